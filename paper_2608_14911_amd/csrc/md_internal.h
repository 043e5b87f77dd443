// Internal definitions shared by the host runtime and the gfx950 kernels of
// the short-range MD step.  Not part of the public ABI (see include/md.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/md.h"

namespace md {

constexpr int kBlock = 256;            // threads per block of the streaming kernels
constexpr int kScanBlocks = 1024;      // chunks (blocks) of the cell-count scan (<= 1024)
constexpr int kChunkPad = 32;          // one 128-byte line per chunk sum (atomics on a line serialize)
constexpr int kMaxGrid = 65535 * 16;   // cap for 1-D grids
constexpr int kNacc = 11;              // reduced quantities per step, see Acc
constexpr int kHistRec = 16;           // doubles per history record

// Order of the per-step FP64 reductions.
enum Acc { A_EPAIR = 0, A_EBOND, A_EANGLE, A_EKIN, A_VIR, A_TXX, A_TYY, A_TZZ, A_TXY, A_TXZ, A_TYZ };

// History record layout (doubles): step, e_pair, e_bond, e_angle, e_kin, W,
// tensor[6], n_rebuilds, status, nl_max, pad.
enum Hist { H_STEP = 0, H_EPAIR, H_EBOND, H_EANGLE, H_EKIN, H_VIR, H_T0, H_NREB = 12, H_STATUS, H_NLMAX };

// Device control block, lives at the start of the workspace.
struct DevCtl {
    int64_t step;          // n of the positions x_n currently stored
    int32_t vel_half;      // 1: stored velocity is v_{n-1/2}; 0: on-step v_n
    uint32_t rebuild;      // rebuild the list before the next force evaluation
    uint32_t rebuild_next; // set by the step kernel when a particle moved > skin/2
    uint32_t status;       // sticky MD_FLAG_* bits
    int32_t nl_max;        // longest row at the last build
    int32_t pad0;
    int64_t n_rebuilds;
    int64_t build_step;    // step of the positions the list was last built from
    int64_t pad[10];
};

// One type pair, precomputed on the host in FP64 and rounded once for FP32.
template <typename Real>
struct PairCoef {
    Real eps4;     // 4 eps
    Real eps24;    // 24 eps
    Real sig2;     // sigma^2
    Real rc2;      // rc^2 (FP64 copy is used for the cutoff test)
    Real shift;    // energy shift
    Real cap2;     // caprad^2 (0: no cap)
    Real ucap;     // u(caprad) - shift
    Real fcap;     // |f(caprad)|
};

struct PairTable {
    PairCoef<double> d[MD_MAX_TYPES * MD_MAX_TYPES];
    PairCoef<float> f[MD_MAX_TYPES * MD_MAX_TYPES];
    double rc2d[MD_MAX_TYPES * MD_MAX_TYPES];
    // FP32 path: r^2 below lo interacts, above hi does not; in between the
    // decision is retaken in FP64 from the FP64 positions
    float rc2lo[MD_MAX_TYPES * MD_MAX_TYPES];
    float rc2hi[MD_MAX_TYPES * MD_MAX_TYPES];
    // tabulated pairs: points (0 = Lennard-Jones), rmin and 1 / grid step;
    // values (u, f) in Bufs::tab rows [pair][table_points]
    int32_t tabn[MD_MAX_TYPES * MD_MAX_TYPES];
    float tab_rmin[MD_MAX_TYPES * MD_MAX_TYPES];
    float tab_idr[MD_MAX_TYPES * MD_MAX_TYPES];
    // AdResS coarse-grained tables (rows kCgTableRow + pair): points (0 = none),
    // rmin, 1 / grid step, and the cutoff (FP64, with the fixed-point band)
    int32_t cgn[MD_MAX_TYPES * MD_MAX_TYPES];
    float cg_rmin[MD_MAX_TYPES * MD_MAX_TYPES];
    float cg_idr[MD_MAX_TYPES * MD_MAX_TYPES];
    double cg_rc2d[MD_MAX_TYPES * MD_MAX_TYPES];
    float cg_rc2lo[MD_MAX_TYPES * MD_MAX_TYPES];
    float cg_rc2hi[MD_MAX_TYPES * MD_MAX_TYPES];
};
constexpr int kAngleTableRow = MD_MAX_TYPES * MD_MAX_TYPES;   // row of the angle table in Bufs::tab
constexpr int kCgTableRow = kAngleTableRow + 1;               // first coarse-grained row
constexpr int kTableRows = kCgTableRow + MD_MAX_TYPES * MD_MAX_TYPES;

// Everything a kernel of one handle needs; passed by value.
struct Geom {
    int64_t n;
    double L[3], hL[3];     // box, half box
    double invL[3];         // 1 / L
    double invh[3];         // cells per unit length
    double h[3];            // cell side
    int nc[3];
    int kc;                 // stencil reach in cells (cells of side >= rv / kc)
    int64_t ncell;
    double rv2;             // list radius squared (FP64, exact same ops as the oracle)
    double disp2;           // (skin/2)^2
    int32_t cap;            // ELL capacity
    int32_t ntypes;
    // 32-bit fixed-point positions: q = floor(x * qs), dx = (int32)(q_j - q_i) * ql
    double qs[3];           // 2^32 / L
    float ql[3];            // L / 2^32
    float rv2lo, rv2hi;     // fixed-point list test band; FP64 test in between
    int32_t nl_tile;        // list build: 1 = one wavefront per 64-particle tile with
                            // candidates broadcast through the scalar cache, 0 = one
                            // particle per lane
    int32_t nl_cubic;       // cubic box: the tile build tests r^2 in fixed-point units
    float rq2lo, rq2hi;     // the list band in units of (L 2^-32)^2 (cubic box)
    uint32_t r16lo, r16hi;  // a wider band in units of (L 2^-16)^2 for the 16-bit
                            // prefilter of the tile build (cubic box)
    int32_t x3_on;          // keep the 12-byte position records (systems without bonds,
                            // whose fast step kernel gathers them)
    // Lees-Edwards shear (flow x, gradient y): offset delta(step) =
    // fmod(le_rate_Ly * (step * le_dt), Lx); images one box above move with
    // +le_rate_Ly along x
    int32_t le;
    double le_rate_Ly;      // shear_rate * Ly
    double le_dt;           // dt (the offset assumes a constant time step)
    double skin;
    int32_t table_points;   // row length of Bufs::tab
};

struct Bufs {
    DevCtl* ctl;
    double* partials;       // [kNacc][grid]
    double* hist;           // [MD_HISTORY_CAPACITY][kHistRec]
    double* cur;            // [kHistRec] observables of the last finalize
    double4* x[2];          // positions (w = type), sorted order, by step parity
    int4* xq[2];            // fixed-point positions (w = type), by step parity
    int32_t* x3[2];         // the same x, y, z as 12-byte records, by parity (kept when Geom::x3_on)
    double* v;              // [3][N] SoA, sorted order
    double* xb;             // [3][N] positions at the last build
    int32_t* img;           // [3][N]
    int32_t* type_t;        // [N] particle types in tag order
    int32_t* tag;           // sorted -> tag
    int32_t* inv;           // tag -> sorted
    uint32_t* cellid;       // [N]
    int32_t* ccount;        // [ncell], all zero between rebuilds
    int32_t* cstart;        // [ncell + 1]
    int32_t* bsum;          // [kScanBlocks] chunk sums; one system: [kScanBlocks][kChunkPad], column 0
    int32_t* tmp;           // [N] scatter slots
    double4* xt;            // permute temporaries
    double* vt;
    int32_t* imgt;
    int32_t* tsc;           // [N] tags in scatter order (rank inside a cell)
    int32_t* nl;            // ELL in 64-particle tiles [N/64][cap][64], sorted indices
    int32_t* ncount;        // [N]
    // topology, tag space (static) and sorted space (remapped at each build)
    int32_t* tcnt_t;        // [N] nbond | nangle << 8
    int32_t* bp_t;          // [MAXB][N] partner tags
    int2* ang_t;            // [MAXA][N] (other1 | role << 30, other2) tags
    int32_t* tcnt_s;        // [N]
    int32_t* bp_s;          // [MAXB][N]
    int2* ang_s;            // [MAXA][N]
    int32_t maxb, maxa;     // row counts actually used (<= limits)
    float2* tab;            // [kTableRows][table_points] (u, f) or (u, du/dphi); or null
};

struct Dyn {
    double dt;
    double hdtm[MD_MAX_TYPES];  // dt / (2 m)
    double mass[MD_MAX_TYPES];
    double gm[MD_MAX_TYPES];    // gamma m
    double amp[MD_MAX_TYPES];   // sqrt(2 gamma m kT / dt)
    int32_t langevin;
    uint64_t seed;
    double fene_K, fene_R02;
    double fene_halfKR02;       // K R0^2 / 2
    float fene_Kf, fene_R02f, fene_halfKR02f;
    double k_bend;
    float k_bendf;
    // DPD pair thermostat (integrator MD_DPD): -gamma w^2 (e.v) e + sigma w theta e / sqrt(dt)
    int32_t dpd;
    float dpd_rc, dpd_rc2;
    float dpd_gamma;
    float dpd_sigma_isdt;   // sqrt(2 gamma kT) / sqrt(dt)
    // the generic FP32 step kernel is needed (shear, DPD, tables, angle kinds)
    int32_t gen;
    int32_t angle_kind;     // MD_ANGLE_*
    float angle_K, cos_phi0;
    int32_t ang_n;          // points of the angle table
    float ang_idphi;        // (ang_n - 1) / pi
    const float2* ang_tab;  // the angle table (u, du/dphi), or null
    // AdResS slab along x: weight 1 within d_at of x0, cos^2 switch over d_hy
    int32_t adress;
    float ad_x0, ad_dat, ad_dhy, ad_k;   // ad_k = pi / (2 d_hy)
};

// internal status bit (init only): a particle type outside 0..n_types-1
constexpr uint32_t MD_FLAG_BAD_TYPE = 0x100u;

enum Mode { MODE_STEP = 0, MODE_OBSERVE = 1, MODE_FORCES = 2 };

// Single-type LJ coefficients rescaled to fixed-point length units u = L/2^32
// (cubic box): r2 and the band limits in u^2, sigma^2 / u^2, 24 eps / u.
struct FastCoef {
    float rc2lo, rc2hi;     // band limits on r2 in u^2
    float sig2u;            // sigma^2 / u^2
    float eps24_u;          // 24 eps / u
    float eps4, eps24, shift;
    double rc2d;            // rc^2 (FP64 re-decision)
};

struct StepArgs {
    Geom g;
    Bufs b;
    PairTable pt;
    Dyn dy;
    FastCoef fast;
    int32_t use_fast;
    int32_t parity;
    int32_t mode;
    int32_t tensor;
    double* f_out;              // MODE_FORCES: [N][3] tag order
};

// ------------------------------------------------------------------ surrogate

constexpr int kSurNB = 32;                  // radial basis functions
constexpr int kSurH = 64;                   // hidden width
constexpr int kSurNP = 6337;                // parameters
constexpr int kSurNPpad = 6400;
constexpr int kOW1 = 0, kOB1 = 2048, kOW2 = 2112, kOB2 = 6208, kOW3 = 6272, kOB3 = 6336;
// prepared FP32 weights, rows padded for the LDS image: W1 [64][36],
// W1T [32][68], W2 [64][68], W2T [64][68], then b1, b2, w3 [64], b3
constexpr int kPF1 = 36, kPF64 = 68;
constexpr int kPW1 = 0, kPW1T = 64 * kPF1, kPW2 = kPW1T + 32 * kPF64, kPW2T = kPW2 + 64 * kPF64,
              kPB1 = kPW2T + 64 * kPF64, kPB2 = kPB1 + 64, kPW3 = kPB2 + 64, kPB3 = kPW3 + 64,
              kPrepF = kPB3 + 64;
// prepared BF16 weights, rows padded for the LDS image: W1 [64][40],
// W1T [32][72], W2 [64][72], W2T [64][72]
constexpr int kSW1 = 40, kSW64 = 72;
constexpr int kQW1 = 0, kQW1T = 64 * kSW1, kQW2 = kQW1T + 32 * kSW64, kQW2T = kQW2 + 64 * kSW64,
              kPrepB = kQW2T + 64 * kSW64;
// prepared BF16 weights for the 16x16x32 matrix-core network (inference):
// A-operand images with the K axis in slot order (see md_surrogate.hip):
// W1 [64][40], W2 [64][72], W2^T [64][72], W1^T [32][72]
constexpr int kMS1 = 40, kMS64 = 72;
constexpr int kM1 = 0, kM2 = 64 * kMS1, kM2T = kM2 + 64 * kMS64, kM1T = kM2T + 64 * kMS64,
              kPrepM = kM1T + 32 * kMS64;
constexpr int kSurPart = 9;                 // E, W, tensor[6], loss
constexpr int kSurGradBlocks = 256;         // blocks of the double-backward kernel
constexpr int kSurMomBlocks = 256;          // blocks of the descriptor-moment kernel (partials in gpart)
static_assert(kSurMomBlocks * 2 * kSurNB * 2 <= kSurGradBlocks * kSurNPpad, "moment partials fit in gpart");

struct SurBufs {
    float* G;           // [N][32] descriptors, sorted order
    float* a;           // [N][32] dE_i/dG(i)
    uint16_t* ab;       // [N][32] the same in BF16 (the BF16 form's pair-force pass)
    float* u;           // [N][32] training: dL/da_i
    float4* f;          // [N] surrogate pair force
    float4* delta;      // [N] training: dL/dF_i
    double* part;       // [kSurPart][step grid] block partials
    double* loss;       // [1] loss accumulated over the frames of a call
    float* w;           // [kSurNPpad] master weights
    float* wp;          // [kPrepF] prepared FP32 weights
    uint16_t* wb;       // [kPrepB] prepared BF16 weights
    uint16_t* wm;       // [kPrepM] prepared BF16 weights, matrix-core operand images
    float* gmean;       // [32]
    float* gistd;       // [32]
    float* grad;        // [kSurNPpad]
    float* m1;          // [kSurNPpad] Adam moments
    float* m2;
    float* gpart;       // [kSurGradBlocks][kSurNPpad]
};

struct SurConst {
    float mu[kSurNB];   // basis centres
    float c_exp;        // log2(e) / (2 w^2): phi = exp2(-c_exp (r - mu)^2)
    float inv_w2;       // 1 / w^2
    float rd2;          // r_d^2
    float pi_rd;        // pi / r_d
    float dmu;          // centre spacing
    float ratio;        // exp2(-2 c_exp dmu^2): step of the basis recurrences
};

hipError_t launch_sur_prepare(const SurBufs& s, hipStream_t st);
hipError_t launch_sur_mlp(const SurBufs& s, const float* G, int64_t P, float* a, float* e, double* epart,
                          int bf16, int grid, hipStream_t st, uint16_t* a16 = nullptr);
hipError_t launch_sur_force(const Geom& g, const Bufs& b, const SurBufs& s, const SurConst& c, int parity,
                            const double* fref, double two_over_m, int tensor, int grid, hipStream_t st,
                            int a_bf16 = 0);
hipError_t launch_sur_u(const Geom& g, const Bufs& b, const SurBufs& s, const SurConst& c, int parity, int grid,
                        hipStream_t st);
hipError_t launch_sur_bwd2(const SurBufs& s, int64_t P, int bf16, hipStream_t st);
hipError_t launch_sur_grad_reduce(const SurBufs& s, int nblk, int accumulate, hipStream_t st);
int sur_bwd2_grid(int64_t P);
hipError_t launch_sur_loss_reduce(const SurBufs& s, int grid, int accumulate, hipStream_t st);
hipError_t launch_sur_adam(const SurBufs& s, int64_t t, float lr, float beta1, float beta2, float eps,
                           hipStream_t st);
hipError_t launch_sur_to_tag(const Geom& g, const Bufs& b, const float* src, float* dst, hipStream_t st);
hipError_t launch_sur_moments(const SurBufs& s, int64_t n, int accumulate, hipStream_t st);
hipError_t launch_sur_moments_final(const SurBufs& s, double cnt, double floor_var, float* g_mean, float* g_istd,
                                    hipStream_t st);
hipError_t launch_sur_from_tag(const Geom& g, const Bufs& b, const float* src, float* dst, hipStream_t st);
hipError_t launch_sur_f_to_tag(const Geom& g, const Bufs& b, const float4* src, double* dst, hipStream_t st);
// inference: descriptors (FP32 rows into s.G, or with net != 0 fused with the
// BF16 network: s.ab rows and energy partials in s.part row 0), the BF16
// network on given rows, and the pair force fused with bonded forces and
// integration (the step kernel of the surrogate mode)
hipError_t launch_sur_desc2(const Geom& g, const Bufs& b, const SurBufs& s, const SurConst& c, int parity, int net,
                            hipStream_t st);
hipError_t launch_sur_mlp16(const SurBufs& s, const float* G, int64_t P, float* a, float* e, hipStream_t st);
hipError_t launch_sur_step(const StepArgs& a, const SurBufs& s, const SurConst& c, int bonded, int a_bf16,
                           hipStream_t st);

// ------------------------------------------------------------------ batches

// One system of a batch as the per-tile kernels see it.  Tiles of kBlock
// particles never straddle systems; tile0 is the system's first global tile.
struct SysEntry {
    StepArgs a;             // parity / mode fields unused: kernel arguments
    int64_t tile0;
    int32_t ntiles;
    int32_t bonded;
    int64_t c_off;          // first cell in the concatenated cell arrays
};

// Concatenated cell arrays of a batch and the descriptor of their scan.
struct BatchCells {
    Geom gg;                // gg.ncell = all cells (each system's ncell + 1)
    Bufs gb;                // gb.ccount / gb.cstart / gb.bsum / gb.ctl (any-rebuild flag)
    const SysEntry* tab;    // device table (any parity)
    int64_t* c_off;         // [nsys + 1] first cell per system
    int32_t* base;          // [nsys] scan prefix at each system's first cell
    int32_t nsys;
};

// ev_sorted (or null) is recorded between the cell sort and the list build
hipError_t launch_batch_rebuild(const BatchCells& bc, const SysEntry* tab, const int32_t* tile_sys, int64_t ntiles,
                                int parity, hipStream_t s, hipEvent_t ev_sorted = nullptr);
hipError_t launch_batch_step(const SysEntry* tab, const int32_t* tile_sys, int64_t ntiles, int parity, int mode,
                             int tensor, hipStream_t s);
hipError_t launch_batch_finalize(const SysEntry* tab, int nsys, int mode, hipStream_t s);
hipError_t launch_batch_gather_obs(const SysEntry* tab, int nsys, double* out, hipStream_t s);

// launchers (md_kernels.hip)
hipError_t launch_init_load(const Geom& g, const Bufs& b, int parity, const double* pos,
                            const double* vel, const int32_t* type, const int32_t* image,
                            hipStream_t s);
hipError_t launch_set_ctl(const Bufs& b, int64_t step, int vel_half, int rebuild, int clear_status,
                          hipStream_t s);
hipError_t launch_rebuild(const Geom& g, const Bufs& b, int parity, int bonded, hipStream_t s,
                          hipEvent_t ev_sorted = nullptr);
hipError_t launch_clear_rebuild(const Bufs& b, hipStream_t s);
hipError_t launch_step(const StepArgs& a, int fp64, int single_type, int bonded, int block,
                       hipStream_t s);
int step_grid(int64_t n);
// blocks of the plain force kernel that launch_step runs with `block`
// threads per block (the FP32 fast kernels take 64..512; the others 256)
int step_launch_grid(const StepArgs& a, int fp64, int block);
// spart: surrogate partials (row 0 energy; with spart_rows 8 also virial and
// tensor rows), or nullptr
hipError_t launch_finalize(const Bufs& b, int nblocks, int mode, const double* spart, int tensor, hipStream_t s,
                           int spart_rows = 8);
hipError_t launch_overwrite_state(const Geom& g, const Bufs& b, int parity, const double* pos,
                                  const double* vel, const int32_t* image, hipStream_t s);
hipError_t launch_get_state(const Geom& g, const Bufs& b, int parity, double* pos, double* vel,
                            int32_t* image, double* pos_build, hipStream_t s);
hipError_t launch_copy_i32(int32_t* dst, const int32_t* src, int64_t n, hipStream_t s);
hipError_t launch_get_neighbors(const Geom& g, const Bufs& b, int32_t* count, int32_t* idx,
                                int32_t cap, hipStream_t s);
hipError_t launch_zero_i32(int32_t* p, int64_t n, hipStream_t s);

}  // namespace md
