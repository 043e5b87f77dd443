// Host runtime and C ABI of the short-range MD step (include/md.h).
//
// The handle plans the cell grid, carves the caller's workspace, keeps
// host mirrors of the step counter and the position-buffer parity, and
// enqueues every step as
//     rebuild stage (8 kernels that return at once unless a particle moved
//     more than skin/2) -> fused force+integrate kernel -> 1-block finalize
// on the caller's stream, optionally replayed from a hipGraph of two steps.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "md_internal.h"

using namespace md;

namespace {

thread_local std::string g_last_error;

// e[0] step start, e[4] after the cell sort, e[1] after the list build,
// e[2] after the force stage, e[3] after the finalize
constexpr int kStepEvents = 5;
struct EvQuad {
    hipEvent_t e[kStepEvents];
};

}  // namespace

struct md_handle_s {
    md_config cfg;
    Geom g;
    Bufs b;
    PairTable pt;
    Dyn dy;
    FastCoef fast;
    int32_t use_fast = 0;
    hipStream_t stream = nullptr;
    int parity = 0;
    int64_t host_step = 0;
    int32_t vel_half = 0;
    int bonded = 0, single = 1, fp64 = 0;
    int step_grid = 1;
    int64_t hist_next = 0;
    std::string err;
    uint8_t* ws = nullptr;
    size_t ws_bytes = 0;
    // graph of two steps, valid for one parity
    hipGraphExec_t gexec = nullptr;
    int graph_parity = -1;
    // timing
    bool timing = false;
    std::vector<EvQuad> ev_free, ev_pending;
    md_timing tacc;
    // learned surrogate
    SurBufs sb;
    SurConst sc;
    int has_sur = 0;          // workspace reserved
    int sur_loaded = 0;       // md_sur_set called
    int sur_prec = MD_SUR_FP32;
    int pair_mode = MD_PAIR_PLAIN;
    // device whose static workspace this handle uses (md_init_static), or -1
    int static_dev = -1;
    // tables set so far (kept across md_set_params)
    int32_t tabn[MD_MAX_TYPES * MD_MAX_TYPES] = {};
    double tab_rmin[MD_MAX_TYPES * MD_MAX_TYPES] = {};
    int32_t ang_n = 0;
    int32_t cgn[MD_MAX_TYPES * MD_MAX_TYPES] = {};
    double cg_rmin[MD_MAX_TYPES * MD_MAX_TYPES] = {};
    double cg_rc[MD_MAX_TYPES * MD_MAX_TYPES] = {};
};

// ------------------------------------------------------------------ static workspace
// Workspace of md_init_static: a file-scope device array, one copy per GPU,
// held by the code object until the process ends.  In host code its name is
// only a stand-in; the device address comes from hipGetSymbolAddress, taken
// once per device with that device current.
static __device__ __align__(256) uint8_t scratch[MD_STATIC_WORKSPACE_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
uint8_t* g_static_ptr[kMaxDevices];     // device address of `scratch`, per device
md_handle g_static_owner[kMaxDevices];  // live handle on that device's array, or nullptr
}  // namespace

// ------------------------------------------------------------------ helpers

static md_status fail(md_handle h, md_status st, const std::string& msg) {
    if (h) h->err = msg;
    g_last_error = msg;
    return st;
}

#define HIP_TRY(h, call)                                                                   \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail((h), MD_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static md_status validate(const md_config* c, std::string* why) {
    if (!c) { *why = "config is NULL"; return MD_ERR_ARG; }
    if (c->struct_size != sizeof(md_config)) { *why = "md_config.struct_size mismatch (ABI version)"; return MD_ERR_ARG; }
    if (c->n_types < 1 || c->n_types > MD_MAX_TYPES) { *why = "n_types out of range"; return MD_ERR_ARG; }
    // the step kernels address gathered records with 32-bit byte offsets
    // (16 bytes per particle): at most 2^28 - 1 particles per system
    if (c->n_particles < 1 || c->n_particles > ((int64_t)1 << 28) - 1) {
        *why = "n_particles out of range (1 .. 2^28 - 1)";
        return MD_ERR_ARG;
    }
    for (int d = 0; d < 3; ++d)
        if (!(c->box[d] > 0.0) || !isfinite(c->box[d])) { *why = "box must be positive and finite"; return MD_ERR_ARG; }
    if (!(c->dt > 0.0) || !isfinite(c->dt)) { *why = "dt must be > 0"; return MD_ERR_ARG; }
    if (!(c->skin > 0.0) || !isfinite(c->skin)) { *why = "skin must be > 0"; return MD_ERR_ARG; }
    if (c->integrator != MD_NVE && c->integrator != MD_LANGEVIN && c->integrator != MD_DPD) {
        *why = "unknown integrator";
        return MD_ERR_ARG;
    }
    if (c->force_precision != MD_FP64 && c->force_precision != MD_FP32) { *why = "unknown force precision"; return MD_ERR_ARG; }
    if (c->block_size != 0 && c->block_size != 64 && c->block_size != 128 && c->block_size != 256 &&
        c->block_size != 512) {
        *why = "block_size must be 0, 64, 128, 256 or 512";
        return MD_ERR_ARG;
    }
    if (c->integrator != MD_NVE && (!(c->gamma >= 0.0) || !(c->temperature >= 0.0))) {
        *why = "thermostat gamma and temperature must be >= 0";
        return MD_ERR_ARG;
    }
    if (c->integrator == MD_DPD && !(c->dpd_rc > 0.0 && isfinite(c->dpd_rc))) {
        *why = "DPD needs dpd_rc > 0";
        return MD_ERR_ARG;
    }
    if (!isfinite(c->shear_rate)) { *why = "shear_rate must be finite"; return MD_ERR_ARG; }
    if ((c->integrator == MD_DPD || c->shear_rate != 0.0) && c->force_precision != MD_FP32) {
        *why = "DPD and Lees-Edwards shear run on the FP32 pair path (force_precision MD_FP32)";
        return MD_ERR_ARG;
    }
    const int nt = c->n_types;
    for (int a = 0; a < nt; ++a)
        for (int bb = 0; bb < nt; ++bb) {
            const md_pair_params& p = c->pair[a * MD_MAX_TYPES + bb];
            const md_pair_params& q = c->pair[bb * MD_MAX_TYPES + a];
            if (!(p.rc > 0.0) || !(p.sigma > 0.0) || !(p.eps >= 0.0) || !(p.caprad >= 0.0) || !isfinite(p.rc)) {
                *why = "pair parameters: need rc > 0, sigma > 0, eps >= 0, caprad >= 0";
                return MD_ERR_ARG;
            }
            if (memcmp(&p, &q, sizeof(p)) != 0) { *why = "pair table must be symmetric"; return MD_ERR_ARG; }
        }
    if (c->n_bonds < 0 || c->n_angles < 0) { *why = "negative bond/angle count"; return MD_ERR_ARG; }
    if (c->n_bonds > 0 && !(c->fene_R0 > 0.0 && c->fene_K >= 0.0)) { *why = "FENE needs R0 > 0, K >= 0"; return MD_ERR_ARG; }
    if (c->nl_capacity < 0 || c->nl_capacity > 4096) { *why = "nl_capacity out of range"; return MD_ERR_ARG; }
    if (c->cell_factor < 0 || c->cell_factor > 2) { *why = "cell_factor must be 0, 1 or 2"; return MD_ERR_ARG; }
    if (!(c->list_cutoff >= 0.0) || !isfinite(c->list_cutoff)) { *why = "list_cutoff must be >= 0"; return MD_ERR_ARG; }
    if (c->surrogate != 0 && c->surrogate != 1) { *why = "surrogate must be 0 or 1"; return MD_ERR_ARG; }
    if (c->table_points < 0 || c->table_points > 65536) { *why = "table_points out of range (0 .. 65536)"; return MD_ERR_ARG; }
    if (c->angle_kind < MD_ANGLE_COSINE || c->angle_kind > MD_ANGLE_TABULATED) { *why = "unknown angle kind"; return MD_ERR_ARG; }
    if ((c->table_points > 0 || c->angle_kind != MD_ANGLE_COSINE) && c->force_precision != MD_FP32) {
        *why = "tables and angle kinds other than MD_ANGLE_COSINE run on the FP32 pair path";
        return MD_ERR_ARG;
    }
    if (c->adress != 0 && c->adress != 1) { *why = "adress must be 0 or 1"; return MD_ERR_ARG; }
    if (c->adress && (c->table_points < 2 || !(c->adress_d_at >= 0.0) || !(c->adress_d_hy > 0.0) ||
                      !isfinite(c->adress_x0))) {
        *why = "AdResS needs table_points >= 2, d_at >= 0 and d_hy > 0";
        return MD_ERR_ARG;
    }
    if (c->angle_kind == MD_ANGLE_TABULATED && c->table_points < 2) {
        *why = "MD_ANGLE_TABULATED needs table_points >= 2";
        return MD_ERR_ARG;
    }
    return MD_OK;
}

static double rc_max_of(const md_config* c) {
    double m = 0.0;
    for (int a = 0; a < c->n_types; ++a)
        for (int bb = 0; bb < c->n_types; ++bb) m = fmax(m, c->pair[a * MD_MAX_TYPES + bb].rc);
    return m;
}

// Width of the band around a squared cutoff r2 inside which a decision
// taken on fixed-point coordinates is retaken in FP64: four times a bound on
// |r2_fixed - r2| from the quantisation (L / 2^32 per coordinate), the
// int->float conversion and the FP32 products.
static double fixed_band(double r2, double Lmax) {
    const double r = sqrt(r2);
    const double eq = Lmax * 0x1.0p-32;
    return 4.0 * (2.0 * sqrt(3.0) * r * 2.0 * eq + (4.0 * sqrt(3.0) + 4.0) * 0x1.0p-24 * r2);
}

static md_status plan_geom(const md_config* c, Geom* g, std::string* why) {
    md_status st = validate(c, why);
    if (st != MD_OK) return st;
    memset(g, 0, sizeof(*g));
    g->n = c->n_particles;
    g->ntypes = c->n_types;
    const double rv = fmax(fmax(rc_max_of(c), c->list_cutoff), c->integrator == MD_DPD ? c->dpd_rc : 0.0) + c->skin;
    g->rv2 = rv * rv;
    g->disp2 = (0.5 * c->skin) * (0.5 * c->skin);
    // List build: dense systems (>= 8 particles expected in a cell of side
    // rv) one wavefront per 64-particle tile, others one particle per lane,
    // both on cells of side rv; half-cutoff sub-cells only when the box holds
    // fewer than 3 cells of side rv per axis.  Measured on MI355X (2M-bead
    // melt, 3 beads per cell): the per-particle build on cells of side rv
    // beats half-cutoff sub-cells by 12% in whole-step throughput (fewer
    // stencil rows, each a memory round trip) and the tile build, whose
    // shared candidate stream is 2.4-7.7x longer than a lane's own.
    const double density = (double)c->n_particles / (c->box[0] * c->box[1] * c->box[2]);
    const bool per_particle = (c->flags & MD_CFG_NL_PER_PARTICLE) != 0;
    const bool dense = density * rv * rv * rv >= 8.0 && !per_particle;
    g->kc = c->cell_factor;
    if (g->kc == 0) {
        bool fit1 = true, fit2 = true;
        for (int d = 0; d < 3; ++d) {
            if ((int)floor(c->box[d] / (rv * (1.0 + 1e-12))) < 3) fit1 = false;
            if ((int)floor(c->box[d] * 2.0 / (rv * (1.0 + 1e-12))) < 5) fit2 = false;
        }
        g->kc = fit1 ? 1 : (fit2 ? 2 : 1);
    }
    g->ncell = 1;
    double Lmax = 0.0;
    for (int d = 0; d < 3; ++d) {
        g->L[d] = c->box[d];
        g->hL[d] = 0.5 * c->box[d];
        g->invL[d] = 1.0 / c->box[d];
        Lmax = fmax(Lmax, c->box[d]);
        int nc = (int)floor(c->box[d] * g->kc / (rv * (1.0 + 1e-12)));
        if (nc < 2 * g->kc + 1) {
            char buf[200];
            snprintf(buf, sizeof buf, "box %.6g holds %d cells of side >= (rc+skin)/%d = %.6g along axis %d; need >= %d",
                     c->box[d], nc, g->kc, rv / g->kc, d, 2 * g->kc + 1);
            *why = buf;
            return MD_ERR_BOX_TOO_SMALL;
        }
        if (nc > 4096) nc = 4096;
        g->nc[d] = nc;
        g->invh[d] = (double)nc / c->box[d];
        g->h[d] = c->box[d] / (double)nc;
        g->ncell *= nc;
        g->qs[d] = 0x1.0p32 / c->box[d];
        g->ql[d] = (float)(c->box[d] * 0x1.0p-32);
    }
    const double band = fixed_band(g->rv2, Lmax);
    g->rv2lo = (float)(g->rv2 - band);
    g->rv2hi = (float)(g->rv2 + band);
    if (c->nl_capacity > 0) {
        // rows are padded and streamed in batches of 8 slots, so the capacity
        // is a multiple of 8 (4096 already is): a batch never reads past a row
        g->cap = (c->nl_capacity + 7) & ~7;
    } else {
        const double vol = c->box[0] * c->box[1] * c->box[2];
        const double expect = (double)c->n_particles / vol * (4.0 / 3.0) * M_PI * rv * rv * rv;
        int cap = (int)ceil(1.5 * expect + 32.0);
        cap = (cap + 7) & ~7;
        if (cap < 16) cap = 16;
        if (cap > 4096) cap = 4096;
        g->cap = cap;
    }
    g->nl_tile = (!per_particle && ((c->flags & MD_CFG_NL_TILES) || (dense && g->kc == 1))) ? 1 : 0;
    g->le = c->shear_rate != 0.0 ? 1 : 0;
    g->le_rate_Ly = c->shear_rate * c->box[1];
    g->le_dt = c->dt;
    g->skin = c->skin;
    g->table_points = c->table_points;
    if (g->le) g->nl_tile = 0;   // the sheared stencil is built one particle per lane
    g->nl_cubic = (c->box[0] == c->box[1] && c->box[1] == c->box[2]) ? 1 : 0;
    // the unbonded fast step kernel gathers 12-byte records (fewer L1 lines per
    // gather: 4% faster on the LJ fluid); the bonded one keeps the 16-byte
    // records, for which the extra stores cost more than the gathers save
    g->x3_on = (c->n_bonds == 0 && c->n_angles == 0) ? 1 : 0;
    {
        // rv^2 -/+ band over ql^2 (ql = L 2^-32 exactly), rounded outwards to float
        const double ql = c->box[0] * 0x1.0p-32;
        const double lo = (g->rv2 - band) / (ql * ql), hi = (g->rv2 + band) / (ql * ql);
        float flo = (float)lo, fhi = (float)hi;
        if ((double)flo > lo) flo = nextafterf(flo, 0.0f);
        if ((double)fhi < hi) fhi = nextafterf(fhi, INFINITY);
        g->rq2lo = flo;
        g->rq2hi = fhi;
        // 16-bit prefilter: dx16 = (int32)(q_j - q_i) >> 16 is within e = U + ql
        // of the FP64 difference (U = L 2^-16), so |r16^2 U^2 - r^2| stays
        // below 2 rv sqrt(3) e + 3 e^2 around rv; 1.5x that, rounded outwards
        const double U = c->box[0] * 0x1.0p-16, e = U + ql;
        const double B16 = 1.5 * (2.0 * rv * sqrt(3.0) * e + 3.0 * e * e);
        const double l16 = floor((g->rv2 - B16) / (U * U)), h16 = ceil((g->rv2 + B16) / (U * U));
        g->r16lo = (uint32_t)fmax(0.0, fmin(l16, 4294967295.0));
        g->r16hi = (uint32_t)fmax(0.0, fmin(h16, 4294967295.0));
    }
    return MD_OK;
}

// Partial-sum columns: one per block of the plain force kernel at its
// smallest block (64 threads), at least one per block of the others.
static int64_t part_cols(int64_t n) {
    const int64_t c = (n + 63) / 64;
    return c > (int64_t)step_grid(n) ? c : (int64_t)step_grid(n);
}

// Carve the workspace; with base == nullptr only the size is computed.
static size_t carve(const md_config* c, const Geom& g, int step_grid, uint8_t* base, Bufs* b,
                    SurBufs* sb = nullptr, bool ext_cells = false) {
    const int64_t n = g.n;
    const bool bonded = c->n_bonds > 0 || c->n_angles > 0;
    const int maxb = c->n_bonds > 0 ? MD_MAX_BONDS_PER_PARTICLE : 0;
    const int maxa = c->n_angles > 0 ? MD_MAX_ANGLES_PER_PARTICLE : 0;
    size_t off = 0;
    auto take = [&](size_t bytes) -> void* {
        void* p = base ? (void*)(base + off) : nullptr;
        off += align256(bytes);
        return p;
    };
    Bufs t;
    memset(&t, 0, sizeof(t));
    t.ctl = (DevCtl*)take(sizeof(DevCtl));
    t.cur = (double*)take(sizeof(double) * kHistRec);
    t.hist = (double*)take(sizeof(double) * kHistRec * MD_HISTORY_CAPACITY);
    t.partials = (double*)take(sizeof(double) * kNacc * (size_t)part_cols(n));
    t.x[0] = (double4*)take(sizeof(double4) * n);
    t.x[1] = (double4*)take(sizeof(double4) * n);
    t.xq[0] = (int4*)take(sizeof(int4) * n);
    t.xq[1] = (int4*)take(sizeof(int4) * n);
    t.x3[0] = (int32_t*)take(sizeof(int32_t) * 3 * n);
    t.x3[1] = (int32_t*)take(sizeof(int32_t) * 3 * n);
    t.v = (double*)take(sizeof(double) * 3 * n);
    t.xb = (double*)take(sizeof(double) * 3 * n);
    t.img = (int32_t*)take(sizeof(int32_t) * 3 * n);
    t.type_t = (int32_t*)take(sizeof(int32_t) * n);
    t.tag = (int32_t*)take(sizeof(int32_t) * n);
    t.inv = (int32_t*)take(sizeof(int32_t) * n);
    t.cellid = (uint32_t*)take(sizeof(uint32_t) * n);
    if (!ext_cells) {   // batch members use the batch's concatenated cell arrays
        t.ccount = (int32_t*)take(sizeof(int32_t) * g.ncell);
        t.cstart = (int32_t*)take(sizeof(int32_t) * (g.ncell + 1));
    }
    t.bsum = (int32_t*)take(sizeof(int32_t) * kScanBlocks * kChunkPad);
    t.tmp = (int32_t*)take(sizeof(int32_t) * n);
    t.xt = (double4*)take(sizeof(double4) * n);
    t.vt = (double*)take(sizeof(double) * 3 * n);
    t.imgt = (int32_t*)take(sizeof(int32_t) * 3 * n);
    t.tsc = (int32_t*)take(sizeof(int32_t) * n);
    t.ncount = (int32_t*)take(sizeof(int32_t) * n);
    t.nl = (int32_t*)take(sizeof(int32_t) * (size_t)g.cap * (size_t)((n + 63) / 64 * 64));
    if (bonded) {
        t.tcnt_t = (int32_t*)take(sizeof(int32_t) * n);
        t.tcnt_s = (int32_t*)take(sizeof(int32_t) * n);
        if (maxb) {
            t.bp_t = (int32_t*)take(sizeof(int32_t) * (size_t)maxb * n);
            t.bp_s = (int32_t*)take(sizeof(int32_t) * (size_t)maxb * n);
        }
        if (maxa) {
            t.ang_t = (int2*)take(sizeof(int2) * (size_t)maxa * n);
            t.ang_s = (int2*)take(sizeof(int2) * (size_t)maxa * n);
        }
    }
    t.maxb = maxb;
    t.maxa = maxa;
    if (c->table_points > 0) t.tab = (float2*)take(sizeof(float2) * (size_t)kTableRows * c->table_points);
    if (b) *b = t;
    if (c->surrogate) {
        SurBufs u;
        memset(&u, 0, sizeof(u));
        u.G = (float*)take(sizeof(float) * kSurNB * n);
        u.a = (float*)take(sizeof(float) * kSurNB * n);
        u.ab = (uint16_t*)take(sizeof(uint16_t) * kSurNB * n);
        u.u = (float*)take(sizeof(float) * kSurNB * n);
        u.f = (float4*)take(sizeof(float4) * n);
        u.delta = (float4*)take(sizeof(float4) * n);
        u.part = (double*)take(sizeof(double) * kSurPart * (size_t)step_grid);
        u.loss = (double*)take(sizeof(double) * 4);
        u.w = (float*)take(sizeof(float) * kSurNPpad);
        u.wp = (float*)take(sizeof(float) * kPrepF);
        u.wb = (uint16_t*)take(sizeof(uint16_t) * kPrepB);
        u.wm = (uint16_t*)take(sizeof(uint16_t) * kPrepM);
        u.gmean = (float*)take(sizeof(float) * kSurNB);
        u.gistd = (float*)take(sizeof(float) * kSurNB);
        u.grad = (float*)take(sizeof(float) * kSurNPpad);
        u.m1 = (float*)take(sizeof(float) * kSurNPpad);
        u.m2 = (float*)take(sizeof(float) * kSurNPpad);
        u.gpart = (float*)take(sizeof(float) * kSurNPpad * (size_t)kSurGradBlocks);
        if (sb) *sb = u;
    }
    return off;
}

static int step_grid_of(int64_t n) { return step_grid(n); }

static void fill_params(md_handle h, const md_config* c) {
    PairTable& pt = h->pt;
    memset(&pt, 0, sizeof(pt));
    for (int a = 0; a < c->n_types; ++a)
        for (int bb = 0; bb < c->n_types; ++bb) {
            const int tp = a * MD_MAX_TYPES + bb;
            const md_pair_params& p = c->pair[tp];
            double shift;
            if (isnan(p.shift)) {
                double s2 = (p.sigma * p.sigma) / (p.rc * p.rc);
                double s6 = s2 * s2 * s2;
                shift = 4.0 * p.eps * (s6 * s6 - s6);
            } else {
                shift = p.shift;
            }
            PairCoef<double> d;
            d.eps4 = 4.0 * p.eps;
            d.eps24 = 24.0 * p.eps;
            d.sig2 = p.sigma * p.sigma;
            d.rc2 = p.rc * p.rc;
            d.shift = shift;
            d.cap2 = p.caprad > 0.0 ? p.caprad * p.caprad : 0.0;
            d.ucap = 0.0;
            d.fcap = 0.0;
            if (p.caprad > 0.0) {
                double s2 = d.sig2 / d.cap2, s6 = s2 * s2 * s2, s12 = s6 * s6;
                d.ucap = 4.0 * p.eps * (s12 - s6) - shift;
                d.fcap = 24.0 * p.eps * (2.0 * s12 - s6) / d.cap2 * sqrt(d.cap2);
            }
            pt.d[tp] = d;
            pt.f[tp] = PairCoef<float>{(float)d.eps4, (float)d.eps24, (float)d.sig2, (float)d.rc2,
                                       (float)d.shift, (float)d.cap2, (float)d.ucap, (float)d.fcap};
            pt.rc2d[tp] = p.rc * p.rc;
            double Lmax = fmax(c->box[0], fmax(c->box[1], c->box[2]));
            const double band = fixed_band(p.rc * p.rc, Lmax);
            pt.rc2lo[tp] = (float)(p.rc * p.rc - band);
            pt.rc2hi[tp] = (float)(p.rc * p.rc + band);
        }
    // fast FP32 path: one type, cubic box, no capping radius
    {
        const md_pair_params& p = c->pair[0];
        const bool cubic = c->box[0] == c->box[1] && c->box[1] == c->box[2];
        h->use_fast = (c->n_types == 1 && cubic && !(p.caprad > 0.0) && c->integrator != MD_DPD &&
                       c->shear_rate == 0.0) ? 1 : 0;
        const double u = c->box[0] * 0x1.0p-32;
        FastCoef& f = h->fast;
        memset(&f, 0, sizeof(f));
        f.rc2lo = (float)((double)pt.rc2lo[0] / (u * u));
        f.rc2hi = (float)((double)pt.rc2hi[0] / (u * u));
        f.sig2u = (float)(p.sigma * p.sigma / (u * u));
        f.eps24_u = (float)(24.0 * p.eps / u);
        f.eps4 = (float)(4.0 * p.eps);
        f.eps24 = (float)(24.0 * p.eps);
        f.shift = (float)pt.d[0].shift;
        f.rc2d = pt.rc2d[0];
    }
    Dyn& dy = h->dy;
    memset(&dy, 0, sizeof(dy));
    dy.dt = c->dt;
    dy.langevin = c->integrator == MD_LANGEVIN;
    dy.seed = c->seed;
    dy.fene_K = c->fene_K;
    dy.fene_R02 = c->fene_R0 * c->fene_R0;
    dy.fene_halfKR02 = 0.5 * c->fene_K * c->fene_R0 * c->fene_R0;
    dy.fene_Kf = (float)dy.fene_K;
    dy.fene_R02f = (float)dy.fene_R02;
    dy.fene_halfKR02f = (float)dy.fene_halfKR02;
    dy.k_bend = c->k_bend;
    dy.k_bendf = (float)c->k_bend;
    dy.dpd = c->integrator == MD_DPD ? 1 : 0;
    dy.dpd_rc = (float)c->dpd_rc;
    dy.dpd_rc2 = (float)(c->dpd_rc * c->dpd_rc);
    dy.dpd_gamma = (float)c->gamma;
    dy.dpd_sigma_isdt = (float)(sqrt(2.0 * c->gamma * c->temperature) / sqrt(c->dt));
    // tables set on the handle, against the cutoffs of this configuration
    bool any_tab = false;
    for (int tp = 0; tp < MD_MAX_TYPES * MD_MAX_TYPES; ++tp) {
        pt.tabn[tp] = h->tabn[tp];
        if (h->tabn[tp] > 1) {
            any_tab = true;
            pt.tab_rmin[tp] = (float)h->tab_rmin[tp];
            pt.tab_idr[tp] = (float)((double)(h->tabn[tp] - 1) / (c->pair[tp].rc - h->tab_rmin[tp]));
        }
    }
    dy.angle_kind = c->angle_kind;
    dy.angle_K = (float)c->angle_K;
    dy.cos_phi0 = (float)cos(c->angle_phi0);
    dy.ang_n = h->ang_n;
    dy.ang_idphi = h->ang_n > 1 ? (float)((double)(h->ang_n - 1) / M_PI) : 0.f;
    dy.ang_tab = h->b.tab ? h->b.tab + (size_t)kAngleTableRow * h->g.table_points : nullptr;
    // AdResS coarse-grained tables
    const double Lmax = fmax(c->box[0], fmax(c->box[1], c->box[2]));
    for (int tp = 0; tp < MD_MAX_TYPES * MD_MAX_TYPES; ++tp) {
        pt.cgn[tp] = c->adress ? h->cgn[tp] : 0;
        if (pt.cgn[tp] > 1) {
            const double rc2 = h->cg_rc[tp] * h->cg_rc[tp], band = fixed_band(rc2, Lmax);
            pt.cg_rmin[tp] = (float)h->cg_rmin[tp];
            pt.cg_idr[tp] = (float)((double)(h->cgn[tp] - 1) / (h->cg_rc[tp] - h->cg_rmin[tp]));
            pt.cg_rc2d[tp] = rc2;
            pt.cg_rc2lo[tp] = (float)(rc2 - band);
            pt.cg_rc2hi[tp] = (float)(rc2 + band);
        }
    }
    dy.adress = c->adress;
    dy.ad_x0 = (float)c->adress_x0;
    dy.ad_dat = (float)c->adress_d_at;
    dy.ad_dhy = (float)c->adress_d_hy;
    dy.ad_k = c->adress ? (float)(M_PI / (2.0 * c->adress_d_hy)) : 0.f;
    dy.gen = (c->shear_rate != 0.0 || c->integrator == MD_DPD || any_tab || c->angle_kind != MD_ANGLE_COSINE ||
              c->adress) ? 1 : 0;
    if (dy.gen) h->use_fast = 0;
}

static void fill_masses(md_handle h, const double* mass_by_type) {
    const md_config* c = &h->cfg;
    for (int t = 0; t < MD_MAX_TYPES; ++t) {
        const double m = t < c->n_types ? mass_by_type[t] : 1.0;
        h->dy.mass[t] = m;
        h->dy.hdtm[t] = 0.5 * c->dt / m;
        h->dy.gm[t] = c->gamma * m;
        h->dy.amp[t] = c->integrator == MD_LANGEVIN ? sqrt(2.0 * c->gamma * m * c->temperature / c->dt) : 0.0;
    }
}

static StepArgs make_args(md_handle h, int mode, int tensor, double* f_out) {
    StepArgs a;
    memset(&a, 0, sizeof(a));
    a.g = h->g;
    a.b = h->b;
    a.pt = h->pt;
    a.dy = h->dy;
    a.fast = h->fast;
    a.use_fast = h->use_fast;
    a.parity = h->parity;
    a.mode = mode;
    a.tensor = tensor;
    a.f_out = f_out;
    return a;
}

static void drop_graph(md_handle h) {
    if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
    h->gexec = nullptr;
    h->graph_parity = -1;
}

// Basis constants of the surrogate descriptor: centres
// mu_k = MU0 + k (MU1 - MU0) / 31 rounded once from FP64, exp2 scale
// log2(e) / (2 w^2), cutoff r_d.
static void fill_sur_const(SurConst* c) {
    memset(c, 0, sizeof(*c));
    for (int k = 0; k < kSurNB; ++k) c->mu[k] = (float)(MD_SUR_MU0 + k * (MD_SUR_MU1 - MD_SUR_MU0) / (kSurNB - 1));
    const double w2 = MD_SUR_WIDTH * MD_SUR_WIDTH;
    c->c_exp = (float)(1.4426950408889634 / (2.0 * w2));
    c->inv_w2 = (float)(1.0 / w2);
    c->rd2 = (float)(MD_SUR_RCUT * MD_SUR_RCUT);
    c->pi_rd = (float)(M_PI / MD_SUR_RCUT);
    const double dmu = (MD_SUR_MU1 - MD_SUR_MU0) / (kSurNB - 1);
    c->dmu = (float)dmu;
    c->ratio = (float)exp2(-2.0 * (1.4426950408889634 / (2.0 * w2)) * dmu * dmu);
}

static int block_of(md_handle h) { return h->cfg.block_size ? h->cfg.block_size : kBlock; }

// Force stage: the plain fused kernel, or the surrogate's network stage
// followed by its fused pair-force + bonded + integration kernel.  BF16
// form: descriptors and the matrix-core network in one kernel, the input
// gradients passed on as BF16 rows.  FP32 form: descriptor rows, then the
// FP32 network.  *spart receives the network's energy partials (one row),
// or nullptr.
static hipError_t launch_force_stage(md_handle h, int mode, int tensor, double* f_out, const double** spart) {
    StepArgs a = make_args(h, mode, tensor, f_out);
    *spart = nullptr;
    if (h->pair_mode == MD_PAIR_PLAIN)
        return launch_step(a, h->fp64, h->single, h->bonded, block_of(h), h->stream);
    hipError_t e;
    const SurBufs& s = h->sb;
    const int bf = h->sur_prec == MD_SUR_BF16;
    if (bf) {
        if ((e = launch_sur_desc2(h->g, h->b, s, h->sc, h->parity, 1, h->stream)) != hipSuccess) return e;
    } else {
        if ((e = launch_sur_desc2(h->g, h->b, s, h->sc, h->parity, 0, h->stream)) != hipSuccess) return e;
        if ((e = launch_sur_mlp(s, s.G, h->g.n, s.a, nullptr, s.part, 0, h->step_grid, h->stream)) != hipSuccess)
            return e;
    }
    *spart = s.part;
    return launch_sur_step(a, s, h->sc, h->bonded, bf, h->stream);
}

// the finalize of a force stage: surrogate partials carry the energy only;
// the plain kernels leave one partial column per block they ran
static hipError_t launch_stage_finalize(md_handle h, int mode, const double* spart, int tensor) {
    int nb = h->step_grid;
    if (h->pair_mode == MD_PAIR_PLAIN) nb = step_launch_grid(make_args(h, mode, tensor, nullptr), h->fp64, block_of(h));
    return launch_finalize(h->b, nb, mode, spart, tensor, h->stream, 1);
}

// Enqueue one full step at the handle's current parity and advance the
// host mirrors.  Events (timing mode) bracket the three stages.
static hipError_t enqueue_step(md_handle h, const EvQuad* q) {
    hipError_t e;
    if (q) (void)hipEventRecord(q->e[0], h->stream);
    e = launch_rebuild(h->g, h->b, h->parity, h->bonded, h->stream, q ? q->e[4] : nullptr);
    if (e != hipSuccess) return e;
    if (q) (void)hipEventRecord(q->e[1], h->stream);
    const double* spart = nullptr;
    const int tensor = (h->cfg.flags & MD_CFG_VIRIAL_TENSOR) ? 1 : 0;
    e = launch_force_stage(h, MODE_STEP, tensor, nullptr, &spart);
    if (e != hipSuccess) return e;
    if (q) (void)hipEventRecord(q->e[2], h->stream);
    e = launch_stage_finalize(h, MODE_STEP, spart, tensor);
    if (e != hipSuccess) return e;
    if (q) (void)hipEventRecord(q->e[3], h->stream);
    h->parity ^= 1;
    h->host_step += 1;
    h->vel_half = 1;
    return hipSuccess;
}

static md_status build_graph(md_handle h) {
    drop_graph(h);
    hipGraph_t graph = nullptr;
    const int p0 = h->parity;
    const int64_t s0 = h->host_step;
    HIP_TRY(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e1 = enqueue_step(h, nullptr);
    hipError_t e2 = e1 == hipSuccess ? enqueue_step(h, nullptr) : e1;
    hipError_t e3 = hipStreamEndCapture(h->stream, &graph);
    // capture does not execute anything: restore the mirrors
    h->parity = p0;
    h->host_step = s0;
    if (e2 != hipSuccess || e3 != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(h, MD_ERR_HIP, std::string("graph capture failed: ") +
                                       hipGetErrorString(e2 != hipSuccess ? e2 : e3));
    }
    hipError_t e4 = hipGraphInstantiate(&h->gexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e4 != hipSuccess) {
        h->gexec = nullptr;
        return fail(h, MD_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e4));
    }
    h->graph_parity = p0;
    return MD_OK;
}

static md_status rebuild_now(md_handle h, int force) {
    if (force) HIP_TRY(h, launch_set_ctl(h->b, -1, -1, 1, 0, h->stream));
    HIP_TRY(h, launch_rebuild(h->g, h->b, h->parity, h->bonded, h->stream));
    HIP_TRY(h, launch_clear_rebuild(h->b, h->stream));
    return MD_OK;
}

static md_status status_to_code(md_handle h, uint32_t st, int32_t nl_max) {
    if (st & MD_FLAG_NL_OVERFLOW) {
        char buf[160];
        snprintf(buf, sizeof buf, "neighbour list overflow: a particle has %d neighbours, capacity %d; "
                                  "re-create with md_config.nl_capacity >= %d", nl_max, h->g.cap, (nl_max + 7) & ~7);
        return fail(h, MD_ERR_NL_OVERFLOW, buf);
    }
    if (st & MD_FLAG_BOND_BROKEN) return fail(h, MD_ERR_BOND_BROKEN, "a FENE bond reached R0");
    if (st & MD_FLAG_NONFINITE) return fail(h, MD_ERR_NONFINITE, "non-finite position or velocity");
    if (st & MD_FLAG_BAD_TYPE) return fail(h, MD_ERR_ARG, "particle type outside 0..n_types-1");
    return MD_OK;
}

static md_status read_ctl(md_handle h, DevCtl* c) {
    HIP_TRY(h, hipMemcpyAsync(c, h->b.ctl, sizeof(DevCtl), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return MD_OK;
}

static void fill_obs(md_handle h, const double* rec, md_obs* o) {
    memset(o, 0, sizeof(*o));
    o->step = (int64_t)rec[H_STEP];
    o->e_pair = rec[H_EPAIR];
    o->e_bond = rec[H_EBOND];
    o->e_angle = rec[H_EANGLE];
    o->e_kin = rec[H_EKIN];
    o->e_total = rec[H_EPAIR] + rec[H_EBOND] + rec[H_EANGLE] + rec[H_EKIN];
    o->virial = rec[H_VIR];
    for (int k = 0; k < 6; ++k) o->virial_tensor[k] = rec[H_T0 + k];
    const double V = h->g.L[0] * h->g.L[1] * h->g.L[2];
    o->pressure = (2.0 * rec[H_EKIN] + rec[H_VIR]) / (3.0 * V);
    const double n = (double)h->g.n;
    const double ndof = h->cfg.integrator == MD_LANGEVIN ? 3.0 * n : (n > 1 ? 3.0 * n - 3.0 : 3.0);
    o->temperature = 2.0 * rec[H_EKIN] / ndof;
    o->n_rebuilds = (int64_t)rec[H_NREB];
    o->status_flags = (uint32_t)rec[H_STATUS];
    o->nl_max_count = (int32_t)rec[H_NLMAX];
}

// a tabulated angle kind needs its table before forces are evaluated
static md_status need_tables(md_handle h) {
    if (h->cfg.angle_kind == MD_ANGLE_TABULATED && h->cfg.n_angles > 0 && h->ang_n < 2)
        return fail(h, MD_ERR_STATE, "MD_ANGLE_TABULATED: md_set_angle_table has not been called");
    return MD_OK;
}

static md_status upload_topology(md_handle h, const int32_t* bonds, const int32_t* angles) {
    const md_config* c = &h->cfg;
    const int64_t n = h->g.n;
    std::vector<int32_t> tcnt(n, 0), bp((size_t)h->b.maxb * n, 0);
    std::vector<int32_t> ang((size_t)h->b.maxa * n * 2, 0);
    std::vector<int32_t> nb(n, 0), na(n, 0);
    for (int64_t k = 0; k < c->n_bonds; ++k) {
        const int64_t p = bonds[2 * k], q = bonds[2 * k + 1];
        if (p < 0 || q < 0 || p >= n || q >= n || p == q) return fail(h, MD_ERR_TOPOLOGY, "bond with invalid particle id");
        if (nb[p] >= MD_MAX_BONDS_PER_PARTICLE || nb[q] >= MD_MAX_BONDS_PER_PARTICLE)
            return fail(h, MD_ERR_TOPOLOGY, "more than MD_MAX_BONDS_PER_PARTICLE bonds on a particle");
        bp[(size_t)nb[p]++ * n + p] = (int32_t)q;
        bp[(size_t)nb[q]++ * n + q] = (int32_t)p;
    }
    for (int64_t k = 0; k < c->n_angles; ++k) {
        const int64_t ids[3] = {angles[3 * k], angles[3 * k + 1], angles[3 * k + 2]};
        for (int r = 0; r < 3; ++r)
            if (ids[r] < 0 || ids[r] >= n) return fail(h, MD_ERR_TOPOLOGY, "angle with invalid particle id");
        if (ids[0] == ids[1] || ids[1] == ids[2] || ids[0] == ids[2])
            return fail(h, MD_ERR_TOPOLOGY, "angle with repeated particle");
        for (int r = 0; r < 3; ++r)
            if (na[ids[r]] >= MD_MAX_ANGLES_PER_PARTICLE)
                return fail(h, MD_ERR_TOPOLOGY, "more than MD_MAX_ANGLES_PER_PARTICLE angles on a particle");
        // per member: role and the two other members in (a, b, c) order
        const int64_t others[3][2] = {{ids[1], ids[2]}, {ids[0], ids[2]}, {ids[0], ids[1]}};
        for (int r = 0; r < 3; ++r) {
            const int64_t p = ids[r];
            const size_t slot = (size_t)na[p]++ * n + p;
            ang[2 * slot] = (int32_t)(others[r][0] | ((int64_t)r << 30));
            ang[2 * slot + 1] = (int32_t)others[r][1];
        }
    }
    for (int64_t p = 0; p < n; ++p) tcnt[p] = nb[p] | (na[p] << 8);
    HIP_TRY(h, hipMemcpyAsync(h->b.tcnt_t, tcnt.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, h->stream));
    if (h->b.maxb)
        HIP_TRY(h, hipMemcpyAsync(h->b.bp_t, bp.data(), sizeof(int32_t) * bp.size(), hipMemcpyHostToDevice, h->stream));
    if (h->b.maxa)
        HIP_TRY(h, hipMemcpyAsync(h->b.ang_t, ang.data(), sizeof(int32_t) * ang.size(), hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return MD_OK;
}

// ------------------------------------------------------------------ ABI

extern "C" {

const char* md_status_string(md_status s) {
    switch (s) {
        case MD_OK: return "MD_OK";
        case MD_ERR_ARG: return "MD_ERR_ARG";
        case MD_ERR_HIP: return "MD_ERR_HIP";
        case MD_ERR_BOX_TOO_SMALL: return "MD_ERR_BOX_TOO_SMALL";
        case MD_ERR_NL_OVERFLOW: return "MD_ERR_NL_OVERFLOW";
        case MD_ERR_BOND_BROKEN: return "MD_ERR_BOND_BROKEN";
        case MD_ERR_NONFINITE: return "MD_ERR_NONFINITE";
        case MD_ERR_STATE: return "MD_ERR_STATE";
        case MD_ERR_WORKSPACE: return "MD_ERR_WORKSPACE";
        case MD_ERR_TOPOLOGY: return "MD_ERR_TOPOLOGY";
        default: return "MD_ERR_UNKNOWN";
    }
}

const char* md_last_error(md_handle h) { return h ? h->err.c_str() : g_last_error.c_str(); }

md_status md_workspace_bytes(const md_config* cfg, size_t* bytes) {
    if (!bytes) return fail(nullptr, MD_ERR_ARG, "bytes is NULL");
    Geom g;
    std::string why;
    md_status st = plan_geom(cfg, &g, &why);
    if (st != MD_OK) return fail(nullptr, st, why);
    *bytes = carve(cfg, g, step_grid_of(g.n), nullptr, nullptr);
    return MD_OK;
}

md_status md_plan_config(const md_config* cfg, md_plan* out) {
    if (!out) return fail(nullptr, MD_ERR_ARG, "out is NULL");
    Geom g;
    std::string why;
    md_status st = plan_geom(cfg, &g, &why);
    if (st != MD_OK) return fail(nullptr, st, why);
    for (int d = 0; d < 3; ++d) out->cells[d] = g.nc[d];
    out->cell_factor = g.kc;
    out->nl_capacity = g.cap;
    out->nl_build = g.nl_tile ? MD_NL_BUILD_TILES : MD_NL_BUILD_PER_PARTICLE;
    out->list_radius = sqrt(g.rv2);
    return MD_OK;
}

// External cell arrays of a batch member (nullptr for a standalone handle).
struct CellExt {
    int32_t* ccount;
    int32_t* cstart;
};

static md_status init_core(const md_config* cfg, const double* pos, const double* vel, const int32_t* type,
                           const double* mass_by_type, const int32_t* bonds, const int32_t* angles, void* workspace,
                           size_t ws_bytes, void* stream, const CellExt* ext, md_handle* out);

md_status md_init(const md_config* cfg, const double* pos, const double* vel, const int32_t* type,
                  const double* mass_by_type, const int32_t* bonds, const int32_t* angles, void* workspace,
                  size_t ws_bytes, void* stream, md_handle* out) {
    return init_core(cfg, pos, vel, type, mass_by_type, bonds, angles, workspace, ws_bytes, stream, nullptr, out);
}

static md_status init_core(const md_config* cfg, const double* pos, const double* vel, const int32_t* type,
                           const double* mass_by_type, const int32_t* bonds, const int32_t* angles, void* workspace,
                           size_t ws_bytes, void* stream, const CellExt* ext, md_handle* out) {
    if (!out) return fail(nullptr, MD_ERR_ARG, "out is NULL");
    *out = nullptr;
    Geom g;
    std::string why;
    md_status st = plan_geom(cfg, &g, &why);
    if (st != MD_OK) return fail(nullptr, st, why);
    if (!pos || !vel || !mass_by_type || !workspace) return fail(nullptr, MD_ERR_ARG, "NULL pos/vel/mass/workspace");
    if (cfg->n_bonds > 0 && !bonds) return fail(nullptr, MD_ERR_ARG, "n_bonds > 0 but bonds is NULL");
    if (cfg->n_angles > 0 && !angles) return fail(nullptr, MD_ERR_ARG, "n_angles > 0 but angles is NULL");
    for (int t = 0; t < cfg->n_types; ++t)
        if (!(mass_by_type[t] > 0.0) || !isfinite(mass_by_type[t])) return fail(nullptr, MD_ERR_ARG, "mass must be > 0");
    const int sg = step_grid_of(g.n);
    const size_t need = carve(cfg, g, sg, nullptr, nullptr, nullptr, ext != nullptr);
    if (ws_bytes < need) return fail(nullptr, MD_ERR_WORKSPACE, "workspace smaller than md_workspace_bytes()");
    if (((uintptr_t)workspace & 255) != 0) return fail(nullptr, MD_ERR_WORKSPACE, "workspace must be 256-byte aligned");

    md_handle h = new (std::nothrow) md_handle_s();
    if (!h) return fail(nullptr, MD_ERR_ARG, "out of host memory");
    h->cfg = *cfg;
    h->g = g;
    h->stream = (hipStream_t)stream;
    h->ws = (uint8_t*)workspace;
    h->ws_bytes = ws_bytes;
    h->step_grid = sg;
    h->bonded = (cfg->n_bonds > 0 || cfg->n_angles > 0) ? 1 : 0;
    h->single = cfg->n_types == 1 ? 1 : 0;
    h->fp64 = cfg->force_precision == MD_FP64 ? 1 : 0;
    memset(&h->tacc, 0, sizeof(h->tacc));
    carve(cfg, g, sg, h->ws, &h->b, &h->sb, ext != nullptr);
    if (ext) {
        h->b.ccount = ext->ccount;
        h->b.cstart = ext->cstart;
    }
    h->has_sur = cfg->surrogate;
    fill_sur_const(&h->sc);
    fill_params(h, cfg);
    fill_masses(h, mass_by_type);

    auto bail = [&](md_status s) {
        md_destroy(h);
        return s;
    };
    md_status r;
    // control block and cell counters start at zero
    if (launch_zero_i32((int32_t*)h->b.ctl, sizeof(DevCtl) / 4, h->stream) != hipSuccess ||
        launch_zero_i32(h->b.ccount, g.ncell, h->stream) != hipSuccess ||
        launch_zero_i32(h->b.bsum, kScanBlocks * kChunkPad, h->stream) != hipSuccess ||
        launch_zero_i32(h->b.ncount, g.n, h->stream) != hipSuccess ||
        launch_zero_i32((int32_t*)h->b.partials, 2 * kNacc * part_cols(g.n), h->stream) != hipSuccess)
        return bail(fail(nullptr, MD_ERR_HIP, "kernel launch failed during init"));
    if (type) {
        if (launch_copy_i32(h->b.type_t, type, g.n, h->stream) != hipSuccess)
            return bail(fail(nullptr, MD_ERR_HIP, "type copy failed"));
    } else if (launch_zero_i32(h->b.type_t, g.n, h->stream) != hipSuccess) {
        return bail(fail(nullptr, MD_ERR_HIP, "type init failed"));
    }
    if (launch_init_load(g, h->b, 0, pos, vel, h->b.type_t, nullptr, h->stream) != hipSuccess)
        return bail(fail(nullptr, MD_ERR_HIP, "state upload failed"));
    if (h->bonded && (r = upload_topology(h, bonds, angles)) != MD_OK) {
        g_last_error = h->err;
        return bail(r);
    }
    if (launch_set_ctl(h->b, 0, 0, 1, 0, h->stream) != hipSuccess)
        return bail(fail(nullptr, MD_ERR_HIP, "control init failed"));
    if ((r = rebuild_now(h, 0)) != MD_OK) { g_last_error = h->err; return bail(r); }
    DevCtl c;
    if ((r = read_ctl(h, &c)) != MD_OK) { g_last_error = h->err; return bail(r); }
    if ((r = status_to_code(h, c.status, c.nl_max)) != MD_OK) { g_last_error = h->err; return bail(r); }
    *out = h;
    return MD_OK;
}

md_status md_init_static(const md_config* cfg, const double* pos, const double* vel, const int32_t* type,
                         const double* mass_by_type, const int32_t* bonds, const int32_t* angles, void* stream,
                         md_handle* out) {
    if (!out) return fail(nullptr, MD_ERR_ARG, "out is NULL");
    *out = nullptr;
    size_t need = 0;
    md_status st = md_workspace_bytes(cfg, &need);
    if (st != MD_OK) return st;
    if (need > (size_t)MD_STATIC_WORKSPACE_BYTES) {
        char buf[200];
        snprintf(buf, sizeof buf, "md_init_static: the system needs %zu bytes of workspace, the static workspace "
                                  "holds %zu; use md_init with a caller-owned workspace",
                 need, (size_t)MD_STATIC_WORKSPACE_BYTES);
        return fail(nullptr, MD_ERR_WORKSPACE, buf);
    }
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(nullptr, MD_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(nullptr, MD_ERR_ARG, "device index beyond the static table");
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (g_static_owner[dev])
        return fail(nullptr, MD_ERR_STATE, "md_init_static: a handle on this device's static workspace is still "
                                           "alive; md_destroy it first");
    if (!g_static_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(nullptr, MD_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_static_ptr[dev] = (uint8_t*)p;
    }
    // init_core clears every counter and flag the kernels need at zero, as it
    // does for an uninitialised caller workspace
    st = init_core(cfg, pos, vel, type, mass_by_type, bonds, angles, g_static_ptr[dev], MD_STATIC_WORKSPACE_BYTES,
                   stream, nullptr, out);
    if (st != MD_OK) return st;
    (*out)->static_dev = dev;
    g_static_owner[dev] = *out;
    return MD_OK;
}

md_status md_set_params(md_handle h, const md_config* cfg) {
    if (!h) return fail(nullptr, MD_ERR_ARG, "NULL handle");
    Geom g;
    std::string why;
    md_status st = plan_geom(cfg, &g, &why);
    if (st != MD_OK) return fail(h, st, why);
    const md_config& o = h->cfg;
    if (cfg->n_particles != o.n_particles || cfg->n_types != o.n_types || cfg->n_bonds != o.n_bonds ||
        cfg->n_angles != o.n_angles || memcmp(cfg->box, o.box, sizeof(o.box)) != 0)
        return fail(h, MD_ERR_ARG, "md_set_params cannot change N, types, box or topology");
    // The rebuild threshold (skin/2)^2 and the list radius stay those of
    // md_init.  With the skin fixed, a cutoff that fits inside the list radius
    // leaves at least the full skin between them, so the threshold stays valid;
    // a changed skin would not (a smaller effective skin under the old
    // threshold misses pairs entering the cutoff).
    if (cfg->skin != o.skin) return fail(h, MD_ERR_ARG, "md_set_params cannot change the skin fixed at md_init");
    if (cfg->table_points != o.table_points)
        return fail(h, MD_ERR_ARG, "md_set_params cannot change table_points (workspace layout)");
    if (cfg->shear_rate != o.shear_rate || ((o.shear_rate != 0.0) && cfg->dt != o.dt))
        return fail(h, MD_ERR_ARG, "md_set_params cannot change the shear rate, or the time step under shear");
    if (g.rv2 > h->g.rv2 * (1.0 + 1e-15))
        return fail(h, MD_ERR_ARG, "cutoff + skin exceeds the list radius fixed at md_init");
    double mass[MD_MAX_TYPES];
    for (int t = 0; t < MD_MAX_TYPES; ++t) mass[t] = h->dy.mass[t];
    const double old_disp2 = h->g.disp2;
    h->cfg = *cfg;
    h->fp64 = cfg->force_precision == MD_FP64 ? 1 : 0;
    fill_params(h, cfg);
    fill_masses(h, mass);
    h->g.disp2 = old_disp2;
    drop_graph(h);
    return MD_OK;
}

static md_status upload_table_row(md_handle h, int row, const std::vector<float2>& v) {
    HIP_TRY(h, hipMemcpyAsync(h->b.tab + (size_t)row * h->g.table_points, v.data(), sizeof(float2) * v.size(),
                              hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));   // the host vector goes out of scope
    return MD_OK;
}

md_status md_set_pair_table(md_handle h, int32_t ti, int32_t tj, const double* u, const double* f, int32_t npoints,
                            double rmin) {
    if (!h) return fail(nullptr, MD_ERR_ARG, "NULL handle");
    const md_config& c = h->cfg;
    if (ti < 0 || tj < 0 || ti >= c.n_types || tj >= c.n_types) return fail(h, MD_ERR_ARG, "type out of range");
    if (!u || !f || npoints < 2 || npoints > c.table_points)
        return fail(h, MD_ERR_ARG, "need u, f and 2 <= npoints <= md_config.table_points");
    const double rc = c.pair[ti * MD_MAX_TYPES + tj].rc;
    if (!(rmin >= 0.0 && rmin < rc)) return fail(h, MD_ERR_ARG, "need 0 <= rmin < rc");
    std::vector<float2> v(npoints);
    for (int k = 0; k < npoints; ++k) {
        if (!isfinite(u[k]) || !isfinite(f[k])) return fail(h, MD_ERR_ARG, "non-finite table value");
        v[k] = make_float2((float)u[k], (float)f[k]);
    }
    for (int pass = 0; pass < 2; ++pass) {
        const int tp = pass == 0 ? ti * MD_MAX_TYPES + tj : tj * MD_MAX_TYPES + ti;
        md_status r = upload_table_row(h, tp, v);
        if (r != MD_OK) return r;
        h->tabn[tp] = npoints;
        h->tab_rmin[tp] = rmin;
    }
    double mass[MD_MAX_TYPES];
    for (int t = 0; t < MD_MAX_TYPES; ++t) mass[t] = h->dy.mass[t];
    fill_params(h, &h->cfg);
    fill_masses(h, mass);
    drop_graph(h);
    return MD_OK;
}

md_status md_set_cg_table(md_handle h, int32_t ti, int32_t tj, const double* u, const double* f, int32_t npoints,
                          double rmin, double rc_cg) {
    if (!h) return fail(nullptr, MD_ERR_ARG, "NULL handle");
    const md_config& c = h->cfg;
    if (!c.adress) return fail(h, MD_ERR_ARG, "md_config.adress is 0");
    if (ti < 0 || tj < 0 || ti >= c.n_types || tj >= c.n_types) return fail(h, MD_ERR_ARG, "type out of range");
    if (!u || !f || npoints < 2 || npoints > c.table_points)
        return fail(h, MD_ERR_ARG, "need u, f and 2 <= npoints <= md_config.table_points");
    if (!(rmin >= 0.0 && rmin < rc_cg) || !isfinite(rc_cg)) return fail(h, MD_ERR_ARG, "need 0 <= rmin < rc_cg");
    if ((rc_cg + c.skin) * (rc_cg + c.skin) > h->g.rv2 * (1.0 + 1e-12))
        return fail(h, MD_ERR_ARG, "rc_cg + skin exceeds the list radius; raise md_config.list_cutoff");
    std::vector<float2> v(npoints);
    for (int k = 0; k < npoints; ++k) {
        if (!isfinite(u[k]) || !isfinite(f[k])) return fail(h, MD_ERR_ARG, "non-finite table value");
        v[k] = make_float2((float)u[k], (float)f[k]);
    }
    for (int pass = 0; pass < 2; ++pass) {
        const int tp = pass == 0 ? ti * MD_MAX_TYPES + tj : tj * MD_MAX_TYPES + ti;
        md_status r = upload_table_row(h, kCgTableRow + tp, v);
        if (r != MD_OK) return r;
        h->cgn[tp] = npoints;
        h->cg_rmin[tp] = rmin;
        h->cg_rc[tp] = rc_cg;
    }
    double mass[MD_MAX_TYPES];
    for (int t = 0; t < MD_MAX_TYPES; ++t) mass[t] = h->dy.mass[t];
    fill_params(h, &h->cfg);
    fill_masses(h, mass);
    drop_graph(h);
    return MD_OK;
}

md_status md_set_angle_subens(md_handle h, int32_t ntables, const double* u, const double* dudphi,
                              const double* weights, int32_t npoints) {
    if (!h) return fail(nullptr, MD_ERR_ARG, "NULL handle");
    if (ntables < 1 || !u || !dudphi || !weights || npoints < 2 || npoints > h->cfg.table_points)
        return fail(h, MD_ERR_ARG, "need ntables >= 1, u, dudphi, weights and 2 <= npoints <= table_points");
    std::vector<float2> v(npoints);
    for (int k = 0; k < npoints; ++k) {
        double su = 0.0, sg = 0.0;
        for (int m = 0; m < ntables; ++m) {
            su += weights[m] * u[(size_t)m * npoints + k];
            sg += weights[m] * dudphi[(size_t)m * npoints + k];
        }
        if (!isfinite(su) || !isfinite(sg)) return fail(h, MD_ERR_ARG, "non-finite table value");
        v[k] = make_float2((float)su, (float)sg);
    }
    md_status r = upload_table_row(h, kAngleTableRow, v);
    if (r != MD_OK) return r;
    h->ang_n = npoints;
    double mass[MD_MAX_TYPES];
    for (int t = 0; t < MD_MAX_TYPES; ++t) mass[t] = h->dy.mass[t];
    fill_params(h, &h->cfg);
    fill_masses(h, mass);
    drop_graph(h);
    return MD_OK;
}

md_status md_set_angle_table(md_handle h, const double* u, const double* dudphi, int32_t npoints) {
    const double one = 1.0;
    return md_set_angle_subens(h, 1, u, dudphi, &one, npoints);
}

md_status md_build_neighbors(md_handle h) {
    if (!h) return fail(nullptr, MD_ERR_ARG, "NULL handle");
    return rebuild_now(h, 1);
}

md_status md_forces(md_handle h, double* f_out) {
    if (!h) return fail(nullptr, MD_ERR_ARG, "NULL handle");
    if (need_tables(h) != MD_OK) return MD_ERR_STATE;
    md_status r = rebuild_now(h, 0);
    if (r != MD_OK) return r;
    const double* spart = nullptr;
    HIP_TRY(h, launch_force_stage(h, MODE_FORCES, 1, f_out, &spart));
    HIP_TRY(h, launch_stage_finalize(h, MODE_FORCES, spart, 1));
    return MD_OK;
}

md_status md_step(md_handle h, int64_t nsteps) {
    if (!h) return fail(nullptr, MD_ERR_ARG, "NULL handle");
    if (nsteps < 0) return fail(h, MD_ERR_ARG, "nsteps < 0");
    if (need_tables(h) != MD_OK) return MD_ERR_STATE;
    const bool use_graph = !(h->cfg.flags & MD_CFG_NO_GRAPH) && !h->timing && h->stream != nullptr;
    int64_t left = nsteps;
    while (left > 0) {
        if (use_graph && left >= 2) {
            if (h->graph_parity != h->parity) {
                if (h->gexec && h->graph_parity >= 0) {
                    // single eager step to align the parity with the graph
                    HIP_TRY(h, enqueue_step(h, nullptr));
                    --left;
                    continue;
                }
                md_status r = build_graph(h);
                if (r != MD_OK) return r;
            }
            HIP_TRY(h, hipGraphLaunch(h->gexec, h->stream));
            h->parity ^= 0;  // two steps: parity unchanged
            h->host_step += 2;
            h->vel_half = 1;
            left -= 2;
            continue;
        }
        EvQuad q;
        const EvQuad* qp = nullptr;
        if (h->timing) {
            if (!h->ev_free.empty()) {
                q = h->ev_free.back();
                h->ev_free.pop_back();
            } else {
                for (int k = 0; k < kStepEvents; ++k) HIP_TRY(h, hipEventCreate(&q.e[k]));
            }
            h->ev_pending.push_back(q);
            qp = &h->ev_pending.back();
        }
        HIP_TRY(h, enqueue_step(h, qp));
        --left;
    }
    return MD_OK;
}

md_status md_observables(md_handle h, md_obs* out) {
    if (!h || !out) return fail(h, MD_ERR_ARG, "NULL handle or output");
    if (need_tables(h) != MD_OK) return MD_ERR_STATE;
    md_status r = rebuild_now(h, 0);
    if (r != MD_OK) return r;
    const double* spart = nullptr;
    HIP_TRY(h, launch_force_stage(h, MODE_OBSERVE, 1, nullptr, &spart));
    HIP_TRY(h, launch_stage_finalize(h, MODE_OBSERVE, spart, 1));
    double rec[kHistRec];
    HIP_TRY(h, hipMemcpyAsync(rec, h->b.cur, sizeof(rec), hipMemcpyDeviceToHost, h->stream));
    DevCtl c;
    if ((r = read_ctl(h, &c)) != MD_OK) return r;
    fill_obs(h, rec, out);
    out->status_flags = c.status;
    return status_to_code(h, c.status, c.nl_max);
}

md_status md_history(md_handle h, md_obs* out, int64_t max, int64_t* n) {
    if (!h || !n || (max > 0 && !out)) return fail(h, MD_ERR_ARG, "NULL argument");
    DevCtl c;
    md_status r = read_ctl(h, &c);
    if (r != MD_OK) return r;
    const int64_t end = c.step;
    int64_t first = h->hist_next;
    if (end - first > MD_HISTORY_CAPACITY) first = end - MD_HISTORY_CAPACITY;
    int64_t count = end - first;
    if (count > max) count = max;
    if (count < 0) count = 0;
    std::vector<double> ring((size_t)kHistRec * MD_HISTORY_CAPACITY);
    if (count > 0) {
        HIP_TRY(h, hipMemcpyAsync(ring.data(), h->b.hist, sizeof(double) * ring.size(), hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
    }
    for (int64_t k = 0; k < count; ++k) {
        const int64_t s = first + k;
        fill_obs(h, &ring[(size_t)(s % MD_HISTORY_CAPACITY) * kHistRec], &out[k]);
    }
    h->hist_next = first + count;
    *n = count;
    return MD_OK;
}

md_status md_get_state(md_handle h, double* pos, double* vel, int32_t* image, double* pos_build, int64_t* step,
                       int32_t* vel_half) {
    if (!h) return fail(nullptr, MD_ERR_ARG, "NULL handle");
    md_status r = rebuild_now(h, 0);
    if (r != MD_OK) return r;
    HIP_TRY(h, launch_get_state(h->g, h->b, h->parity, pos, vel, image, pos_build, h->stream));
    if (step) *step = h->host_step;
    if (vel_half) *vel_half = h->vel_half;
    return MD_OK;
}

md_status md_set_state(md_handle h, const double* pos, const double* vel, const int32_t* image,
                       const double* pos_build, int64_t step, int32_t vel_half) {
    if (!h) return fail(nullptr, MD_ERR_ARG, "NULL handle");
    if (!pos || !vel) return fail(h, MD_ERR_ARG, "NULL pos or vel");
    if (step < 0 || (vel_half != 0 && vel_half != 1)) return fail(h, MD_ERR_ARG, "bad step or vel_half");
    h->parity = 0;
    drop_graph(h);
    HIP_TRY(h, launch_init_load(h->g, h->b, 0, pos_build ? pos_build : pos, vel, h->b.type_t, image, h->stream));
    HIP_TRY(h, launch_set_ctl(h->b, step, vel_half, 1, 1, h->stream));
    md_status r = rebuild_now(h, 0);
    if (r != MD_OK) return r;
    if (pos_build) HIP_TRY(h, launch_overwrite_state(h->g, h->b, 0, pos, vel, image, h->stream));
    h->host_step = step;
    h->vel_half = vel_half;
    h->hist_next = step;
    return MD_OK;
}

md_status md_get_neighbors(md_handle h, int32_t* count, int32_t* idx, int32_t cap) {
    if (!h || !count || !idx || cap < 1) return fail(h, MD_ERR_ARG, "bad argument");
    md_status r = rebuild_now(h, 0);
    if (r != MD_OK) return r;
    HIP_TRY(h, launch_get_neighbors(h->g, h->b, count, idx, cap, h->stream));
    DevCtl c;
    if ((r = read_ctl(h, &c)) != MD_OK) return r;
    if ((r = status_to_code(h, c.status, c.nl_max)) != MD_OK) return r;
    if (c.nl_max > cap) return fail(h, MD_ERR_NL_OVERFLOW, "cap smaller than the longest neighbour row");
    return MD_OK;
}

md_status md_status_check(md_handle h) {
    if (!h) return fail(nullptr, MD_ERR_ARG, "NULL handle");
    DevCtl c;
    md_status r = read_ctl(h, &c);
    if (r != MD_OK) return r;
    return status_to_code(h, c.status, c.nl_max);
}

md_status md_timing_enable(md_handle h, int32_t enable) {
    if (!h) return fail(nullptr, MD_ERR_ARG, "NULL handle");
    h->timing = enable != 0;
    return MD_OK;
}

md_status md_timing_read(md_handle h, md_timing* out) {
    if (!h || !out) return fail(h, MD_ERR_ARG, "NULL argument");
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    for (const EvQuad& q : h->ev_pending) {
        float a = 0, b = 0, c = 0, d = 0;
        HIP_TRY(h, hipEventElapsedTime(&a, q.e[0], q.e[1]));
        HIP_TRY(h, hipEventElapsedTime(&b, q.e[1], q.e[2]));
        HIP_TRY(h, hipEventElapsedTime(&c, q.e[2], q.e[3]));
        HIP_TRY(h, hipEventElapsedTime(&d, q.e[0], q.e[4]));
        h->tacc.n_rebuild += 1;
        h->tacc.ms_rebuild += a;
        h->tacc.ms_bin_sort += d;
        h->tacc.n_step_kernels += 1;
        h->tacc.ms_step_kernels += b;
        h->tacc.n_finalize += 1;
        h->tacc.ms_finalize += c;
        h->ev_free.push_back(q);
    }
    h->ev_pending.clear();
    *out = h->tacc;
    memset(&h->tacc, 0, sizeof(h->tacc));
    return MD_OK;
}

// ------------------------------------------------------------------ surrogate ABI

static md_status need_sur(md_handle h) {
    if (!h) return fail(nullptr, MD_ERR_ARG, "NULL handle");
    if (!h->has_sur) return fail(h, MD_ERR_ARG, "created without md_config.surrogate = 1");
    return MD_OK;
}

md_status md_sur_set(md_handle h, const float* theta, const float* g_mean, const float* g_istd, int32_t precision) {
    md_status r = need_sur(h);
    if (r != MD_OK) return r;
    if (!theta || !g_mean || !g_istd) return fail(h, MD_ERR_ARG, "NULL theta / mean / istd");
    if (precision != MD_SUR_FP32 && precision != MD_SUR_BF16) return fail(h, MD_ERR_ARG, "bad precision");
    const SurBufs& s = h->sb;
    HIP_TRY(h, hipMemcpyAsync(s.w, theta, sizeof(float) * kSurNP, hipMemcpyDeviceToDevice, h->stream));
    HIP_TRY(h, hipMemcpyAsync(s.gmean, g_mean, sizeof(float) * kSurNB, hipMemcpyDeviceToDevice, h->stream));
    HIP_TRY(h, hipMemcpyAsync(s.gistd, g_istd, sizeof(float) * kSurNB, hipMemcpyDeviceToDevice, h->stream));
    HIP_TRY(h, launch_zero_i32((int32_t*)s.m1, kSurNPpad, h->stream));
    HIP_TRY(h, launch_zero_i32((int32_t*)s.m2, kSurNPpad, h->stream));
    HIP_TRY(h, launch_zero_i32((int32_t*)s.grad, kSurNPpad, h->stream));
    HIP_TRY(h, launch_sur_prepare(s, h->stream));
    h->sur_prec = precision;
    h->sur_loaded = 1;
    drop_graph(h);
    return MD_OK;
}

md_status md_sur_get(md_handle h, float* theta) {
    md_status r = need_sur(h);
    if (r != MD_OK) return r;
    if (!theta) return fail(h, MD_ERR_ARG, "NULL theta");
    HIP_TRY(h, hipMemcpyAsync(theta, h->sb.w, sizeof(float) * kSurNP, hipMemcpyDeviceToDevice, h->stream));
    return MD_OK;
}

md_status md_set_pair_mode(md_handle h, int32_t mode) {
    if (!h) return fail(nullptr, MD_ERR_ARG, "NULL handle");
    if (mode == MD_PAIR_PLAIN) {
        h->pair_mode = mode;
        drop_graph(h);
        return MD_OK;
    }
    if (mode != MD_PAIR_SURROGATE) return fail(h, MD_ERR_ARG, "bad pair mode");
    if (h->g.le || h->dy.dpd) return fail(h, MD_ERR_ARG, "the surrogate runs without DPD and shear");
    md_status r = need_sur(h);
    if (r != MD_OK) return r;
    if (!h->sur_loaded) return fail(h, MD_ERR_ARG, "md_sur_set has not been called");
    if (sqrt(h->g.rv2) - h->cfg.skin < MD_SUR_RCUT * (1.0 - 1e-12))
        return fail(h, MD_ERR_ARG, "list radius minus skin is below the descriptor cutoff; set md_config.list_cutoff");
    h->pair_mode = mode;
    drop_graph(h);
    return MD_OK;
}

md_status md_sur_descriptors(md_handle h, float* G) {
    md_status r = need_sur(h);
    if (r != MD_OK) return r;
    if (!G) return fail(h, MD_ERR_ARG, "NULL output");
    if (sqrt(h->g.rv2) - h->cfg.skin < MD_SUR_RCUT * (1.0 - 1e-12))
        return fail(h, MD_ERR_ARG, "list radius minus skin is below the descriptor cutoff");
    if ((r = rebuild_now(h, 0)) != MD_OK) return r;
    HIP_TRY(h, launch_sur_desc2(h->g, h->b, h->sb, h->sc, h->parity, 0, h->stream));
    HIP_TRY(h, launch_sur_to_tag(h->g, h->b, h->sb.G, G, h->stream));
    return MD_OK;
}

md_status md_sur_desc_stats(md_handle h, const double* frames, int32_t nf, float* g_mean, float* g_istd) {
    md_status r = need_sur(h);
    if (r != MD_OK) return r;
    if (!frames || nf < 1) return fail(h, MD_ERR_ARG, "bad frames");
    if (!g_mean || !g_istd) return fail(h, MD_ERR_ARG, "NULL output");
    if (sqrt(h->g.rv2) - h->cfg.skin < MD_SUR_RCUT * (1.0 - 1e-12))
        return fail(h, MD_ERR_ARG, "list radius minus skin is below the descriptor cutoff");
    const int64_t n = h->g.n;
    drop_graph(h);
    h->parity = 0;
    for (int32_t f = 0; f < nf; ++f) {
        const double* pos = frames + (size_t)f * 3 * n;
        HIP_TRY(h, launch_init_load(h->g, h->b, 0, pos, nullptr, h->b.type_t, nullptr, h->stream));
        HIP_TRY(h, launch_set_ctl(h->b, 0, 0, 1, 1, h->stream));
        if ((r = rebuild_now(h, 0)) != MD_OK) return r;
        HIP_TRY(h, launch_sur_desc2(h->g, h->b, h->sb, h->sc, 0, 0, h->stream));
        HIP_TRY(h, launch_sur_moments(h->sb, n, f > 0, h->stream));
    }
    HIP_TRY(h, launch_sur_moments_final(h->sb, (double)n * (double)nf, MD_SUR_VAR_FLOOR, g_mean, g_istd, h->stream));
    h->host_step = 0;
    h->vel_half = 0;
    h->hist_next = 0;
    return MD_OK;
}

md_status md_sur_mlp_eval(md_handle h, const float* G, int64_t P, float* e, float* dedg) {
    md_status r = need_sur(h);
    if (r != MD_OK) return r;
    if (!h->sur_loaded) return fail(h, MD_ERR_ARG, "md_sur_set has not been called");
    if (P < 0 || (P > 0 && (!G || !dedg))) return fail(h, MD_ERR_ARG, "bad arguments");
    if (P == 0) return MD_OK;
    if (h->sur_prec == MD_SUR_BF16) {
        HIP_TRY(h, launch_sur_mlp16(h->sb, G, P, dedg, e, h->stream));
        return MD_OK;
    }
    const int64_t tiles = (P + 63) / 64;
    const int grid = (int)(tiles < 4096 ? tiles : 4096);
    HIP_TRY(h, launch_sur_mlp(h->sb, G, P, dedg, e, nullptr, 0, grid, h->stream));
    return MD_OK;
}

md_status md_sur_pair_forces(md_handle h, const float* dedg, double* f_out) {
    md_status r = need_sur(h);
    if (r != MD_OK) return r;
    if (!dedg || !f_out) return fail(h, MD_ERR_ARG, "NULL argument");
    if (sqrt(h->g.rv2) - h->cfg.skin < MD_SUR_RCUT * (1.0 - 1e-12))
        return fail(h, MD_ERR_ARG, "list radius minus skin is below the descriptor cutoff");
    if ((r = rebuild_now(h, 0)) != MD_OK) return r;
    const SurBufs& s = h->sb;
    HIP_TRY(h, launch_sur_from_tag(h->g, h->b, dedg, s.a, h->stream));
    HIP_TRY(h, launch_sur_force(h->g, h->b, s, h->sc, h->parity, nullptr, 0.0, 0, h->step_grid, h->stream));
    HIP_TRY(h, launch_sur_f_to_tag(h->g, h->b, s.f, f_out, h->stream));
    return MD_OK;
}

md_status md_sur_loss_grad(md_handle h, const double* frames, const double* f_ref, int32_t nf, float* grad,
                           double* loss) {
    md_status r = need_sur(h);
    if (r != MD_OK) return r;
    if (!h->sur_loaded) return fail(h, MD_ERR_ARG, "md_sur_set has not been called");
    if (!frames || !f_ref || nf < 1) return fail(h, MD_ERR_ARG, "bad frames");
    if (sqrt(h->g.rv2) - h->cfg.skin < MD_SUR_RCUT * (1.0 - 1e-12))
        return fail(h, MD_ERR_ARG, "list radius minus skin is below the descriptor cutoff");
    const int64_t n = h->g.n;
    const double two_over_m = 2.0 / (3.0 * (double)n * (double)nf);
    const SurBufs& s = h->sb;
    const int bf = h->sur_prec == MD_SUR_BF16;
    drop_graph(h);
    h->parity = 0;
    for (int32_t f = 0; f < nf; ++f) {
        const double* pos = frames + (size_t)f * 3 * n;
        HIP_TRY(h, launch_init_load(h->g, h->b, 0, pos, nullptr, h->b.type_t, nullptr, h->stream));
        HIP_TRY(h, launch_set_ctl(h->b, 0, 0, 1, 1, h->stream));
        if ((r = rebuild_now(h, 0)) != MD_OK) return r;
        HIP_TRY(h, launch_sur_desc2(h->g, h->b, s, h->sc, 0, 0, h->stream));
        HIP_TRY(h, launch_sur_mlp(s, s.G, n, s.a, nullptr, nullptr, bf, h->step_grid, h->stream));
        HIP_TRY(h, launch_sur_force(h->g, h->b, s, h->sc, 0, f_ref + (size_t)f * 3 * n, two_over_m, 0, h->step_grid,
                                    h->stream));
        HIP_TRY(h, launch_sur_loss_reduce(s, h->step_grid, f > 0, h->stream));
        HIP_TRY(h, launch_sur_u(h->g, h->b, s, h->sc, 0, h->step_grid, h->stream));
        HIP_TRY(h, launch_sur_bwd2(s, n, bf, h->stream));
        HIP_TRY(h, launch_sur_grad_reduce(s, sur_bwd2_grid(n), f > 0, h->stream));
    }
    h->host_step = 0;
    h->vel_half = 0;
    h->hist_next = 0;
    if (grad) HIP_TRY(h, hipMemcpyAsync(grad, s.grad, sizeof(float) * kSurNP, hipMemcpyDeviceToDevice, h->stream));
    if (loss) {
        double l = 0.0;
        HIP_TRY(h, hipMemcpyAsync(&l, s.loss, sizeof(double), hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        *loss = l / (3.0 * (double)n * (double)nf);
        DevCtl c;
        if ((r = read_ctl(h, &c)) != MD_OK) return r;
        if ((r = status_to_code(h, c.status, c.nl_max)) != MD_OK) return r;
    }
    return MD_OK;
}

md_status md_sur_adam(md_handle h, int64_t t, double lr, double beta1, double beta2, double eps) {
    md_status r = need_sur(h);
    if (r != MD_OK) return r;
    if (!h->sur_loaded) return fail(h, MD_ERR_ARG, "md_sur_set has not been called");
    if (t < 1 || !(lr >= 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0))
        return fail(h, MD_ERR_ARG, "bad Adam parameters");
    HIP_TRY(h, launch_sur_adam(h->sb, t, (float)lr, (float)beta1, (float)beta2, (float)eps, h->stream));
    HIP_TRY(h, launch_sur_prepare(h->sb, h->stream));
    return MD_OK;
}

// ------------------------------------------------------------------ batches

}  // extern "C"

struct md_batch_s {
    int nsys = 0;
    std::vector<md_handle> sys;
    hipStream_t stream = nullptr;
    BatchCells bc;
    SysEntry* tabs[2][2] = {};      // device [nsys] per (mode: step / observe, parity)
    int32_t* tile_sys = nullptr;    // device [ntiles]
    int64_t ntiles = 0;
    double* obs = nullptr;          // device [nsys][kHistRec]
    int parity = 0;
    int64_t host_step = 0;
    hipGraphExec_t gexec = nullptr;
    int graph_parity = -1;
    std::string err;
    bool timing = false;
    std::vector<EvQuad> ev_free, ev_pending;
    md_timing tacc;
};

namespace {

struct BatchPlan {
    std::vector<Geom> g;
    std::vector<size_t> ws_off, ws_size;
    std::vector<int64_t> c_off, tile0;
    std::vector<int32_t> ntiles;
    int64_t ncell_total = 0, ntiles_total = 0, n_total = 0;
    size_t off_ctl = 0, off_count = 0, off_start = 0, off_bsum = 0, off_coff = 0, off_base = 0, off_tiles = 0,
           off_tab = 0, off_obs = 0, total = 0;
};

md_status plan_batch(const md_config* cfgs, int32_t nsys, BatchPlan* p, std::string* why) {
    if (!cfgs || nsys < 1) {
        *why = "need at least one system";
        return MD_ERR_ARG;
    }
    p->g.resize(nsys);
    p->ws_off.resize(nsys);
    p->ws_size.resize(nsys);
    p->c_off.resize(nsys + 1);
    p->tile0.resize(nsys);
    p->ntiles.resize(nsys);
    for (int s = 0; s < nsys; ++s) {
        const md_config* c = &cfgs[s];
        md_status st = plan_geom(c, &p->g[s], why);
        if (st != MD_OK) {
            *why = "system " + std::to_string(s) + ": " + *why;
            return st;
        }
        const md_pair_params& pp = c->pair[0];
        if (c->n_types != 1 || c->force_precision != MD_FP32 || pp.caprad > 0.0 || c->box[0] != c->box[1] ||
            c->box[1] != c->box[2] || c->surrogate || c->integrator == MD_DPD || c->shear_rate != 0.0 ||
            c->table_points != 0 || c->angle_kind != MD_ANGLE_COSINE || c->adress) {
            *why = "system " + std::to_string(s) +
                   ": batch members need one particle type, FP32 pair math, a cubic box, no capping radius, "
                   "no surrogate, no DPD, no shear, no tables, the cosine angle and no AdResS";
            return MD_ERR_ARG;
        }
        if (c->n_particles > (int64_t)kBlock * 1024) {
            *why = "system " + std::to_string(s) + ": batch members hold at most 262144 particles";
            return MD_ERR_ARG;
        }
        const int64_t nt = (c->n_particles + kBlock - 1) / kBlock;
        p->ntiles[s] = (int32_t)nt;
        p->tile0[s] = p->ntiles_total;
        p->ntiles_total += nt;
        p->n_total += c->n_particles;
        p->c_off[s] = p->ncell_total;
        p->ncell_total += p->g[s].ncell + 1;   // each system's cells and its end sentinel
        p->ws_size[s] = carve(c, p->g[s], (int)nt, nullptr, nullptr, nullptr, true);
    }
    p->c_off[nsys] = p->ncell_total;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align256(bytes);
        return o;
    };
    p->off_ctl = take(sizeof(DevCtl));
    p->off_count = take(sizeof(int32_t) * (p->ncell_total + 1));
    p->off_start = take(sizeof(int32_t) * (p->ncell_total + 1));
    p->off_bsum = take(sizeof(int32_t) * kScanBlocks);
    p->off_coff = take(sizeof(int64_t) * (nsys + 1));
    p->off_base = take(sizeof(int32_t) * nsys);
    p->off_tiles = take(sizeof(int32_t) * p->ntiles_total);
    p->off_tab = take(sizeof(SysEntry) * nsys * 4);
    p->off_obs = take(sizeof(double) * kHistRec * nsys);
    for (int s = 0; s < nsys; ++s) p->ws_off[s] = take(p->ws_size[s]);
    p->total = off;
    return MD_OK;
}

md_status bfail(md_batch b, md_status st, const std::string& msg) {
    if (b) b->err = msg;
    g_last_error = msg;
    return st;
}

#define BHIP_TRY(b, call)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return bfail((b), MD_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

hipError_t batch_enqueue_step(md_batch b, const EvQuad* q = nullptr) {
    if (q) (void)hipEventRecord(q->e[0], b->stream);
    hipError_t e = launch_batch_rebuild(b->bc, b->tabs[0][b->parity], b->tile_sys, b->ntiles, b->parity, b->stream,
                                        q ? q->e[4] : nullptr);
    if (e != hipSuccess) return e;
    if (q) (void)hipEventRecord(q->e[1], b->stream);
    e = launch_batch_step(b->tabs[0][b->parity], b->tile_sys, b->ntiles, b->parity, MODE_STEP, 0, b->stream);
    if (e != hipSuccess) return e;
    if (q) (void)hipEventRecord(q->e[2], b->stream);
    e = launch_batch_finalize(b->tabs[0][b->parity], b->nsys, MODE_STEP, b->stream);
    if (e != hipSuccess) return e;
    if (q) (void)hipEventRecord(q->e[3], b->stream);
    b->parity ^= 1;
    b->host_step += 1;
    return hipSuccess;
}

void batch_sync_members(md_batch b) {
    for (md_handle h : b->sys) {
        h->parity = b->parity;
        h->host_step = b->host_step;
        h->vel_half = 1;
        drop_graph(h);
    }
}

void batch_drop_graph(md_batch b) {
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    b->gexec = nullptr;
    b->graph_parity = -1;
}

}  // namespace

extern "C" {

md_status md_batch_workspace_bytes(const md_config* cfgs, int32_t nsys, size_t* bytes) {
    if (!bytes) return fail(nullptr, MD_ERR_ARG, "bytes is NULL");
    BatchPlan p;
    std::string why;
    md_status st = plan_batch(cfgs, nsys, &p, &why);
    if (st != MD_OK) return fail(nullptr, st, why);
    *bytes = p.total;
    return MD_OK;
}

md_status md_batch_destroy(md_batch b) {
    if (!b) return MD_OK;
    (void)hipStreamSynchronize(b->stream);
    batch_drop_graph(b);
    for (auto& q : b->ev_free)
        for (int k = 0; k < kStepEvents; ++k) (void)hipEventDestroy(q.e[k]);
    for (auto& q : b->ev_pending)
        for (int k = 0; k < kStepEvents; ++k) (void)hipEventDestroy(q.e[k]);
    for (md_handle h : b->sys) md_destroy(h);
    delete b;
    return MD_OK;
}

md_status md_batch_init(const md_config* cfgs, int32_t nsys, const double* const* pos, const double* const* vel,
                        const double* const* mass_by_type, const int32_t* const* bonds,
                        const int32_t* const* angles, void* workspace, size_t ws_bytes, void* stream,
                        md_batch* out) {
    if (!out) return fail(nullptr, MD_ERR_ARG, "out is NULL");
    *out = nullptr;
    BatchPlan p;
    std::string why;
    md_status st = plan_batch(cfgs, nsys, &p, &why);
    if (st != MD_OK) return fail(nullptr, st, why);
    if (!pos || !vel || !mass_by_type || !workspace) return fail(nullptr, MD_ERR_ARG, "NULL argument");
    if (ws_bytes < p.total) return fail(nullptr, MD_ERR_WORKSPACE, "workspace smaller than md_batch_workspace_bytes()");
    if (((uintptr_t)workspace & 255) != 0) return fail(nullptr, MD_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    md_batch b = new (std::nothrow) md_batch_s();
    if (!b) return fail(nullptr, MD_ERR_ARG, "out of host memory");
    memset(&b->tacc, 0, sizeof(b->tacc));
    b->nsys = nsys;
    b->stream = (hipStream_t)stream;
    uint8_t* ws = (uint8_t*)workspace;
    int32_t* gcount = (int32_t*)(ws + p.off_count);
    int32_t* gstart = (int32_t*)(ws + p.off_start);
    for (int m = 0; m < 2; ++m)
        for (int q = 0; q < 2; ++q) b->tabs[m][q] = (SysEntry*)(ws + p.off_tab) + (size_t)(2 * m + q) * nsys;
    b->tile_sys = (int32_t*)(ws + p.off_tiles);
    b->ntiles = p.ntiles_total;
    b->obs = (double*)(ws + p.off_obs);
    memset(&b->bc, 0, sizeof(b->bc));
    b->bc.gg.ncell = p.ncell_total;
    b->bc.gg.n = p.n_total;
    b->bc.gb.ctl = (DevCtl*)(ws + p.off_ctl);
    b->bc.gb.ccount = gcount;
    b->bc.gb.cstart = gstart;
    b->bc.gb.bsum = (int32_t*)(ws + p.off_bsum);
    b->bc.tab = b->tabs[0][0];
    b->bc.c_off = (int64_t*)(ws + p.off_coff);
    b->bc.base = (int32_t*)(ws + p.off_base);
    b->bc.nsys = nsys;
    auto bail = [&](md_status r) {
        md_batch_destroy(b);
        return r;
    };
    if (launch_zero_i32((int32_t*)b->bc.gb.ctl, sizeof(DevCtl) / 4, b->stream) != hipSuccess ||
        launch_zero_i32(gcount, p.ncell_total + 1, b->stream) != hipSuccess)
        return bail(fail(nullptr, MD_ERR_HIP, "batch init: kernel launch failed"));
    for (int s = 0; s < nsys; ++s) {
        CellExt ext{gcount + p.c_off[s], gstart + p.c_off[s]};
        md_handle h = nullptr;
        md_status r = init_core(&cfgs[s], pos[s], vel[s], nullptr, mass_by_type[s], bonds ? bonds[s] : nullptr,
                                angles ? angles[s] : nullptr, ws + p.ws_off[s], p.ws_size[s], stream, &ext, &h);
        if (r != MD_OK) {
            std::string m = "system " + std::to_string(s) + ": " + g_last_error;
            md_batch_destroy(b);
            return fail(nullptr, r, m);
        }
        b->sys.push_back(h);
    }
    std::vector<SysEntry> tab((size_t)4 * nsys);
    std::vector<int32_t> tiles(p.ntiles_total);
    for (int s = 0; s < nsys; ++s) {
        md_handle h = b->sys[s];
        if (!h->use_fast) return bail(fail(nullptr, MD_ERR_ARG, "batch member outside the FP32 fast path"));
        for (int m = 0; m < 2; ++m)
            for (int q = 0; q < 2; ++q) {
                SysEntry& e = tab[(size_t)(2 * m + q) * nsys + s];
                memset(&e, 0, sizeof(SysEntry));
                e.a = make_args(h, m == 0 ? MODE_STEP : MODE_OBSERVE, m, nullptr);
                e.a.parity = q;
                e.a.use_fast = 1;
                e.tile0 = p.tile0[s];
                e.ntiles = p.ntiles[s];
                e.bonded = h->bonded;
                e.c_off = p.c_off[s];
            }
        for (int64_t t = 0; t < p.ntiles[s]; ++t) tiles[p.tile0[s] + t] = s;
    }
    if (hipMemcpyAsync(b->tabs[0][0], tab.data(), sizeof(SysEntry) * tab.size(), hipMemcpyHostToDevice,
                       b->stream) != hipSuccess ||
        hipMemcpyAsync(b->tile_sys, tiles.data(), sizeof(int32_t) * tiles.size(), hipMemcpyHostToDevice,
                       b->stream) != hipSuccess ||
        hipMemcpyAsync(b->bc.c_off, p.c_off.data(), sizeof(int64_t) * (nsys + 1), hipMemcpyHostToDevice,
                       b->stream) != hipSuccess ||
        hipStreamSynchronize(b->stream) != hipSuccess)
        return bail(fail(nullptr, MD_ERR_HIP, "batch table upload failed"));
    *out = b;
    return MD_OK;
}

md_status md_batch_step(md_batch b, int64_t nsteps) {
    if (!b) return fail(nullptr, MD_ERR_ARG, "NULL batch");
    if (nsteps < 0) return bfail(b, MD_ERR_ARG, "nsteps < 0");
    int64_t left = nsteps;
    while (left > 0) {
        if (b->timing) {
            EvQuad q;
            if (!b->ev_free.empty()) {
                q = b->ev_free.back();
                b->ev_free.pop_back();
            } else {
                for (int k = 0; k < kStepEvents; ++k) BHIP_TRY(b, hipEventCreate(&q.e[k]));
            }
            b->ev_pending.push_back(q);
            BHIP_TRY(b, batch_enqueue_step(b, &b->ev_pending.back()));
            --left;
            continue;
        }
        if (left >= 2 && b->stream != nullptr) {
            if (b->graph_parity != b->parity) {
                batch_drop_graph(b);
                hipGraph_t graph = nullptr;
                const int p0 = b->parity;
                const int64_t s0 = b->host_step;
                BHIP_TRY(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
                hipError_t e1 = batch_enqueue_step(b);
                hipError_t e2 = e1 == hipSuccess ? batch_enqueue_step(b) : e1;
                hipError_t e3 = hipStreamEndCapture(b->stream, &graph);
                b->parity = p0;
                b->host_step = s0;
                if (e2 != hipSuccess || e3 != hipSuccess) {
                    if (graph) (void)hipGraphDestroy(graph);
                    return bfail(b, MD_ERR_HIP, "batch graph capture failed");
                }
                hipError_t e4 = hipGraphInstantiate(&b->gexec, graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                if (e4 != hipSuccess) {
                    b->gexec = nullptr;
                    return bfail(b, MD_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e4));
                }
                b->graph_parity = p0;
            }
            BHIP_TRY(b, hipGraphLaunch(b->gexec, b->stream));
            b->host_step += 2;
            left -= 2;
            continue;
        }
        BHIP_TRY(b, batch_enqueue_step(b));
        --left;
    }
    batch_sync_members(b);
    return MD_OK;
}

md_status md_batch_observables(md_batch b, md_obs* out) {
    if (!b || !out) return fail(nullptr, MD_ERR_ARG, "NULL argument");
    SysEntry* to = b->tabs[1][b->parity];
    BHIP_TRY(b, launch_batch_rebuild(b->bc, to, b->tile_sys, b->ntiles, b->parity, b->stream));
    BHIP_TRY(b, launch_batch_step(to, b->tile_sys, b->ntiles, b->parity, MODE_OBSERVE, 1, b->stream));
    BHIP_TRY(b, launch_batch_finalize(to, b->nsys, MODE_OBSERVE, b->stream));
    BHIP_TRY(b, launch_batch_gather_obs(to, b->nsys, b->obs, b->stream));
    std::vector<double> rec((size_t)kHistRec * b->nsys);
    BHIP_TRY(b, hipMemcpyAsync(rec.data(), b->obs, sizeof(double) * rec.size(), hipMemcpyDeviceToHost, b->stream));
    BHIP_TRY(b, hipStreamSynchronize(b->stream));
    md_status worst = MD_OK;
    for (int s = 0; s < b->nsys; ++s) {
        fill_obs(b->sys[s], &rec[(size_t)s * kHistRec], &out[s]);
        const md_status r = status_to_code(b->sys[s], out[s].status_flags, out[s].nl_max_count);
        if (r != MD_OK && worst == MD_OK) {
            worst = r;
            b->err = "system " + std::to_string(s) + ": " + b->sys[s]->err;
            g_last_error = b->err;
        }
    }
    return worst;
}

md_status md_batch_get_state(md_batch b, int32_t sys, double* pos, double* vel, int32_t* image, double* pos_build,
                             int64_t* step, int32_t* vel_half) {
    if (!b || sys < 0 || sys >= b->nsys) return fail(nullptr, MD_ERR_ARG, "bad batch or system index");
    md_status r = md_get_state(b->sys[sys], pos, vel, image, pos_build, step, vel_half);
    if (r != MD_OK) bfail(b, r, b->sys[sys]->err);
    return r;
}

const char* md_batch_last_error(md_batch b) { return b ? b->err.c_str() : g_last_error.c_str(); }

md_status md_batch_timing_enable(md_batch b, int32_t enable) {
    if (!b) return fail(nullptr, MD_ERR_ARG, "NULL batch");
    b->timing = enable != 0;
    return MD_OK;
}

md_status md_batch_timing_read(md_batch b, md_timing* out) {
    if (!b || !out) return fail(nullptr, MD_ERR_ARG, "NULL argument");
    BHIP_TRY(b, hipStreamSynchronize(b->stream));
    for (const EvQuad& q : b->ev_pending) {
        float x = 0, y = 0, z = 0, w = 0;
        BHIP_TRY(b, hipEventElapsedTime(&x, q.e[0], q.e[1]));
        BHIP_TRY(b, hipEventElapsedTime(&y, q.e[1], q.e[2]));
        BHIP_TRY(b, hipEventElapsedTime(&z, q.e[2], q.e[3]));
        BHIP_TRY(b, hipEventElapsedTime(&w, q.e[0], q.e[4]));
        b->tacc.n_rebuild += 1;
        b->tacc.ms_rebuild += x;
        b->tacc.ms_bin_sort += w;
        b->tacc.n_step_kernels += 1;
        b->tacc.ms_step_kernels += y;
        b->tacc.n_finalize += 1;
        b->tacc.ms_finalize += z;
        b->ev_free.push_back(q);
    }
    b->ev_pending.clear();
    *out = b->tacc;
    memset(&b->tacc, 0, sizeof(b->tacc));
    return MD_OK;
}

md_status md_destroy(md_handle h) {
    if (!h) return MD_OK;
    (void)hipStreamSynchronize(h->stream);
    drop_graph(h);
    if (h->static_dev >= 0) {
        std::lock_guard<std::mutex> lk(g_static_mu);
        if (g_static_owner[h->static_dev] == h) g_static_owner[h->static_dev] = nullptr;
    }
    for (auto& q : h->ev_free)
        for (int k = 0; k < kStepEvents; ++k) (void)hipEventDestroy(q.e[k]);
    for (auto& q : h->ev_pending)
        for (int k = 0; k < kStepEvents; ++k) (void)hipEventDestroy(q.e[k]);
    delete h;
    return MD_OK;
}

}  // extern "C"
