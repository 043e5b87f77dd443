// gfx950 kernels of the per-timestep short-range MD step (ESPResSo++,
// arXiv 2608.14911): cell binning and stable cell sort (CellGrid, section
// "Software design"), Verlet-list build with a skin (VerletList +
// system.skin, section "Example usage"), LJ / capped-LJ pair forces
// (LennardJones, LennardJonesCapped with shift='auto'), FENE + cosine
// bending bonded forces (bonded interactions, section "Functionality"),
// velocity Verlet with the Langevin force (VelocityVerlet +
// LangevinThermostat) and FP64 energy / virial reductions
// (computeEnergy()).
//
// Layout: particles are kept sorted by cell so that a wavefront's 64 lanes
// stream neighbouring particles; positions are double4 (x, y, z, type) so a
// gathered neighbour is one 32-byte segment; velocities and build positions
// are SoA planes; the Verlet list is ELL, neighbour-major (entry k of
// particle i at k*N + i) so that lane i reads consecutive words.
#include "md_internal.h"

namespace md {

// ------------------------------------------------------------------ helpers

// Minimum image by compare-and-shift: the same IEEE operations on every
// side, and exactly antisymmetric (d_ji = -d_ij).
__device__ __forceinline__ double mimg(double d, double L, double hL) {
    if (d > hL) d -= L;
    else if (d < -hL) d += L;
    return d;
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

__device__ __forceinline__ void cell_coords(const Geom& g, double x, double y, double z, int& cx,
                                            int& cy, int& cz) {
    // positions are in [0, L); the clamp covers rounding at L and NaN
    double fx = x * g.invh[0], fy = y * g.invh[1], fz = z * g.invh[2];
    cx = (fx >= 0.0) ? (int)fx : 0;
    cy = (fy >= 0.0) ? (int)fy : 0;
    cz = (fz >= 0.0) ? (int)fz : 0;
    cx = clampi(cx, 0, g.nc[0] - 1);
    cy = clampi(cy, 0, g.nc[1] - 1);
    cz = clampi(cz, 0, g.nc[2] - 1);
}

__device__ __forceinline__ uint32_t cell_of(const Geom& g, const double4& p) {
    int cx, cy, cz;
    cell_coords(g, p.x, p.y, p.z, cx, cy, cz);
    return (uint32_t)(((int64_t)cz * g.nc[1] + cy) * g.nc[0] + cx);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of two
// 64x64->128 multiplies with the published multipliers, key bumped by the
// published Weyl constants between rounds.
__device__ __forceinline__ void philox4x64_10(uint64_t& x0, uint64_t& x1, uint64_t& x2, uint64_t& x3,
                                              uint64_t k0, uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t hi0 = __umul64hi(M0, x0), lo0 = M0 * x0;
        uint64_t hi1 = __umul64hi(M1, x2), lo1 = M1 * x2;
        uint64_t n0 = hi1 ^ x1 ^ k0;
        uint64_t n2 = hi0 ^ x3 ^ k1;
        x0 = n0;
        x1 = lo1;
        x2 = n2;
        x3 = lo0;
        k0 += 0x9E3779B97F4A7C15ull;
        k1 += 0xBB67AE8584CAA73Bull;
    }
}

// Three N(0,1) draws keyed (seed, stream) at counter (step, tag, 0, 0):
// uniforms ((w >> 11) + 1/2) 2^-53 in (0,1), Box-Muller in FP64.
__device__ __forceinline__ void gauss3(uint64_t seed, uint64_t stream, uint64_t step, uint64_t tag,
                                       double& g0, double& g1, double& g2) {
    uint64_t x0 = step, x1 = tag, x2 = 0, x3 = 0;
    philox4x64_10(x0, x1, x2, x3, seed, stream);
    const double two_pi = 6.283185307179586;
    double u0 = ((double)(x0 >> 11) + 0.5) * 0x1.0p-53;
    double u1 = ((double)(x1 >> 11) + 0.5) * 0x1.0p-53;
    double u2 = ((double)(x2 >> 11) + 0.5) * 0x1.0p-53;
    double u3 = ((double)(x3 >> 11) + 0.5) * 0x1.0p-53;
    double r0 = sqrt(-2.0 * log(u0));
    double r1 = sqrt(-2.0 * log(u2));
    g0 = r0 * cos(two_pi * u1);
    g1 = r0 * sin(two_pi * u1);
    g2 = r1 * cos(two_pi * u3);
}

template <typename Real>
__device__ __forceinline__ Real rcp(Real x);
template <>
__device__ __forceinline__ float rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <>
__device__ __forceinline__ double rcp<double>(double x) { return 1.0 / x; }

template <typename Real>
__device__ __forceinline__ Real rsq(Real x);
template <>
__device__ __forceinline__ float rsq<float>(float x) { return __builtin_amdgcn_rsqf(x); }
template <>
__device__ __forceinline__ double rsq<double>(double x) { return 1.0 / sqrt(x); }

template <typename Real>
__device__ __forceinline__ Real logr(Real x);
template <>
__device__ __forceinline__ float logr<float>(float x) { return logf(x); }
template <>
__device__ __forceinline__ double logr<double>(double x) { return log(x); }

template <typename Real>
__device__ __forceinline__ const PairCoef<Real>& coef(const PairTable& pt, int tp);
template <>
__device__ __forceinline__ const PairCoef<float>& coef<float>(const PairTable& pt, int tp) { return pt.f[tp]; }
template <>
__device__ __forceinline__ const PairCoef<double>& coef<double>(const PairTable& pt, int tp) { return pt.d[tp]; }

__device__ __forceinline__ bool rebuild_requested(const Bufs& b) {
    return __atomic_load_n(&b.ctl->rebuild, __ATOMIC_RELAXED) != 0;
}

__device__ __forceinline__ int64_t gtid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ int64_t gstride() { return (int64_t)gridDim.x * blockDim.x; }

// ------------------------------------------------------------------ init / state I/O

// Load tag-ordered FP64 state into the (identity-ordered) sorted arrays,
// folding positions into [0, L) with image counters.
__global__ void __launch_bounds__(kBlock) k_init_load(Geom g, Bufs b, int parity, const double* pos,
                                                      const double* vel, const int32_t* type,
                                                      const int32_t* image) {
    const int64_t n = g.n;
    for (int64_t i = gtid(); i < n; i += gstride()) {
        double p[3];
        for (int d = 0; d < 3; ++d) {
            double x = pos[3 * i + d];
            int im = image ? image[3 * i + d] : 0;
            double k = floor(x / g.L[d]);
            if (k != 0.0 && isfinite(k)) {
                x -= k * g.L[d];
                im += (int)k;
            }
            if (x < 0.0) { x += g.L[d]; im -= 1; }
            if (x >= g.L[d]) { x -= g.L[d]; im += 1; }
            p[d] = x;
            b.img[d * n + i] = im;
            b.v[d * n + i] = vel[3 * i + d];
        }
        int ty = type ? type[i] : 0;
        if (ty < 0 || ty >= g.ntypes) {
            atomicOr(&b.ctl->status, MD_FLAG_BAD_TYPE);
            ty = 0;
        }
        b.x[parity][i] = make_double4(p[0], p[1], p[2], (double)ty);
        b.tag[i] = (int32_t)i;
        b.inv[i] = (int32_t)i;
    }
}

// After a rebuild from the build positions, put the current state into the
// slots the sort assigned (used by md_set_state with a build snapshot).
__global__ void __launch_bounds__(kBlock) k_overwrite_state(Geom g, Bufs b, int parity,
                                                            const double* pos, const double* vel,
                                                            const int32_t* image) {
    const int64_t n = g.n;
    for (int64_t s = gtid(); s < n; s += gstride()) {
        int64_t t = b.tag[s];
        double4 old = b.x[parity][s];
        double p[3];
        for (int d = 0; d < 3; ++d) {
            double x = pos[3 * t + d];
            int im = image ? image[3 * t + d] : 0;
            if (x < 0.0) { x += g.L[d]; im -= 1; }
            if (x >= g.L[d]) { x -= g.L[d]; im += 1; }
            p[d] = x;
            b.img[d * n + s] = im;
            b.v[d * n + s] = vel[3 * t + d];
        }
        b.x[parity][s] = make_double4(p[0], p[1], p[2], old.w);
    }
}

__global__ void __launch_bounds__(kBlock) k_get_state(Geom g, Bufs b, int parity, double* pos,
                                                      double* vel, int32_t* image, double* pos_build) {
    const int64_t n = g.n;
    for (int64_t s = gtid(); s < n; s += gstride()) {
        int64_t t = b.tag[s];
        double4 p = b.x[parity][s];
        if (pos) { pos[3 * t] = p.x; pos[3 * t + 1] = p.y; pos[3 * t + 2] = p.z; }
        for (int d = 0; d < 3; ++d) {
            if (vel) vel[3 * t + d] = b.v[d * n + s];
            if (image) image[3 * t + d] = b.img[d * n + s];
            if (pos_build) pos_build[3 * t + d] = b.xb[d * n + s];
        }
    }
}

__global__ void __launch_bounds__(kBlock) k_get_neighbors(Geom g, Bufs b, int32_t* count,
                                                          int32_t* idx, int32_t cap) {
    const int64_t n = g.n;
    for (int64_t s = gtid(); s < n; s += gstride()) {
        int64_t t = b.tag[s];
        int c = b.ncount[s];
        int cc = c < g.cap ? c : g.cap;
        count[t] = c;
        for (int k = 0; k < cc && k < cap; ++k) idx[t * (int64_t)cap + k] = b.tag[b.nl[(int64_t)k * n + s]];
    }
}

__global__ void k_set_ctl(Bufs b, int64_t step, int vel_half, int rebuild, int clear_status) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        DevCtl* c = b.ctl;
        if (step >= 0) c->step = step;
        if (vel_half >= 0) c->vel_half = vel_half;
        if (rebuild >= 0) c->rebuild = (uint32_t)rebuild;
        c->rebuild_next = 0;
        if (clear_status) { c->status = 0; c->nl_max = 0; }
    }
}

__global__ void __launch_bounds__(kBlock) k_zero_i32(int32_t* p, int64_t n) {
    for (int64_t i = gtid(); i < n; i += gstride()) p[i] = 0;
}

__global__ void __launch_bounds__(kBlock) k_copy_i32(int32_t* dst, const int32_t* src, int64_t n) {
    for (int64_t i = gtid(); i < n; i += gstride()) dst[i] = src[i];
}

// ------------------------------------------------------------------ rebuild: cell sort
// Every rebuild kernel returns at once unless the device flag asks for a
// rebuild, so the whole step can be enqueued (and graph-captured) without a
// host round trip.

__global__ void __launch_bounds__(kBlock) k_bin(Geom g, Bufs b, int parity) {
    if (!rebuild_requested(b)) return;
    const double4* __restrict__ x = b.x[parity];
    for (int64_t i = gtid(); i < g.n; i += gstride()) {
        uint32_t c = cell_of(g, x[i]);
        b.cellid[i] = c;
        atomicAdd(&b.ccount[c], 1);
    }
}

__device__ int block_exclusive_scan(int v, int& total) {
    __shared__ int wsum[kBlock / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < kBlock / 64; ++k) {
        if (k < w) off += wsum[k];
        tot += wsum[k];
    }
    __syncthreads();
    total = tot;
    return off + x - v;
}

__device__ __forceinline__ void scan_chunk(const Geom& g, int blk, int64_t& lo, int64_t& hi) {
    int64_t chunk = (g.ncell + kScanBlocks - 1) / kScanBlocks;
    lo = blk * chunk;
    hi = lo + chunk;
    if (hi > g.ncell) hi = g.ncell;
    if (lo > g.ncell) lo = g.ncell;
}

__global__ void __launch_bounds__(kBlock) k_scan_reduce(Geom g, Bufs b) {
    if (!rebuild_requested(b)) return;
    int64_t lo, hi;
    scan_chunk(g, blockIdx.x, lo, hi);
    int s = 0;
    for (int64_t c = lo + threadIdx.x; c < hi; c += kBlock) s += b.ccount[c];
    __shared__ int red[kBlock];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) b.bsum[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(1024) k_scan_top(Bufs b) {
    if (!rebuild_requested(b)) return;
    __shared__ int wsum[16];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int v = b.bsum[threadIdx.x];
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    int off = 0;
    for (int k = 0; k < w; ++k) off += wsum[k];
    b.bsum[threadIdx.x] = off + x - v;
}

__global__ void __launch_bounds__(kBlock) k_scan_apply(Geom g, Bufs b) {
    if (!rebuild_requested(b)) return;
    int64_t lo, hi;
    scan_chunk(g, blockIdx.x, lo, hi);
    int running = b.bsum[blockIdx.x];
    for (int64_t base = lo; base < hi; base += kBlock) {
        int64_t c = base + threadIdx.x;
        int v = (c < hi) ? b.ccount[c] : 0;
        int tot;
        int e = block_exclusive_scan(v, tot);
        if (c < hi) b.cstart[c] = running + e;
        running += tot;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) b.cstart[g.ncell] = (int32_t)g.n;
}

// Scatter into cell segments; counts return to zero for the next build.
__global__ void __launch_bounds__(kBlock) k_scatter(Geom g, Bufs b) {
    if (!rebuild_requested(b)) return;
    for (int64_t i = gtid(); i < g.n; i += gstride()) {
        uint32_t c = b.cellid[i];
        int slot = b.cstart[c] + atomicSub(&b.ccount[c], 1) - 1;
        b.tmp[slot] = (int32_t)i;
    }
}

// Order inside a cell by particle tag: the sorted order is then a function
// of the positions alone, so a run resumed from a saved build snapshot
// reproduces it exactly.  Gathers all per-particle arrays into temporaries.
__global__ void __launch_bounds__(kBlock) k_rank_permute(Geom g, Bufs b, int parity) {
    if (!rebuild_requested(b)) return;
    const int64_t n = g.n;
    for (int64_t s = gtid(); s < n; s += gstride()) {
        int32_t i = b.tmp[s];
        uint32_t c = b.cellid[i];
        int32_t ti = b.tag[i];
        int st = b.cstart[c], en = b.cstart[c + 1];
        int r = 0;
        for (int u = st; u < en; ++u) r += (b.tag[b.tmp[u]] < ti);
        int64_t nw = st + r;
        b.xt[nw] = b.x[parity][i];
        for (int d = 0; d < 3; ++d) {
            b.vt[d * n + nw] = b.v[d * n + i];
            b.imgt[d * n + nw] = b.img[d * n + i];
        }
        b.tagt[nw] = ti;
    }
}

__global__ void __launch_bounds__(kBlock) k_commit(Geom g, Bufs b, int parity, int bonded) {
    if (!rebuild_requested(b)) return;
    const int64_t n = g.n;
    if (gtid() == 0) {
        b.ctl->n_rebuilds += 1;
        b.ctl->nl_max = 0;
    }
    for (int64_t s = gtid(); s < n; s += gstride()) {
        double4 p = b.xt[s];
        b.x[parity][s] = p;
        b.xb[s] = p.x;
        b.xb[n + s] = p.y;
        b.xb[2 * n + s] = p.z;
        for (int d = 0; d < 3; ++d) {
            b.v[d * n + s] = b.vt[d * n + s];
            b.img[d * n + s] = b.imgt[d * n + s];
        }
        int32_t t = b.tagt[s];
        b.tag[s] = t;
        b.inv[t] = (int32_t)s;
        if (bonded) b.tcnt_s[s] = b.tcnt_t[t];
    }
}

// ------------------------------------------------------------------ rebuild: Verlet list

// NL(i) = { j != i : r_ij^2 < rv^2 } over the 27 surrounding cells, with
// r^2 = (dx*dx + dy*dy) + dz*dz in FP64 and no fused multiply-add, so the
// sets equal those of any implementation performing the same IEEE
// operations.  Row order: stencil (z, y, x offsets -1..1), then sorted index.
// Also remaps the bonded topology from tags to sorted indices.
__global__ void __launch_bounds__(kBlock) k_nl_build(Geom g, Bufs b, int parity, int bonded) {
#pragma clang fp contract(off)
    if (!rebuild_requested(b)) return;
    const int64_t n = g.n;
    const double4* __restrict__ x = b.x[parity];
    int local_max = 0;
    bool overflow = false;
    for (int64_t i = gtid(); i < n; i += gstride()) {
        double4 xi = x[i];
        int cx, cy, cz;
        cell_coords(g, xi.x, xi.y, xi.z, cx, cy, cz);
        int cnt = 0;
        for (int oz = -1; oz <= 1; ++oz) {
            int nz = cz + oz;
            nz = nz < 0 ? nz + g.nc[2] : (nz >= g.nc[2] ? nz - g.nc[2] : nz);
            for (int oy = -1; oy <= 1; ++oy) {
                int ny = cy + oy;
                ny = ny < 0 ? ny + g.nc[1] : (ny >= g.nc[1] ? ny - g.nc[1] : ny);
                for (int ox = -1; ox <= 1; ++ox) {
                    int nx = cx + ox;
                    nx = nx < 0 ? nx + g.nc[0] : (nx >= g.nc[0] ? nx - g.nc[0] : nx);
                    int64_t c = ((int64_t)nz * g.nc[1] + ny) * g.nc[0] + nx;
                    int st = b.cstart[c], en = b.cstart[c + 1];
                    for (int j = st; j < en; ++j) {
                        if (j == i) continue;
                        double4 xj = x[j];
                        double dx = mimg(xj.x - xi.x, g.L[0], g.hL[0]);
                        double dy = mimg(xj.y - xi.y, g.L[1], g.hL[1]);
                        double dz = mimg(xj.z - xi.z, g.L[2], g.hL[2]);
                        double r2 = (dx * dx + dy * dy) + dz * dz;
                        if (r2 < g.rv2) {
                            if (cnt < g.cap) b.nl[(int64_t)cnt * n + i] = j;
                            ++cnt;
                        }
                    }
                }
            }
        }
        b.ncount[i] = cnt;
        if (cnt > local_max) local_max = cnt;
        if (cnt > g.cap) overflow = true;
        if (bonded) {
            int32_t t = b.tag[i];
            int tc = b.tcnt_t[t];
            int nb = tc & 0xff, na = tc >> 8;
            for (int k = 0; k < nb; ++k) b.bp_s[(int64_t)k * n + i] = b.inv[b.bp_t[(int64_t)k * n + t]];
            for (int k = 0; k < na; ++k) {
                int2 e = b.ang_t[(int64_t)k * n + t];
                int role = (int)((uint32_t)e.x >> 30);
                int o1 = e.x & 0x3fffffff;
                b.ang_s[(int64_t)k * n + i] = make_int2(b.inv[o1] | (role << 30), b.inv[e.y]);
            }
        }
    }
    // one atomic per wave
    for (int o = 32; o >= 1; o >>= 1) {
        int y = __shfl_xor(local_max, o, 64);
        local_max = y > local_max ? y : local_max;
    }
    if ((threadIdx.x & 63) == 0 && local_max > 0) atomicMax(&b.ctl->nl_max, local_max);
    if (__any(overflow) && (threadIdx.x & 63) == 0) atomicOr(&b.ctl->status, MD_FLAG_NL_OVERFLOW);
}

__global__ void k_clear_rebuild(Bufs b) {
    if (threadIdx.x == 0 && blockIdx.x == 0) b.ctl->rebuild = 0;
}

// ------------------------------------------------------------------ forces + integration

// Fused per-particle kernel: pair forces over the Verlet row, bonded forces,
// then (MODE_STEP) the velocity-Verlet update with the Langevin force, the
// periodic wrap, the half-skin displacement test, and per-block FP64 partial
// sums of energy, kinetic energy and virial.  Positions are double-buffered
// by step parity so that the update can run in the same kernel as the
// neighbour gathers.  Real is the precision of the pair / bonded math;
// coordinate differences are always taken in FP64.
template <typename Real, bool SINGLE, bool BONDED>
__global__ void __launch_bounds__(kBlock) k_step(const StepArgs a) {
    const Geom& g = a.g;
    const Bufs& b = a.b;
    const int64_t n = g.n;
    const double4* __restrict__ xin = b.x[a.parity];
    double acc[kNacc];
#pragma unroll
    for (int k = 0; k < kNacc; ++k) acc[k] = 0.0;
    bool flag_rebuild = false, flag_bond = false, flag_nonfinite = false;

    const int64_t i = gtid();
    if (i < n) {
        const double4 xi = xin[i];
        const int ti = SINGLE ? 0 : (int)xi.w;
        Real fx = 0, fy = 0, fz = 0, ui = 0, wi = 0;
        Real txx = 0, tyy = 0, tzz = 0, txy = 0, txz = 0, tyz = 0;
        const bool tensor = a.tensor != 0;
        int cnt = b.ncount[i];
        cnt = cnt < g.cap ? cnt : g.cap;
        const int32_t* __restrict__ row = b.nl + i;

        auto pair = [&](const double4& xj) {
            double dx = mimg(xj.x - xi.x, g.L[0], g.hL[0]);
            double dy = mimg(xj.y - xi.y, g.L[1], g.hL[1]);
            double dz = mimg(xj.z - xi.z, g.L[2], g.hL[2]);
            double r2d = dx * dx + dy * dy + dz * dz;
            const int tp = SINGLE ? 0 : ti * MD_MAX_TYPES + (int)xj.w;
            if (r2d < a.pt.rc2d[tp]) {
                const PairCoef<Real>& c = coef<Real>(a.pt, tp);
                Real r2 = (Real)r2d;
                Real fr, u;
                if (c.cap2 > Real(0) && r2 < c.cap2) {
                    fr = c.fcap * rsq<Real>(r2);
                    u = c.ucap;
                } else {
                    Real inv = rcp<Real>(r2);
                    Real s2 = c.sig2 * inv;
                    Real s6 = s2 * s2 * s2;
                    fr = c.eps24 * s6 * (Real(2) * s6 - Real(1)) * inv;
                    u = c.eps4 * s6 * (s6 - Real(1)) - c.shift;
                }
                Real rx = -(Real)dx, ry = -(Real)dy, rz = -(Real)dz;  // r_i - r_j
                fx += fr * rx;
                fy += fr * ry;
                fz += fr * rz;
                ui += u;
                wi += fr * r2;
                if (tensor) {
                    txx += fr * rx * rx; tyy += fr * ry * ry; tzz += fr * rz * rz;
                    txy += fr * rx * ry; txz += fr * rx * rz; tyz += fr * ry * rz;
                }
            }
        };

        int k = 0;
        for (; k + 4 <= cnt; k += 4) {
            const int j0 = row[(int64_t)(k + 0) * n];
            const int j1 = row[(int64_t)(k + 1) * n];
            const int j2 = row[(int64_t)(k + 2) * n];
            const int j3 = row[(int64_t)(k + 3) * n];
            const double4 x0 = xin[j0], x1 = xin[j1], x2 = xin[j2], x3 = xin[j3];
            pair(x0);
            pair(x1);
            pair(x2);
            pair(x3);
        }
        for (; k < cnt; ++k) pair(xin[row[(int64_t)k * n]]);

        acc[A_EPAIR] = 0.5 * (double)ui;
        acc[A_VIR] = 0.5 * (double)wi;
        if (tensor) {
            acc[A_TXX] = 0.5 * (double)txx; acc[A_TYY] = 0.5 * (double)tyy; acc[A_TZZ] = 0.5 * (double)tzz;
            acc[A_TXY] = 0.5 * (double)txy; acc[A_TXZ] = 0.5 * (double)txz; acc[A_TYZ] = 0.5 * (double)tyz;
        }

        if (BONDED) {
            const int tc = b.tcnt_s[i];
            const int nb = tc & 0xff, na = tc >> 8;
            const Real K = sizeof(Real) == 8 ? (Real)a.dy.fene_K : (Real)a.dy.fene_Kf;
            const Real R02 = sizeof(Real) == 8 ? (Real)a.dy.fene_R02 : (Real)a.dy.fene_R02f;
            const Real hKR02 = sizeof(Real) == 8 ? (Real)a.dy.fene_halfKR02 : (Real)a.dy.fene_halfKR02f;
            Real eb = 0, wb = 0;
            for (int q = 0; q < nb; ++q) {
                const int m = b.bp_s[(int64_t)q * n + i];
                const double4 xm = xin[m];
                Real rx = -(Real)mimg(xm.x - xi.x, g.L[0], g.hL[0]);
                Real ry = -(Real)mimg(xm.y - xi.y, g.L[1], g.hL[1]);
                Real rz = -(Real)mimg(xm.z - xi.z, g.L[2], g.hL[2]);
                Real r2 = rx * rx + ry * ry + rz * rz;
                Real qq = r2 / R02;
                if (!(qq < Real(1))) {
                    flag_bond = true;
                    continue;
                }
                Real om = Real(1) - qq;
                Real fr = -K / om;
                fx += fr * rx;
                fy += fr * ry;
                fz += fr * rz;
                eb += -hKR02 * logr<Real>(om);
                wb += fr * r2;
                if (tensor) {
                    acc[A_TXX] += 0.5 * (double)(fr * rx * rx); acc[A_TYY] += 0.5 * (double)(fr * ry * ry);
                    acc[A_TZZ] += 0.5 * (double)(fr * rz * rz); acc[A_TXY] += 0.5 * (double)(fr * rx * ry);
                    acc[A_TXZ] += 0.5 * (double)(fr * rx * rz); acc[A_TYZ] += 0.5 * (double)(fr * ry * rz);
                }
            }
            acc[A_EBOND] = 0.5 * (double)eb;
            acc[A_VIR] += 0.5 * (double)wb;
            const Real kb = sizeof(Real) == 8 ? (Real)a.dy.k_bend : (Real)a.dy.k_bendf;
            Real ea = 0, wa = 0;
            for (int q = 0; q < na; ++q) {
                const int2 e = b.ang_s[(int64_t)q * n + i];
                const int role = (int)((uint32_t)e.x >> 30);
                const int o1 = e.x & 0x3fffffff, o2 = e.y;
                const double4 p1 = xin[o1], p2 = xin[o2];
                // particles (A, B, C) with B the centre
                const double4& pa = role == 0 ? xi : p1;
                const double4& pb = role == 1 ? xi : (role == 0 ? p1 : p2);
                const double4& pc = role == 2 ? xi : p2;
                Real b1x = (Real)mimg(pb.x - pa.x, g.L[0], g.hL[0]);
                Real b1y = (Real)mimg(pb.y - pa.y, g.L[1], g.hL[1]);
                Real b1z = (Real)mimg(pb.z - pa.z, g.L[2], g.hL[2]);
                Real b2x = (Real)mimg(pc.x - pb.x, g.L[0], g.hL[0]);
                Real b2y = (Real)mimg(pc.y - pb.y, g.L[1], g.hL[1]);
                Real b2z = (Real)mimg(pc.z - pb.z, g.L[2], g.hL[2]);
                Real l1sq = b1x * b1x + b1y * b1y + b1z * b1z;
                Real l2sq = b2x * b2x + b2y * b2y + b2z * b2z;
                Real il1l2 = rsq<Real>(l1sq * l2sq);
                Real cs = (b1x * b2x + b1y * b2y + b1z * b2z) * il1l2;
                Real i1 = rcp<Real>(l1sq), i2 = rcp<Real>(l2sq);
                // dcos/db1 and dcos/db2
                Real g1x = b2x * il1l2 - cs * b1x * i1, g1y = b2y * il1l2 - cs * b1y * i1, g1z = b2z * il1l2 - cs * b1z * i1;
                Real g2x = b1x * il1l2 - cs * b2x * i2, g2y = b1y * il1l2 - cs * b2y * i2, g2z = b1z * il1l2 - cs * b2z * i2;
                Real Fx, Fy, Fz;
                if (role == 0) {
                    Fx = -kb * g1x; Fy = -kb * g1y; Fz = -kb * g1z;
                    wa += -(b1x * Fx + b1y * Fy + b1z * Fz);
                    if (tensor) {
                        acc[A_TXX] += (double)(-b1x * Fx); acc[A_TYY] += (double)(-b1y * Fy); acc[A_TZZ] += (double)(-b1z * Fz);
                        acc[A_TXY] += 0.5 * (double)(-b1x * Fy - b1y * Fx); acc[A_TXZ] += 0.5 * (double)(-b1x * Fz - b1z * Fx);
                        acc[A_TYZ] += 0.5 * (double)(-b1y * Fz - b1z * Fy);
                    }
                } else if (role == 2) {
                    Fx = kb * g2x; Fy = kb * g2y; Fz = kb * g2z;
                    wa += b2x * Fx + b2y * Fy + b2z * Fz;
                    if (tensor) {
                        acc[A_TXX] += (double)(b2x * Fx); acc[A_TYY] += (double)(b2y * Fy); acc[A_TZZ] += (double)(b2z * Fz);
                        acc[A_TXY] += 0.5 * (double)(b2x * Fy + b2y * Fx); acc[A_TXZ] += 0.5 * (double)(b2x * Fz + b2z * Fx);
                        acc[A_TYZ] += 0.5 * (double)(b2y * Fz + b2z * Fy);
                    }
                } else {
                    Fx = kb * (g1x - g2x); Fy = kb * (g1y - g2y); Fz = kb * (g1z - g2z);
                    ea += kb * (Real(1) - cs);
                }
                fx += Fx;
                fy += Fy;
                fz += Fz;
            }
            acc[A_EANGLE] = (double)ea;
            acc[A_VIR] += (double)wa;
        }

        const double F[3] = {(double)fx, (double)fy, (double)fz};
        const int tm = SINGLE ? 0 : ti;
        const double hdtm = a.dy.hdtm[tm];
        const double m = a.dy.mass[tm];
        double vp[3], ft[3];
        for (int d = 0; d < 3; ++d) vp[d] = b.v[d * n + i];
        int32_t tg = -1;
        if (a.dy.langevin || a.mode == MODE_FORCES) tg = b.tag[i];
        if (a.dy.langevin) {
            double g0, g1, g2;
            gauss3(a.dy.seed, 0, (uint64_t)b.ctl->step, (uint64_t)tg, g0, g1, g2);
            const double gm = a.dy.gm[tm], amp = a.dy.amp[tm];
            ft[0] = (F[0] - gm * vp[0]) + amp * g0;
            ft[1] = (F[1] - gm * vp[1]) + amp * g1;
            ft[2] = (F[2] - gm * vp[2]) + amp * g2;
        } else {
            ft[0] = F[0]; ft[1] = F[1]; ft[2] = F[2];
        }
        const bool vh_in = b.ctl->vel_half != 0;
        double von[3], ke = 0.0;
        for (int d = 0; d < 3; ++d) {
            von[d] = vh_in ? vp[d] + hdtm * ft[d] : vp[d];
            ke += von[d] * von[d];
        }
        acc[A_EKIN] = 0.5 * m * ke;

        if (a.mode == MODE_STEP) {
            double xo[3] = {xi.x, xi.y, xi.z};
            double d2 = 0.0;
            for (int d = 0; d < 3; ++d) {
                const double vh = von[d] + hdtm * ft[d];
                double xn = xo[d] + a.dy.dt * vh;
                if (xn < 0.0 || xn >= g.L[d]) {
                    int im = b.img[d * n + i];
                    if (xn < 0.0) { xn += g.L[d]; im -= 1; }
                    if (xn >= g.L[d]) { xn -= g.L[d]; im += 1; }
                    b.img[d * n + i] = im;
                }
                if (!isfinite(xn) || !isfinite(vh)) flag_nonfinite = true;
                xo[d] = xn;
                b.v[d * n + i] = vh;
                const double dd = mimg(xn - b.xb[d * n + i], g.L[d], g.hL[d]);
                d2 += dd * dd;
            }
            if (d2 > g.disp2) flag_rebuild = true;
            b.x[a.parity ^ 1][i] = make_double4(xo[0], xo[1], xo[2], xi.w);
        } else if (a.mode == MODE_FORCES && a.f_out) {
            a.f_out[3 * (int64_t)tg] = F[0];
            a.f_out[3 * (int64_t)tg + 1] = F[1];
            a.f_out[3 * (int64_t)tg + 2] = F[2];
        }
    }

    // flags: one store / atomic per wave
    const bool any_reb = __any(flag_rebuild);
    const bool any_bond = __any(flag_bond);
    const bool any_nf = __any(flag_nonfinite);
    if ((threadIdx.x & 63) == 0) {
        if (any_reb) __atomic_store_n(&b.ctl->rebuild_next, 1u, __ATOMIC_RELAXED);
        if (any_bond) atomicOr(&b.ctl->status, MD_FLAG_BOND_BROKEN);
        if (any_nf) atomicOr(&b.ctl->status, MD_FLAG_NONFINITE);
    }

    // deterministic block reduction: wave butterfly, then waves in order
    __shared__ double red[kBlock / 64][kNacc];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nacc = a.tensor ? kNacc : A_VIR + 1;
    for (int q = 0; q < nacc; ++q) {
        double s = wave_sum(acc[q]);
        if (lane == 0) red[w][q] = s;
    }
    __syncthreads();
    if (threadIdx.x < kNacc) {
        double s = 0.0;
        if ((int)threadIdx.x < nacc)
            for (int ww = 0; ww < kBlock / 64; ++ww) s += red[ww][threadIdx.x];
        b.partials[(int64_t)blockIdx.x * kNacc + threadIdx.x] = s;
    }
}

// One block: reduce the per-block partials in a fixed order, record the
// step's observables, and (MODE_STEP) advance the step counter and move the
// rebuild request to the next step.
constexpr int kFinal = 256;
__global__ void __launch_bounds__(kFinal) k_finalize(Bufs b, int nblocks, int mode) {
    __shared__ double red[kFinal / 64][kNacc];
    double s[kNacc];
#pragma unroll
    for (int k = 0; k < kNacc; ++k) s[k] = 0.0;
    for (int blk = threadIdx.x; blk < nblocks; blk += kFinal)
#pragma unroll
        for (int k = 0; k < kNacc; ++k) s[k] += b.partials[(int64_t)blk * kNacc + k];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < kNacc; ++k) {
        double v = wave_sum(s[k]);
        if (lane == 0) red[w][k] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot[kNacc];
        for (int k = 0; k < kNacc; ++k) {
            double v = 0.0;
            for (int ww = 0; ww < kFinal / 64; ++ww) v += red[ww][k];
            tot[k] = v;
        }
        DevCtl* c = b.ctl;
        const int64_t step = c->step;
        double rec[kHistRec];
        rec[H_STEP] = (double)step;
        rec[H_EPAIR] = tot[A_EPAIR];
        rec[H_EBOND] = tot[A_EBOND];
        rec[H_EANGLE] = tot[A_EANGLE];
        rec[H_EKIN] = tot[A_EKIN];
        rec[H_VIR] = tot[A_VIR];
        for (int k = 0; k < 6; ++k) rec[H_T0 + k] = tot[A_TXX + k];
        rec[H_NREB] = (double)c->n_rebuilds;
        rec[H_STATUS] = (double)c->status;
        rec[H_NLMAX] = (double)c->nl_max;
        rec[15] = 0.0;
        for (int k = 0; k < kHistRec; ++k) b.cur[k] = rec[k];
        if (mode == MODE_STEP) {
            double* h = b.hist + (int64_t)(step % MD_HISTORY_CAPACITY) * kHistRec;
            for (int k = 0; k < kHistRec; ++k) h[k] = rec[k];
            c->step = step + 1;
            c->vel_half = 1;
            c->rebuild = c->rebuild_next;
            c->rebuild_next = 0;
        } else {
            c->rebuild = 0;
        }
    }
}

// ------------------------------------------------------------------ launchers

static inline int grid_for(int64_t n, int cap_blocks = 4096) {
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > cap_blocks) g = cap_blocks;
    return (int)g;
}

hipError_t launch_init_load(const Geom& g, const Bufs& b, int parity, const double* pos,
                            const double* vel, const int32_t* type, const int32_t* image,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_init_load, dim3(grid_for(g.n)), dim3(kBlock), 0, s, g, b, parity, pos, vel, type,
                       image);
    return hipGetLastError();
}

hipError_t launch_overwrite_state(const Geom& g, const Bufs& b, int parity, const double* pos,
                                  const double* vel, const int32_t* image, hipStream_t s) {
    hipLaunchKernelGGL(k_overwrite_state, dim3(grid_for(g.n)), dim3(kBlock), 0, s, g, b, parity, pos, vel,
                       image);
    return hipGetLastError();
}

hipError_t launch_get_state(const Geom& g, const Bufs& b, int parity, double* pos, double* vel,
                            int32_t* image, double* pos_build, hipStream_t s) {
    hipLaunchKernelGGL(k_get_state, dim3(grid_for(g.n)), dim3(kBlock), 0, s, g, b, parity, pos, vel, image,
                       pos_build);
    return hipGetLastError();
}

hipError_t launch_get_neighbors(const Geom& g, const Bufs& b, int32_t* count, int32_t* idx, int32_t cap,
                                hipStream_t s) {
    hipLaunchKernelGGL(k_get_neighbors, dim3(grid_for(g.n)), dim3(kBlock), 0, s, g, b, count, idx, cap);
    return hipGetLastError();
}

hipError_t launch_set_ctl(const Bufs& b, int64_t step, int vel_half, int rebuild, int clear_status,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_set_ctl, dim3(1), dim3(64), 0, s, b, step, vel_half, rebuild, clear_status);
    return hipGetLastError();
}

hipError_t launch_zero_i32(int32_t* p, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_i32, dim3(grid_for(n)), dim3(kBlock), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_copy_i32(int32_t* dst, const int32_t* src, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_copy_i32, dim3(grid_for(n)), dim3(kBlock), 0, s, dst, src, n);
    return hipGetLastError();
}

hipError_t launch_clear_rebuild(const Bufs& b, hipStream_t s) {
    hipLaunchKernelGGL(k_clear_rebuild, dim3(1), dim3(64), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_rebuild(const Geom& g, const Bufs& b, int parity, int bonded, hipStream_t s,
                          hipEvent_t ev0, hipEvent_t ev1) {
    const int gs = grid_for(g.n, 2048);
    if (ev0) (void)hipEventRecord(ev0, s);
    hipLaunchKernelGGL(k_bin, dim3(gs), dim3(kBlock), 0, s, g, b, parity);
    hipLaunchKernelGGL(k_scan_reduce, dim3(kScanBlocks), dim3(kBlock), 0, s, g, b);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, b);
    hipLaunchKernelGGL(k_scan_apply, dim3(kScanBlocks), dim3(kBlock), 0, s, g, b);
    hipLaunchKernelGGL(k_scatter, dim3(gs), dim3(kBlock), 0, s, g, b);
    hipLaunchKernelGGL(k_rank_permute, dim3(gs), dim3(kBlock), 0, s, g, b, parity);
    hipLaunchKernelGGL(k_commit, dim3(gs), dim3(kBlock), 0, s, g, b, parity, bonded);
    hipLaunchKernelGGL(k_nl_build, dim3(grid_for(g.n, 8192)), dim3(kBlock), 0, s, g, b, parity, bonded);
    if (ev1) (void)hipEventRecord(ev1, s);
    return hipGetLastError();
}

hipError_t launch_step(const StepArgs& a, int fp64, int single_type, int bonded, int block, hipStream_t s) {
    (void)block;
    const int64_t nb = (a.g.n + kBlock - 1) / kBlock;
    dim3 grid((unsigned)nb), blk(kBlock);
#define MD_LAUNCH(R, S, B) hipLaunchKernelGGL((k_step<R, S, B>), grid, blk, 0, s, a)
    if (fp64) {
        if (single_type) { if (bonded) MD_LAUNCH(double, true, true); else MD_LAUNCH(double, true, false); }
        else { if (bonded) MD_LAUNCH(double, false, true); else MD_LAUNCH(double, false, false); }
    } else {
        if (single_type) { if (bonded) MD_LAUNCH(float, true, true); else MD_LAUNCH(float, true, false); }
        else { if (bonded) MD_LAUNCH(float, false, true); else MD_LAUNCH(float, false, false); }
    }
#undef MD_LAUNCH
    return hipGetLastError();
}

hipError_t launch_finalize(const Bufs& b, int nblocks, int mode, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinal), 0, s, b, nblocks, mode);
    return hipGetLastError();
}

}  // namespace md
