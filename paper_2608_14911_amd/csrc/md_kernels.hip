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
// stream neighbouring particles; positions are double4 (x, y, z, type) and
// fixed-point int4 (qx, qy, qz, type), so a gathered neighbour is one 32- or
// 16-byte segment; velocities and build positions are SoA planes; the
// Verlet list is ELL in tiles of 64 particles (entry k of particle i at
// (i / 64) * cap * 64 + k * 64 + i % 64), so that the 64 lanes of a
// wavefront read 256 contiguous bytes per entry.
#include "md_device.h"


namespace md {

// ------------------------------------------------------------------ helpers

// Minimum image d - L rint(d / L), branch-free.  For |d| < L (positions in
// [0, L)) the shift is 0 or +-L and the result is d -/+ L rounded once, the
// same value a compare-and-shift gives except within an ulp of |d| = L/2,
// which is never inside the list radius (L >= 3 cells >= 2 rv).  Exactly
// antisymmetric: d_ji = -d_ij.
__device__ __forceinline__ double mimg(double d, double L, double invL) {
    return fma(-L, rint(d * invL), d);
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

// Philox4x32-10 (the same paper): four 32-bit words, 10 rounds of two
// 32x32->64 multiplies with the published multipliers, the key bumped by the
// published Weyl constants between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t& x0, uint32_t& x1, uint32_t& x2, uint32_t& x3,
                                              uint32_t k0, uint32_t k1) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hi0 = __umulhi(M0, x0), lo0 = M0 * x0;
        const uint32_t hi1 = __umulhi(M1, x2), lo1 = M1 * x2;
        const uint32_t n0 = hi1 ^ x1 ^ k0;
        const uint32_t n2 = hi0 ^ x3 ^ k1;
        x0 = n0;
        x1 = lo1;
        x2 = n2;
        x3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
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
            b.v[d * n + i] = vel ? vel[3 * i + d] : 0.0;
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
        const int4 q = quantize4(g, p[0], p[1], p[2], old.w);
        b.xq[parity][s] = q;
        if (g.x3_on) store_q3(b.x3[parity], s, q);
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
        const int32_t* row = b.nl + nl_base(s, g.cap);
        for (int k = 0; k < cc && k < cap; ++k) idx[t * (int64_t)cap + k] = b.tag[row[nl_off(k)]];
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

// Runs of equal cells over the lanes of a wavefront.  Particles arrive in
// the previous build's cell order, so a run is usually a whole cell's share
// of the wavefront and one atomic serves it.  Active lanes are a prefix of
// the wavefront.  Returns the run's first lane and its length.
__device__ __forceinline__ void cell_run(uint32_t c, bool active, int& first, int& len) {
    const int lane = threadIdx.x & 63;
    const uint32_t prev = __shfl_up(c, 1, 64);
    const uint64_t heads = __ballot(active && (lane == 0 || c != prev));
    // bits 0 .. k: (2 << k) - 1, which is all ones for k = 63
    const uint64_t upto = heads & ((2ull << lane) - 1);
    first = upto ? 63 - __clzll(upto) : 0;
    const uint64_t after = heads & ~((2ull << first) - 1);
    const int nact = __popcll(__ballot(active));
    const int next = after ? __ffsll((unsigned long long)after) - 1 : nact;
    len = next - first;
}

__device__ __forceinline__ uint32_t bin_one(const Geom& g, const Bufs& b, int64_t i, bool active, int parity) {
    uint32_t c = 0xffffffffu;
    if (active) {
        c = cell_of(g, b.x[parity][i]);
        b.cellid[i] = c;
    }
    int first, len;
    cell_run(c, active, first, len);
    if (active && (threadIdx.x & 63) == first) atomicAdd(&b.ccount[c], len);
    return c;
}

// Cells are scanned in kScanBlocks chunks of consecutive cells.  Binning also
// sums each chunk's particles (one atomic per run of equal chunks in a
// wavefront, each chunk's sum on a 128-byte line of its own), so the scan
// needs no separate reduction pass.
__device__ __forceinline__ int64_t scan_chunk_cells(const Geom& g) {
    return (g.ncell + kScanBlocks - 1) / kScanBlocks;
}

__global__ void __launch_bounds__(kBlock) k_bin(Geom g, Bufs b, int parity) {
    if (!rebuild_requested(b)) return;
    const int64_t chunk = scan_chunk_cells(g);
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < g.n; i0 += gstride()) {
        const int64_t i = i0 + threadIdx.x;
        const bool active = i < g.n;
        const uint32_t c = bin_one(g, b, i, active, parity);
        const uint32_t ch = active ? (uint32_t)(c / chunk) : 0xffffffffu;
        int first, len;
        cell_run(ch, active, first, len);
        if (active && (threadIdx.x & 63) == first) atomicAdd(&b.bsum[(int64_t)ch * kChunkPad], len);
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
    const int64_t chunk = scan_chunk_cells(g);
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

// Exclusive scan of the kScanBlocks chunk sums by one block.
__global__ void __launch_bounds__(kScanBlocks) k_scan_top(Bufs b) {
    if (!rebuild_requested(b)) return;
    __shared__ int wsum[kScanBlocks / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int v = b.bsum[threadIdx.x];
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    int off = 0;
    for (int k = 0; k < w; ++k) off += wsum[k];
    b.bsum[threadIdx.x] = off + x - v;
}

__device__ __forceinline__ void scan_apply_body(const Geom& g, const Bufs& b, int running) {
    int64_t lo, hi;
    scan_chunk(g, blockIdx.x, lo, hi);
    // four consecutive cells per thread and step
    for (int64_t base = lo; base < hi; base += 4 * kBlock) {
        const int64_t c0 = base + 4 * (int64_t)threadIdx.x;
        int v[4], sum = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            v[u] = (c0 + u < hi) ? b.ccount[c0 + u] : 0;
            sum += v[u];
        }
        int tot;
        int e = block_exclusive_scan(sum, tot);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (c0 + u < hi) b.cstart[c0 + u] = running + e;
            e += v[u];
        }
        running += tot;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) b.cstart[g.ncell] = (int32_t)g.n;
}

// Batches: chunk offsets from k_scan_reduce and k_scan_top.
__global__ void __launch_bounds__(kBlock) k_scan_apply(Geom g, Bufs b) {
    if (!rebuild_requested(b)) return;
    scan_apply_body(g, b, b.bsum[blockIdx.x]);
}

// One system: the chunk sums come from k_bin, and each block adds up the
// sums of the chunks before its own (at most kScanBlocks values, read from
// the L2), which replaces the reduction and top-level scan kernels.
__global__ void __launch_bounds__(kBlock) k_scan_chunks(Geom g, Bufs b) {
    if (!rebuild_requested(b)) return;
    int part = 0;
    for (int k = threadIdx.x; k < (int)blockIdx.x; k += kBlock) part += b.bsum[k * kChunkPad];
    int off;
    (void)block_exclusive_scan(part, off);
    scan_apply_body(g, b, off);
}

// Scatter into cell segments, one atomic per run of equal cells; counts
// return to zero for the next build.  The tags are copied beside the slots
// so that the ranking below reads them contiguously.
__device__ __forceinline__ void scatter_one(const Bufs& b, int64_t i, bool active) {
    const uint32_t c = active ? b.cellid[i] : 0xffffffffu;
    int first, len;
    cell_run(c, active, first, len);
    const int lane = threadIdx.x & 63;
    int top = 0;
    if (active && lane == first) top = atomicSub(&b.ccount[c], len);
    top = __shfl(top, first, 64);
    if (active) {
        // the run owns slots [start + top - len, start + top)
        const int slot = b.cstart[c] + top - len + (lane - first);
        b.tmp[slot] = (int32_t)i;
        b.tsc[slot] = b.tag[i];
    }
}

__global__ void __launch_bounds__(kBlock) k_scatter(Geom g, Bufs b) {
    if (!rebuild_requested(b)) return;
    // the chunk sums were read by the scan: clear them for the next build
    for (int64_t k = gtid(); k < kScanBlocks; k += gstride()) b.bsum[k * kChunkPad] = 0;
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < g.n; i0 += gstride()) {
        const int64_t i = i0 + threadIdx.x;
        scatter_one(b, i, i < g.n);
    }
}

// Order inside a cell by particle tag: the sorted order is then a function
// of the positions alone, so a run resumed from a saved build snapshot
// reproduces it exactly.  Gathers the positions, velocities and images into
// temporaries; the tags, which no thread of this pass reads, go straight to
// their sorted slots.
__device__ __forceinline__ void permute_one(const Geom& g, const Bufs& b, int64_t s, int parity) {
    const int64_t n = g.n;
    {
        int32_t i = b.tmp[s];
        uint32_t c = b.cellid[i];
        int32_t ti = b.tsc[s];
        int st = b.cstart[c], en = b.cstart[c + 1];
        int r = 0;
        int u = st;
        for (; u + 4 <= en; u += 4) {
            const int a0 = b.tsc[u], a1 = b.tsc[u + 1], a2 = b.tsc[u + 2], a3 = b.tsc[u + 3];
            r += (a0 < ti) + (a1 < ti) + (a2 < ti) + (a3 < ti);
        }
        for (; u < en; ++u) r += (b.tsc[u] < ti);
        int64_t nw = st + r;
        // every load before the first store: a load after a store it may
        // alias cannot be moved above it, and would wait in turn
        const double4 p = b.x[parity][i];
        double vv[3];
        int32_t im[3];
        for (int d = 0; d < 3; ++d) {
            vv[d] = b.v[d * n + i];
            im[d] = b.img[d * n + i];
        }
        b.xt[nw] = p;
        for (int d = 0; d < 3; ++d) {
            b.vt[d * n + nw] = vv[d];
            b.imgt[d * n + nw] = im[d];
        }
        b.tag[nw] = ti;
    }
}

__global__ void __launch_bounds__(kBlock) k_rank_permute(Geom g, Bufs b, int parity) {
    if (!rebuild_requested(b)) return;
    for (int64_t s = gtid(); s < g.n; s += gstride()) permute_one(g, b, s, parity);
}

__device__ __forceinline__ void commit_one(const Geom& g, const Bufs& b, int64_t s, int parity, int bonded) {
    const int64_t n = g.n;
    if (s == 0) {
        b.ctl->n_rebuilds += 1;
        b.ctl->nl_max = 0;
        b.ctl->build_step = b.ctl->step;
    }
    {
        // loads first, as in permute_one
        const double4 p = b.xt[s];
        double vv[3];
        int32_t im[3];
        for (int d = 0; d < 3; ++d) {
            vv[d] = b.vt[d * n + s];
            im[d] = b.imgt[d * n + s];
        }
        const int32_t t = bonded ? b.tag[s] : 0;
        b.x[parity][s] = p;
        const int4 q = quantize4(g, p.x, p.y, p.z, p.w);
        b.xq[parity][s] = q;
        if (g.x3_on) store_q3(b.x3[parity], s, q);
        b.xb[s] = p.x;
        b.xb[n + s] = p.y;
        b.xb[2 * n + s] = p.z;
        for (int d = 0; d < 3; ++d) {
            b.v[d * n + s] = vv[d];
            b.img[d * n + s] = im[d];
        }
        // the inverse permutation serves only the bonded remap of the list
        // build, which also copies the per-particle bond and angle counts
        if (bonded) b.inv[t] = (int32_t)s;
    }
}

__global__ void __launch_bounds__(kBlock) k_commit(Geom g, Bufs b, int parity, int bonded) {
    if (!rebuild_requested(b)) return;
    for (int64_t s = gtid(); s < g.n; s += gstride()) commit_one(g, b, s, parity, bonded);
}

// ------------------------------------------------------------------ rebuild: Verlet list

// r_ij^2 in FP64 with the operation order of the plain definition
// ((dx*dx + dy*dy) + dz*dz, no fused multiply-add): the list and cutoff
// decisions taken with it equal those of any implementation doing the same
// IEEE operations on the same positions.
__device__ __forceinline__ double exact_r2(const Geom& g, const double4& a, const double4& b) {
#pragma clang fp contract(off)
    const double dx = mimg(b.x - a.x, g.L[0], g.invL[0]);
    const double dy = mimg(b.y - a.y, g.L[1], g.invL[1]);
    const double dz = mimg(b.z - a.z, g.L[2], g.invL[2]);
    return (dx * dx + dy * dy) + dz * dz;
}

// distance along one axis from a point at offset u inside its cell to the
// cell o cells away
__device__ __forceinline__ float cell_gap(int o, float u, float h) {
    float d = o > 0 ? (float)o * h - u : (o < 0 ? u + (float)(-o - 1) * h : 0.0f);
    return d > 0.0f ? d : 0.0f;
}

__device__ __forceinline__ int wrapc(int c, int nc) { return c < 0 ? c + nc : (c >= nc ? c - nc : c); }

// Bond and angle counts and partners of sorted particle i, partners from
// tags to sorted indices.
__device__ __forceinline__ void remap_bonded(const Bufs& b, int64_t n, int64_t i) {
    const int32_t t = b.tag[i];
    const int tc = b.tcnt_t[t];
    b.tcnt_s[i] = tc;
    const int nb = tc & 0xff, na = tc >> 8;
    for (int k = 0; k < nb; ++k) b.bp_s[(int64_t)k * n + i] = b.inv[b.bp_t[(int64_t)k * n + t]];
    for (int k = 0; k < na; ++k) {
        const int2 e = b.ang_t[(int64_t)k * n + t];
        const int role = (int)((uint32_t)e.x >> 30);
        const int o1 = e.x & 0x3fffffff;
        b.ang_s[(int64_t)k * n + i] = make_int2(b.inv[o1] | (role << 30), b.inv[e.y]);
    }
}

// NL(i) = { j != i : r_ij^2 < rv^2 } over the cells within rv of particle i
// (stencil of (2kc+1)^3 cells of side >= rv/kc, cells farther than rv
// skipped).  The test runs on the fixed-point positions and is retaken in
// FP64 (exact_r2) inside a band around rv that bounds the fixed-point
// rounding, so the sets are those of the FP64 definition.  Row order:
// stencil (z, y, x offsets), then sorted index.  Also remaps the bonded
// topology from tags to sorted indices.
constexpr int kNlLds = 24;  // row slots staged in LDS by the per-particle build (25 KB per block with the spare row)

// Store a group of four tested candidates j0..j0+3 (hits flagged in `in`) to
// a per-particle row: its first kNlLds slots in LDS (buf, [slot][lane] of the
// wavefront, row kNlLds a spare), the rest in the list.  While the next four
// slots lie in LDS every candidate is stored, a miss to the spare row, with
// no branch; past them (LIST_PATH) one masked store per hit; otherwise, and
// for the group that crosses from LDS to the list, the general path.  Hits
// beyond the capacity are counted, not stored.  The list-only path pays where
// rows run well past the LDS slots (the dense fluids of a batch); where rows
// end near them (the sheared DPD fluid, ~28 slots) the lanes split over three
// paths and it cost 11 % of the build, so that build leaves it out.
template <bool LIST_PATH>
__device__ __forceinline__ void nl_store4(int32_t (*buf)[64], int ln, int32_t* __restrict__ nlrow, int cap,
                                          const bool (&in)[4], int j0, int& cnt) {
    if (cnt + 4 <= kNlLds) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            buf[in[u] ? cnt : kNlLds][ln] = j0 + u;
            cnt += in[u] ? 1 : 0;
        }
    } else if (LIST_PATH && cnt >= kNlLds) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (in[u] & (cnt < cap)) nlrow[nl_off(cnt)] = j0 + u;
            cnt += in[u] ? 1 : 0;
        }
    } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (in[u]) {
                if (cnt < cap) {
                    if (cnt < kNlLds) buf[cnt][ln] = j0 + u;
                    else nlrow[nl_off(cnt)] = j0 + u;
                }
                ++cnt;
            }
        }
    }
}
__device__ __forceinline__ void nl_one(const Geom& g, const Bufs& b, int64_t i, int parity, int bonded,
                                       int& local_max, bool& overflow) {
    const int64_t n = g.n;
    const double4* __restrict__ x = b.x[parity];
    const int4* __restrict__ xq = b.xq[parity];
    const float hy = (float)g.h[1], hz = (float)g.h[2];
    const int kc = g.kc;
    {
        const double4 xi = x[i];
        const int4 qi = xq[i];
        int cx, cy, cz;
        cell_coords(g, xi.x, xi.y, xi.z, cx, cy, cz);
        const float uy = (float)(xi.y - cy * g.h[1]);
        const float uz = (float)(xi.z - cz * g.h[2]);
        int cnt = 0;
        const int self = (int)i;
        int32_t* __restrict__ nlrow = b.nl + nl_base(i, g.cap);
        // The first kNlLds slots of each row collect in LDS, [slot][lane] per
        // wavefront, and leave in whole-wavefront stores at the end: the
        // hits of the lanes fall in different iterations, so direct stores
        // would cost one partly masked store instruction per hit event.
        // Row kNlLds is a spare that takes the stores of candidates that miss.
        __shared__ int32_t nlbuf[kBlock / 64][kNlLds + 1][64];
        const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
        auto put = [&](int k, int j) {
            if (k < kNlLds) nlbuf[wv][k][ln] = j;
            else nlrow[nl_off(k)] = j;
        };
        // Cells cx-kc .. cx+kc of one (y, z) row are consecutive in the cell
        // order, so their particles form one contiguous range of the sorted
        // arrays (two when the row wraps around the box).  Candidates are
        // gathered four at a time, the last one repeated past the end of the
        // range, so a short range costs one memory round trip.  The four
        // tests become flags with one branch for the rare FP64 band, and the
        // stores take as few branches as the row's position allows
        // (nl_store4): per-candidate branches cost more scalar and branch
        // issue than the tests themselves.
        auto test_range = [&](int st, int en) {
            for (int j = st; j < en; j += 4) {
                int4 qq[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) qq[u] = xq[min(j + u, en - 1)];
                bool in[4], band[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const float dx = qdiff(qq[u].x, qi.x, g.ql[0]);
                    const float dy = qdiff(qq[u].y, qi.y, g.ql[1]);
                    const float dz = qdiff(qq[u].z, qi.z, g.ql[2]);
                    const float r2 = dx * dx + dy * dy + dz * dz;
                    // bitwise, not short-circuit: no branch around the test
                    const bool ok = (j + u < en) & (j + u != self);
                    in[u] = ok & (r2 < g.rv2lo);
                    band[u] = ok & (r2 >= g.rv2lo) & (r2 < g.rv2hi);
                }
                if (band[0] | band[1] | band[2] | band[3]) {
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        if (band[u]) in[u] = exact_r2(g, xi, x[j + u]) < g.rv2;
                }
                nl_store4<true>(nlbuf[wv], ln, nlrow, g.cap, in, j, cnt);
            }
        };
        const int xlo = cx - kc, xhi = cx + kc;   // inclusive cell range along x
        const int nx = g.nc[0];
        const bool wl = xlo < 0, wh = xhi >= nx;
        const int side = 2 * kc + 1, nv = 2 * side * side;
        const int32_t* __restrict__ cs = b.cstart;
        // Piece v is the first or second range of stencil row v / 2 (rows
        // z-major, empty when the row is out of reach or does not wrap).  The
        // cell bounds of piece v + 1 are loaded before the candidates of
        // piece v are tested, so the two loads overlap.
        auto piece = [&](int v, int& a, int& e) {
            a = e = 0;
            const int r = v >> 1, pc = v & 1;
            const int oz = r / side - kc, oy = r % side - kc;
            const float gz = cell_gap(oz, uz, hz);
            const float gz2 = gz * gz;
            if (gz2 > g.rv2hi) return;
            const float gy = cell_gap(oy, uy, hy);
            if (gz2 + gy * gy > g.rv2hi) return;
            const int nz = wrapc(cz + oz, g.nc[2]), ny = wrapc(cy + oy, g.nc[1]);
            const int64_t rowc = ((int64_t)nz * g.nc[1] + ny) * nx;
            if (!wl && !wh) {
                if (pc == 0) { a = cs[rowc + xlo]; e = cs[rowc + xhi + 1]; }
            } else if (wl) {
                if (pc == 0) { a = cs[rowc + nx + xlo]; e = cs[rowc + nx]; }
                else { a = cs[rowc]; e = cs[rowc + xhi + 1]; }
            } else {
                if (pc == 0) { a = cs[rowc + xlo]; e = cs[rowc + nx]; }
                else { a = cs[rowc]; e = cs[rowc + xhi - nx + 1]; }
            }
        };
        int pa, pe;
        piece(0, pa, pe);
        for (int v = 0; v < nv; ++v) {
            int na = 0, ne = 0;
            if (v + 1 < nv) piece(v + 1, na, ne);
            test_range(pa, pe);
            pa = na;
            pe = ne;
        }
        b.ncount[i] = cnt;
        if (cnt > local_max) local_max = cnt;
        if (cnt > g.cap) overflow = true;
        // pad the row to a multiple of 8 with the particle itself (r = 0,
        // never inside a cutoff) so that step kernels stream whole batches
        const int nslot = min(((cnt + 7) & ~7), g.cap);
        for (int k = cnt; k < nslot; ++k) put(k, (int)i);
#pragma unroll
        for (int k = 0; k < kNlLds; ++k)
            if (k < nslot) nlrow[nl_off(k)] = nlbuf[wv][k][ln];
        if (bonded) remap_bonded(b, n, i);
    }
}

// Longest row and overflow flag.  Atomics on one address serialize (tens of
// ns each, measured), so a wavefront raises the maximum only when its own
// row is longer than the value it reads; a stale read costs one redundant
// atomic, never a wrong maximum.
__device__ __forceinline__ void nl_epilogue(const Bufs& b, int local_max, bool overflow) {
    for (int o = 32; o >= 1; o >>= 1) {
        const int y = __shfl_xor(local_max, o, 64);
        local_max = y > local_max ? y : local_max;
    }
    if ((threadIdx.x & 63) == 0 && local_max > 0) {
        const int cur = __hip_atomic_load(&b.ctl->nl_max, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (local_max > cur) atomicMax(&b.ctl->nl_max, local_max);
    }
    if (__any(overflow) && (threadIdx.x & 63) == 0) atomicOr(&b.ctl->status, MD_FLAG_NL_OVERFLOW);
}

__global__ void __launch_bounds__(kBlock) k_nl_build(Geom g, Bufs b, int parity, int bonded) {
    if (!rebuild_requested(b)) return;
    int local_max = 0;
    bool overflow = false;
    for (int64_t i = gtid_xcd(); i < g.n; i += gstride()) nl_one(g, b, i, parity, bonded, local_max, overflow);
    nl_epilogue(b, local_max, overflow);
}

// The same lists built one wavefront per 64-particle tile of the sorted order
// (the tile of the list layout).  The tile's particles lie in a few
// consecutive cells; lanes of one (y, z) cell row form a segment whose x-cells
// span [x0, x1].  The segment's candidates are the particles of cells
// [x0 - kc, x1 + kc] in each of the (2kc+1)^2 neighbouring rows, streamed in
// nl_one's order (rows z-major, a wrapped x-range high part first, sorted
// index) through the scalar cache: every lane tests every candidate, so there
// are no per-lane gathers.  A candidate outside a lane's own stencil is at
// least kc cell sides >= rv away and never passes the test, and a lane's own
// candidates keep their relative order, so each row equals nl_one's entry for
// entry.  A segment is cut where its x-span plus the stencil would exceed the
// row (no candidate twice).  Cubic boxes prefilter on the upper 16 bits of
// the fixed-point differences with integer r^2 (two 24-bit multiplies of
// sign-extended upper words per axis), with a band that bounds the
// truncation; inside it the 32-bit test and then FP64 decide.
typedef int int4v __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(4))) int4v* __restrict__ scalar_int4_ptr;
typedef const __attribute__((address_space(4))) int32_t* __restrict__ scalar_i32_ptr;

// Row builder state of one lane (one particle of a tile): its fixed-point
// and FP64 position, its row in the tile's list block and the row length.
struct NlRow {
    uint32_t qx, qy, qz;
    double4 xi;
    int self, cnt, cap;
    char* tnlb;          // byte base of the tile's list block (32-bit offsets from it)
    uint32_t lane4;

    // A hit goes to slot min(cnt, cap - 1): an overflowing row overwrites its
    // last slot, and the overflow flag then voids the list.
    __device__ __forceinline__ void hit(int j) {
        const int slot = cnt < cap ? cnt : cap - 1;
        *(uint32_t*)(tnlb + (((uint32_t)slot << 8) | lane4)) = (uint32_t)j;
        ++cnt;
    }

    // Candidate j at fixed-point position qj, counted when ok.  All lanes of
    // the wavefront call it together (the band test is a wavefront mask).
    template <bool CUBIC>
    __device__ __forceinline__ void test(const Geom& g, const double4* __restrict__ x, int j, const int4v qj,
                                         bool ok) {
        const int lane = threadIdx.x & 63;
        if (CUBIC) {
            // 16-bit prefilter: the high halves of the fixed-point differences
            // (24-bit multiplies of the upper words), decided outside a band
            // that bounds its truncation; inside it the 32-bit test, then FP64
            const int32_t ex = (int32_t)((uint32_t)qj.x - qx), ey = (int32_t)((uint32_t)qj.y - qy),
                          ez = (int32_t)((uint32_t)qj.z - qz);
            const int hx = ex >> 16, hy = ey >> 16, hz = ez >> 16;
            const uint32_t r16 = (uint32_t)__mul24(hx, hx) + (uint32_t)__mul24(hy, hy) + (uint32_t)__mul24(hz, hz);
            if (ok && r16 < g.r16lo && j != self) hit(j);
            // lanes with r16 in [lo, hi): one unsigned compare, as a wave mask
            const uint64_t band = __builtin_amdgcn_uicmp(r16 - g.r16lo, g.r16hi - g.r16lo, 36 /* ult */);
            if (__builtin_expect(band != 0, 0)) {
                if (ok && ((band >> lane) & 1)) {
                    const float dx = (float)ex, dy = (float)ey, dz = (float)ez;
                    const float r2 = dx * dx + dy * dy + dz * dz;
                    bool in = r2 < g.rq2lo;
                    if (!in && r2 < g.rq2hi) in = exact_r2(g, xi, x[j]) < g.rv2;
                    if (in && j != self) hit(j);
                }
            }
        } else {
            const float dx = qdiff((uint32_t)qj.x, qx, g.ql[0]);
            const float dy = qdiff((uint32_t)qj.y, qy, g.ql[1]);
            const float dz = qdiff((uint32_t)qj.z, qz, g.ql[2]);
            const float r2 = dx * dx + dy * dy + dz * dz;
            if (ok && r2 < g.rv2lo && j != self) hit(j);
            const uint64_t band = __builtin_amdgcn_uicmp(__float_as_uint(r2) - __float_as_uint(g.rv2lo),
                                                         __float_as_uint(g.rv2hi) - __float_as_uint(g.rv2lo), 36);
            if (__builtin_expect(band != 0, 0)) {
                if (ok && ((band >> lane) & 1) && exact_r2(g, xi, x[j]) < g.rv2 && j != self) hit(j);
            }
        }
    }
};

// Lane setup shared by the tile builds: particle p = t*64 + lane, its cell
// and its row state.
__device__ __forceinline__ NlRow nl_row_setup(const Geom& g, const Bufs& b, int64_t t, int parity, bool valid,
                                              int& cxl, int& cyl, int& czl) {
    const int lane = threadIdx.x & (kTile - 1);
    const int64_t p = t * kTile + lane;
    NlRow r;
    r.qx = r.qy = r.qz = 0;
    r.xi = make_double4(0.0, 0.0, 0.0, 0.0);
    cxl = cyl = czl = -1;
    if (valid) {
        r.xi = b.x[parity][p];
        cell_coords(g, r.xi.x, r.xi.y, r.xi.z, cxl, cyl, czl);
        const int4 q = b.xq[parity][p];
        r.qx = (uint32_t)q.x;
        r.qy = (uint32_t)q.y;
        r.qz = (uint32_t)q.z;
    }
    r.self = (int)p;
    r.cnt = 0;
    r.cap = g.cap;
    r.tnlb = (char*)(b.nl + t * (int64_t)g.cap * kTile);
    r.lane4 = (uint32_t)lane << 2;
    return r;
}

// Row count, padding to a multiple of 8 with the particle itself, and the
// bonded remap.
__device__ __forceinline__ void nl_row_finish(const Geom& g, const Bufs& b, const NlRow& r, bool valid, int bonded,
                                              int& local_max, bool& overflow) {
    if (!valid) return;
    const int64_t p = r.self;
    b.ncount[p] = r.cnt;
    if (r.cnt > local_max) local_max = r.cnt;
    if (r.cnt > g.cap) overflow = true;
    for (int k = r.cnt; k < ((r.cnt + 7) & ~7) && k < g.cap; ++k)
        *(uint32_t*)(r.tnlb + (((uint32_t)k << 8) | r.lane4)) = (uint32_t)p;
    if (bonded) remap_bonded(b, g.n, p);
}

template <bool CUBIC>
__device__ __forceinline__ void nl_tile(const Geom& g, const Bufs& b, int64_t t, int parity, int bonded,
                                        int& local_max, bool& overflow) {
    const int lane = threadIdx.x & (kTile - 1);
    const int64_t n = g.n;
    const int nv = (n - t * kTile < kTile) ? (int)(n - t * kTile) : kTile;
    const bool valid = lane < nv;
    const double4* __restrict__ x = b.x[parity];
    // the particle data are not written by this kernel: uniform loads through
    // the constant address space become scalar loads
    const scalar_int4_ptr xqs = (scalar_int4_ptr)(const void*)b.xq[parity];
    const scalar_i32_ptr cs = (scalar_i32_ptr)(const void*)b.cstart;
    const int kc = g.kc, nx = g.nc[0];
    int cxl, cyl, czl;
    NlRow row = nl_row_setup(g, b, t, parity, valid, cxl, cyl, czl);
    // candidates [j, e) through the scalar cache, 8 and 4 at a time; the
    // next batch of 8 is loaded before the current one is tested, so its
    // scalar-cache latency overlaps the tests (measured: 697 -> 643 us per
    // LJ-1M build)
    auto scan = [&](int j, const int e) {
        if (j + 8 <= e) {
            int4v q[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) q[u] = xqs[j + u];
            for (; j + 16 <= e; j += 8) {
                int4v nq[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) nq[u] = xqs[j + 8 + u];
#pragma unroll
                for (int u = 0; u < 8; ++u) row.test<CUBIC>(g, x, j + u, q[u], true);
#pragma unroll
                for (int u = 0; u < 8; ++u) q[u] = nq[u];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) row.test<CUBIC>(g, x, j + u, q[u], true);
            j += 8;
        }
        for (; j + 4 <= e; j += 4) {
            const int4v q0 = xqs[j], q1 = xqs[j + 1], q2 = xqs[j + 2], q3 = xqs[j + 3];
            row.test<CUBIC>(g, x, j, q0, true);
            row.test<CUBIC>(g, x, j + 1, q1, true);
            row.test<CUBIC>(g, x, j + 2, q2, true);
            row.test<CUBIC>(g, x, j + 3, q3, true);
        }
        for (; j < e; ++j) row.test<CUBIC>(g, x, j, xqs[j], true);
    };
    int lo = 0;
    while (lo < nv) {
        const int x0 = __builtin_amdgcn_readlane(cxl, lo);
        const int y0 = __builtin_amdgcn_readlane(cyl, lo);
        const int z0 = __builtin_amdgcn_readlane(czl, lo);
        const int xlim = x0 + nx - 2 * kc - 1;
        const int hi = lo + (int)__popcll(__ballot(valid && lane >= lo && cyl == y0 && czl == z0 && cxl <= xlim));
        const int x1 = __builtin_amdgcn_readlane(cxl, hi - 1);
        if (lane >= lo && lane < hi) {
            const int xa = x0 - kc, xb = x1 + kc;
            const bool wl = xa < 0, wh = xb >= nx;
            const int side = 2 * kc + 1, np = 2 * side * side;
            // piece p: the first or second range of stencil row p / 2 (rows
            // z-major); the next piece's bounds are loaded before the
            // current piece is scanned
            auto piece = [&](int p, int& a, int& e) {
                a = e = 0;
                const int r = p >> 1, pc = p & 1;
                const int nz = wrapc(z0 + r / side - kc, g.nc[2]), ny = wrapc(y0 + r % side - kc, g.nc[1]);
                const int64_t rowc = ((int64_t)nz * g.nc[1] + ny) * nx;
                if (!wl && !wh) {
                    if (pc == 0) { a = cs[rowc + xa]; e = cs[rowc + xb + 1]; }
                } else if (wl) {
                    if (pc == 0) { a = cs[rowc + nx + xa]; e = cs[rowc + nx]; }
                    else { a = cs[rowc]; e = cs[rowc + xb + 1]; }
                } else {
                    if (pc == 0) { a = cs[rowc + xa]; e = cs[rowc + nx]; }
                    else { a = cs[rowc]; e = cs[rowc + xb - nx + 1]; }
                }
            };
            int pa, pe;
            piece(0, pa, pe);
            for (int p = 0; p < np; ++p) {
                int na = 0, ne = 0;
                if (p + 1 < np) piece(p + 1, na, ne);
                scan(pa, pe);
                pa = na;
                pe = ne;
            }
        }
        lo = hi;
    }
    nl_row_finish(g, b, row, valid, bonded, local_max, overflow);
}

constexpr int kNlBlock = kBlock;
__global__ void __launch_bounds__(kNlBlock) k_nl_tiles(Geom g, Bufs b, int parity, int bonded) {
    if (!rebuild_requested(b)) return;
    // wave-uniform tile index (readfirstlane keeps it in scalar registers)
    const int64_t t = (int64_t)xcd_block(blockIdx.x, gridDim.x) * (kNlBlock / kTile) +
                      __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kTile));
    int local_max = 0;
    bool overflow = false;
    if (t * kTile < g.n) {
        if (g.nl_cubic) nl_tile<true>(g, b, t, parity, bonded, local_max, overflow);
        else nl_tile<false>(g, b, t, parity, bonded, local_max, overflow);
    }
    nl_epilogue(b, local_max, overflow);
}

// ------------------------------------------------------------------ Lees-Edwards shear
//
// Flow along x, gradient along y (section "New Features": Lees-Edwards
// boundary conditions).  The image one box above is displaced by
// delta(step) = fmod(shear_rate Ly (step dt), Lx) and moves with
// +shear_rate Ly along x.  Minimum image of d = r_j - r_i: dy by
// compare-and-shift, s = +1 when dy > Ly/2 (j's nearest image lies one box
// below: x_j - delta), -1 when dy < -Ly/2; dx = the x minimum image of
// x_j - x_i, then for s != 0 the x minimum image of dx - s delta_w
// (delta_w = delta folded into (-Lx/2, Lx/2]).  FP64 operations in that
// order, so list and cutoff decisions equal any implementation doing the
// same operations.

__device__ __forceinline__ double le_delta(const Geom& g, int64_t step) {
    double d = fmod(g.le_rate_Ly * ((double)step * g.le_dt), g.L[0]);
    return d < 0.0 ? d + g.L[0] : d;
}
__device__ __forceinline__ double le_fold(const Geom& g, double d) { return d > g.hL[0] ? d - g.L[0] : d; }

__device__ __forceinline__ double exact_r2_le(const Geom& g, const double4& a, const double4& b, double dw) {
#pragma clang fp contract(off)
    double dy = b.y - a.y;
    int sy = 0;
    if (dy > g.hL[1]) { dy -= g.L[1]; sy = 1; }
    else if (dy < -g.hL[1]) { dy += g.L[1]; sy = -1; }
    double dx = mimg(b.x - a.x, g.L[0], g.invL[0]);
    if (sy != 0) dx = mimg(dx - sy * dw, g.L[0], g.invL[0]);
    const double dz = mimg(b.z - a.z, g.L[2], g.invL[2]);
    return (dx * dx + dy * dy) + dz * dz;
}

// Sign s of the sheared image from the fixed-point y coordinates: the raw
// difference beyond half the box (2^31 units).
__device__ __forceinline__ int le_sign_q(uint32_t qiy, uint32_t qjy) {
    const int64_t d = (int64_t)qjy - (int64_t)qiy;
    return d > 0x80000000LL ? 1 : (d < -0x80000000LL ? -1 : 0);
}

// Fixed-point differences r_j - r_i under the shear (qd = the offset delta in
// units of Lx 2^-32); s as above.
struct DiffLEQ {
    float l0, l1, l2;
    uint32_t qd;
    __device__ int operator()(const int4& a, const int4& b, float& dx, float& dy, float& dz) const {
        const int s = le_sign_q((uint32_t)a.y, (uint32_t)b.y);
        dx = (float)(int32_t)((uint32_t)b.x - (uint32_t)a.x - (uint32_t)(s * (int64_t)qd)) * l0;
        dy = qdiff(b.y, a.y, l1);
        dz = qdiff(b.z, a.z, l2);
        return s;
    }
};

// NL(i) under the shear, one particle per lane: as nl_one, except that a
// stencil row reached across the y boundary (s != 0) scans the x cells
// around x_i + s delta (one cell of margin each side, the whole row when that
// covers it).  Rows are in stencil order; sets equal the FP64 definition.
__device__ __forceinline__ void nl_one_le(const Geom& g, const Bufs& b, int64_t i, int parity, int bonded,
                                          double delta, double dw, uint32_t qd, int& local_max, bool& overflow) {
    const int64_t n = g.n;
    const double4* __restrict__ x = b.x[parity];
    const int4* __restrict__ xq = b.xq[parity];
    const int kc = g.kc, nx = g.nc[0];
    const double4 xi = x[i];
    const int4 qi = xq[i];
    int cx, cy, cz;
    cell_coords(g, xi.x, xi.y, xi.z, cx, cy, cz);
    const float uy = (float)(xi.y - cy * g.h[1]);
    const float uz = (float)(xi.z - cz * g.h[2]);
    const DiffLEQ df{g.ql[0], g.ql[1], g.ql[2], qd};
    int32_t* __restrict__ nlrow = b.nl + nl_base(i, g.cap);
    int cnt = 0;
    // the first kNlLds slots collect in LDS, [slot][lane] per wavefront, and
    // leave in whole-wavefront stores at the end (as in the plain build)
    // (row kNlLds is the spare of the misses, as there)
    __shared__ int32_t nlbuf_le[kBlock / 64][kNlLds + 1][64];
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
    const int self = (int)i;
    auto put = [&](int k, int j) {
        if (k < kNlLds) nlbuf_le[wv][k][ln] = j;
        else nlrow[nl_off(k)] = j;
    };
    // candidates gathered four at a time, the last one repeated past the end
    // of the range; tests as flags and stores as in the plain build
    auto test_range = [&](int st, int en) {
        for (int j0 = st; j0 < en; j0 += 4) {
            int4 qq[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) qq[u] = xq[min(j0 + u, en - 1)];
            bool in[4], band[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                float dx, dy, dz;
                df(qi, qq[u], dx, dy, dz);
                const float r2 = dx * dx + dy * dy + dz * dz;
                const bool ok = (j0 + u < en) & (j0 + u != self);
                in[u] = ok & (r2 < g.rv2lo);
                band[u] = ok & (r2 >= g.rv2lo) & (r2 < g.rv2hi);
            }
            if (band[0] | band[1] | band[2] | band[3]) {
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (band[u]) in[u] = exact_r2_le(g, xi, x[j0 + u], dw) < g.rv2;
            }
            nl_store4<false>(nlbuf_le[wv], ln, nlrow, g.cap, in, j0, cnt);
        }
    };
    // Piece v is the first or second contiguous range of stencil row v / 2
    // (rows z-major; empty when the row is out of reach or does not wrap).
    // Across the y-boundary the row's x-range is re-centred on x_i +- delta
    // with one cell of margin each side (the whole row when that covers it).
    // The bounds of piece v + 1 are loaded before piece v is tested.
    const int32_t* __restrict__ cs = b.cstart;
    const int side = 2 * kc + 1, nv = 2 * side * side;
    const double rv = sqrt(g.rv2);
    auto piece = [&](int v, int& a, int& e) {
        a = e = 0;
        const int r = v >> 1, pc = v & 1;
        const int oz = r / side - kc, oy = r % side - kc;
        const float gz = cell_gap(oz, uz, (float)g.h[2]);
        if (gz * gz > g.rv2hi) return;
        const float gy = cell_gap(oy, uy, (float)g.h[1]);
        if (gz * gz + gy * gy > g.rv2hi) return;
        const int nz = wrapc(cz + oz, g.nc[2]);
        const int yraw = cy + oy;
        const int sh = yraw < 0 ? 1 : (yraw >= g.nc[1] ? -1 : 0);
        const int ny = wrapc(yraw, g.nc[1]);
        const int64_t rowc = ((int64_t)nz * g.nc[1] + ny) * nx;
        int lo = cx - kc, hi = cx + kc;
        if (sh != 0) {
            const double c0 = xi.x + sh * delta;
            lo = (int)floor((c0 - rv) * g.invh[0]) - 1;
            hi = (int)floor((c0 + rv) * g.invh[0]) + 1;
        }
        if (hi - lo + 1 >= nx) {
            if (pc == 0) { a = cs[rowc]; e = cs[rowc + nx]; }
            return;
        }
        // [lo, hi] modulo nx: one or two contiguous ranges of cells
        const int l = ((lo % nx) + nx) % nx;
        const int h = l + (hi - lo);
        if (h < nx) {
            if (pc == 0) { a = cs[rowc + l]; e = cs[rowc + h + 1]; }
        } else if (pc == 0) {
            a = cs[rowc + l]; e = cs[rowc + nx];
        } else {
            a = cs[rowc]; e = cs[rowc + h - nx + 1];
        }
    };
    int pa, pe;
    piece(0, pa, pe);
    for (int v = 0; v < nv; ++v) {
        int na = 0, ne = 0;
        if (v + 1 < nv) piece(v + 1, na, ne);
        test_range(pa, pe);
        pa = na;
        pe = ne;
    }
    b.ncount[i] = cnt;
    if (cnt > local_max) local_max = cnt;
    if (cnt > g.cap) overflow = true;
    const int nslot = min(((cnt + 7) & ~7), g.cap);
    for (int k = cnt; k < nslot; ++k) put(k, (int)i);
#pragma unroll
    for (int k = 0; k < kNlLds; ++k)
        if (k < nslot) nlrow[nl_off(k)] = nlbuf_le[wv][k][ln];
    if (bonded) remap_bonded(b, n, i);
}

__global__ void __launch_bounds__(kBlock) k_nl_build_le(Geom g, Bufs b, int parity, int bonded) {
    if (!rebuild_requested(b)) return;
    const double delta = le_delta(g, b.ctl->step);
    const double dw = le_fold(g, delta);
    const uint32_t qd = quantize(delta, g.qs[0]);
    int local_max = 0;
    bool overflow = false;
    for (int64_t i = gtid_xcd(); i < g.n; i += gstride())
        nl_one_le(g, b, i, parity, bonded, delta, dw, qd, local_max, overflow);
    nl_epilogue(b, local_max, overflow);
}

__global__ void k_clear_rebuild(Bufs b) {
    if (threadIdx.x == 0 && blockIdx.x == 0) b.ctl->rebuild = 0;
}

// ------------------------------------------------------------------ bonded forces

// Coordinate differences b - a for the two position formats.
struct DiffQ {
    float l0, l1, l2;
    __device__ void operator()(const int4& a, const int4& b, float& dx, float& dy, float& dz) const {
        dx = qdiff(b.x, a.x, l0);
        dy = qdiff(b.y, a.y, l1);
        dz = qdiff(b.z, a.z, l2);
    }
};
struct Diff64 {
    double L0, L1, L2, i0, i1, i2;
    __device__ void operator()(const double4& a, const double4& b, double& dx, double& dy, double& dz) const {
        dx = mimg(b.x - a.x, L0, i0);
        dy = mimg(b.y - a.y, L1, i1);
        dz = mimg(b.z - a.z, L2, i2);
    }
};

__device__ __forceinline__ void add_tensor(double* acc, double s, double rx, double ry, double rz, double fx,
                                           double fy, double fz) {
    acc[A_TXX] += s * rx * fx;
    acc[A_TYY] += s * ry * fy;
    acc[A_TZZ] += s * rz * fz;
    acc[A_TXY] += s * 0.5 * (rx * fy + ry * fx);
    acc[A_TXZ] += s * 0.5 * (rx * fz + rz * fx);
    acc[A_TYZ] += s * 0.5 * (ry * fz + rz * fy);
}

// FENE bonds and cosine bending angles acting on particle i, from its own
// rows of the sorted-space topology.  Each bond is evaluated by both ends
// (half the energy each), each angle by its three members (energy counted
// by the centre); no atomics.
// EXT (the generic FP32 kernel): the angle kinds MD_ANGLE_COSINE_SQUARED
// and MD_ANGLE_TABULATED besides the cosine bending, through
// dU/dcos(theta), theta = pi - phi the angle between b1 and b2.
template <typename Real, typename P, typename Diff, bool EXT = false>
__device__ __forceinline__ void bonded_forces(const Bufs& b, const Dyn& dyn, int64_t n, int64_t i,
                                              const P* __restrict__ xs, const P& pi, const Diff& diff,
                                              Real& fx, Real& fy, Real& fz, double* acc, bool tensor,
                                              bool& flag_bond) {
    const bool f64 = sizeof(Real) == 8;
    const int tc = b.tcnt_s[i];
    const int nb = tc & 0xff, na = tc >> 8;
    const Real K = f64 ? (Real)dyn.fene_K : (Real)dyn.fene_Kf;
    const Real R02 = f64 ? (Real)dyn.fene_R02 : (Real)dyn.fene_R02f;
    const Real hKR02 = f64 ? (Real)dyn.fene_halfKR02 : (Real)dyn.fene_halfKR02f;
    // The first kPreB bonds and kPreA angles (all of a linear chain's) load
    // their partner indices together and then gather the partners' records
    // together: two memory round trips instead of two per term.  Rows past a
    // particle's own counts hold no partner, so those gathers read the
    // particle itself and their terms are skipped; the terms are summed in
    // the same order as before.
    constexpr int kPreB = 2, kPreA = 3;
    int mb[kPreB];
    int2 ex[kPreA];
#pragma unroll
    for (int q = 0; q < kPreB; ++q) mb[q] = q < b.maxb ? b.bp_s[(int64_t)q * n + i] : 0;
#pragma unroll
    for (int q = 0; q < kPreA; ++q) ex[q] = q < b.maxa ? b.ang_s[(int64_t)q * n + i] : make_int2(0, 0);
    P pbq[kPreB], pa1[kPreA], pa2[kPreA];
#pragma unroll
    for (int q = 0; q < kPreB; ++q) pbq[q] = xs[q < nb ? mb[q] : (int)i];
#pragma unroll
    for (int q = 0; q < kPreA; ++q) {
        pa1[q] = xs[q < na ? (ex[q].x & 0x3fffffff) : (int)i];
        pa2[q] = xs[q < na ? ex[q].y : (int)i];
    }
    Real eb = 0, wb = 0;
    auto bond = [&](const P& pm) {
        Real dx, dy, dz;
        diff(pi, pm, dx, dy, dz);                    // x_m - x_i
        const Real rx = -dx, ry = -dy, rz = -dz;     // r_i - r_m
        const Real r2 = rx * rx + ry * ry + rz * rz;
        const Real qq = r2 / R02;
        if (!(qq < Real(1))) {
            flag_bond = true;
            return;
        }
        const Real om = Real(1) - qq;
        const Real fr = -K / om;
        fx += fr * rx;
        fy += fr * ry;
        fz += fr * rz;
        eb += -hKR02 * logr<Real>(om);
        wb += fr * r2;
        if (tensor) add_tensor(acc, 0.5, rx, ry, rz, fr * rx, fr * ry, fr * rz);
    };
#pragma unroll
    for (int q = 0; q < kPreB; ++q)
        if (q < nb) bond(pbq[q]);
    for (int q = kPreB; q < nb; ++q) bond(xs[b.bp_s[(int64_t)q * n + i]]);
    acc[A_EBOND] += 0.5 * (double)eb;
    acc[A_VIR] += 0.5 * (double)wb;
    const Real kb = f64 ? (Real)dyn.k_bend : (Real)dyn.k_bendf;
    Real ea = 0, wa = 0;
    auto angle = [&](const int2 e, const P& p1, const P& p2) {
        const int role = (int)((uint32_t)e.x >> 30);
        // members (A, B, C), B the centre; i is the one named by role
        const P& pa = role == 0 ? pi : p1;
        const P& pb = role == 1 ? pi : (role == 0 ? p1 : p2);
        const P& pc = role == 2 ? pi : p2;
        Real b1x, b1y, b1z, b2x, b2y, b2z;
        diff(pa, pb, b1x, b1y, b1z);                 // b1 = x_B - x_A
        diff(pb, pc, b2x, b2y, b2z);                 // b2 = x_C - x_B
        const Real l1sq = b1x * b1x + b1y * b1y + b1z * b1z;
        const Real l2sq = b2x * b2x + b2y * b2y + b2z * b2z;
        const Real il1l2 = rsq<Real>(l1sq * l2sq);
        const Real cs = (b1x * b2x + b1y * b2y + b1z * b2z) * il1l2;
        const Real i1 = rcp<Real>(l1sq), i2 = rcp<Real>(l2sq);
        Real Fx, Fy, Fz;
        if (EXT && dyn.angle_kind != MD_ANGLE_COSINE) {
            // dUdc = dU/dcos(theta); cos(phi) = -cs
            Real dUdc, ua;
            if (dyn.angle_kind == MD_ANGLE_COSINE_SQUARED) {
                const Real d = -cs - (Real)dyn.cos_phi0;
                ua = (Real)dyn.angle_K * d * d;
                dUdc = Real(-2) * (Real)dyn.angle_K * d;
            } else {
                const float cphi = (float)(-cs > Real(1) ? Real(1) : (-cs < Real(-1) ? Real(-1) : -cs));
                const float phi = acosf(cphi);
                const float q = phi * dyn.ang_idphi;
                int k = (int)q;
                k = k > dyn.ang_n - 2 ? dyn.ang_n - 2 : k;
                const float al = q - (float)k;
                const float2 t0 = dyn.ang_tab[k], t1 = dyn.ang_tab[k + 1];
                ua = (Real)((1.f - al) * t0.x + al * t1.x);
                const float gphi = (1.f - al) * t0.y + al * t1.y;       // du/dphi
                const float sn = sinf(phi);
                dUdc = (Real)(gphi / (sn > 1e-8f ? sn : 1e-8f));        // dU/dcos(theta) = -dU/dcos(phi)
            }
            const Real dA0 = b2x * il1l2 - cs * b1x * i1, dA1 = b2y * il1l2 - cs * b1y * i1,
                       dA2 = b2z * il1l2 - cs * b1z * i1;          // dcos/db1
            const Real dC0 = b1x * il1l2 - cs * b2x * i2, dC1 = b1y * il1l2 - cs * b2y * i2,
                       dC2 = b1z * il1l2 - cs * b2z * i2;          // dcos/db2
            if (role == 0) {
                Fx = dUdc * dA0; Fy = dUdc * dA1; Fz = dUdc * dA2;
                wa += -(b1x * Fx + b1y * Fy + b1z * Fz);
                if (tensor) add_tensor(acc, 1.0, -b1x, -b1y, -b1z, Fx, Fy, Fz);
            } else if (role == 2) {
                Fx = -dUdc * dC0; Fy = -dUdc * dC1; Fz = -dUdc * dC2;
                wa += b2x * Fx + b2y * Fy + b2z * Fz;
                if (tensor) add_tensor(acc, 1.0, b2x, b2y, b2z, Fx, Fy, Fz);
            } else {
                Fx = -(dUdc * dA0 - dUdc * dC0);
                Fy = -(dUdc * dA1 - dUdc * dC1);
                Fz = -(dUdc * dA2 - dUdc * dC2);
                ea += ua;
            }
        } else if (role == 0) {          // F_A = -k dcos/db1
            Fx = -kb * (b2x * il1l2 - cs * b1x * i1);
            Fy = -kb * (b2y * il1l2 - cs * b1y * i1);
            Fz = -kb * (b2z * il1l2 - cs * b1z * i1);
            wa += -(b1x * Fx + b1y * Fy + b1z * Fz);                 // (x_A - x_B) . F_A
            if (tensor) add_tensor(acc, 1.0, -b1x, -b1y, -b1z, Fx, Fy, Fz);
        } else if (role == 2) {   // F_C = k dcos/db2
            Fx = kb * (b1x * il1l2 - cs * b2x * i2);
            Fy = kb * (b1y * il1l2 - cs * b2y * i2);
            Fz = kb * (b1z * il1l2 - cs * b2z * i2);
            wa += b2x * Fx + b2y * Fy + b2z * Fz;                    // (x_C - x_B) . F_C
            if (tensor) add_tensor(acc, 1.0, b2x, b2y, b2z, Fx, Fy, Fz);
        } else {                  // F_B = -(F_A + F_C)
            Fx = kb * ((b2x * il1l2 - cs * b1x * i1) - (b1x * il1l2 - cs * b2x * i2));
            Fy = kb * ((b2y * il1l2 - cs * b1y * i1) - (b1y * il1l2 - cs * b2y * i2));
            Fz = kb * ((b2z * il1l2 - cs * b1z * i1) - (b1z * il1l2 - cs * b2z * i2));
            ea += kb * (Real(1) - cs);
        }
        fx += Fx;
        fy += Fy;
        fz += Fz;
    };
#pragma unroll
    for (int q = 0; q < kPreA; ++q)
        if (q < na) angle(ex[q], pa1[q], pa2[q]);
    for (int q = kPreA; q < na; ++q) {
        const int2 e = b.ang_s[(int64_t)q * n + i];
        angle(e, xs[e.x & 0x3fffffff], xs[e.y]);
    }
    acc[A_EANGLE] += (double)ea;
    acc[A_VIR] += (double)wa;
}

// ------------------------------------------------------------------ integration

// Velocity Verlet with the Langevin force for one particle (MODE_STEP), or
// only the on-step kinetic energy (MODE_OBSERVE / MODE_FORCES):
//   F_tot   = F(x_n) [- gamma m v' + sqrt(2 gamma m kT/dt) xi_n]
//   v_n     = v' + dt/(2m) F_tot          (v_n = v' before the first step)
//   v_{n+h} = v_n + dt/(2m) F_tot,  x_{n+1} = x_n + dt v_{n+h}, wrapped
// plus the half-skin displacement test against the build positions.
// Lees-Edwards data of one step: the offset at the new positions' step and
// the offset's change since the list was built (the rebuild criterion).
struct LeStep {
    double delta_next;     // delta(step + 1) in [0, Lx)
    double drift;          // |shear_rate Ly (step + 1 - build_step) dt|
};

__device__ __forceinline__ void finish_particle(const StepArgs& a, int64_t i, const double4& xi, int tm,
                                               const double F[3], double* acc, bool& flag_reb,
                                               bool& flag_nf, const LeStep* le = nullptr) {
    const Geom& g = a.g;
    const Bufs& b = a.b;
    const int64_t n = g.n;
    const double hdtm = a.dy.hdtm[tm];
    const double m = a.dy.mass[tm];
    double vp[3], ft[3], xbv[3];
    for (int d = 0; d < 3; ++d) vp[d] = b.v[d * n + i];
    // the build positions load with the velocities: read after the velocity
    // stores below, each would wait on its own round trip (the compiler cannot
    // move a load above a store it may alias)
    if (a.mode == MODE_STEP)
        for (int d = 0; d < 3; ++d) xbv[d] = b.xb[d * n + i];
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
        ft[0] = F[0];
        ft[1] = F[1];
        ft[2] = F[2];
    }
    const bool vh_in = b.ctl->vel_half != 0;
    double von[3], ke = 0.0;
    for (int d = 0; d < 3; ++d) {
        von[d] = vh_in ? vp[d] + hdtm * ft[d] : vp[d];
        ke += von[d] * von[d];
    }
    acc[A_EKIN] += 0.5 * m * ke;
    if (a.mode == MODE_STEP && le) {
        // sheared boundaries: crossing y = Ly (y = 0) shifts x by -delta (+delta)
        // and v_x by -shear_rate Ly (+), before the x fold; the build position
        // moves with the particle, so the displacement stays the physical one
        double xn[3], vh[3];
        for (int d = 0; d < 3; ++d) {
            vh[d] = von[d] + hdtm * ft[d];
            xn[d] = (d == 0 ? xi.x : d == 1 ? xi.y : xi.z) + a.dy.dt * vh[d];
        }
        int sc = 0;
        if (xn[1] >= g.L[1]) { xn[1] -= g.L[1]; xn[0] -= le->delta_next; vh[0] -= g.le_rate_Ly; sc = 1; }
        else if (xn[1] < 0.0) { xn[1] += g.L[1]; xn[0] += le->delta_next; vh[0] += g.le_rate_Ly; sc = -1; }
        if (sc != 0) {
            b.img[n + i] += sc;
            xbv[0] -= sc * le->delta_next;
            b.xb[i] = xbv[0];
        }
        double d2 = 0.0;
        for (int d = 0; d < 3; ++d) {
            if (xn[d] < 0.0 || xn[d] >= g.L[d]) {
                int im = b.img[d * n + i];
                if (xn[d] < 0.0) { xn[d] += g.L[d]; im -= 1; }
                if (xn[d] >= g.L[d]) { xn[d] -= g.L[d]; im += 1; }
                b.img[d * n + i] = im;
            }
            if (!isfinite(xn[d]) || !isfinite(vh[d])) flag_nf = true;
            b.v[d * n + i] = vh[d];
            const double dd = mimg(xn[d] - xbv[d], g.L[d], g.invL[d]);
            d2 += dd * dd;
        }
        // a pair's separation changes by at most both displacements plus the
        // offset's change since the build: rebuild before that reaches the skin
        if (2.0 * sqrt(d2) + le->drift >= g.skin) flag_reb = true;
        b.x[a.parity ^ 1][i] = make_double4(xn[0], xn[1], xn[2], xi.w);
        const int4 qn = quantize4(g, xn[0], xn[1], xn[2], xi.w);
        b.xq[a.parity ^ 1][i] = qn;
        if (g.x3_on) store_q3(b.x3[a.parity ^ 1], i, qn);
    } else if (a.mode == MODE_STEP) {
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
            if (!isfinite(xn) || !isfinite(vh)) flag_nf = true;
            xo[d] = xn;
            b.v[d * n + i] = vh;
            const double dd = mimg(xn - xbv[d], g.L[d], g.invL[d]);
            d2 += dd * dd;
        }
        if (d2 > g.disp2) flag_reb = true;
        b.x[a.parity ^ 1][i] = make_double4(xo[0], xo[1], xo[2], xi.w);
        const int4 qn = quantize4(g, xo[0], xo[1], xo[2], xi.w);
        b.xq[a.parity ^ 1][i] = qn;
        if (g.x3_on) store_q3(b.x3[a.parity ^ 1], i, qn);
    } else if (a.mode == MODE_FORCES && a.f_out) {
        a.f_out[3 * (int64_t)tg] = F[0];
        a.f_out[3 * (int64_t)tg + 1] = F[1];
        a.f_out[3 * (int64_t)tg + 2] = F[2];
    }
}

// Flags (one store or atomic per wave) and the deterministic block
// reduction of the per-particle sums into partials[k][block]; BS threads per
// block.
template <int BS = kBlock>
__device__ __forceinline__ void block_epilogue(const StepArgs& a, const double* acc, bool flag_reb,
                                              bool flag_bond, bool flag_nf, int nacc, int64_t slot = -1,
                                              int64_t nslots = 0) {
    if (slot < 0) {
        slot = blockIdx.x;
        nslots = gridDim.x;
    }
    const Bufs& b = a.b;
    const bool any_reb = __any(flag_reb);
    const bool any_bond = __any(flag_bond);
    const bool any_nf = __any(flag_nf);
    if ((threadIdx.x & 63) == 0) {
        // Stores to one address from many wavefronts serialize, and under a
        // drifting sheared image nearly every wavefront of a step can ask for
        // the rebuild, so a wavefront sets the flag only when it reads it
        // clear; a stale read costs one redundant store, never a lost request.
        if (any_reb && __hip_atomic_load(&b.ctl->rebuild_next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u)
            __atomic_store_n(&b.ctl->rebuild_next, 1u, __ATOMIC_RELAXED);
        if (any_bond) atomicOr(&b.ctl->status, MD_FLAG_BOND_BROKEN);
        if (any_nf) atomicOr(&b.ctl->status, MD_FLAG_NONFINITE);
    }
    __shared__ double red[BS / 64][kNacc];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int q = 0; q < nacc; ++q) {
        const double s = wave_sum(acc[q]);
        if (lane == 0) red[w][q] = s;
    }
    __syncthreads();
    if (threadIdx.x < kNacc) {
        double s = 0.0;
        if ((int)threadIdx.x < nacc)
            for (int ww = 0; ww < BS / 64; ++ww) s += red[ww][threadIdx.x];
        b.partials[(int64_t)threadIdx.x * nslots + slot] = s;
    }
}

// ------------------------------------------------------------------ step kernels

// FP64 pair path: FP64 positions gathered from the double-buffered double4
// array, all pair and bonded math in FP64.
template <bool SINGLE, bool BONDED>
__global__ void __launch_bounds__(kBlock) k_step64(const StepArgs a) {
    const Geom& g = a.g;
    const Bufs& b = a.b;
    const int64_t n = g.n;
    const double4* __restrict__ xin = b.x[a.parity];
    double acc[kNacc];
#pragma unroll
    for (int k = 0; k < kNacc; ++k) acc[k] = 0.0;
    bool flag_reb = false, flag_bond = false, flag_nf = false;
    const bool tensor = a.tensor != 0;
    const int64_t ntile = (n + kBlock - 1) / kBlock;
    const int64_t bt = xcd_block(blockIdx.x, gridDim.x);
    for (int64_t t = bt * ntile / gridDim.x; t < (bt + 1) * ntile / gridDim.x; ++t) {
    const int64_t i = t * kBlock + threadIdx.x;
    if (i < n) {
        const double4 xi = xin[i];
        const int ti = SINGLE ? 0 : (int)xi.w;
        double fx = 0, fy = 0, fz = 0, ui = 0, wi = 0;
        int cnt = b.ncount[i];
        cnt = cnt < g.cap ? cnt : g.cap;
        const int32_t* __restrict__ row = b.nl + nl_base(i, g.cap);
        for (int k = 0; k < cnt; ++k) {
            const double4 xj = xin[row[nl_off(k)]];
            const double dx = mimg(xj.x - xi.x, g.L[0], g.invL[0]);
            const double dy = mimg(xj.y - xi.y, g.L[1], g.invL[1]);
            const double dz = mimg(xj.z - xi.z, g.L[2], g.invL[2]);
            const double r2 = dx * dx + dy * dy + dz * dz;
            const int tp = SINGLE ? 0 : ti * MD_MAX_TYPES + (int)xj.w;
            if (exact_r2(g, xi, xj) < a.pt.rc2d[tp]) {
                const PairCoef<double>& c = a.pt.d[tp];
                double fr, u;
                if (c.cap2 > 0.0 && r2 < c.cap2) {
                    fr = c.fcap / sqrt(r2);
                    u = c.ucap;
                } else {
                    const double inv = 1.0 / r2;
                    const double s2 = c.sig2 * inv;
                    const double s6 = s2 * s2 * s2;
                    fr = c.eps24 * s6 * (2.0 * s6 - 1.0) * inv;
                    u = c.eps4 * s6 * (s6 - 1.0) - c.shift;
                }
                fx -= fr * dx;
                fy -= fr * dy;
                fz -= fr * dz;
                ui += u;
                wi += fr * r2;
                if (tensor) add_tensor(acc, 0.5, -dx, -dy, -dz, -fr * dx, -fr * dy, -fr * dz);
            }
        }
        acc[A_EPAIR] += 0.5 * ui;
        acc[A_VIR] += 0.5 * wi;
        if (BONDED) {
            const Diff64 df{g.L[0], g.L[1], g.L[2], g.invL[0], g.invL[1], g.invL[2]};
            bonded_forces<double, double4, Diff64>(b, a.dy, n, i, xin, xi, df, fx, fy, fz, acc, tensor, flag_bond);
        }
        const double F[3] = {fx, fy, fz};
        finish_particle(a, i, xi, SINGLE ? 0 : ti, F, acc, flag_reb, flag_nf);
    }
    }
    block_epilogue(a, acc, flag_reb, flag_bond, flag_nf, tensor ? kNacc : A_VIR + 1);
}

// FP32 pair path.  Neighbours are gathered as 16-byte fixed-point records;
// dx = (int32)(q_j - q_i) * L/2^32 is the minimum image with no branch and
// an absolute error of a few 1e-8; the pair and bonded math is FP32.  A
// cutoff decision inside the rounding band around rc is retaken in FP64
// from the FP64 positions, so the set of interacting pairs is that of the
// FP64 definition.  Neighbour indices are loaded one batch of 8 ahead of
// the gathers that use them.
template <bool SINGLE, bool BONDED, bool TENSOR>
__global__ void __launch_bounds__(kBlock) k_step_q(const StepArgs a) {
    const Geom& g = a.g;
    const Bufs& b = a.b;
    const int64_t n = g.n;
    const int4* __restrict__ xq = b.xq[a.parity];
    const double4* __restrict__ x64 = b.x[a.parity];
    double acc[kNacc];
#pragma unroll
    for (int k = 0; k < kNacc; ++k) acc[k] = 0.0;
    bool flag_reb = false, flag_bond = false, flag_nf = false;
    const int64_t ntile = (n + kBlock - 1) / kBlock;
    const int64_t bt = xcd_block(blockIdx.x, gridDim.x);
    for (int64_t t = bt * ntile / gridDim.x; t < (bt + 1) * ntile / gridDim.x; ++t) {
    const int64_t i = t * kBlock + threadIdx.x;
    if (i < n) {
        const double4 xi = x64[i];
        const int4 qi = quantize4(g, xi.x, xi.y, xi.z, xi.w);  // equals xq[i]: same function
        const int ti = SINGLE ? 0 : qi.w;
        const float l0 = g.ql[0], l1 = g.ql[1], l2 = g.ql[2];
        float fx = 0.f, fy = 0.f, fz = 0.f, ue = 0.f, we = 0.f;
        float txx = 0.f, tyy = 0.f, tzz = 0.f, txy = 0.f, txz = 0.f, tyz = 0.f;
        int cnt = b.ncount[i];
        cnt = cnt < g.cap ? cnt : g.cap;
        const int32_t* __restrict__ row = b.nl + nl_base(i, g.cap);
        const int self = (int)i;

        auto pair = [&](const int4& qj, int j, bool valid) {
            const float dx = qdiff(qj.x, qi.x, l0);
            const float dy = qdiff(qj.y, qi.y, l1);
            const float dz = qdiff(qj.z, qi.z, l2);
            const float r2 = dx * dx + dy * dy + dz * dz;
            const int tp = SINGLE ? 0 : ti * MD_MAX_TYPES + qj.w;
            bool in = valid && r2 < a.pt.rc2lo[tp];
            if (valid && !in && r2 < a.pt.rc2hi[tp]) in = exact_r2(g, xi, x64[j]) < a.pt.rc2d[tp];
            if (in) {
                const PairCoef<float>& c = a.pt.f[tp];
                float fr, u;
                if (a.pt.tabn[tp] > 1) {
                    // tabulated: u and f = -du/dr linear in r on the pair's grid
                    const float r = sqrtf(r2);
                    float q = (r - a.pt.tab_rmin[tp]) * a.pt.tab_idr[tp];
                    q = q > 0.f ? q : 0.f;
                    int kq = (int)q;
                    kq = kq > a.pt.tabn[tp] - 2 ? a.pt.tabn[tp] - 2 : kq;
                    const float al = q - (float)kq;
                    const float2* trow = b.tab + (int64_t)tp * g.table_points;
                    const float2 t0 = trow[kq], t1 = trow[kq + 1];
                    u = (1.f - al) * t0.x + al * t1.x;
                    fr = ((1.f - al) * t0.y + al * t1.y) * __builtin_amdgcn_rcpf(r);
                } else if (c.cap2 > 0.f && r2 < c.cap2) {
                    fr = c.fcap * __builtin_amdgcn_rsqf(r2);
                    u = c.ucap;
                } else {
                    const float inv = __builtin_amdgcn_rcpf(r2);
                    const float s2 = c.sig2 * inv;
                    const float s6 = s2 * s2 * s2;
                    fr = c.eps24 * s6 * (2.f * s6 - 1.f) * inv;
                    u = c.eps4 * s6 * (s6 - 1.f) - c.shift;
                }
                fx -= fr * dx;
                fy -= fr * dy;
                fz -= fr * dz;
                ue += u;
                we += fr * r2;
                if (TENSOR) {
                    txx += fr * dx * dx; tyy += fr * dy * dy; tzz += fr * dz * dz;
                    txy += fr * dx * dy; txz += fr * dx * dz; tyz += fr * dy * dz;
                }
            }
        };

        // Neighbour indices are prefetched one batch of 8 ahead.  The loads
        // are unconditional (slot clamped inside the row capacity) so the
        // compiler can count them and wait only for the gathers in use;
        // slots past the row's count select the particle itself, masked.
        constexpr int B = 8;
        const int last = cnt > 0 ? cnt - 1 : 0;   // loads past the row repeat its last slot
        const char* __restrict__ xqb = reinterpret_cast<const char*>(xq);
        int jn[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const int v = row[nl_off(u < last ? u : last)];
            jn[u] = u < cnt ? v : self;
        }
        for (int k0 = 0; k0 < cnt; k0 += B) {
            int jc[B];
            int4 q[B];
#pragma unroll
            for (int u = 0; u < B; ++u) {
                jc[u] = jn[u];
                q[u] = *reinterpret_cast<const int4*>(xqb + ((uint32_t)jc[u] << 4));
            }
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const int kk = k0 + B + u;
                const int v = row[nl_off(kk < last ? kk : last)];
                jn[u] = kk < cnt ? v : self;
            }
#pragma unroll
            for (int u = 0; u < B; ++u) pair(q[u], jc[u], k0 + u < cnt);
        }
        acc[A_EPAIR] += 0.5 * (double)ue;
        acc[A_VIR] += 0.5 * (double)we;
        if (TENSOR) {
            acc[A_TXX] += 0.5 * (double)txx; acc[A_TYY] += 0.5 * (double)tyy; acc[A_TZZ] += 0.5 * (double)tzz;
            acc[A_TXY] += 0.5 * (double)txy; acc[A_TXZ] += 0.5 * (double)txz; acc[A_TYZ] += 0.5 * (double)tyz;
        }
        if (BONDED) {
            const DiffQ df{l0, l1, l2};
            bonded_forces<float, int4, DiffQ>(b, a.dy, n, i, xq, qi, df, fx, fy, fz, acc, TENSOR, flag_bond);
        }
        const double F[3] = {(double)fx, (double)fy, (double)fz};
        finish_particle(a, i, xi, SINGLE ? 0 : ti, F, acc, flag_reb, flag_nf);
    }
    }
    block_epilogue(a, acc, flag_reb, flag_bond, flag_nf, TENSOR ? kNacc : A_VIR + 1);
}


// FP32 fast path: one particle type, cubic box, no capping radius.  The pair
// math runs in fixed-point length units (u = L / 2^32): r2 = |dq|^2, the
// coefficients are rescaled on the host, out-of-range pairs get inv = 0 so
// that every term vanishes without a branch, and the FP64 re-decision of the
// rounding band around rc costs one rarely taken branch per batch of 8.
//   F_i = -(24 eps / u) sum a b-weighted dq,  a = s6 (2 s6 - 1), b = a / r2
//   U_i = 1/2 (4 eps sum s6 (s6 - 1) - n_in shift),  W_i = 1/2 24 eps sum a
template <bool BONDED, bool TENSOR>
__device__ __forceinline__ void fast_particle(const StepArgs& a, int64_t i, double* acc, bool& flag_reb,
                                              bool& flag_bond, bool& flag_nf) {
    const Geom& g = a.g;
    const Bufs& b = a.b;
    const int64_t n = g.n;
    const int4* __restrict__ xq = b.xq[a.parity];
    const double4* __restrict__ x64 = b.x[a.parity];
    {
        const double4 xi = x64[i];
        const int4 qi = quantize4(g, xi.x, xi.y, xi.z, xi.w);  // equals xq[i]: same function
        const FastCoef& fc = a.fast;
        float fx = 0.f, fy = 0.f, fz = 0.f, ea = 0.f, wa = 0.f, nin = 0.f;
        float txx = 0.f, tyy = 0.f, tzz = 0.f, txy = 0.f, txz = 0.f, tyz = 0.f;
        int cnt = b.ncount[i];
        cnt = cnt < g.cap ? cnt : g.cap;
        // the capacity is a multiple of 8, so the padded row stays inside it
        const int nslots = min((cnt + 7) & ~7, g.cap);
        const int32_t* __restrict__ row = b.nl + nl_base(i, g.cap);
        // unbonded: 12-byte records (Geom::x3_on); bonded: the 16-byte ones
        const char* __restrict__ recb = BONDED ? reinterpret_cast<const char*>(xq)
                                              : reinterpret_cast<const char*>(b.x3[a.parity]);
        const int last = nslots > 0 ? nslots - 1 : 0;  // loads past the row repeat its last slot
        // Indices are loaded two batches ahead of their gathers (16 loads
        // of 256 bytes in flight per wavefront) to cover HBM latency.
        constexpr int B = 8;
        int jn[B], jn2[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            jn[u] = row[(u < last ? u : last) * kTile];
            jn2[u] = row[(B + u < last ? B + u : last) * kTile];
        }
        for (int k0 = 0; k0 < nslots; k0 += B) {
            int jc[B];
            Q3 q[B];
#pragma unroll
            for (int u = 0; u < B; ++u) {
                jc[u] = jn[u];
                if (BONDED) {
                    const int4 r = *reinterpret_cast<const int4*>(recb + ((uint32_t)jc[u] << 4));
                    q[u] = Q3{r.x, r.y, r.z};
                } else {
                    q[u] = *reinterpret_cast<const Q3*>(recb + (uint32_t)jc[u] * 12u);
                }
            }
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const int kk = k0 + 2 * B + u;
                jn[u] = jn2[u];
                jn2[u] = row[nl_off(kk < last ? kk : last)];
            }
            float dx[B], dy[B], dz[B], r2[B];
            uint32_t inmask = 0, bandmask = 0;
#pragma unroll
            for (int u = 0; u < B; ++u) {
                dx[u] = (float)(int32_t)((uint32_t)q[u].x - (uint32_t)qi.x);
                dy[u] = (float)(int32_t)((uint32_t)q[u].y - (uint32_t)qi.y);
                dz[u] = (float)(int32_t)((uint32_t)q[u].z - (uint32_t)qi.z);
                r2[u] = dx[u] * dx[u] + dy[u] * dy[u] + dz[u] * dz[u];
                // r2 > 0 excludes the padding self entries
                const bool lo = r2[u] > 0.f && r2[u] < fc.rc2lo;
                const bool band = r2[u] >= fc.rc2lo && r2[u] < fc.rc2hi;
                inmask |= (uint32_t)lo << u;
                bandmask |= (uint32_t)band << u;
            }
            if (__builtin_expect(bandmask != 0, 0)) {
#pragma unroll
                for (int u = 0; u < B; ++u)
                    if ((bandmask >> u) & 1u)
                        if (exact_r2(g, xi, x64[jc[u]]) < fc.rc2d) inmask |= 1u << u;
            }
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const bool in = (inmask >> u) & 1u;
                const float inv = in ? __builtin_amdgcn_rcpf(r2[u]) : 0.f;
                const float s2 = fc.sig2u * inv;
                const float s6 = s2 * s2 * s2;
                const float aa = s6 * (2.f * s6 - 1.f);
                const float bb = aa * inv;
                fx += bb * dx[u];
                fy += bb * dy[u];
                fz += bb * dz[u];
                wa += aa;
                ea += s6 * s6 - s6;
                nin += in ? 1.f : 0.f;
                if (TENSOR) {
                    txx += bb * dx[u] * dx[u]; tyy += bb * dy[u] * dy[u]; tzz += bb * dz[u] * dz[u];
                    txy += bb * dx[u] * dy[u]; txz += bb * dx[u] * dz[u]; tyz += bb * dy[u] * dz[u];
                }
            }
        }
        fx *= -fc.eps24_u;
        fy *= -fc.eps24_u;
        fz *= -fc.eps24_u;
        acc[A_EPAIR] += 0.5 * ((double)fc.eps4 * (double)ea - (double)fc.shift * (double)nin);
        acc[A_VIR] += 0.5 * (double)fc.eps24 * (double)wa;
        if (TENSOR) {
            // r_ij f_ij = 24 eps b dq dq (units cancel: b carries 1/u^2)
            const double s = 0.5 * (double)fc.eps24;
            acc[A_TXX] += s * txx; acc[A_TYY] += s * tyy; acc[A_TZZ] += s * tzz;
            acc[A_TXY] += s * txy; acc[A_TXZ] += s * txz; acc[A_TYZ] += s * tyz;
        }
        if (BONDED) {
            const DiffQ df{g.ql[0], g.ql[1], g.ql[2]};
            bonded_forces<float, int4, DiffQ>(b, a.dy, n, i, xq, qi, df, fx, fy, fz, acc, TENSOR, flag_bond);
        }
        const double F[3] = {(double)fx, (double)fy, (double)fz};
        finish_particle(a, i, xi, 0, F, acc, flag_reb, flag_nf);
    }
}

// BS particles per block (64 .. 512, the block dimension the autotuner
// picks); one block per BS-particle tile, blocks in XCD-contiguous order.
template <bool BONDED, bool TENSOR, int BS>
__device__ __forceinline__ void step_fast_body(const StepArgs& a) {
    const int64_t n = a.g.n;
    double acc[kNacc];
#pragma unroll
    for (int k = 0; k < kNacc; ++k) acc[k] = 0.0;
    bool flag_reb = false, flag_bond = false, flag_nf = false;
    const int64_t ntile = (n + BS - 1) / BS;
    const int64_t bt = xcd_block(blockIdx.x, gridDim.x);
    for (int64_t t = bt * ntile / gridDim.x; t < (bt + 1) * ntile / gridDim.x; ++t) {
        const int64_t i = t * BS + threadIdx.x;
        if (i < n) fast_particle<BONDED, TENSOR>(a, i, acc, flag_reb, flag_bond, flag_nf);
    }
    block_epilogue<BS>(a, acc, flag_reb, flag_bond, flag_nf, TENSOR ? kNacc : A_VIR + 1);
}

// The LJ form: 139-142 VGPRs, 3 wavefronts per SIMD, at every block size.
template <bool TENSOR, int BS>
__global__ void __launch_bounds__(BS)
k_step_fast(const StepArgs a) {
    step_fast_body<false, TENSOR, BS>(a);
}

// The bonded form is capped at 128 VGPRs (4 wavefronts per SIMD instead of
// 3, a few bytes of spill): 6% faster on the 2M-bead melt, whose list is
// short and whose bonded partners add gathers; the same cap costs the LJ
// kernel 4%, so it keeps its 144 registers.
template <bool TENSOR, int BS>
__global__ void __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(4)))
k_step_fast_bonded(const StepArgs a) {
    step_fast_body<true, TENSOR, BS>(a);
}

// AdResS weight of a position x along the slab axis: 1 within d_at of x0
// (minimum image), cos^2(pi (d - d_at) / (2 d_hy)) over the hybrid zone, 0
// beyond.
__device__ __forceinline__ float adress_weight(const Dyn& dy, float x, float Lx) {
    float d = x - dy.ad_x0;
    if (d > 0.5f * Lx) d -= Lx;
    else if (d < -0.5f * Lx) d += Lx;
    d = fabsf(d);
    if (d < dy.ad_dat) return 1.f;
    if (d >= dy.ad_dat + dy.ad_dhy) return 0.f;
    // cos^2 z = (1 + cos 2z) / 2, with the revolution-scaled hardware cosine
    return 0.5f + 0.5f * __builtin_amdgcn_cosf(dy.ad_k * (d - dy.ad_dat) * 0.3183098861837907f);
}

// theta_ij of the DPD thermostat: Philox4x32-10 at counter (step low word,
// step high word, min id, max id) with key (seed low word, seed high word
// ^ 6), Box-Muller on the first two words as uniforms (w + 1/2) 2^-32,
// evaluated in FP32 with the hardware log2 and cosine (cos(2 pi u) from the
// revolution-scaled instruction): within a few 1e-7 of the FP64 draw, far
// below the FP32 force rounding.
__device__ __forceinline__ float dpd_theta(uint64_t seed, uint64_t step, uint32_t ti, uint32_t tj) {
    uint32_t x0 = (uint32_t)step, x1 = (uint32_t)(step >> 32), x2 = ti < tj ? ti : tj, x3 = ti < tj ? tj : ti;
    philox4x32_10(x0, x1, x2, x3, (uint32_t)seed, (uint32_t)(seed >> 32) ^ 6u);
    const float u0 = fmaf((float)x0, 0x1.0p-32f, 0x1.0p-33f);
    const float u1 = fmaf((float)x1, 0x1.0p-32f, 0x1.0p-33f);
    // -2 ln u0 = -2 ln 2 log2 u0
    const float rr = sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u0));
    return rr * __builtin_amdgcn_cosf(u1);
}

// Generic FP32 step, one 256-particle tile per block, for what the fast
// kernels leave out: the DPD pair thermostat (MD_DPD), Lees-Edwards shear,
// tabulated pair potentials and the angle kinds beyond the cosine bending.
// The pair table (any types, capping radius, or a tabulated pair: u and f
// interpolated linearly in r) and the bonded terms under the sheared minimum
// image, the DPD forces from the half-step velocities (MODE_STEP only: a
// thermostat force, not part of md_forces), then the integration with the
// sheared boundary crossing.  The DPD pair force on i, with e = (r_i - r_j)/r, w = 1 - r/rc_d:
//   (-gamma w^2 (e . v_ij) + sigma w theta_ij / sqrt(dt)) e,
// computed by both members of a pair with the same theta_ij, so the two
// contributions cancel to FP32 rounding.
// SINGLE: one particle type, so the pair parameters are uniform and held in
// scalar registers.  LDSTAB: the tables the kernel reads (the pair row of
// type pair 0 and the AdResS coarse-grained row) are first copied into LDS,
// [2][table_points] (u, f) pairs, so that their lookups do not wait on
// global memory.  The neighbour row is pipelined: the index two slots ahead
// and the record (and DPD velocity) one slot ahead of the pair arithmetic.
template <bool BONDED, bool SINGLE, bool LDSTAB>
__global__ void __launch_bounds__(kBlock) k_step_gen(const StepArgs a) {
    extern __shared__ float2 stab[];
    const Geom& g = a.g;
    const Bufs& b = a.b;
    const int64_t n = g.n;
    const int4* __restrict__ xq = b.xq[a.parity];
    const double4* __restrict__ x64 = b.x[a.parity];
    if (LDSTAB) {
        const int np = g.table_points;
        const float2* __restrict__ src0 = b.tab;
        const float2* __restrict__ src1 = b.tab + (int64_t)kCgTableRow * np;
        for (int k = threadIdx.x; k < np; k += kBlock) {
            stab[k] = src0[k];
            stab[np + k] = src1[k];
        }
        __syncthreads();
    }
    double acc[kNacc];
#pragma unroll
    for (int k = 0; k < kNacc; ++k) acc[k] = 0.0;
    bool flag_reb = false, flag_bond = false, flag_nf = false;
    const bool tensor = a.tensor != 0;
    const int64_t step = b.ctl->step;
    double delta = 0.0, dw = 0.0;
    uint32_t qd = 0;
    LeStep les{0.0, 0.0};
    if (g.le) {
        delta = le_delta(g, step);
        dw = le_fold(g, delta);
        qd = quantize(delta, g.qs[0]);
        les.delta_next = le_delta(g, step + 1);
        les.drift = fabs(g.le_rate_Ly * ((double)(step + 1 - b.ctl->build_step) * g.le_dt));
    }
    const bool dpd = a.dy.dpd && a.mode == MODE_STEP;
    const int64_t i = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (i < n) {
        const double4 xi = x64[i];
        const int4 qi = quantize4(g, xi.x, xi.y, xi.z, xi.w);
        const int ti = qi.w;
        const DiffLEQ df{g.ql[0], g.ql[1], g.ql[2], qd};
        float fx = 0.f, fy = 0.f, fz = 0.f, ue = 0.f, we = 0.f;
        float txx = 0.f, tyy = 0.f, tzz = 0.f, txy = 0.f, txz = 0.f, tyz = 0.f;
        const float wi = a.dy.adress ? adress_weight(a.dy, (float)xi.x, (float)g.L[0]) : 1.f;
        // DPD reads the half-step velocities and ids from the snapshot in
        // b.vt taken before this kernel (b.v is overwritten here as particles
        // finish): one 16-byte record (vx, vy, vz, id) per particle
        const float4* __restrict__ vs = reinterpret_cast<const float4*>(b.vt);
        float4 vi = make_float4(0.f, 0.f, 0.f, 0.f);
        if (dpd) vi = vs[i];
        int cnt = b.ncount[i];
        cnt = cnt < g.cap ? cnt : g.cap;
        const int32_t* __restrict__ row = b.nl + nl_base(i, g.cap);
        // slots past the end repeat the last one (every slot below cnt holds
        // a particle index); an empty row reads the particle itself
        const int last = cnt > 0 ? cnt - 1 : 0;
        auto slot = [&](int k) { return cnt > 0 ? row[nl_off(k < last ? k : last)] : (int)i; };
        int jA = slot(0), jB = slot(1);
        int4 qA = xq[jA];
        float4 vA = dpd ? vs[jA] : make_float4(0.f, 0.f, 0.f, 0.f);
        for (int k = 0; k < cnt; ++k) {
            const int j = jA;
            const int4 qj = qA;
            const float4 vj = vA;
            jA = jB;
            jB = slot(k + 2);
            qA = xq[jA];
            if (dpd) vA = vs[jA];
            float dx, dy, dz;
            const int s = df(qi, qj, dx, dy, dz);
            const float r2 = dx * dx + dy * dy + dz * dz;
            const int tp = SINGLE ? 0 : ti * MD_MAX_TYPES + qj.w;
            bool in = r2 < a.pt.rc2lo[tp];
            if (!in && r2 < a.pt.rc2hi[tp]) in = exact_r2_le(g, xi, x64[j], dw) < a.pt.rc2d[tp];
            // AdResS: the coarse-grained force of the pair, to be mixed in below
            bool cg_in = false;
            float ucg = 0.f, frcg = 0.f;
            if (a.dy.adress && a.pt.cgn[tp] > 1) {
                cg_in = r2 < a.pt.cg_rc2lo[tp];
                if (!cg_in && r2 < a.pt.cg_rc2hi[tp]) cg_in = exact_r2_le(g, xi, x64[j], dw) < a.pt.cg_rc2d[tp];
                if (cg_in) {
                    const float r = sqrtf(r2);
                    float q = (r - a.pt.cg_rmin[tp]) * a.pt.cg_idr[tp];
                    q = q > 0.f ? q : 0.f;
                    int kq = (int)q;
                    kq = kq > a.pt.cgn[tp] - 2 ? a.pt.cgn[tp] - 2 : kq;
                    const float al = q - (float)kq;
                    const float2* trow = LDSTAB ? stab + g.table_points
                                                : b.tab + (int64_t)(kCgTableRow + tp) * g.table_points;
                    const float2 t0 = trow[kq], t1 = trow[kq + 1];
                    ucg = (1.f - al) * t0.x + al * t1.x;
                    frcg = ((1.f - al) * t0.y + al * t1.y) * __builtin_amdgcn_rcpf(r);
                }
            }
            if (in || cg_in) {
                const PairCoef<float>& c = a.pt.f[tp];
                float fr = 0.f, u = 0.f;
                if (!in) {
                } else if (a.pt.tabn[tp] > 1) {
                    // tabulated: u and f = -du/dr linear in r on the pair's grid
                    const float r = sqrtf(r2);
                    float q = (r - a.pt.tab_rmin[tp]) * a.pt.tab_idr[tp];
                    q = q > 0.f ? q : 0.f;
                    int kq = (int)q;
                    kq = kq > a.pt.tabn[tp] - 2 ? a.pt.tabn[tp] - 2 : kq;
                    const float al = q - (float)kq;
                    const float2* trow = LDSTAB ? stab : b.tab + (int64_t)tp * g.table_points;
                    const float2 t0 = trow[kq], t1 = trow[kq + 1];
                    u = (1.f - al) * t0.x + al * t1.x;
                    fr = ((1.f - al) * t0.y + al * t1.y) * __builtin_amdgcn_rcpf(r);
                } else if (c.cap2 > 0.f && r2 < c.cap2) {
                    fr = c.fcap * __builtin_amdgcn_rsqf(r2);
                    u = c.ucap;
                } else {
                    const float inv = __builtin_amdgcn_rcpf(r2);
                    const float s2 = c.sig2 * inv;
                    const float s6 = s2 * s2 * s2;
                    fr = c.eps24 * s6 * (2.f * s6 - 1.f) * inv;
                    u = c.eps4 * s6 * (s6 - 1.f) - c.shift;
                }
                if (a.dy.adress) {
                    // x_j from its fixed-point coordinate (positions lie in [0, L))
                    const float lam = wi * adress_weight(a.dy, (float)(uint32_t)qj.x * g.ql[0], (float)g.L[0]);
                    u = lam * u + (1.f - lam) * ucg;
                    fr = lam * fr + (1.f - lam) * frcg;
                }
                fx -= fr * dx;
                fy -= fr * dy;
                fz -= fr * dz;
                ue += u;
                we += fr * r2;
                if (tensor) {
                    txx += fr * dx * dx; tyy += fr * dy * dy; tzz += fr * dz * dz;
                    txy += fr * dx * dy; txz += fr * dx * dz; tyz += fr * dy * dz;
                }
            }
            if (dpd && r2 < a.dy.dpd_rc2 && r2 > 0.f) {
                const float ir = __builtin_amdgcn_rsqf(r2);
                const float r = r2 * ir;
                const float w = 1.f - r * __builtin_amdgcn_rcpf(a.dy.dpd_rc);
                const float ex = -dx * ir, ey = -dy * ir, ez = -dz * ir;
                // v_i - (v_j - s shear_rate Ly e_x)
                const float vx = vi.x - vj.x + (float)(s * g.le_rate_Ly);
                const float vy = vi.y - vj.y;
                const float vz = vi.z - vj.z;
                const float ev = ex * vx + ey * vy + ez * vz;
                const float th = dpd_theta(a.dy.seed, (uint64_t)step, __float_as_uint(vi.w), __float_as_uint(vj.w));
                const float A = -a.dy.dpd_gamma * w * w * ev + a.dy.dpd_sigma_isdt * w * th;
                fx += A * ex;
                fy += A * ey;
                fz += A * ez;
            }
        }
        acc[A_EPAIR] += 0.5 * (double)ue;
        acc[A_VIR] += 0.5 * (double)we;
        if (tensor) {
            acc[A_TXX] += 0.5 * (double)txx; acc[A_TYY] += 0.5 * (double)tyy; acc[A_TZZ] += 0.5 * (double)tzz;
            acc[A_TXY] += 0.5 * (double)txy; acc[A_TXZ] += 0.5 * (double)txz; acc[A_TYZ] += 0.5 * (double)tyz;
        }
        if (BONDED) {
            const auto dfb = [&df](const int4& p, const int4& q, float& ddx, float& ddy, float& ddz) {
                (void)df(p, q, ddx, ddy, ddz);
            };
            bonded_forces<float, int4, decltype(dfb), true>(b, a.dy, n, i, xq, qi, dfb, fx, fy, fz, acc, tensor,
                                                            flag_bond);
        }
        const double F[3] = {(double)fx, (double)fy, (double)fz};
        finish_particle(a, i, xi, ti, F, acc, flag_reb, flag_nf, g.le ? &les : nullptr);
    }
    block_epilogue(a, acc, flag_reb, flag_bond, flag_nf, tensor ? kNacc : A_VIR + 1);
}

// Step of the surrogate mode, one 256-particle tile per block: the
// network's pair force from the per-particle input gradients a_i = dE_i/dG(i),
//   F_i = sum_j ((a_i + a_j) . g'(r_ij)) (x_j - x_i) / r_ij  over r_ij < r_d,
//   g'_k(r) = phi_k(r) (f_c'(r) - (r - mu_k) f_c(r) / w^2),
// then the bonded forces, the integration and the reductions of the plain
// step kernels.  The list row is pipelined: positions are gathered two slots
// ahead and the a_j rows of in-range neighbours one slot ahead of the pair
// arithmetic that uses them.  BF16 form (A16): a rows are
// BF16; g' is rounded to BF16 pairs and dotted with a_i and a_j by
// v_dot2_f32_bf16 with FP32 accumulation.  FP32 form: FP32 rows and FP32
// multiply-adds.  The pair virial goes to the step's reductions; the
// network energy comes from the network kernel's partials.
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));

template <bool BONDED, bool TENSOR, bool A16>
__global__ void __launch_bounds__(kBlock) k_sur_step(const StepArgs a, const SurBufs s, const SurConst c) {
    constexpr int AW = A16 ? 16 : 32;       // 32-bit words per a row
    const Geom& g = a.g;
    const Bufs& b = a.b;
    const int64_t n = g.n;
    double acc[kNacc];
#pragma unroll
    for (int k = 0; k < kNacc; ++k) acc[k] = 0.0;
    bool flag_reb = false, flag_bond = false, flag_nf = false;
    const int64_t i = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (i < n) {
        const int4* __restrict__ xq = b.xq[a.parity];
        const double4 xi = b.x[a.parity][i];
        const int4 qi = quantize4(g, xi.x, xi.y, xi.z, xi.w);
        const uint32_t* __restrict__ arow = A16 ? reinterpret_cast<const uint32_t*>(s.ab)
                                                : reinterpret_cast<const uint32_t*>(s.a);
        uint32_t ai[AW];
#pragma unroll
        for (int q = 0; q < AW / 4; ++q) {
            const uint4 v = reinterpret_cast<const uint4*>(arow + i * AW)[q];
            ai[4 * q] = v.x; ai[4 * q + 1] = v.y; ai[4 * q + 2] = v.z; ai[4 * q + 3] = v.w;
        }
        int cnt = b.ncount[i];
        cnt = cnt < g.cap ? cnt : g.cap;
        const int nslots = min((cnt + 7) & ~7, g.cap);
        const int32_t* __restrict__ row = b.nl + nl_base(i, g.cap);
        const int last = nslots > 0 ? nslots - 1 : 0;
        float fx = 0.f, fy = 0.f, fz = 0.f, wv = 0.f;
        float txx = 0.f, tyy = 0.f, tzz = 0.f, txy = 0.f, txz = 0.f, tyz = 0.f;
        auto idx = [&](int slot) { return row[nl_off(slot < last ? slot : last)]; };
        auto geom = [&](const int4& qj, float& dx, float& dy, float& dz) {
            dx = qdiff(qj.x, qi.x, g.ql[0]);
            dy = qdiff(qj.y, qi.y, g.ql[1]);
            dz = qdiff(qj.z, qi.z, g.ql[2]);
            return dx * dx + dy * dy + dz * dz;
        };
        auto load_row = [&](int j, uint32_t* out) {
#pragma unroll
            for (int q = 0; q < AW / 4; ++q) {
                const uint4 v = reinterpret_cast<const uint4*>(arow + (int64_t)j * AW)[q];
                out[4 * q] = v.x; out[4 * q + 1] = v.y; out[4 * q + 2] = v.z; out[4 * q + 3] = v.w;
            }
        };
        auto pair = [&](const int4& qj, const uint32_t* aj) {
            float dx, dy, dz;
            const float r2 = geom(qj, dx, dy, dz);
            const float r = sqrtf(r2);
            float dfc;
            const float fc = sur_cutoff(c, r, dfc);
            float ph[kSurNB];
            sur_basis(c, r, ph);
            const float Bc = c.inv_w2 * fc;
            float cij = 0.f;
            if (A16) {
                // g'_k = phi_k (dfc - (r - mu_k) Bc) = phi_k (mu_k Bc + al): one
                // FMA and one product per term (the FP32 cancellation of
                // mu_k Bc against al is far below the BF16 rounding that follows)
                const float al = fmaf(-r, Bc, dfc);
#pragma unroll
                for (int k2 = 0; k2 < kSurNB / 2; ++k2) {
                    const float g0 = ph[2 * k2] * fmaf(c.mu[2 * k2], Bc, al);
                    const float g1 = ph[2 * k2 + 1] * fmaf(c.mu[2 * k2 + 1], Bc, al);
                    const bf16x2v gp = {(__bf16)g0, (__bf16)g1};
                    cij = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2v, ai[k2]), gp, cij, false);
                    cij = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2v, aj[k2]), gp, cij, false);
                }
            } else {
#pragma unroll
                for (int k = 0; k < kSurNB; ++k) {
                    const float dg = ph[k] * fmaf(-(r - c.mu[k]), Bc, dfc);
                    cij = fmaf(__uint_as_float(ai[k]) + __uint_as_float(aj[k]), dg, cij);
                }
            }
            const float sc = cij * __builtin_amdgcn_rcpf(r);
            fx += sc * dx;
            fy += sc * dy;
            fz += sc * dz;
            wv -= cij * r;
            if (TENSOR) {
                // r_ij f_ij with r_ij = -(dx, dy, dz), f_ij = sc (dx, dy, dz)
                txx -= sc * dx * dx; tyy -= sc * dy * dy; tzz -= sc * dz * dz;
                txy -= sc * dx * dy; txz -= sc * dx * dz; tyz -= sc * dy * dz;
            }
        };
        auto in_range = [&](const int4& qj) {
            float dx, dy, dz;
            const float r2 = geom(qj, dx, dy, dz);
            return r2 < c.rd2 && r2 > 0.f;   // r2 = 0: the row's padding (the particle itself)
        };
        if (nslots > 0) {
            // slot k: index jA, position qA, a row aX (in range: inX); slot k+1:
            // index jB, position qB (in flight); slot k+2: index jC.  Rows hold
            // a multiple of 8 slots, so slots come in pairs and the a rows
            // alternate between aX and aY without copies.
            int jA = idx(0), jB = idx(1), jC = idx(2);
            int4 qA = xq[jA], qB = xq[jB];
            uint32_t aX[AW], aY[AW];
            bool inX = in_range(qA), inY = false;
            if (inX) load_row(jA, aX);
            for (int k0 = 0; k0 < nslots; k0 += 2) {
                // slot k0 (row aX); prefetch: a row of k0 + 1, position of k0 + 2
                inY = in_range(qB);
                if (inY) load_row(jB, aY);
                int4 qC = xq[jC];
                int jD = idx(k0 + 3);
                if (inX) pair(qA, aX);
                qA = qB; qB = qC; jA = jB; jB = jC; jC = jD;
                // slot k0 + 1 (row aY); prefetch: a row of k0 + 2, position of k0 + 3
                inX = k0 + 2 < nslots && in_range(qB);
                if (inX) load_row(jB, aX);
                qC = xq[jC];
                jD = idx(k0 + 4);
                if (inY) pair(qA, aY);
                qA = qB; qB = qC; jA = jB; jB = jC; jC = jD;
            }
        }
        acc[A_VIR] += 0.5 * (double)wv;
        if (TENSOR) {
            acc[A_TXX] += 0.5 * (double)txx; acc[A_TYY] += 0.5 * (double)tyy; acc[A_TZZ] += 0.5 * (double)tzz;
            acc[A_TXY] += 0.5 * (double)txy; acc[A_TXZ] += 0.5 * (double)txz; acc[A_TYZ] += 0.5 * (double)tyz;
        }
        if (BONDED) {
            const DiffQ df{g.ql[0], g.ql[1], g.ql[2]};
            bonded_forces<float, int4, DiffQ>(b, a.dy, n, i, xq, qi, df, fx, fy, fz, acc, TENSOR, flag_bond);
        }
        const double F[3] = {(double)fx, (double)fy, (double)fz};
        finish_particle(a, i, xi, (int)xi.w, F, acc, flag_reb, flag_nf);
    }
    block_epilogue(a, acc, flag_reb, flag_bond, flag_nf, TENSOR ? kNacc : A_VIR + 1);
}

// One block: reduce partials[k][block] in a fixed order, record the step's
// observables, and (MODE_STEP) advance the step counter and move the
// rebuild request to the next step.
constexpr int kFinal = 1024;
// nacc: the number of quantities the step kernel accumulated (the virial
// tensor only when it was asked for); the others are zero and not read.
__device__ __forceinline__ void finalize_body(const Bufs& b, int nblocks, int mode, const double* spart, int nacc,
                                              int spart_rows = 8) {
    __shared__ double red[kFinal / 64][kNacc];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double s[kNacc];
#pragma unroll
    for (int k = 0; k < kNacc; ++k) s[k] = 0.0;
    for (int blk0 = 0; blk0 < nblocks; blk0 += 4 * kFinal) {
        double v[4][kNacc];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int blk = blk0 + r * kFinal + threadIdx.x;
#pragma unroll
            for (int k = 0; k < kNacc; ++k)
                v[r][k] = (k < nacc && blk < nblocks) ? b.partials[(int64_t)k * nblocks + blk] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int k = 0; k < kNacc; ++k) s[k] += v[r][k];
        if (spart) {
            // surrogate pair energy (row 0), virial (row 1) and tensor (rows 2..7)
            for (int r = 0; r < 4; ++r) {
                const int blk = blk0 + r * kFinal + threadIdx.x;
                if (blk >= nblocks) continue;
                s[A_EPAIR] += spart[blk];
                if (spart_rows > 1) {
                    s[A_VIR] += spart[(int64_t)nblocks + blk];
                    if (nacc == kNacc)
                        for (int k = 0; k < 6; ++k) s[A_TXX + k] += spart[(int64_t)(2 + k) * nblocks + blk];
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < kNacc; ++k) {
        const double t = k < nacc ? wave_sum(s[k]) : 0.0;
        if (lane == 0) red[w][k] = t;
    }
    __syncthreads();
    // one lane per quantity sums the wavefront totals (fixed order), so the
    // serial part below reads finished sums only
    __shared__ double fin[kNacc];
    if (threadIdx.x < kNacc) {
        double v = 0.0;
        for (int ww = 0; ww < kFinal / 64; ++ww) v += red[ww][threadIdx.x];
        fin[threadIdx.x] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot[kNacc];
        for (int k = 0; k < kNacc; ++k) tot[k] = fin[k];
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

__global__ void __launch_bounds__(kFinal) k_finalize(Bufs b, int nblocks, int mode, const double* spart, int nacc,
                                                     int spart_rows) {
    finalize_body(b, nblocks, mode, spart, nacc, spart_rows);
}

// ------------------------------------------------------------------ batches
//
// Per-tile kernels of a batch: block -> global tile (XCD-aware order) ->
// system -> the single-system body on that system's arrays.  The rebuild
// kernels return at once for systems whose own rebuild flag is clear.

struct TileRef {
    const SysEntry* e;
    int64_t lt;     // tile inside the system
    int64_t i;      // particle inside the system
};

__device__ __forceinline__ TileRef tile_ref(const SysEntry* __restrict__ tab, const int32_t* __restrict__ tile_sys) {
    const int64_t t = xcd_block(blockIdx.x, gridDim.x);
    const SysEntry* e = tab + tile_sys[t];
    const int64_t lt = t - e->tile0;
    return TileRef{e, lt, lt * kBlock + threadIdx.x};
}

// Rebuild kernels of a batch take the plain block order instead: only the
// members whose own trigger fired have work, and the XCD-contiguous order
// would put all of a rebuilding member's tiles on one XCD while the others
// idle.  Spread round-robin, every member's tiles use all XCDs (measured: the
// 256-replica batch 3.62e9 -> 4.15e9 atom-steps/s).
__device__ __forceinline__ TileRef tile_ref_spread(const SysEntry* __restrict__ tab,
                                                   const int32_t* __restrict__ tile_sys) {
    const int64_t t = blockIdx.x;
    const SysEntry* e = tab + tile_sys[t];
    const int64_t lt = t - e->tile0;
    return TileRef{e, lt, lt * kBlock + threadIdx.x};
}

__global__ void k_batch_any(BatchCells bc) {
    __shared__ int any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    for (int s = threadIdx.x; s < bc.nsys; s += blockDim.x)
        if (rebuild_requested(bc.tab[s].a.b)) any = 1;
    __syncthreads();
    if (threadIdx.x == 0) bc.gb.ctl->rebuild = (uint32_t)any;
}

__global__ void __launch_bounds__(kBlock) k_batch_bin(const SysEntry* __restrict__ tab,
                                                      const int32_t* __restrict__ tile_sys, int parity) {
    const TileRef r = tile_ref_spread(tab, tile_sys);
    const Bufs& b = r.e->a.b;
    if (!rebuild_requested(b)) return;
    const Geom& g = r.e->a.g;
    bin_one(g, b, r.i, r.i < g.n, parity);
}

// prefix of the concatenated counts at each system's first cell
__global__ void k_batch_bases(BatchCells bc) {
    if (!rebuild_requested(bc.gb)) return;
    for (int s = threadIdx.x; s < bc.nsys; s += blockDim.x) bc.base[s] = bc.gb.cstart[bc.c_off[s]];
}

// cell starts of rebuilding systems become offsets inside the system
__global__ void __launch_bounds__(kBlock) k_batch_localize(BatchCells bc) {
    if (!rebuild_requested(bc.gb)) return;
    for (int64_t c = gtid(); c < bc.gg.ncell; c += gstride()) {
        int lo = 0, hi = bc.nsys;   // system with c_off[s] <= c < c_off[s + 1]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (bc.c_off[mid] <= c) lo = mid; else hi = mid;
        }
        if (rebuild_requested(bc.tab[lo].a.b)) bc.gb.cstart[c] -= bc.base[lo];
    }
}

__global__ void __launch_bounds__(kBlock) k_batch_scatter(const SysEntry* __restrict__ tab,
                                                          const int32_t* __restrict__ tile_sys) {
    const TileRef r = tile_ref_spread(tab, tile_sys);
    const Bufs& b = r.e->a.b;
    if (!rebuild_requested(b)) return;
    scatter_one(b, r.i, r.i < r.e->a.g.n);
}

__global__ void __launch_bounds__(kBlock) k_batch_permute(const SysEntry* __restrict__ tab,
                                                          const int32_t* __restrict__ tile_sys, int parity) {
    const TileRef r = tile_ref_spread(tab, tile_sys);
    const Bufs& b = r.e->a.b;
    if (!rebuild_requested(b)) return;
    const Geom& g = r.e->a.g;
    if (r.i < g.n) permute_one(g, b, r.i, parity);
}

__global__ void __launch_bounds__(kBlock) k_batch_commit(const SysEntry* __restrict__ tab,
                                                         const int32_t* __restrict__ tile_sys, int parity) {
    const TileRef r = tile_ref_spread(tab, tile_sys);
    const Bufs& b = r.e->a.b;
    if (!rebuild_requested(b)) return;
    const Geom& g = r.e->a.g;
    if (r.i < g.n) commit_one(g, b, r.i, parity, r.e->bonded);
}

__global__ void __launch_bounds__(kBlock) k_batch_nl(const SysEntry* __restrict__ tab,
                                                     const int32_t* __restrict__ tile_sys, int parity) {
    const TileRef r = tile_ref_spread(tab, tile_sys);
    const Bufs& b = r.e->a.b;
    if (!rebuild_requested(b)) return;
    const Geom& g = r.e->a.g;
    int local_max = 0;
    bool overflow = false;
    if (g.nl_tile) {
        const int64_t t = r.lt * (kBlock / kTile) + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kTile));
        if (t * kTile < g.n) {
            if (g.nl_cubic) nl_tile<true>(g, b, t, parity, r.e->bonded, local_max, overflow);
            else nl_tile<false>(g, b, t, parity, r.e->bonded, local_max, overflow);
        }
    } else if (r.i < g.n) {
        nl_one(g, b, r.i, parity, r.e->bonded, local_max, overflow);
    }
    nl_epilogue(b, local_max, overflow);
}

// Fused force + integrate for one tile of one system (FP32 fast path: one
// particle type, cubic box, no capping radius), partials at the tile's slot.
// The table holds each system's arguments for one (mode, parity); they are
// read in place, never copied.
// Capped at 128 VGPRs like the bonded single-system kernel (the batch holds
// melts): 637 -> 615 us per step for the 256-replica batch.
template <bool TENSOR>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4)))
k_batch_step(const SysEntry* __restrict__ tab, const int32_t* __restrict__ tile_sys) {
    const TileRef r = tile_ref(tab, tile_sys);
    const StepArgs& a = r.e->a;
    double acc[kNacc];
#pragma unroll
    for (int k = 0; k < kNacc; ++k) acc[k] = 0.0;
    bool flag_reb = false, flag_bond = false, flag_nf = false;
    if (r.i < a.g.n) {
        if (r.e->bonded) fast_particle<true, TENSOR>(a, r.i, acc, flag_reb, flag_bond, flag_nf);
        else fast_particle<false, TENSOR>(a, r.i, acc, flag_reb, flag_bond, flag_nf);
    }
    block_epilogue(a, acc, flag_reb, flag_bond, flag_nf, TENSOR ? kNacc : A_VIR + 1, r.lt, r.e->ntiles);
}

__global__ void __launch_bounds__(kFinal) k_batch_finalize(const SysEntry* __restrict__ tab, int mode) {
    const SysEntry& e = tab[blockIdx.x];
    finalize_body(e.a.b, e.ntiles, mode, nullptr, kNacc);
}

__global__ void k_batch_gather_obs(const SysEntry* __restrict__ tab, int nsys, double* out) {
    for (int k = threadIdx.x; k < nsys * kHistRec; k += blockDim.x) out[k] = tab[k / kHistRec].a.b.cur[k % kHistRec];
}

// ------------------------------------------------------------------ launchers

static inline int grid_for(int64_t n, int cap_blocks = 4096) {
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > cap_blocks) g = cap_blocks;
    return (int)g;
}

// One 256-particle tile per block: with about three resident blocks per CU a
// capped grid of multi-tile blocks leaves a partial second wave; single-tile
// blocks let the dispatcher balance the tail (measured: 8 % faster for the
// LJ fluid, 19 % for the melt than 1,024 blocks of 4 tiles).
int step_grid(int64_t n) {
    const int64_t t = (n + kBlock - 1) / kBlock;
    return (int)(t < 1 ? 1 : t);
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
                          hipEvent_t ev_sorted) {
    // the sort passes stride over the particles with at most 2048 blocks:
    // against 512 (2M-bead melt, binning and sort per step) 62.0 -> 56.4 us,
    // and one block per 256 particles 59.2 us
    const int gs = grid_for(g.n, 2048);
    hipLaunchKernelGGL(k_bin, dim3(gs), dim3(kBlock), 0, s, g, b, parity);
    hipLaunchKernelGGL(k_scan_chunks, dim3(kScanBlocks), dim3(kBlock), 0, s, g, b);
    hipLaunchKernelGGL(k_scatter, dim3(gs), dim3(kBlock), 0, s, g, b);
    hipLaunchKernelGGL(k_rank_permute, dim3(gs), dim3(kBlock), 0, s, g, b, parity);
    hipLaunchKernelGGL(k_commit, dim3(gs), dim3(kBlock), 0, s, g, b, parity, bonded);
    if (ev_sorted) (void)hipEventRecord(ev_sorted, s);
    if (g.le)
        hipLaunchKernelGGL(k_nl_build_le, dim3(grid_for(g.n, 1 << 20)), dim3(kBlock), 0, s, g, b, parity, bonded);
    else if (g.nl_tile)
        hipLaunchKernelGGL(k_nl_tiles, dim3((unsigned)((g.n + kNlBlock - 1) / kNlBlock)), dim3(kNlBlock), 0, s, g, b,
                           parity, bonded);
    else
        hipLaunchKernelGGL(k_nl_build, dim3(grid_for(g.n, 1 << 20)), dim3(kBlock), 0, s, g, b, parity, bonded);
    return hipGetLastError();
}

int step_launch_grid(const StepArgs& a, int fp64, int block) {
    if (a.dy.gen || fp64 || !a.use_fast || block == kBlock) return step_grid(a.g.n);
    const int64_t t = (a.g.n + block - 1) / block;
    return (int)(t < 1 ? 1 : t);
}

template <bool BONDED, bool TENSOR>
static void launch_fast(const StepArgs& a, int block, hipStream_t s) {
    const dim3 grid((unsigned)step_launch_grid(a, 0, block)), blk((unsigned)block);
#define MD_LF(BS)                                                                                  \
    do {                                                                                           \
        if (BONDED) hipLaunchKernelGGL((k_step_fast_bonded<TENSOR, BS>), grid, blk, 0, s, a);     \
        else hipLaunchKernelGGL((k_step_fast<TENSOR, BS>), grid, blk, 0, s, a);                   \
    } while (0)
    switch (block) {
        case 64: MD_LF(64); break;
        case 128: MD_LF(128); break;
        case 512: MD_LF(512); break;
        default: MD_LF(256); break;
    }
#undef MD_LF
}

// Velocity snapshot for the DPD pair term into b.vt (the sort's scratch,
// free after the rebuild stage): (vx, vy, vz, id bits) per particle, FP32.
__global__ void __launch_bounds__(kBlock) k_snapshot_v(const Bufs b, int64_t n) {
    float4* __restrict__ out = reinterpret_cast<float4*>(b.vt);
    for (int64_t k = gtid(); k < n; k += gstride())
        out[k] = make_float4((float)b.v[k], (float)b.v[n + k], (float)b.v[2 * n + k], __uint_as_float((uint32_t)b.tag[k]));
}

hipError_t launch_step(const StepArgs& a, int fp64, int single_type, int bonded, int block, hipStream_t s) {
    dim3 grid((unsigned)step_grid(a.g.n)), blk(kBlock);
    if (a.dy.gen && a.dy.dpd && a.mode == MODE_STEP)
        hipLaunchKernelGGL(k_snapshot_v, dim3(grid_for(a.g.n)), dim3(kBlock), 0, s, a.b, a.g.n);
    if (a.dy.gen) {
        // tables in LDS for one particle type, when both rows fit in 32 KB
        const size_t tab_lds = 2 * sizeof(float2) * (size_t)a.g.table_points;
        const bool lds = single_type && a.b.tab && a.g.table_points >= 2 && tab_lds <= 32768;
#define MD_LG(B, S, T) hipLaunchKernelGGL((k_step_gen<B, S, T>), grid, blk, T ? tab_lds : 0, s, a)
        if (bonded) {
            if (lds) MD_LG(true, true, true);
            else if (single_type) MD_LG(true, true, false);
            else MD_LG(true, false, false);
        } else {
            if (lds) MD_LG(false, true, true);
            else if (single_type) MD_LG(false, true, false);
            else MD_LG(false, false, false);
        }
#undef MD_LG
    } else if (fp64) {
#define MD_L64(S, B) hipLaunchKernelGGL((k_step64<S, B>), grid, blk, 0, s, a)
        if (single_type) { if (bonded) MD_L64(true, true); else MD_L64(true, false); }
        else { if (bonded) MD_L64(false, true); else MD_L64(false, false); }
#undef MD_L64
    } else if (a.use_fast) {
        const bool t = a.tensor != 0;
        if (bonded) {
            if (t) launch_fast<true, true>(a, block, s);
            else launch_fast<true, false>(a, block, s);
        } else {
            if (t) launch_fast<false, true>(a, block, s);
            else launch_fast<false, false>(a, block, s);
        }
    } else {
#define MD_LQ(S, B, T) hipLaunchKernelGGL((k_step_q<S, B, T>), grid, blk, 0, s, a)
        const bool t = a.tensor != 0;
        if (single_type) {
            if (bonded) { if (t) MD_LQ(true, true, true); else MD_LQ(true, true, false); }
            else { if (t) MD_LQ(true, false, true); else MD_LQ(true, false, false); }
        } else {
            if (bonded) { if (t) MD_LQ(false, true, true); else MD_LQ(false, true, false); }
            else { if (t) MD_LQ(false, false, true); else MD_LQ(false, false, false); }
        }
#undef MD_LQ
    }
    return hipGetLastError();
}

hipError_t launch_finalize(const Bufs& b, int nblocks, int mode, const double* spart, int tensor, hipStream_t s,
                           int spart_rows) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinal), 0, s, b, nblocks, mode, spart, tensor ? kNacc : A_VIR + 1,
                       spart_rows);
    return hipGetLastError();
}

hipError_t launch_sur_step(const StepArgs& a, const SurBufs& sb, const SurConst& c, int bonded, int a_bf16,
                           hipStream_t s) {
    dim3 grid((unsigned)step_grid(a.g.n)), blk(kBlock);
    const bool t = a.tensor != 0;
#define MD_LS(BO, T, A) hipLaunchKernelGGL((k_sur_step<BO, T, A>), grid, blk, 0, s, a, sb, c)
    if (a_bf16) {
        if (bonded) { if (t) MD_LS(true, true, true); else MD_LS(true, false, true); }
        else { if (t) MD_LS(false, true, true); else MD_LS(false, false, true); }
    } else {
        if (bonded) { if (t) MD_LS(true, true, false); else MD_LS(true, false, false); }
        else { if (t) MD_LS(false, true, false); else MD_LS(false, false, false); }
    }
#undef MD_LS
    return hipGetLastError();
}

}  // namespace md

namespace md {

hipError_t launch_batch_rebuild(const BatchCells& bc, const SysEntry* tab, const int32_t* tile_sys, int64_t ntiles,
                                int parity, hipStream_t s, hipEvent_t ev_sorted) {
    const dim3 tg((unsigned)ntiles), blk(kBlock);
    hipLaunchKernelGGL(k_batch_any, dim3(1), dim3(256), 0, s, bc);
    hipLaunchKernelGGL(k_batch_bin, tg, blk, 0, s, tab, tile_sys, parity);
    hipLaunchKernelGGL(k_scan_reduce, dim3(kScanBlocks), dim3(kBlock), 0, s, bc.gg, bc.gb);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanBlocks), 0, s, bc.gb);
    hipLaunchKernelGGL(k_scan_apply, dim3(kScanBlocks), dim3(kBlock), 0, s, bc.gg, bc.gb);
    hipLaunchKernelGGL(k_batch_bases, dim3(1), dim3(256), 0, s, bc);
    hipLaunchKernelGGL(k_batch_localize, dim3(grid_for(bc.gg.ncell, 4096)), blk, 0, s, bc);
    hipLaunchKernelGGL(k_batch_scatter, tg, blk, 0, s, tab, tile_sys);
    hipLaunchKernelGGL(k_batch_permute, tg, blk, 0, s, tab, tile_sys, parity);
    hipLaunchKernelGGL(k_batch_commit, tg, blk, 0, s, tab, tile_sys, parity);
    if (ev_sorted) (void)hipEventRecord(ev_sorted, s);
    hipLaunchKernelGGL(k_batch_nl, tg, blk, 0, s, tab, tile_sys, parity);
    return hipGetLastError();
}

hipError_t launch_batch_step(const SysEntry* tab, const int32_t* tile_sys, int64_t ntiles, int parity, int mode,
                             int tensor, hipStream_t s) {
    (void)parity;
    (void)mode;
    if (tensor)
        hipLaunchKernelGGL(k_batch_step<true>, dim3((unsigned)ntiles), dim3(kBlock), 0, s, tab, tile_sys);
    else
        hipLaunchKernelGGL(k_batch_step<false>, dim3((unsigned)ntiles), dim3(kBlock), 0, s, tab, tile_sys);
    return hipGetLastError();
}

hipError_t launch_batch_finalize(const SysEntry* tab, int nsys, int mode, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_finalize, dim3(nsys), dim3(kFinal), 0, s, tab, mode);
    return hipGetLastError();
}

hipError_t launch_batch_gather_obs(const SysEntry* tab, int nsys, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_gather_obs, dim3(1), dim3(256), 0, s, tab, nsys, out);
    return hipGetLastError();
}

}  // namespace md
