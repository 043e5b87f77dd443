// Device helpers shared by the gfx950 kernel files of the MD step: fixed-
// point coordinates, wavefront sums, the XCD-aware block order and the
// Verlet-list layout.
#pragma once

#include "md_internal.h"

namespace md {

// 32-bit fixed-point coordinate: q = floor(x 2^32 / L) for x in [0, L); a
// product that rounds up to 2^32 wraps to 0, the same point of the periodic
// box.  The difference (int32)(q_j - q_i) is the minimum image.
__device__ __forceinline__ uint32_t quantize(double x, double qs) { return (uint32_t)(uint64_t)(x * qs); }
__device__ __forceinline__ float qdiff(uint32_t a, uint32_t b, float ql) {
    return (float)(int32_t)(a - b) * ql;
}
__device__ __forceinline__ int4 quantize4(const Geom& g, double x, double y, double z, double w) {
    return make_int4((int)quantize(x, g.qs[0]), (int)quantize(y, g.qs[1]), (int)quantize(z, g.qs[2]), (int)w);
}

// 12-byte fixed-point record (x, y, z): the fast step kernel gathers these,
// 25 instead of 29 distinct 128-byte lines per 64-lane gather on the LJ
// fluid's lists (counted on the CPU) against 16-byte records.
struct alignas(4) Q3 {
    int32_t x, y, z;
};
__device__ __forceinline__ void store_q3(int32_t* p, int64_t i, const int4& q) {
    p[3 * i] = q.x;
    p[3 * i + 1] = q.y;
    p[3 * i + 2] = q.z;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ int64_t gtid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }

// Workgroups are handed to the 8 XCDs round-robin (block b -> XCD b % 8),
// and each XCD has its own L2.  Remap so that XCD x works on one contiguous
// 1/8 of the cell-sorted particles: a spatially compact slab whose gathered
// neighbour records stay in that XCD's L2.  Bijective for any grid size.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block(int b, int G) {
    const int q = G / kXcds, r = G % kXcds;
    const int x = b % kXcds, k = b / kXcds;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}
// Verlet-list layout: tiles of 64 particles (one wavefront); inside a tile
// slot k of all 64 particles is contiguous (256 bytes), and a tile's slots
// follow each other, so a wavefront streams one contiguous block.  (Chunks of
// 4 slots per lane, written by the tile build as 16-byte stores, were slower:
// the register shifting cost the build more VALU than the stores it saved.)
constexpr int kTile = 64;
__device__ __forceinline__ int64_t nl_base(int64_t i, int cap) {
    return (i >> 6) * (int64_t)cap * kTile + (i & (kTile - 1));
}
// offset of slot k from a row's base (nl_base), in entries
__device__ __forceinline__ int nl_off(int k) { return k * kTile; }

__device__ __forceinline__ int64_t gtid_xcd() {
    return (int64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
}
__device__ __forceinline__ int64_t gstride() { return (int64_t)gridDim.x * blockDim.x; }

// ------------------------------------------------------------------ surrogate helpers

// FP32 -> BF16, round to nearest even (NaN stays NaN).
__device__ __forceinline__ short bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (short)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint32_t h) { return __uint_as_float(h << 16); }

// f_c(r) = (cos(pi r / r_d) + 1) / 2 and its derivative.
__device__ __forceinline__ float sur_cutoff(const SurConst& c, float r, float& dfc) {
    // argument in [0, pi]: the hardware sine / cosine are accurate to a few
    // 1e-7 there
    float sn, cs;
    __sincosf(c.pi_rd * r, &sn, &cs);
    dfc = -0.5f * c.pi_rd * sn;
    return 0.5f * (cs + 1.f);
}

// phi_k(r) = exp(-(r - mu_k)^2 / (2 w^2)) for k = 0..31 by two-sided
// recurrences from pivots k = 8 and 24: with t = r - mu_p,
//   phi_{p+1} / phi_p = exp2(c (2 D t - D^2)),  phi_{p-1} / phi_p = exp2(c (-2 D t - D^2)),
// and each further ratio is the previous one times exp2(-2 c D^2)
// (c = log2(e) / (2 w^2), D the centre spacing): 6 exponentials per pair
// instead of 32, chains of at most 8 products.
__device__ __forceinline__ void sur_basis(const SurConst& c, float r, float* phi) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int p = 8 + 16 * h;
        const float t = r - c.mu[p];
        phi[p] = __builtin_amdgcn_exp2f(-c.c_exp * t * t);
        float up = __builtin_amdgcn_exp2f(c.c_exp * (2.f * c.dmu * t - c.dmu * c.dmu));
        float dn = __builtin_amdgcn_exp2f(c.c_exp * (-2.f * c.dmu * t - c.dmu * c.dmu));
#pragma unroll
        for (int m = 1; m <= 8; ++m) {
            phi[p - m] = phi[p - m + 1] * dn;
            dn *= c.ratio;
            if (m <= 7) {
                phi[p + m] = phi[p + m - 1] * up;
                up *= c.ratio;
            }
        }
    }
}

}  // namespace md
