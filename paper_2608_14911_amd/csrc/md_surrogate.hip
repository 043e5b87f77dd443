// gfx950 kernels of the learned non-bonded surrogate: radial descriptors over
// the Verlet list, the 32 -> 64 -> 64 -> 1 SiLU network (forward and input
// gradient) on tiles of 64 particles, the pair force from the per-particle
// input gradients, and the force-matching training path (loss sensitivity
// pass, analytic double backward with block-level weight-gradient products,
// deterministic reduction, Adam).
//
// Network tiles.  A block of 256 threads (4 wavefronts) works on 64
// particles; activations live in LDS as FP32 rows, weights in LDS as a
// padded image.  Every product O[p][c] = sum_k A[p][k] W[c][k] leaves its
// result with one ownership: wavefront w holds particles 16w..16w+15, lane l
// holds particle 16w + (l & 15) and, per 16-column block cb, the columns
// 16 cb + 4 (l >> 4) + e, e = 0..3.  The FP32 form computes these dot
// products on the vector ALUs; the BF16 form issues
// v_mfma_f32_16x16x16_bf16 with the weights as the 16x16 A operand and the
// activations as the B operand, whose accumulator layout is that same
// ownership, so the two forms share every elementwise step.
#include "md_device.h"

namespace md {

typedef short short4v __attribute__((ext_vector_type(4)));
typedef float float4v __attribute__((ext_vector_type(4)));

constexpr int kSB = 256;          // threads per block of the network kernels
constexpr int kSA32 = 36;         // LDS row stride of 32-wide activations (floats)
constexpr int kSA64 = 68;         // LDS row stride of 64-wide activations

// Matrix-core network (see "inference on the matrix cores" below): the
// feature of K slot s in its 32-wide block, and its inverse.
__host__ __device__ constexpr int slot_feature(int s) {
    return (s & 7) < 4 ? 4 * (s >> 3) + (s & 7) : 16 + 4 * (s >> 3) + (s & 7) - 4;
}
__host__ __device__ constexpr int feature_slot(int k) {
    return k < 16 ? 8 * (k >> 2) + (k & 3) : 8 * ((k - 16) >> 2) + 4 + ((k - 16) & 3);
}
static_assert(feature_slot(slot_feature(13)) == 13 && slot_feature(feature_slot(21)) == 21 &&
                  slot_feature(4) == 16 && feature_slot(31) == 31,
              "slot permutation");

__device__ __forceinline__ float sigm(float z) { return __builtin_amdgcn_rcpf(1.f + __expf(-z)); }

// ------------------------------------------------------------------ block sums

// Deterministic block sum of NV doubles into part[k * gridDim.x + blockIdx.x].
template <int NV>
__device__ __forceinline__ void block_store(const double* v, double* part) {
    __shared__ double red[kBlock / 64][NV];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const double t = wave_sum(v[k]);
        if (lane == 0) red[w][k] = t;
    }
    __syncthreads();
    if ((int)threadIdx.x < NV) {
        double t = 0.0;
        for (int ww = 0; ww < (int)(blockDim.x >> 6); ++ww) t += red[ww][threadIdx.x];
        part[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = t;
    }
}

// ------------------------------------------------------------------ pair force

// F_i = sum_j ((a_i + a_j) . g'(r_ij)) (x_j - x_i) / r_ij over r_ij < r_d.
// Inference: F into s.f, per-block virial (and tensor) partials into
// s.part rows 1..7.  Training: delta_i = (2/M) (F_i - F_ref) into s.delta
// and the squared residual into s.part row 8.

// Row of 32 input gradients: FP32, or BF16 (A16).
template <bool A16>
__device__ __forceinline__ void load_a(const SurBufs& s, int64_t j, float* av) {
    if (A16) {
        const uint4* p = reinterpret_cast<const uint4*>(s.ab + j * kSurNB);
#pragma unroll
        for (int q = 0; q < kSurNB / 8; ++q) {
            const uint4 v = p[q];
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                av[8 * q + 2 * e] = bf16_to_f32(w[e] & 0xffffu);
                av[8 * q + 2 * e + 1] = bf16_to_f32(w[e] >> 16);
            }
        }
    } else {
        const float4* p = reinterpret_cast<const float4*>(s.a + j * kSurNB);
#pragma unroll
        for (int q = 0; q < kSurNB / 4; ++q) {
            const float4 v = p[q];
            av[4 * q] = v.x; av[4 * q + 1] = v.y; av[4 * q + 2] = v.z; av[4 * q + 3] = v.w;
        }
    }
}

template <bool TRAIN, bool A16>
__global__ void __launch_bounds__(kBlock) k_sur_force(Geom g, Bufs b, SurBufs s, SurConst c, int parity,
                                                     const double* __restrict__ fref, double two_over_m,
                                                     int tensor) {
    const int64_t n = g.n;
    const int4* __restrict__ xq = b.xq[parity];
    double acc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = 0.0;
    for (int64_t i = gtid_xcd(); i < n; i += gstride()) {
        const int4 qi = xq[i];
        float ai[kSurNB];
        load_a<A16>(s, i, ai);
        int cnt = b.ncount[i];
        cnt = cnt < g.cap ? cnt : g.cap;
        const int32_t* __restrict__ row = b.nl + nl_base(i, g.cap);
        float fx = 0.f, fy = 0.f, fz = 0.f, w = 0.f;
        float txx = 0.f, tyy = 0.f, tzz = 0.f, txy = 0.f, txz = 0.f, tyz = 0.f;
        for (int k = 0; k < cnt; ++k) {
            const int j = row[nl_off(k)];
            const int4 qj = xq[j];
            const float dx = qdiff(qj.x, qi.x, g.ql[0]);
            const float dy = qdiff(qj.y, qi.y, g.ql[1]);
            const float dz = qdiff(qj.z, qi.z, g.ql[2]);
            const float r2 = dx * dx + dy * dy + dz * dz;
            if (r2 < c.rd2 && r2 > 0.f) {
                const float r = sqrtf(r2);
                float dfc;
                const float fc = sur_cutoff(c, r, dfc);
                float av[kSurNB];
                load_a<A16>(s, j, av);
                float ph[kSurNB];
                sur_basis(c, r, ph);
                // g'_k = phi_k (f_c' - (r - mu_k) f_c / w^2): one subtract, two
                // fused multiply-adds and a multiply per basis function
                const float B = c.inv_w2 * fc;
                float cij = 0.f;
#pragma unroll
                for (int kk = 0; kk < kSurNB; ++kk) {
                    const float t = r - c.mu[kk];
                    const float dg = ph[kk] * fmaf(-t, B, dfc);
                    cij = fmaf(ai[kk] + av[kk], dg, cij);
                }
                const float sc = cij / r;
                fx += sc * dx;
                fy += sc * dy;
                fz += sc * dz;
                w -= cij * r;
                if (!TRAIN && tensor) {
                    // r_ij f_ij with r_ij = -(dx, dy, dz), f_ij = sc (dx, dy, dz)
                    txx -= sc * dx * dx; tyy -= sc * dy * dy; tzz -= sc * dz * dz;
                    txy -= sc * dx * dy; txz -= sc * dx * dz; tyz -= sc * dy * dz;
                }
            }
        }
        if (TRAIN) {
            const int64_t t = b.tag[i];
            const double ex = (double)fx - fref[3 * t], ey = (double)fy - fref[3 * t + 1],
                         ez = (double)fz - fref[3 * t + 2];
            acc[0] += ex * ex + ey * ey + ez * ez;
            s.delta[i] = make_float4((float)(two_over_m * ex), (float)(two_over_m * ey), (float)(two_over_m * ez), 0.f);
        } else {
            s.f[i] = make_float4(fx, fy, fz, 0.f);
            acc[0] += 0.5 * (double)w;
            if (tensor) {
                acc[1] += 0.5 * (double)txx; acc[2] += 0.5 * (double)tyy; acc[3] += 0.5 * (double)tzz;
                acc[4] += 0.5 * (double)txy; acc[5] += 0.5 * (double)txz; acc[6] += 0.5 * (double)tyz;
            }
        }
    }
    if (TRAIN) {
        block_store<1>(acc, s.part + (int64_t)8 * gridDim.x);
    } else {
        block_store<7>(acc, s.part + (int64_t)1 * gridDim.x);
    }
}

// u_i = sum_j ((delta_i - delta_j) . (x_j - x_i) / r_ij) g'(r_ij): the
// sensitivity of the loss to a_i (each a_i enters the pair terms of i as
// the first and of its neighbours as the second index).
__global__ void __launch_bounds__(kBlock) k_sur_u(Geom g, Bufs b, SurBufs s, SurConst c, int parity) {
    const int64_t n = g.n;
    const int4* __restrict__ xq = b.xq[parity];
    for (int64_t i = gtid_xcd(); i < n; i += gstride()) {
        const int4 qi = xq[i];
        const float4 di = s.delta[i];
        int cnt = b.ncount[i];
        cnt = cnt < g.cap ? cnt : g.cap;
        const int32_t* __restrict__ row = b.nl + nl_base(i, g.cap);
        float U[kSurNB];
#pragma unroll
        for (int k = 0; k < kSurNB; ++k) U[k] = 0.f;
        for (int k = 0; k < cnt; ++k) {
            const int j = row[nl_off(k)];
            const int4 qj = xq[j];
            const float dx = qdiff(qj.x, qi.x, g.ql[0]);
            const float dy = qdiff(qj.y, qi.y, g.ql[1]);
            const float dz = qdiff(qj.z, qi.z, g.ql[2]);
            const float r2 = dx * dx + dy * dy + dz * dz;
            if (r2 < c.rd2 && r2 > 0.f) {
                const float r = sqrtf(r2);
                float dfc;
                const float fc = sur_cutoff(c, r, dfc);
                const float4 dj = s.delta[j];
                const float proj = ((di.x - dj.x) * dx + (di.y - dj.y) * dy + (di.z - dj.z) * dz) / r;
                float ph[kSurNB];
                sur_basis(c, r, ph);
                const float B = c.inv_w2 * fc;
#pragma unroll
                for (int q = 0; q < kSurNB; ++q) {
                    const float t = r - c.mu[q];
                    U[q] = fmaf(proj * ph[q], fmaf(-t, B, dfc), U[q]);
                }
            }
        }
        float4* out = reinterpret_cast<float4*>(s.u + i * kSurNB);
#pragma unroll
        for (int q = 0; q < kSurNB / 4; ++q) out[q] = make_float4(U[4 * q], U[4 * q + 1], U[4 * q + 2], U[4 * q + 3]);
    }
}

// ------------------------------------------------------------------ network tiles

// Weight images in LDS.  FP32: the prepared FP32 image (row strides 36/68)
// with the biases; BF16: the prepared BF16 image (row strides 40/72) and the
// FP32 biases.
template <bool BF16>
struct WImage;
template <>
struct WImage<false> {
    alignas(16) float w[kPrepF];
    __device__ const float* W1() const { return w + kPW1; }
    __device__ const float* W1T() const { return w + kPW1T; }
    __device__ const float* W2() const { return w + kPW2; }
    __device__ const float* W2T() const { return w + kPW2T; }
    __device__ const float* bias() const { return w + kPB1; }   // b1, b2, w3, b3
    __device__ void load(const SurBufs& s) {
        const float4* src = reinterpret_cast<const float4*>(s.wp);
        float4* dst = reinterpret_cast<float4*>(w);
        for (int k = threadIdx.x; k < kPrepF / 4; k += blockDim.x) dst[k] = src[k];
    }
};
template <>
struct WImage<true> {
    alignas(16) uint16_t w[kPrepB];
    alignas(16) float bb[kPrepF - kPB1];
    __device__ const uint16_t* W1() const { return w + kQW1; }
    __device__ const uint16_t* W1T() const { return w + kQW1T; }
    __device__ const uint16_t* W2() const { return w + kQW2; }
    __device__ const uint16_t* W2T() const { return w + kQW2T; }
    __device__ const float* bias() const { return bb; }
    __device__ void load(const SurBufs& s) {
        const uint4* src = reinterpret_cast<const uint4*>(s.wb);
        uint4* dst = reinterpret_cast<uint4*>(w);
        for (int k = threadIdx.x; k < kPrepB / 8; k += blockDim.x) dst[k] = src[k];
        for (int k = threadIdx.x; k < kPrepF - kPB1; k += blockDim.x) bb[k] = s.wp[kPB1 + k];
    }
};

// O[p][c] = sum_k A[p][k] W[c][k] for the NC columns this lane owns (see the
// file comment).  A: LDS rows of stride SA; W: LDS rows of stride SW.
template <int NC, int K, int SA, int SW>
__device__ __forceinline__ void tile_gemm(const float* __restrict__ A, const float* __restrict__ W, float* out,
                                          int p, int hq) {
#pragma unroll
    for (int v = 0; v < NC / 4; ++v) out[v] = 0.f;
#pragma unroll 2
    for (int k = 0; k < K; k += 4) {
        const float4 x = *reinterpret_cast<const float4*>(A + p * SA + k);
#pragma unroll
        for (int cb = 0; cb < NC / 16; ++cb)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float4 wv = *reinterpret_cast<const float4*>(W + (16 * cb + 4 * hq + e) * SW + k);
                out[4 * cb + e] += x.x * wv.x + x.y * wv.y + x.z * wv.z + x.w * wv.w;
            }
    }
}

template <int NC, int K, int SA, int SW>
__device__ __forceinline__ void tile_gemm(const float* __restrict__ A, const uint16_t* __restrict__ W, float* out,
                                          int p, int hq) {
    const int r = threadIdx.x & 15;
#pragma unroll
    for (int cb = 0; cb < NC / 16; ++cb) {
        float4v acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < K / 16; ++kb) {
            const float4 x = *reinterpret_cast<const float4*>(A + p * SA + 16 * kb + 4 * hq);
            const short4v bop = {bf16_rne(x.x), bf16_rne(x.y), bf16_rne(x.z), bf16_rne(x.w)};
            const short4v aop = *reinterpret_cast<const short4v*>(W + (16 * cb + r) * SW + 16 * kb + 4 * hq);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(aop, bop, acc, 0, 0, 0);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) out[4 * cb + e] = acc[e];
    }
}

// C[h][m] += sum over the tile's 64 particles p of A[p][h] B[p][m] for the
// entries this lane accumulates: h = 16 w + 4 (l >> 4) + e, m = 16 mb + (l & 15).
template <bool BF16, int NM, int SA, int SB>
__device__ __forceinline__ void tile_wgrad(const float* __restrict__ A, const float* __restrict__ B, float* acc) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, hq = lane >> 4, r = lane & 15;
    if (BF16) {
#pragma unroll
        for (int pb = 0; pb < 4; ++pb) {
            short4v aop, bop[NM / 16];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int p = 16 * pb + 4 * hq + j;
                aop[j] = bf16_rne(A[p * SA + 16 * w + r]);
#pragma unroll
                for (int mb = 0; mb < NM / 16; ++mb) bop[mb][j] = bf16_rne(B[p * SB + 16 * mb + r]);
            }
#pragma unroll
            for (int mb = 0; mb < NM / 16; ++mb) {
                float4v c = {acc[4 * mb], acc[4 * mb + 1], acc[4 * mb + 2], acc[4 * mb + 3]};
                c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(aop, bop[mb], c, 0, 0, 0);
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[4 * mb + e] = c[e];
            }
        }
    } else {
#pragma unroll 4
        for (int p = 0; p < 64; ++p) {
            const float4 a4 = *reinterpret_cast<const float4*>(A + p * SA + 16 * w + 4 * hq);
            const float av[4] = {a4.x, a4.y, a4.z, a4.w};
#pragma unroll
            for (int mb = 0; mb < NM / 16; ++mb) {
                const float bv = B[p * SB + 16 * mb + r];
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[4 * mb + e] += av[e] * bv;
            }
        }
    }
}

// Sum over the 16 lanes that share (l >> 4) (the wavefront's particles).
__device__ __forceinline__ float sum16(float v) {
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Load 64 rows of raw descriptors, standardised: X[p][k] = (G - mean) istd,
// and optionally V[p][k] = U[p][k] istd.  Rows at or past P are zero.
__device__ __forceinline__ void load_rows(const SurBufs& s, const float* __restrict__ G, const float* __restrict__ U,
                                          int64_t base, int64_t P, float* sX, float* sV) {
    const int t = threadIdx.x;
    const int p = t >> 2, c0 = (t & 3) * 8;
    const bool ok = base + p < P;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int c = c0 + 4 * h;
        float4 gv = make_float4(0.f, 0.f, 0.f, 0.f), uv = gv;
        if (ok) {
            gv = *reinterpret_cast<const float4*>(G + (base + p) * kSurNB + c);
            if (U) uv = *reinterpret_cast<const float4*>(U + (base + p) * kSurNB + c);
        }
        const float4 m = *reinterpret_cast<const float4*>(s.gmean + c);
        const float4 is = *reinterpret_cast<const float4*>(s.gistd + c);
        float4 x = make_float4((gv.x - m.x) * is.x, (gv.y - m.y) * is.y, (gv.z - m.z) * is.z, (gv.w - m.w) * is.w);
        if (!ok) x = make_float4(0.f, 0.f, 0.f, 0.f);
        *reinterpret_cast<float4*>(sX + p * kSA32 + c) = x;
        if (U) *reinterpret_cast<float4*>(sV + p * kSA32 + c) = make_float4(uv.x * is.x, uv.y * is.y, uv.z * is.z, uv.w * is.w);
    }
}

// Activation storage of the inference tiles: FP32 rows, or BF16 rows in
// the BF16 form (each value rounded once when stored, then used as a
// matrix-core operand by every product that reads it).
template <bool BF16>
struct Act {
    using T = float;
    static constexpr int S32 = kSA32, S64 = kSA64;
    __device__ static T put(float v) { return v; }
};
template <>
struct Act<true> {
    using T = uint16_t;
    static constexpr int S32 = 40, S64 = 72;
    __device__ static T put(float v) { return (uint16_t)bf16_rne(v); }
};

template <int NC, int K, int SA, int SW>
__device__ __forceinline__ void tile_gemm(const uint16_t* __restrict__ A, const uint16_t* __restrict__ W,
                                          float* out, int p, int hq) {
    const int r = threadIdx.x & 15;
#pragma unroll
    for (int cb = 0; cb < NC / 16; ++cb) {
        float4v acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < K / 16; ++kb) {
            const short4v bop = *reinterpret_cast<const short4v*>(A + p * SA + 16 * kb + 4 * hq);
            const short4v aop = *reinterpret_cast<const short4v*>(W + (16 * cb + r) * SW + 16 * kb + 4 * hq);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(aop, bop, acc, 0, 0, 0);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) out[4 * cb + e] = acc[e];
    }
}

template <bool BF16>
__device__ __forceinline__ void load_x(const SurBufs& s, const float* __restrict__ G, int64_t base, int64_t P,
                                       typename Act<BF16>::T* sX) {
    const int t = threadIdx.x;
    const int p = t >> 2, c0 = (t & 3) * 8;
    const bool ok = base + p < P;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int c = c0 + 4 * h;
        float4 gv = make_float4(0.f, 0.f, 0.f, 0.f);
        if (ok) gv = *reinterpret_cast<const float4*>(G + (base + p) * kSurNB + c);
        const float4 m = *reinterpret_cast<const float4*>(s.gmean + c);
        const float4 is = *reinterpret_cast<const float4*>(s.gistd + c);
        const float xv[4] = {(gv.x - m.x) * is.x, (gv.y - m.y) * is.y, (gv.z - m.z) * is.z, (gv.w - m.w) * is.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) sX[p * Act<BF16>::S32 + c + e] = Act<BF16>::put(ok ? xv[e] : 0.f);
    }
}

// Forward and input gradient on tiles of 64 rows:
//   z1 = W1 x + b1, h1 = silu(z1), z2 = W2 h1 + b2, E = w3 . silu(z2) + b3,
//   gz2 = w3 silu'(z2), gz1 = (W2^T gz2) silu'(z1), dE/dG = (W1^T gz1) istd.
template <bool BF16>
__global__ void __launch_bounds__(kSB) k_sur_mlp(SurBufs s, const float* __restrict__ G, int64_t P,
                                                 float* __restrict__ aout, float* __restrict__ eout,
                                                 double* __restrict__ epart, uint16_t* __restrict__ aout16) {
    using AT = typename Act<BF16>::T;
    constexpr int S32 = Act<BF16>::S32, S64 = Act<BF16>::S64;
    __shared__ WImage<BF16> wi;
    __shared__ __attribute__((aligned(16))) AT sX[64 * S32];
    __shared__ __attribute__((aligned(16))) AT sA[64 * S64];
    __shared__ __attribute__((aligned(16))) AT sB[64 * S64];
    wi.load(s);
    __syncthreads();   // the weight image is complete before any lane reads it
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, hq = lane >> 4;
    const int p = 16 * w + (lane & 15);
    const float* b1 = wi.bias();
    const float* b2 = b1 + 64;
    const float* w3 = b1 + 128;
    const float b3 = b1[192];
    double esum = 0.0;
    const int64_t ntile = (P + 63) / 64;
    for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
        const int64_t base = tile * 64;
        __syncthreads();   // previous tile done with sX/sA/sB
        load_x<BF16>(s, G, base, P, sX);
        __syncthreads();
        float z[16], s1[16];
        tile_gemm<64, 32, S32, BF16 ? kSW1 : kPF1>(sX, wi.W1(), z, p, hq);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int h = 16 * (v >> 2) + 4 * hq + (v & 3);
            const float zz = z[v] + b1[h];
            const float sg = sigm(zz);
            s1[v] = sg * (1.f + zz * (1.f - sg));
            sA[p * S64 + h] = Act<BF16>::put(zz * sg);
        }
        __syncthreads();
        tile_gemm<64, 64, S64, BF16 ? kSW64 : kPF64>(sA, wi.W2(), z, p, hq);
        float e = 0.f;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int h = 16 * (v >> 2) + 4 * hq + (v & 3);
            const float zz = z[v] + b2[h];
            const float sg = sigm(zz);
            e += w3[h] * zz * sg;
            sB[p * S64 + h] = Act<BF16>::put(w3[h] * sg * (1.f + zz * (1.f - sg)));
        }
        e += __shfl_xor(e, 16, 64);
        e += __shfl_xor(e, 32, 64);
        const bool valid = base + p < P;
        if (hq == 0 && valid) {
            if (eout) eout[base + p] = e + b3;
            esum += (double)(e + b3);
        }
        __syncthreads();
        tile_gemm<64, 64, S64, BF16 ? kSW64 : kPF64>(sB, wi.W2T(), z, p, hq);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int h = 16 * (v >> 2) + 4 * hq + (v & 3);
            sA[p * S64 + h] = Act<BF16>::put(z[v] * s1[v]);
        }
        __syncthreads();
        float gx[8];
        tile_gemm<32, 64, S64, BF16 ? kSW64 : kPF64>(sA, wi.W1T(), gx, p, hq);
        if (valid) {
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                const int k0 = 16 * cb + 4 * hq;
                const float4 is = *reinterpret_cast<const float4*>(s.gistd + k0);
                const float4 av = make_float4(gx[4 * cb] * is.x, gx[4 * cb + 1] * is.y, gx[4 * cb + 2] * is.z,
                                              gx[4 * cb + 3] * is.w);
                if (aout) *reinterpret_cast<float4*>(aout + (base + p) * kSurNB + k0) = av;
                if (aout16) {
                    const uint32_t lo = (uint16_t)bf16_rne(av.x) | ((uint32_t)(uint16_t)bf16_rne(av.y) << 16);
                    const uint32_t hi = (uint16_t)bf16_rne(av.z) | ((uint32_t)(uint16_t)bf16_rne(av.w) << 16);
                    *reinterpret_cast<uint2*>(aout16 + (base + p) * kSurNB + k0) = make_uint2(lo, hi);
                }
            }
        }
    }
    if (epart) {
        __syncthreads();
        block_store<1>(&esum, epart);
    }
}

// Double backward on tiles of 64 rows.  With x = standardised G, v = u istd
// (u = dL/da): forward z1, z2; tangents t1 = W1 v, t2 = W2 (silu'(z1) t1);
//   dW1 += r1 x^T + gz1 v^T,  db1 += r1,
//   dW2 += r2 h1^T + gz2 (silu'(z1) t1)^T,  db2 += r2,  dw3 += silu'(z2) t2,
// with gz2 = w3 silu'(z2), r2 = w3 silu''(z2) t2, gh1 = W2^T gz2,
// r1 = (W2^T r2) silu'(z1) + gh1 t1 silu''(z1), gz1 = gh1 silu'(z1).
// Each block accumulates over its tiles and writes one partial gradient row.
template <bool BF16>
__global__ void __launch_bounds__(kSB) k_sur_bwd2(SurBufs s, int64_t P) {
    __shared__ WImage<BF16> wi;
    __shared__ __attribute__((aligned(16))) float sX[64 * kSA32];
    __shared__ __attribute__((aligned(16))) float sV[64 * kSA32];
    __shared__ __attribute__((aligned(16))) float sH[64 * kSA64];    // h1, then r1
    __shared__ __attribute__((aligned(16))) float sT[64 * kSA64];    // silu'(z1) t1, then gz1
    __shared__ __attribute__((aligned(16))) float sG[64 * kSA64];    // gz2
    __shared__ __attribute__((aligned(16))) float sR[64 * kSA64];    // r2
    wi.load(s);
    __syncthreads();   // the weight image is complete before any lane reads it
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, hq = lane >> 4;
    const int p = 16 * w + (lane & 15);
    const float* b1 = wi.bias();
    const float* b2 = b1 + 64;
    const float* w3 = b1 + 128;
    float aW1[8], aW2[16], aB1[16], aB2[16], aW3[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) { aW2[v] = 0.f; aB1[v] = 0.f; aB2[v] = 0.f; aW3[v] = 0.f; }
#pragma unroll
    for (int v = 0; v < 8; ++v) aW1[v] = 0.f;
    const int64_t ntile = (P + 63) / 64;
    for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
        const int64_t base = tile * 64;
        const bool valid = base + p < P;
        __syncthreads();
        load_rows(s, s.G, s.u, base, P, sX, sV);
        __syncthreads();
        float z1[16], t1[16], s1[16], d1[16];
        tile_gemm<64, 32, kSA32, BF16 ? kSW1 : kPF1>(sX, wi.W1(), z1, p, hq);
        tile_gemm<64, 32, kSA32, BF16 ? kSW1 : kPF1>(sV, wi.W1(), t1, p, hq);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int h = 16 * (v >> 2) + 4 * hq + (v & 3);
            const float zz = z1[v] + b1[h];
            const float sg = sigm(zz);
            s1[v] = sg * (1.f + zz * (1.f - sg));
            d1[v] = sg * (1.f - sg) * (2.f + zz * (1.f - 2.f * sg));
            sH[p * kSA64 + h] = valid ? zz * sg : 0.f;
            sT[p * kSA64 + h] = valid ? s1[v] * t1[v] : 0.f;
        }
        __syncthreads();
        float z2[16], t2[16];
        tile_gemm<64, 64, kSA64, BF16 ? kSW64 : kPF64>(sH, wi.W2(), z2, p, hq);
        tile_gemm<64, 64, kSA64, BF16 ? kSW64 : kPF64>(sT, wi.W2(), t2, p, hq);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int h = 16 * (v >> 2) + 4 * hq + (v & 3);
            const float zz = z2[v] + b2[h];
            const float sg = sigm(zz);
            const float s2 = sg * (1.f + zz * (1.f - sg));
            const float d2 = sg * (1.f - sg) * (2.f + zz * (1.f - 2.f * sg));
            const float r2 = valid ? w3[h] * d2 * t2[v] : 0.f;
            sG[p * kSA64 + h] = valid ? w3[h] * s2 : 0.f;
            sR[p * kSA64 + h] = r2;
            aB2[v] += sum16(r2);
            aW3[v] += sum16(valid ? s2 * t2[v] : 0.f);
        }
        __syncthreads();
        float gh[16], q[16];
        tile_gemm<64, 64, kSA64, BF16 ? kSW64 : kPF64>(sG, wi.W2T(), gh, p, hq);
        tile_gemm<64, 64, kSA64, BF16 ? kSW64 : kPF64>(sR, wi.W2T(), q, p, hq);
        tile_wgrad<BF16, 64, kSA64, kSA64>(sR, sH, aW2);
        tile_wgrad<BF16, 64, kSA64, kSA64>(sG, sT, aW2);
        __syncthreads();   // sH / sT are rewritten below
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int h = 16 * (v >> 2) + 4 * hq + (v & 3);
            const float r1 = valid ? q[v] * s1[v] + gh[v] * t1[v] * d1[v] : 0.f;
            sH[p * kSA64 + h] = r1;
            sT[p * kSA64 + h] = valid ? gh[v] * s1[v] : 0.f;
            aB1[v] += sum16(r1);
        }
        __syncthreads();
        tile_wgrad<BF16, 32, kSA64, kSA32>(sH, sX, aW1);
        tile_wgrad<BF16, 32, kSA64, kSA32>(sT, sV, aW1);
    }
    // write this block's partial gradient
    float* out = s.gpart + (int64_t)blockIdx.x * kSurNPpad;
    const int r = lane & 15;
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int e = 0; e < 4; ++e) out[kOW2 + (16 * w + 4 * hq + e) * 64 + 16 * mb + r] = aW2[4 * mb + e];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int e = 0; e < 4; ++e) out[kOW1 + (16 * w + 4 * hq + e) * 32 + 16 * mb + r] = aW1[4 * mb + e];
    __syncthreads();
    float* red = sX;   // [4 waves][3][64]
    if (r == 0) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int h = 16 * (v >> 2) + 4 * hq + (v & 3);
            red[(w * 3 + 0) * 64 + h] = aB1[v];
            red[(w * 3 + 1) * 64 + h] = aB2[v];
            red[(w * 3 + 2) * 64 + h] = aW3[v];
        }
    }
    __syncthreads();
    if (threadIdx.x < 192) {
        const int kind = threadIdx.x >> 6, h = threadIdx.x & 63;
        float t = 0.f;
        for (int ww = 0; ww < 4; ++ww) t += red[(ww * 3 + kind) * 64 + h];
        out[(kind == 0 ? kOB1 : kind == 1 ? kOB2 : kOW3) + h] = t;
    }
    if (threadIdx.x == 192) out[kOB3] = 0.f;
}

// grad[k] (+)= sum over blocks of gpart[blk][k], in block order.
__global__ void __launch_bounds__(kBlock) k_sur_grad_reduce(SurBufs s, int nblk, int accumulate) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= kSurNP) return;
    float t = 0.f;
    for (int b = 0; b < nblk; ++b) t += s.gpart[(int64_t)b * kSurNPpad + k];
    s.grad[k] = accumulate ? s.grad[k] + t : t;
}

// loss (+)= sum of the loss partials, in block order.
__global__ void k_sur_loss_reduce(SurBufs s, int grid, int accumulate) {
    if (threadIdx.x != 0) return;
    double t = 0.0;
    for (int b = 0; b < grid; ++b) t += s.part[(int64_t)8 * grid + b];
    s.loss[0] = accumulate ? s.loss[0] + t : t;
}

// Adam (Kingma and Ba 2015) on the master weights, then nothing else: the
// caller refreshes the prepared images.
__global__ void __launch_bounds__(kBlock) k_sur_adam(SurBufs s, float lr, float beta1, float beta2, float eps,
                                                     float bc1, float bc2) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= kSurNP) return;
    const float g = s.grad[k];
    const float m = beta1 * s.m1[k] + (1.f - beta1) * g;
    const float v = beta2 * s.m2[k] + (1.f - beta2) * g * g;
    s.m1[k] = m;
    s.m2[k] = v;
    s.w[k] -= lr * (m / bc1) / (sqrtf(v / bc2) + eps);
}

// Prepared images of the master weights: FP32 W1, W1^T, W2, W2^T with padded
// rows plus the biases, and the BF16 (round to nearest even) copies.
__global__ void __launch_bounds__(kBlock) k_sur_prepare(SurBufs s) {
    const float* w = s.w;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < 64 * 64; k += gridDim.x * blockDim.x) {
        const int r = k >> 6, c = k & 63;
        // W2 [r][c] and its transpose
        const float w2 = w[kOW2 + r * 64 + c];
        s.wp[kPW2 + r * kPF64 + c] = w2;
        s.wp[kPW2T + c * kPF64 + r] = w2;
        s.wb[kQW2 + r * kSW64 + c] = (uint16_t)bf16_rne(w2);
        s.wb[kQW2T + c * kSW64 + r] = (uint16_t)bf16_rne(w2);
        if (c < 32) {
            const float w1 = w[kOW1 + r * 32 + c];
            s.wp[kPW1 + r * kPF1 + c] = w1;
            s.wp[kPW1T + c * kPF64 + r] = w1;
            s.wb[kQW1 + r * kSW1 + c] = (uint16_t)bf16_rne(w1);
            s.wb[kQW1T + c * kSW64 + r] = (uint16_t)bf16_rne(w1);
        }
        // matrix-core images, K axis in slot order: W1 [64][K=32], W2 [64][K=64],
        // W2^T [64 (h1)][K=64 (h2)], W1^T [32 (input)][K=64 (h1)]
        {
            const int kb = c >> 5, sl = 32 * kb + feature_slot(c & 31);
            s.wm[kM2 + r * kMS64 + sl] = (uint16_t)bf16_rne(w2);
            const int kbr = r >> 5, slr = 32 * kbr + feature_slot(r & 31);
            s.wm[kM2T + c * kMS64 + slr] = (uint16_t)bf16_rne(w2);          // W2^T[c][r] = W2[r][c]
            if (c < 32) {
                const float w1 = w[kOW1 + r * 32 + c];
                s.wm[kM1 + r * kMS1 + feature_slot(c)] = (uint16_t)bf16_rne(w1);
                s.wm[kM1T + c * kMS64 + slr] = (uint16_t)bf16_rne(w1);      // W1^T[c][r] = W1[r][c]
            }
        }
        if (r == 0) {
            s.wp[kPB1 + c] = w[kOB1 + c];
            s.wp[kPB2 + c] = w[kOB2 + c];
            s.wp[kPW3 + c] = w[kOW3 + c];
            if (c == 0) s.wp[kPB3] = w[kOB3];
        }
    }
}

// Descriptor moments for the standardisation constants.  Block b owns rows
// 8b + r, 8b + r + 8 kSurMomBlocks, ... (r = threadIdx / 32) and keeps its
// FP64 sums of G and G^2 per basis function in its own slot of gpart, added
// to across the frames of a call, so that the totals do not depend on timing.
__global__ void __launch_bounds__(kBlock) k_sur_moments(SurBufs s, int64_t n, int accumulate) {
    __shared__ double red[2][kBlock / kSurNB][kSurNB];
    const int col = threadIdx.x & (kSurNB - 1), rl = threadIdx.x / kSurNB;
    constexpr int kRows = kBlock / kSurNB;
    double s1 = 0.0, s2 = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * kRows + rl; r < n; r += (int64_t)gridDim.x * kRows) {
        const double v = s.G[r * kSurNB + col];
        s1 += v;
        s2 += v * v;
    }
    red[0][rl][col] = s1;
    red[1][rl][col] = s2;
    __syncthreads();
    if (threadIdx.x < 2 * kSurNB) {
        const int q = threadIdx.x / kSurNB;
        double t = 0.0;
        for (int k = 0; k < kRows; ++k) t += red[q][k][col];
        double* p = reinterpret_cast<double*>(s.gpart) + (int64_t)blockIdx.x * 2 * kSurNB + q * kSurNB + col;
        *p = accumulate ? *p + t : t;
    }
}

// mean_k = S1_k / cnt and istd_k = 1 / sqrt(S2_k / cnt - mean_k^2 + floor),
// the block sums taken in block order (population variance, clamped at 0).
__global__ void k_sur_moments_final(SurBufs s, int nblk, double cnt, double floor_var, float* g_mean,
                                    float* g_istd) {
    const int col = threadIdx.x;
    if (col >= kSurNB) return;
    const double* p = reinterpret_cast<const double*>(s.gpart);
    double s1 = 0.0, s2 = 0.0;
    for (int b = 0; b < nblk; ++b) {
        s1 += p[(int64_t)b * 2 * kSurNB + col];
        s2 += p[(int64_t)b * 2 * kSurNB + kSurNB + col];
    }
    const double m = s1 / cnt;
    double var = s2 / cnt - m * m;
    if (var < 0.0) var = 0.0;
    g_mean[col] = (float)m;
    g_istd[col] = (float)(1.0 / sqrt(var + floor_var));
}

__global__ void __launch_bounds__(kBlock) k_sur_to_tag(Geom g, Bufs b, const float* src, float* dst) {
    for (int64_t i = gtid(); i < g.n; i += gstride()) {
        const int64_t t = b.tag[i];
        const float4* a = reinterpret_cast<const float4*>(src + i * kSurNB);
        float4* o = reinterpret_cast<float4*>(dst + t * kSurNB);
#pragma unroll
        for (int q = 0; q < kSurNB / 4; ++q) o[q] = a[q];
    }
}

__global__ void __launch_bounds__(kBlock) k_sur_from_tag(Geom g, Bufs b, const float* src, float* dst) {
    for (int64_t i = gtid(); i < g.n; i += gstride()) {
        const int64_t t = b.tag[i];
        const float4* a = reinterpret_cast<const float4*>(src + t * kSurNB);
        float4* o = reinterpret_cast<float4*>(dst + i * kSurNB);
#pragma unroll
        for (int q = 0; q < kSurNB / 4; ++q) o[q] = a[q];
    }
}

__global__ void __launch_bounds__(kBlock) k_sur_f_to_tag(Geom g, Bufs b, const float4* src, double* dst) {
    for (int64_t i = gtid(); i < g.n; i += gstride()) {
        const int64_t t = b.tag[i];
        const float4 f = src[i];
        dst[3 * t] = f.x;
        dst[3 * t + 1] = f.y;
        dst[3 * t + 2] = f.z;
    }
}


// ------------------------------------------------------------------ inference on the matrix cores
//
// The BF16 network on v_mfma_f32_16x16x32_bf16, weights as the A operand
// (16 output features x 32 inputs), 16 particles as the B operand
// (32 inputs x 16 particles).  Lane l of a wavefront holds, with
// q = l >> 4 and n = l & 15: A[n][8q + j] and B[8q + j][n] (j = 0..7) and
// the accumulator D[4q + e][n] (e = 0..3).  A layer's outputs therefore sit
// in lane group q as rows 4q..4q+3 of each 16-row block.  The K axis of every
// weight image is stored in "slot order": in a 32-wide K block, slot
// 8q + j stands for feature 4q + j (j < 4) or 16 + 4q + (j - 4) (j >= 4) of
// the block, which is exactly what lane group q holds of two consecutive
// 16-row output blocks.  One layer's activations thus feed the next layer's
// B operand from registers, with no LDS round trip or lane exchange.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));


constexpr int kXS = 40;          // LDS row stride (bf16) of the per-wave input / output rows

// LDS image of the matrix-core weights and the FP32 biases b1, b2, w3, b3.
struct MImage {
    alignas(16) uint16_t w[kPrepM];
    alignas(16) float bb[196];
    __device__ void load(const SurBufs& s) {
        const uint4* src = reinterpret_cast<const uint4*>(s.wm);
        uint4* dst = reinterpret_cast<uint4*>(w);
        for (int k = threadIdx.x; k < kPrepM / 8; k += blockDim.x) dst[k] = src[k];
        for (int k = threadIdx.x; k < 193; k += blockDim.x) bb[k] = s.wp[kPB1 + k];
    }
};

__device__ __forceinline__ bf16x8 lds_op(const uint16_t* p) { return *reinterpret_cast<const bf16x8*>(p); }

// The network on the 64 particles of one wavefront, in 4 groups of 16.  xs:
// the wave's 64 LDS rows (stride kXS) of standardised inputs in slot order,
// rounded to BF16.  For group g, emit(g, E, a) receives, in every lane, the
// particle's energy E (lane n: particle 16g + n) and a[mb][e] = dE/dx for
// input feature 16 mb + 4q + e.  Activations are rounded to BF16 as matrix
// operands; sums, biases, SiLU and its derivative are FP32.
//   z1 = W1 x + b1, h1 = silu(z1), z2 = W2 h1 + b2, E = w3 . silu(z2) + b3,
//   gz2 = w3 silu'(z2), gz1 = (W2^T gz2) silu'(z1), dE/dx = W1^T gz1.
template <typename Emit>
__device__ __forceinline__ void net16_wave(const MImage& wi, const uint16_t* __restrict__ xs, Emit emit) {
    const int lane = threadIdx.x & 63, q = lane >> 4, n = lane & 15;
    const float* b1 = wi.bb;
    const float* b2 = wi.bb + 64;
    const float* w3 = wi.bb + 128;
    const float b3 = wi.bb[192];
    const uint16_t* W1 = wi.w + kM1;
    const uint16_t* W2 = wi.w + kM2;
    const uint16_t* W2T = wi.w + kM2T;
    const uint16_t* W1T = wi.w + kM1T;
#pragma unroll 1
    for (int g = 0; g < 4; ++g) {
        const bf16x8 x = lds_op(xs + (16 * g + n) * kXS + 8 * q);
        f32x4 z[4];
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
            const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
            z[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lds_op(W1 + (16 * mb + n) * kMS1 + 8 * q), x, zero, 0, 0,
                                                             0);
        }
        __builtin_amdgcn_sched_barrier(0);
        float s1[16];
        bf16x8 h[2];
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
            const float4 bv = *reinterpret_cast<const float4*>(b1 + 16 * mb + 4 * q);
            const float bs[4] = {bv.x, bv.y, bv.z, bv.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float zz = z[mb][e] + bs[e];
                const float sg = sigm(zz);
                s1[4 * mb + e] = sg * (1.f + zz * (1.f - sg));
                h[mb >> 1][4 * (mb & 1) + e] = (__bf16)(zz * sg);
            }
        }
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < 2; ++kb)
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lds_op(W2 + (16 * mb + n) * kMS64 + 32 * kb + 8 * q),
                                                              h[kb], acc, 0, 0, 0);
            z[mb] = acc;
        }
        __builtin_amdgcn_sched_barrier(0);
        float en = 0.f;
        bf16x8 gz[2];
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
            const float4 bv = *reinterpret_cast<const float4*>(b2 + 16 * mb + 4 * q);
            const float4 wv = *reinterpret_cast<const float4*>(w3 + 16 * mb + 4 * q);
            const float bs[4] = {bv.x, bv.y, bv.z, bv.w}, ws[4] = {wv.x, wv.y, wv.z, wv.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float zz = z[mb][e] + bs[e];
                const float sg = sigm(zz);
                en += ws[e] * zz * sg;
                gz[mb >> 1][4 * (mb & 1) + e] = (__bf16)(ws[e] * sg * (1.f + zz * (1.f - sg)));
            }
        }
        en += __shfl_xor(en, 16, 64);
        en += __shfl_xor(en, 32, 64);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < 2; ++kb)
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lds_op(W2T + (16 * mb + n) * kMS64 + 32 * kb + 8 * q),
                                                              gz[kb], acc, 0, 0, 0);
            z[mb] = acc;
        }
        __builtin_amdgcn_sched_barrier(0);
        bf16x8 g1[2];
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
#pragma unroll
            for (int e = 0; e < 4; ++e) g1[mb >> 1][4 * (mb & 1) + e] = (__bf16)(z[mb][e] * s1[4 * mb + e]);
        f32x4 a[2];
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < 2; ++kb)
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lds_op(W1T + (16 * mb + n) * kMS64 + 32 * kb + 8 * q),
                                                              g1[kb], acc, 0, 0, 0);
            a[mb] = acc;
        }
        emit(g, en + b3, a);
    }
}

// Standardise a descriptor row (FP32, natural order) into the lane's LDS row
// in slot order, rounded to BF16; rows of absent particles are zero.
__device__ __forceinline__ void put_x_row(const float* G, const float* __restrict__ gmean,
                                          const float* __restrict__ gistd, bool ok, uint16_t* row) {
#pragma unroll
    for (int s8 = 0; s8 < 4; ++s8) {
        bf16x8 v;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = slot_feature(8 * s8 + j);
            v[j] = (__bf16)(ok ? (G[k] - gmean[k]) * gistd[k] : 0.f);
        }
        *reinterpret_cast<bf16x8*>(row + 8 * s8) = v;
    }
}

// Descriptor G(i) of one particle (FP32): its list row streamed in batches
// of 4 slots, the next batch's indices loaded before this batch's position
// gathers are used.  Rows are padded to a multiple of 8 slots with the
// particle itself (r = 0, skipped).
__device__ __forceinline__ void desc_row(const Geom& g, const Bufs& b, const SurConst& c, const int4* __restrict__ xq,
                                         int64_t i, float* G) {
    const int4 qi = xq[i];
    int cnt = b.ncount[i];
    cnt = cnt < g.cap ? cnt : g.cap;
    const int nslots = min((cnt + 7) & ~7, g.cap);
    const int32_t* __restrict__ row = b.nl + nl_base(i, g.cap);
#pragma unroll
    for (int k = 0; k < kSurNB; ++k) G[k] = 0.f;
    constexpr int B = 4;
    const int last = nslots > 0 ? nslots - 1 : 0;
    int jn[B];
#pragma unroll
    for (int u = 0; u < B; ++u) jn[u] = row[nl_off(u < last ? u : last)];
    for (int k0 = 0; k0 < nslots; k0 += B) {
        int4 qj[B];
#pragma unroll
        for (int u = 0; u < B; ++u) qj[u] = xq[jn[u]];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const int kk = k0 + B + u;
            jn[u] = row[nl_off(kk < last ? kk : last)];
        }
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const float dx = qdiff(qj[u].x, qi.x, g.ql[0]);
            const float dy = qdiff(qj[u].y, qi.y, g.ql[1]);
            const float dz = qdiff(qj[u].z, qi.z, g.ql[2]);
            const float r2 = dx * dx + dy * dy + dz * dz;
            if (r2 < c.rd2 && r2 > 0.f) {
                const float r = sqrtf(r2);
                float dfc;
                const float fc = sur_cutoff(c, r, dfc);
                float ph[kSurNB];
                sur_basis(c, r, ph);
#pragma unroll
                for (int k = 0; k < kSurNB; ++k) G[k] = fmaf(ph[k], fc, G[k]);
            }
        }
    }
}

// Descriptors of one 256-particle tile per block (XCD-aware block order).
// NET = false: the FP32 rows go to s.G.  NET = true: each wavefront runs the
// BF16 network on its 64 particles straight from registers and LDS, writes
// the BF16 input gradients a_i to s.ab and the block's energy sum to
// s.part row 0; the descriptors never reach HBM.
template <bool NET>
__global__ void __launch_bounds__(kBlock) k_sur_desc2(Geom g, Bufs b, SurBufs s, SurConst c, int parity) {
    const int64_t n = g.n;
    const int64_t tile = xcd_block(blockIdx.x, gridDim.x);
    const int64_t i = tile * kBlock + threadIdx.x;
    const bool ok = i < n;
    float G[kSurNB];
    if (!NET) {
        if (ok) {
            desc_row(g, b, c, b.xq[parity], i, G);
            float4* out = reinterpret_cast<float4*>(s.G + i * kSurNB);
#pragma unroll
            for (int q = 0; q < kSurNB / 4; ++q) out[q] = make_float4(G[4 * q], G[4 * q + 1], G[4 * q + 2], G[4 * q + 3]);
        }
        return;
    }
    __shared__ MImage wi;
    __shared__ __attribute__((aligned(16))) uint16_t xs[kBlock / 64][64 * kXS];
    __shared__ float es[kBlock / 64][64];
    wi.load(s);
    if (ok) desc_row(g, b, c, b.xq[parity], i, G);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, q = lane >> 4, nn = lane & 15;
    uint16_t* xw = xs[w];
    put_x_row(G, s.gmean, s.gistd, ok, xw + lane * kXS);
    __syncthreads();   // weight image and input rows complete
    net16_wave(wi, xw, [&](int gi, float e, const f32x4* a) {
        // the group's rows were read by its first product: reuse them for
        // dE/dG = (dE/dx) istd in natural feature order
        uint16_t* orow = xw + (16 * gi + nn) * kXS;
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
            const int k0 = 16 * mb + 4 * q;
            const float4 is = *reinterpret_cast<const float4*>(s.gistd + k0);
            const uint32_t lo = (uint16_t)bf16_rne(a[mb][0] * is.x) | ((uint32_t)(uint16_t)bf16_rne(a[mb][1] * is.y) << 16);
            const uint32_t hi = (uint16_t)bf16_rne(a[mb][2] * is.z) | ((uint32_t)(uint16_t)bf16_rne(a[mb][3] * is.w) << 16);
            *reinterpret_cast<uint2*>(orow + k0) = make_uint2(lo, hi);
        }
        if (q == 0) es[w][16 * gi + nn] = e;
    });
    __syncthreads();   // output rows complete
    // the wave's 64 consecutive particles: 4 KB of contiguous BF16 rows
    const int64_t base = tile * kBlock + 64 * w;
#pragma unroll
    for (int cch = 0; cch < 4; ++cch) {
        const int idx = 64 * cch + lane, r = idx >> 2, part = idx & 3;
        if (base + r < n)
            *reinterpret_cast<uint4*>(s.ab + (base + r) * kSurNB + 8 * part) =
                *reinterpret_cast<const uint4*>(xw + r * kXS + 8 * part);
    }
    double esum = ok ? (double)es[w][lane] : 0.0;
    block_store<1>(&esum, s.part);
}

// The BF16 network on given descriptor rows G [P][32] (raw; the handle's
// standardisation is applied): energies e [P] (may be null) and FP32 input
// gradients a [P][32].  One wavefront per 64 rows.
__global__ void __launch_bounds__(kBlock) k_sur_mlp16(SurBufs s, const float* __restrict__ G, int64_t P,
                                                     float* __restrict__ aout, float* __restrict__ eout) {
    __shared__ MImage wi;
    __shared__ __attribute__((aligned(16))) uint16_t xs[kBlock / 64][64 * kXS];
    wi.load(s);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, q = lane >> 4, nn = lane & 15;
    const int64_t base = (int64_t)blockIdx.x * kBlock + 64 * w;
    const bool ok = base + lane < P;
    float Gr[kSurNB];
#pragma unroll
    for (int k = 0; k < kSurNB; ++k) Gr[k] = ok ? G[(base + lane) * kSurNB + k] : 0.f;
    put_x_row(Gr, s.gmean, s.gistd, ok, xs[w] + lane * kXS);
    __syncthreads();
    net16_wave(wi, xs[w], [&](int gi, float e, const f32x4* a) {
        const int64_t p = base + 16 * gi + nn;
        if (p >= P) return;
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
            const int k0 = 16 * mb + 4 * q;
            const float4 is = *reinterpret_cast<const float4*>(s.gistd + k0);
            *reinterpret_cast<float4*>(aout + p * kSurNB + k0) =
                make_float4(a[mb][0] * is.x, a[mb][1] * is.y, a[mb][2] * is.z, a[mb][3] * is.w);
        }
        if (q == 0 && eout) eout[p] = e;
    });
}

// ------------------------------------------------------------------ launchers

static inline int sgrid(int64_t n, int cap_blocks) {
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > cap_blocks) g = cap_blocks;
    return (int)g;
}

int sur_bwd2_grid(int64_t P) {
    int64_t t = (P + 63) / 64;
    if (t < 1) t = 1;
    return (int)(t < kSurGradBlocks ? t : kSurGradBlocks);
}

hipError_t launch_sur_prepare(const SurBufs& s, hipStream_t st) {
    hipLaunchKernelGGL(k_sur_prepare, dim3(16), dim3(kBlock), 0, st, s);
    return hipGetLastError();
}

hipError_t launch_sur_mlp(const SurBufs& s, const float* G, int64_t P, float* a, float* e, double* epart,
                          int bf16, int grid, hipStream_t st, uint16_t* a16) {
    if (bf16)
        hipLaunchKernelGGL(k_sur_mlp<true>, dim3(grid), dim3(kSB), 0, st, s, G, P, a, e, epart, a16);
    else
        hipLaunchKernelGGL(k_sur_mlp<false>, dim3(grid), dim3(kSB), 0, st, s, G, P, a, e, epart, a16);
    return hipGetLastError();
}

hipError_t launch_sur_force(const Geom& g, const Bufs& b, const SurBufs& s, const SurConst& c, int parity,
                            const double* fref, double two_over_m, int tensor, int grid, hipStream_t st,
                            int a_bf16) {
    if (fref)
        hipLaunchKernelGGL((k_sur_force<true, false>), dim3(grid), dim3(kBlock), 0, st, g, b, s, c, parity, fref,
                           two_over_m, 0);
    else if (a_bf16)
        hipLaunchKernelGGL((k_sur_force<false, true>), dim3(grid), dim3(kBlock), 0, st, g, b, s, c, parity, nullptr,
                           0.0, tensor);
    else
        hipLaunchKernelGGL((k_sur_force<false, false>), dim3(grid), dim3(kBlock), 0, st, g, b, s, c, parity,
                           nullptr, 0.0, tensor);
    return hipGetLastError();
}

hipError_t launch_sur_desc2(const Geom& g, const Bufs& b, const SurBufs& s, const SurConst& c, int parity, int net,
                            hipStream_t st) {
    const dim3 grid((unsigned)((g.n + kBlock - 1) / kBlock)), blk(kBlock);
    if (net)
        hipLaunchKernelGGL(k_sur_desc2<true>, grid, blk, 0, st, g, b, s, c, parity);
    else
        hipLaunchKernelGGL(k_sur_desc2<false>, grid, blk, 0, st, g, b, s, c, parity);
    return hipGetLastError();
}

hipError_t launch_sur_mlp16(const SurBufs& s, const float* G, int64_t P, float* a, float* e, hipStream_t st) {
    const int64_t blocks = (P + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_sur_mlp16, dim3((unsigned)(blocks < 1 ? 1 : blocks)), dim3(kBlock), 0, st, s, G, P, a, e);
    return hipGetLastError();
}

hipError_t launch_sur_u(const Geom& g, const Bufs& b, const SurBufs& s, const SurConst& c, int parity, int grid,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_sur_u, dim3(grid), dim3(kBlock), 0, st, g, b, s, c, parity);
    return hipGetLastError();
}

hipError_t launch_sur_bwd2(const SurBufs& s, int64_t P, int bf16, hipStream_t st) {
    const int grid = sur_bwd2_grid(P);
    if (bf16)
        hipLaunchKernelGGL(k_sur_bwd2<true>, dim3(grid), dim3(kSB), 0, st, s, P);
    else
        hipLaunchKernelGGL(k_sur_bwd2<false>, dim3(grid), dim3(kSB), 0, st, s, P);
    return hipGetLastError();
}

hipError_t launch_sur_grad_reduce(const SurBufs& s, int nblk, int accumulate, hipStream_t st) {
    hipLaunchKernelGGL(k_sur_grad_reduce, dim3((kSurNP + kBlock - 1) / kBlock), dim3(kBlock), 0, st, s, nblk,
                       accumulate);
    return hipGetLastError();
}

hipError_t launch_sur_loss_reduce(const SurBufs& s, int grid, int accumulate, hipStream_t st) {
    hipLaunchKernelGGL(k_sur_loss_reduce, dim3(1), dim3(64), 0, st, s, grid, accumulate);
    return hipGetLastError();
}

hipError_t launch_sur_adam(const SurBufs& s, int64_t t, float lr, float beta1, float beta2, float eps,
                           hipStream_t st) {
    const float bc1 = (float)(1.0 - pow((double)beta1, (double)t));
    const float bc2 = (float)(1.0 - pow((double)beta2, (double)t));
    hipLaunchKernelGGL(k_sur_adam, dim3((kSurNP + kBlock - 1) / kBlock), dim3(kBlock), 0, st, s, lr, beta1, beta2,
                       eps, bc1, bc2);
    return hipGetLastError();
}

hipError_t launch_sur_moments(const SurBufs& s, int64_t n, int accumulate, hipStream_t st) {
    hipLaunchKernelGGL(k_sur_moments, dim3(kSurMomBlocks), dim3(kBlock), 0, st, s, n, accumulate);
    return hipGetLastError();
}

hipError_t launch_sur_moments_final(const SurBufs& s, double cnt, double floor_var, float* g_mean, float* g_istd,
                                    hipStream_t st) {
    hipLaunchKernelGGL(k_sur_moments_final, dim3(1), dim3(64), 0, st, s, kSurMomBlocks, cnt, floor_var, g_mean,
                       g_istd);
    return hipGetLastError();
}

hipError_t launch_sur_to_tag(const Geom& g, const Bufs& b, const float* src, float* dst, hipStream_t st) {
    hipLaunchKernelGGL(k_sur_to_tag, dim3(sgrid(g.n, 4096)), dim3(kBlock), 0, st, g, b, src, dst);
    return hipGetLastError();
}

}  // namespace md

namespace md {
hipError_t launch_sur_from_tag(const Geom& g, const Bufs& b, const float* src, float* dst, hipStream_t st) {
    hipLaunchKernelGGL(k_sur_from_tag, dim3(sgrid(g.n, 4096)), dim3(kBlock), 0, st, g, b, src, dst);
    return hipGetLastError();
}

hipError_t launch_sur_f_to_tag(const Geom& g, const Bufs& b, const float4* src, double* dst, hipStream_t st) {
    hipLaunchKernelGGL(k_sur_f_to_tag, dim3(sgrid(g.n, 4096)), dim3(kBlock), 0, st, g, b, src, dst);
    return hipGetLastError();
}
}  // namespace md
