// Shared device helpers for librmips (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rmips {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int WAVE = 64;
constexpr int KMAX = 32;          // largest k (matches RMIPS_K_MAX)
constexpr int TILE_ITEMS = 64;    // items per streamed tile in stage (a)
constexpr int LDS_PAD = 4;        // floats added to an LDS row (bank spread)
// Absolute term of every screening error bound: covers the rounding of
// products and sums that fall into the FP32 subnormal range.
constexpr float E_ABS = 0x1p-99f;

// Padded dimensionality of the FP32 matrix-core path: the 32x32x2 product
// is fed four k-steps at a time from LDS (one 16-byte read per lane), and
// each half-wave owns a contiguous half of the row, so D is a multiple of 8.
__host__ __device__ inline int padded_dim_fp32(int d) { return (d + 7) & ~7; }

// Output layout of a 32x32 matrix-core block: lane l holds column (l & 31)
// and, in register i, row 8*(i/4) + 4*(l/32) + (i%4).
__device__ __forceinline__ int mfma32_row(int i, int lane) {
    return 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
}

// One 32x32 block of Out[r][c] = sum_k A[r][k] * B[c][k] in FP32 on the
// matrix cores.  A and B are row-major in LDS with row stride `ld` floats;
// both operands hold rows of length D = 2*ks, and half-wave h supplies the
// dims [h*ks, (h+1)*ks) of its row (any split of the dims between the two
// halves gives the same sum; this one makes every read contiguous).
__device__ __forceinline__ void mfma32_f32(f32x16 &acc, const float *A,
                                           const float *B, int ld, int ks,
                                           int lane) {
    const int r = lane & 31, h = lane >> 5;
    const float *a = A + r * ld + h * ks;
    const float *b = B + r * ld + h * ks;
    for (int s = 0; s < ks; s += 4) {
        f32x4 av = *reinterpret_cast<const f32x4 *>(a + s);
        f32x4 bv = *reinterpret_cast<const f32x4 *>(b + s);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[0], bv[0], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[1], bv[1], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[2], bv[2], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[3], bv[3], acc, 0, 0, 0);
    }
}

// Two blocks sharing the B operand (rows rb0 and rb1 of A), interleaved so
// the two accumulation chains overlap in the matrix pipeline.
__device__ __forceinline__ void mfma32x2_f32(f32x16 &acc0, f32x16 &acc1,
                                             const float *A0, const float *A1,
                                             const float *B, int ld, int ks,
                                             int lane) {
    const int r = lane & 31, h = lane >> 5;
    const float *a0 = A0 + r * ld + h * ks;
    const float *a1 = A1 + r * ld + h * ks;
    const float *b = B + r * ld + h * ks;
    for (int s = 0; s < ks; s += 4) {
        f32x4 av0 = *reinterpret_cast<const f32x4 *>(a0 + s);
        f32x4 av1 = *reinterpret_cast<const f32x4 *>(a1 + s);
        f32x4 bv = *reinterpret_cast<const f32x4 *>(b + s);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(av0[q], bv[q], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(av1[q], bv[q], acc1, 0, 0, 0);
        }
    }
}

// Exact value of u . p: FP64 sum of the exact products of the FP32 inputs,
// taken in index order from +0.0.  fma() adds the exact product with one
// rounding, which is what a separate multiply (exact) and add would give.
__device__ __forceinline__ double ip64(const float *__restrict__ u,
                                       const float *__restrict__ p, int d) {
    double acc = 0.0;
    for (int i = 0; i < d; ++i)
        acc = __fma_rn((double)u[i], (double)p[i], acc);
    return acc;
}

// Pair rule of the tie order: item `id` with value v belongs to S_k(u) iff
// (v, -id) >= (tau, -tau_id) lexicographically.
__device__ __forceinline__ bool in_topk(double v, int id, double tau, int tau_id) {
    return v > tau || (v == tau && id <= tau_id);
}

// Monotone map from float to uint32 (ascending float -> ascending key).
__device__ __forceinline__ uint32_t float_key(float f) {
    uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__device__ __forceinline__ float wave_min(float x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = fminf(x, __shfl_xor(x, o));
    return x;
}

__device__ __forceinline__ int wave_sum(int x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

}  // namespace rmips
