// Shared device helpers for librmips (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <type_traits>
#include <stdint.h>

namespace rmips {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

// Screening precisions (values of rmips_prec).  FP8 e4m3, FP6 e2m3 and FP4
// e2m1 share one layout: a 32-byte slot per 32 elements (one element per byte
// for FP8; FP6 and FP4 pack the block's codes from the slot's first bit, 24 or
// 16 bytes, the rest zero), a power-of-two scale per vector.
enum { PREC_FP32 = 0, PREC_BF16 = 1, PREC_FP8 = 2, PREC_FP6 = 3, PREC_FP4 = 4 };
__host__ __device__ constexpr bool scaled_prec(int prec) { return prec >= PREC_FP8; }
// format code of the f8f6f4 matrix-core instruction and bits per element
__host__ __device__ constexpr int mx_format(int prec) {
    return prec == PREC_FP6 ? 2 : prec == PREC_FP4 ? 4 : 0;
}
__host__ __device__ constexpr int mx_bits(int prec) {
    return prec == PREC_FP6 ? 6 : prec == PREC_FP4 ? 4 : 8;
}
// largest magnitude of the element format (the scale maps a row's largest
// value at or below it)
__host__ __device__ constexpr float mx_max(int prec) {
    return prec == PREC_FP6 ? 7.5f : prec == PREC_FP4 ? 6.0f : 448.0f;
}

constexpr int WAVE = 64;
constexpr int KMAX = 32;          // largest k (matches RMIPS_K_MAX)
constexpr int DMAX = 256;         // largest d (matches RMIPS_D_MAX)
constexpr int TILE_ITEMS = 64;    // items per streamed tile in stage (a)
constexpr int LDS_PAD = 4;        // floats added to an LDS row (bank spread)
// Absolute term of every screening error bound: covers the rounding of
// products and sums that fall into the FP32 subnormal range.
constexpr float E_ABS = 0x1p-99f;

// FP32 rows split at h = ceil(d / 2): values 0..h-1 open the first half
// (D / 2 slots), values h..d-1 the second, each half padded with zeros at
// its end, so that value slots 4c + q >= h of both halves are zero and their
// matrix-core steps can be skipped.  Slot of value (or padding entry) c < D:
__host__ __device__ inline int fp32_slot(int c, int d, int D) {
    const int h = (d + 1) / 2, gap = D / 2 - h;  // zeros closing the first half
    if (c < h) return c;
    if (c < d) return D / 2 + (c - h);
    if (c < d + gap) return h + (c - d);
    return c;  // zeros closing the second half
}

// Padded dimensionality and element size per screening precision: each
// half-wave owns half of the row; a BF16 step takes 8 elements per lane
// (D multiple of 16), an FP8 step 32 (D multiple of 64).
__host__ __device__ inline int padded_dim(int prec, int d) {
    return prec == PREC_FP32 ? (d + 7) & ~7 : prec == PREC_BF16 ? (d + 15) & ~15 : (d + 63) & ~63;
}
__host__ __device__ inline int elem_bytes(int prec) {
    return prec == PREC_FP32 ? 4 : prec == PREC_BF16 ? 2 : 1;
}
// LDS row stride in bytes (16 bytes of padding spread the banks).
__host__ __device__ inline int lds_row_bytes(int prec, int D) { return D * elem_bytes(prec) + 16; }

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
#pragma unroll 4
    for (int s = 0; s < ks; s += 4) {
        f32x4 av = *reinterpret_cast<const f32x4 *>(a + s);
        f32x4 bv = *reinterpret_cast<const f32x4 *>(b + s);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[0], bv[0], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[1], bv[1], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[2], bv[2], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[3], bv[3], acc, 0, 0, 0);
    }
}

// 32 bytes of FP8 (e4m3) values from LDS as the 8-register operand of the
// FP8 matrix-core product (format code 0, unit block scales 0x7f = 2^0).
__device__ __forceinline__ i32x8 ld_fp8x32(const uint8_t *p) {
    const i32x4 lo = *reinterpret_cast<const i32x4 *>(p);
    const i32x4 hi = *reinterpret_cast<const i32x4 *>(p + 16);
    return i32x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
}

// Products with the stationary operand held in registers: each lane's half
// row as NCH 16-byte chunks (FP32: 4 elements, BF16: 8, FP8: 16), the other
// operand's rows in LDS (row stride ls bytes; half-wave h feeds the dims
// [h*D/2, (h+1)*D/2) of its row, which pairs the same dims of both rows).
// rows2: c0 += A0 B^T, c1 += A1 B^T with B in registers; cols2: c0 += A
// B0^T, c1 += A B1^T with A in registers.  All NCH chunks are multiplied
// without branches, so that the LDS reads run ahead of the products: the
// register chunks past nch are zero and add exact zeros, and the LDS reads
// past a row end stay in the next row or in the LDS_GUARD bytes of zeros
// that follow each buffer (finite values, so 0 * x = 0).  FP32 skips the
// steps of the zero slots of its split layout in the last chunk.
constexpr int LDS_GUARD = 512;  // >= 16 * (32 - 1) bytes of overread

// Register-operand widths that are compiled: BF16 and FP8 rows are multiplied
// over the smallest even chunk count >= nch (every even count up to the
// largest row), FP32 rows over every count up to 16 and multiples of 4
// above.  with_nch calls f(std::integral_constant<int, NCH>).
template <int LO, int HI, class F> void with_exact(int nch, F &&f) {
    if constexpr (LO <= HI) {
        if (nch == LO) f(std::integral_constant<int, LO>{});
        else with_exact<LO + 1, HI>(nch, f);
    }
}
template <int PREC, class F> void with_nch(int nch, F &&f) {
    if constexpr (PREC == PREC_FP32) {
        // every count up to 16 (each chunk costs eight FP32 products), then
        // multiples of 4
        if (nch <= 16) with_exact<1, 16>(nch, f);
        else if (nch <= 20) f(std::integral_constant<int, 20>{});
        else if (nch <= 24) f(std::integral_constant<int, 24>{});
        else if (nch <= 28) f(std::integral_constant<int, 28>{});
        else f(std::integral_constant<int, 32>{});
    } else {
        switch ((nch + 1) & ~1) {
        case 2: f(std::integral_constant<int, 2>{}); break;
        case 4: f(std::integral_constant<int, 4>{}); break;
        case 6: f(std::integral_constant<int, 6>{}); break;
        case 8: f(std::integral_constant<int, 8>{}); break;
        default:
            if constexpr (PREC == PREC_BF16) {  // FP8/FP6/FP4 rows have at most 8 chunks
                switch ((nch + 1) & ~1) {
                case 10: f(std::integral_constant<int, 10>{}); break;
                case 12: f(std::integral_constant<int, 12>{}); break;
                case 14: f(std::integral_constant<int, 14>{}); break;
                default: f(std::integral_constant<int, 16>{}); break;
                }
            }
        }
    }
}
template <int PREC, int NCH> struct MMR;

template <int NCH> struct MMR<PREC_FP32, NCH> {
    // all NCH chunks without branches: chunks from nch on are zero in the
    // register operand and add exact zeros (the LDS reads past a row end
    // land in the next row, the row padding or the zero guard: finite)
    // (h = ceil(d / 2): the steps of value slots 4c + q >= h multiply zeros
    // in both halves, see fp32_slot, and are skipped in the last chunk)
    static __device__ __forceinline__ void rows2(f32x16 &c0, f32x16 &c1, const uint8_t *A0,
                                                 const uint8_t *A1, const uint4 (&b)[NCH],
                                                 int ls, int nch, int D, int h, int lane) {
        const int off = (lane & 31) * ls + (lane >> 5) * (D / 2) * 4;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const f32x4 x0 = *reinterpret_cast<const f32x4 *>(A0 + off + 16 * c);
            const f32x4 x1 = *reinterpret_cast<const f32x4 *>(A1 + off + 16 * c);
            const float y[4] = {__uint_as_float(b[c].x), __uint_as_float(b[c].y),
                                __uint_as_float(b[c].z), __uint_as_float(b[c].w)};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (c < NCH - 1 || 4 * c + q < h) {
                    c0 = __builtin_amdgcn_mfma_f32_32x32x2f32(x0[q], y[q], c0, 0, 0, 0);
                    c1 = __builtin_amdgcn_mfma_f32_32x32x2f32(x1[q], y[q], c1, 0, 0, 0);
                }
            }
        }
    }
    static __device__ __forceinline__ void cols2(f32x16 &c0, f32x16 &c1, const uint4 (&a)[NCH],
                                                 const uint8_t *B0, const uint8_t *B1, int ls,
                                                 int nch, int D, int h, int lane) {
        const int off = (lane & 31) * ls + (lane >> 5) * (D / 2) * 4;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const f32x4 y0 = *reinterpret_cast<const f32x4 *>(B0 + off + 16 * c);
            const f32x4 y1 = *reinterpret_cast<const f32x4 *>(B1 + off + 16 * c);
            const float x[4] = {__uint_as_float(a[c].x), __uint_as_float(a[c].y),
                                __uint_as_float(a[c].z), __uint_as_float(a[c].w)};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (c < NCH - 1 || 4 * c + q < h) {
                    c0 = __builtin_amdgcn_mfma_f32_32x32x2f32(x[q], y0[q], c0, 0, 0, 0);
                    c1 = __builtin_amdgcn_mfma_f32_32x32x2f32(x[q], y1[q], c1, 0, 0, 0);
                }
            }
        }
    }
};

template <int NCH> struct MMR<PREC_BF16, NCH> {
    static __device__ __forceinline__ bf16x8 as_bf(const uint4 &v) {
        return __builtin_bit_cast(bf16x8, v);
    }
    static __device__ __forceinline__ void rows2(f32x16 &c0, f32x16 &c1, const uint8_t *A0,
                                                 const uint8_t *A1, const uint4 (&b)[NCH],
                                                 int ls, int nch, int D, int /*h*/, int lane) {
        const int off = (lane & 31) * ls + (lane >> 5) * (D / 2) * 2;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const bf16x8 x0 = *reinterpret_cast<const bf16x8 *>(A0 + off + 16 * c);
            const bf16x8 x1 = *reinterpret_cast<const bf16x8 *>(A1 + off + 16 * c);
            c0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x0, as_bf(b[c]), c0, 0, 0, 0);
            c1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x1, as_bf(b[c]), c1, 0, 0, 0);
        }
    }
    static __device__ __forceinline__ void cols2(f32x16 &c0, f32x16 &c1, const uint4 (&a)[NCH],
                                                 const uint8_t *B0, const uint8_t *B1, int ls,
                                                 int nch, int D, int /*h*/, int lane) {
        const int off = (lane & 31) * ls + (lane >> 5) * (D / 2) * 2;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const bf16x8 y0 = *reinterpret_cast<const bf16x8 *>(B0 + off + 16 * c);
            const bf16x8 y1 = *reinterpret_cast<const bf16x8 *>(B1 + off + 16 * c);
            c0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf(a[c]), y0, c0, 0, 0, 0);
            c1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf(a[c]), y1, c1, 0, 0, 0);
        }
    }
    // c[h][j] += A_j B_h^T for two register operands B_0, B_1: each chunk
    // read from LDS feeds two products
    static __device__ __forceinline__ void rows4(f32x16 (&c)[2][2], const uint8_t *A0,
                                                 const uint8_t *A1, const uint4 (&b0)[NCH],
                                                 const uint4 (&b1)[NCH], int ls, int D,
                                                 int lane) {
        const int off = (lane & 31) * ls + (lane >> 5) * (D / 2) * 2;
#pragma unroll
        for (int q = 0; q < NCH; ++q) {
            const bf16x8 x0 = *reinterpret_cast<const bf16x8 *>(A0 + off + 16 * q);
            const bf16x8 x1 = *reinterpret_cast<const bf16x8 *>(A1 + off + 16 * q);
            c[0][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x0, as_bf(b0[q]), c[0][0], 0, 0, 0);
            c[0][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x1, as_bf(b0[q]), c[0][1], 0, 0, 0);
            c[1][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x0, as_bf(b1[q]), c[1][0], 0, 0, 0);
            c[1][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x1, as_bf(b1[q]), c[1][1], 0, 0, 0);
        }
    }
};

// FP8 e4m3, FP6 e2m3 and FP4 e2m1: one f8f6f4 product per pair of 16-byte
// chunks (a lane's 32 elements of one block), unit block scales (the
// per-vector power-of-two scales are applied outside).  FMT: the
// instruction's format code for both operands.
template <int FMT, int NCH> struct MMRx {
    static __device__ __forceinline__ i32x8 pair(const uint4 &lo, const uint4 &hi) {
        return i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w,
                     (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
    }
    static __device__ __forceinline__ void rows2(f32x16 &c0, f32x16 &c1, const uint8_t *A0,
                                                 const uint8_t *A1, const uint4 (&b)[NCH],
                                                 int ls, int nch, int D, int /*h*/, int lane) {
        const int off = (lane & 31) * ls + (lane >> 5) * (D / 2);
#pragma unroll
        for (int c = 0; c + 1 < NCH; c += 2) {
            const i32x8 x0 = ld_fp8x32(A0 + off + 16 * c);
            const i32x8 x1 = ld_fp8x32(A1 + off + 16 * c);
            const i32x8 y = pair(b[c], b[c + 1]);
            c0 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(x0, y, c0, FMT, FMT, 0,
                                                                 0x7f7f7f7f, 0, 0x7f7f7f7f);
            c1 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(x1, y, c1, FMT, FMT, 0,
                                                                 0x7f7f7f7f, 0, 0x7f7f7f7f);
        }
    }
    static __device__ __forceinline__ void cols2(f32x16 &c0, f32x16 &c1, const uint4 (&a)[NCH],
                                                 const uint8_t *B0, const uint8_t *B1, int ls,
                                                 int nch, int D, int /*h*/, int lane) {
        const int off = (lane & 31) * ls + (lane >> 5) * (D / 2);
#pragma unroll
        for (int c = 0; c + 1 < NCH; c += 2) {
            const i32x8 x = pair(a[c], a[c + 1]);
            const i32x8 y0 = ld_fp8x32(B0 + off + 16 * c);
            const i32x8 y1 = ld_fp8x32(B1 + off + 16 * c);
            c0 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(x, y0, c0, FMT, FMT, 0,
                                                                 0x7f7f7f7f, 0, 0x7f7f7f7f);
            c1 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(x, y1, c1, FMT, FMT, 0,
                                                                 0x7f7f7f7f, 0, 0x7f7f7f7f);
        }
    }
    // as MMR<PREC_BF16>::rows4
    static __device__ __forceinline__ void rows4(f32x16 (&c)[2][2], const uint8_t *A0,
                                                 const uint8_t *A1, const uint4 (&b0)[NCH],
                                                 const uint4 (&b1)[NCH], int ls, int D,
                                                 int lane) {
        const int off = (lane & 31) * ls + (lane >> 5) * (D / 2);
#pragma unroll
        for (int q = 0; q + 1 < NCH; q += 2) {
            const i32x8 x0 = ld_fp8x32(A0 + off + 16 * q);
            const i32x8 x1 = ld_fp8x32(A1 + off + 16 * q);
            const i32x8 y0 = pair(b0[q], b0[q + 1]);
            const i32x8 y1 = pair(b1[q], b1[q + 1]);
            c[0][0] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(x0, y0, c[0][0], FMT, FMT, 0,
                                                                      0x7f7f7f7f, 0, 0x7f7f7f7f);
            c[0][1] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(x1, y0, c[0][1], FMT, FMT, 0,
                                                                      0x7f7f7f7f, 0, 0x7f7f7f7f);
            c[1][0] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(x0, y1, c[1][0], FMT, FMT, 0,
                                                                      0x7f7f7f7f, 0, 0x7f7f7f7f);
            c[1][1] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(x1, y1, c[1][1], FMT, FMT, 0,
                                                                      0x7f7f7f7f, 0, 0x7f7f7f7f);
        }
    }
};
template <int NCH> struct MMR<PREC_FP8, NCH> : MMRx<0, NCH> {};
template <int NCH> struct MMR<PREC_FP6, NCH> : MMRx<2, NCH> {};
template <int NCH> struct MMR<PREC_FP4, NCH> : MMRx<4, NCH> {};

// Index (0..3) of the SIMD that runs this wave: bits 5:4 of the HW_ID
// hardware register.
__device__ __forceinline__ int simd_id() {
    return __builtin_amdgcn_s_getreg((1 << 11) | (4 << 6) | 4) & 3;  // hwreg(HW_ID, 4, 2)
}

// 1 / x for a power of two x whose reciprocal is a normal float: exact.
__device__ __forceinline__ float pow2_rcp(float x) {
    return __uint_as_float((254u << 23) - (__float_as_uint(x) & 0x7f800000u));
}

// Direct global-to-LDS copies (no registers): each lane copies 16 (or 4)
// bytes from its own global address; lane l's bytes land at lds + 16 l (or
// 4 l), lds being the wave's common LDS address.  They complete under the
// vector-memory counter: dma_wait() before a barrier publishes them.
__device__ __forceinline__ void dma16(const void *g, void *lds) {
    __builtin_amdgcn_global_load_lds(g, (__attribute__((address_space(3))) void *)lds, 16, 0, 0);
}
__device__ __forceinline__ void dma4(const void *g, void *lds) {
    __builtin_amdgcn_global_load_lds(g, (__attribute__((address_space(3))) void *)lds, 4, 0, 0);
}
__device__ __forceinline__ void dma_wait() { __builtin_amdgcn_s_waitcnt(0); }

// Rows 0..63 (row r at src + min(r, rlast) * rowb) into LDS rows of ls =
// rowb + 16 bytes: 64 * (w16 + 1) 16-byte slots, 64 per wave instruction,
// wave w taking instructions w, w + nw, ...  The last slot of each LDS row
// is padding and gets a copy of the row's last vector.  magic =
// ceil(2^32 / (w16 + 1)) splits a slot index into (row, vector) exactly
// for the slot counts used here (at most 64 * 129 slots).
__device__ __forceinline__ void rows_dma(const uint8_t *src, int rowb, int w16, uint32_t magic,
                                         int rlast, uint8_t *dst, int w, int nw, int lane) {
    const int spr = w16 + 1;
    for (int j = w; j < spr; j += nw) {
        const uint32_t s = 64u * (uint32_t)j + (uint32_t)lane;
        const uint32_t r = __umulhi(s, magic);
        uint32_t c = s - r * (uint32_t)spr;
        c = c < (uint32_t)w16 ? c : (uint32_t)(w16 - 1);
        const uint32_t rr = r < (uint32_t)rlast ? r : (uint32_t)rlast;
        dma16(src + (size_t)rr * rowb + 16 * c, dst + 1024 * j);
    }
}
__host__ __device__ inline uint32_t slot_magic(int w16) { return 0xffffffffu / (uint32_t)(w16 + 1) + 1u; }

// Load this lane's half row (nch 16-byte chunks) of row `row` of a
// quantized array with rows of rowb bytes; zeros when row is invalid.
template <int NCH>
__device__ __forceinline__ void load_half_row(uint4 (&r)[NCH], const uint8_t *X, int64_t row,
                                              bool valid, int rowb, int nch, int lane) {
    const uint4 *src = reinterpret_cast<const uint4 *>(X + row * rowb + (lane >> 5) * (rowb / 2));
#pragma unroll
    for (int c = 0; c < NCH; ++c) r[c] = (valid && c < nch) ? src[c] : make_uint4(0, 0, 0, 0);
}

// Round to nearest even BF16; returns the bits, q = the value represented.
__device__ __forceinline__ uint16_t to_bf16(float x, float &q) {
    uint32_t b = __float_as_uint(x);
    b += 0x7fffu + ((b >> 16) & 1u);
    const uint16_t h = (uint16_t)(b >> 16);
    q = __uint_as_float((uint32_t)h << 16);
    return h;
}

// Round to nearest even OCP FP8 e4m3 (bias 7, largest finite 448, no
// infinities); |y| <= 448 is required.  Returns the byte, q = its value.
__device__ __forceinline__ uint8_t to_e4m3(float y, float &q) {
    const float a = fabsf(y);
    const uint8_t sg = (y < 0.0f) ? 0x80 : 0x00;
    if (a == 0.0f) {
        q = 0.0f;
        return 0;
    }
    int e = (int)((__float_as_uint(a) >> 23) & 0xff) - 127;  // floor(log2 a) for normal a
    if (e < -6) e = -6;                                        // subnormal range: step 2^-9
    const float step = __uint_as_float((uint32_t)(e - 3 + 127) << 23);
    float m = rintf(a / step) * step;                          // exact scaling, RNE
    int em = (int)((__float_as_uint(m) >> 23) & 0xff) - 127;
    uint8_t code;
    if (m == 0.0f) {
        code = 0;
    } else if (em < -6) {                                      // subnormal: mant * 2^-9
        code = (uint8_t)(m * 512.0f);
    } else {
        const uint32_t mant = (__float_as_uint(m) >> 20) & 0x7u;
        code = (uint8_t)(((em + 7) << 3) | mant);
    }
    q = (y < 0.0f) ? -m : m;
    return (uint8_t)(sg | code);
}

// Round-to-nearest-even encoding of y (|y| <= the format's largest value)
// into an OCP element format with 2 exponent bits (bias 1) and M mantissa
// bits, no infinities: e2m3 (FP6, M = 3) or e2m1 (FP4, M = 1).  Subnormals
// (exponent field 0) step by 2^-M.  q receives the encoded value.
template <int M>
__device__ __forceinline__ uint8_t to_e2m(float y, float &q) {
    const float a = fabsf(y);
    const uint8_t sg = (y < 0.0f) ? (uint8_t)(1u << (M + 2)) : 0;
    if (a == 0.0f) {
        q = 0.0f;
        return 0;
    }
    int e = (int)((__float_as_uint(a) >> 23) & 0xff) - 127;  // floor(log2 a) for normal a
    if (e < 0) e = 0;                                          // subnormal range: step 2^-M
    const float step = __uint_as_float((uint32_t)(e - M + 127) << 23);
    float m = rintf(a / step) * step;                          // exact scaling, RNE
    const float mx = (2.0f - __uint_as_float((uint32_t)(127 - M) << 23)) * 4.0f;
    if (m > mx) m = mx;
    int em = (int)((__float_as_uint(m) >> 23) & 0xff) - 127;
    uint8_t code;
    if (m == 0.0f) {
        code = 0;
    } else if (em < 0) {                                       // subnormal: mant * 2^-M
        code = (uint8_t)(m * (float)(1 << M));
    } else {
        const uint32_t mant = (__float_as_uint(m) >> (23 - M)) & ((1u << M) - 1u);
        code = (uint8_t)(((em + 1) << M) | mant);
    }
    q = (y < 0.0f) ? -m : m;
    return (uint8_t)(sg | code);
}

// Exact value of u . p: FP64 sum of the exact products of the FP32 inputs,
// taken in index order from +0.0.  fma() adds the exact product with one
// rounding, which is what a separate multiply (exact) and add would give.
// The operands are loaded a block of 16 values per row at a time, ahead of
// the dependent chain and with no branch between the loads: as 16-byte
// vectors when both rows are 16-byte aligned and d is a multiple of 4, as
// 8-byte vectors when they are 8-byte aligned and d is even, else one value
// per load.  In the last, partial block indexes past the end are clamped
// (every load stays in bounds) and their values replaced by zeros, which add
// +0 and leave the sum unchanged (the sum is never -0: it starts at +0 and
// +0 + -0 = +0).  BLK: values of each row per block (a multiple of 4).
template <int BLK = 16>
__device__ __forceinline__ double ip64(const float *__restrict__ u,
                                       const float *__restrict__ p, int d) {
    static_assert(BLK % 4 == 0, "whole 16-byte vectors per block");
    double acc = 0.0;
    const uintptr_t al = reinterpret_cast<uintptr_t>(u) | reinterpret_cast<uintptr_t>(p);
    if ((d & 3) == 0 && (al & 15) == 0) {
        constexpr int RV = BLK / 4;
        const float4 *u4 = reinterpret_cast<const float4 *>(u);
        const float4 *p4 = reinterpret_cast<const float4 *>(p);
        const int d4 = d >> 2;
        for (int i = 0; i < d4; i += RV) {
            float4 x[RV], y[RV];
#pragma unroll
            for (int j = 0; j < RV; ++j) {
                const bool ok = i + j < d4;
                const int t = ok ? i + j : d4 - 1;
                const float4 a = u4[t], b = p4[t];
                x[j] = ok ? a : make_float4(0.f, 0.f, 0.f, 0.f);
                y[j] = ok ? b : make_float4(0.f, 0.f, 0.f, 0.f);
            }
#pragma unroll
            for (int j = 0; j < RV; ++j) {
                acc = __fma_rn((double)x[j].x, (double)y[j].x, acc);
                acc = __fma_rn((double)x[j].y, (double)y[j].y, acc);
                acc = __fma_rn((double)x[j].z, (double)y[j].z, acc);
                acc = __fma_rn((double)x[j].w, (double)y[j].w, acc);
            }
        }
        return acc;
    }
    if ((d & 1) == 0 && (al & 7) == 0) {
        constexpr int RV = BLK / 2;
        const float2 *u2 = reinterpret_cast<const float2 *>(u);
        const float2 *p2 = reinterpret_cast<const float2 *>(p);
        const int d2 = d >> 1;
        for (int i = 0; i < d2; i += RV) {
            float2 x[RV], y[RV];
#pragma unroll
            for (int j = 0; j < RV; ++j) {
                const bool ok = i + j < d2;
                const int t = ok ? i + j : d2 - 1;
                const float2 a = u2[t], b = p2[t];
                x[j] = ok ? a : make_float2(0.f, 0.f);
                y[j] = ok ? b : make_float2(0.f, 0.f);
            }
#pragma unroll
            for (int j = 0; j < RV; ++j) {
                acc = __fma_rn((double)x[j].x, (double)y[j].x, acc);
                acc = __fma_rn((double)x[j].y, (double)y[j].y, acc);
            }
        }
        return acc;
    }
    for (int i = 0; i < d; i += BLK) {
        float x[BLK], y[BLK];
#pragma unroll
        for (int j = 0; j < BLK; ++j) {
            const bool ok = i + j < d;
            const int t = ok ? i + j : d - 1;
            const float a = u[t], b = p[t];
            x[j] = ok ? a : 0.0f;
            y[j] = ok ? b : 0.0f;
        }
#pragma unroll
        for (int j = 0; j < BLK; ++j) acc = __fma_rn((double)x[j], (double)y[j], acc);
    }
    return acc;
}

// Exact values of u . p0 and u . p1 (ip64's arithmetic, term by term), the
// two rows' blocks loaded together so that twice the bytes are in flight per
// lane, and the user's block once for both.
__device__ __forceinline__ void ip64x2(const float *__restrict__ u, const float *__restrict__ p0,
                                       const float *__restrict__ p1, int d, double &r0,
                                       double &r1) {
    const uintptr_t al = reinterpret_cast<uintptr_t>(u) | reinterpret_cast<uintptr_t>(p0) |
                         reinterpret_cast<uintptr_t>(p1);
    if ((d & 3) != 0 || (al & 15) != 0) {
        r0 = ip64(u, p0, d);
        r1 = ip64(u, p1, d);
        return;
    }
    constexpr int RV = 4;
    const float4 *u4 = reinterpret_cast<const float4 *>(u);
    const float4 *a4 = reinterpret_cast<const float4 *>(p0);
    const float4 *b4 = reinterpret_cast<const float4 *>(p1);
    const int d4 = d >> 2;
    double s0 = 0.0, s1 = 0.0;
    for (int i = 0; i < d4; i += RV) {
        float4 x[RV], y[RV], z[RV];
#pragma unroll
        for (int j = 0; j < RV; ++j) {
            const bool ok = i + j < d4;
            const int t = ok ? i + j : d4 - 1;
            const float4 a = u4[t], b = a4[t], c = b4[t];
            // (selects per value: a select between two vectors in memory
            // would be made through private memory)
            x[j] = make_float4(ok ? a.x : 0.f, ok ? a.y : 0.f, ok ? a.z : 0.f, ok ? a.w : 0.f);
            y[j] = make_float4(ok ? b.x : 0.f, ok ? b.y : 0.f, ok ? b.z : 0.f, ok ? b.w : 0.f);
            z[j] = make_float4(ok ? c.x : 0.f, ok ? c.y : 0.f, ok ? c.z : 0.f, ok ? c.w : 0.f);
        }
#pragma unroll
        for (int j = 0; j < RV; ++j) {
            s0 = __fma_rn((double)x[j].x, (double)y[j].x, s0);
            s1 = __fma_rn((double)x[j].x, (double)z[j].x, s1);
            s0 = __fma_rn((double)x[j].y, (double)y[j].y, s0);
            s1 = __fma_rn((double)x[j].y, (double)z[j].y, s1);
            s0 = __fma_rn((double)x[j].z, (double)y[j].z, s0);
            s1 = __fma_rn((double)x[j].z, (double)z[j].z, s1);
            s0 = __fma_rn((double)x[j].w, (double)y[j].w, s0);
            s1 = __fma_rn((double)x[j].w, (double)z[j].w, s1);
        }
    }
    r0 = s0;
    r1 = s1;
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
