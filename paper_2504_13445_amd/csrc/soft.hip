// Relaxed, differentiable score for query item vectors q (not in the paper;
// a smooth stand-in for |T_k(q)| used to design new items):
//   S(q)  = sum_u sigmoid(z_u),          z_u = (u . q - tau_u) / T
//   dS/dq = sum_u sigmoid'(z_u) / T * u
//
// One workgroup takes 64 queries and a slice of the users, streamed 64 at a
// time through LDS.  Z = Q U^T comes from the FP32 matrix cores (each wave
// one 32x32 block); sigmoid or sigmoid' is applied in registers.  For the
// gradient the weights W = sigmoid'(z) / T go through LDS (the product's
// output layout is not its input layout) and a second product accumulates
// G += W U over the chunk.  Per-slice partial sums are added in FP64 in a
// fixed order by a second kernel, so results do not depend on scheduling.
#include <mutex>

#include "common.h"
#include "kernels.h"

namespace rmips {

constexpr int SQ = 64;          // queries per workgroup
constexpr int SUC = 64;         // users per chunk
constexpr int S_SPLITS = 128;   // user slices (workgroups per query tile)

struct SoftDims {
    int d, D, Dg, ld, ldw;  // dims, padded for Z (x8), padded for G (x32), LDS strides
};

// LDS row stride ld = D + LDS_PAD (not Dg): the gradient's last 32-wide dim
// block then reads past a user row's end, into the next row or, from the
// last row, into the weights that follow; those values are finite and only
// reach dims >= d, which are dropped.  The smaller stride lets two
// workgroups share a compute unit for d <= 104.
__host__ __device__ inline SoftDims soft_dims(int d) {
    SoftDims s;
    s.d = d;
    s.D = (d + 7) & ~7;
    s.Dg = (d + 31) & ~31;
    s.ld = s.D + LDS_PAD;
    s.ldw = SUC + LDS_PAD;
    return s;
}

size_t soft_lds(int d) {
    SoftDims s = soft_dims(d);
    // Q and U rows, the weights, and the reads of the last dim block past U
    // (which land in the weights: Dg - ld <= SQ * ldw floats)
    return (size_t)(2 * SQ * s.ld + SQ * s.ldw) * sizeof(float) + 4 * SQ * sizeof(float);
}

// sigmoid and its derivative from t = exp(-|z|), which never overflows
__device__ __forceinline__ void sig(float z, float &s, float &ds) {
    const float t = __expf(-fabsf(z));
    const float r = __builtin_amdgcn_rcpf(1.0f + t);
    s = (z >= 0.0f) ? r : t * r;
    ds = t * r * r;
}

// CPL: 64-wide column groups per user row (ceil(d / 64)).
template <bool BWD, int CPL>
__global__ __launch_bounds__(256) void k_soft(const float *__restrict__ U, int64_t n,
                                              const float *__restrict__ tau,
                                              const float *__restrict__ Q, int64_t nq, int d,
                                              float invT, float *__restrict__ Sp,
                                              float *__restrict__ Gp) {
    extern __shared__ float smem[];
    __shared__ float tsh[SUC];
    const SoftDims sd = soft_dims(d);
    const int ld = sd.ld, ldw = sd.ldw, ks = sd.D / 2;
    float *Qsh = smem;
    float *Ush = Qsh + SQ * ld;
    float *Wsh = Ush + SUC * ld;
    float *Ssh = Wsh + SQ * ldw;  // [4 waves][SQ]

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t q0 = (int64_t)blockIdx.x * SQ;
    const int split = blockIdx.y, nsplit = gridDim.y;
    const int64_t per = (n + nsplit - 1) / nsplit;
    const int64_t ub = (int64_t)split * per;
    const int64_t ue = (ub + per < n) ? ub + per : n;

    for (int e = tid; e < SQ * ld; e += 256) {
        const int r = e / ld, c = e - r * ld;
        float v = 0.0f;
        if (q0 + r < nq && c < d) v = Q[(q0 + r) * d + c];
        Qsh[r * ld + c] = v;
    }
    for (int e = tid; e < SQ * 4; e += 256) Ssh[e] = 0.0f;

    // Z block of this wave: query rows rbq*32.., user columns cbu*32..
    const int rbq = w >> 1, cbu = w & 1;
    // forward, up to 64 dims per half row (d <= 128): the wave's query
    // operand stays in registers for the whole kernel (the same products, in
    // the same order, as from LDS; the backward kernel keeps its registers
    // for the gradient blocks)
    constexpr bool QREG = !BWD && CPL <= 2;
    float qa[QREG ? 32 * CPL : 1];
    if constexpr (QREG) {
        __syncthreads();  // the query tile is in LDS
        const float *a = Qsh + (rbq * 32 + (lane & 31)) * ld + (lane >> 5) * ks;
#pragma unroll
        for (int q = 0; q < 32 * CPL; ++q) qa[q] = (q < ks) ? a[q] : 0.0f;
    }
    float ssum[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) ssum[i] = 0.0f;
    // G blocks of this wave: query rows rbq*32.., dim columns (cbu + 2j)*32
    f32x16 g[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) g[j] = f32x16{0};
    const int ncb = sd.Dg / 32;  // 32-wide dim blocks (<= 8)

    // users are staged through registers (wave w takes rows w, w+4, ...,
    // lanes take columns), so the next chunk loads during compute
    constexpr int RPW = SUC / 4;  // rows per wave
    float pf[RPW][CPL];
    float ptau = 0.0f;
    auto fetch = [&](int64_t u0) {
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
            const int64_t u = u0 + w + 4 * i;
#pragma unroll
            for (int j = 0; j < CPL; ++j) {
                const int c = lane + 64 * j;
                pf[i][j] = (u < ue && c < d) ? U[u * d + c] : 0.0f;
            }
        }
        ptau = (tid < SUC && u0 + tid < ue) ? tau[u0 + tid] : INFINITY;
    };
    auto stash = [&]() {
#pragma unroll
        for (int i = 0; i < RPW; ++i)
#pragma unroll
            for (int j = 0; j < CPL; ++j) {
                const int c = lane + 64 * j;
                if (c < ld) Ush[(w + 4 * i) * ld + c] = pf[i][j];
            }
    };

    if (ub < ue) fetch(ub);
    for (int64_t u0 = ub; u0 < ue; u0 += SUC) {
        __syncthreads();  // previous chunk fully consumed
        stash();
        if (tid < SUC) tsh[tid] = ptau;
        __syncthreads();
        if (u0 + SUC < ue) fetch(u0 + SUC);
        f32x16 z = {0};
        if constexpr (QREG) {
            const float *b = Ush + (cbu * 32 + (lane & 31)) * ld + (lane >> 5) * ks;
#pragma unroll
            for (int q = 0; q < 32 * CPL; q += 4) {
                if (q < ks) {  // (uniform; ks is a multiple of 4)
                    const f32x4 bv = *reinterpret_cast<const f32x4 *>(b + q);
                    z = __builtin_amdgcn_mfma_f32_32x32x2f32(qa[q], bv[0], z, 0, 0, 0);
                    z = __builtin_amdgcn_mfma_f32_32x32x2f32(qa[q + 1], bv[1], z, 0, 0, 0);
                    z = __builtin_amdgcn_mfma_f32_32x32x2f32(qa[q + 2], bv[2], z, 0, 0, 0);
                    z = __builtin_amdgcn_mfma_f32_32x32x2f32(qa[q + 3], bv[3], z, 0, 0, 0);
                }
            }
        } else {
            mfma32_f32(z, Qsh + rbq * 32 * ld, Ush + cbu * 32 * ld, ld, ks, lane);
        }
        const float tu = tsh[cbu * 32 + (lane & 31)];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            float s, ds;
            sig((z[i] - tu) * invT, s, ds);
            if (BWD) {
                Wsh[(rbq * 32 + mfma32_row(i, lane)) * ldw + cbu * 32 + (lane & 31)] = ds * invT;
            } else {
                ssum[i] += s;
            }
        }
        if (BWD) {
            __syncthreads();
            // G[q][dim] += sum_u W[q][u] U[u][dim]; k = users in steps of 2
            const int r = lane & 31, h = lane >> 5;
            const float *wa = Wsh + (rbq * 32 + r) * ldw;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int cb = cbu + 2 * j;
                if (cb < ncb) {
#pragma unroll 8
                    for (int s2 = 0; s2 < SUC; s2 += 2)
                        g[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(
                            wa[s2 + h], Ush[(s2 + h) * ld + cb * 32 + r], g[j], 0, 0, 0);
                }
            }
        }
    }
    if (!BWD) {
        // per-query sums: over the 32 lanes of a half, then over the 2 waves
        // sharing the query rows
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            float x = ssum[i];
#pragma unroll
            for (int o = 16; o > 0; o >>= 1) x += __shfl_xor(x, o);
            if ((lane & 31) == 0) Ssh[w * SQ + rbq * 32 + mfma32_row(i, lane)] = x;
        }
        __syncthreads();
        if (tid < SQ && q0 + tid < nq) {
            const int rb = tid >> 5;
            const float x = Ssh[(2 * rb) * SQ + tid] + Ssh[(2 * rb + 1) * SQ + tid];
            Sp[(int64_t)split * nq + q0 + tid] = x;
        }
    } else {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int64_t q = q0 + rbq * 32 + mfma32_row(i, lane);
            if (q >= nq) continue;
            float *dst = Gp + ((int64_t)split * nq + q) * sd.Dg;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int cb = cbu + 2 * j;
                if (cb < ncb) dst[cb * 32 + (lane & 31)] = g[j][i];
            }
        }
    }
}

// out[q][c] = scale_q * (sum over slices k of P[k][q][c]) in FP64, for
// c < width.  One workgroup per query and 64 columns: each of its four waves
// adds a quarter of the slices in slice order (loads in batches of 8), then
// the four partial sums are added in wave order, a fixed order in every call.
__global__ __launch_bounds__(256) void k_soft_reduce(const float *__restrict__ P, int nsplit,
                                                     int64_t cols, int64_t ld_in, int64_t width,
                                                     const float *__restrict__ dS,
                                                     float *__restrict__ out, int64_t ld_out) {
    __shared__ double part[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t q = blockIdx.x;
    const int64_t c = (int64_t)blockIdx.y * 64 + lane;
    const bool ok = c < width;
    const int per = (nsplit + 3) / 4, k0 = w * per, k1 = min(nsplit, k0 + per);
    double s = 0.0;
    if (ok) {
        const float *p = P + q * ld_in + c;
        const int64_t step = cols * ld_in;
        int k = k0;
        for (; k + 8 <= k1; k += 8) {
            float v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = p[(int64_t)(k + j) * step];
#pragma unroll
            for (int j = 0; j < 8; ++j) s += (double)v[j];
        }
        for (; k < k1; ++k) s += (double)p[(int64_t)k * step];
    }
    part[w][lane] = s;
    __syncthreads();
    if (w == 0 && ok) {
        double t = part[0][lane] + part[1][lane];
        t += part[2][lane];
        t += part[3][lane];
        if (dS) t *= (double)dS[q];
        out[q * ld_out + c] = (float)t;
    }
}

// Scratch of the entry point that allocates nothing (rmips_soft_bwd_noalloc):
// the gradient's per-slice partial sums live in this file-scope array, one
// copy per device, held until the process ends.  It takes nq * Dg <=
// SOFT_NOALLOC_COLS (Dg = d rounded up to 32).  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in): it passes
// the device address that hipGetSymbolAddress returns for the device, taken
// once per device with that device current.
constexpr int64_t SOFT_NOALLOC_COLS = 65536;
constexpr size_t SOFT_SCRATCH_BYTES = (size_t)S_SPLITS * SOFT_NOALLOC_COLS * sizeof(float) + 256;
static __device__ __align__(256) uint8_t scratch[SOFT_SCRATCH_BYTES];

namespace {
constexpr int SCRATCH_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[SCRATCH_DEVICES] = {};
}  // namespace

hipError_t soft_scratch_init(int device, void **out) {
    *out = nullptr;
    if (device < 0 || device >= SCRATCH_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device] == nullptr) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;  // the caller makes it current
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

bool soft_noalloc_fits(int64_t nq, int d) {
    return nq * (int64_t)soft_dims(d).Dg <= SOFT_NOALLOC_COLS &&
           soft_ws_bytes(0, nq, d) <= SOFT_SCRATCH_BYTES;
}

size_t soft_ws_bytes(int64_t n, int64_t nq, int d) {
    (void)n;
    SoftDims s = soft_dims(d);
    return (size_t)S_SPLITS * nq * s.Dg * sizeof(float) + 256;
}

void launch_soft(const float *U, int64_t n, const float *tau, const float *Q, int64_t nq,
                 int d, float T, const float *dS, float *S, float *dQ, void *ws,
                 hipStream_t st) {
    const SoftDims sd = soft_dims(d);
    int nsplit = S_SPLITS;
    if ((int64_t)nsplit * SUC > n) nsplit = (int)((n + SUC - 1) / SUC);
    dim3 g((unsigned)((nq + SQ - 1) / SQ), (unsigned)nsplit);
    float *part = reinterpret_cast<float *>(ws);
    const size_t lds = soft_lds(d);
    const int cpl = (sd.Dg + 63) / 64;
    const float invT = 1.0f / T;
#define RMIPS_SOFT(B, C)                                                               \
    k_soft<B, C><<<g, 256, lds, st>>>(U, n, tau, Q, nq, d, invT, B ? nullptr : part,   \
                                      B ? part : nullptr)
    if (dQ) {
        {
            RMIPS_PROF(st, "k_soft/bwd");
            if (cpl == 1) RMIPS_SOFT(true, 1);
            else if (cpl == 2) RMIPS_SOFT(true, 2);
            else if (cpl == 3) RMIPS_SOFT(true, 3);
            else RMIPS_SOFT(true, 4);
        }
        RMIPS_PROF(st, "k_soft_reduce");
        k_soft_reduce<<<dim3((unsigned)nq, (unsigned)((d + 63) / 64)), 256, 0, st>>>(
            part, nsplit, nq, sd.Dg, d, dS, dQ, d);
    } else {
        {
            RMIPS_PROF(st, "k_soft/fwd");
            if (cpl == 1) RMIPS_SOFT(false, 1);
            else if (cpl == 2) RMIPS_SOFT(false, 2);
            else if (cpl == 3) RMIPS_SOFT(false, 3);
            else RMIPS_SOFT(false, 4);
        }
        RMIPS_PROF(st, "k_soft_reduce");
        k_soft_reduce<<<dim3((unsigned)nq, 1u), 256, 0, st>>>(part, nsplit, nq, 1, 1, nullptr, S,
                                                              1);
    }
#undef RMIPS_SOFT
}

}  // namespace rmips
