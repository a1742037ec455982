// Relaxed, differentiable score for query item vectors q (not in the paper;
// a smooth stand-in for |T_k(q)| used to design new items):
//   S(q)  = sum_u sigmoid(z_u),          z_u = (u . q - tau_u) / T
//   dS/dq = sum_u sigmoid'(z_u) / T * u
//
// One workgroup takes 64 QB queries (16 QB per wave, QB = 2 up to d = 128)
// and a slice of the users, streamed 64 at a time through LDS.  For each
// block of 16 users a wave forms Z^T = U Q^T for each of its query blocks on
// the FP32 matrix cores (v_mfma_f32_16x16x4f32; K-slot
// k of step s takes dim 4 s + k; the users' rows from LDS, the wave's query
// rows in registers).  The product leaves users 4 (l / 16) + i of register i
// in lane l beside query l % 16, which is the A-operand layout of K-step i
// of the gradient product G = W^T U (W = sigmoid'(z) / T, K-slot k = users
// 4 k + i): the weights feed that product straight from registers, with the
// same users' rows from LDS as its B operand.  S and G come from one pass
// (Z once).  Per-slice partial sums are added in FP64 in a fixed order by a
// second kernel, so results do not depend on scheduling.
#include <mutex>

#include "common.h"
#include "kernels.h"

namespace rmips {

constexpr int SUC = 64;         // users per chunk (four blocks of 16)
constexpr int S_SPLITS = 384;   // user slices at most (workspace); launches aim at
                                // three workgroups per CU (d <= 128)

struct SoftDims {
    int d, kq, Dg, ld;  // dims, steps of the Z product (ceil(d / 4)), d rounded up to
                        // 16 (the gradient's dim blocks), LDS row stride
};

// Row stride: 4 kq or 4 kq + 4 floats, whichever is an odd number of
// 16-byte vectors, so that the 16 rows x 4 consecutive floats that a Z step
// reads, and the 4 rows x 16 floats of a gradient step, fall on 64 distinct
// banks.  The gradient's last dim block reads up to Dg - 1 - ... past a row
// end (into the next row, the next buffer or the zero guard): finite values
// that reach only dims >= d, which are dropped.
__host__ __device__ inline SoftDims soft_dims(int d) {
    SoftDims s;
    s.d = d;
    s.kq = (d + 3) / 4;
    s.Dg = (d + 15) & ~15;
    s.ld = (s.kq & 1) ? 4 * s.kq : 4 * s.kq + 4;
    return s;
}
constexpr int SOFT_GUARD = 64;  // floats of zeros after the buffers (>= Dg - ld)

size_t soft_lds(int d) {
    SoftDims s = soft_dims(d);
    // two user chunks, the zero guard, the chunks' thresholds (two)
    return (size_t)(2 * SUC * s.ld + SOFT_GUARD + 2 * SUC) * sizeof(float);
}

// sigmoid and its derivative from t = exp(-|z|), which never overflows
__device__ __forceinline__ void sig(float z, float &s, float &ds) {
    const float t = __expf(-fabsf(z));
    const float r = __builtin_amdgcn_rcpf(1.0f + t);
    s = (z >= 0.0f) ? r : t * r;
    ds = t * r * r;
}

// Waves per SIMD: three where the registers allow it (the LDS holds three
// workgroups up to d = 128), else two.
__host__ __device__ constexpr int soft_wpe(int qn, int qb) { return qn * qb <= 48 ? 3 : 2; }

// QN: registers of the query operand (kq rounded up to 8); NCB: 16-wide dim
// blocks of G (at most; Dg / 16 at run time); QB: query blocks of 16 per
// wave (each user-row read from LDS feeds QB products); WS / WG: form S / G.
template <int QN, int NCB, int QB, bool WS, bool WG>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(soft_wpe(QN, QB))))
void k_soft(const float *__restrict__ U, int64_t n, const float *__restrict__ tau,
            const float *__restrict__ Q, int64_t nq, int d, float invT,
            float *__restrict__ Sp, float *__restrict__ Gp) {
    extern __shared__ float smem[];
    const SoftDims sd = soft_dims(d);
    const int ld = sd.ld, kq = sd.kq, Dg = sd.Dg, ncb = Dg / 16;
    float *Ubuf = smem;                     // 2 x SUC x ld
    float *guard = Ubuf + 2 * SUC * ld;     // zeros
    float *tsh = guard + SOFT_GUARD;        // 2 x SUC

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int r16 = lane & 15, k4 = lane >> 4;
    const int64_t q0 = (int64_t)blockIdx.x * (64 * QB) + w * (16 * QB);  // the wave's queries
    const int split = blockIdx.y, nsplit = gridDim.y;
    const int64_t per = (n + nsplit - 1) / nsplit;
    const int64_t ubeg = (int64_t)split * per;
    const int64_t uend = (ubeg + per < n) ? ubeg + per : n;

    for (int e = tid; e < SOFT_GUARD; e += 256) guard[e] = 0.0f;
    // this lane's query of block b (q0 + 16 b + r16): dims 4 s + k4
    float qa[QB][QN];
#pragma unroll
    for (int b = 0; b < QB; ++b) {
        const int64_t qrow = q0 + 16 * b + r16;
        const float *qp = Q + (qrow < nq ? qrow : 0) * d;
#pragma unroll
        for (int j = 0; j < QN; ++j) {
            const int c = 4 * j + k4;
            qa[b][j] = (qrow < nq && j < kq && c < d) ? qp[c] : 0.0f;
        }
    }
    float ssum[QB];  // S of this lane's queries over its users
    f32x4 g[QB][WG ? NCB : 1];
#pragma unroll
    for (int b = 0; b < QB; ++b) {
        ssum[b] = 0.0f;
#pragma unroll
        for (int j = 0; j < (WG ? NCB : 1); ++j) g[b][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    }

    // user chunks are copied straight from global memory into LDS (no
    // registers), the next chunk while the current one is multiplied: rows
    // of whole 16-byte vectors 16 bytes per lane (vector slots), others 4
    // bytes per lane (float slots).  Slot s of a chunk is row s / spr,
    // position s % spr (spr slots per LDS row); positions past the row and
    // rows past the slice hold a finite copy of an element inside it (the
    // padding columns meet zero query entries, rows past the slice are
    // dropped by their validity).
    const bool v16 = (d % 4) == 0 && (reinterpret_cast<uintptr_t>(U) & 15) == 0;
    const int spr = v16 ? ld / 4 : ld;            // slots per LDS row
    const int rlen = v16 ? d / 4 : d;             // valid slots per row
    const uint32_t magic = 0xffffffffu / (uint32_t)spr + 1u;  // s / spr = umulhi(s, magic)
    auto issue = [&](int64_t u0, int b) {
        float *dst = Ubuf + b * SUC * ld;
        const int64_t left = uend - u0;
        for (int j = w; j < spr; j += 4) {  // SUC * spr slots, 64 per instruction
            const uint32_t sl = 64u * (uint32_t)j + (uint32_t)lane;
            const uint32_t r = __umulhi(sl, magic);
            const uint32_t c = sl - r * (uint32_t)spr;
            const int64_t ur = u0 + ((int64_t)r < left ? (int64_t)r : left - 1);
            const int cc = (int)c < rlen ? (int)c : rlen - 1;
            if (v16) dma16(U + ur * d + 4 * cc, dst + 256 * j);
            else dma4(U + ur * d + cc, dst + 64 * j);
        }
        if (w == 3) dma4(tau + u0 + (lane < left ? lane : left - 1), tsh + b * SUC);
    };

    int buf = 0;
    if (ubeg < uend) issue(ubeg, 0);
    for (int64_t u0 = ubeg; u0 < uend; u0 += SUC) {
        dma_wait();
        __syncthreads();  // chunk u0 is in buffer buf; the other buffer is free
        if (u0 + SUC < uend) issue(u0 + SUC, buf ^ 1);
        const float *Uc = Ubuf + buf * SUC * ld;
        const float *tc = tsh + buf * SUC;
        const int64_t left = uend - u0;
        // one user block at a time (unrolling the blocks makes the compiler
        // hold every block's operands at once and spill)
#pragma unroll 1
        for (int ub = 0; ub < SUC / 16; ++ub) {
            // Z^T blocks: users ub * 16 + (0..15), the wave's query blocks
            f32x4 z[QB];
#pragma unroll
            for (int b = 0; b < QB; ++b) z[b] = f32x4{0.f, 0.f, 0.f, 0.f};
            const float *a = Uc + (ub * 16 + r16) * ld + k4;
            // the reads of the next 8 steps issued before this group's
            // products, none behind a branch: reads for steps past kq land at
            // most 4 QN - 4 kq + 27 < 32 floats past a row end (the next row,
            // the other buffer or the zero guard, all inside the LDS block)
            // and are not multiplied
            float av[2][8];
#pragma unroll
            for (int j = 0; j < 8; ++j) av[0][j] = a[4 * j];
#pragma unroll
            for (int j0 = 0; j0 < QN; j0 += 8) {
                const int cg = (j0 / 8) & 1;
                if (j0 + 8 < QN) {
#pragma unroll
                    for (int j = 0; j < 8; ++j) av[cg ^ 1][j] = a[4 * (j0 + 8 + j)];
                }
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    if (j0 + j < kq) {
#pragma unroll
                        for (int b = 0; b < QB; ++b)
                            z[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[cg][j], qa[b][j0 + j],
                                                                       z[b], 0, 0, 0);
                    }
                }
                // (no read of a later group moves above this group)
                __builtin_amdgcn_sched_barrier(0);
            }
            // register i: user ub * 16 + 4 k4 + i; a user past the slice
            // contributes nothing (explicit validity)
            float wv[QB][4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int ur = ub * 16 + 4 * k4 + i;
                const bool ok = ur < left;
                const float tu = tc[ur];
#pragma unroll
                for (int b = 0; b < QB; ++b) {
                    float sv, dv;
                    sig((z[b][i] - tu) * invT, sv, dv);
                    if (WS) ssum[b] += ok ? sv : 0.0f;
                    wv[b][i] = ok ? dv * invT : 0.0f;
                }
            }
            if constexpr (WG) {
                // (the next dim block's reads before this block's products, as
                // above; blocks from ncb on read at most 16 NCB - ld < 32
                // floats past a row end and are not multiplied)
                const float *ur = Uc + (ub * 16 + 4 * k4) * ld + r16;
                float uv[2][4];
#pragma unroll
                for (int i = 0; i < 4; ++i) uv[0][i] = ur[i * ld];
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) {
                    if (cb + 1 < NCB) {
#pragma unroll
                        for (int i = 0; i < 4; ++i) uv[(cb + 1) & 1][i] = ur[i * ld + (cb + 1) * 16];
                    }
                    if (cb < ncb) {
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
#pragma unroll
                            for (int b = 0; b < QB; ++b)
                                g[b][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                                    wv[b][i], uv[cb & 1][i], g[b][cb], 0, 0, 0);
                        }
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        }
        buf ^= 1;
    }
    if constexpr (WS) {
        // the four lanes of a query (k4 = 0..3), in a fixed order
#pragma unroll
        for (int b = 0; b < QB; ++b) {
            float x = ssum[b] + __shfl_xor(ssum[b], 16);
            x += __shfl_xor(x, 32);
            const int64_t qrow = q0 + 16 * b + r16;
            if (k4 == 0 && qrow < nq) Sp[(int64_t)split * nq + qrow] = x;
        }
    }
    if constexpr (WG) {
        // g[b][cb][i]: query q0 + 16 b + 4 k4 + i, dim cb * 16 + r16
#pragma unroll
        for (int b = 0; b < QB; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t q = q0 + 16 * b + 4 * k4 + i;
                if (q >= nq) continue;
                float *dst = Gp + ((int64_t)split * nq + q) * Dg;
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb)
                    if (cb < ncb) dst[cb * 16 + r16] = g[b][cb][i];
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
// SOFT_NOALLOC_COLS (Dg = d rounded up to 16).  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in): it passes
// the device address that hipGetSymbolAddress returns for the device, taken
// once per device with that device current.
constexpr int64_t SOFT_NOALLOC_COLS = 65536;
constexpr int SOFT_NOALLOC_SPLITS = 192;  // user slices of that entry point at most
constexpr size_t SOFT_SCRATCH_BYTES =
    (size_t)SOFT_NOALLOC_SPLITS * SOFT_NOALLOC_COLS * sizeof(float);
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

// (the gradient alone uses the G partial sums at the start of the scratch)
bool soft_noalloc_fits(int64_t nq, int d) {
    return nq * (int64_t)soft_dims(d).Dg <= SOFT_NOALLOC_COLS;
}
int soft_noalloc_splits() { return SOFT_NOALLOC_SPLITS; }
int soft_max_splits() { return S_SPLITS; }

size_t soft_ws_bytes(int64_t n, int64_t nq, int d) {
    (void)n;
    SoftDims s = soft_dims(d);
    // per-slice partial sums of G, then of S
    return (size_t)S_SPLITS * nq * (s.Dg + 1) * sizeof(float) + 512;
}

// Per-slice partial sums (G then S) in ws; S, G (unscaled) and dQ (G scaled
// by dS) are written where not NULL.
void launch_soft(const float *U, int64_t n, const float *tau, const float *Q, int64_t nq,
                 int d, float T, const float *dS, float *S, float *G, float *dQ, void *ws,
                 hipStream_t st, int max_splits) {
    const SoftDims sd = soft_dims(d);
    const float invT = 1.0f / T;
    const bool ws_ = S != nullptr, wg = G != nullptr || dQ != nullptr;
    // two query blocks per wave up to d = 128, one above (registers)
    const int qb = sd.kq <= 32 ? 2 : 1;
    const int64_t tiles = (nq + 64 * qb - 1) / (64 * qb);
    // slices: one resident round of workgroups (each has one wave per SIMD,
    // so as many per compute unit as the registers give waves per SIMD, at
    // most as many as the LDS holds), at least one chunk of users each; a
    // partial second round would leave compute units idle at the end
    const int qn = 8 * ((sd.kq + 7) / 8);
    const int resident =
        std::max(1, std::min(soft_wpe(qn, qb), (int)((size_t)(160 * 1024) / soft_lds(d))));
    int64_t ns = (256 * (int64_t)resident + tiles - 1) / tiles;
    ns = std::min<int64_t>(ns, std::min<int64_t>(max_splits, (n + SUC - 1) / SUC));
    const int nsplit = (int)std::max<int64_t>(1, ns);
    dim3 g((unsigned)tiles, (unsigned)nsplit);
    float *gpart = reinterpret_cast<float *>(ws);
    float *spart = gpart + (size_t)max_splits * nq * sd.Dg;
    const size_t lds = soft_lds(d);
    {
        RMIPS_PROF(st, ws_ && wg ? "k_soft/fwd+grad" : (wg ? "k_soft/grad" : "k_soft/fwd"));
        // QN = kq rounded up to 8 registers of the query operand, NCB = QN / 4
        // dim blocks (>= Dg / 16)
        with_exact<1, 8>((sd.kq + 7) / 8, [&](auto q8) {
            constexpr int QN = 8 * decltype(q8)::value, NCB = QN / 4, QB = QN <= 32 ? 2 : 1;
            if (ws_ && wg)
                k_soft<QN, NCB, QB, true, true><<<g, 256, lds, st>>>(U, n, tau, Q, nq, d, invT,
                                                                     spart, gpart);
            else if (wg)
                k_soft<QN, NCB, QB, false, true><<<g, 256, lds, st>>>(U, n, tau, Q, nq, d, invT,
                                                                      nullptr, gpart);
            else
                k_soft<QN, NCB, QB, true, false><<<g, 256, lds, st>>>(U, n, tau, Q, nq, d, invT,
                                                                      spart, nullptr);
        });
    }
    RMIPS_PROF(st, "k_soft_reduce");
    if (G)
        k_soft_reduce<<<dim3((unsigned)nq, (unsigned)((d + 63) / 64)), 256, 0, st>>>(
            gpart, nsplit, nq, sd.Dg, d, nullptr, G, d);
    if (dQ)
        k_soft_reduce<<<dim3((unsigned)nq, (unsigned)((d + 63) / 64)), 256, 0, st>>>(
            gpart, nsplit, nq, sd.Dg, d, dS, dQ, d);
    if (S)
        k_soft_reduce<<<dim3((unsigned)nq, 1u), 256, 0, st>>>(spart, nsplit, nq, 1, 1, nullptr,
                                                              S, 1);
}

// dQ[i][:] = dS[i] * G[i][:]
__global__ void k_soft_scale(const float *__restrict__ G, int64_t nq, int d,
                             const float *__restrict__ dS, float *__restrict__ dQ) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nq * d) return;
    dQ[e] = dS[e / d] * G[e];
}

void launch_soft_scale(const float *G, int64_t nq, int d, const float *dS, float *dQ,
                       hipStream_t st) {
    RMIPS_PROF(st, "k_soft_scale");
    k_soft_scale<<<(unsigned)((nq * d + 255) / 256), 256, 0, st>>>(G, nq, d, dS, dQ);
}

}  // namespace rmips
