// Stage (b): exact scores |T_k(p)| (Def. 2, Eq. 1) of a set of items, and
// stage (c): the Eq. (3)/(6) upper-bound counts uscore(p) and the running
// top-N of the bound-ordered visit (Alg. 2).
//
// Both counting kernels keep a tile of 64 items in LDS and stream users
// through LDS 128 at a time; the matrix cores give an FP32 value per
// (item, user) pair, each lane owns one user column and 16 item rows of a
// 32x32 block, and counts accumulate per lane and item row, so no global
// atomics are needed: each workgroup writes one partial count per item,
// and a second pass sums the partials in a fixed order.
#include "common.h"
#include "kernels.h"

namespace rmips {

constexpr int CI = 64;    // items per counting workgroup
constexpr int CU = 128;   // users per streamed chunk of the bound kernel

// The counting kernel streams 32 users per wave; NW = 4 waves, or 2 when
// long rows would not fit four waves' users in LDS.
size_t count_lds_nw(int D, int nw) {
    const int ld = D + LDS_PAD;
    return (size_t)(CI + 32 * nw) * ld * sizeof(float) + nw * CI * sizeof(int);
}

int count_waves(int D) { return count_lds_nw(D, 4) <= 96 * 1024 ? 4 : 2; }

size_t count_lds(int D) { return count_lds_nw(D, count_waves(D)); }

// Sum of a per-slot count over the 32 lanes of each half-wave; afterwards
// lanes 0 and 32 hold the totals of their rows.
__device__ __forceinline__ int half_sum(int x) {
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

// Exact count.  For a pair with screened value vh and bound E:
//   vh - E > tau_hi  =>  v > tau_u           (in S_k(u))
//   vh + E < tau_lo  =>  v < tau_u           (not in S_k(u))
// and otherwise the pair is recomputed in FP64 and decided by the tie rule.
template <int NW>
__global__ __launch_bounds__(64 * NW) void k_count(CountArgs a) {
    constexpr int CUW = 32 * NW, NT = 64 * NW;
    extern __shared__ float smem[];
    const int D = a.D, ld = D + LDS_PAD, ks = D / 2, D4 = D / 4;
    float *Psh = smem;
    float *Ush = Psh + CI * ld;
    int *wsum = reinterpret_cast<int *>(Ush + CUW * ld);  // [NW][CI]

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t ib = (int64_t)blockIdx.x * CI;
    const int split = blockIdx.y;

    for (int e = tid; e < CI * D4; e += NT) {
        int r = e / D4, c = e - r * D4;
        int64_t it = ib + r;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (it < a.nb) {
            int64_t row = a.rows ? a.rows[it] : it;
            v = reinterpret_cast<const float4 *>(a.Pk)[row * D4 + c];
        }
        *reinterpret_cast<float4 *>(Psh + r * ld + 4 * c) = v;
    }
    // this lane's 32 item rows: norm (0 for rows past the batch)
    float np[32];
    bool rvalid[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) {
        const int r = mfma32_row(i & 15, lane) + ((i < 16) ? 0 : 32);
        const int64_t it = ib + r;
        rvalid[i] = it < a.nb;
        np[i] = 0.0f;
        if (rvalid[i]) np[i] = a.Np[a.rows ? a.rows[it] : it];
    }
    int cnt[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) cnt[i] = 0;
    int64_t nrecheck = 0;

    const int64_t nchunks = (a.ulen + CUW - 1) / CUW;
    for (int64_t ch = split; ch < nchunks; ch += a.nsplit) {
        const int64_t u0 = ch * CUW;
        __syncthreads();
        for (int e = tid; e < CUW * D4; e += NT) {
            int r = e / D4, c = e - r * D4;
            int64_t us = u0 + r;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (us < a.ulen) v = reinterpret_cast<const float4 *>(a.Us)[us * D4 + c];
            *reinterpret_cast<float4 *>(Ush + r * ld + 4 * c) = v;
        }
        __syncthreads();
        const int64_t us = u0 + w * 32 + (lane & 31);
        const bool cvalid = us < a.ulen;
        const float ua = cvalid ? a.us.a[us] : 0.0f;
        const float thi = cvalid ? a.us.tau_hi[us] : INFINITY;
        const float tlo = cvalid ? a.us.tau_lo[us] : INFINITY;
        f32x16 acc0 = {0}, acc1 = {0};
        mfma32x2_f32(acc0, acc1, Psh, Psh + 32 * ld, Ush + w * 32 * ld, ld, ks, lane);
        bool amb_any = false;
        uint32_t ambm = 0;
#pragma unroll
        for (int i = 0; i < 32; ++i) {
            const float v = (i < 16) ? acc0[i] : acc1[i - 16];
            const float e = fmaf(ua, np[i], E_ABS);
            const bool in = (v - e) > thi;
            const bool out = (v + e) < tlo;
            cnt[i] += in ? 1 : 0;
            const bool amb = !(in || out) && cvalid && rvalid[i];
            ambm |= amb ? (1u << i) : 0u;
            amb_any |= amb;
        }
        if (__ballot(amb_any) != 0ull) {
            const int64_t uid = cvalid ? a.us.uid[us] : 0;
            const double tau = cvalid ? a.us.tau[us] : 0.0;
            const int tid_k = cvalid ? a.us.tau_id[us] : 0;
            const float *urow = a.Uorig + uid * a.d;
#pragma unroll
            for (int i = 0; i < 32; ++i) {
                const bool amb = (ambm >> i) & 1u;
                if (__ballot(amb) != 0ull && amb) {
                    const int r = mfma32_row(i & 15, lane) + ((i < 16) ? 0 : 32);
                    const int64_t it = ib + r;
                    const int64_t row = a.rows ? a.rows[it] : it;
                    const int64_t orow = a.item_orig ? a.item_orig[row] : row;
                    const int tie = a.item_tie ? a.item_tie[row] : 0x7fffffff;
                    const double v = ip64(urow, a.Porig + orow * a.d, a.d);
                    cnt[i] += in_topk(v, tie < 0 ? 0x7fffffff : tie, tau, tid_k) ? 1 : 0;
                    ++nrecheck;
                }
            }
        }
    }
    // reduce: rows of half 0 live in lanes 0..31, of half 1 in 32..63
#pragma unroll
    for (int i = 0; i < 32; ++i) {
        const int s = half_sum(cnt[i]);
        const int r = mfma32_row(i & 15, lane) + ((i < 16) ? 0 : 32);
        if ((lane & 31) == 0) wsum[w * CI + r] = s;
    }
    __syncthreads();
    if (tid < CI) {
        const int64_t it = ib + tid;
        int s = 0;
#pragma unroll
        for (int q = 0; q < NW; ++q) s += wsum[q * CI + tid];
        if (it < a.nb) a.partial[(int64_t)split * a.nb + it] = s;
    }
    if (a.rechecks) {
        int64_t tot = nrecheck;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o);
        if (lane == 0 && tot) atomicAdd(reinterpret_cast<unsigned long long *>(a.rechecks),
                                        (unsigned long long)tot);
    }
}

void launch_count(const CountArgs &a, hipStream_t st) {
    if (a.nb <= 0) return;
    dim3 g((unsigned)((a.nb + CI - 1) / CI), (unsigned)a.nsplit);
    if (count_waves(a.D) == 4)
        k_count<4><<<g, 256, count_lds_nw(a.D, 4), st>>>(a);
    else
        k_count<2><<<g, 128, count_lds_nw(a.D, 2), st>>>(a);
}

// Eq. (3)/(6) bound count over the users of the item tile's Cauchy-Schwarz
// prefix.  Rows are augmented so that one product gives the bound plus its
// rounding slack: [W p, tail(p), ||p||] . [W u, tail(u), s ||u||].
constexpr int BA = 16;            // augmented row length
constexpr int BLD = BA + LDS_PAD;

__global__ __launch_bounds__(256) void k_bound(BoundArgs a) {
    __shared__ float Psh[CI * BLD];
    __shared__ float Ush[CU * BLD];
    __shared__ int wsum[4 * CI];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t ib = (int64_t)blockIdx.x * CI;
    const int split = blockIdx.y;
    for (int e = tid; e < CI * 4; e += 256) {
        int r = e >> 2, c = e & 3;
        int64_t it = ib + r;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (it < a.m) v = reinterpret_cast<const float4 *>(a.Pa)[it * 4 + c];
        *reinterpret_cast<float4 *>(Psh + r * BLD + 4 * c) = v;
    }
    int cnt[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) cnt[i] = 0;
    const int64_t ulen = a.cs[ib];  // largest prefix of the tile (norm order)
    const int64_t nchunks = (ulen + CU - 1) / CU;
    for (int64_t ch = split; ch < nchunks; ch += a.nsplit) {
        const int64_t u0 = ch * CU;
        __syncthreads();
        for (int e = tid; e < CU * 4; e += 256) {
            int r = e >> 2, c = e & 3;
            int64_t us = u0 + r;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (us < ulen) v = reinterpret_cast<const float4 *>(a.Ua)[us * 4 + c];
            *reinterpret_cast<float4 *>(Ush + r * BLD + 4 * c) = v;
        }
        __syncthreads();
        const int64_t us = u0 + w * 32 + (lane & 31);
        const float tlo = (us < ulen) ? a.tau_lo[us] : INFINITY;
        f32x16 acc0 = {0}, acc1 = {0};
        mfma32x2_f32(acc0, acc1, Psh, Psh + 32 * BLD, Ush + w * 32 * BLD, BLD, BA / 2, lane);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            cnt[i] += (acc0[i] >= tlo) ? 1 : 0;
            cnt[16 + i] += (acc1[i] >= tlo) ? 1 : 0;
        }
    }
#pragma unroll
    for (int i = 0; i < 32; ++i) {
        const int s = half_sum(cnt[i]);
        const int r = mfma32_row(i & 15, lane) + ((i < 16) ? 0 : 32);
        if ((lane & 31) == 0) wsum[w * CI + r] = s;
    }
    __syncthreads();
    if (tid < CI) {
        const int64_t it = ib + tid;
        const int s = wsum[tid] + wsum[CI + tid] + wsum[2 * CI + tid] + wsum[3 * CI + tid];
        if (it < a.m) a.partial[(int64_t)split * a.m + it] = s;
    }
    if (a.pairs && tid == 0) {
        // statistics only: pairs of the user chunks this workgroup evaluated
        int64_t np = 0;
        const int64_t rows = (a.m - ib < CI) ? (a.m - ib) : CI;
        for (int64_t ch = split; ch < nchunks; ch += a.nsplit) {
            const int64_t u0 = ch * CU;
            np += rows * ((ulen - u0 < CU) ? (ulen - u0) : CU);
        }
        atomicAdd(a.pairs, (unsigned long long)np);
    }
}

void launch_bound(const BoundArgs &a, hipStream_t st) {
    dim3 g((unsigned)((a.m + CI - 1) / CI), (unsigned)a.nsplit);
    k_bound<<<g, 256, 0, st>>>(a);
}

__global__ void k_colsum(const int32_t *__restrict__ partial, int nsplit, int64_t cols,
                         int32_t *__restrict__ out) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= cols) return;
    int s = 0;
    for (int q = 0; q < nsplit; ++q) s += partial[(int64_t)q * cols + j];
    out[j] = s;
}

void launch_colsum(const int32_t *partial, int nsplit, int64_t cols, int32_t *out,
                   hipStream_t st) {
    k_colsum<<<(unsigned)((cols + 255) / 256), 256, 0, st>>>(partial, nsplit, cols, out);
}

__global__ void k_visit_keys(const int32_t *__restrict__ us, const int32_t *__restrict__ inv,
                             int64_t m, uint32_t *__restrict__ key, int32_t *__restrict__ val) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= m) return;
    int r = inv[c];
    key[c] = ~(uint32_t)us[r];
    val[c] = r;
}

void launch_visit_keys(const int32_t *uscore, const int32_t *inv, int64_t m, uint32_t *key,
                       int32_t *val, hipStream_t st) {
    k_visit_keys<<<(unsigned)((m + 255) / 256), 256, 0, st>>>(uscore, inv, m, key, val);
}

__global__ void k_gather_i32(const int32_t *__restrict__ src, const int32_t *__restrict__ idx,
                             int64_t n, int32_t *__restrict__ dst) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[idx[i]];
}

void launch_gather_i32(const int32_t *src, const int32_t *idx, int64_t n, int32_t *dst,
                       hipStream_t st) {
    k_gather_i32<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(src, idx, n, dst);
}

// ------------------------------------------------------------------ top-N
// One workgroup: the kept list plus the batch items that can enter it are
// sorted (bitonic, descending keys score<<32 | ~id) in LDS.
constexpr int TOPN_CAP = 8192;

__global__ __launch_bounds__(1024) void k_topn_merge(const int32_t *__restrict__ partial,
                                                     int nsplit, int64_t nb,
                                                     const int32_t *__restrict__ batch_ids,
                                                     int N, uint64_t *__restrict__ top,
                                                     int32_t *__restrict__ status,
                                                     int32_t *__restrict__ batch_scores) {
    __shared__ uint64_t key[TOPN_CAP];
    __shared__ int cnt;
    const int t = threadIdx.x;
    const int kept = status[1];
    const int tauN = status[0];
    if (t == 0) cnt = kept;
    for (int i = t; i < kept; i += 1024) key[i] = top[i];
    __syncthreads();
    for (int64_t j = t; j < nb; j += 1024) {
        int s = 0;
        for (int q = 0; q < nsplit; ++q) s += partial[(int64_t)q * nb + j];
        if (batch_scores) batch_scores[j] = s;
        if (s >= tauN) {
            int pos = atomicAdd(&cnt, 1);
            key[pos] = ((uint64_t)(uint32_t)s << 32) | (uint64_t)(~(uint32_t)batch_ids[j]);
        }
    }
    __syncthreads();
    const int total = cnt;
    int P2 = 1;
    while (P2 < total) P2 <<= 1;
    for (int i = total + t; i < P2; i += 1024) key[i] = 0ull;
    __syncthreads();
    for (int kk = 2; kk <= P2; kk <<= 1) {
        for (int j = kk >> 1; j > 0; j >>= 1) {
            for (int i = t; i < P2; i += 1024) {
                int l = i ^ j;
                if (l > i) {
                    uint64_t x = key[i], y = key[l];
                    bool desc = (i & kk) == 0;
                    if ((x < y) == desc) {
                        key[i] = y;
                        key[l] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
    const int keep = total < N ? total : N;
    for (int i = t; i < keep; i += 1024) top[i] = key[i];
    if (t == 0) {
        status[1] = keep;
        status[0] = (keep == N) ? (int)(key[N - 1] >> 32) : -1;
    }
}

void launch_topn_merge(const int32_t *partial, int nsplit, int64_t nb, const int32_t *batch_ids,
                       int N, uint64_t *top, int32_t *status, int32_t *batch_scores,
                       hipStream_t st) {
    k_topn_merge<<<1, 1024, 0, st>>>(partial, nsplit, nb, batch_ids, N, top, status,
                                     batch_scores);
}

}  // namespace rmips
