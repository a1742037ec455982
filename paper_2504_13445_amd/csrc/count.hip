// Stage (b): exact scores |T_k(p)| (Def. 2, Eq. 1) of a set of items, and
// stage (c): the Eq. (3)/(6) upper-bound counts uscore(p) and the running
// top-N of the bound-ordered visit (Alg. 2).
//
// Both counting kernels keep a tile of items in LDS and stream users through
// LDS; the matrix cores give an FP32 value per (item, user) pair, each lane
// owns one user column and 16 item rows of a 32x32 block, and counts
// accumulate per lane and item row, so no global atomics are needed: each
// workgroup writes one partial count per item, and a second pass sums the
// partials in a fixed order.
#include "common.h"
#include "kernels.h"

namespace rmips {


// Sum of a per-slot count over the 32 lanes of each half-wave; afterwards
// lanes 0 and 32 hold the totals of their rows.
__device__ __forceinline__ int half_sum(int x) {
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

// Counting workgroup: 8 waves, each owning 32 items (the row operand, kept
// in registers for the whole kernel); users stream through LDS 64 at a time
// (two column blocks), double-buffered where LDS allows, so the next chunk
// loads while the current one is multiplied.
constexpr int CNT_USERS = 64;            // users per chunk
constexpr int AMB_CAP = 1024;            // deferred FP64 rechecks per workgroup
constexpr int AMB_FLUSH = AMB_CAP / 2;   // list length that triggers a flush between chunks

// Counting configuration: waves of 32 items (the items' rows stay in
// registers), two user-chunk buffers in LDS (the next chunk is copied in
// while the current one is used).  8 waves while a half row fits in 16
// chunks (two waves per SIMD, 256 registers each), 4 for longer rows; either
// way the registers allow one workgroup per CU, which has the LDS to itself
// (at most 143 KB, for D = 256 in FP32).
constexpr int CNT_NW = 8;  // at most
__host__ __device__ constexpr int count_waves(int nch) { return nch <= 16 ? 8 : 4; }

// The wide-band precisions (e4m3, e2m3, e2m1) leave a large share of the
// pairs ambiguous (about one in six at d = 200): their rechecks are taken
// chunk by chunk with the chunk's FP32 user rows staged in LDS once, instead
// of one user-row gather per pair.  A lane's ambiguous pairs of a chunk are
// one 32-bit word (16 rows x two user columns) in LDS.
__host__ __device__ constexpr bool count_staged(int prec) { return prec >= PREC_FP8; }
__host__ __device__ inline int staged_stride(int D) { return D + 4; }  // floats per staged row

size_t count_lds(int prec, int D) {
    const int ls = lds_row_bytes(prec, D);
    size_t b = 2 * (size_t)(CNT_USERS * ls + LDS_GUARD) + AMB_CAP * sizeof(int2) +
               32 * CNT_NW * sizeof(int) + 32;
    if (count_staged(prec))
        b += 64 * CNT_NW * sizeof(uint32_t) + (size_t)CNT_USERS * staged_stride(D) * sizeof(float) +
             2 * 32 * CNT_NW * sizeof(int);
    return b;
}

// u . p (ip64's arithmetic: FP64 fused multiply-adds in index order) with
// u staged in LDS, 16-byte aligned; p's 16-byte vectors are read four at a
// time.  Rows that are not whole vectors take one value at a time.
__device__ __forceinline__ double ip64_staged(const float *ul, const float *__restrict__ p, int d) {
    double acc = 0.0;
    if ((d & 3) == 0 && (reinterpret_cast<uintptr_t>(p) & 15) == 0) {
        constexpr int RV = 4;
        const float4 *u4 = reinterpret_cast<const float4 *>(ul);
        const float4 *p4 = reinterpret_cast<const float4 *>(p);
        const int d4 = d >> 2;
        for (int i = 0; i < d4; i += RV) {
            float4 y[RV];
#pragma unroll
            for (int j = 0; j < RV; ++j) y[j] = p4[i + j < d4 ? i + j : d4 - 1];
#pragma unroll
            for (int j = 0; j < RV; ++j) {
                const bool ok = i + j < d4;
                const float4 x = u4[ok ? i + j : d4 - 1];
                acc = __fma_rn((double)(ok ? x.x : 0.f), (double)(ok ? y[j].x : 0.f), acc);
                acc = __fma_rn((double)(ok ? x.y : 0.f), (double)(ok ? y[j].y : 0.f), acc);
                acc = __fma_rn((double)(ok ? x.z : 0.f), (double)(ok ? y[j].z : 0.f), acc);
                acc = __fma_rn((double)(ok ? x.w : 0.f), (double)(ok ? y[j].w : 0.f), acc);
            }
        }
        return acc;
    }
    for (int i = 0; i < d; ++i) acc = __fma_rn((double)ul[i], (double)p[i], acc);
    return acc;
}

// FP64 decision of one (item row, user) pair by the tie rule.
__device__ __forceinline__ bool recheck_pair(const CountArgs &a, int64_t row, int64_t us) {
    const int64_t uid = a.us.uid[us];
    const int64_t orow = a.item_orig ? a.item_orig[row] : row;
    int tie = a.item_tie ? a.item_tie[row] : -1;
    if (tie < 0) tie = 0x7fffffff;  // outside P: after every item of P
    const double v = ip64(a.Uorig + uid * a.d, a.Porig + orow * a.d, a.d);
    return in_topk(v, tie, a.us.tau[us], a.us.tau_id[us]);
}

// Exact count.  For a pair with screened value vh and bound E:
//   vh - E > tau_hi  =>  v > tau_u           (in S_k(u))
//   vh + E < tau_lo  =>  v < tau_u           (not in S_k(u))
// E is taken with the largest N, Nh and R of the wave's 32 items, so both
// tests fold into two per-user thresholds; other pairs are recomputed in
// FP64 and decided by the tie rule.
// NW waves of 32 items; NCH: 16-byte chunks of the register operand.
template <int PREC, int NCH>
// two waves per SIMD where the row fits in 16 chunks
__global__ __launch_bounds__(64 * count_waves(NCH)) __attribute__((amdgpu_waves_per_eu(NCH <= 16 ? 2 : 1)))
void k_count(CountArgs a) {
    constexpr int NW = count_waves(NCH), NT = 64 * NW, CNT_ITEMS = 32 * NW;
    extern __shared__ __align__(16) uint8_t smem8[];
    const int D = a.D, ls = lds_row_bytes(PREC, D), w16 = D * elem_bytes(PREC) / 16;
    const int rowb = D * elem_bytes(PREC), nch = rowb / 32;
    // each user buffer is followed by LDS_GUARD bytes of zeros
    const int bstride = CNT_USERS * ls + LDS_GUARD;
    uint8_t *Ush0 = smem8;
    uint8_t *Ush1 = Ush0 + bstride;
    int2 *amb = reinterpret_cast<int2 *>(Ush0 + 2 * bstride);
    int *cntl = reinterpret_cast<int *>(amb + AMB_CAP);
    int *ambn = cntl + CNT_ITEMS;
    // (wide bands) the lanes' ambiguity words and the chunk's FP32 user
    // rows, after the fixed part of count_lds (16-byte aligned)
    constexpr bool STAGED = count_staged(PREC);
    uint32_t *ambw = reinterpret_cast<uint32_t *>(smem8 + (2 * (size_t)bstride + AMB_CAP * sizeof(int2) +
                                                           32 * CNT_NW * sizeof(int) + 32));
    float *urow_s = reinterpret_cast<float *>(ambw + 64 * CNT_NW);
    const int ustride = staged_stride(D);
    // (wide bands) each item row's original row and tie id
    int *orow_s = reinterpret_cast<int *>(urow_s + (size_t)CNT_USERS * ustride);
    int *tie_s = orow_s + CNT_NW * 32;

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    // item-block-major order: the blocks of the longest prefixes start first
    const int64_t ib = (int64_t)(blockIdx.x / a.nsplit) * CNT_ITEMS;
    const int split = (int)(blockIdx.x % a.nsplit);

    // this lane's half of its item's row (row lane & 31 of the wave's 32),
    // kept in registers for the whole kernel
    uint4 ia[NCH];
    {
        const int64_t it = ib + w * 32 + (lane & 31);
        const bool ok = it < a.nb;
        const int64_t row = ok ? (a.rows ? a.rows[it] : it) : 0;
        load_half_row<NCH>(ia, reinterpret_cast<const uint8_t *>(a.Pq), row, ok, rowb, nch, lane);
    }
    if (tid < CNT_ITEMS) cntl[tid] = 0;
    if constexpr (STAGED) {
        if (tid < CNT_ITEMS) {
            const int64_t it = ib + tid;
            int orow = 0, tie = 0x7fffffff;
            if (it < a.nb) {
                const int64_t row = a.rows ? a.rows[it] : it;
                orow = (int)(a.item_orig ? a.item_orig[row] : row);
                tie = a.item_tie ? a.item_tie[row] : -1;
                if (tie < 0) tie = 0x7fffffff;  // outside P: after every item of P
            }
            orow_s[tid] = orow;
            tie_s[tid] = tie;
        }
    }
    if (tid == 0) *ambn = 0;
    if (tid < 2 * LDS_GUARD / 16) {
        const int g = tid / (LDS_GUARD / 16), e = tid % (LDS_GUARD / 16);
        reinterpret_cast<uint4 *>(Ush0 + g * bstride + CNT_USERS * ls)[e] = make_uint4(0, 0, 0, 0);
    }

    // largest N, Nh, R among this wave's 32 items; row validity bits; row scales
    float mn = 0.0f, mh = 0.0f, mr = 0.0f;
    {
        const int64_t it = ib + w * 32 + (lane & 31);
        if (it < a.nb) {
            const int64_t row = a.rows ? a.rows[it] : it;
            mn = a.Np[row];
            mh = a.Nhp[row];
            mr = a.Rp[row];
        }
#pragma unroll
        for (int o = 1; o < 32; o <<= 1) {
            mn = fmaxf(mn, __shfl_xor(mn, o));
            mh = fmaxf(mh, __shfl_xor(mh, o));
            mr = fmaxf(mr, __shfl_xor(mr, o));
        }
    }
    uint32_t rvalid = 0;
    float srow[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int64_t it = ib + w * 32 + mfma32_row(i, lane);
        const bool ok = it < a.nb;
        rvalid |= ok ? (1u << i) : 0u;
        srow[i] = 1.0f;
        if (scaled_prec(PREC) && ok) srow[i] = a.sp[a.rows ? a.rows[it] : it];
    }

    int cnt[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) cnt[i] = 0;

    const int64_t ulen = a.ulen_dev ? (int64_t)*a.ulen_dev : a.ulen;
    const int64_t nchunks = (ulen + CNT_USERS - 1) / CNT_USERS;
    const uint32_t magic = slot_magic(w16);
    // chunk ch of users into an LDS buffer by direct copies; rows past the
    // last user repeat it (their columns are masked out)
    auto chunk_copy = [&](int64_t ch, uint8_t *dst) {
        const int64_t u0 = ch * CNT_USERS;
        const int64_t left = ulen - u0;
        const int rlast = (int)((left < CNT_USERS ? left : CNT_USERS) - 1);
        rows_dma(reinterpret_cast<const uint8_t *>(a.Us) + u0 * rowb, rowb, w16, magic, rlast,
                 dst, w, NW, lane);
    };
    // per-user fields of a chunk's two user columns, loaded one chunk ahead
    const float mrh = fmaf(a.c_err, mh, mr);
    float4 uq0 = make_float4(0.f, 0.f, 0.f, 0.f), uq1 = uq0;
    float uqs0 = 1.0f, uqs1 = 1.0f;
    auto user_fetch = [&](int64_t c) {
        const int64_t v0 = c * CNT_USERS + (lane & 31), v1 = v0 + 32;
        if (c < nchunks && v0 < ulen) {
            uq0 = a.us.thr[v0];
            uqs0 = a.us.sinv[v0];
        }
        if (c < nchunks && v1 < ulen) {
            uq1 = a.us.thr[v1];
            uqs1 = a.us.sinv[v1];
        }
    };
    // thresholds of one user column against this wave's items, in the
    // units of the screened products (sinv = 1 / s exactly: s is a power of two)
    auto thresholds = [&](const float4 &q, float sinv, float &tin, float &tout) {
        const float e = fmaf(q.z, mn, fmaf(q.w, mrh, a.e_abs));
        tin = (q.x + e) * sinv;
        tout = (q.y - e) * sinv;
    };

    // FP64 rechecks of the first na listed pairs, spread over the workgroup
    auto flush = [&](int na) {
        for (int e = tid; e < na; e += NT) {
            const int2 q = amb[e];
            const int64_t row = a.rows ? a.rows[ib + q.x] : ib + q.x;
            if (recheck_pair(a, row, q.y)) atomicAdd(&cntl[q.x], 1);
        }
    };
    int nall = 0;  // pairs listed (statistics)
    int nst = 0;   // (wide bands) this thread's rechecks from staged rows

    // Phases: the two waves that share a SIMD work in opposite order
    // between the barriers.  An early wave multiplies chunk c and then
    // classifies it; a late wave first classifies chunk c - 1 (products kept
    // from the previous iteration) and then multiplies chunk c.  So one
    // wave's matrix products overlap the other's vector work.  Roles come
    // from the hardware SIMD id, one ticket per wave.
    int *simdc = ambn + 1;
    if (tid < 4) simdc[tid] = 0;

    int64_t ch = split;
    user_fetch(ch);
    if (ch < nchunks) chunk_copy(ch, Ush0);
    dma_wait();
    __syncthreads();
    bool late = false;
    {
        int t = 0;
        if (lane == 0) t = atomicAdd(&simdc[simd_id()], 1);
        late = (__builtin_amdgcn_readfirstlane(t) & 1) != 0;  // uniform in the wave
        // (wide bands: every wave classifies its chunk before the barrier,
        // so that all the words of a chunk are there after it)
        if (STAGED) late = false;
    }
    // the pending classification: products acc0/acc1 of the user columns
    // pus0 and pus0 + 32 with their thresholds
    f32x16 acc0 = {0}, acc1 = {0};
    float ptin0 = INFINITY, ptout0 = INFINITY, ptin1 = INFINITY, ptout1 = INFINITY;
    int64_t pus0 = 0;
    bool pending = false;
    auto classify = [&]() {
        const int64_t us0 = pus0, us1 = pus0 + 32;
        const bool c0 = us0 < ulen, c1 = us1 < ulen;
        // a column past the last user counts nothing (explicit validity)
        const int m0 = c0 ? 1 : 0, m1 = c1 ? 1 : 0;
        // counts, and whether any pair falls between the two thresholds:
        // with e = med3(v, tout, tin) (tout <= tin), v > tin <=> v > e and
        // tout <= v <= tin <=> v == e
        bool anyamb = false;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const float v0 = scaled_prec(PREC) ? acc0[i] * srow[i] : acc0[i];
            const float v1 = scaled_prec(PREC) ? acc1[i] * srow[i] : acc1[i];
            const float e0 = __builtin_amdgcn_fmed3f(v0, ptout0, ptin0);
            const float e1 = __builtin_amdgcn_fmed3f(v1, ptout1, ptin1);
            cnt[i] += (v0 > e0) ? m0 : 0;
            cnt[i] += (v1 > e1) ? m1 : 0;
            anyamb |= (v0 == e0) | (v1 == e1);
        }
        if constexpr (STAGED) {
            // this lane's ambiguous pairs as one word, rechecked after the
            // chunk's barrier (bit i: register i & 15 of block i >> 4)
            uint32_t word = 0u;
            if (__ballot(anyamb) != 0ull) {
                uint32_t ambm0 = 0, ambm1 = 0;
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const float v0 = scaled_prec(PREC) ? acc0[i] * srow[i] : acc0[i];
                    const float v1 = scaled_prec(PREC) ? acc1[i] * srow[i] : acc1[i];
                    ambm0 |= (v0 == __builtin_amdgcn_fmed3f(v0, ptout0, ptin0)) ? (1u << i) : 0u;
                    ambm1 |= (v1 == __builtin_amdgcn_fmed3f(v1, ptout1, ptin1)) ? (1u << i) : 0u;
                }
                ambm0 = c0 ? (ambm0 & rvalid) : 0u;
                ambm1 = c1 ? (ambm1 & rvalid) : 0u;
                word = ambm0 | (ambm1 << 16);
            }
            ambw[w * 64 + lane] = word;
        } else if (__ballot(anyamb) != 0ull) {
            uint32_t ambm0 = 0, ambm1 = 0;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const float v0 = scaled_prec(PREC) ? acc0[i] * srow[i] : acc0[i];
                const float v1 = scaled_prec(PREC) ? acc1[i] * srow[i] : acc1[i];
                ambm0 |= (v0 == __builtin_amdgcn_fmed3f(v0, ptout0, ptin0)) ? (1u << i) : 0u;
                ambm1 |= (v1 == __builtin_amdgcn_fmed3f(v1, ptout1, ptin1)) ? (1u << i) : 0u;
            }
            ambm0 = c0 ? (ambm0 & rvalid) : 0u;
            ambm1 = c1 ? (ambm1 & rvalid) : 0u;
            // this lane's ambiguous pairs, one set bit at a time (bit i:
            // register i & 15 of block i >> 4)
            uint32_t pend = ambm0 | (ambm1 << 16);
            while (pend != 0u) {
                const int i = __builtin_ctz(pend);
                pend &= pend - 1u;
                const int rl = w * 32 + mfma32_row(i & 15, lane);
                const int64_t us = (i < 16) ? us0 : us1;
                const int s = atomicAdd(ambn, 1);
                if (s < AMB_CAP) {
                    amb[s] = make_int2(rl, (int)us);
                } else {
                    const int64_t row = a.rows ? a.rows[ib + rl] : ib + rl;
                    if (recheck_pair(a, row, us)) atomicAdd(&cntl[rl], 1);
                }
            }
        }
        pending = false;
    };
    int buf = 0;
    for (; ch < nchunks; ch += a.nsplit) {
        const int64_t nxt = ch + a.nsplit;
        // the other buffer was last read before the previous barrier
        if (nxt < nchunks) chunk_copy(nxt, buf ? Ush0 : Ush1);
        const uint8_t *Ub = buf ? Ush1 : Ush0;
        const int64_t us0 = ch * CNT_USERS + (lane & 31), us1 = us0 + 32;
        // (a column past the last user keeps these values; classify() counts
        // nothing in it, whatever its products hold)
        float tin0 = INFINITY, tout0 = INFINITY, tin1 = INFINITY, tout1 = INFINITY;
        if (us0 < ulen) thresholds(uq0, uqs0, tin0, tout0);
        if (us1 < ulen) thresholds(uq1, uqs1, tin1, tout1);
        user_fetch(nxt);
        // rows: this wave's items (shared); columns: the two user blocks
        auto multiply = [&]() {
            acc0 = f32x16{0};
            acc1 = f32x16{0};
            MMR<PREC, NCH>::cols2(acc0, acc1, ia, Ub, Ub + 32 * ls, ls, nch, D, (a.d + 1) / 2, lane);
            ptin0 = tin0;
            ptout0 = tout0;
            ptin1 = tin1;
            ptout1 = tout1;
            pus0 = us0;
            pending = true;
        };
        if (!late) multiply();
        if (pending) classify();
        if (late) multiply();
        if (nxt < nchunks) dma_wait();
        __syncthreads();
        buf ^= 1;
        if constexpr (STAGED) {
            // the chunk's rechecks: its users' FP32 rows staged once (a wave
            // per row at a time), then each thread takes the word of the lane
            // with its index, its items' original rows and tie ids from LDS
            const uint32_t myw = ambw[tid];
            if (__syncthreads_or(myw != 0u)) {
                const int64_t u0 = ch * CNT_USERS;
                for (int sl = w; sl < CNT_USERS; sl += NW) {
                    if (u0 + sl >= ulen) break;
                    const float *src = a.Uorig + (int64_t)a.us.uid[u0 + sl] * a.d;
                    for (int i = lane; i < a.d; i += 64) urow_s[sl * ustride + i] = src[i];
                }
                __syncthreads();
                uint32_t bits = myw;
                const int wv = tid >> 6, ln = tid & 63;
                while (bits != 0u) {
                    const int i = __builtin_ctz(bits);
                    bits &= bits - 1u;
                    const int rl = wv * 32 + mfma32_row(i & 15, ln);
                    const int sl = (ln & 31) + (i >= 16 ? 32 : 0);
                    const int64_t usr = u0 + sl;
                    const double v = ip64_staged(urow_s + sl * ustride,
                                                 a.Porig + (int64_t)orow_s[rl] * a.d, a.d);
                    if (in_topk(v, tie_s[rl], a.us.tau[usr], a.us.tau_id[usr]))
                        atomicAdd(&cntl[rl], 1);
                    ++nst;
                }
                __syncthreads();  // (the words and rows of the next chunk)
            }
        }
        // a long list is rechecked by the whole workgroup now, so that the
        // list rarely fills and rechecks rarely run inside one wave
        const int nq = *ambn;  // the same for all threads after the barrier
        if (nq >= AMB_FLUSH) {
            flush(nq < AMB_CAP ? nq : AMB_CAP);
            nall += nq;
            __syncthreads();
            if (tid == 0) *ambn = 0;
            __syncthreads();
        }
    }
    // a late wave's last chunk
    if (pending) classify();
    __syncthreads();
    // deferred FP64 rechecks, spread over the whole workgroup
    {
        const int nq = *ambn;
        flush(nq < AMB_CAP ? nq : AMB_CAP);
        nall += nq;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int s = half_sum(cnt[i]);
        const int rl = w * 32 + mfma32_row(i, lane);
        if ((lane & 31) == 0 && ib + rl < a.nb)
            a.partial[(int64_t)split * a.nb + ib + rl] = s + cntl[rl];
    }
    if (a.rechecks && tid == 0 && nall > 0)
        atomicAdd(reinterpret_cast<unsigned long long *>(a.rechecks), (unsigned long long)nall);
    if constexpr (STAGED) {
        const int ws = wave_sum(nst);
        if (a.rechecks && lane == 0 && ws > 0)
            atomicAdd(reinterpret_cast<unsigned long long *>(a.rechecks), (unsigned long long)ws);
    }
}

template <int PREC>
void launch_count_p(const CountArgs &a, size_t lds, hipStream_t st) {
    with_nch<PREC>(a.D * elem_bytes(PREC) / 32, [&](auto n) {
        constexpr int NCH = decltype(n)::value, NW = count_waves(NCH);
        const unsigned g = (unsigned)((a.nb + 32 * NW - 1) / (32 * NW) * a.nsplit);
        RMIPS_PROF(st, "k_count");
        k_count<PREC, NCH><<<g, 64 * NW, lds, st>>>(a);
    });
}

__global__ __launch_bounds__(256) void k_max_i32(const int32_t *__restrict__ x, int64_t n,
                                                 int32_t *__restrict__ out) {
    __shared__ int32_t wm[4];
    int32_t v = 0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) v = max(v, x[i]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) *out = max(max(wm[0], wm[1]), max(wm[2], wm[3]));
}

void launch_max_i32(const int32_t *x, int64_t n, int32_t *out, hipStream_t st) {
    RMIPS_PROF(st, "k_max_i32");
    k_max_i32<<<1, 256, 0, st>>>(x, n, out);
}

void launch_count(const CountArgs &a, hipStream_t st) {
    if (a.nb <= 0) return;
    const size_t lds = count_lds(a.prec, a.D);
    if (a.prec == PREC_FP32) launch_count_p<PREC_FP32>(a, lds, st);
    else if (a.prec == PREC_BF16) launch_count_p<PREC_BF16>(a, lds, st);
    else if (a.prec == PREC_FP8) launch_count_p<PREC_FP8>(a, lds, st);
    else if (a.prec == PREC_FP6) launch_count_p<PREC_FP6>(a, lds, st);
    else launch_count_p<PREC_FP4>(a, lds, st);
}

// The slots of one batch of the visit in item-row order: the rows index the
// norm-ordered item arrays, so a counting wave's 32 items then have close
// norms, and the error band it takes from their largest N, Nh and R is close
// to each item's own (fewer pairs to recheck in FP64).  Rows and caller ids
// move together, so each count still goes with its item.  One workgroup,
// a bitonic sort of at most BATCH_ORDER_MAX (row, id) pairs in LDS.
constexpr int BATCH_ORDER_MAX = 4096;
__global__ __launch_bounds__(1024) void k_batch_order(int32_t *__restrict__ rows,
                                                      int32_t *__restrict__ cid, int nb) {
    __shared__ uint64_t kv[BATCH_ORDER_MAX];
    int P2 = 1;
    while (P2 < nb) P2 <<= 1;
    for (int i = threadIdx.x; i < P2; i += blockDim.x)
        kv[i] = i < nb ? ((uint64_t)(uint32_t)rows[i] << 32) | (uint32_t)cid[i] : ~0ull;
    __syncthreads();
    for (int kk = 2; kk <= P2; kk <<= 1)
        for (int j = kk >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < P2; i += blockDim.x) {
                const int l = i ^ j;
                if (l > i) {
                    const uint64_t x = kv[i], y = kv[l];
                    if ((x > y) == ((i & kk) == 0)) {
                        kv[i] = y;
                        kv[l] = x;
                    }
                }
            }
            __syncthreads();
        }
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
        rows[i] = (int32_t)(kv[i] >> 32);
        cid[i] = (int32_t)(uint32_t)kv[i];
    }
}

void launch_batch_order(int32_t *rows, int32_t *cid, int64_t nb, hipStream_t st) {
    if (nb < 2 || nb > BATCH_ORDER_MAX) return;  // (larger batches keep the visit order)
    RMIPS_PROF(st, "k_batch_order");
    k_batch_order<<<1, 1024, 0, st>>>(rows, cid, (int)nb);
}

// Eq. (3)/(6) bound count over the users of the item block's Cauchy-Schwarz
// prefix.  Rows are augmented so that one ka-term product gives the bound
// plus its rounding slack: [W p, tail(p), ||p||] . [W u, tail(u), s ||u||],
// each row stored in BF16 (round to nearest) and multiplied in one BF16
// matrix-core step per 16 terms, the rounding of the rows and of the sums
// being covered by s.
//
// A workgroup of BW waves holds 32 * TI items (TI 32-row tiles)
// in every wave's registers; each wave reads blocks of 32 users straight from
// memory into registers (one block ahead), with no LDS and no barrier until
// the final sum of the waves' counts.  KS = ka / 16 steps of K per product.
constexpr int BW = 4;  // waves per bound workgroup
__host__ __device__ constexpr int bound_tiles(int ks) { return ks <= 2 ? 4 : 2; }

// The largest float below t (t finite).  For y = rn(x), pred(y) <= x: the
// subtraction below is thus rounded down.
__device__ __forceinline__ float float_pred(float t) {
    const uint32_t b = __float_as_uint(t);
    return __uint_as_float(t > 0.0f ? b - 1u : (t < 0.0f ? b + 1u : 0x80000001u));
}

template <int KS>
__global__ __launch_bounds__(64 * BW) void k_bound(BoundArgs a) {
    constexpr int TI = bound_tiles(KS), BI = 32 * TI, RW = 2 * KS;  // RW: 16-byte words per row
    __shared__ int wsum[BW][BI];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int h = lane >> 5, col = lane & 31;
    // workgroups in item-block-major order (all splits of a block, then the
    // next block): the blocks of the longest prefixes start first
    const int64_t ib = (int64_t)(blockIdx.x / a.nsplit) * BI;
    const int split = (int)(blockIdx.x % a.nsplit);
    // the items' rows: row col of each tile, K half h of each step
    bf16x8 ah[TI][KS];
#pragma unroll
    for (int t = 0; t < TI; ++t) {
        const int64_t r = ib + 32 * t + col;
#pragma unroll
        for (int q = 0; q < KS; ++q) {
            uint4 x = make_uint4(0, 0, 0, 0);
            if (r < a.mpad) x = a.Pb[r * RW + 2 * q + h];
            ah[t][q] = __builtin_bit_cast(bf16x8, x);
        }
    }
    int cnt[TI][16];
#pragma unroll
    for (int t = 0; t < TI; ++t)
#pragma unroll
        for (int i = 0; i < 16; ++i) cnt[t][i] = 0;

    const int64_t ulen = a.cs[ib];  // largest prefix of the block (norm order)
    const int64_t nblk = (ulen + 31) / 32;
    const int64_t step = (int64_t)a.nsplit * BW;
    // one user column per lane: its row, its threshold lowered
    // by the absolute slack, and whether the column is a user of the prefix
    // (vm = 1) or past it (vm = 0: nothing it holds is counted); clamped
    // index, so every load is in bounds
    auto fetch = [&](int64_t j, uint4 (&bh)[KS], float &tl, int &vm) {
        const int64_t us = j * 32 + col;
        const bool ok = j < nblk && us < ulen;
        const int64_t uc = ok ? us : 0;
#pragma unroll
        for (int q = 0; q < KS; ++q) bh[q] = a.Ub[uc * RW + 2 * q + h];
        tl = float_pred(a.tau_lo[uc] - a.abs_slack);
        vm = ok ? 1 : 0;
    };
    int64_t j = (int64_t)split * BW + w;
    uint4 bh[KS];
    float tl;
    int vm;
    fetch(j, bh, tl, vm);
    int64_t npairs = 0;  // statistics: users of this wave's blocks
    for (; j < nblk; j += step) {
        uint4 nh[KS];
        float nt;
        int nvm;
        fetch(j + step, nh, nt, nvm);
        // the products of tile t + 1 run while tile t's counts are taken
        auto prod = [&](int t, f32x16 &acc) {
            acc = f32x16{0};
#pragma unroll
            for (int q = 0; q < KS; ++q)
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                    ah[t][q], __builtin_bit_cast(bf16x8, bh[q]), acc, 0, 0, 0);
        };
        auto tally = [&](int t, const f32x16 &acc) {
#pragma unroll
            for (int i = 0; i < 16; ++i) cnt[t][i] += (acc[i] >= tl) ? vm : 0;
        };
        f32x16 p0, p1;
        prod(0, p0);
        prod(1, p1);
        tally(0, p0);
        if constexpr (TI == 4) {
            prod(2, p0);
            tally(1, p1);
            prod(3, p1);
            tally(2, p0);
            tally(3, p1);
        } else {
            tally(1, p1);
        }
        npairs += (ulen - j * 32 < 32) ? (ulen - j * 32) : 32;
#pragma unroll
        for (int q = 0; q < KS; ++q) bh[q] = nh[q];
        tl = nt;
        vm = nvm;
    }
#pragma unroll
    for (int t = 0; t < TI; ++t)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int sm = half_sum(cnt[t][i]);
            if (col == 0) wsum[w][32 * t + mfma32_row(i, lane)] = sm;
        }
    __syncthreads();
    if (tid < BI) {
        const int64_t it = ib + tid;
        int sm = 0;
#pragma unroll
        for (int q = 0; q < BW; ++q) sm += wsum[q][tid];
        if (it < a.m) a.partial[(int64_t)split * a.m + it] = sm;
    }
    if (a.pairs && lane == 0 && npairs > 0) {
        const int64_t rows = (a.m - ib < BI) ? (a.m - ib) : BI;
        atomicAdd(a.pairs, (unsigned long long)(rows * npairs));
    }
}

// Longer rows (KS >= 3): a workgroup of BLW waves holds 64 items per wave
// (512 in all) in registers, and every stage of bl_users(KS) users is
// copied into LDS once (direct copies, double-buffered) and read by all the
// waves, so that a user row is fetched once per 512 items.
constexpr int BLW = 8;  // waves per workgroup
// users per stage: 256 while two such stages (rows of 2 KS + 1 16-byte
// slots) and their thresholds fit in the 160 KB of LDS, else 128
__host__ __device__ constexpr int bl_users(int ks) {
    return 2 * 256 * (2 * ks + 1) * 16 + 2 * 256 * 4 <= 160 * 1024 ? 256 : 128;
}
constexpr size_t bound_lds_bytes(int ks) {
    return 2 * (size_t)bl_users(ks) * (2 * ks + 1) * 16 + 2 * (size_t)bl_users(ks) * 4;
}

template <int KS>
__global__ __launch_bounds__(64 * BLW) __attribute__((amdgpu_waves_per_eu(2)))
void k_bound_lds(BoundArgs a) {
    constexpr int TI = 2, BI = 32 * TI * BLW, RW = 2 * KS, LSL = RW + 1;  // LSL: LDS row slots
    constexpr int BL_USERS = bl_users(KS);
    static_assert(KS <= 11, "longer rows take k_bound16");
    // two stage buffers of user rows, then their thresholds (dynamic LDS,
    // bound_lds_bytes(KS))
    extern __shared__ __align__(16) uint8_t smem_b[];
    uint4 (*ush)[BL_USERS * LSL] = reinterpret_cast<uint4 (*)[BL_USERS * LSL]>(smem_b);
    float (*tsh)[BL_USERS] = reinterpret_cast<float (*)[BL_USERS]>(smem_b + 2 * BL_USERS * LSL * 16);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int h = lane >> 5, col = lane & 31;
    // workgroups in item-block-major order (all splits of a block, then the
    // next block): the blocks of the longest prefixes start first
    const int64_t ib = (int64_t)(blockIdx.x / a.nsplit) * BI;
    const int split = (int)(blockIdx.x % a.nsplit);
    // this wave's items: rows ib + 64 w + 32 t + col, K half h
    bf16x8 ah[TI][KS];
#pragma unroll
    for (int t = 0; t < TI; ++t) {
        const int64_t r = ib + 64 * w + 32 * t + col;
#pragma unroll
        for (int q = 0; q < KS; ++q) {
            uint4 x = make_uint4(0, 0, 0, 0);
            if (r < a.mpad) x = a.Pb[r * RW + 2 * q + h];
            ah[t][q] = __builtin_bit_cast(bf16x8, x);
        }
    }
    int cnt[TI][16];
#pragma unroll
    for (int t = 0; t < TI; ++t)
#pragma unroll
        for (int i = 0; i < 16; ++i) cnt[t][i] = 0;

    const int64_t ulen = a.cs[ib];  // largest prefix of the block (norm order)
    const int64_t nblk = (ulen + BL_USERS - 1) / BL_USERS;
    const uint32_t magic = slot_magic(RW);
    // stage j: users [BL_USERS j, BL_USERS (j + 1)) in groups of 64 rows
    // (rows past the prefix repeat its last user, groups wholly past it are
    // not copied: their LDS rows hold whatever an earlier stage left, and
    // only the columns' validity bits keep them out of the counts) and
    // their thresholds
    auto stage = [&](int64_t j, int b) {
#pragma unroll
        for (int g = 0; g < BL_USERS / 64; ++g) {
            const int64_t u0 = j * BL_USERS + 64 * g;
            const int64_t left = ulen - u0;
            if (left <= 0) break;
            const int rlast = (int)((left < 64 ? left : 64) - 1);
            rows_dma(reinterpret_cast<const uint8_t *>(a.Ub + u0 * RW), RW * 16, RW, magic, rlast,
                     reinterpret_cast<uint8_t *>(ush[b] + 64 * g * LSL), w, BLW, lane);
            if (w == BLW - 1) dma4(a.tau_lo + u0 + (lane < rlast ? lane : rlast), tsh[b] + 64 * g);
        }
    };
    int64_t j = split;
    int buf = 0;
    if (j < nblk) stage(j, 0);
    dma_wait();
    __syncthreads();
    int64_t npairs = 0;  // statistics: users of this workgroup's stages
    // products of the last column block not counted yet (from the previous
    // stage), their thresholds and the validity of their user column (none
    // at first)
    f32x16 pc[TI];
#pragma unroll
    for (int t = 0; t < TI; ++t) pc[t] = f32x16{0};
    float tprev = 0.0f;
    int vprev = 0;
    for (; j < nblk; j += a.nsplit) {
        const int64_t nx = j + a.nsplit;
        if (nx < nblk) stage(nx, buf ^ 1);  // the other buffer was last read before the barrier
        const uint4 *U = ush[buf];
        // column blocks of 32 users: the products of block cb run while the
        // counts of block cb - 1 (for cb = 0: the previous stage's last
        // block) are taken, one product and a few compares at a time
#pragma unroll
        for (int cb = 0; cb < BL_USERS / 32; ++cb) {
            const int ul = 32 * cb + col;
            // a column past the prefix counts nothing, whatever its LDS row
            // and threshold hold (explicit validity, not a masking value)
            const int vm = (j * BL_USERS + ul < ulen) ? 1 : 0;
            // read for every lane (stale past the prefix, and then not
            // counted), so that the block has no branch and the products and
            // counts below can interleave
            const float tl = float_pred(tsh[buf][ul] - a.abs_slack);
            f32x16 nc[TI];
#pragma unroll
            for (int t = 0; t < TI; ++t) nc[t] = f32x16{0};
#pragma unroll
            for (int q = 0; q < KS; ++q) {
                const bf16x8 yh = __builtin_bit_cast(bf16x8, U[ul * LSL + 2 * q + h]);
#pragma unroll
                for (int t = 0; t < TI; ++t)
                    nc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[t][q], yh, nc[t], 0, 0, 0);
            }
#pragma unroll
            for (int t = 0; t < TI; ++t)
#pragma unroll
                for (int i = 0; i < 16; ++i) cnt[t][i] += (pc[t][i] >= tprev) ? vprev : 0;
            // the counts (about 72 vector instructions) spread over the products
            constexpr int NPROD = KS * TI, NV = (72 + NPROD - 1) / NPROD;
#pragma unroll
            for (int g = 0; g < NPROD; ++g) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // one product
                __builtin_amdgcn_sched_group_barrier(0x002, NV, 0);  // vector ops
            }
#pragma unroll
            for (int t = 0; t < TI; ++t) pc[t] = nc[t];
            tprev = tl;
            vprev = vm;
        }
        // the counts are taken before the barrier (not moved past it)
#pragma unroll
        for (int t = 0; t < TI; ++t)
#pragma unroll
            for (int i = 0; i < 16; ++i) asm volatile("" : "+v"(cnt[t][i]));
        npairs += (ulen - j * BL_USERS < BL_USERS) ? (ulen - j * BL_USERS) : BL_USERS;
        if (nx < nblk) dma_wait();
        __syncthreads();
        buf ^= 1;
    }
#pragma unroll
    for (int t = 0; t < TI; ++t)
#pragma unroll
        for (int i = 0; i < 16; ++i) cnt[t][i] += (pc[t][i] >= tprev) ? vprev : 0;
#pragma unroll
    for (int t = 0; t < TI; ++t)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int sm = half_sum(cnt[t][i]);
            const int64_t it = ib + 64 * w + 32 * t + mfma32_row(i, lane);
            if (col == 0 && it < a.m) a.partial[(int64_t)split * a.m + it] = sm;
        }
    if (a.pairs && tid == 0 && npairs > 0) {
        const int64_t rows = (a.m - ib < BI) ? (a.m - ib) : BI;
        atomicAdd(a.pairs, (unsigned long long)(rows * npairs));
    }
}

// The longest rows (ka = 32 KT > 176, KT = 6..9 steps of 32 terms): the
// 16x16x32 matrix-core step, so that a wave's items (48: three tiles of 16
// rows) take 12 KT registers and, up to KT = 7, three waves fit on a SIMD (a
// workgroup of 12 waves, 576 items; two waves and 384 items for longer
// rows).  User stages of 128 rows are copied into LDS as in k_bound_lds.
// Operand layout of v_mfma_f32_16x16x32_bf16: lane l feeds row (or column)
// l % 16 with terms 8 (l / 16) .. 8 (l / 16) + 7 of the step, and holds
// result rows 4 (l / 16) + i (i = 0..3) of column l % 16.  Each 32-user
// block is counted right after its products (the other waves of the SIMD
// multiply meanwhile).
__host__ __device__ constexpr int b16_waves(int kt) { return kt <= 7 ? 12 : 8; }  // per workgroup
constexpr int B16_TI = 3;       // 16-row item tiles per wave
constexpr int B16_USERS = 128;  // users per stage
constexpr size_t bound16_lds_bytes(int kt) {
    return 2 * (size_t)B16_USERS * (4 * kt + 1) * 16 + 2 * (size_t)B16_USERS * 4;
}

template <int KT>
__global__ __launch_bounds__(64 * b16_waves(KT)) __attribute__((amdgpu_waves_per_eu(b16_waves(KT) / 4)))
void k_bound16(BoundArgs a) {
    constexpr int B16_W = b16_waves(KT);
    constexpr int BI = 16 * B16_TI * B16_W, RW = 4 * KT, LSL = RW + 1;  // LSL: LDS row slots
    extern __shared__ __align__(16) uint8_t smem_b[];
    uint4 (*ush)[B16_USERS * LSL] = reinterpret_cast<uint4 (*)[B16_USERS * LSL]>(smem_b);
    float (*tsh)[B16_USERS] = reinterpret_cast<float (*)[B16_USERS]>(smem_b + 2 * B16_USERS * LSL * 16);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int c16 = lane & 15, kq = lane >> 4;  // row / column, term block of a step
    const int64_t ib = (int64_t)(blockIdx.x / a.nsplit) * BI;
    const int split = (int)(blockIdx.x % a.nsplit);
    // this wave's items: rows ib + 48 w + 16 t + c16, term block kq of each step
    bf16x8 ah[B16_TI][KT];
#pragma unroll
    for (int t = 0; t < B16_TI; ++t) {
        const int64_t r = ib + 48 * w + 16 * t + c16;
#pragma unroll
        for (int q = 0; q < KT; ++q) {
            uint4 x = make_uint4(0, 0, 0, 0);
            if (r < a.mpad) x = a.Pb[r * RW + 4 * q + kq];
            ah[t][q] = __builtin_bit_cast(bf16x8, x);
        }
    }
    // counts per item row held by this lane: rows 16 t + 4 kq + i
    int cnt[B16_TI][4];
#pragma unroll
    for (int t = 0; t < B16_TI; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) cnt[t][i] = 0;

    const int64_t ulen = a.cs[ib];  // largest prefix of the block (norm order)
    const int64_t nblk = (ulen + B16_USERS - 1) / B16_USERS;
    const uint32_t magic = slot_magic(RW);
    // stage j: users [128 j, 128 (j + 1)) in groups of 64 rows (rows past
    // the prefix repeat its last user, groups wholly past it are not copied:
    // only the columns' validity bits keep them out of the counts) and their
    // thresholds
    auto stage = [&](int64_t j, int b) {
#pragma unroll
        for (int g = 0; g < B16_USERS / 64; ++g) {
            const int64_t u0 = j * B16_USERS + 64 * g;
            const int64_t left = ulen - u0;
            if (left <= 0) break;
            const int rlast = (int)((left < 64 ? left : 64) - 1);
            rows_dma(reinterpret_cast<const uint8_t *>(a.Ub + u0 * RW), RW * 16, RW, magic, rlast,
                     reinterpret_cast<uint8_t *>(ush[b] + 64 * g * LSL), w, B16_W, lane);
            if (w == B16_W - 1) dma4(a.tau_lo + u0 + (lane < rlast ? lane : rlast), tsh[b] + 64 * g);
        }
    };
    int64_t j = split;
    int buf = 0;
    if (j < nblk) stage(j, 0);
    dma_wait();
    __syncthreads();
    int64_t npairs = 0;  // statistics: users of this workgroup's stages
    for (; j < nblk; j += a.nsplit) {
        const int64_t nx = j + a.nsplit;
        if (nx < nblk) stage(nx, buf ^ 1);  // the other buffer was last read before the barrier
        const uint4 *U = ush[buf];
#pragma unroll
        for (int cb = 0; cb < B16_USERS / 32; ++cb) {
            // the two 16-user columns of this block held by this lane, their
            // validity (explicit, not a masking value) and thresholds (read
            // for every lane, so that the block has no branch)
            int vm[2];
            float tl[2];
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int ul = 32 * cb + 16 * c + c16;
                vm[c] = (j * B16_USERS + ul < ulen) ? 1 : 0;
                tl[c] = float_pred(tsh[buf][ul] - a.abs_slack);
            }
            f32x4 acc[B16_TI][2];
#pragma unroll
            for (int t = 0; t < B16_TI; ++t) acc[t][0] = acc[t][1] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int q = 0; q < KT; ++q) {
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const bf16x8 yb = __builtin_bit_cast(
                        bf16x8, U[(32 * cb + 16 * c + c16) * LSL + 4 * q + kq]);
#pragma unroll
                    for (int t = 0; t < B16_TI; ++t)
                        acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[t][q], yb, acc[t][c], 0, 0, 0);
                }
            }
#pragma unroll
            for (int t = 0; t < B16_TI; ++t)
#pragma unroll
                for (int c = 0; c < 2; ++c)
#pragma unroll
                    for (int i = 0; i < 4; ++i) cnt[t][i] += (acc[t][c][i] >= tl[c]) ? vm[c] : 0;
        }
        // the counts are taken before the barrier (not moved past it)
#pragma unroll
        for (int t = 0; t < B16_TI; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) asm volatile("" : "+v"(cnt[t][i]));
        npairs += (ulen - j * B16_USERS < B16_USERS) ? (ulen - j * B16_USERS) : B16_USERS;
        if (nx < nblk) dma_wait();
        __syncthreads();
        buf ^= 1;
    }
    // each row's count: the sum over the 16 lanes of its term block
#pragma unroll
    for (int t = 0; t < B16_TI; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            int x = cnt[t][i];
#pragma unroll
            for (int o = 8; o > 0; o >>= 1) x += __shfl_xor(x, o);
            const int64_t it = ib + 48 * w + 16 * t + 4 * kq + i;
            if (c16 == 0 && it < a.m) a.partial[(int64_t)split * a.m + it] = x;
        }
    if (a.pairs && tid == 0 && npairs > 0) {
        const int64_t rows = (a.m - ib < BI) ? (a.m - ib) : BI;
        atomicAdd(a.pairs, (unsigned long long)(rows * npairs));
    }
}

__host__ __device__ constexpr int bound_items(int ks) {
    return ks >= 12 ? 16 * B16_TI * b16_waves(ks / 2) : ks >= 3 ? 64 * BLW : 32 * bound_tiles(ks);
}

void launch_bound(const BoundArgs &a, hipStream_t st, const char *prof_name) {
    auto go = [&](auto ks) {
        constexpr int KS = decltype(ks)::value, BI = bound_items(KS);
        const unsigned g = (unsigned)((a.m + BI - 1) / BI * a.nsplit);
        RMIPS_PROF(st, prof_name);
        if constexpr (KS >= 12) {
            static_assert(KS % 2 == 0, "rows past 176 terms come in steps of 32");
            k_bound16<KS / 2><<<g, 64 * b16_waves(KS / 2), bound16_lds_bytes(KS / 2), st>>>(a);
        } else if constexpr (KS >= 3) {
            k_bound_lds<KS><<<g, 64 * BLW, bound_lds_bytes(KS), st>>>(a);
        } else {
            k_bound<KS><<<g, 64 * BW, 0, st>>>(a);
        }
    };
    // ka = 16 KS: KS <= 11, or an even KS up to 18 (rows past 176 terms are
    // padded to a multiple of 32)
    switch (a.ka / 16) {
#define RMIPS_BOUND_KS(K) case K: go(std::integral_constant<int, K>{}); break;
        RMIPS_BOUND_KS(1) RMIPS_BOUND_KS(2) RMIPS_BOUND_KS(3) RMIPS_BOUND_KS(4)
        RMIPS_BOUND_KS(5) RMIPS_BOUND_KS(6) RMIPS_BOUND_KS(7) RMIPS_BOUND_KS(8)
        RMIPS_BOUND_KS(9) RMIPS_BOUND_KS(10) RMIPS_BOUND_KS(11) RMIPS_BOUND_KS(12)
        RMIPS_BOUND_KS(14) RMIPS_BOUND_KS(16)
#undef RMIPS_BOUND_KS
    default: go(std::integral_constant<int, 18>{}); break;
    }
}

// splits of each item block's user prefix: about 4096 workgroups, 1 to smax
int bound_splits(int64_t m, int ka, int smax) {
    const int64_t bi = bound_items(ka / 16);
    const int64_t blocks = (m + bi - 1) / bi;
    const int64_t s = (4096 + blocks - 1) / blocks;
    return (int)(s < 1 ? 1 : (s > smax ? smax : s));
}

// out[j] = sum over q of partial[q][j].  A 256-thread block covers 16
// columns with 16 threads each (a thread adds every 16th split, eight loads
// in flight), then adds the 16 partial sums per column through LDS.
__global__ __launch_bounds__(256) void k_colsum(const int32_t *__restrict__ partial, int nsplit,
                                                int64_t cols, int32_t *__restrict__ out) {
    __shared__ int part[16][17];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int64_t j = (int64_t)blockIdx.x * 16 + tx;
    int s = 0;
    if (j < cols) {
        int q = ty;
        for (; q + 16 * 7 < nsplit; q += 16 * 8) {
            int t[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) t[e] = partial[(int64_t)(q + 16 * e) * cols + j];
#pragma unroll
            for (int e = 0; e < 8; ++e) s += t[e];
        }
        for (; q < nsplit; q += 16) s += partial[(int64_t)q * cols + j];
    }
    part[ty][tx] = s;
    __syncthreads();
    if (ty == 0 && j < cols) {
        int t = 0;
#pragma unroll
        for (int e = 0; e < 16; ++e) t += part[e][tx];
        out[j] = t;
    }
}

void launch_colsum(const int32_t *partial, int nsplit, int64_t cols, int32_t *out,
                   hipStream_t st) {
    RMIPS_PROF(st, "k_colsum");
    k_colsum<<<(unsigned)((cols + 15) / 16), 256, 0, st>>>(partial, nsplit, cols, out);
}

__global__ void k_visit_keys(const int32_t *__restrict__ us, const int32_t *__restrict__ inv,
                             int64_t m, uint32_t *__restrict__ key, int32_t *__restrict__ val,
                             int32_t *__restrict__ status) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c == 0 && status) {  // a new running top-N: no N-th score, none kept
        status[0] = -1;
        status[1] = 0;
    }
    if (c >= m) return;
    int r = inv[c];
    key[c] = ~(uint32_t)us[r];
    val[c] = r;
}

void launch_visit_keys(const int32_t *uscore, const int32_t *inv, int64_t m, uint32_t *key,
                       int32_t *val, int32_t *status, hipStream_t st) {
    RMIPS_PROF(st, "k_visit_keys");
    k_visit_keys<<<(unsigned)((m + 255) / 256), 256, 0, st>>>(uscore, inv, m, key, val, status);
}

__global__ void k_gather_i32(const int32_t *__restrict__ src, const int32_t *__restrict__ idx,
                             int64_t n, int32_t *__restrict__ dst) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[idx[i]];
}

void launch_gather_i32(const int32_t *src, const int32_t *idx, int64_t n, int32_t *dst,
                       hipStream_t st) {
    RMIPS_PROF(st, "k_gather_i32");
    k_gather_i32<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(src, idx, n, dst);
}

__global__ void k_gather3_i32(const int32_t *__restrict__ a, const int32_t *__restrict__ b,
                              const int32_t *__restrict__ c, const int32_t *__restrict__ idx,
                              int64_t n, int32_t *__restrict__ da, int32_t *__restrict__ db,
                              int32_t *__restrict__ dc) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t j = idx[i];
    da[i] = a[j];
    db[i] = b[j];
    dc[i] = c[j];
}

void launch_gather3_i32(const int32_t *a, const int32_t *b, const int32_t *c,
                        const int32_t *idx, int64_t n, int32_t *da, int32_t *db, int32_t *dc,
                        hipStream_t st) {
    RMIPS_PROF(st, "k_gather3_i32");
    k_gather3_i32<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(a, b, c, idx, n, da, db, dc);
}

// A segment of the visit order re-bounded: key[i] = id[i], val[i] = i
// (the local slots, to be sorted by id), and the bound of each slot tightened
// to the smaller of its two counts, also written to the norm-order array.
__global__ void k_seg_init(const int32_t *__restrict__ id, int64_t n, uint32_t *__restrict__ key,
                           int32_t *__restrict__ val) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    key[i] = (uint32_t)id[i];
    val[i] = (int32_t)i;
}

void launch_seg_init(const int32_t *id, int64_t n, uint32_t *key, int32_t *val, hipStream_t st) {
    RMIPS_PROF(st, "k_seg_init");
    k_seg_init<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(id, n, key, val);
}

__global__ void k_seg_bound(int32_t *__restrict__ b, const int32_t *__restrict__ b0,
                            const int32_t *__restrict__ rows, int64_t n,
                            int32_t *__restrict__ uscore) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t v = min(b[i], b0[i]);
    b[i] = v;
    uscore[rows[i]] = v;
}

void launch_seg_bound(int32_t *b, const int32_t *b0, const int32_t *rows, int64_t n,
                      int32_t *uscore, hipStream_t st) {
    RMIPS_PROF(st, "k_seg_bound");
    k_seg_bound<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(b, b0, rows, n, uscore);
}

// ------------------------------------------------------------------ top-N
// One workgroup: the kept list plus the batch items that can enter it are
// sorted (bitonic, descending keys score<<32 | ~id) in LDS.
constexpr int TOPN_CAP = 8192;

__global__ __launch_bounds__(1024) void k_topn_merge(const int32_t *__restrict__ scores,
                                                     int64_t nb,
                                                     const int32_t *__restrict__ batch_ids,
                                                     int N, uint64_t *__restrict__ top,
                                                     int32_t *__restrict__ status) {
    __shared__ uint64_t key[TOPN_CAP];
    __shared__ int cnt;
    const int t = threadIdx.x;
    const int kept = status[1];
    const int tauN = status[0];
    if (t == 0) cnt = kept;
    for (int i = t; i < kept; i += 1024) key[i] = top[i];
    __syncthreads();
    for (int64_t j = t; j < nb; j += 1024) {
        const int s = scores[j];
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

void launch_topn_merge(const int32_t *scores, int64_t nb, const int32_t *batch_ids, int N,
                       uint64_t *top, int32_t *status, hipStream_t st) {
    RMIPS_PROF(st, "k_topn_merge");
    k_topn_merge<<<1, 1024, 0, st>>>(scores, nb, batch_ids, N, top, status);
}

}  // namespace rmips
