// Stage (a): tau_u, the k-th largest u . p over all items (Def. 1), exact.
//
// Screening.  A workgroup holds 32 users per wave in registers and streams the
// items in descending-norm order (Alg. 1 step (1)), 64 per tile, through
// the matrix cores in FP32, BF16 or FP8 (e4m3, a power-of-two scale per
// user and per item tile).  With N = ||x||, Nh = ||xq|| and R = ||x - xq||
// of the quantized copies xq (all rounded up), every screened value vh
// satisfies |vh - v| <= E(u, p) = R_u N_p + Nh_u R_p + c Nh_u Nh_p +
// c2 N_u N_p + e_abs against the exact value v: the quantisation error by
// Cauchy-Schwarz, c bounds the matrix-core accumulation, c2 the FP64
// definition's own rounding and the FP32 comparisons.
//
// Phase 1 (first t0 tiles): per lane and register slot the running maximum
// of the lower bounds vh - E; the k-th largest of the 64 slot maxima of a
// user (each slot covers a distinct set of items) is a value L0 that at
// least k items reach, so L0 <= tau_u.
// Phase 2 (all tiles, interleaved over `nsplit` workgroups): an item is a
// candidate when vh + E >= L0; S_k(u) lies among the candidates because
// v >= tau_u >= L0.  A tile whose largest norm satisfies
// N_u * N_p * (1 + 2 c) < L0 for every user of the workgroup ends the scan:
// by Cauchy-Schwarz (Eq. 2) no later item can be a candidate (the early stop
// of the paper's norm-ordered scan, Sec. 4.2); the quantisation terms enter
// through the largest R_p / N_p over all items.
// Final: per user, L* = k-th largest lower bound among the candidates (the
// candidates hold every item whose lower bound reaches L0, so this is the
// k-th largest over all items), the candidates with vh + E >= L* are
// recomputed in FP64, and the k-th in (value desc, id asc) order is tau_u.
// A user whose candidates overflow the list is recomputed by brute force.
#include "common.h"
#include "kernels.h"

namespace rmips {


// Bitonic sort of 32 registers, descending.
__device__ __forceinline__ void cas_desc(float &a, float &b) {
    float hi = fmaxf(a, b), lo = fminf(a, b);
    a = hi;
    b = lo;
}

__device__ __forceinline__ void sort32_desc(float (&v)[32]) {
#pragma unroll
    for (int k = 2; k <= 32; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
            for (int i = 0; i < 32; ++i) {
                int l = i ^ j;
                if (l > i) {
                    if ((i & k) == 0) cas_desc(v[i], v[l]);
                    else cas_desc(v[l], v[i]);
                }
            }
        }
    }
}

// Sort a bitonic sequence of 32 registers, descending.
__device__ __forceinline__ void merge32_desc(float (&v)[32]) {
#pragma unroll
    for (int j = 16; j > 0; j >>= 1) {
#pragma unroll
        for (int i = 0; i < 32; ++i) {
            int l = i ^ j;
            if (l > i) cas_desc(v[i], v[l]);
        }
    }
}

// Screening configuration: up to 12 waves of 32 users (the users' rows stay
// in registers), two item-tile buffers in LDS (the next tile is copied in while
// the current one is used; the registers allow one workgroup per CU, which
// has the LDS to itself), nch 16-byte chunks per half row.
constexpr int SCR_NW = 12;  // at most
// 12 waves while a half row fits in 8 chunks, or 14 in BF16 (three waves
// per SIMD, 168 registers each: the FP32 rows take more matrix steps per
// chunk, so a third wave gains nothing there and the longer rows spill), 8 up
// to 28 chunks (two per SIMD, 256 registers each: a wave's band test then
// runs while the other wave of its SIMD multiplies), 4 for longer rows,
// whose waves need more registers
__host__ __device__ constexpr int screen_waves(int prec, int nch) {
    return (nch <= 8 || (prec == PREC_BF16 && nch <= 14)) ? 12 : nch <= 28 ? 8 : 4;
}
// the bounds-only pass (phase 1 alone, fewer registers): 8 waves, two
// workgroups per CU (128 registers) while a half row fits in 8 chunks
__host__ __device__ constexpr int screen_waves_p1(int prec, int nch) {
    return nch <= 8 ? 8 : screen_waves(prec, nch);
}
template <bool LISTED> __host__ __device__ constexpr int screen_nw(int prec, int nch) {
    return LISTED ? screen_waves(prec, nch) : screen_waves_p1(prec, nch);
}
template <bool LISTED> __host__ __device__ constexpr int screen_wpe(int prec, int nch) {
    return (!LISTED && nch <= 8) ? 4 : screen_waves(prec, nch) / 4;
}
// per tile buffer: N, Nh, R of the 64 items, the tile's largest Nh and R
// and its scale in the first three of 64 slots, and the items' caller ids
// (copied in with the tile, so that no global load is waited for)
constexpr int NSTRIDE = 5 * TILE_ITEMS;
size_t thresh_screen_lds(int prec, int D) {
    const int ls = lds_row_bytes(prec, D);
    return 2 * (size_t)(TILE_ITEMS * ls + LDS_GUARD) + 2 * (size_t)NSTRIDE * 4 +
           16 * sizeof(float);
}

// Item tile t (64 rows, and per item N, Nh, R, and the tile's scalars) into
// LDS buffer b by direct copies; the last wave also takes the per-item
// arrays.  Completion: dma_wait() and a barrier.
template <int NW>
__device__ __forceinline__ void tile_copy(const ThreshArgs &a, int t, int rowb, int w16,
                                          uint32_t magic, int ls, uint8_t *Pbase, float *Nbase,
                                          int b, int w, int lane) {
    const int64_t rb = (int64_t)t * TILE_ITEMS;
    rows_dma(reinterpret_cast<const uint8_t *>(a.Pq) + rb * rowb, rowb, w16, magic,
             TILE_ITEMS - 1, Pbase + (size_t)b * (TILE_ITEMS * ls + LDS_GUARD), w, NW, lane);
    if (w == NW - 1) {
        float *nb = Nbase + b * NSTRIDE;
        dma4(a.Np + rb + lane, nb);
        dma4(a.Nhp + rb + lane, nb + TILE_ITEMS);
        dma4(a.Rp + rb + lane, nb + 2 * TILE_ITEMS);
        const float *sc = lane == 1 ? a.tmax_r + t : (lane == 2 ? a.sp + rb : a.tmax_nh + t);
        dma4(sc, nb + 3 * TILE_ITEMS);
        const int64_t pr = rb + lane < a.m ? rb + lane : a.m - 1;  // padding rows: never candidates
        dma4(a.perm + pr, nb + 4 * TILE_ITEMS);
    }
}

// Element i (0..31) of the pair of accumulators (register i & 15 of block
// i >> 4) for a per-lane i, by selects (no dynamic register index).
__device__ __forceinline__ float pick32(const f32x16 &a0, const f32x16 &a1, int i) {
    const int j = i & 15;
    float x = a0[0], y = a1[0];
#pragma unroll
    for (int q = 1; q < 16; ++q) {
        x = (j == q) ? a0[q] : x;
        y = (j == q) ? a1[q] : y;
    }
    return (i & 16) ? y : x;
}

// Users of one screening workgroup: 32 per wave.  Without a user list the
// grid covers all users once; with one (refinement passes) the workgroups
// stride over the list, whose length is read on the device.
__device__ __forceinline__ int64_t screen_blocks(const ThreshArgs &a, int tu) {
    const int64_t cnt = a.ulist ? (int64_t)*a.ulist_cnt : a.n;
    return (cnt + tu - 1) / tu;
}

// LISTED: a refinement pass over a user list (its own kernel symbol)
template <int PREC, int NCH, bool LISTED>
// three, two or one waves per SIMD, as the wave count above sets
__global__ __launch_bounds__(64 * screen_nw<LISTED>(PREC, NCH)) __attribute__((amdgpu_waves_per_eu(screen_wpe<LISTED>(PREC, NCH))))
void k_thresh_screen(ThreshArgs a) {
    constexpr int NW = screen_nw<LISTED>(PREC, NCH), TU = 32 * NW;
    extern __shared__ __align__(16) uint8_t smem8[];
    const int D = a.D, ls = lds_row_bytes(PREC, D), rowb = D * elem_bytes(PREC);
    const int nch = rowb / 32;
    // item tiles, each followed by LDS_GUARD bytes of zeros; then N, Nh, R
    const int bstride = TILE_ITEMS * ls + LDS_GUARD;
    uint8_t *Pbase = smem8;
    float *Nbase = reinterpret_cast<float *>(Pbase + 2 * bstride);
    float *red = reinterpret_cast<float *>(Nbase + 2 * NSTRIDE);

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int split = blockIdx.y;
    const int w16 = rowb / 16;
    const int ucol = w * 32 + (lane & 31);
    constexpr bool listed = LISTED;
    const int64_t nlist = listed ? (int64_t)*a.ulist_cnt : a.n;
    const int64_t nblk = screen_blocks(a, TU);
    const float rmax = __uint_as_float(*a.rmax_bits);
    // phase 1 only without a list: listed users come with their bound
    const int t0 = listed ? 0 : (a.t0tiles < a.ntiles ? a.t0tiles : a.ntiles);
    auto tile_of = [&](int it) { return it < t0 ? it : split + (it - t0) * a.nsplit; };

    const uint32_t magic = slot_magic(w16);
    unsigned long long pacc = 0;  // statistics: phase-2 pairs screened
    if (tid < 2 * LDS_GUARD / 16) {
        const int g = tid / (LDS_GUARD / 16), e = tid % (LDS_GUARD / 16);
        reinterpret_cast<uint4 *>(Pbase + g * bstride + TILE_ITEMS * ls)[e] =
            make_uint4(0, 0, 0, 0);
    }

    for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        __syncthreads();  // the previous block is done with the tile buffers
        const int64_t pos = blk * TU + ucol;
        const bool uvalid = pos < nlist;
        const int64_t ug = uvalid ? (listed ? (int64_t)a.ulist[pos] : pos) : 0;
        const int64_t nub = (nlist - blk * TU < TU) ? (nlist - blk * TU) : TU;
        int64_t ntile_p2 = 0;
        // this lane's half of its user's row, kept in registers for the whole scan
        uint4 ub[NCH];
        load_half_row<NCH>(ub, reinterpret_cast<const uint8_t *>(a.Uq), ug, uvalid, rowb, nch,
                           lane);
        const float nu = uvalid ? a.Nu[ug] : 0.0f;
        const float nhu = uvalid ? a.Nhu[ug] : 0.0f;
        const float ru = uvalid ? a.Ru[ug] : 0.0f;
        const float su = uvalid ? a.su[ug] : 1.0f;
        const float su_inv = pow2_rcp(su);

        // error bound of this user against an item: E(u,p)
        auto ebound = [&](float n_p, float nh_p, float r_p) {
            return fmaf(ru, n_p,
                        fmaf(nhu, r_p, fmaf(a.c_err * nhu, nh_p, fmaf(a.c2 * nu, n_p, a.e_abs))));
        };
        // exit ratio: vh + E <= K_u * N_p + 2 e_abs for every item p, so no
        // item of norm below (L - 2 e_abs) / K_u reaches L
        auto exit_ratio = [&](float L) {
            float rr = INFINITY;
            if (uvalid) {
                const float K = nu * (1.0f + a.g64 + 2.0f * a.c2) + 2.0f * ru +
                                2.0f * nhu * (rmax + a.c_err * (1.0f + rmax));
                rr = (L > 2.0f * a.e_abs && K > 0.0f) ? (L - 2.0f * a.e_abs) / K * (1.0f - 0x1p-20f)
                                                      : 0.0f;
            }
            return wave_min(rr);
        };

        float L0 = -INFINITY, rwg = INFINITY;
        if (listed) {
            L0 = uvalid ? a.Luse[ug] : INFINITY;
            const float rr = exit_ratio(L0);
            if (lane == 0) red[w] = rr;
        }
        // the user's list for this split holds two halves of cap / 2 entries,
        // one per half-wave (each half-wave sees other item rows), so that
        // each lane appends to its own half with a register count: no
        // atomics.  The final selection reads them as 2 * nsplit lists.
        const int half = a.cap / 2, hw = lane >> 5;
        float2 *mycand = a.cand + (ug * a.nsplit + split) * a.cap + hw * half;
        int32_t *mycid = a.cand_id + (ug * a.nsplit + split) * a.cap + hw * half;
        int myc = 0;  // candidates of this lane's half, stored or not

        // (the barrier at the top of this loop: the previous block is done
        // with the tile buffers)
        tile_copy<NW>(a, tile_of(0), rowb, w16, magic, ls, Pbase, Nbase, 0, w, lane);
        dma_wait();
        __syncthreads();
        if (listed) {
            rwg = red[0];
#pragma unroll
            for (int q = 1; q < NW; ++q) rwg = fminf(rwg, red[q]);
        }
        int buf = 0;
        // phase 1: per-slot maxima of the lower bounds vh - E over the first
        // t0 tiles, then L0 = k-th largest of the user's 64 slot maxima
        if (t0 > 0) {
            float M[32];
#pragma unroll
            for (int i = 0; i < 32; ++i) M[i] = -INFINITY;
            for (int it = 0; it < t0; ++it) {
                const int t = it;
                const int tn = tile_of(it + 1);
                const bool pre = tn < a.ntiles;
                if (pre)
                    tile_copy<NW>(a, tn, rowb, w16, magic, ls, Pbase, Nbase, buf ^ 1, w, lane);
                const uint8_t *Psh = Pbase + buf * bstride;
                const float *Nsh = Nbase + buf * NSTRIDE;
                const int64_t rb = (int64_t)t * TILE_ITEMS;
                const float e_t = ebound(Nsh[0], Nsh[3 * TILE_ITEMS], Nsh[3 * TILE_ITEMS + 1]);
                const float sc = su * Nsh[3 * TILE_ITEMS + 2];
                f32x16 acc0 = {0}, acc1 = {0};
                MMR<PREC, NCH>::rows2(acc0, acc1, Psh, Psh + 32 * ls, ub, ls, nch, D, (a.d + 1) / 2, lane);
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const int r = mfma32_row(i, lane);
                    if (rb + r < a.m) M[i] = fmaxf(M[i], fmaf(acc0[i], sc, -e_t));
                    if (rb + r + 32 < a.m) M[16 + i] = fmaxf(M[16 + i], fmaf(acc1[i], sc, -e_t));
                }
                if (pre) dma_wait();
                __syncthreads();
                buf ^= 1;
            }
            sort32_desc(M);
            float Bv[32];
#pragma unroll
            for (int j = 0; j < 32; ++j) Bv[j] = __shfl_xor(M[31 - j], 32);
#pragma unroll
            for (int j = 0; j < 32; ++j) M[j] = fmaxf(M[j], Bv[j]);
            merge32_desc(M);
            L0 = M[0];
#pragma unroll
            for (int j = 1; j < 32; ++j)
                if (j == a.k - 1) L0 = M[j];
            const float rr = exit_ratio(L0);
            if (lane == 0) red[w] = rr;
            __syncthreads();
            rwg = red[0];
#pragma unroll
            for (int q = 1; q < NW; ++q) rwg = fminf(rwg, red[q]);
        }
        if constexpr (!LISTED) {
            // the bounds-only pass (the launch without a user list): keep L0
            // and go to the next block
            if (split == 0 && lane < 32 && uvalid) a.Luse[ug] = L0;
            continue;
        }
        // phase 2 (tiles split, split + nsplit, ...): candidates vh + E >= L0
        for (int it = t0;; ++it) {
            const int t = tile_of(it);
            if (t >= a.ntiles) break;
            const float *Nsh = Nbase + buf * NSTRIDE;
            if (Nsh[0] < rwg) break;  // Cauchy-Schwarz exit (N is sorted: Nsh[0] is the largest)
            ++ntile_p2;
            const int tn = tile_of(it + 1);
            const bool pre = tn < a.ntiles;
            if (pre)
                tile_copy<NW>(a, tn, rowb, w16, magic, ls, Pbase, Nbase, buf ^ 1, w, lane);
            const uint8_t *Psh = Pbase + buf * bstride;
            const int64_t rb = (int64_t)t * TILE_ITEMS;
            // tile maxima: N is sorted (first item), Nh and R staged with the tile
            const float e_t = ebound(Nsh[0], Nsh[3 * TILE_ITEMS], Nsh[3 * TILE_ITEMS + 1]);
            const float sp_t = Nsh[3 * TILE_ITEMS + 2];
            const float sc = su * sp_t;  // product scale of this (user, tile)
            f32x16 acc0 = {0}, acc1 = {0};
            MMR<PREC, NCH>::rows2(acc0, acc1, Psh, Psh + 32 * ls, ub, ls, nch, D, (a.d + 1) / 2, lane);
            // first on the tile bound, then per item; the scales are powers of
            // two, so multiplying by their exact reciprocals divides exactly
            const float thr = (L0 - e_t) * (su_inv * pow2_rcp(sp_t));
            // (a linear chain: it compiles to three-input maxima)
            float vmax = acc0[0];
#pragma unroll
            for (int i = 1; i < 16; ++i) vmax = fmaxf(vmax, acc0[i]);
#pragma unroll
            for (int i = 0; i < 16; ++i) vmax = fmaxf(vmax, acc1[i]);
            if (__ballot(vmax >= thr && uvalid) != 0ull) {
                // this lane's slots that pass the tile bound (bit i: register
                // i & 15 of block i >> 4), then each of them once
                uint32_t pend = 0u;
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    pend |= (acc0[i] >= thr) ? (1u << i) : 0u;
                    pend |= (acc1[i] >= thr) ? (1u << (16 + i)) : 0u;
                }
                if (!uvalid) pend = 0u;
                while (pend != 0u) {
                    const int i = __builtin_ctz(pend);
                    pend &= pend - 1u;
                    const int r = mfma32_row(i & 15, lane) + (i >> 4) * 32;
                    if (rb + r >= a.m) continue;  // padding rows of the last tile
                    const float v = pick32(acc0, acc1, i) * sc;
                    const float eb = ebound(Nsh[r], Nsh[TILE_ITEMS + r], Nsh[2 * TILE_ITEMS + r]);
                    if (v + eb >= L0) {
                        if (myc < half) {
                            mycand[myc] = make_float2(v, eb);
                            mycid[myc] = __float_as_int(Nsh[4 * TILE_ITEMS + r]);
                        }
                        ++myc;
                    }
                }
            }
            if (pre) dma_wait();
            __syncthreads();
            buf ^= 1;
        }
        if (listed && uvalid) a.cand_cnt[(ug * a.nsplit + split) * 2 + hw] = myc;
        // the bound this pass used (equal for the two lanes of a user)
        if (!listed && split == 0 && lane < 32 && uvalid) a.Luse[ug] = L0;
        pacc += (unsigned long long)(ntile_p2 * TILE_ITEMS * nub);
    }
    if (a.pairs && tid == 0 && pacc)
        atomicAdd(a.pairs + (blockIdx.x & (CSTAT_SLOTS - 1)), pacc);
}

// The passes with a user list (phase 2 alone) for BF16 and the f8f6f4
// formats, with two blocks of 32 users per wave: each item chunk read from
// LDS feeds four products (two item blocks x two user blocks), half the LDS
// reads per product of k_thresh_screen.  8 waves of 64 users (two per SIMD:
// both users' half rows stay in registers).  The band test, the candidate
// lists and the exit are k_thresh_screen's, per user block.
constexpr int SCR2_NW = 8;
__host__ __device__ constexpr bool screen_u2(int prec, int nch) {
    return prec != PREC_FP32 && nch <= 16;
}
template <int PREC, int NCH>
__global__ __launch_bounds__(64 * SCR2_NW) __attribute__((amdgpu_waves_per_eu(2)))
void k_thresh_screen_u2(ThreshArgs a) {
    constexpr int NW = SCR2_NW, TU = 64 * NW;
    extern __shared__ __align__(16) uint8_t smem8[];
    const int D = a.D, ls = lds_row_bytes(PREC, D), rowb = D * elem_bytes(PREC);
    const int nch = rowb / 32;
    const int bstride = TILE_ITEMS * ls + LDS_GUARD;
    uint8_t *Pbase = smem8;
    float *Nbase = reinterpret_cast<float *>(Pbase + 2 * bstride);
    float *red = reinterpret_cast<float *>(Nbase + 2 * NSTRIDE);

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int split = blockIdx.y;
    const int w16 = rowb / 16;
    const int64_t nlist = (int64_t)*a.ulist_cnt;
    const int64_t nblk = (nlist + TU - 1) / TU;
    const float rmax = __uint_as_float(*a.rmax_bits);
    auto tile_of = [&](int it) { return split + it * a.nsplit; };

    const uint32_t magic = slot_magic(w16);
    unsigned long long pacc = 0;  // statistics: pairs screened
    if (tid < 2 * LDS_GUARD / 16) {
        const int g = tid / (LDS_GUARD / 16), e = tid % (LDS_GUARD / 16);
        reinterpret_cast<uint4 *>(Pbase + g * bstride + TILE_ITEMS * ls)[e] =
            make_uint4(0, 0, 0, 0);
    }
    const int half = a.cap / 2, hw = lane >> 5;

    for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        __syncthreads();  // the previous block is done with the tile buffers
        const int64_t nub = (nlist - blk * TU < TU) ? (nlist - blk * TU) : TU;
        int64_t ntile_p2 = 0;
        // user block h of this wave: users w * 64 + 32 h + (lane & 31)
        bool uvalid[2];
        int64_t ug[2];
        uint4 ub0[NCH], ub1[NCH];
        float nu[2], nhu[2], ru[2], su[2], su_inv[2], L0[2];
        float2 *mycand[2];
        int32_t *mycid[2];
        int myc[2] = {0, 0};
        float rr = INFINITY;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int64_t pos = blk * TU + w * 64 + 32 * h + (lane & 31);
            uvalid[h] = pos < nlist;
            ug[h] = uvalid[h] ? (int64_t)a.ulist[pos] : 0;
            nu[h] = uvalid[h] ? a.Nu[ug[h]] : 0.0f;
            nhu[h] = uvalid[h] ? a.Nhu[ug[h]] : 0.0f;
            ru[h] = uvalid[h] ? a.Ru[ug[h]] : 0.0f;
            su[h] = uvalid[h] ? a.su[ug[h]] : 1.0f;
            su_inv[h] = pow2_rcp(su[h]);
            L0[h] = uvalid[h] ? a.Luse[ug[h]] : INFINITY;
            mycand[h] = a.cand + (ug[h] * a.nsplit + split) * a.cap + hw * half;
            mycid[h] = a.cand_id + (ug[h] * a.nsplit + split) * a.cap + hw * half;
            // exit ratio as in k_thresh_screen
            if (uvalid[h]) {
                const float K = nu[h] * (1.0f + a.g64 + 2.0f * a.c2) + 2.0f * ru[h] +
                                2.0f * nhu[h] * (rmax + a.c_err * (1.0f + rmax));
                const float r = (L0[h] > 2.0f * a.e_abs && K > 0.0f)
                                    ? (L0[h] - 2.0f * a.e_abs) / K * (1.0f - 0x1p-20f)
                                    : 0.0f;
                rr = fminf(rr, r);
            }
        }
        load_half_row<NCH>(ub0, reinterpret_cast<const uint8_t *>(a.Uq), ug[0], uvalid[0], rowb,
                           nch, lane);
        load_half_row<NCH>(ub1, reinterpret_cast<const uint8_t *>(a.Uq), ug[1], uvalid[1], rowb,
                           nch, lane);
        rr = wave_min(rr);
        if (lane == 0) red[w] = rr;
        auto ebound = [&](int h, float n_p, float nh_p, float r_p) {
            return fmaf(ru[h], n_p, fmaf(nhu[h], r_p,
                                         fmaf(a.c_err * nhu[h], nh_p, fmaf(a.c2 * nu[h], n_p, a.e_abs))));
        };
        tile_copy<NW>(a, tile_of(0), rowb, w16, magic, ls, Pbase, Nbase, 0, w, lane);
        dma_wait();
        __syncthreads();
        float rwg = red[0];
#pragma unroll
        for (int q = 1; q < NW; ++q) rwg = fminf(rwg, red[q]);
        int buf = 0;
        for (int it = 0;; ++it) {
            const int t = tile_of(it);
            if (t >= a.ntiles) break;
            const float *Nsh = Nbase + buf * NSTRIDE;
            if (Nsh[0] < rwg) break;  // Cauchy-Schwarz exit (N is sorted: Nsh[0] is the largest)
            ++ntile_p2;
            const int tn = tile_of(it + 1);
            const bool pre = tn < a.ntiles;
            if (pre)
                tile_copy<NW>(a, tn, rowb, w16, magic, ls, Pbase, Nbase, buf ^ 1, w, lane);
            const uint8_t *Psh = Pbase + buf * bstride;
            const int64_t rb = (int64_t)t * TILE_ITEMS;
            const float sp_t = Nsh[3 * TILE_ITEMS + 2];
            f32x16 acc[2][2];
#pragma unroll
            for (int h = 0; h < 2; ++h) acc[h][0] = acc[h][1] = f32x16{0};
            MMR<PREC, NCH>::rows4(acc, Psh, Psh + 32 * ls, ub0, ub1, ls, D, lane);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const float e_t = ebound(h, Nsh[0], Nsh[3 * TILE_ITEMS], Nsh[3 * TILE_ITEMS + 1]);
                const float sc = su[h] * sp_t;
                const float thr = (L0[h] - e_t) * (su_inv[h] * pow2_rcp(sp_t));
                float vmax = acc[h][0][0];
#pragma unroll
                for (int i = 1; i < 16; ++i) vmax = fmaxf(vmax, acc[h][0][i]);
#pragma unroll
                for (int i = 0; i < 16; ++i) vmax = fmaxf(vmax, acc[h][1][i]);
                if (__ballot(vmax >= thr && uvalid[h]) != 0ull) {
                    uint32_t pend = 0u;
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        pend |= (acc[h][0][i] >= thr) ? (1u << i) : 0u;
                        pend |= (acc[h][1][i] >= thr) ? (1u << (16 + i)) : 0u;
                    }
                    if (!uvalid[h]) pend = 0u;
                    while (pend != 0u) {
                        const int i = __builtin_ctz(pend);
                        pend &= pend - 1u;
                        const int r = mfma32_row(i & 15, lane) + (i >> 4) * 32;
                        if (rb + r >= a.m) continue;  // padding rows of the last tile
                        const float v = pick32(acc[h][0], acc[h][1], i) * sc;
                        const float eb =
                            ebound(h, Nsh[r], Nsh[TILE_ITEMS + r], Nsh[2 * TILE_ITEMS + r]);
                        if (v + eb >= L0[h]) {
                            if (myc[h] < half) {
                                mycand[h][myc[h]] = make_float2(v, eb);
                                mycid[h][myc[h]] = __float_as_int(Nsh[4 * TILE_ITEMS + r]);
                            }
                            ++myc[h];
                        }
                    }
                }
            }
            if (pre) dma_wait();
            __syncthreads();
            buf ^= 1;
        }
#pragma unroll
        for (int h = 0; h < 2; ++h)
            if (uvalid[h]) a.cand_cnt[(ug[h] * a.nsplit + split) * 2 + hw] = myc[h];
        pacc += (unsigned long long)(ntile_p2 * TILE_ITEMS * nub);
    }
    if (a.pairs && tid == 0 && pacc)
        atomicAdd(a.pairs + (blockIdx.x & (CSTAT_SLOTS - 1)), pacc);
}

// ------------------------------------------------------------------ final
// Wave-level bitonic sort of (value, id) pairs in LDS in the order (value
// desc, id asc); the slots from n up to the next power of two are filled
// first.
__device__ void wave_sort_pairs(double *v, int *id, int n, int lane) {
    int P2 = 1;
    while (P2 < n) P2 <<= 1;
    for (int i = n + lane; i < P2; i += 64) {
        v[i] = -INFINITY;
        id[i] = 0x7fffffff;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    for (int kk = 2; kk <= P2; kk <<= 1)
        for (int j = kk >> 1; j > 0; j >>= 1) {
            for (int i = lane; i < P2; i += 64) {
                const int l = i ^ j;
                if (l > i) {
                    const double x = v[i], y = v[l];
                    const int xi = id[i], yi = id[l];
                    const bool y_first = (y > x) || (y == x && yi < xi);
                    const bool desc = (i & kk) == 0;
                    if (y_first == desc) {
                        v[i] = y; v[l] = x;
                        id[i] = yi; id[l] = xi;
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
            __builtin_amdgcn_wave_barrier();
        }
}


constexpr int FIN_WAVES = 4;
constexpr int FIN_WPE = 4;  // waves per SIMD of the final selection
constexpr int FIN_ENTRY_BYTES = 12;  // LDS bytes per list entry of the final selection
size_t final_entry_bytes() { return FIN_ENTRY_BYTES; }
// recomputations per user handed from k_thresh_final to k_thresh_exact;
// more, up to EXACT_WIDE, go to k_thresh_exact_wide
constexpr int EXACT_SLOTS = 8;
constexpr int EXACT_WIDE_J = 16;  // values per lane in k_thresh_exact_wide
constexpr int EXACT_WIDE = 64 * EXACT_WIDE_J;

// Orders this wave's LDS accesses (every list of the final selection is
// private to one wave, so no workgroup barrier is needed).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Wave-wide maximum and sum by DPP steps (no LDS traffic): quad_perm
// [1,0,3,2] and [2,3,0,1] combine the lanes of each quad, row_half_mirror
// and row_mirror the quads of each row of 16, row_bcast:15 (rows 1, 3) and
// row_bcast:31 (rows 2, 3) the rows; lane 63 then holds the result, read
// back as a wave-uniform value.  Lanes left out of a step keep `old`, the
// operation's identity.
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_from(int identity, int v) {
    return __builtin_amdgcn_update_dpp(identity, v, CTRL, ROWS, 0xf, false);
}
__device__ __forceinline__ float dpp_wave_max(float x) {
    const int id = __float_as_int(-INFINITY);
    x = fmaxf(x, __int_as_float(dpp_from<0xB1, 0xf>(id, __float_as_int(x))));
    x = fmaxf(x, __int_as_float(dpp_from<0x4E, 0xf>(id, __float_as_int(x))));
    x = fmaxf(x, __int_as_float(dpp_from<0x141, 0xf>(id, __float_as_int(x))));
    x = fmaxf(x, __int_as_float(dpp_from<0x140, 0xf>(id, __float_as_int(x))));
    x = fmaxf(x, __int_as_float(dpp_from<0x142, 0xa>(id, __float_as_int(x))));
    x = fmaxf(x, __int_as_float(dpp_from<0x143, 0xc>(id, __float_as_int(x))));
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}
__device__ __forceinline__ int dpp_wave_sum(int x) {
    x += dpp_from<0xB1, 0xf>(0, x);
    x += dpp_from<0x4E, 0xf>(0, x);
    x += dpp_from<0x141, 0xf>(0, x);
    x += dpp_from<0x140, 0xf>(0, x);
    x += dpp_from<0x142, 0xa>(0, x);
    x += dpp_from<0x143, 0xc>(0, x);
    return __builtin_amdgcn_readlane(x, 63);
}

// The k-th largest of x[0..n) counting repetitions (-inf when n < k), by
// rounds of the largest value below the previous round's, each counted with
// its repetitions, until k values are reached.  Lists of up to 64 KR values
// are held in registers for the rounds (lane l: values l, l + 64, ...; the
// -inf padding can only be counted once every value is taken, and then the
// result is -inf anyway); longer ones are read from LDS in every round.
constexpr int KTH_KR = 12;
__device__ float wave_kth_largest(const float *x, int n, int k, int lane) {
    float prev = INFINITY, v = -INFINITY;
    int acc = 0;
    if (n <= 64 * KTH_KR) {
        float r[KTH_KR];
#pragma unroll
        for (int j = 0; j < KTH_KR; ++j) r[j] = (lane + 64 * j < n) ? x[lane + 64 * j] : -INFINITY;
        for (int rd = 0; rd < k && acc < k; ++rd) {
            float mx = -INFINITY;
#pragma unroll
            for (int j = 0; j < KTH_KR; ++j) mx = (r[j] < prev) ? fmaxf(mx, r[j]) : mx;
            mx = dpp_wave_max(mx);
            int c = 0;
#pragma unroll
            for (int j = 0; j < KTH_KR; ++j) c += (r[j] == mx) ? 1 : 0;
            acc += dpp_wave_sum(c);
            prev = mx;
            v = mx;
        }
    } else {
        for (int rd = 0; rd < k && acc < k; ++rd) {
            float mx = -INFINITY;
            for (int e = lane; e < n; e += 64) {
                const float y = x[e];
                mx = (y < prev) ? fmaxf(mx, y) : mx;
            }
            mx = dpp_wave_max(mx);
            int c = 0;
            for (int e = lane; e < n; e += 64) c += (x[e] == mx) ? 1 : 0;
            acc += dpp_wave_sum(c);
            prev = mx;
            v = mx;
        }
    }
    return acc >= k ? v : -INFINITY;
}

// One wave per user.  The lists of the user's splits are gathered into
// LDS with lower and upper bounds vh -/+ E; L* = k-th largest lower bound.
// A user whose lists overflowed is not resolved here: the k-th largest lower
// bound among its stored candidates (distinct items, so at most tau_u) is a
// tighter starting bound for another screening pass, or, when it does not
// improve on the bound used, the user goes to the exact fallback.
// capT: longest candidate list taken; capP: array stride, capT rounded up
// to a power of two so that the bitonic sorts can pad in place.
// Four waves per SIMD: the FP64 recomputations load 16 values per row at a
// time (latency), which needs more than the registers of six.
template <bool LISTED>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(FIN_WPE)))
void k_thresh_final(ThreshArgs a, int capT, int capP) {
    extern __shared__ float smem[];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int nw = blockDim.x >> 6;  // waves per block (one user each)
    // per-wave LDS (FIN_ENTRY_BYTES per entry): lo, hi (float), cidx (int),
    // the survivors and then the values to recompute compacted in place; the
    // FP64 values v64 take the place of lo and hi once those are no longer
    // read
    uint8_t *base = reinterpret_cast<uint8_t *>(smem) + (size_t)w * capP * FIN_ENTRY_BYTES;
    float *lo = reinterpret_cast<float *>(base);
    float *hi = lo + capP;
    double *v64 = reinterpret_cast<double *>(base);
    int *cidx = reinterpret_cast<int *>(hi + capP);
    __shared__ float Lstar[FIN_WAVES];
    __shared__ int nsurv[FIN_WAVES];
    constexpr bool listed = LISTED;
    const int64_t nlist = listed ? (int64_t)*a.ulist_cnt : a.n;
    unsigned long long *cs = a.cstats ? a.cstats + (blockIdx.x & (CSTAT_SLOTS - 1)) * 4 : nullptr;
    // statistics of this wave's users (candidates, recomputed), added to
    // the counters once at the end
    unsigned long long st_cand = 0, st_rec = 0;

    for (int64_t b0 = (int64_t)blockIdx.x * nw; b0 < nlist; b0 += (int64_t)gridDim.x * nw) {
        const int64_t pos = b0 + w;
        const bool valid = pos < nlist;
        const int64_t u = valid ? (listed ? (int64_t)a.ulist[pos] : pos) : 0;
        // the split counts, one per lane (nsplit <= 64), and their sums;
        // stored entries are laid out split after split
        int cl = 0;
        if (valid && lane < a.nsplit) cl = a.cand_cnt[u * a.nsplit + lane];
        bool over = __ballot(cl > a.cap) != 0ull;
        const int sl = cl < a.cap ? cl : a.cap;
        int pre = sl;  // inclusive prefix of the stored counts
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(pre, o);
            if (lane >= o) pre += y;
        }
        const int stored = __builtin_amdgcn_readlane(pre, 63);
        int total = 0;  // statistics: candidates found, stored or not
        if (cs) {
            int t = cl;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) t += __shfl_xor(t, o);
            total = __builtin_amdgcn_readlane(t, 0);
        }
        if (stored > capT) over = true;  // cannot happen: nsplit * cap <= capT
        wave_sync();  // this wave's previous user is done with its LDS lists
        if (lane == 0) Lstar[w] = -INFINITY;
        if (valid && stored <= capT) {
            // entry g of the joined list (64 at a time, from every split
            // at once): split s = number of inclusive prefixes <= g, entry
            // g - (prefix before s); FIN_GU rounds of loads are issued before
            // their entries are stored, so that their latencies overlap
            constexpr int FIN_GU = 4;
            for (int g0 = 0; g0 < stored; g0 += 64 * FIN_GU) {
                float2 cv[FIN_GU];  // (screened value, its bound E)
                int ci[FIN_GU];
#pragma unroll
                for (int t = 0; t < FIN_GU; ++t) {
                    const int g = g0 + 64 * t + lane;
                    int sp = 0, before = 0;
                    for (int q = 0; q < a.nsplit; ++q) {
                        const int pq = __builtin_amdgcn_readlane(pre, q);
                        if (pq <= g) {
                            sp = q + 1;
                            before = pq;
                        }
                    }
                    cv[t] = make_float2(0.0f, 0.0f);
                    ci[t] = 0;
                    if (g < stored) {
                        const int64_t e = (u * a.nsplit + sp) * a.cap + (g - before);
                        cv[t] = a.cand[e];
                        ci[t] = a.cand_id[e];
                    }
                }
#pragma unroll
                for (int t = 0; t < FIN_GU; ++t) {
                    const int g = g0 + 64 * t + lane;
                    if (g < stored) {
                        lo[g] = cv[t].x - cv[t].y;
                        hi[g] = cv[t].x + cv[t].y;
                        cidx[g] = ci[t];
                    }
                }
            }
        }
        wave_sync();
        // L* = k-th largest lower bound: by ranks for short lists, else by
        // rounds of the largest value below the previous round's, counted
        // with its repetitions, until k values are reached (the list stays
        // in place, paired with the upper bounds and ids)
        if (valid && stored <= capT) {
            if (stored <= 128) {
                for (int e = lane; e < stored; e += 64) {
                    const float x = lo[e];
                    int rank = 0;
                    for (int f = 0; f < stored; ++f) {
                        const float y = lo[f];
                        rank += (y > x) || (y == x && f < e);
                    }
                    if (rank == a.k - 1) Lstar[w] = x;
                }
            } else {
                const float Ls = wave_kth_largest(lo, stored, a.k, lane);
                if (lane == 0) Lstar[w] = Ls;
            }
        }
        wave_sync();
        if (valid && over) {
            if (lane == 0) {
                const float Lprev = a.Luse[u];
                const float Lnew = stored >= a.k ? fmaxf(Lstar[w], Lprev) : Lprev;
                if (a.rlist && Lnew > Lprev) {
                    a.Luse[u] = Lnew;
                    a.rlist[atomicAdd(a.rcnt, 1)] = (int)u;
                    if (cs) atomicAdd(cs + 3, 1ull);
                } else {
                    a.flist[atomicAdd(a.fcnt, 1)] = (int)u;
                    if (cs) atomicAdd(cs + 2, 1ull);
                }
            }
        }
        const bool work = valid && !over;
        if (work) st_cand += (unsigned long long)total;
        // survivors: upper bound reaches L*; their caller ids and bounds
        // compacted in place (a survivor's slot is at most its index, and each
        // round of 64 reads its entries before it writes)
        if (work) {
            const float Ls = Lstar[w];
            int cntw = 0;
            // (no list overflowed: every candidate is stored)
            for (int e0 = 0; e0 < stored; e0 += 64) {
                const int e = e0 + lane;
                float l = 0.0f, h = 0.0f;
                int c = 0;
                if (e < stored) {
                    l = lo[e];
                    h = hi[e];
                    c = cidx[e];
                }
                const bool keep = e < stored && h >= Ls;
                const uint64_t bal = __ballot(keep);
                const int p = cntw + __popcll(bal & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
                __builtin_amdgcn_wave_barrier();
                if (keep) {
                    cidx[p] = c;
                    lo[p] = l;
                    hi[p] = h;
                }
                cntw += __popcll(bal);
            }
            if (lane == 0) nsurv[w] = cntw;
        }
        wave_sync();
        // When only tau is asked for, a survivor whose lower bound exceeds the
        // upper bounds of all but at most k - 2 others ranks above the k-th
        // item; with A such survivors, tau is the (k - A)-th of the others, and
        // only those are recomputed.  A survivor p is such another one when
        // at least k upper bounds (its own included) reach lo[p], that is
        // when lo[p] <= H_k, the k-th largest upper bound of the survivors
        // (counted directly for short lists, where that is cheaper).
        const bool band = a.topk == nullptr;
        int *rid = cidx;
        if (work) {
            const int ns = nsurv[w];
            int nrec = ns;
            if (band) {
                const bool direct = ns <= 128;
                const float Hk = direct ? 0.0f : wave_kth_largest(hi, ns, a.k, lane);
                int cntb = 0;
                for (int p0 = 0; p0 < ns; p0 += 64) {
                    const int p = p0 + lane;
                    bool unc = false;
                    int id = 0;
                    if (p < ns) {
                        const float x = lo[p];
                        if (direct) {
                            int c = 0;
                            for (int q = 0; q < ns; ++q) c += hi[q] >= x;
                            unc = c >= a.k;
                        } else {
                            unc = x <= Hk;
                        }
                        id = cidx[p];
                    }
                    const uint64_t bal = __ballot(unc);
                    const int q = cntb + __popcll(bal & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
                    if (unc) cidx[q] = id;
                    cntb += __popcll(bal);
                }
                nrec = cntb;
            }
            if (lane == 0) nsurv[w] = nrec | ((ns - nrec) << 16);
            st_rec += (unsigned long long)nrec;
        }
        wave_sync();
        // Only tau asked for: the values to recompute are left to
        // k_thresh_exact (at most EXACT_SLOTS, several users per wave) or
        // k_thresh_exact_wide (up to EXACT_WIDE, a wave per user), which hold
        // no lists in LDS and so keep many more row gathers in flight than
        // this kernel.  The ids go to this user's candidate slots (read
        // above), the target rank and the count to its first count slot; -1
        // there for every other user of the list.
        const int nrec_w = nsurv[w] & 0xffff;
        const bool defer = work && band && nrec_w <= EXACT_WIDE;
        if (valid) {
            if (defer) {
                const int64_t c0 = u * a.nsplit * (int64_t)a.cap;
                for (int q = lane; q < nrec_w; q += 64) a.cand_id[c0 + q] = rid[q];
                if (lane == 0)
                    a.cand_cnt[u * a.nsplit] = (a.k - 1 - (nsurv[w] >> 16)) | (nrec_w << 8);
            } else if (lane == 0) {
                a.cand_cnt[u * a.nsplit] = -1;
            }
        }
        wave_sync();  // (v64 takes the place of lo and hi)
        if (work && !defer) {
            const float *urow = a.U + u * a.d;
            for (int q = lane; q < nrec_w; q += 64)
                v64[q] = ip64<16>(urow, a.P + (int64_t)rid[q] * a.d, a.d);
        }
        wave_sync();
        if (work && !defer) {
            const int nrec = nsurv[w] & 0xffff, nabove = nsurv[w] >> 16;
            const int tgt = a.k - 1 - nabove;  // rank of tau among the recomputed
            if (nrec <= 128) {
                for (int q = lane; q < nrec; q += 64) {
                    const double x = v64[q];
                    const int c = rid[q];
                    int rank = 0;
                    for (int f = 0; f < nrec; ++f) {
                        const double y = v64[f];
                        rank += (y > x) || (y == x && rid[f] < c);
                    }
                    if (rank == tgt) {
                        a.tau[u] = x;
                        a.tau_id[u] = c;
                    }
                    if (a.topk && rank < a.k) a.topk[u * a.k + rank] = c;
                    if (a.topv && rank < a.k) a.topv[u * a.k + rank] = x;
                }
            } else {
                wave_sort_pairs(v64, rid, nrec, lane);
                if (lane == 0) {
                    a.tau[u] = v64[tgt];
                    a.tau_id[u] = rid[tgt];
                }
                if (a.topk)
                    for (int r = lane; r < a.k; r += 64) a.topk[u * a.k + r] = rid[r];
                if (a.topv)
                    for (int r = lane; r < a.k; r += 64) a.topv[u * a.k + r] = v64[r];
            }
        }
    }
    if (cs && lane == 0) {
        if (st_cand) atomicAdd(cs, st_cand);
        if (st_rec) atomicAdd(cs + 1, st_rec);
    }
}

// u . p (ip64's arithmetic, term by term) with the user's row staged in LDS
// (ul, 16-byte aligned): 32 values of the item row per step, so that a
// lane's loads of a step cover whole 128-byte blocks of it.  Rows that are
// not 16-byte vectors go through ip64 with the user's row from memory.
__device__ __forceinline__ double ip64_lds_user(const float *ul, const float *ug,
                                                const float *__restrict__ p, int d) {
    if ((d & 3) != 0 || (reinterpret_cast<uintptr_t>(p) & 15) != 0) return ip64<16>(ug, p, d);
    constexpr int RV = 8;
    const float4 *u4 = reinterpret_cast<const float4 *>(ul);
    const float4 *p4 = reinterpret_cast<const float4 *>(p);
    const int d4 = d >> 2;
    double acc = 0.0;
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

// The recomputations left by k_thresh_final: EXACT_SLOTS lanes per user,
// 64 / EXACT_SLOTS users per wave over the same list.  Lane q of a user with
// n <= EXACT_SLOTS values to recompute takes the q-th id; the value of rank
// tgt among the n, in the order (value desc, id asc), is tau_u.  Each user's
// row is staged in LDS once for its lanes (workgroups of four waves).
template <bool LISTED>
__global__ __launch_bounds__(256) void k_thresh_exact(ThreshArgs a) {
    constexpr int UPW = 64 / EXACT_SLOTS;  // users per wave
    __shared__ __align__(16) float urow_s[4][UPW][DMAX];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int grp = lane / EXACT_SLOTS, q = lane % EXACT_SLOTS;
    const int nw = blockDim.x >> 6;
    const int64_t nlist = LISTED ? (int64_t)*a.ulist_cnt : a.n;
    for (int64_t b0 = ((int64_t)blockIdx.x * nw + w) * UPW; b0 < nlist;
         b0 += (int64_t)gridDim.x * nw * UPW) {
        const int64_t pos = b0 + grp;
        const bool valid = pos < nlist;
        const int64_t u = valid ? (LISTED ? (int64_t)a.ulist[pos] : pos) : 0;
        const int meta = valid ? a.cand_cnt[u * a.nsplit] : -1;
        // (longer lists are k_thresh_exact_wide's)
        const int nrec = (meta < 0 || (meta >> 8) > EXACT_SLOTS) ? 0 : meta >> 8;
        const int tgt = meta & 255;
        const bool have = q < nrec;
        const float *ug = a.U + u * a.d;
        float *ul = urow_s[w][grp];
        wave_sync();  // the previous users' rows are no longer read
        if (nrec > 0)
            for (int i = q; i < a.d; i += EXACT_SLOTS) ul[i] = ug[i];
        wave_sync();
        int id = 0;
        double v = 0.0;
        if (have) {
            id = a.cand_id[u * a.nsplit * (int64_t)a.cap + q];
            v = ip64_lds_user(ul, ug, a.P + (int64_t)id * a.d, a.d);
        }
        // rank among the user's values: the lanes of its group
        int rank = 0;
#pragma unroll
        for (int j = 0; j < EXACT_SLOTS; ++j) {
            const int src = grp * EXACT_SLOTS + j;
            const double y = __shfl(v, src);
            const int yi = __shfl(id, src);
            rank += (j < nrec && ((y > v) || (y == v && yi < id))) ? 1 : 0;
        }
        if (have && rank == tgt) {
            a.tau[u] = v;
            a.tau_id[u] = id;
        }
    }
}

// The recomputations of users with more than EXACT_SLOTS (at most
// EXACT_WIDE) values: a wave per user, lane l computing values l, l + 64,
// ... (up to EXACT_WIDE_J of them) into the wave's LDS slice; tau_u, the value
// of rank tgt in the order (value desc, id asc), by tgt + 1 rounds of a
// wave-wide maximum over the values not yet taken.  Each wave reads the
// metadata of 64 users at a time and takes the wide ones in turn.
template <bool LISTED>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
void k_thresh_exact_wide(ThreshArgs a) {
    __shared__ __align__(16) float urow_s[4][DMAX];
    __shared__ double val_s[4][EXACT_WIDE];
    __shared__ int id_s[4][EXACT_WIDE];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int nw = blockDim.x >> 6;
    const int64_t nlist = LISTED ? (int64_t)*a.ulist_cnt : a.n;
    const int64_t capU = (int64_t)a.nsplit * a.cap;
    float *ul = urow_s[w];
    double *vw = val_s[w];
    int *iw = id_s[w];
    for (int64_t c0 = ((int64_t)blockIdx.x * nw + w) * 64; c0 < nlist;
         c0 += (int64_t)gridDim.x * nw * 64) {
        const int64_t pos = c0 + lane;
        int64_t myu = 0;
        int meta = -1;
        if (pos < nlist) {
            myu = LISTED ? (int64_t)a.ulist[pos] : pos;
            meta = a.cand_cnt[myu * a.nsplit];
        }
        uint64_t wide = __ballot(meta >= 0 && (meta >> 8) > EXACT_SLOTS);
        while (wide != 0ull) {
            const int src = __builtin_ctzll(wide);
            wide &= wide - 1ull;
            // (wave-uniform)
            const int64_t u = __builtin_amdgcn_readfirstlane((int)__shfl(myu, src));
            const int mt = __builtin_amdgcn_readfirstlane(__shfl(meta, src));
            const int nrec = mt >> 8, tgt = mt & 255;
            const int32_t *ids = a.cand_id + u * capU;
            const float *urow = a.U + u * a.d;
            wave_sync();  // the previous user's row and values are no longer read
            for (int i = lane; i < a.d; i += 64) ul[i] = urow[i];
            wave_sync();
            uint32_t avail = 0u;  // bit j: value lane + 64 j held and not yet taken
            for (int j = 0; j < EXACT_WIDE_J && 64 * j < nrec; ++j) {
                const int q = lane + 64 * j;
                if (q < nrec) {
                    const int id = ids[q];
                    vw[q] = ip64_lds_user(ul, urow, a.P + (int64_t)id * a.d, a.d);
                    iw[q] = id;
                    avail |= 1u << j;
                }
            }
            // (each lane reads back only the values it wrote)
            const int jn = (nrec + 63) / 64;
            double bv = -INFINITY;
            int bi = 0x7fffffff;
            for (int r = 0; r <= tgt; ++r) {
                // this lane's best value not yet taken, then the wave's
                double lv = -INFINITY;
                int li = 0x7fffffff, lj = -1;
                for (int j = 0; j < jn; ++j) {
                    if (!((avail >> j) & 1u)) continue;
                    const double x = vw[lane + 64 * j];
                    const int xi = iw[lane + 64 * j];
                    if (lj < 0 || x > lv || (x == lv && xi < li)) {
                        lv = x;
                        li = xi;
                        lj = j;
                    }
                }
                bv = lv;
                bi = li;
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) {
                    const double ov = __shfl_xor(bv, o);
                    const int oi = __shfl_xor(bi, o);
                    if (ov > bv || (ov == bv && oi < bi)) {
                        bv = ov;
                        bi = oi;
                    }
                }
                // the ids are distinct: the lane holding the maximum takes it
                if (lj >= 0 && li == bi) avail &= ~(1u << lj);
            }
            if (lane == 0) {
                a.tau[u] = bv;
                a.tau_id[u] = bi;
            }
        }
    }
}

// ------------------------------------------------------------------ fallback
// Brute force for users whose candidate list overflowed: one wave per user,
// every item in FP64, per-lane top-k lists merged by k rounds of a wave-wide
// maximum under (value desc, id asc).
constexpr int FB_WAVES = 2;

__global__ __launch_bounds__(64 * FB_WAVES) void k_thresh_fallback(ThreshArgs a) {
    __shared__ double lv[FB_WAVES][64][KMAX];
    __shared__ int li[FB_WAVES][64][KMAX];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int k = a.k;
    const int64_t nf = *a.fcnt;
    for (int64_t i = (int64_t)blockIdx.x * FB_WAVES + w; i < nf;
         i += (int64_t)gridDim.x * FB_WAVES) {
        const int64_t u = a.flist[i];
        const float *urow = a.U + u * a.d;
        double *myv = lv[w][lane];
        int *myi = li[w][lane];
        int cnt = 0;
        for (int64_t j = lane; j < a.m; j += 64) {
            const int c = (int)j;  // caller id
            const double v = ip64(urow, a.P + j * a.d, a.d);
            if (cnt == k) {
                const double tv = myv[k - 1];
                const int ti = myi[k - 1];
                if (!(v > tv || (v == tv && c < ti))) continue;
            }
            int pos = (cnt < k) ? cnt : k - 1;
            while (pos > 0 && (myv[pos - 1] < v || (myv[pos - 1] == v && myi[pos - 1] > c))) {
                myv[pos] = myv[pos - 1];
                myi[pos] = myi[pos - 1];
                --pos;
            }
            myv[pos] = v;
            myi[pos] = c;
            if (cnt < k) ++cnt;
        }
        int head = 0;
        for (int r = 0; r < k; ++r) {
            double bv = (head < cnt) ? myv[head] : -INFINITY;
            int bi = (head < cnt) ? myi[head] : 0x7fffffff;
            int bl = lane;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                double ov = __shfl_xor(bv, o);
                int oi = __shfl_xor(bi, o);
                int ol = __shfl_xor(bl, o);
                if (ov > bv || (ov == bv && oi < bi)) {
                    bv = ov;
                    bi = oi;
                    bl = ol;
                }
            }
            if (lane == bl) ++head;
            if (lane == 0) {
                if (a.topk) a.topk[u * k + r] = bi;
                if (a.topv) a.topv[u * k + r] = bv;
                if (r == k - 1) {
                    a.tau[u] = bv;
                    a.tau_id[u] = bi;
                }
            }
        }
    }
}

template <int PREC>
void launch_screen(const ThreshArgs &a, int nch, dim3 g, size_t lds, hipStream_t st,
                   const char *name) {
    RMIPS_PROF(st, name);
    with_nch<PREC>(nch, [&](auto n) {
        constexpr int NCH = decltype(n)::value;
        if constexpr (screen_u2(PREC, NCH)) {
            if (a.ulist) {
                k_thresh_screen_u2<PREC, NCH><<<g, 64 * SCR2_NW, lds, st>>>(a);
                return;
            }
        }
        if (a.ulist) k_thresh_screen<PREC, NCH, true><<<g, 64 * screen_nw<true>(PREC, NCH), lds, st>>>(a);
        else k_thresh_screen<PREC, NCH, false><<<g, 64 * screen_nw<false>(PREC, NCH), lds, st>>>(a);
    });
}

// Sort keys of the users' early-exit ratios (ascending): the norm below
// which no item reaches the user's starting bound, as in the screening
// kernel; users whose bound is not positive scan every tile (ratio 0).
__global__ void k_exit_keys(ThreshArgs a, uint32_t *__restrict__ key, int32_t *__restrict__ val) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u == 0) {  // the list counters of the passes that follow
        a.lcnt[0] = 0;
        a.lcnt[1] = 0;
        a.lcnt[2] = 0;
        a.lcnt[3] = 0;
        *a.nall = (int32_t)a.n;  // the main pass takes every user
    }
    if (u >= a.n) return;
    const float rmax = __uint_as_float(*a.rmax_bits);
    const float nu = a.Nu[u], nhu = a.Nhu[u], ru = a.Ru[u], L = a.Luse[u];
    const float K = nu * (1.0f + a.g64 + 2.0f * a.c2) + 2.0f * ru +
                    2.0f * nhu * (rmax + a.c_err * (1.0f + rmax));
    const float rr = (L > 2.0f * a.e_abs && K > 0.0f) ? (L - 2.0f * a.e_abs) / K : 0.0f;
    key[u] = float_key(rr);
    val[u] = (int32_t)u;
}

void launch_thresh(const ThreshArgs &a0, hipStream_t st) {
    const int nch = a0.D * elem_bytes(a0.prec) / 32;
    // users per workgroup of the passes with a user list
    const int tu = screen_u2(a0.prec, nch) ? 64 * SCR2_NW : 32 * screen_waves(a0.prec, nch);
    const size_t lds = thresh_screen_lds(a0.prec, a0.D);
    const int64_t ublocks = (a0.n + tu - 1) / tu;
    const int capU = a0.cap * a0.nsplit;
    const int capP = final_stride(capU);
    int fw = (int)((150 * 1024) / ((size_t)capP * FIN_ENTRY_BYTES));  // waves whose lists fit in LDS
    fw = fw < 1 ? 1 : (fw > FIN_WAVES ? FIN_WAVES : fw);
    const size_t lds_fin = (size_t)fw * capP * FIN_ENTRY_BYTES;
    // one resident round of workgroups (FIN_WPE per CU, fewer when their
    // lists fill the LDS): each wave takes many users in turn
    const int64_t fres =
        256 * std::max<int64_t>(1, std::min<int64_t>(FIN_WPE * 4 / fw, (160 * 1024) / lds_fin));
    const int64_t fblocks = std::min<int64_t>((a0.n + fw - 1) / fw, fres);
    // (four 4-wave workgroups per CU are resident)
    const int64_t eblocks = std::min<int64_t>(
        (a0.n + 4 * (64 / EXACT_SLOTS) - 1) / (4 * (64 / EXACT_SLOTS)), 4 * 256);
    // a wave per 64 users of the list, four per workgroup, a few resident
    // rounds
    const int64_t wblocks = std::min<int64_t>((a0.n + 255) / 256, 8 * 256);
    int32_t *LA = a0.lists, *LB = a0.lists + a0.n, *LF = a0.lists + 2 * a0.n;
    auto screen = [&](const ThreshArgs &a, dim3 g, const char *name) {
        if (a.prec == PREC_FP32) launch_screen<PREC_FP32>(a, nch, g, lds, st, name);
        else if (a.prec == PREC_BF16) launch_screen<PREC_BF16>(a, nch, g, lds, st, name);
        else if (a.prec == PREC_FP8) launch_screen<PREC_FP8>(a, nch, g, lds, st, name);
        else if (a.prec == PREC_FP6) launch_screen<PREC_FP6>(a, nch, g, lds, st, name);
        else launch_screen<PREC_FP4>(a, nch, g, lds, st, name);
    };
    // the screening pass writes each (user, split) list as two halves of
    // cap / 2 entries with their own counts: the final selection and the
    // deferred recomputations read them as 2 * nsplit lists
    auto final = [&](const ThreshArgs &a, int capT, const char *nf, const char *ne,
                     const char *nw) {
        ThreshArgs h = a;
        h.nsplit = 2 * a.nsplit;
        h.cap = a.cap / 2;
        {
            RMIPS_PROF(st, nf);
            k_thresh_final<true><<<(unsigned)fblocks, 64 * fw, lds_fin, st>>>(h, capT, capP);
        }
        {
            RMIPS_PROF(st, ne);
            k_thresh_exact<true><<<(unsigned)eblocks, 256, 0, st>>>(h);
        }
        RMIPS_PROF(st, nw);
        k_thresh_exact_wide<true><<<(unsigned)wblocks, 256, 0, st>>>(h);
    };
    // bounds-only pass (the launch without a user list): every user's L0
    // from the first tiles (phase 1), in workgroups of its own size
    ThreshArgs b0 = a0;
    b0.ulist = nullptr;
    b0.ulist_cnt = nullptr;
    b0.nsplit = 1;
    b0.pairs = nullptr;
    const int tu1 = 32 * screen_waves_p1(a0.prec, nch);
    screen(b0, dim3((unsigned)((a0.n + tu1 - 1) / tu1), 1u), "k_thresh_screen/bounds");
    // users in the order of their early-exit ratios, so that the users of a
    // workgroup stop their scans at about the same tile
    {
        RMIPS_PROF(st, "k_exit_keys");
        k_exit_keys<<<(unsigned)((a0.n + 255) / 256), 256, 0, st>>>(a0, a0.ukey, a0.uord);
    }
    // a grouping only: the top 16 bits of the ratio (sign, exponent and 7
    // mantissa bits) are enough, ties stay in user order
    (void)radix_sort_u32(a0.ukey, a0.uord, a0.n, a0.usort, st, 16, 32);
    // main pass: all users, in that order, from their L0
    ThreshArgs a = a0;
    a.ulist = a0.uord;
    a.ulist_cnt = a0.nall;
    a.rlist = a0.refine > 0 ? LA : nullptr;
    a.rcnt = a0.lcnt;
    a.flist = LF;
    a.fcnt = a0.lcnt + 2;
    if (a.ev0) (void)hipEventRecord(a.ev0, st);
    screen(a, dim3((unsigned)ublocks, (unsigned)a.nsplit), "k_thresh_screen/main");
    if (a.ev1) (void)hipEventRecord(a.ev1, st);
    final(a, capU, "k_thresh_final/main", "k_thresh_exact/main", "k_thresh_exact_wide/main");
    // refinement passes over the users whose lists overflowed: the same
    // per-user capacity in fewer, longer lists per split
    int nsr = capU / 64;
    nsr = nsr < 1 ? 1 : (nsr > 8 ? 8 : nsr);
    for (int r = 1; r <= a0.refine && r <= 2; ++r) {
        ThreshArgs b = a0;
        b.ulist = (r == 1) ? LA : LB;
        b.ulist_cnt = a0.lcnt + (r == 1 ? 0 : 1);
        b.rlist = (r < a0.refine && r < 2) ? LB : nullptr;
        b.rcnt = a0.lcnt + 1;
        b.flist = LF;
        b.fcnt = a0.lcnt + 2;
        b.nsplit = nsr;
        b.cap = (capU / nsr) & ~1;  // (even: two halves per list)
        b.t0tiles = 0;
        b.pairs = a0.rpairs;
        // one resident round (one screening workgroup per CU): the lists
        // are usually empty, and the workgroups loop over long ones
        const int64_t gx = ublocks < 256 / nsr ? ublocks : 256 / nsr;
        screen(b, dim3((unsigned)gx, (unsigned)nsr), "k_thresh_screen/refine");
        final(b, b.nsplit * b.cap, "k_thresh_final/refine", "k_thresh_exact/refine",
              "k_thresh_exact_wide/refine");
    }
    int64_t fb = (a0.n + FB_WAVES - 1) / FB_WAVES;
    if (fb > 1024) fb = 1024;
    a.flist = LF;
    a.fcnt = a0.lcnt + 2;
    RMIPS_PROF(st, "k_thresh_fallback");
    k_thresh_fallback<<<(unsigned)fb, 64 * FB_WAVES, 0, st>>>(a);
}

}  // namespace rmips
