// Stable LSD radix sort of (uint32 key, int32 value) pairs, 8 bits per pass.
//
// Used for the orderings the method needs: items by norm (descending),
// users by their pruning ratio tau_u/||u||, and items by upper-bound score
// (descending) with ties kept in item-id order.  Stability is what carries
// the id tie order through: inputs are laid out in id order.
#include "common.h"
#include "kernels.h"

namespace rmips {

constexpr int SORT_THREADS = 256;
constexpr int SORT_ROUNDS = 4;                        // 256-element rounds per block
constexpr int SORT_CHUNK = SORT_THREADS * SORT_ROUNDS;  // elements per block
// Up to this many blocks a pass needs no scan kernels: every scatter block
// sums the digit counts of all blocks itself.  Counts of a pass are then
// laid out [block][digit], otherwise [digit][block] (scanned in place).
constexpr int PREFIX_MAX_BLOCKS = 128;

__device__ __forceinline__ int64_t count_index(bool small, uint32_t dig, int64_t blk,
                                               int nblocks) {
    return small ? blk * 256 + dig : (int64_t)dig * nblocks + blk;
}

// Digit counts of the first pass per block; clears the counts of the later
// passes, which the scatter of the pass before each of them accumulates.
__global__ __launch_bounds__(SORT_THREADS) void k_radix_hist(
    const uint32_t *__restrict__ keys, int64_t n, int shift, int nblocks, int npass,
    uint32_t *__restrict__ counts) {
    __shared__ uint32_t hist[256];
    const int t = threadIdx.x;
    const bool small = nblocks <= PREFIX_MAX_BLOCKS;
    hist[t] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * SORT_CHUNK;
    uint32_t kr[SORT_ROUNDS];
#pragma unroll
    for (int r = 0; r < SORT_ROUNDS; ++r) {
        const int64_t e = base + (int64_t)r * SORT_THREADS + t;
        kr[r] = e < n ? keys[e] : 0u;
    }
#pragma unroll
    for (int r = 0; r < SORT_ROUNDS; ++r)
        if (base + (int64_t)r * SORT_THREADS + t < n) atomicAdd(&hist[(kr[r] >> shift) & 255u], 1u);
    __syncthreads();
    const int64_t stride = (int64_t)256 * nblocks;
    const int64_t ci = count_index(small, t, blockIdx.x, nblocks);
    counts[ci] = hist[t];
    for (int q = 1; q < npass; ++q) counts[q * stride + ci] = 0;
}

// Exclusive scan of counts[0, total) in place, in tiles of SCAN_TILE
// entries: the first kernel sums each tile, the second scans each tile from
// the sum of the tiles before it (at most a few dozen, read by every block).
constexpr int SCAN_PER_THREAD = 16;
constexpr int SCAN_TILE = SORT_THREADS * SCAN_PER_THREAD;

__global__ __launch_bounds__(SORT_THREADS) void k_scan_reduce(const uint32_t *__restrict__ counts,
                                                              int64_t total,
                                                              uint32_t *__restrict__ tsum) {
    __shared__ uint32_t ws[SORT_THREADS / WAVE];
    const int t = threadIdx.x;
    const int64_t b0 = (int64_t)blockIdx.x * SCAN_TILE;
    uint32_t s = 0;
#pragma unroll
    for (int r = 0; r < SCAN_PER_THREAD; ++r) {
        const int64_t e = b0 + (int64_t)r * SORT_THREADS + t;
        s += (e < total) ? counts[e] : 0u;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((t & 63) == 0) ws[t >> 6] = s;
    __syncthreads();
    if (t == 0) {
        uint32_t x = 0;
        for (int q = 0; q < SORT_THREADS / WAVE; ++q) x += ws[q];
        tsum[blockIdx.x] = x;
    }
}

__global__ __launch_bounds__(SORT_THREADS) void k_scan_down(uint32_t *__restrict__ counts,
                                                            int64_t total,
                                                            const uint32_t *__restrict__ tsum) {
    __shared__ uint32_t tot[SORT_THREADS];
    __shared__ uint32_t base;
    const int t = threadIdx.x;
    if (t == 0) {
        uint32_t x = 0;
        for (int q = 0; q < (int)blockIdx.x; ++q) x += tsum[q];
        base = x;
    }
    // each thread: SCAN_PER_THREAD consecutive entries
    const int64_t e0 = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)t * SCAN_PER_THREAD;
    uint32_t v[SCAN_PER_THREAD];
    uint32_t s = 0;
#pragma unroll
    for (int r = 0; r < SCAN_PER_THREAD; ++r) {
        v[r] = (e0 + r < total) ? counts[e0 + r] : 0u;
        s += v[r];
    }
    tot[t] = s;
    __syncthreads();
    // inclusive scan of the thread sums
    for (int o = 1; o < SORT_THREADS; o <<= 1) {
        const uint32_t y = (t >= o) ? tot[t - o] : 0u;
        __syncthreads();
        tot[t] += y;
        __syncthreads();
    }
    uint32_t run = base + tot[t] - s;
#pragma unroll
    for (int r = 0; r < SCAN_PER_THREAD; ++r) {
        if (e0 + r < total) counts[e0 + r] = run;
        run += v[r];
    }
}

// One pass: block b moves its SORT_CHUNK elements to their places.  Its
// first output slot per digit comes either from the scanned counts, or
// (small) from summing the counts of all blocks here: digits before this one
// over all blocks, plus this digit over the blocks before b.  With nshift >=
// 0 the pass also counts the next pass's digits per destination block.
__global__ __launch_bounds__(SORT_THREADS) void k_radix_scatter(
    const uint32_t *__restrict__ kin, const int32_t *__restrict__ vin,
    uint32_t *__restrict__ kout, int32_t *__restrict__ vout, int64_t n,
    int shift, int nshift, int nblocks, const uint32_t *__restrict__ counts,
    uint32_t *__restrict__ cnext) {
    __shared__ uint32_t base[256];
    __shared__ uint32_t wcnt[SORT_THREADS / WAVE][256];
    __shared__ uint32_t ptot[SORT_THREADS / WAVE][256];
    __shared__ uint32_t wsum[SORT_THREADS / WAVE];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const bool small = nblocks <= PREFIX_MAX_BLOCKS;
    // this thread's elements of all rounds, loaded before the offsets are
    // summed
    const int64_t b0 = (int64_t)blockIdx.x * SORT_CHUNK;
    uint32_t kr[SORT_ROUNDS];
    int32_t vr[SORT_ROUNDS];
#pragma unroll
    for (int r = 0; r < SORT_ROUNDS; ++r) {
        const int64_t e = b0 + (int64_t)r * SORT_THREADS + t;
        kr[r] = e < n ? kin[e] : 0u;
        vr[r] = e < n ? vin[e] : 0;
    }
    if (small) {
        // wave w sums the rows w, w + 4, ...: lane l holds digits 4l..4l+3;
        // wcnt collects the rows before this block, ptot all rows
        const uint4 *c4 = reinterpret_cast<const uint4 *>(counts);
        uint4 pre = make_uint4(0, 0, 0, 0), tot = make_uint4(0, 0, 0, 0);
#pragma unroll 8
        for (int b = w; b < nblocks; b += SORT_THREADS / WAVE) {
            const uint4 c = c4[(int64_t)b * 64 + lane];
            tot.x += c.x; tot.y += c.y; tot.z += c.z; tot.w += c.w;
            if (b < (int)blockIdx.x) { pre.x += c.x; pre.y += c.y; pre.z += c.z; pre.w += c.w; }
        }
        reinterpret_cast<uint4 *>(&ptot[w][0])[lane] = tot;
        reinterpret_cast<uint4 *>(&wcnt[w][0])[lane] = pre;
        __syncthreads();
        uint32_t T = 0, P = 0;
#pragma unroll
        for (int q = 0; q < SORT_THREADS / WAVE; ++q) {
            T += ptot[q][t];
            P += wcnt[q][t];
        }
        // exclusive scan of the digit totals over the 256 digits
        uint32_t x = T;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[w] = x;
        __syncthreads();
        uint32_t before = 0;
        for (int q = 0; q < w; ++q) before += wsum[q];
        base[t] = before + x - T + P;
        for (int q = 0; q < SORT_THREADS / WAVE; ++q) wcnt[q][t] = 0;
    } else {
        base[t] = counts[count_index(false, t, blockIdx.x, nblocks)];
        for (int q = 0; q < SORT_THREADS / WAVE; ++q) wcnt[q][t] = 0;
    }
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int r = 0; r < SORT_ROUNDS; ++r) {
        const int64_t e = b0 + (int64_t)r * SORT_THREADS + t;
        const bool active = e < n;
        const uint32_t key = kr[r];
        const int32_t val = vr[r];
        uint32_t dig = (key >> shift) & 255u;
        // lanes of this wave holding the same digit
        uint64_t peers = __ballot(active);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            uint64_t bb = __ballot((dig >> b) & 1u);
            peers &= ((dig >> b) & 1u) ? bb : ~bb;
        }
        const uint32_t rank = __popcll(peers & lt);
        if (active && rank == 0) wcnt[w][dig] = __popcll(peers);
        __syncthreads();
        uint32_t off = base[dig] + rank;
        for (int q = 0; q < w; ++q) off += wcnt[q][dig];
        if (active) {
            kout[off] = key;
            vout[off] = val;
        }
        if (nshift >= 0) {
            // the next digits per destination block: one atomic per group of
            // peers with the same next digit and block (a digit's peers fill
            // consecutive slots, so they meet at most two blocks, told apart
            // by the block's lowest bit)
            const uint32_t nd = (key >> nshift) & 255u, db = off / SORT_CHUNK;
            uint64_t grp = peers;
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const uint64_t bb = __ballot((nd >> b) & 1u);
                grp &= ((nd >> b) & 1u) ? bb : ~bb;
            }
            const uint64_t bb = __ballot(db & 1u);
            grp &= (db & 1u) ? bb : ~bb;
            if (active && (grp & lt) == 0ull)
                atomicAdd(&cnext[count_index(small, nd, db, nblocks)], (uint32_t)__popcll(grp));
        }
        __syncthreads();
        uint32_t add = 0;
        for (int q = 0; q < SORT_THREADS / WAVE; ++q) {
            add += wcnt[q][t];
            wcnt[q][t] = 0;
        }
        base[t] += add;
        __syncthreads();
    }
}

size_t radix_sort_scratch_bytes(int64_t n) {
    int64_t nblocks = (n + SORT_CHUNK - 1) / SORT_CHUNK;
    if (nblocks < 1) nblocks = 1;
    const int64_t ntiles = (256 * nblocks + SCAN_TILE - 1) / SCAN_TILE;
    return (size_t)(4 * 256 * nblocks) * sizeof(uint32_t) +
           2 * ((size_t)n * (sizeof(uint32_t) + sizeof(int32_t)) + 256) +
           (size_t)ntiles * 4 + 1024;
}

// Sort (keys, vals) ascending by the key bits [lo_bit, hi_bit), stably; the
// bits at and above hi_bit must be the same in every key (then the order is
// that of the whole keys).  8 bits per pass, the result in the input
// buffers; `scratch` holds radix_sort_scratch_bytes(n) bytes.
hipError_t radix_sort_u32(uint32_t *keys, int32_t *vals, int64_t n, void *scratch,
                          hipStream_t st, int lo_bit, int hi_bit) {
    if (n <= 1 || hi_bit <= lo_bit) return hipSuccess;
    if (lo_bit < 0 || hi_bit > 32) return hipErrorInvalidValue;
    const int npass = (hi_bit - lo_bit + 7) / 8;
    const int nblocks = (int)((n + SORT_CHUNK - 1) / SORT_CHUNK);
    const bool small = nblocks <= PREFIX_MAX_BLOCKS;
    const int64_t total = (int64_t)256 * nblocks;
    uint32_t *counts = (uint32_t *)scratch;
    uint8_t *p = (uint8_t *)scratch + (size_t)4 * total * sizeof(uint32_t);
    auto carve = [&](size_t bytes) {
        p = (uint8_t *)(((uintptr_t)p + 255) & ~(uintptr_t)255);
        uint8_t *q = p;
        p += bytes;
        return q;
    };
    uint32_t *k1 = (uint32_t *)carve((size_t)n * 4), *k2 = (uint32_t *)carve((size_t)n * 4);
    int32_t *v1 = (int32_t *)carve((size_t)n * 4), *v2 = (int32_t *)carve((size_t)n * 4);
    uint32_t *tsum = (uint32_t *)carve(0);
    const int ntiles = (int)((total + SCAN_TILE - 1) / SCAN_TILE);
    {
        RMIPS_PROF(st, "k_radix_hist");
        k_radix_hist<<<nblocks, SORT_THREADS, 0, st>>>(keys, n, lo_bit, nblocks, npass, counts);
    }
    // the passes run keys -> 1 -> 2 -> 1 ... and the last one writes keys
    const uint32_t *ks = keys;
    const int32_t *vs = vals;
    for (int q = 0; q < npass; ++q) {
        const int shift = lo_bit + 8 * q;
        const bool last = q == npass - 1;
        uint32_t *kd = last ? keys : ((q & 1) ? k2 : k1);
        int32_t *vd = last ? vals : ((q & 1) ? v2 : v1);
        uint32_t *cq = counts + q * total;
        if (!small) {
            RMIPS_PROF(st, "k_scan");
            k_scan_reduce<<<ntiles, SORT_THREADS, 0, st>>>(cq, total, tsum);
            k_scan_down<<<ntiles, SORT_THREADS, 0, st>>>(cq, total, tsum);
        }
        RMIPS_PROF(st, "k_radix_scatter");
        k_radix_scatter<<<nblocks, SORT_THREADS, 0, st>>>(
            ks, vs, kd, vd, n, shift, last ? -1 : shift + 8, nblocks, cq, cq + total);
        ks = kd;
        vs = vd;
    }
    return hipGetLastError();
}

}  // namespace rmips
