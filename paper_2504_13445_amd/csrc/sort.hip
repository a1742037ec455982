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
constexpr int SORT_ROUNDS = 16;                       // 256-element rounds per block
constexpr int SORT_CHUNK = SORT_THREADS * SORT_ROUNDS;  // elements per block

__global__ __launch_bounds__(SORT_THREADS) void k_radix_hist(
    const uint32_t *__restrict__ keys, int64_t n, int shift, int nblocks,
    uint32_t *__restrict__ counts) {
    __shared__ uint32_t hist[256];
    const int t = threadIdx.x;
    hist[t] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * SORT_CHUNK;
    for (int r = 0; r < SORT_ROUNDS; ++r) {
        int64_t e = base + (int64_t)r * SORT_THREADS + t;
        if (e < n) atomicAdd(&hist[(keys[e] >> shift) & 255u], 1u);
    }
    __syncthreads();
    counts[(int64_t)t * nblocks + blockIdx.x] = hist[t];
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

__global__ __launch_bounds__(SORT_THREADS) void k_radix_scatter(
    const uint32_t *__restrict__ kin, const int32_t *__restrict__ vin,
    uint32_t *__restrict__ kout, int32_t *__restrict__ vout, int64_t n,
    int shift, int nblocks, const uint32_t *__restrict__ offsets) {
    __shared__ uint32_t base[256];
    __shared__ uint32_t wcnt[SORT_THREADS / WAVE][256];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    base[t] = offsets[(int64_t)t * nblocks + blockIdx.x];
    for (int q = 0; q < SORT_THREADS / WAVE; ++q) wcnt[q][t] = 0;
    __syncthreads();
    const int64_t b0 = (int64_t)blockIdx.x * SORT_CHUNK;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int r = 0; r < SORT_ROUNDS; ++r) {
        const int64_t e = b0 + (int64_t)r * SORT_THREADS + t;
        const bool active = e < n;
        uint32_t key = active ? kin[e] : 0u;
        int32_t val = active ? vin[e] : 0;
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
        if (active) {
            uint32_t off = base[dig] + rank;
            for (int q = 0; q < w; ++q) off += wcnt[q][dig];
            kout[off] = key;
            vout[off] = val;
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
    return (size_t)(256 * nblocks) * sizeof(uint32_t) +
           (size_t)n * (sizeof(uint32_t) + sizeof(int32_t)) + (size_t)ntiles * 4 + 1024;
}

// Sort (keys, vals) ascending by key, stably; `scratch` holds
// radix_sort_scratch_bytes(n) bytes.  Four passes, so the result ends in
// the input buffers.
hipError_t radix_sort_u32(uint32_t *keys, int32_t *vals, int64_t n,
                          void *scratch, hipStream_t st) {
    if (n <= 1) return hipSuccess;
    int nblocks = (int)((n + SORT_CHUNK - 1) / SORT_CHUNK);
    uint32_t *counts = (uint32_t *)scratch;
    uint8_t *p = (uint8_t *)scratch + (size_t)256 * nblocks * sizeof(uint32_t);
    p = (uint8_t *)(((uintptr_t)p + 255) & ~(uintptr_t)255);
    uint32_t *ktmp = (uint32_t *)p;
    int32_t *vtmp = (int32_t *)(p + (size_t)n * sizeof(uint32_t));
    uint32_t *tsum = (uint32_t *)(vtmp + n);
    const int64_t total = (int64_t)256 * nblocks;
    const int ntiles = (int)((total + SCAN_TILE - 1) / SCAN_TILE);
    uint32_t *ka = keys, *kb = ktmp;
    int32_t *va = vals, *vb = vtmp;
    for (int pass = 0; pass < 4; ++pass) {
        int shift = 8 * pass;
        k_radix_hist<<<nblocks, SORT_THREADS, 0, st>>>(ka, n, shift, nblocks, counts);
        k_scan_reduce<<<ntiles, SORT_THREADS, 0, st>>>(counts, total, tsum);
        k_scan_down<<<ntiles, SORT_THREADS, 0, st>>>(counts, total, tsum);
        k_radix_scatter<<<nblocks, SORT_THREADS, 0, st>>>(ka, va, kb, vb, n, shift,
                                                          nblocks, counts);
        uint32_t *tk = ka; ka = kb; kb = tk;
        int32_t *tv = va; va = vb; vb = tv;
    }
    return hipGetLastError();
}

}  // namespace rmips
