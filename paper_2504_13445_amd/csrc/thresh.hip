// Stage (a): tau_u, the k-th largest u . p over all items (Def. 1), exact.
//
// Screening.  A workgroup holds 32 users per wave in LDS and streams the
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

// Users per screening workgroup: 32 per wave, NW waves (4, or 2 when the
// rows are long enough that four waves' users would not fit in LDS).

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

// Screening configuration: nw waves (32 users each), nb item-tile buffers
// in LDS (2 = the next tile loads while the current one is used), pf 16-byte
// vectors of a tile staged per thread (0 = tiles load synchronously).
struct ScreenCfg { int nw, nb, pf; };

size_t thresh_screen_lds_cfg(int prec, int D, int nw, int nb) {
    const int ls = lds_row_bytes(prec, D);
    return (size_t)(32 * nw + nb * TILE_ITEMS) * ls + (size_t)nb * 3 * TILE_ITEMS * 4 +
           32 * nw * sizeof(int) + 16 * sizeof(float);
}

ScreenCfg screen_cfg(int prec, int D) {
    ScreenCfg c{4, 2, 0};
    if (thresh_screen_lds_cfg(prec, D, 4, 2) > 96 * 1024) c.nw = 2;
    if (thresh_screen_lds_cfg(prec, D, c.nw, 2) > 160 * 1024) c.nb = 1;
    const int need = TILE_ITEMS * D * elem_bytes(prec) / 16, nt = 64 * c.nw;
    if (c.nb == 2) c.pf = (need <= 4 * nt) ? 4 : (need <= 8 * nt) ? 8 : 0;
    return c;
}

size_t thresh_screen_lds(int prec, int D) {
    ScreenCfg c = screen_cfg(prec, D);
    return thresh_screen_lds_cfg(prec, D, c.nw, c.nb);
}

// Item tile t (64 rows of D elements, and per item N, Nh, R) into registers,
// then into LDS buffer b; or straight into LDS.
struct TileIO {
    const uint4 *src;   // the tile's rows, 16-byte vectors
    int nvec;           // 16-byte vectors per tile
    int w16;            // 16-byte vectors per row
    int ls;             // LDS row stride (bytes)
};

template <int PFN, int NT>
__device__ __forceinline__ void tile_fetch(uint4 (&pf)[PFN], float (&pn)[3], const ThreshArgs &a,
                                           const TileIO &io, int t, int tid) {
    const uint4 *src = io.src + (int64_t)t * io.nvec;
#pragma unroll
    for (int q = 0; q < PFN; ++q) {
        const int e = tid + q * NT;
        pf[q] = (e < io.nvec) ? src[e] : make_uint4(0, 0, 0, 0);
    }
    if (tid < TILE_ITEMS) {
        const int64_t r = (int64_t)t * TILE_ITEMS + tid;
        pn[0] = a.Np[r];
        pn[1] = a.Nhp[r];
        pn[2] = a.Rp[r];
    }
}

template <int PFN, int NT>
__device__ __forceinline__ void tile_stash(const uint4 (&pf)[PFN], const float (&pn)[3],
                                           uint8_t *Pbase, float *Nbase, int b,
                                           const TileIO &io, int tid) {
#pragma unroll
    for (int q = 0; q < PFN; ++q) {
        const int e = tid + q * NT;
        if (e < io.nvec) {
            const int r = e / io.w16, c = e - r * io.w16;
            *reinterpret_cast<uint4 *>(Pbase + (b * TILE_ITEMS + r) * io.ls + 16 * c) = pf[q];
        }
    }
    if (tid < TILE_ITEMS) {
        float *nb = Nbase + b * 3 * TILE_ITEMS;
        nb[tid] = pn[0];
        nb[TILE_ITEMS + tid] = pn[1];
        nb[2 * TILE_ITEMS + tid] = pn[2];
    }
}

template <int NT>
__device__ __forceinline__ void tile_load(const ThreshArgs &a, const TileIO &io, int t,
                                          uint8_t *Pbase, float *Nbase, int b, int tid) {
    const uint4 *src = io.src + (int64_t)t * io.nvec;
    for (int e = tid; e < io.nvec; e += NT) {
        const int r = e / io.w16, c = e - r * io.w16;
        *reinterpret_cast<uint4 *>(Pbase + (b * TILE_ITEMS + r) * io.ls + 16 * c) = src[e];
    }
    if (tid < TILE_ITEMS) {
        const int64_t r = (int64_t)t * TILE_ITEMS + tid;
        float *nb = Nbase + b * 3 * TILE_ITEMS;
        nb[tid] = a.Np[r];
        nb[TILE_ITEMS + tid] = a.Nhp[r];
        nb[2 * TILE_ITEMS + tid] = a.Rp[r];
    }
}

template <int PREC, int NW, int PF, int NB>
__global__ __launch_bounds__(64 * NW) void k_thresh_screen(ThreshArgs a) {
    constexpr int TU = 32 * NW, NT = 64 * NW;
    extern __shared__ __align__(16) uint8_t smem8[];
    const int D = a.D, ls = lds_row_bytes(PREC, D), rowb = D * elem_bytes(PREC);
    uint8_t *Ush = smem8;
    uint8_t *Pbase = Ush + TU * ls;                                   // item tiles
    float *Nbase = reinterpret_cast<float *>(Pbase + NB * TILE_ITEMS * ls);  // N, Nh, R
    int *cntsh = reinterpret_cast<int *>(Nbase + NB * 3 * TILE_ITEMS);
    float *red = reinterpret_cast<float *>(cntsh + TU);

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t ubase = (int64_t)blockIdx.x * TU;
    const int split = blockIdx.y;
    const int w16 = rowb / 16;

    for (int e = tid; e < TU * w16; e += NT) {
        int r = e / w16, c = e - r * w16;
        int64_t u = ubase + r;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (u < a.n) v = reinterpret_cast<const uint4 *>(a.Uq)[u * w16 + c];
        *reinterpret_cast<uint4 *>(Ush + r * ls + 16 * c) = v;
    }
    if (tid < TU) cntsh[tid] = 0;

    const int ucol = w * 32 + (lane & 31);
    const int64_t ug = ubase + ucol;
    const bool uvalid = ug < a.n;
    const float nu = uvalid ? a.Nu[ug] : 0.0f;
    const float nhu = uvalid ? a.Nhu[ug] : 0.0f;
    const float ru = uvalid ? a.Ru[ug] : 0.0f;
    const float su = uvalid ? a.su[ug] : 1.0f;
    const uint8_t *Bw = Ush + w * 32 * ls;
    const float rmax = __uint_as_float(*a.rmax_bits);

    // error bound of this user against a tile: E(u,p) <= eu(maxN, maxNh, maxR)
    auto ebound = [&](float n_p, float nh_p, float r_p) {
        return fmaf(ru, n_p, fmaf(nhu, r_p, fmaf(a.c_err * nhu, nh_p, fmaf(a.c2 * nu, n_p, a.e_abs))));
    };

    // tile sequence: phase 1 = tiles 0..t0-1, phase 2 = split, split+nsplit, ...
    const int t0 = a.t0tiles < a.ntiles ? a.t0tiles : a.ntiles;
    auto tile_of = [&](int it) { return it < t0 ? it : split + (it - t0) * a.nsplit; };

    TileIO io;
    io.src = reinterpret_cast<const uint4 *>(a.Pq);
    io.w16 = w16;
    io.nvec = TILE_ITEMS * w16;
    io.ls = ls;
    constexpr int PFN = PF > 0 ? PF : 1;
    uint4 pf[PFN];
    float pn[3] = {0.f, 0.f, 0.f};

    float M[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) M[i] = -INFINITY;
    float L0 = -INFINITY, rwg = INFINITY;
    float2 *mycand = a.cand + ((int64_t)ug * a.nsplit + split) * a.cap;
    int64_t ntile_p2 = 0;

    if (PF > 0) {
        tile_fetch<PFN, NT>(pf, pn, a, io, 0, tid);
        tile_stash<PFN, NT>(pf, pn, Pbase, Nbase, 0, io, tid);
    } else {
        tile_load<NT>(a, io, 0, Pbase, Nbase, 0, tid);
    }
    __syncthreads();
    int buf = 0;
    for (int it = 0;; ++it) {
        const int t = tile_of(it);
        if (it >= t0) {
            if (t >= a.ntiles) break;
            if (a.Np[(int64_t)t * TILE_ITEMS] < rwg) break;  // Cauchy-Schwarz exit
            ++ntile_p2;
        }
        const int tn = tile_of(it + 1);
        const bool pre = tn < a.ntiles;
        if (PF > 0 && pre) tile_fetch<PFN, NT>(pf, pn, a, io, tn, tid);
        const uint8_t *Psh = Pbase + buf * TILE_ITEMS * ls;
        const float *Nsh = Nbase + buf * 3 * TILE_ITEMS;
        const int64_t rb = (int64_t)t * TILE_ITEMS;
        // tile maxima: N is sorted (first item), Nh and R from the precomputed arrays
        const float e_t = ebound(Nsh[0], a.tmax_nh[t], a.tmax_r[t]);
        const float sc = su * a.sp[rb];  // product scale of this (user, tile)
        f32x16 acc0 = {0}, acc1 = {0};
        MM<PREC>::rows2(acc0, acc1, Psh, Psh + 32 * ls, Bw, ls, D, lane);
        if (it < t0) {
            // phase 1: per-slot maxima of the lower bounds vh - E
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int r = mfma32_row(i, lane);
                if (rb + r < a.m) M[i] = fmaxf(M[i], fmaf(acc0[i], sc, -e_t));
                if (rb + r + 32 < a.m) M[16 + i] = fmaxf(M[16 + i], fmaf(acc1[i], sc, -e_t));
            }
            if (it == t0 - 1) {
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
                // exit ratio: vh + E <= K_u * N_p + 2 e_abs for every item p
                float rr = INFINITY;
                if (uvalid) {
                    const float K = nu * (1.0f + a.g64 + 2.0f * a.c2) + 2.0f * ru +
                                    2.0f * nhu * (rmax + a.c_err * (1.0f + rmax));
                    rr = (L0 > 2.0f * a.e_abs && K > 0.0f)
                             ? (L0 - 2.0f * a.e_abs) / K * (1.0f - 0x1p-20f)
                             : 0.0f;
                }
                rr = wave_min(rr);
                if (lane == 0) red[w] = rr;
            }
        } else {
            // phase 2: candidates vh + E >= L0, first on the tile bound
            const float thr = (L0 - e_t) / sc;  // exact: sc is a power of two
            bool any = false;
#pragma unroll
            for (int i = 0; i < 16; ++i) any |= (acc0[i] >= thr) | (acc1[i] >= thr);
            if (__ballot(any && uvalid) != 0ull) {
#pragma unroll
                for (int i = 0; i < 32; ++i) {
                    const float v = ((i < 16) ? acc0[i] : acc1[i - 16]) * sc;
                    const int r = mfma32_row(i & 15, lane) + ((i < 16) ? 0 : 32);
                    const bool p = uvalid && ((i < 16) ? acc0[i] : acc1[i - 16]) >= thr &&
                                   rb + r < a.m;
                    if (p) {
                        const float h = v + ebound(Nsh[r], Nsh[TILE_ITEMS + r],
                                                   Nsh[2 * TILE_ITEMS + r]);
                        if (h >= L0) {
                            int s = atomicAdd(&cntsh[ucol], 1);
                            if (s < a.cap)
                                mycand[s] = make_float2(v, __int_as_float((int)(rb + r)));
                        }
                    }
                }
            }
        }
        if (pre) {
            if (NB == 1) {
                __syncthreads();  // every wave is done with the only buffer
                tile_load<NT>(a, io, tn, Pbase, Nbase, 0, tid);
            } else if (PF > 0) {
                tile_stash<PFN, NT>(pf, pn, Pbase, Nbase, buf ^ 1, io, tid);
            } else {
                tile_load<NT>(a, io, tn, Pbase, Nbase, buf ^ 1, tid);
            }
        }
        __syncthreads();
        if (it == t0 - 1) {
            rwg = red[0];
#pragma unroll
            for (int q = 1; q < NW; ++q) rwg = fminf(rwg, red[q]);
        }
        if (NB == 2) buf ^= 1;
    }
    __syncthreads();
    if (tid < TU && ubase + tid < a.n) a.cand_cnt[(ubase + tid) * a.nsplit + split] = cntsh[tid];
    if (a.pairs && tid == 0) {
        // statistics only: pairs of the phase-2 tiles this workgroup screened
        const int64_t nu_valid = (a.n - ubase < TU) ? (a.n - ubase) : TU;
        atomicAdd(a.pairs, (unsigned long long)(ntile_p2 * TILE_ITEMS * nu_valid));
    }
}

// ------------------------------------------------------------------ final
constexpr int FIN_WAVES = 4;

__global__ __launch_bounds__(256) void k_thresh_final(ThreshArgs a, int capT) {
    extern __shared__ float smem[];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int nw = blockDim.x >> 6;  // waves per block (one user each)
    const int64_t u = (int64_t)blockIdx.x * nw + w;
    const bool valid = u < a.n;
    // per-wave LDS: v64[capT] (double), lo, hi (float), cidx, sid (int)
    uint8_t *base = reinterpret_cast<uint8_t *>(smem) + (size_t)w * capT * 24;
    double *v64 = reinterpret_cast<double *>(base);
    float *lo = reinterpret_cast<float *>(base + (size_t)capT * 8);
    float *hi = lo + capT;
    int *cidx = reinterpret_cast<int *>(hi + capT);
    int *sid = cidx + capT;
    __shared__ float Lstar[FIN_WAVES];
    __shared__ int nsurv[FIN_WAVES];

    int total = 0;
    bool over = false;
    if (valid) {
        for (int s = 0; s < a.nsplit; ++s) {
            int c = a.cand_cnt[u * a.nsplit + s];
            over |= c > a.cap;
            total += c;
        }
        if (total > capT) over = true;
        if (lane == 0) a.flag[u] = over ? 1 : 0;
    }
    const bool work = valid && !over;
    const float nu = valid ? a.Nu[u] : 0.0f;
    const float nhu = valid ? a.Nhu[u] : 0.0f;
    const float ru = valid ? a.Ru[u] : 0.0f;
    if (lane == 0) Lstar[w] = -INFINITY;
    if (work) {
        int off = 0;
        for (int s = 0; s < a.nsplit; ++s) {
            const int c = a.cand_cnt[u * a.nsplit + s];
            const float2 *src = a.cand + (u * a.nsplit + s) * a.cap;
            for (int e = lane; e < c; e += 64) {
                float2 cv = src[e];
                int idx = __float_as_int(cv.y);
                const float eb =
                    fmaf(ru, a.Np[idx],
                         fmaf(nhu, a.Rp[idx],
                              fmaf(a.c_err * nhu, a.Nhp[idx], fmaf(a.c2 * nu, a.Np[idx], a.e_abs))));
                lo[off + e] = cv.x - eb;
                hi[off + e] = cv.x + eb;
                cidx[off + e] = idx;
            }
            off += c;
        }
    }
    __syncthreads();
    // L* = k-th largest lower bound (rank by value desc, position asc)
    if (work) {
        for (int e = lane; e < total; e += 64) {
            const float x = lo[e];
            int rank = 0;
            for (int f = 0; f < total; ++f) {
                float y = lo[f];
                rank += (y > x) || (y == x && f < e);
            }
            if (rank == a.k - 1) Lstar[w] = x;
        }
    }
    __syncthreads();
    // survivors: upper bound reaches L*; keep their caller ids
    if (work) {
        const float Ls = Lstar[w];
        int cntw = 0;
        for (int e0 = 0; e0 < total; e0 += 64) {
            const int e = e0 + lane;
            const bool keep = e < total && hi[e] >= Ls;
            const uint64_t bal = __ballot(keep);
            const int pos = cntw + __popcll(bal & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
            if (keep) sid[pos] = a.perm[cidx[e]];
            cntw += __popcll(bal);
        }
        if (lane == 0) nsurv[w] = cntw;
    }
    __syncthreads();
    if (work) {
        const int ns = nsurv[w];
        const float *urow = a.U + u * a.d;
        for (int s = lane; s < ns; s += 64)
            v64[s] = ip64(urow, a.P + (int64_t)sid[s] * a.d, a.d);
    }
    __syncthreads();
    if (work) {
        const int ns = nsurv[w];
        for (int s = lane; s < ns; s += 64) {
            const double x = v64[s];
            const int c = sid[s];
            int rank = 0;
            for (int f = 0; f < ns; ++f) {
                double y = v64[f];
                rank += (y > x) || (y == x && sid[f] < c);
            }
            if (rank == a.k - 1) {
                a.tau[u] = x;
                a.tau_id[u] = c;
            }
            if (a.topk && rank < a.k) a.topk[u * a.k + rank] = c;
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
    for (int64_t u = (int64_t)blockIdx.x * FB_WAVES + w; u < a.n;
         u += (int64_t)gridDim.x * FB_WAVES) {
        if (a.flag[u] == 0) continue;
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
                if (r == k - 1) {
                    a.tau[u] = bv;
                    a.tau_id[u] = bi;
                }
            }
        }
    }
}

void launch_thresh(const ThreshArgs &a, hipStream_t st) {
    const ScreenCfg c = screen_cfg(a.prec, a.D);
    const int tu = 32 * c.nw;
    const size_t lds = thresh_screen_lds_cfg(a.prec, a.D, c.nw, c.nb);
    dim3 g((unsigned)((a.n + tu - 1) / tu), (unsigned)a.nsplit);
    if (a.ev0) (void)hipEventRecord(a.ev0, st);
#define RMIPS_SCREEN(P)                                                                   \
    do {                                                                                  \
        if (c.nw == 4 && c.pf == 4) k_thresh_screen<P, 4, 4, 2><<<g, 256, lds, st>>>(a);  \
        else if (c.nw == 4 && c.pf == 8) k_thresh_screen<P, 4, 8, 2><<<g, 256, lds, st>>>(a); \
        else if (c.nw == 4) k_thresh_screen<P, 4, 0, 2><<<g, 256, lds, st>>>(a);          \
        else if (c.nb == 2 && c.pf == 4) k_thresh_screen<P, 2, 4, 2><<<g, 128, lds, st>>>(a); \
        else if (c.nb == 2 && c.pf == 8) k_thresh_screen<P, 2, 8, 2><<<g, 128, lds, st>>>(a); \
        else if (c.nb == 2) k_thresh_screen<P, 2, 0, 2><<<g, 128, lds, st>>>(a);          \
        else k_thresh_screen<P, 2, 0, 1><<<g, 128, lds, st>>>(a);                         \
    } while (0)
    if (a.prec == PREC_FP32) RMIPS_SCREEN(PREC_FP32);
    else if (a.prec == PREC_BF16) RMIPS_SCREEN(PREC_BF16);
    else RMIPS_SCREEN(PREC_FP8);
#undef RMIPS_SCREEN
    if (a.ev1) (void)hipEventRecord(a.ev1, st);
    const int capT = a.cap * a.nsplit;
    int fw = (int)((150 * 1024) / ((size_t)capT * 24));  // waves whose lists fit in LDS
    fw = fw < 1 ? 1 : (fw > FIN_WAVES ? FIN_WAVES : fw);
    const size_t lds_fin = (size_t)fw * capT * 24;
    k_thresh_final<<<(unsigned)((a.n + fw - 1) / fw), 64 * fw, lds_fin, st>>>(a, capT);
    int64_t fb = (a.n + FB_WAVES - 1) / FB_WAVES;
    if (fb > 1024) fb = 1024;
    k_thresh_fallback<<<(unsigned)fb, 64 * FB_WAVES, 0, st>>>(a);
}

}  // namespace rmips
