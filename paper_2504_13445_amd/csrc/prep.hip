// Preparation kernels: norms, padded copies, gathers into the orders the
// method works in (items by descending norm, Alg. 1 step (1); users by
// pruning ratio), the Gram matrix of the rotation (Alg. 1 step (2)) and the
// rotated, augmented rows of the Eq. (3) bound.
#include "common.h"
#include "kernels.h"

namespace rmips {

// One wave per row: coalesced loads, FP64 sum of squares.
__global__ __launch_bounds__(256) void k_rows_prep(const float *__restrict__ X, int64_t rows,
                                                   int d, int D, float *__restrict__ Xpad,
                                                   float *__restrict__ norm,
                                                   uint32_t *__restrict__ key,
                                                   int32_t *__restrict__ val,
                                                   int *__restrict__ flag) {
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= rows) return;
    const float *x = X + r * d;
    double s = 0.0;
    bool bad = false;
    for (int i = lane; i < D; i += 64) {
        float v = (i < d) ? x[i] : 0.0f;
        if (!isfinite(v)) bad = true;
        s += (double)v * (double)v;
        if (Xpad) Xpad[r * D + i] = v;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (__ballot(bad) != 0ull && lane == 0) *flag = 1;
    if (lane == 0) {
        // the FP64 sum and sqrt are within 1e-13 relative of ||x||; the
        // factor and the upward conversion make the FP32 value an upper bound
        float nf = __double2float_ru(sqrt(s) * (1.0 + 0x1p-40));
        if (!(nf <= 0x1p60f)) *flag = 1;
        norm[r] = nf;
        if (key) {
            key[r] = ~__float_as_uint(nf);
            val[r] = (int32_t)r;
        }
    }
}

void launch_rows_prep(const float *X, int64_t rows, int d, int D, float *Xpad, float *norm,
                      uint32_t *key, int32_t *val, int *flag, hipStream_t st) {
    if (rows <= 0) return;
    RMIPS_PROF(st, "k_rows_prep");
    k_rows_prep<<<(unsigned)((rows + 3) / 4), 256, 0, st>>>(X, rows, d, D, Xpad, norm, key,
                                                            val, flag);
}

// Padded, quantized copy of rows, 64 rows per block (wave w takes rows w,
// w+4, ...).  Row r of the output is row order[r] of X (identity if NULL);
// rows past `rows` are zero.  Rows of a group share one power-of-two scale
// s (FP8: the smallest with max |x_i| / s <= 448, but at least 2^-63 so
// that 1/s and the product of two scales' reciprocals stay finite; FP32
// and BF16: 1).  Per row: N = ||x||, Nh = ||xq||, R = ||x - xq|| (FP64
// sums, rounded up to FP32), sc = s; the largest R/N of the rows goes to
// *rmax (a monotone atomic maximum of non-negative floats).
//
// Subnormal operands: the matrix cores may flush them to zero, so the
// copy never holds one.  An FP32 or BF16 value below 2^-126 in magnitude,
// and an e4m3 code in the format's subnormal range (scaled magnitude below
// 2^-6), is stored as zero and its whole value counts in R.  The error
// bound, which takes the quantisation error from R by Cauchy-Schwarz, then
// holds whatever the hardware does with subnormal inputs.  FP6 e2m3 and
// FP4 e2m1 keep their subnormal codes (values below 1 before scaling, a
// large part of a row with two exponent bits): the f8f6f4 instruction
// decodes every code of both formats exactly on gfx950 (measured over all
// codes, no difference from the decoded products).
template <int PREC>
__global__ __launch_bounds__(256) void k_quant(const float *__restrict__ X,
                                               const int32_t *__restrict__ order, int64_t rows,
                                               int64_t rows_pad, int d, int D, int group,
                                               uint8_t *__restrict__ Xq, float *__restrict__ N,
                                               float *__restrict__ Nh, float *__restrict__ R,
                                               float *__restrict__ sc,
                                               unsigned int *__restrict__ rmax,
                                               int *__restrict__ flag) {
    // 64 rows per block, 16 per wave; a row's values (D <= 256: at most 4
    // per lane) stay in registers between the two passes
    __shared__ float rowmax[64];
    __shared__ float rmx[4];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t r0 = (int64_t)blockIdx.x * 64;
    // the source rows of the wave's 16 rows, all requested before the first
    // is used (-1: past the end)
    // (lane j < 16 loads the entry of row j; one load for all)
    int64_t src[16];
    {
        const int64_t rl = r0 + w + 4 * (lane & 15);
        const int32_t ol = (order && lane < 16 && rl < rows) ? order[rl] : (int32_t)rl;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int64_t r = r0 + w + 4 * j;
            src[j] = (r < rows) ? (int64_t)__builtin_amdgcn_readlane(ol, j) : -1;
        }
    }
    float v[16][4];
    float mx[16];
    bool bad = false;
    // pass 1: load, finiteness, max |x_i| per row
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const float *x = (src[j] >= 0) ? X + src[j] * d : nullptr;
        mx[j] = 0.0f;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = lane + 64 * q;
            const float t = (x && c < d) ? x[c] : 0.0f;
            v[j][q] = t;
            bad |= !isfinite(t);
            mx[j] = fmaxf(mx[j], fabsf(t));
        }
    }
    if (__ballot(bad) != 0ull && lane == 0) *flag = 1;
    if (scaled_prec(PREC)) {
        // the 16 row maxima reduced together (a maximum in any order)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1)
#pragma unroll
            for (int j = 0; j < 16; ++j) mx[j] = fmaxf(mx[j], __shfl_xor(mx[j], o));
        if (lane == 0)
#pragma unroll
            for (int j = 0; j < 16; ++j) rowmax[w + 4 * j] = mx[j];
        __syncthreads();
    }
    // pass 2: quantize with the group's scale, residual sums in FP64; four
    // rows at a time, whose lane sums are reduced together (each row's sums
    // in the same order as alone)
    float rrmax = 0.0f;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        double sx[4], sq[4], sr[4];
        float sc4[4];
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int j = 4 * g + jj;
            const int i = w + 4 * j;
            const int64_t r = r0 + i;
            float s = 1.0f;
            if (scaled_prec(PREC)) {
                const int g0 = (i / group) * group;
                float m = 0.0f;
                for (int t = g0; t < g0 + group && t < 64; ++t) m = fmaxf(m, rowmax[t]);
                if (m > 0.0f) {
                    // smallest power of two s with m / s <= the format's largest value
                    constexpr float FMAX = mx_max(PREC);
                    int e;
                    frexpf(m / FMAX, &e);  // m/FMAX = f * 2^e, f in [0.5, 1)
                    s = ldexpf(1.0f, e);
                    if (m / ldexpf(1.0f, e - 1) <= FMAX) s = ldexpf(1.0f, e - 1);
                    s = fmaxf(s, 0x1p-63f);
                }
            }
            sc4[jj] = s;
            const float inv = 1.0f / s;  // exact: s is a power of two
            sx[jj] = 0.0;
            sq[jj] = 0.0;
            sr[jj] = 0.0;
            const bool live = r < rows_pad;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int c = lane + 64 * q;
                if (c < D) {
                    const float t = v[j][q];
                    float qv;
                    // (values below 2^-126 are zero in the copy)
                    const bool sub = fabsf(t) < 0x1p-126f;
                    if (PREC == PREC_FP32) {
                        qv = sub ? 0.0f : t;
                        if (live) reinterpret_cast<float *>(Xq)[r * D + fp32_slot(c, d, D)] = qv;
                    } else if (PREC == PREC_BF16) {
                        uint16_t h = to_bf16(t, qv);
                        if (sub) {
                            h = 0;
                            qv = 0.0f;
                        }
                        if (live) reinterpret_cast<uint16_t *>(Xq)[r * D + c] = h;
                    } else if (PREC == PREC_FP8) {
                        float yq;
                        uint8_t b8 = to_e4m3(t * inv, yq);
                        if ((b8 & 0x78u) == 0u) {  // zero or an e4m3 subnormal code
                            b8 = 0;
                            yq = 0.0f;
                        }
                        if (live) Xq[r * D + c] = b8;
                        qv = yq * s;
                    } else {
                        // FP6 / FP4: the 32 codes of a block (held by 32
                        // consecutive lanes) packed from the slot's first
                        // bit, code e at bits [B e, B e + B); lane e < B of
                        // the block assembles dword e from the codes that
                        // reach into it, lanes B..7 write the slot's zero
                        // dwords
                        float yq;
                        const uint32_t code = (PREC == PREC_FP6) ? to_e2m<3>(t * inv, yq)
                                                                 : to_e2m<1>(t * inv, yq);
                        qv = yq * s;
                        constexpr int B = mx_bits(PREC);
                        const int e = lane & 31, base = lane & 32;
                        const int wsel = (e < B) ? e : 0;
                        const int t0 = (32 * wsel) / B;
                        uint32_t word = 0u;
#pragma unroll
                        for (int k = 0; k < 32 / B + 2; ++k) {
                            const int tk = t0 + k;
                            const uint32_t ck = __shfl(code, base + (tk < 32 ? tk : 31));
                            const int sh = B * tk - 32 * wsel;
                            if (tk < 32 && sh > -B && sh < 32)
                                word |= (sh >= 0) ? (ck << sh) : (ck >> (-sh));
                        }
                        if (live && e < 8)
                            reinterpret_cast<uint32_t *>(Xq + r * D + (c - e))[e] =
                                (e < B) ? word : 0u;
                    }
                    sx[jj] += (double)t * (double)t;
                    sq[jj] += (double)qv * (double)qv;
                    const double df = (double)t - (double)qv;  // exact: both are FP32
                    sr[jj] += df * df;
                }
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1)
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                sx[jj] += __shfl_xor(sx[jj], o);
                sq[jj] += __shfl_xor(sq[jj], o);
                sr[jj] += __shfl_xor(sr[jj], o);
            }
        if (lane == 0) {
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                const int64_t r = r0 + w + 4 * (4 * g + jj);
                if (r >= rows_pad) continue;
                const double up = 1.0 + 0x1p-40;
                const float nx = __double2float_ru(sqrt(sx[jj]) * up);
                // (FP32: R is zero unless the row holds subnormal values)
                const float rr = __double2float_ru(sqrt(sr[jj]) * up);
                if (!(nx <= 0x1p60f)) *flag = 1;
                N[r] = nx;
                Nh[r] = __double2float_ru(sqrt(sq[jj]) * up);
                R[r] = rr;
                sc[r] = sc4[jj];
                if (nx > 0.0f && rr > 0.0f)
                    rrmax = fmaxf(rrmax, __double2float_ru((double)rr / (double)nx));
            }
        }
    }
    // largest R / N of the block, one atomic per block (non-negative floats
    // order like their bit patterns)
    if (rmax) {
        if (lane == 0) rmx[w] = rrmax;
        __syncthreads();
        if (threadIdx.x == 0) {
            const float m = fmaxf(fmaxf(rmx[0], rmx[1]), fmaxf(rmx[2], rmx[3]));
            if (m > 0.0f) atomicMax(rmax, __float_as_uint(m));
        }
    }
}

void launch_quant(int prec, const float *X, const int32_t *order, int64_t rows,
                  int64_t rows_pad, int d, int D, int group, void *Xq, float *N, float *Nh,
                  float *R, float *sc, unsigned int *rmax, int *flag, hipStream_t st) {
    const unsigned g = (unsigned)((rows_pad + 63) / 64);
    uint8_t *q = reinterpret_cast<uint8_t *>(Xq);
    RMIPS_PROF(st, "k_quant");
    if (prec == PREC_FP32)
        k_quant<PREC_FP32><<<g, 256, 0, st>>>(X, order, rows, rows_pad, d, D, group, q, N, Nh, R,
                                              sc, rmax, flag);
    else if (prec == PREC_BF16)
        k_quant<PREC_BF16><<<g, 256, 0, st>>>(X, order, rows, rows_pad, d, D, group, q, N, Nh, R,
                                              sc, rmax, flag);
    else if (prec == PREC_FP8)
        k_quant<PREC_FP8><<<g, 256, 0, st>>>(X, order, rows, rows_pad, d, D, group, q, N, Nh, R,
                                             sc, rmax, flag);
    else if (prec == PREC_FP6)
        k_quant<PREC_FP6><<<g, 256, 0, st>>>(X, order, rows, rows_pad, d, D, group, q, N, Nh, R,
                                             sc, rmax, flag);
    else
        k_quant<PREC_FP4><<<g, 256, 0, st>>>(X, order, rows, rows_pad, d, D, group, q, N, Nh, R,
                                             sc, rmax, flag);
}

__global__ void k_tile_max(const float *__restrict__ Nh, const float *__restrict__ R, int ntiles,
                           float *__restrict__ tnh, float *__restrict__ tr) {
    const int lane = threadIdx.x & 63;
    const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (t >= ntiles) return;
    float a = Nh[(int64_t)t * 64 + lane], b = R[(int64_t)t * 64 + lane];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a = fmaxf(a, __shfl_xor(a, o));
        b = fmaxf(b, __shfl_xor(b, o));
    }
    if (lane == 0) {
        tnh[t] = a;
        tr[t] = b;
    }
}

void launch_tile_max(const float *Nh, const float *R, int ntiles, float *tmax_nh, float *tmax_r,
                     hipStream_t st) {
    RMIPS_PROF(st, "k_tile_max");
    k_tile_max<<<(unsigned)((ntiles + 3) / 4), 256, 0, st>>>(Nh, R, ntiles, tmax_nh, tmax_r);
}

__global__ void k_gather_rows(const float *__restrict__ P, const int32_t *__restrict__ perm,
                              const float *__restrict__ nb_id, int64_t m, int64_t rows_pad,
                              int d, int D, float *__restrict__ Pk, float *__restrict__ Np) {
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= rows_pad) return;
    if (r < m) {
        const int64_t src = perm[r];
        for (int i = lane; i < D; i += 64) Pk[r * D + i] = (i < d) ? P[src * d + i] : 0.0f;
        if (lane == 0) Np[r] = nb_id[src];
    } else {
        for (int i = lane; i < D; i += 64) Pk[r * D + i] = 0.0f;
        if (lane == 0) Np[r] = 0.0f;
    }
}

void launch_gather_rows(const float *P, const int32_t *perm, const float *norm_by_id,
                        int64_t m, int64_t rows_pad, int d, int D, float *Pk, float *Np,
                        hipStream_t st) {
    RMIPS_PROF(st, "k_gather_rows");
    k_gather_rows<<<(unsigned)((rows_pad + 3) / 4), 256, 0, st>>>(P, perm, norm_by_id, m,
                                                                  rows_pad, d, D, Pk, Np);
}

__global__ void k_invert_perm(const int32_t *__restrict__ perm, int64_t m,
                              int32_t *__restrict__ inv) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < m) inv[perm[r]] = (int32_t)r;
}

void launch_invert_perm(const int32_t *perm, int64_t m, int32_t *inv, hipStream_t st) {
    RMIPS_PROF(st, "k_invert_perm");
    k_invert_perm<<<(unsigned)((m + 255) / 256), 256, 0, st>>>(perm, m, inv);
}

__global__ void k_user_side(const double *__restrict__ tau, const int32_t *__restrict__ tau_id,
                            const float *__restrict__ Nu, const float *__restrict__ Nhu,
                            const float *__restrict__ Ru, const float *__restrict__ su,
                            const int32_t *__restrict__ order, int64_t n, float c2,
                            UserSide out) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    int64_t u = order ? order[r] : r;
    double t = tau[u];
    out.N[r] = Nu[u];
    out.Nh[r] = Nhu[u];
    out.R[r] = Ru[u];
    out.sinv[r] = 1.0f / su[u];  // exact: su is a power of two
    out.tau_hi[r] = __double2float_ru(t);
    out.tau_lo[r] = __double2float_rd(t);
    out.tau[r] = t;
    out.tau_id[r] = tau_id[u];
    out.uid[r] = (int32_t)u;
    out.thr[r] = make_float4(__double2float_ru(t), __double2float_rd(t), fmaf(c2, Nu[u], Ru[u]),
                             Nhu[u]);
}

void launch_user_side(const double *tau, const int32_t *tau_id, const float *Nu,
                      const float *Nhu, const float *Ru, const float *su,
                      const int32_t *order, int64_t n, float c2, UserSide out, hipStream_t st) {
    RMIPS_PROF(st, "k_user_side");
    k_user_side<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(tau, tau_id, Nu, Nhu, Ru, su, order,
                                                             n, c2, out);
}

// tau[u] = topv[u][k - 1], tau_id[u] = topk[u][k - 1]: the threshold of
// S_k(u) from the user's list of its kmax largest values (kmax >= k).
__global__ void k_kth_column(const double *__restrict__ topv, const int32_t *__restrict__ topk,
                             int64_t n, int kmax, int k, double *__restrict__ tau,
                             int32_t *__restrict__ tau_id) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    tau[u] = topv[u * kmax + (k - 1)];
    tau_id[u] = topk[u * kmax + (k - 1)];
}

void launch_kth_column(const double *topv, const int32_t *topk, int64_t n, int kmax, int k,
                       double *tau, int32_t *tau_id, hipStream_t st) {
    RMIPS_PROF(st, "k_kth_column");
    k_kth_column<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(topv, topk, n, kmax, k, tau,
                                                               tau_id);
}

__global__ void k_rho_keys(const double *__restrict__ tau, const float *__restrict__ Nu,
                           int64_t n, uint32_t *__restrict__ key, int32_t *__restrict__ val) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    double t = tau[u];
    float nu = Nu[u];
    float rho = -INFINITY;
    // a user with tau <= 0 (or a zero vector) can hold any item: ratio -inf
    if (t > 0.0 && nu > 0.0f) rho = __double2float_rd(t / (double)nu);
    key[u] = float_key(rho);
    val[u] = (int32_t)u;
}

void launch_rho_keys(const double *tau, const float *Nu, int64_t n, uint32_t *key,
                     int32_t *val, hipStream_t st) {
    RMIPS_PROF(st, "k_rho_keys");
    k_rho_keys<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(tau, Nu, n, key, val);
}

__global__ void k_gather_padded(const uint4 *__restrict__ X, const int32_t *__restrict__ order,
                                int64_t rows, int W16, uint4 *__restrict__ Y) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * W16) return;
    int64_t r = e / W16, c = e - r * W16;
    Y[e] = X[(int64_t)order[r] * W16 + c];
}

// Ys[r] = Xs[order[r]], rows of row_bytes (a multiple of 16)
void launch_gather_padded(const void *X, const int32_t *order, int64_t rows, int row_bytes,
                          void *Y, hipStream_t st) {
    const int W16 = row_bytes / 16;
    int64_t tot = rows * W16;
    RMIPS_PROF(st, "k_gather_padded");
    k_gather_padded<<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(
        reinterpret_cast<const uint4 *>(X), order, rows, W16, reinterpret_cast<uint4 *>(Y));
}

// The keys are ordered by their bits from lo_bit up only: the prefix then
// takes every user whose key agrees with the item's in those bits or is
// below, a superset of the users of Eq. (2) (ratios up to 2^(lo_bit-23)
// relative above the item's norm also come in).
__global__ void k_cs_prefix(const uint32_t *__restrict__ keys, int64_t n,
                            const float *__restrict__ norm, int64_t m, int lo_bit,
                            int32_t *__restrict__ cs) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    // v <= (1 + d 2^-53) ||u|| ||p|| for the exact value; 2^-18 covers that
    // and the FP32 rounding of this product
    const uint32_t x = float_key(norm[j] * (1.0f + 0x1p-18f)) >> lo_bit;
    int64_t lo = 0, hi = n;  // first position with a larger key
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if ((keys[mid] >> lo_bit) <= x) lo = mid + 1; else hi = mid;
    }
    cs[j] = (int32_t)lo;
}

void launch_cs_prefix(const uint32_t *rho_sorted_keys, int64_t n, const float *norm,
                      int64_t m, int lo_bit, int32_t *cs, hipStream_t st) {
    RMIPS_PROF(st, "k_cs_prefix");
    k_cs_prefix<<<(unsigned)((m + 255) / 256), 256, 0, st>>>(rho_sorted_keys, n, norm, m, lo_bit,
                                                             cs);
}

// 32x32 tile of G per block over one slice of the sampled rows (blockIdx.z),
// staged through LDS; slices are summed afterwards in a fixed order.
constexpr int GRAM_SLICES = 64;

__global__ __launch_bounds__(256) void k_gram(const float *__restrict__ X, int64_t ns,
                                              int64_t stride, int d, double *__restrict__ Gp) {
    __shared__ float xa[64][33];
    __shared__ float xb[64][33];
    const int i0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
    const int t = threadIdx.x, ti = t & 31, tj = t >> 5;  // tj in [0, 8)
    const int64_t per = (ns + GRAM_SLICES - 1) / GRAM_SLICES;
    const int64_t sb = (int64_t)blockIdx.z * per;
    const int64_t se = (sb + per < ns) ? sb + per : ns;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t s0 = sb; s0 < se; s0 += 64) {
        for (int e = t; e < 64 * 32; e += 256) {
            int rr = e >> 5, cc = e & 31;
            int64_t s = s0 + rr;
            float va = 0.f, vb = 0.f;
            if (s < se) {
                const float *x = X + s * stride * d;
                if (i0 + cc < d) va = x[i0 + cc];
                if (j0 + cc < d) vb = x[j0 + cc];
            }
            xa[rr][cc] = va;
            xb[rr][cc] = vb;
        }
        __syncthreads();
        for (int rr = 0; rr < 64; ++rr) {
            double a = xa[rr][ti];
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] += a * (double)xb[rr][tj + 8 * q];
        }
        __syncthreads();
    }
    double *G = Gp + (int64_t)blockIdx.z * d * d;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        int i = i0 + ti, j = j0 + tj + 8 * q;
        if (i < d && j < d) G[(int64_t)i * d + j] = acc[q];
    }
}

__global__ void k_gram_sum(const double *__restrict__ Gp, int dd, double *__restrict__ G) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= dd) return;
    double s = 0.0;
    for (int z = 0; z < GRAM_SLICES; ++z) s += Gp[(int64_t)z * dd + e];
    G[e] = s;
}

size_t gram_scratch_bytes(int d) { return (size_t)GRAM_SLICES * d * d * sizeof(double); }

void launch_gram(const float *X, int64_t ns, int64_t stride, int d, double *G, double *scratch,
                 hipStream_t st) {
    dim3 g((d + 31) / 32, (d + 31) / 32, GRAM_SLICES);
    {
        RMIPS_PROF(st, "k_gram");
        k_gram<<<g, 256, 0, st>>>(X, ns, stride, d, scratch);
    }
    RMIPS_PROF(st, "k_gram_sum");
    k_gram_sum<<<(d * d + 255) / 256, 256, 0, st>>>(scratch, d * d, G);
}

// Augmented rows of the Eq. (3) bound, one thread per row over a
// persistent grid: y = W x in FP64 with W (dp x d, FP64, orthonormal rows)
// on the FP64 matrix cores; ||x||^2 in FP64.  Row layout: a = [y (dp values,
// rounded to FP32), tail(x), scale * ||x||, 0...] (ka values, a multiple of
// 16), stored as BF16 rn(a) (2 ka bytes).  tail(x) = sqrt(||x||^2 -
// ||W x||^2), rounded up and widened
// by 1e-12 ||x||^2 under the root for the FP64 rounding (in any summation
// order) and the departure of W from exact orthonormality.
//
// Each wave projects 16 rows at a time onto the 64 output columns (zero past
// dp) with v_mfma_f64_16x16x4_f64, four column tiles of 16 per step of 4
// terms.  Operand layout of that instruction: lane l feeds row l % 16 of A
// and column l % 16 of B at k-slot l / 16, and holds result rows
// l / 16 + 4 i (i = 0..3) of column l % 16.  k-slot g of a step s takes term
// g * Kq + s (Kq = ceil(d / 4)), so each lane reads one contiguous quarter of
// its row.  W is staged once per workgroup in LDS in the same order:
// Wt[(s * 4 + g) * 64 + j] = W[j][g * Kq + s].
constexpr int DP_MAX = 62;
constexpr int KA_MAX = 64;
constexpr int ROT_WAVES = 8;
typedef double d4_t __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(64 * ROT_WAVES) __attribute__((amdgpu_waves_per_eu(2)))
void k_rotate_aug(const float *__restrict__ X, const int32_t *__restrict__ order, int64_t rows,
                  int64_t rows_pad, int d, const double *__restrict__ W, int dp, int ka,
                  float scale, uint4 *__restrict__ out) {
    extern __shared__ double Wt[];
    const int Kq = (d + 3) / 4;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, c16 = lane & 15;
    for (int e = threadIdx.x; e < 4 * Kq * 64; e += blockDim.x) {
        const int ri = e >> 6, j = e & 63, k = (ri & 3) * Kq + (ri >> 2);
        Wt[e] = (j < dp && k < d) ? W[(int64_t)j * d + k] : 0.0;
    }
    __syncthreads();
    uint16_t *o16 = reinterpret_cast<uint16_t *>(out);
    const int64_t rstride = (int64_t)gridDim.x * ROT_WAVES * 16;
    for (int64_t r0 = ((int64_t)blockIdx.x * ROT_WAVES + w) * 16; r0 < rows_pad; r0 += rstride) {
        // A operand: row r0 + c16, terms g * Kq .. g * Kq + Kq - 1 (zero past
        // d and for padding rows), in blocks of 16 terms, the next block
        // loaded while the current one is multiplied
        const int64_t ra = r0 + c16;
        const bool live = ra < rows;
        const float *x = X + (int64_t)(live ? (order ? order[ra] : ra) : 0) * d;
        // (unconditional loads of indexes clamped into the row, so that none
        // waits for another; values past d and of padding rows are zero)
        auto load16 = [&](float (&v)[16], int q0) {
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int k = g * Kq + q0 + j;
                const bool ok = live && q0 + j < Kq && k < d;
                const float t = x[ok ? k : 0];
                v[j] = ok ? t : 0.0f;
            }
        };
        double s = 0.0;
        d4_t acc[4] = {};
        float xa[16], xb[16];
        load16(xa, 0);
        for (int q0 = 0; q0 < Kq; q0 += 16) {
            if (q0 + 16 < Kq) load16(xb, q0 + 16);  // (uniform)
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                if (q0 + j < Kq) {  // (uniform)
                    const double a = (double)xa[j];
                    s = fma(a, a, s);
                    const double *wr = Wt + ((q0 + j) * 4 + g) * 64 + c16;
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, wr[16 * t], acc[t], 0, 0,
                                                                       0);
                }
            }
#pragma unroll
            for (int j = 0; j < 16; ++j) xa[j] = xb[j];
        }
        // ||x||^2 of row c16 over the four k-slots, then of this lane's result
        // rows g + 4 i (held by lane g + 4 i)
        s += __shfl_xor(s, 16);
        s += __shfl_xor(s, 32);
        double y2[4], sr[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            double v = 0.0;
#pragma unroll
            for (int t = 0; t < 4; ++t) v = fma(acc[t][i], acc[t][i], v);
            y2[i] = v;
            sr[i] = __shfl(s, g + 4 * i);
        }
#pragma unroll
        for (int o = 1; o < 16; o <<= 1)
#pragma unroll
            for (int i = 0; i < 4; ++i) y2[i] += __shfl_xor(y2[i], o);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t R = r0 + g + 4 * i;
            if (R >= rows_pad) continue;
            double t2 = sr[i] - y2[i];
            if (t2 < 0.0) t2 = 0.0;
            const float tail = __double2float_ru(sqrt(t2 + 1e-12 * sr[i]));
            const float nrm = scale * __double2float_ru(sqrt(sr[i]) * (1.0 + 0x1p-40));
            uint16_t *orow = o16 + R * ka;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int C = 16 * t + c16;
                if (C >= ka) continue;
                float v = (C < dp) ? (float)acc[t][i] : 0.0f;
                v = (C == dp) ? tail : v;
                v = (C == dp + 1) ? nrm : v;
                float h;
                orow[C] = to_bf16(v, h);
            }
        }
    }
}

// The same rows when W is the identity (dp = d <= 256, ka <= 288): y = x
// exactly, and ||W x||^2 is the same FP64 sum as ||x||^2, so the tail is the
// widening alone.  Up to the FP64 summation order of the norm (both rounded
// up) these are the rows k_rotate_aug gives with W = I.  One wave per row:
// lane j holds values 8j .. 8j + 7 of the augmented row and writes its
// 16-byte word j (at most 36 words).
constexpr int AUG_ROWS = 4;  // rows (waves) per workgroup
__global__ __launch_bounds__(64 * AUG_ROWS) void k_aug_ident(const float *__restrict__ X,
                                                            const int32_t *__restrict__ order,
                                                            int64_t rows, int64_t rows_pad, int d,
                                                            int ka, float scale,
                                                            uint4 *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * AUG_ROWS + (threadIdx.x >> 6);
    if (r >= rows_pad) return;
    const int kw = ka / 8;
    uint4 *o = out + r * kw;
    if (r >= rows) {
        if (lane < kw) o[lane] = make_uint4(0, 0, 0, 0);
        return;
    }
    const float *x = X + (int64_t)(order ? order[r] : r) * d;
    float v[8];
    if ((d & 3) == 0 && (reinterpret_cast<uintptr_t>(x) & 15) == 0) {  // 16-byte vectors: two loads per lane
        const float4 *x4 = reinterpret_cast<const float4 *>(x);
        const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
        const float4 y0 = 8 * lane < d ? x4[2 * lane] : z;
        const float4 y1 = 8 * lane + 4 < d ? x4[2 * lane + 1] : z;
        v[0] = y0.x; v[1] = y0.y; v[2] = y0.z; v[3] = y0.w;
        v[4] = y1.x; v[5] = y1.y; v[6] = y1.z; v[7] = y1.w;
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = 8 * lane + e < d ? x[8 * lane + e] : 0.0f;
    }
    double s = 0.0;
#pragma unroll
    for (int e = 0; e < 8; ++e) s = fma((double)v[e], (double)v[e], s);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    const float tail = __double2float_ru(sqrt(0.0 + 1e-12 * s));
    const float nrm = scale * __double2float_ru(sqrt(s) * (1.0 + 0x1p-40));
    if (lane >= kw) return;
    uint32_t hw[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        uint16_t b[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int c = 8 * lane + 2 * e + h;
            float y = v[2 * e + h];
            y = (c == d) ? tail : y;
            y = (c == d + 1) ? nrm : y;
            float q;
            b[h] = to_bf16(y, q);
        }
        hw[e] = (uint32_t)b[0] | ((uint32_t)b[1] << 16);
    }
    o[lane] = make_uint4(hw[0], hw[1], hw[2], hw[3]);
}

size_t rotate_lds_bytes(int d) { return (size_t)4 * ((d + 3) / 4) * 64 * sizeof(double); }

void launch_rotate_aug(const float *X, const int32_t *order, int64_t rows, int64_t rows_pad,
                       int d, const double *W, int dp, int ka, float scale, uint4 *out,
                       hipStream_t st) {
    if (W == nullptr) {  // the identity, dp = d
        RMIPS_PROF(st, "k_aug_ident");
        k_aug_ident<<<(unsigned)((rows_pad + AUG_ROWS - 1) / AUG_ROWS), 64 * AUG_ROWS, 0, st>>>(
            X, order, rows, rows_pad, d, ka, scale, out);
        return;
    }
    // persistent: W is staged once per workgroup, one workgroup per compute
    // unit (its LDS), 16 rows per wave at a time
    int64_t g = (rows_pad + 16 * ROT_WAVES - 1) / (16 * ROT_WAVES);
    if (g > 256) g = 256;
    RMIPS_PROF(st, "k_rotate_aug");
    k_rotate_aug<<<(unsigned)g, 64 * ROT_WAVES, rotate_lds_bytes(d), st>>>(
        X, order, rows, rows_pad, d, W, dp, ka, scale, out);
}

}  // namespace rmips
