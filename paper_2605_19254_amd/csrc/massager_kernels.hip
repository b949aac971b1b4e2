// Local Smith forms with transforms on the GPU (Section 2.2, Phase 2, item 2:
// the modular Smith form of the n x t projection P_1 over Z/sZ, for the
// massager's batches whose modulus s fits a machine word).
//
// s is split into prime powers m_f = q_f^e_f on the host; plane f holds
// W_f = P_1 mod m_f (n x t), its row transform E_f (n x n) and column
// transform R_f (t x t), the latter stored transposed (row j of the buffer
// is column j of R_f), so that the column operations of the elimination
// read and write contiguous rows.  Step c takes, in every plane at once, an entry of
// minimal q-adic valuation v in rows >= c and columns >= c (a global minimum
// of keys (v, row, column)), exchanges it to (c, c), and clears column c below
// it and row c right of it; v is minimal, so the pivot divides every entry it
// clears and the diagonal comes out in order of valuation, i.e. in
// divisibility order.  Then E_f P_1 R_f = diag(q^v_0 u_0, q^v_1 u_1, ...) with
// units u_c, which the host combines over the planes by the CRT.
//
// Arithmetic: odd m in Montgomery form (R = 2^64; every value < m < 2^62), a
// power of two by masking; exact division by q^v through the inverse of q
// modulo 2^64 (odd q) or a shift.
#include "smith_internal.hpp"

namespace rns {
namespace {

__device__ __forceinline__ uint64_t ls_mul(const LsnfPlane &P, uint64_t a, uint64_t b) {
    if (P.pow2) return (a * b) & (P.m - 1);
    const uint64_t lo = a * b, hi = __umul64hi(a, b);
    const uint64_t u = lo * P.minv;                      // lo + u m = 0 (mod 2^64)
    const uint64_t r = hi + __umul64hi(u, P.m) + (lo != 0 ? 1 : 0);
    return r >= P.m ? r - P.m : r;
}
__device__ __forceinline__ uint64_t ls_sub(const LsnfPlane &P, uint64_t a, uint64_t b) {
    return a >= b ? a - b : a + P.m - b;
}
__device__ __forceinline__ uint64_t ls_add(const LsnfPlane &P, uint64_t a, uint64_t b) {
    const uint64_t r = a + b;
    return r >= P.m ? r - P.m : r;
}
// q-adic valuation of x in [0, m), e for x = 0.
__device__ __forceinline__ int ls_val(const LsnfPlane &P, uint64_t x) {
    if (x == 0) return P.e;
    if (P.pow2) return min(__ffsll((long long)x) - 1, P.e);
    int v = 0;
    while (v < P.e && x * P.qinv <= P.qmax) {
        x *= P.qinv;
        ++v;
    }
    return v;
}
// x / q^v for q^v dividing x.
__device__ __forceinline__ uint64_t ls_divq(const LsnfPlane &P, uint64_t x, int v) {
    if (P.pow2) return x >> v;
    for (int i = 0; i < v; ++i) x *= P.qinv;
    return x;
}
__device__ __forceinline__ uint64_t ls_mulmod(uint64_t a, uint64_t b, uint64_t m) {
    return (uint64_t)((unsigned __int128)a * b % m);
}
// a^-1 mod m for a prime to m (extended Euclid, signed 128-bit cofactors).
__device__ uint64_t ls_inv(uint64_t a, uint64_t m) {
    if (m == 1) return 0;
    __int128 r0 = m, r1 = a % m, t0 = 0, t1 = 1;
    while (r1) {
        const __int128 q = r0 / r1;
        __int128 x = r0 - q * r1;
        r0 = r1;
        r1 = x;
        x = t0 - q * t1;
        t0 = t1;
        t1 = x;
    }
    if (t0 < 0) t0 += m;
    return (uint64_t)t0;
}

constexpr uint64_t kKeyNone = ~0ull;

// W_f = P mod m_f (Montgomery form for odd m), Pf = P mod m_f (plain, kept
// for P R), E_f = I, R_f = I; the step records cleared.
__global__ __launch_bounds__(256) void k_ls_load(const uint64_t *__restrict__ P, int64_t n, int64_t t,
                                                 const LsnfPlane *__restrict__ pl, uint64_t *__restrict__ W,
                                                 uint64_t *__restrict__ Pf, uint64_t *__restrict__ E,
                                                 uint64_t *__restrict__ R, LsnfStep *__restrict__ st) {
    const int f = blockIdx.y;
    const LsnfPlane P0 = pl[f];
    const int64_t nt = n * t, nn = n * n, tt = t * t;
    const uint64_t one = ls_mul(P0, 1, P0.r2);
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < nt + nn + tt; k += (int64_t)gridDim.x * 256) {
        if (k < nt) {
            const uint64_t x = P[k] % P0.m;
            Pf[f * nt + k] = x;
            W[f * nt + k] = ls_mul(P0, x, P0.r2);
        } else if (k < nt + nn) {
            const int64_t e = k - nt;
            E[f * nn + e] = (e / n == e % n) ? one : 0;
        } else {
            const int64_t e = k - nt - nn;
            R[f * tt + e] = (e / t == e % t) ? one : 0;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st[f].key = kKeyNone;
        st[f].done = 0;
    }
}

// Minimal key (v << 42 | row << 21 | column) over rows >= c, columns >= c.
__global__ __launch_bounds__(256) void k_ls_key(const uint64_t *__restrict__ W, int64_t n, int64_t t, int64_t c,
                                                const LsnfPlane *__restrict__ pl, LsnfStep *__restrict__ st) {
    const int f = blockIdx.y;
    if (st[f].done) return;
    const LsnfPlane P0 = pl[f];
    const int64_t w = t - c, cnt = (n - c) * w;
    uint64_t best = kKeyNone;
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < cnt; k += (int64_t)gridDim.x * 256) {
        const int64_t i = c + k / w, j = c + k % w;
        const uint64_t x = W[f * n * t + i * t + j];
        if (x == 0) continue;
        const uint64_t key = ((uint64_t)ls_val(P0, x) << 42) | ((uint64_t)i << 21) | (uint64_t)j;
        best = key < best ? key : best;
    }
    __shared__ uint64_t red[256];
    red[threadIdx.x] = best;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] = min(red[threadIdx.x], red[threadIdx.x + h]);
        __syncthreads();
    }
    if (threadIdx.x == 0 && red[0] != kKeyNone) atomicMin((unsigned long long *)&st[f].key, (unsigned long long)red[0]);
}

// Row exchange c <-> pivot row in W and E.
__global__ __launch_bounds__(256) void k_ls_swap_rows(uint64_t *__restrict__ W, uint64_t *__restrict__ E, int64_t n,
                                                      int64_t t, int64_t c, const LsnfStep *__restrict__ st) {
    const int f = blockIdx.y;
    const uint64_t key = st[f].key;
    if (st[f].done || key == kKeyNone) return;
    const int64_t i = (int64_t)((key >> 21) & 0x1FFFFF);
    if (i == c) return;
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k < t) {
        uint64_t *a = W + f * n * t + c * t + k, *b = W + f * n * t + i * t + k;
        const uint64_t x = *a;
        *a = *b;
        *b = x;
    }
    if (k < n) {
        uint64_t *a = E + f * n * n + c * n + k, *b = E + f * n * n + i * n + k;
        const uint64_t x = *a;
        *a = *b;
        *b = x;
    }
}

// Column exchange c <-> pivot column in W and R (rows of the transposed R).
__global__ __launch_bounds__(256) void k_ls_swap_cols(uint64_t *__restrict__ W, uint64_t *__restrict__ R, int64_t n,
                                                      int64_t t, int64_t c, const LsnfStep *__restrict__ st) {
    const int f = blockIdx.y;
    const uint64_t key = st[f].key;
    if (st[f].done || key == kKeyNone) return;
    const int64_t j = (int64_t)(key & 0x1FFFFF);
    if (j == c) return;
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k < n) {
        uint64_t *a = W + f * n * t + k * t + c, *b = W + f * n * t + k * t + j;
        const uint64_t x = *a;
        *a = *b;
        *b = x;
    }
    if (k < t) {
        uint64_t *a = R + f * t * t + c * t + k, *b = R + f * t * t + j * t + k;
        const uint64_t x = *a;
        *a = *b;
        *b = x;
    }
}

// The pivot of step c: v, q^v, m / q^v and the inverse of the pivot's unit
// part modulo m / q^v; vals[f][c] = v (e once the rest is zero) and
// units[f][c] = the plain unit part modulo m / q^v.  Resets the key.
__global__ void k_ls_pivot(const uint64_t *__restrict__ W, int64_t n, int64_t t, int64_t c,
                           const LsnfPlane *__restrict__ pl, LsnfStep *__restrict__ st, int32_t *__restrict__ vals,
                           uint64_t *__restrict__ units) {
    const int f = blockIdx.x;
    if (threadIdx.x != 0) return;
    const LsnfPlane P0 = pl[f];
    LsnfStep &S = st[f];
    if (S.done || S.key == kKeyNone) {
        S.done = 1;
        vals[f * t + c] = P0.e;
        units[f * t + c] = 0;
        return;
    }
    const int v = (int)(S.key >> 42);
    uint64_t qv = 1;
    for (int i = 0; i < v; ++i) qv *= P0.q;
    const uint64_t mq = P0.m / qv;
    const uint64_t ap = ls_divq(P0, W[f * n * t + c * t + c], v) % mq;   // (a / q^v) R (mod m / q^v)
    S.v = v;
    S.qv = qv;
    S.mq = mq;
    S.uinv = ls_inv(ap, mq);
    vals[f * t + c] = v;
    units[f * t + c] = P0.pow2 ? ap : ls_mulmod(ap, P0.rinv % mq, mq);     // a / q^v, plain
    S.key = kKeyNone;
}

// Rows r > c: row r -= f_r row c in W (columns > c) and in E (all columns),
// f_r = (W[r][c] / q^v) (a / q^v)^-1 mod m / q^v; one work-group per row.
__global__ __launch_bounds__(256) void k_ls_elim_rows(uint64_t *__restrict__ W, uint64_t *__restrict__ E, int64_t n,
                                                      int64_t t, int64_t c, const LsnfPlane *__restrict__ pl,
                                                      const LsnfStep *__restrict__ st) {
    const int f = blockIdx.y;
    const LsnfStep &S = st[f];
    if (S.done) return;
    const LsnfPlane P0 = pl[f];
    const int64_t r = c + 1 + blockIdx.x;
    uint64_t *Wf = W + f * n * t, *Ef = E + f * n * n;
    const uint64_t b = Wf[r * t + c];
    if (b == 0) return;
    const uint64_t fr = ls_mulmod(ls_divq(P0, b, S.v) % S.mq, S.uinv, S.mq);   // plain
    const uint64_t fm = ls_mul(P0, fr, P0.r2);                                // its Montgomery form
    for (int64_t j = c + 1 + threadIdx.x; j < t; j += 256)
        Wf[r * t + j] = ls_sub(P0, Wf[r * t + j], ls_mul(P0, fm, Wf[c * t + j]));
    for (int64_t k = threadIdx.x; k < n; k += 256) Ef[r * n + k] = ls_sub(P0, Ef[r * n + k], ls_mul(P0, fm, Ef[c * n + k]));
    __syncthreads();
    if (threadIdx.x == 0) Wf[r * t + c] = 0;
}

// Columns j > c: column j -= g_j column c in R (row j of the transposed
// buffer -= g_j row c), W[c][j] = 0, g_j = (W[c][j] / q^v) (a / q^v)^-1
// mod m / q^v; one work-group per column.
__global__ __launch_bounds__(256) void k_ls_elim_cols(uint64_t *__restrict__ W, uint64_t *__restrict__ R, int64_t n,
                                                      int64_t t, int64_t c, const LsnfPlane *__restrict__ pl,
                                                      const LsnfStep *__restrict__ st) {
    const int f = blockIdx.y;
    const LsnfStep &S = st[f];
    if (S.done) return;
    const LsnfPlane P0 = pl[f];
    const int64_t j = c + 1 + blockIdx.x;
    uint64_t *Wf = W + f * n * t, *Rf = R + f * t * t;
    const uint64_t w = Wf[c * t + j];
    if (w == 0) return;
    const uint64_t g = ls_mulmod(ls_divq(P0, w, S.v) % S.mq, S.uinv, S.mq);
    const uint64_t gm = ls_mul(P0, g, P0.r2);
    for (int64_t k = threadIdx.x; k < t; k += 256) Rf[j * t + k] = ls_sub(P0, Rf[j * t + k], ls_mul(P0, gm, Rf[c * t + k]));
    __syncthreads();
    if (threadIdx.x == 0) Wf[c * t + j] = 0;
}

// out[f][i][j] = sum_k Pf[i][k] R_f[k][j] (plain, mod m_f) for j < take, R_f
// from its transposed buffer.  A work-group takes 16 rows i x 64 columns j:
// chunks of 32 k of those 16 rows of Pf and of the 64 rows j of the
// transposed R are staged in LDS (both read along k, contiguously), and
// thread (w, l) accumulates rows 4 w .. 4 w + 3 against column l.
constexpr int kPrTI = 16, kPrTJ = 64, kPrKC = 32;
__global__ __launch_bounds__(256) void k_ls_pr(const uint64_t *__restrict__ Pf, const uint64_t *__restrict__ R,
                                               int64_t n, int64_t t, int64_t take, const LsnfPlane *__restrict__ pl,
                                               uint64_t *__restrict__ out) {
    __shared__ uint64_t ps[kPrTI][kPrKC + 1];
    __shared__ uint64_t rs[kPrTJ][kPrKC + 1];
    const int f = blockIdx.z;
    const LsnfPlane P0 = pl[f];
    const int64_t i0 = (int64_t)blockIdx.y * kPrTI, j0 = (int64_t)blockIdx.x * kPrTJ;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t *pf = Pf + f * n * t;
    const uint64_t *rf = R + f * t * t;
    uint64_t acc[4] = {0, 0, 0, 0};
    for (int64_t k0 = 0; k0 < t; k0 += kPrKC) {
        // 16 x 32 of Pf and 64 x 32 of the transposed R, zero past the edges
        for (int e = threadIdx.x; e < kPrTI * kPrKC; e += 256) {
            const int r = e / kPrKC, kk = e % kPrKC;
            const int64_t i = i0 + r, k = k0 + kk;
            ps[r][kk] = i < n && k < t ? pf[i * t + k] : 0;
        }
        for (int e = threadIdx.x; e < kPrTJ * kPrKC; e += 256) {
            const int r = e / kPrKC, kk = e % kPrKC;
            const int64_t j = j0 + r, k = k0 + kk;
            rs[r][kk] = j < take && k < t ? rf[j * t + k] : 0;
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < kPrKC; ++kk) {
            const uint64_t rv = rs[lane][kk];
#pragma unroll
            for (int a = 0; a < 4; ++a) acc[a] = ls_add(P0, acc[a], ls_mul(P0, ps[4 * w + a][kk], rv));   // plain x Montgomery
        }
        __syncthreads();
    }
    const int64_t j = j0 + lane;
    if (j >= take) return;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int64_t i = i0 + 4 * w + a;
        if (i < n) out[(f * n + i) * take + j] = acc[a];
    }
}

// Rows 0 .. rows-1 of every E_f from Montgomery to plain form.
__global__ __launch_bounds__(256) void k_ls_plain(uint64_t *__restrict__ E, int64_t n, int64_t rows,
                                                  const LsnfPlane *__restrict__ pl) {
    const int f = blockIdx.y;
    const LsnfPlane P0 = pl[f];
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < rows * n; k += (int64_t)gridDim.x * 256)
        E[f * n * n + k] = ls_mul(P0, E[f * n * n + k], 1);
}

}  // namespace

void launch_ls_load(const uint64_t *P, int64_t n, int64_t t, const LsnfPlane *pl, int F, uint64_t *W, uint64_t *Pf,
                    uint64_t *E, uint64_t *R, LsnfStep *st, hipStream_t s) {
    ProfScope trace_(tl_trace, "k_ls_load", s);
    const int64_t total = n * t + n * n + t * t;
    const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(k_ls_load, dim3(blocks, (unsigned)F), dim3(256), 0, s, P, n, t, pl, W, Pf, E, R, st);
}

void launch_ls_step(uint64_t *W, uint64_t *E, uint64_t *R, int64_t n, int64_t t, int64_t c, const LsnfPlane *pl,
                    int F, LsnfStep *st, int32_t *vals, uint64_t *units, hipStream_t s) {
    ProfScope trace_(tl_trace, "k_ls_step", s, 6);
    const int64_t cnt = (n - c) * (t - c);
    const unsigned kb = (unsigned)std::min<int64_t>(std::max<int64_t>((cnt + 255) / 256, 1), 4096);
    hipLaunchKernelGGL(k_ls_key, dim3(kb, (unsigned)F), dim3(256), 0, s, W, n, t, c, pl, st);
    const unsigned sb = (unsigned)((std::max(n, t) + 255) / 256);
    hipLaunchKernelGGL(k_ls_swap_rows, dim3(sb, (unsigned)F), dim3(256), 0, s, W, E, n, t, c, st);
    hipLaunchKernelGGL(k_ls_swap_cols, dim3(sb, (unsigned)F), dim3(256), 0, s, W, R, n, t, c, st);
    hipLaunchKernelGGL(k_ls_pivot, dim3((unsigned)F), dim3(64), 0, s, W, n, t, c, pl, st, vals, units);
    if (n - c - 1 > 0)
        hipLaunchKernelGGL(k_ls_elim_rows, dim3((unsigned)(n - c - 1), (unsigned)F), dim3(256), 0, s, W, E, n, t, c,
                           pl, st);
    if (t - c - 1 > 0)
        hipLaunchKernelGGL(k_ls_elim_cols, dim3((unsigned)(t - c - 1), (unsigned)F), dim3(256), 0, s, W, R, n, t, c,
                           pl, st);
}

void launch_ls_pr(const uint64_t *Pf, const uint64_t *R, int64_t n, int64_t t, int64_t take, const LsnfPlane *pl,
                  int F, uint64_t *out, hipStream_t s) {
    if (take <= 0) return;
    ProfScope trace_(tl_trace, "k_ls_pr", s);
    hipLaunchKernelGGL(k_ls_pr, dim3((unsigned)((take + kPrTJ - 1) / kPrTJ), (unsigned)((n + kPrTI - 1) / kPrTI),
                                     (unsigned)F), dim3(256), 0, s, Pf, R, n, t, take, pl, out);
}

void launch_ls_plain(uint64_t *E, int64_t n, int64_t rows, const LsnfPlane *pl, int F, hipStream_t s) {
    if (rows <= 0) return;
    ProfScope trace_(tl_trace, "k_ls_plain", s);
    const unsigned blocks = (unsigned)std::min<int64_t>((rows * n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_ls_plain, dim3(blocks, (unsigned)F), dim3(256), 0, s, E, n, rows, pl);
}

}  // namespace rns
