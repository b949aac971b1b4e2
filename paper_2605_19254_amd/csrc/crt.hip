// crt_reconstruct: L residue planes -> signed integers in W 64-bit words
// (Section 3.1: the integer result is rebuilt by the Chinese Remainder
// Theorem; the bullet on fast base conversion adds the Lagrange form with a
// floating-point correction factor).  One thread per matrix entry; the
// residues of an entry are read from the L planes with coalesced loads.
//
// Exact form (Garner).  Mixed-radix digits v_j with
//   x = v_0 + v_1 p_0 + v_2 p_0 p_1 + ... ,  0 <= v_j < p_j,
// from t_j = (((r_j - v_0) p_0^-1 - v_1) p_1^-1 - ...) mod p_j.  Each modular
// product has factors below 1.5*2^26 and 2^26, so it is exact in a double and
// reduced with the rounded reciprocal.  x > (M-1)/2 (digit-wise comparison
// from the top) means the symmetric representative is x - M < 0; its
// magnitude M - x = (M-1-x) + 1 has the borrow-free digits p_j - 1 - v_j.
// The magnitude is evaluated by Horner's rule into W words with a sticky bit
// for anything beyond, which decides overflow exactly.
//
// Lagrange form.  y_j = r_j * (M/p_j)^-1 mod p_j, then
//   x = sum_j y_j (M/p_j) - alpha M,   alpha = round(sum_j y_j / p_j),
// evaluated modulo 2^(64W).  alpha is exact when a caller-supplied bound B
// leaves the margin B/M <= 1/2 - 2^-40 (the double sum of at most 64 terms
// below 1 errs by less than 2^-40.9), which the host checks before choosing
// this form; it also requires B < 2^(64W-1), so the result cannot overflow.
//
// Exact Lagrange form (k_crt_exact, no bound needed).  The same sum S over
// 32-bit limbs: each limb column accumulates y_j times limb k of M/p_j with
// 32 x 32 -> 64-bit multiply-adds (products below 2^58, so 32 primes fit a
// 64-bit column before the carries are propagated), then a = floor(alpha)
// and x = S - a M.  alpha errs by less than 2^-40, so a is floor(S / M) or
// one off when S / M lies that close to an integer; one addition or
// subtraction of M brings x into [0, M) in every case, and x > M - x picks
// the negative representative x - M.  Exact for any residues.
//
// The kernels take one job by value or a table of jobs in device memory
// (every product of a batched plan in one launch).
#include "reduce_crt.hpp"

#include <algorithm>
#include <cmath>

using namespace rns;

namespace {

constexpr int kBlock = 128;
constexpr int kLagEntries = 4;

struct PC2 {
    double pf, pinv;
};

__device__ __forceinline__ double modp(double x, const PC2 &P) {
    return fma(-rint(x * P.pinv), P.pf, x);                 // |result| <= (p+1)/2
}

// With a job table, blocks take runs of `chunk` consecutive tiles, job by job
// (for_job_tiles).  A single job uses runs of one tile.
constexpr int kChunk = 8;

template <int WT>
__global__ __launch_bounds__(kBlock) void k_crt_garner(CrtJob job0, const CrtJob *__restrict__ jobs,
                                                      int njobs, int64_t total_tiles,
                                                      const PrimeConst *__restrict__ pc_all,
                                                      const double *__restrict__ garner_all, int W,
                                                      int chunk) {
    __shared__ uint32_t vd[kCrtMaxL][kBlock];
    const int tid = threadIdx.x;
    const int64_t nchunks = (total_tiles + chunk - 1) / chunk;
    for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
      const int64_t t0 = ch * chunk;
      const int64_t t1 = t0 + chunk < total_tiles ? t0 + chunk : total_tiles;
      for_job_tiles(job0, jobs, njobs, total_tiles, t0, t1, [&](const CrtJob &J, int64_t t) {
        const int64_t u = t - J.tile_begin;
        const int64_t i = u / J.col_tiles;
        // Lanes past the last column work on the last column and store
        // nothing, so control flow stays uniform (uniform loads stay scalar).
        const int64_t c_lane = (u - i * J.col_tiles) * kBlock + tid;
        const bool valid = c_lane < J.cols;
        const int64_t c = valid ? c_lane : J.cols - 1;
        const auto src = gptr(J.res + i * J.ldr + c);
        const auto pc = cptr(pc_all + J.prime_begin);
        const auto garner = cptr(garner_all + (int64_t)J.prime_begin * kCrtMaxL);
        const auto half = cptr(J.half);
        const int L = J.L;
        const int64_t ps = J.ps;
        // All residues of this entry into its digit column, eight loads in
        // flight at a time.
        for (int j0 = 0; j0 < L; j0 += 8) {
            uint32_t r[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) r[q] = src[(int64_t)min(j0 + q, L - 1) * ps];   // in bounds
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (j0 + q < L) vd[j0 + q][tid] = r[q];
        }
        // Garner digits, each overwriting its residue.
        for (int j = 0; j < L; ++j) {
            const PC2 P{pc[j].pf, pc[j].pinv};
            double tj = (double)vd[j][tid];
            const auto gj = garner + (int64_t)j * kCrtMaxL;
            for (int q = 0; q < j; ++q) {
                const double x = (tj - (double)vd[q][tid]) * gj[j - q];
                tj = modp(x, P);
            }
            tj = tj < 0.0 ? tj + P.pf : tj;
            vd[j][tid] = (uint32_t)tj;
        }
        // Sign: compare with the digits of (M-1)/2 from the top.
        bool neg = false;
        for (int j = L - 1; j >= 0; --j) {
            const uint32_t a = vd[j][tid], h = half[j];
            if (a != h) {
                neg = a > h;
                break;
            }
        }
        // Magnitude by Horner's rule, low WT words plus a sticky overflow bit.
        uint64_t w[WT];
#pragma unroll
        for (int k = 0; k < WT; ++k) w[k] = 0;
        bool sticky = false;
        for (int j = L - 1; j >= 0; --j) {
            const uint32_t p = pc[j].p;
            const uint32_t u = neg ? p - 1 - vd[j][tid] : vd[j][tid];
            uint64_t carry = u;
#pragma unroll
            for (int k = 0; k < WT; ++k) {
                const uint64_t lo = w[k] * (uint64_t)p;
                const uint64_t hi = __umul64hi(w[k], (uint64_t)p);
                const uint64_t s = lo + carry;
                carry = hi + (s < lo ? 1 : 0);
                w[k] = s;
            }
            sticky |= carry != 0;
        }
        if (neg) {
            uint64_t carry = 1;
#pragma unroll
            for (int k = 0; k < WT; ++k) {
                const uint64_t s = w[k] + carry;
                carry = (s < w[k]) ? 1 : 0;
                w[k] = s;
            }
            sticky |= carry != 0;
        }
        // Fits in W words?  Positive: mag < 2^(64W-1).  Negative: mag <= 2^(64W-1).
        bool high_zero = !sticky;
#pragma unroll
        for (int k = 0; k < WT; ++k)
            if (k >= W && w[k] != 0) high_zero = false;
        uint64_t top = 0;
        bool low_zero = true;
#pragma unroll
        for (int k = 0; k < WT; ++k) {
            if (k == W - 1) top = w[k];
            if (k < W - 1 && w[k] != 0) low_zero = false;
        }
        bool fits;
        if (!neg) fits = high_zero && (top >> 63) == 0;
        else fits = high_zero && ((top >> 63) == 0 || (top == (1ull << 63) && low_zero));
        if (!valid) return;
        if (!fits) atomicOr(J.status, 1);
        // Two's complement of the signed value, low W words.
        const auto dst = gptr_w(J.out + (i * J.ldo + c) * W);
        uint64_t carry = 1;
#pragma unroll
        for (int k = 0; k < WT; ++k) {
            if (k < W) {
                uint64_t v = w[k];
                if (neg) {
                    const uint64_t nv = ~v;
                    v = nv + carry;
                    carry = (v < nv) ? 1 : 0;
                }
                dst[k] = v;
            }
        }
      });
    }
}

// Lagrange form, one prime's term for one entry: y = r (M/p_j)^-1 mod p_j in
// [0, p_j), alpha += y / p_j, x += y (M/p_j) over the low WT words.
template <int WT>
__device__ __forceinline__ void lag_term(uint64_t (&x)[WT], double &alpha, uint32_t r, int j,
                                         const __attribute__((address_space(4))) PrimeConst *pc,
                                         const __attribute__((address_space(4))) double *cinv,
                                         const __attribute__((address_space(4))) uint64_t *mj, int W) {
    const PC2 P{pc[j].pf, pc[j].pinv};
    double y = modp((double)r * cinv[j], P);
    y = y < 0.0 ? y + P.pf : y;
    alpha = fma(y, P.pinv, alpha);
    const uint64_t yi = (uint64_t)y;
    const auto m = mj + (int64_t)j * W;
    uint64_t carry = 0;
#pragma unroll
    for (int k = 0; k < WT; ++k) {
        if (k < W) {
            const uint64_t lo = m[k] * yi;
            const uint64_t hi = __umul64hi(m[k], yi);
            const uint64_t s1 = lo + carry;
            const uint64_t c1 = s1 < lo ? 1 : 0;
            const uint64_t s2 = x[k] + s1;
            const uint64_t c2 = s2 < x[k] ? 1 : 0;
            x[k] = s2;
            carry = hi + c1 + c2;
        }
    }
}

// x -= round(alpha) M over the low WT words: the symmetric representative.
template <int WT>
__device__ __forceinline__ void lag_finish(uint64_t (&x)[WT], double alpha,
                                           const __attribute__((address_space(4))) uint64_t *mw, int W) {
    const uint64_t a = (uint64_t)rint(alpha);
    uint64_t borrow = 0;
    uint64_t carry = 0;
#pragma unroll
    for (int k = 0; k < WT; ++k) {
        if (k < W) {
            const uint64_t lo = mw[k] * a;
            const uint64_t hi = __umul64hi(mw[k], a);
            const uint64_t s1 = lo + carry;
            carry = hi + (s1 < lo ? 1 : 0);
            const uint64_t d1 = x[k] - s1;
            const uint64_t b1 = x[k] < s1 ? 1 : 0;
            const uint64_t d2 = d1 - borrow;
            const uint64_t b2 = d1 < borrow ? 1 : 0;
            x[k] = d2;
            borrow = b1 + b2;
        }
    }
}

// One entry of the Lagrange form: column c_lane of a row whose residues start
// at res_row (planes ps apart) and whose output words start at out_row.  The
// job's fields come in as values, which keeps them uniform (scalar) after
// inlining.
template <int WT>
__device__ __forceinline__ void lagrange_entry(const uint32_t *res_row, uint64_t *out_row, int64_t cols,
                                               int64_t ps, int L, const PrimeConst *pc_job,
                                               const double *lag_c, const uint64_t *lag_mj,
                                               const uint64_t *lag_m, int W, int64_t c_lane) {
    // Lanes past the last column work on the last column and store nothing,
    // so control flow stays uniform (uniform loads stay scalar).
    const bool valid = c_lane < cols;
    const int64_t c = valid ? c_lane : cols - 1;
    const auto src = gptr(res_row + c);
    const auto pc = cptr(pc_job);
    const auto cinv = cptr(lag_c);
    const auto mj = cptr(lag_mj);
    uint64_t x[WT];
#pragma unroll
    for (int k = 0; k < WT; ++k) x[k] = 0;
    double alpha = 0.0;
    for (int j0 = 0; j0 < L; j0 += 8) {
        uint32_t r[8];                        // eight loads in flight at a time
#pragma unroll
        for (int q = 0; q < 8; ++q) r[q] = src[(int64_t)min(j0 + q, L - 1) * ps];   // in bounds
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            if (j0 + q >= L) break;
            lag_term<WT>(x, alpha, r[q], j0 + q, pc, cinv, mj, W);
        }
    }
    lag_finish<WT>(x, alpha, cptr(lag_m), W);
    if (!valid) return;
    const auto dst = gptr_w(out_row + c * W);
#pragma unroll
    for (int k = 0; k < WT; ++k)
        if (k < W) dst[k] = x[k];
}

// Short bases (L <= kShortL): E entries per thread, kBlock apart, whose
// residues are all loaded (E*kShortL loads in flight; planes past L repeat
// the last one) before any is combined.
constexpr int kShortL = 4;

template <int WT, int E>
__device__ __forceinline__ void lagrange_short(const uint32_t *res_row, uint64_t *out_row, int64_t cols,
                                               int64_t ps, int L, const PrimeConst *pc_job,
                                               const double *lag_c, const uint64_t *lag_mj,
                                               const uint64_t *lag_m, int W, int64_t base) {
    const auto pc = cptr(pc_job);
    const auto cinv = cptr(lag_c);
    const auto mj = cptr(lag_mj);
    uint32_t r[E][kShortL];
    int64_t c[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int64_t c_lane = base + (int64_t)e * kBlock;
        c[e] = c_lane < cols ? c_lane : cols - 1;        // in bounds; stores are skipped below
        const auto src = gptr(res_row + c[e]);
#pragma unroll
        for (int q = 0; q < kShortL; ++q) r[e][q] = src[(int64_t)min(q, L - 1) * ps];   // no branch per load
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        uint64_t x[WT];
#pragma unroll
        for (int k = 0; k < WT; ++k) x[k] = 0;
        double alpha = 0.0;
#pragma unroll
        for (int q = 0; q < kShortL; ++q)
            if (q < L) lag_term<WT>(x, alpha, r[e][q], q, pc, cinv, mj, W);
        lag_finish<WT>(x, alpha, cptr(lag_m), W);
        if (base + (int64_t)e * kBlock < cols) {
            const auto dst = gptr_w(out_row + c[e] * W);
#pragma unroll
            for (int k = 0; k < WT; ++k)
                if (k < W) dst[k] = x[k];
        }
    }
}

// E entries per thread: a tile covers E * kBlock columns of one row.
template <int WT, int E>
__global__ __launch_bounds__(kBlock) void k_crt_lagrange(CrtJob job0, const CrtJob *__restrict__ jobs,
                                                        int njobs, int64_t total_tiles,
                                                        const PrimeConst *__restrict__ pc_all, int W,
                                                        int chunk) {
    const int64_t nchunks = (total_tiles + chunk - 1) / chunk;
    for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
      const int64_t t0 = ch * chunk;
      const int64_t t1 = t0 + chunk < total_tiles ? t0 + chunk : total_tiles;
      for_job_tiles(job0, jobs, njobs, total_tiles, t0, t1, [&](const CrtJob &J, int64_t t) {
        const int64_t u = t - J.tile_begin;
        const int64_t i = u / J.col_tiles;
        const int64_t base = (u - i * J.col_tiles) * kBlock * E + threadIdx.x;
        const uint32_t *res_row = J.res + i * J.ldr;
        uint64_t *out_row = J.out + i * J.ldo * W;
        if constexpr (E > 1) {
            lagrange_short<WT, E>(res_row, out_row, J.cols, J.ps, J.L, pc_all + J.prime_begin, J.lag_c,
                                  J.lag_mj, J.lag_m, W, base);
        } else {
            lagrange_entry<WT>(res_row, out_row, J.cols, J.ps, J.L, pc_all + J.prime_begin, J.lag_c, J.lag_mj,
                               J.lag_m, W, base);
        }
      });
    }
}

// Host helpers on 32-bit limb vectors.
Limbs limbs_from_words(const uint64_t *w, int W) {
    Limbs a;
    for (int k = 0; k < W; ++k) {
        a.push_back((uint32_t)w[k]);
        a.push_back((uint32_t)(w[k] >> 32));
    }
    limbs_trim(a);
    return a;
}

// a - b for a >= b.
Limbs limbs_sub(const Limbs &a, const Limbs &b) {
    Limbs r(a);
    int64_t borrow = 0;
    for (size_t i = 0; i < r.size(); ++i) {
        int64_t t = (int64_t)r[i] - (i < b.size() ? (int64_t)b[i] : 0) - borrow;
        borrow = t < 0;
        r[i] = (uint32_t)(t + (borrow ? (1ll << 32) : 0));
    }
    limbs_trim(r);
    return r;
}

Limbs limbs_shr(const Limbs &a, int bits, bool round_up) {
    Limbs r;
    const int wsh = bits / 32, bsh = bits % 32;
    bool lost = false;
    for (int i = 0; i < (int)a.size(); ++i) {
        if (i < wsh) {
            lost |= a[i] != 0;
            continue;
        }
    }
    if (bsh && wsh < (int)a.size()) lost |= (a[wsh] & ((1u << bsh) - 1)) != 0;
    for (int i = wsh; i < (int)a.size(); ++i) {
        uint64_t lo = a[i] >> bsh;
        uint64_t hi = (bsh && i + 1 < (int)a.size()) ? ((uint64_t)a[i + 1] << (32 - bsh)) : 0;
        r.push_back((uint32_t)(lo | hi));
    }
    limbs_trim(r);
    if (round_up && lost) {
        size_t i = 0;
        for (;; ++i) {
            if (i == r.size()) { r.push_back(1); break; }
            if (++r[i] != 0) break;
        }
    }
    return r;
}

}  // namespace

namespace rns {

// Entries per thread: 4 for the Lagrange form with at most two output words
// and at most 4 primes (little work per entry, so a tile's job lookup is
// shared by more entries), otherwise 1 (more threads in flight).
int crt_entries(bool fast, int W, int L) { return fast && W <= 2 && L <= kShortL ? kLagEntries : 1; }
int64_t crt_col_tiles(int64_t cols, int entries) { return (cols + kBlock * entries - 1) / (kBlock * entries); }
int64_t crt_tiles(int64_t rows, int64_t cols, int entries) { return rows * crt_col_tiles(cols, entries); }

bool crt_fast_ok(const rns_ctx *ctx, int begin, int L, const uint64_t *bound_words, int Wb, int W) {
    if (!bound_words || Wb <= 0) return false;
    Limbs B = limbs_from_words(bound_words, Wb);
    Limbs M{1};
    for (int j = 0; j < L; ++j) limbs_mul_small(M, ctx->primes[begin + j]);
    Limbs twoB = B;
    limbs_mul_small(twoB, 2);
    Limbs lim_w{1};                    // 2^(64W-1)
    for (int k = 0; k < 64 * W - 1; ++k) limbs_mul_small(lim_w, 2);
    if (limbs_cmp(twoB, M) >= 0 || limbs_cmp(B, lim_w) >= 0) return false;
    Limbs D = limbs_sub(M, twoB);
    Limbs T = limbs_shr(M, 39, true);
    return limbs_cmp(D, T) >= 0;
}

// One entry per thread; KT bounds the 32-bit limbs K of the computation (K is
// even: the table's words of M / p_j and M, two limbs each).
template <int KT>
__global__ __launch_bounds__(kBlock) void k_crt_exact(CrtJob J, int64_t total_tiles,
                                                     const PrimeConst *__restrict__ pc_all, int W, int K) {
    const int tid = threadIdx.x;
    for (int64_t t = blockIdx.x; t < total_tiles; t += gridDim.x) {
        const int64_t i = t / J.col_tiles;
        const int64_t c_lane = (t - i * J.col_tiles) * kBlock + tid;
        const bool valid = c_lane < J.cols;
        const int64_t c = valid ? c_lane : J.cols - 1;        // in bounds; the store is skipped below
        const auto src = gptr(J.res + i * J.ldr + c);
        const auto pc = cptr(pc_all + J.prime_begin);
        const auto cinv = cptr(J.lag_c);
        const auto mj = cptr(reinterpret_cast<const uint32_t *>(J.lag_mj));
        const auto m32 = cptr(reinterpret_cast<const uint32_t *>(J.lag_m));
        const int L = J.L;
        const int64_t ps = J.ps;
        uint64_t acc[KT];
#pragma unroll
        for (int k = 0; k < KT; ++k) acc[k] = 0;
        double alpha = 0.0;
        auto settle = [&]() {                       // carries up, every column below 2^32 again
            uint64_t carry = 0;
#pragma unroll
            for (int k = 0; k < KT; ++k) {
                if (k < K) {
                    const uint64_t v = acc[k] + carry;
                    acc[k] = v & 0xFFFFFFFFull;
                    carry = v >> 32;
                }
            }
        };
        for (int j0 = 0; j0 < L; j0 += 8) {
            uint32_t r[8];                          // eight loads in flight at a time
#pragma unroll
            for (int q = 0; q < 8; ++q) r[q] = src[(int64_t)min(j0 + q, L - 1) * ps];   // in bounds
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int j = j0 + q;
                if (j >= L) break;
                const PC2 P{pc[j].pf, pc[j].pinv};
                double y = modp((double)r[q] * cinv[j], P);
                y = y < 0.0 ? y + P.pf : y;
                alpha = fma(y, P.pinv, alpha);
                const uint64_t yi = (uint64_t)y;
                const auto m = mj + (int64_t)j * K;
#pragma unroll
                for (int k = 0; k < KT; ++k)
                    if (k < K) acc[k] += yi * (uint64_t)m[k];
            }
            if ((j0 & 31) == 24) settle();          // at most 32 terms per column between settles
        }
        settle();
        // x = S - a M with a = floor(alpha) (a < 64), as K limbs with a sign.
        const uint64_t a = (uint64_t)floor(alpha);
        int64_t borrow = 0;
        uint64_t mc = 0;
#pragma unroll
        for (int k = 0; k < KT; ++k) {
            if (k < K) {
                const uint64_t prod = a * (uint64_t)m32[k] + mc;
                mc = prod >> 32;
                const int64_t d = (int64_t)acc[k] - (int64_t)(prod & 0xFFFFFFFFull) - borrow;
                borrow = d < 0 ? 1 : 0;
                acc[k] = (uint64_t)(d + (borrow << 32));
            }
        }
        const bool below = borrow != 0 || mc != 0;  // x < 0: S < a M
        // One correction: x + M when below, x - M when x >= M.
        // x >= M, compared from the top limb (a branch-free scan over the
        // unrolled limbs: the first difference from the top decides).
        bool ge = !below, decided = false;
#pragma unroll
        for (int k = KT - 1; k >= 0; --k) {
            if (k < K && !decided && acc[k] != m32[k]) {
                ge = ge && acc[k] > m32[k];
                decided = true;
            }
        }
        if (below || ge) {
            int64_t cb = 0;
#pragma unroll
            for (int k = 0; k < KT; ++k) {
                if (k < K) {
                    const int64_t d = below ? (int64_t)acc[k] + (int64_t)m32[k] + cb
                                            : (int64_t)acc[k] - (int64_t)m32[k] + cb;
                    cb = d >> 32;                                   // -1, 0 or 1
                    acc[k] = (uint64_t)d & 0xFFFFFFFFull;
                }
            }
        }
        // 0 <= x < M; the negative representative when x > M - x.
        uint64_t dm[KT];
        int64_t cb = 0;
#pragma unroll
        for (int k = 0; k < KT; ++k) {
            if (k < K) {
                const int64_t d = (int64_t)m32[k] - (int64_t)acc[k] + cb;
                cb = d >> 32;
                dm[k] = (uint64_t)d & 0xFFFFFFFFull;
            }
        }
        bool neg = false, dec = false;
#pragma unroll
        for (int k = KT - 1; k >= 0; --k) {
            if (k < K && !dec && acc[k] != dm[k]) {
                neg = acc[k] > dm[k];
                dec = true;
            }
        }
        // Magnitude into W words; it fits when below 2^(64W-1) (or equal, for
        // a negative value).
        bool high = false, at_limit = true;
        uint64_t mag_top = 0;
#pragma unroll
        for (int k = 0; k < KT; ++k) {
            if (k >= K) continue;
            const uint64_t v = neg ? dm[k] : acc[k];
            if (k >= 2 * W && v) high = true;
            if (k == 2 * W - 1) mag_top = v;
            else if (k < 2 * W - 1 && v) at_limit = false;
        }
        bool fits = !high && (mag_top >> 31) == 0;
        if (neg && !high && mag_top == 0x80000000ull && at_limit) fits = true;
        if (!valid) continue;
        if (!fits) atomicOr(J.status, 1);
        const auto dst = gptr_w(J.out + (i * J.ldo + c) * W);
        uint64_t carry = 1;
        for (int w = 0; w < W; ++w) {
            const int k0 = 2 * w, k1 = 2 * w + 1;
            uint64_t lo = 0, hi = 0;
#pragma unroll
            for (int k = 0; k < KT; ++k) {
                if (k == k0 && k < K) lo = neg ? dm[k] : acc[k];
                if (k == k1 && k < K) hi = neg ? dm[k] : acc[k];
            }
            uint64_t v = lo | (hi << 32);
            if (neg) {
                const uint64_t nv = ~v;
                v = nv + carry;
                carry = (v < nv) ? 1 : 0;
            }
            dst[w] = v;
        }
    }
}

int launch_crt_exact(const CrtJob &j, int64_t total_tiles, const PrimeConst *pc, int W, int K, hipStream_t s) {
    const unsigned grid = (unsigned)std::min<int64_t>(total_tiles, 1 << 20);
#define RNS_EX(KT_) hipLaunchKernelGGL(k_crt_exact<KT_>, dim3(grid), dim3(kBlock), 0, s, j, total_tiles, pc, W, K)
    if (K <= 8) RNS_EX(8);
    else if (K <= 16) RNS_EX(16);
    else if (K <= 24) RNS_EX(24);
    else if (K <= 32) RNS_EX(32);
    else if (K <= 44) RNS_EX(44);
    else if (K <= 56) RNS_EX(56);
    else return RNS_ENOTSUP;
#undef RNS_EX
    return RNS_OK;
}

void launch_crt(bool fast, int W, int E, const CrtJob &job0, const CrtJob *jobs, int njobs,
                int64_t total_tiles, const PrimeConst *pc, const double *garner, hipStream_t s) {
    const int chunk = njobs > 1 ? kChunk : 1;
    const unsigned grid = (unsigned)std::min<int64_t>((total_tiles + chunk - 1) / chunk, 1 << 20);
    if (fast) {
#define RNS_LAG(WT_, E_) \
    hipLaunchKernelGGL((k_crt_lagrange<WT_, E_>), dim3(grid), dim3(kBlock), 0, s, job0, jobs, njobs, total_tiles, pc, W, chunk)
        if (W <= 1 && E > 1) RNS_LAG(1, kLagEntries);
        else if (W <= 1) RNS_LAG(1, 1);
        else if (W <= 2 && E > 1) RNS_LAG(2, kLagEntries);
        else if (W <= 2) RNS_LAG(2, 1);
        else if (W <= 4) RNS_LAG(4, 1);
        else if (W <= 8) RNS_LAG(8, 1);
        else if (W <= 16) RNS_LAG(16, 1);
        else RNS_LAG(32, 1);
#undef RNS_LAG
    } else {
#define RNS_GAR(WT_) \
    hipLaunchKernelGGL(k_crt_garner<WT_>, dim3(grid), dim3(kBlock), 0, s, job0, jobs, njobs, total_tiles, pc, garner, W, chunk)
        if (W <= 1) RNS_GAR(1);
        else if (W <= 2) RNS_GAR(2);
        else if (W <= 4) RNS_GAR(4);
        else if (W <= 8) RNS_GAR(8);
        else if (W <= 16) RNS_GAR(16);
        else RNS_GAR(32);
#undef RNS_GAR
    }
}

}  // namespace rns

extern "C" int crt_reconstruct(rns_ctx *ctx, const uint32_t *res, int64_t rows, int64_t cols,
                               int64_t ldr, int64_t plane_stride, int prime_begin, int L,
                               const uint64_t *bound_words, int Wb, uint64_t *out, int W,
                               int64_t ldo, int32_t *d_status, void *stream) {
    if (!ctx || rows < 0 || cols < 0) return RNS_EINVAL;
    if (L < 1 || L > kCrtMaxL || W < 1 || W > kCrtMaxW) return RNS_EINVAL;
    if (prime_begin < 0 || prime_begin + L > ctx->L) return RNS_EINVAL;
    if (Wb < 0 || (Wb > 0 && !bound_words)) return RNS_EINVAL;
    if (rows == 0 || cols == 0) return RNS_OK;
    if (!res || !out || ldr < cols || ldo < cols) return RNS_EINVAL;
    if (L > 1 && plane_stride < (rows - 1) * ldr + cols) return RNS_EINVAL;
    std::lock_guard<std::mutex> guard(ctx->mu);
    RNS_HIP(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    CrtJob j{};
    j.res = res; j.rows = rows; j.cols = cols; j.ldr = ldr; j.ps = plane_stride;
    j.prime_begin = prime_begin; j.L = L; j.out = out; j.ldo = ldo;
    j.status = d_status ? d_status : ctx->d_status;
    j.tile_begin = 0;
    const bool fast = crt_fast_ok(ctx, prime_begin, L, bound_words, Wb, W);
    if (!fast && ctx->crt_form == 1)   // the exact form on the matrix cores (digits_gemm.hip)
        return crt_mfma(ctx, res, rows, cols, ldr, plane_stride, prime_begin, L, out, W, ldo, j.status, s);
    if (!fast && ctx->crt_form == 0) {  // the exact Lagrange form on 32-bit limbs
        int Wm = 1;                      // words of M, plus one for S < L M
        {
            double bits = 0;
            for (int q = 0; q < L; ++q) bits += std::log2((double)ctx->primes[prime_begin + q]);
            Wm = (int)((bits + 7.0) / 64.0) + 1;
        }
        const LagrangeTable *lt = nullptr;
        int st = lagrange_table(ctx, prime_begin, L, Wm, &lt, s);
        if (st != RNS_OK) return st;
        j.lag_c = lt->d_c; j.lag_mj = lt->d_mj; j.lag_m = lt->d_m;
        j.col_tiles = crt_col_tiles(cols, 1);
        ProfScope ps(ctx, "k_crt_exact", s);
        st = launch_crt_exact(j, crt_tiles(rows, cols, 1), ctx->d_prime, W, 2 * Wm, s);
        if (st != RNS_OK) return st;
        RNS_HIP(hipGetLastError());
        return RNS_OK;
    }
    const int E = crt_entries(fast, W, L);
    j.col_tiles = crt_col_tiles(cols, E);
    if (fast) {
        const LagrangeTable *lt = nullptr;
        int st = lagrange_table(ctx, prime_begin, L, W, &lt, s);
        if (st != RNS_OK) return st;
        j.lag_c = lt->d_c; j.lag_mj = lt->d_mj; j.lag_m = lt->d_m;
    } else {
        int st = mixed_radix_half(ctx, prime_begin, L, &j.half, s);
        if (st != RNS_OK) return st;
    }
    ProfScope ps(ctx, fast ? "k_crt_lagrange" : "k_crt_garner", s);
    launch_crt(fast, W, E, j, nullptr, 0, crt_tiles(rows, cols, E), ctx->d_prime, ctx->d_garner, s);
    RNS_HIP(hipGetLastError());
    return RNS_OK;
}
