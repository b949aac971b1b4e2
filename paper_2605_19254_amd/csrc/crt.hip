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
#include "internal.hpp"

#include <algorithm>

using namespace rns;

namespace {

constexpr int kBlock = 128;

__device__ __forceinline__ double modp(double x, const PrimeConst &P) {
    return fma(-rint(x * P.pinv), P.pf, x);                 // |result| <= (p+1)/2
}

template <int WT>
__global__ __launch_bounds__(kBlock) void k_crt_garner(
    const uint32_t *__restrict__ res, int64_t rows, int64_t cols, int64_t ldr, int64_t ps,
    const PrimeConst *__restrict__ pc, const double *__restrict__ garner,
    const uint32_t *__restrict__ half, int L, uint64_t *__restrict__ out, int W, int64_t ldo,
    int32_t *__restrict__ status, int64_t col_tiles) {
    __shared__ uint32_t vd[kCrtMaxL][kBlock];
    const int tid = threadIdx.x;
    const int64_t ntiles = rows * col_tiles;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t i = t / col_tiles;
        const int64_t c = (t - i * col_tiles) * kBlock + tid;
        if (c >= cols) continue;
        const uint32_t *src = res + i * ldr + c;
        // Garner digits.
        for (int j = 0; j < L; ++j) {
            const PrimeConst P = pc[j];
            double tj = (double)src[(int64_t)j * ps];
            const double *gj = garner + (int64_t)j * kCrtMaxL;
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
        if (!fits) atomicOr(status, 1);
        // Two's complement of the signed value, low W words.
        uint64_t *dst = out + (i * ldo + c) * W;
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
    }
}

template <int WT>
__global__ __launch_bounds__(kBlock) void k_crt_lagrange(
    const uint32_t *__restrict__ res, int64_t rows, int64_t cols, int64_t ldr, int64_t ps,
    const PrimeConst *__restrict__ pc, const double *__restrict__ cinv,
    const uint64_t *__restrict__ mj, const uint64_t *__restrict__ mw, int L,
    uint64_t *__restrict__ out, int W, int64_t ldo, int64_t col_tiles) {
    const int64_t ntiles = rows * col_tiles;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t i = t / col_tiles;
        const int64_t c = (t - i * col_tiles) * kBlock + threadIdx.x;
        if (c >= cols) continue;
        const uint32_t *src = res + i * ldr + c;
        uint64_t x[WT];
#pragma unroll
        for (int k = 0; k < WT; ++k) x[k] = 0;
        double alpha = 0.0;
        for (int j = 0; j < L; ++j) {
            const PrimeConst P = pc[j];
            double y = modp((double)src[(int64_t)j * ps] * cinv[j], P);
            y = y < 0.0 ? y + P.pf : y;
            alpha = fma(y, P.pinv, alpha);
            const uint64_t yi = (uint64_t)y;
            const uint64_t *m = mj + (int64_t)j * W;
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
        uint64_t *dst = out + (i * ldo + c) * W;
#pragma unroll
        for (int k = 0; k < WT; ++k)
            if (k < W) dst[k] = x[k];
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
    const int64_t col_tiles = (cols + kBlock - 1) / kBlock;
    const int64_t ntiles = rows * col_tiles;
    const unsigned grid = (unsigned)std::min<int64_t>(ntiles, 1 << 20);
    const PrimeConst *pc = ctx->d_prime + prime_begin;

    // Decide whether the caller's bound allows the Lagrange form.
    bool fast = false;
    if (bound_words && Wb > 0) {
        Limbs B = limbs_from_words(bound_words, Wb);
        Limbs M{1};
        for (int j = 0; j < L; ++j) limbs_mul_small(M, ctx->primes[prime_begin + j]);
        Limbs twoB = B;
        limbs_mul_small(twoB, 2);
        Limbs lim_w{1};                    // 2^(64W-1)
        for (int k = 0; k < 64 * W - 1; ++k) limbs_mul_small(lim_w, 2);
        if (limbs_cmp(twoB, M) < 0 && limbs_cmp(B, lim_w) < 0) {
            Limbs D = limbs_sub(M, twoB);
            Limbs T = limbs_shr(M, 39, true);
            fast = limbs_cmp(D, T) >= 0;
        }
    }
    if (fast) {
        const LagrangeTable *lt = nullptr;
        int st = lagrange_table(ctx, prime_begin, L, W, &lt);
        if (st != RNS_OK) return st;
        ProfScope ps(ctx, "k_crt_lagrange", s);
#define RNS_LAG(WT_)                                                                       \
    hipLaunchKernelGGL(k_crt_lagrange<WT_>, dim3(grid), dim3(kBlock), 0, s, res, rows, cols, \
                       ldr, plane_stride, pc, lt->d_c, lt->d_mj, lt->d_m, L, out, W, ldo,   \
                       col_tiles)
        if (W <= 1) RNS_LAG(1);
        else if (W <= 2) RNS_LAG(2);
        else if (W <= 4) RNS_LAG(4);
        else if (W <= 8) RNS_LAG(8);
        else if (W <= 16) RNS_LAG(16);
        else RNS_LAG(32);
#undef RNS_LAG
    } else {
        const uint32_t *half = nullptr;
        int st = mixed_radix_half(ctx, prime_begin, L, &half);
        if (st != RNS_OK) return st;
        int32_t *status = d_status ? d_status : ctx->d_status;
        const double *garner = ctx->d_garner + (int64_t)prime_begin * kCrtMaxL;
        ProfScope ps(ctx, "k_crt_garner", s);
#define RNS_GAR(WT_)                                                                      \
    hipLaunchKernelGGL(k_crt_garner<WT_>, dim3(grid), dim3(kBlock), 0, s, res, rows, cols, \
                       ldr, plane_stride, pc, garner, half, L, out, W, ldo, status,        \
                       col_tiles)
        if (W <= 1) RNS_GAR(1);
        else if (W <= 2) RNS_GAR(2);
        else if (W <= 4) RNS_GAR(4);
        else if (W <= 8) RNS_GAR(8);
        else if (W <= 16) RNS_GAR(16);
        else RNS_GAR(32);
#undef RNS_GAR
    }
    RNS_HIP(hipGetLastError());
    return RNS_OK;
}
