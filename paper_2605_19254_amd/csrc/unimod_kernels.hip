// Elementwise kernels of the unimodularity certificate (Section 2.2,
// Phase 3): high-order X-adic residues by double-plus-one steps
//
//     Y = Z Z,   K = cmod(C Y, X),   Z' = (Y - D K) / X,
//
// with X the product of the primes p_1 .. p_j of one residue basis and the
// exact value of Z' recovered from a second basis q_1 .. q_l.  The three
// products are residue products (the INT8 matrix-core GEMM); these kernels do
// the parts between them:
//
//   k_uc_convert  K mod p_i (i <= j)  ->  K mod q_k: Garner's mixed radix
//                 digits of K mod X, the symmetric representative chosen by
//                 comparing the digits with those of (X - 1) / 2, then Horner
//                 modulo each q_k.
//   k_uc_identity Z_0 = I.
//   k_uc_tail     (Y - D K) mod q_k  ->  Z' = (Y - D K) X^-1 as int64: the
//                 residues times X^-1 mod q_k, Garner over the q_k, the
//                 symmetric representative as above, its bound checked; one
//                 flag records a nonzero entry, another an entry beyond the
//                 bound.
//
// All moduli are below 2^26, so every product of two residues is below 2^52
// and fits a 64-bit integer; reductions use the integer remainder.
#include "smith_internal.hpp"

namespace rns {
namespace {

__device__ __forceinline__ uint64_t sub_mod(uint64_t a, uint64_t b, uint64_t m) {
    return a >= b ? a - b : a + m - b;
}

// Mixed-radix digits of the residues r[0..k) (moduli m[0..k)): value =
// d_0 + m_0 (d_1 + m_1 (d_2 + ...)); inv[a][b] = m_a^-1 mod m_b for a < b.
__device__ __forceinline__ void garner(const uint64_t *r, const uint32_t *m, const uint32_t (*inv)[kUcMaxPrimes],
                                       int k, uint64_t *d) {
    for (int b = 0; b < k; ++b) {
        uint64_t t = r[b];
        for (int a = 0; a < b; ++a) t = (sub_mod(t, d[a] % m[b], m[b]) * inv[a][b]) % m[b];
        d[b] = t;
    }
}

// Whether the mixed-radix value with digits d exceeds the one with digits h
// (both over the same radices; the most significant digit is the last).
__device__ __forceinline__ bool mr_greater(const uint64_t *d, const uint32_t *h, int k) {
    for (int b = k - 1; b >= 0; --b) {
        if (d[b] != h[b]) return d[b] > h[b];
    }
    return false;
}

__global__ __launch_bounds__(256) void k_uc_convert(const uint32_t *__restrict__ Kp, uint32_t *__restrict__ Kq,
                                                    int64_t count, int64_t plane_stride, UcBasis b) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x) {
        uint64_t r[kUcMaxPrimes], d[kUcMaxPrimes];
        for (int i = 0; i < b.j; ++i) r[i] = Kp[i * plane_stride + e];
        garner(r, b.p, b.pinv, b.j, d);
        const bool neg = mr_greater(d, b.phalf, b.j);     // K = value - X
        for (int k = 0; k < b.l; ++k) {
            const uint64_t q = b.q[k];
            uint64_t w = d[b.j - 1] % q;
            for (int i = b.j - 2; i >= 0; --i) w = (w * (b.p[i] % q) + d[i] % q) % q;
            if (neg) w = sub_mod(w, b.x_mod_q[k], q);
            Kq[k * plane_stride + e] = (uint32_t)w;
        }
    }
}

__global__ __launch_bounds__(256) void k_uc_tail(const uint32_t *__restrict__ Rq, int64_t *__restrict__ Z,
                                                 int64_t count, int64_t plane_stride, UcBasis b,
                                                 int32_t *__restrict__ flags) {
    int nonzero = 0, beyond = 0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x) {
        uint64_t r[kUcMaxPrimes], d[kUcMaxPrimes];
        for (int k = 0; k < b.l; ++k) r[k] = ((uint64_t)Rq[k * plane_stride + e] * b.xinv_q[k]) % b.q[k];
        garner(r, b.q, b.qinv, b.l, d);
        const bool neg = mr_greater(d, b.qhalf, b.l);
        // |z| (or |z| - 1 for negative z, from the complemented digits) as an
        // unsigned 128-bit value, so that an entry beyond the bound is seen.
        unsigned __int128 v = 0;
        for (int k = b.l - 1; k >= 0; --k) {
            const uint64_t dk = neg ? (uint64_t)b.q[k] - 1 - d[k] : d[k];
            v = v * b.q[k] + dk;
        }
        if (neg) v += 1;
        int64_t z = 0;
        if (v > (unsigned __int128)b.bound) {
            beyond = 1;
        } else {
            z = neg ? -(int64_t)(uint64_t)v : (int64_t)(uint64_t)v;
        }
        nonzero |= z != 0;
        Z[e] = z;
    }
    nonzero = __syncthreads_or(nonzero);
    beyond = __syncthreads_or(beyond);
    if (threadIdx.x == 0) {
        if (nonzero) atomicOr(flags, 1);
        if (beyond) atomicOr(flags + 1, 1);
    }
}

__global__ __launch_bounds__(256) void k_uc_identity(int64_t *__restrict__ Z, int64_t n) {
    const int64_t count = n * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x)
        Z[e] = (e / n == e % n) ? 1 : 0;
}

unsigned uc_blocks(int64_t count) {
    const int64_t b = (count + 255) / 256;
    return (unsigned)std::min<int64_t>(std::max<int64_t>(b, 1), 8192);
}

}  // namespace

void launch_uc_identity(int64_t *Z, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    ProfScope trace_(tl_trace, "k_uc_identity", s);
    hipLaunchKernelGGL(k_uc_identity, dim3(uc_blocks(n * n)), dim3(256), 0, s, Z, n);
}

void launch_uc_convert(const uint32_t *Kp, uint32_t *Kq, int64_t count, int64_t plane_stride, const UcBasis &b,
                       hipStream_t s) {
    if (count <= 0) return;
    ProfScope trace_(tl_trace, "k_uc_convert", s);
    hipLaunchKernelGGL(k_uc_convert, dim3(uc_blocks(count)), dim3(256), 0, s, Kp, Kq, count, plane_stride, b);
}

void launch_uc_tail(const uint32_t *Rq, int64_t *Z, int64_t count, int64_t plane_stride, const UcBasis &b,
                    int32_t *flags, hipStream_t s) {
    if (count <= 0) return;
    ProfScope trace_(tl_trace, "k_uc_tail", s);
    hipLaunchKernelGGL(k_uc_tail, dim3(uc_blocks(count)), dim3(256), 0, s, Rq, Z, count, plane_stride, b, flags);
}

}  // namespace rns
