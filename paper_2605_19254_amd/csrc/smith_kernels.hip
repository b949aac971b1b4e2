// GPU kernels of the Smith-form driver.
//
//   Blocked Gauss-Jordan inversion and forward elimination modulo many primes
//   at once (pivot blocks, row exchanges; the block updates are residue
//   products), for A^-1 mod q and det A mod q.
//   p-adic lifting steps and projections of the lifted digits.
//   Residues of multiword integers, scaling of residue planes, and an exact
//   comparison of a residue product with s I (the integrality check).
//   Elimination over Z/q^e with minimal-valuation pivoting, which gives the
//   local Smith form of an integer matrix at the prime q.
//
// Arithmetic modulo a 26-bit prime uses exact doubles (products < 2^52) and
// the rounded reciprocal; modulo q^e < 2^34 the first factor is split at bit 17
// so that every partial product stays below 2^52.
#include "smith_internal.hpp"

namespace rns {
namespace {

__device__ __forceinline__ uint32_t mulmod_p(uint32_t a, uint32_t b, double pf, double pinv) {
    const double x = (double)a * (double)b;
    double r = fma(-rint(x * pinv), pf, x);
    r = r < 0.0 ? r + pf : r;
    return (uint32_t)r;
}

__device__ __forceinline__ uint32_t powmod_p(uint32_t a, uint32_t e, double pf, double pinv) {
    uint32_t r = 1;
    while (e) {
        if (e & 1) r = mulmod_p(r, a, pf, pinv);
        a = mulmod_p(a, a, pf, pinv);
        e >>= 1;
    }
    return r;
}

// Loads A (int64) reduced mod each prime into [A mod p | I] (ld = 2n) or
// A mod p (ld = n).
__global__ __launch_bounds__(256) void k_gj_load(const int64_t *__restrict__ A, int64_t n, int64_t ld,
                                                 uint32_t *__restrict__ M,
                                                 const GjPrime *__restrict__ pr) {
    const int q = blockIdx.z;
    const int64_t i = blockIdx.y;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= ld) return;
    uint32_t v;
    if (j < n) {
        const int64_t x = A[i * n + j];
        const int64_t p = pr[q].p;
        int64_t r = x % p;
        v = (uint32_t)(r < 0 ? r + p : r);
    } else {
        v = (j - n == i) ? 1u : 0u;
    }
    M[((int64_t)q * n + i) * ld + j] = v;
}

// ------------------------------------------ blocked elimination mod p --
// Elimination of P planes M [P][n][ld] in blocks of bw <= kGjBlock columns
// (ld = 2n: Gauss-Jordan on [A | I]; ld = n: forward elimination for the
// determinant).  Per block starting at row and column r0:
//   k_gj_blockinv (mode 0) inverts the block P11 = M[r0.., r0..] without row
//                 exchanges; it succeeds when the leading minors of P11 are
//                 nonzero mod p, which for a 26-bit prime fails only rarely,
//                 and then multiplies det[q] by its pivots; on a zero pivot
//                 it marks the plane in need[q] instead.
//   For the marked planes only:
//   k_gj_panel    eliminates a copy of the block's columns below row r0 with
//                 the first nonzero entry as pivot, recording the row swaps
//                 and multiplying det[q] by the pivots (no pivot: singular);
//   k_gj_swap     applies those swaps to the whole rows of M;
//   k_gj_blockinv (mode 1) inverts the new P11 (its leading minors are the
//                 pivots just found, so no pivoting is needed).
// The driver completes the block with two residue products:
//   pivot rows <- P11^-1 (pivot rows),   other rows -= (their panel) (pivot rows),
// which is Gauss-Jordan (or LU's Schur complement) for bw columns at once.

constexpr int kGjBlockMax = kGjBlock;

__global__ __launch_bounds__(1024) void k_gj_panel(const uint32_t *__restrict__ M, int64_t n, int64_t ld,
                                                   int64_t r0, int bw, const GjPrime *__restrict__ pr,
                                                   uint32_t *__restrict__ S, int32_t *__restrict__ piv,
                                                   int32_t *__restrict__ singular,
                                                   const int32_t *__restrict__ need,
                                                   uint32_t *__restrict__ det) {
    const int q = blockIdx.x;
    if (singular[q] || !need[q]) return;
    const uint32_t *Mq = M + (int64_t)q * n * ld;
    const int64_t rows = n - r0;
    uint32_t *Sq = S + (int64_t)q * n * kGjBlockMax;           // [rows][bw]
    for (int64_t e = threadIdx.x; e < rows * bw; e += blockDim.x) {
        const int64_t i = e / bw;
        const int c = (int)(e - i * bw);
        Sq[e] = Mq[(r0 + i) * ld + r0 + c];
    }
    __syncthreads();
    const double pf = pr[q].pf, pinv = pr[q].pinv;
    const uint32_t p = pr[q].p;
    __shared__ int best;
    __shared__ uint32_t inv;
    for (int j = 0; j < bw; ++j) {
        if (threadIdx.x == 0) best = (int)rows;
        __syncthreads();
        for (int64_t i = j + threadIdx.x; i < rows; i += blockDim.x)
            if (Sq[i * bw + j] != 0) atomicMin(&best, (int)i);
        __syncthreads();
        const int r = best;                                    // the same on every thread
        if (r >= rows) {
            if (threadIdx.x == 0) singular[q] = 1;
            return;
        }
        if (r != j)
            for (int c = threadIdx.x; c < bw; c += blockDim.x) {
                const uint32_t t = Sq[(int64_t)j * bw + c];
                Sq[(int64_t)j * bw + c] = Sq[(int64_t)r * bw + c];
                Sq[(int64_t)r * bw + c] = t;
            }
        __syncthreads();
        if (threadIdx.x == 0) {
            piv[q * kGjBlockMax + j] = (int)(r0 + r);
            const uint32_t pv = Sq[(int64_t)j * bw + j];
            if (det) {
                const uint32_t d = mulmod_p(det[q], pv, pf, pinv);
                det[q] = (r != j && d != 0) ? p - d : d;
            }
            inv = powmod_p(pv, p - 2, pf, pinv);
        }
        __syncthreads();
        const int w = bw - j - 1;                              // columns right of the pivot
        if (w > 0)
            for (int64_t e = threadIdx.x; e < (rows - j - 1) * (int64_t)w; e += blockDim.x) {
                const int64_t i = j + 1 + e / w;
                const int c = j + 1 + (int)(e % w);
                const uint32_t f = Sq[i * bw + j];
                if (f == 0) continue;
                const uint32_t t = mulmod_p(mulmod_p(f, inv, pf, pinv), Sq[(int64_t)j * bw + c], pf, pinv);
                const uint32_t a = Sq[i * bw + c];
                Sq[i * bw + c] = a >= t ? a - t : a + p - t;
            }
        __syncthreads();
    }
}

// Applies the recorded swaps (row r0+j <-> row piv[j], j = 0..bw-1, in order)
// to every column; one thread per column.
__global__ __launch_bounds__(256) void k_gj_swap(uint32_t *__restrict__ M, int64_t n, int64_t ld, int64_t r0,
                                                 int bw, const int32_t *__restrict__ piv,
                                                 const int32_t *__restrict__ singular,
                                                 const int32_t *__restrict__ need) {
    const int q = blockIdx.y;
    if (singular[q] || !need[q]) return;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ld) return;
    uint32_t *Mq = M + (int64_t)q * n * ld;
    for (int j = 0; j < bw; ++j) {
        const int64_t r = piv[q * kGjBlockMax + j];
        if (r != r0 + j) {
            const uint32_t t = Mq[(r0 + j) * ld + c];
            Mq[(r0 + j) * ld + c] = Mq[r * ld + c];
            Mq[r * ld + c] = t;
        }
    }
}

// (a b - f c) mod p for a, b, f, c in [0, p), p < 2^26: both products are
// below 2^52, so the difference is an exact double and one reduction finishes.
__device__ __forceinline__ uint32_t mulsub_p(uint32_t a, uint32_t b, uint32_t f, uint32_t c, double pf,
                                             double pinv) {
    const double x = fma((double)a, (double)b, -((double)f * (double)c));
    double r = fma(-rint(x * pinv), pf, x);
    r = r < 0.0 ? r + pf : r;
    return (uint32_t)r;
}

// W[q] = P11^-1 for the pivot block M[r0.., r0..] (bw x bw) by fraction-free
// Gauss-Jordan on [P11 | I] in LDS without row exchanges: step j leaves the
// pivot row alone and replaces every other row i by pv_j row_i - T[i][j]
// row_j (pv_j = T[j][j]), so no step waits for a modular inverse.  Row i then
// changes only in columns j+1 .. bw+j (beyond them row j is zero) and in its
// own column (its diagonal, i < j, or its unit column bw+i, i > j), which is
// only scaled; column j becomes zero.  At the end the left block is diag(d)
// and the right block R = E (the product of the steps), so P11^-1 = D^-1 R,
// with the bw inverses taken in parallel.  Each step scales bw-1 rows by
// pv_j, so det(P11) = prod d_i / prod_j pv_j^(bw-1).  A zero pivot means a
// zero leading minor, as in the scaled form.  Mode 0 runs on every plane,
// sets need[q] = 0 and multiplies det[q] by det(P11) on success, or sets
// need[q] = 1 on a zero pivot (W is then not used); mode 1 runs on the planes
// with need[q] = 1 after their rows were exchanged (a zero pivot then means
// a singular plane).
__global__ __launch_bounds__(1024) void k_gj_blockinv(const uint32_t *__restrict__ M, int64_t n, int64_t ld,
                                                      int64_t r0, int bw, const GjPrime *__restrict__ pr,
                                                      uint32_t *__restrict__ W, int32_t *__restrict__ singular,
                                                      int32_t *__restrict__ need, uint32_t *__restrict__ det,
                                                      int mode) {
    __shared__ uint32_t T[kGjBlockMax][2 * kGjBlockMax];
    __shared__ uint32_t F[kGjBlockMax];
    __shared__ uint32_t PV[kGjBlockMax];
    __shared__ uint32_t Dinv[kGjBlockMax];
    __shared__ uint32_t red[kGjBlockMax];
    const int q = blockIdx.x;
    if (singular[q] || (mode == 1 && !need[q])) return;
    const uint32_t *Mq = M + (int64_t)q * n * ld;
    const int w2 = 2 * bw;
    for (int e = threadIdx.x; e < bw * w2; e += blockDim.x) {
        const int i = e / w2, c = e % w2;
        T[i][c] = c < bw ? Mq[(r0 + i) * ld + r0 + c] : (uint32_t)(c - bw == i);
    }
    __syncthreads();
    const double pf = pr[q].pf, pinv = pr[q].pinv;
    const uint32_t p = pr[q].p;
    // Thread t updates window column a0 = t % bw of rows i0, i0 + rstep, ...
    // (rstep = threads / bw; the threads beyond rstep * bw stay idle).
    const int rstep = (int)blockDim.x / bw;
    const int a0 = (int)threadIdx.x % bw, i0 = (int)threadIdx.x / bw;
    bool failed = false;
    for (int j = 0; j < bw; ++j) {
        const uint32_t pv = T[j][j];                          // the same on every thread
        if (pv == 0) {
            failed = true;
            break;
        }
        for (int i = threadIdx.x; i < bw; i += blockDim.x) F[i] = T[i][j];
        if (threadIdx.x == 0) PV[j] = pv;
        __syncthreads();
        if (i0 < rstep) {
            const int c = j + 1 + a0;                         // window column, j+1 .. bw+j
            const uint32_t tj = T[j][c];
            for (int i = i0; i < bw; i += rstep)
                if (i != j) T[i][c] = mulsub_p(pv, T[i][c], F[i], tj, pf, pinv);
        }
        for (int i = threadIdx.x; i < bw; i += blockDim.x) {
            if (i == j) continue;
            const int own = i < j ? i : bw + i;               // outside the window above
            T[i][own] = mulmod_p(pv, T[i][own], pf, pinv);
            T[i][j] = 0;
        }
        __syncthreads();
    }
    if (failed) {
        if (threadIdx.x == 0) {
            if (mode == 0) need[q] = 1;
            else singular[q] = 1;                             // cannot happen after k_gj_panel
        }
        return;
    }
    const bool want_det = mode == 0 && det != nullptr;
    for (int i = threadIdx.x; i < bw; i += blockDim.x) {
        const uint32_t d = T[i][i];
        Dinv[i] = powmod_p(d, p - 2, pf, pinv);
        if (want_det) red[i] = mulmod_p(d, powmod_p(PV[i], p - (uint32_t)bw, pf, pinv), pf, pinv);   // d_i pv_i^-(bw-1)
    }
    __syncthreads();
    if (want_det)
        for (int h = 1; h < bw; h *= 2) {                     // product of red[0 .. bw-1] into red[0]
            for (int i = threadIdx.x; i < bw; i += blockDim.x)
                if (i % (2 * h) == 0 && i + h < bw) red[i] = mulmod_p(red[i], red[i + h], pf, pinv);
            __syncthreads();
        }
    if (threadIdx.x == 0) {
        if (mode == 0) {
            need[q] = 0;
            if (want_det) det[q] = mulmod_p(det[q], red[0], pf, pinv);
        }
    }
    uint32_t *Wq = W + (int64_t)q * kGjBlockMax * kGjBlockMax;   // [bw][bw], stride kGjBlockMax
    for (int e = threadIdx.x; e < bw * bw; e += blockDim.x) {
        const int i = e / bw, c = e % bw;
        Wq[i * kGjBlockMax + c] = mulmod_p(Dinv[i], T[i][bw + c], pf, pinv);
    }
}

// ----------------------------------------------------- p-adic lifting --
// Dixon's iteration for A Y = J with C = A^-1 mod p resident: with R_0 = J,
//   X_i = C R_i mod p,   R_{i+1} = (R_i - A X_i) / p   (an exact division),
// so that Y = sum_i X_i p^i in the p-adic integers.  The t right-hand sides
// are stored column by column ([t][n]); one wave handles one row.

constexpr int kLiftMaxT = 16;

// Rows of C and A, and the vectors R, Rm, X, have a padded stride ld (a
// multiple of 4); C and A are zero beyond column n, so every row is read with
// 16-byte loads and the padding contributes nothing.

// Each work-group handles RW consecutive rows; its four waves take one
// quarter of the columns k each and add their sums through LDS at the end.
// Every load of the right-hand sides (from L2) serves RW rows, and splitting
// the columns gives four times as many independent waves as one wave per row
// block would (the launcher takes RW = 1 for small n and up to 4 for large n).

// X[c][r] = sum_k C[r][k] Rm[c][k] mod p.  Each lane sums at most ld/64
// products below 2^52 per row (ld <= 65536 keeps that below 2^62), reduces
// its sums mod p, and the wave adds the 64 reduced sums.
// The residual update's division by p (exact for a correct C): q = num / p
// rounded toward zero, and q mod p in [0, p).  For odd p, v = num p^-1 mod
// 2^64 satisfies v p = num mod 2^64, so when |v| <= lim with lim p < 2^63,
// v p = num exactly and v is the quotient; a correct step's quotients are far
// below lim = min(6.9e18 / p, 2^50), so the integer division runs only where
// the step is wrong (or its quotient is that large), and there it decides
// exactness as before.  Below 2^50, q - p rint(q / p) in doubles is exact:
// the rounding error of q / p stays below 1 / (4p), while q / p lies at
// least 1 / (2p) from every half-integer (p odd); one +p then gives [0, p).
struct LiftDiv {
    uint64_t pinv64;   // p^-1 mod 2^64
    int64_t lim;
    uint32_t p;
    double pf, pinv;
    __device__ explicit LiftDiv(uint32_t p_) : p(p_) {
        uint64_t x = p;                                  // p^-1 mod 2^3 (odd p)
#pragma unroll
        for (int i = 0; i < 5; ++i) x *= 2 - (uint64_t)p * x;   // Newton: 3 -> 6 -> ... -> 96 bits
        pinv64 = x;
        pf = (double)p;
        pinv = 1.0 / pf;
        const double l = 6.9e18 * pinv;
        lim = l < 0x1p50 ? (int64_t)l : ((int64_t)1 << 50);
    }
    // false when p does not divide num
    __device__ __forceinline__ bool div(int64_t num, int64_t &q, uint32_t &qm) const {
        q = (int64_t)((uint64_t)num * pinv64);
        if (q <= lim && q >= -lim) {
            const double qd = (double)q;
            const double r = fma(-rint(qd * pinv), pf, qd);
            qm = (uint32_t)(r < 0.0 ? r + pf : r);
            return true;
        }
        q = num / (int64_t)p;
        const int64_t m = q % (int64_t)p;
        qm = (uint32_t)(m < 0 ? m + (int64_t)p : m);
        return q * (int64_t)p == num;
    }
};

// Step i = *base + off: it reads Rm[i & 1] and R[i & 1], writes its digits to
// Xh + i t ld and the next residuals to the other buffers.  *base lives in
// device memory and is advanced by k_lift_advance after a run of steps, so a
// run of steps (offsets 0, 1, ...) takes the same arguments every time and
// can be replayed from a captured graph.
template <int T, int kLiftRows>
__global__ __launch_bounds__(256) void k_lift_x(const uint32_t *__restrict__ C, int64_t n, int64_t ld,
                                                const uint32_t *__restrict__ Rm0, const uint32_t *__restrict__ Rm1,
                                                int t, uint32_t p, uint32_t *__restrict__ Xh,
                                                const int64_t *__restrict__ base, int off) {
    static_assert(kLiftRows * T <= 64, "one lane of wave 0 per (row, column) in the final sum");
    __shared__ uint64_t part[4][kLiftRows][T];
    const int64_t i_step = *base + off;
    const uint32_t *__restrict__ Rm = (i_step & 1) ? Rm1 : Rm0;
    uint32_t *__restrict__ X = Xh + i_step * t * ld;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * kLiftRows;
    if (r0 >= n) return;                                 // whole work-groups only
    const int64_t q = ld / 4;
    const int64_t kb = q * wave / 4, ke = q * (wave + 1) / 4;
    const uint4 *Cr[kLiftRows];
#pragma unroll
    for (int rr = 0; rr < kLiftRows; ++rr)               // rows past n re-read row r0 and store nothing
        Cr[rr] = reinterpret_cast<const uint4 *>(C + (r0 + rr < n ? r0 + rr : r0) * ld);
    uint64_t acc[kLiftRows][T];
#pragma unroll
    for (int rr = 0; rr < kLiftRows; ++rr)
#pragma unroll
        for (int c = 0; c < T; ++c) acc[rr][c] = 0;
#pragma unroll 2
    for (int64_t k = kb + lane; k < ke; k += 64) {
        uint4 rv[T];
#pragma unroll
        for (int c = 0; c < T; ++c)
            if (c < t) rv[c] = reinterpret_cast<const uint4 *>(Rm + (int64_t)c * ld)[k];
#pragma unroll
        for (int rr = 0; rr < kLiftRows; ++rr) {
            const uint4 cv = Cr[rr][k];
#pragma unroll
            for (int c = 0; c < T; ++c)
                if (c < t)
                    acc[rr][c] += (uint64_t)cv.x * rv[c].x + (uint64_t)cv.y * rv[c].y +
                                  (uint64_t)cv.z * rv[c].z + (uint64_t)cv.w * rv[c].w;
        }
    }
#pragma unroll
    for (int rr = 0; rr < kLiftRows; ++rr)
#pragma unroll
        for (int c = 0; c < T; ++c) {
            if (c < t) {
                uint64_t v = acc[rr][c] % p;
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
                if (lane == 0) part[wave][rr][c] = v;    // below 64 p < 2^32
            }
        }
    __syncthreads();
    if (wave == 0) {
        const int rr = lane / T, c = lane % T;
        if (rr < kLiftRows && c < t && r0 + rr < n) {
            const uint64_t v = part[0][rr][c] + part[1][rr][c] + part[2][rr][c] + part[3][rr][c];
            X[(int64_t)c * ld + r0 + rr] = (uint32_t)(v % p);
        }
    }
}

// --------------------------------------- lifting products on the matrix cores
// X = C Rm mod p is a residue product with at most 16 columns.  C is fixed
// for a whole lifting, so its balanced residues are split once into four
// signed base-256 digits and tiled in the INT8 MFMA operand layout (per
// 16-row block and 64-column step, four 1 KiB fragments, lane l holding row
// l%16 and the 16 columns 16(l/16) .. +15).  Each step splits Rm the same way
// in registers (lane l: right-hand side l%16), or takes it as balanced digit
// fragments written by the residual update, and runs the 16 digit-pair
// products v_mfma_i32_16x16x64_i8 per block and step, summed in int32 per
// shift group s = i+j; the sums of one group over k <= 43690 columns stay
// below 2^31: both operands' digits are balanced (d0..d2 in [-128, 127],
// |d3| <= 2), so a group adds per column at most three products of two full
// digits (3 * 2^14) or two of them and two with a top digit (2^15 + 2^9).

typedef int v4i_l __attribute__((ext_vector_type(4)));

// Balanced signed base-256 digits of a balanced residue |r| <= (p-1)/2 < 2^25:
// r = d0 + 2^8 d1 + 2^16 d2 + 2^24 d3, d0..d2 in [-128, 127], |d3| <= 2.
__device__ __forceinline__ void lift_digits(int32_t r, int32_t (&d)[4]) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        d[i] = (int32_t)(int8_t)(r & 0xFF);
        r = (r - d[i]) >> 8;
    }
    d[3] = r;
}

// Digit fragments of 16 residues x[0..15] in [0, p): byte j of word w of
// fragment i is digit i of x[4w + j].
__device__ __forceinline__ void lift_pack(const uint32_t (&x)[16], uint32_t p, v4i_l (&f)[4]) {
    uint32_t w[4][4] = {};
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int32_t r = x[e] > (p >> 1) ? (int32_t)x[e] - (int32_t)p : (int32_t)x[e];
        int32_t d[4];
        lift_digits(r, d);
#pragma unroll
        for (int i = 0; i < 4; ++i) w[i][e >> 2] |= ((uint32_t)d[i] & 0xFFu) << (8 * (e & 3));
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) f[i] = v4i_l{(int)w[i][0], (int)w[i][1], (int)w[i][2], (int)w[i][3]};
}

// 16 consecutive entries v[k0 .. k0+15] of a padded row (stride ld, a
// multiple of 4): whole 4-entry chunks at or past ld read as zero.
__device__ __forceinline__ void lift_load16(const uint32_t *v, int64_t k0, int64_t ld, bool valid,
                                            uint32_t (&x)[16]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        uint4 u = {0u, 0u, 0u, 0u};
        if (valid && k0 + 4 * q < ld) u = *reinterpret_cast<const uint4 *>(v + k0 + 4 * q);
        x[4 * q] = u.x; x[4 * q + 1] = u.y; x[4 * q + 2] = u.z; x[4 * q + 3] = u.w;
    }
}

// One wave per (64-column step kt, 16-row block rb).
__global__ __launch_bounds__(64) void k_lift_tile_c(const uint32_t *__restrict__ C, int64_t n, int64_t ld,
                                                    uint32_t p, int KT, v4i_l *__restrict__ Ct) {
    const int kt = blockIdx.x;
    const int64_t rb = blockIdx.y;
    const int lane = threadIdx.x;
    const int64_t row = rb * 16 + (lane & 15);
    uint32_t x[16];
    lift_load16(C + row * ld, (int64_t)kt * 64 + 16 * (lane >> 4), ld, row < n, x);
    v4i_l f[4];
    lift_pack(x, p, f);
#pragma unroll
    for (int i = 0; i < 4; ++i) Ct[((rb * KT + kt) * 4 + i) * 64 + lane] = f[i];
}

// (sum_s C_s 2^(8s)) mod p in [0, p) for the seven shift-group sums, every
// step an exact double operation (|C_s| < 2^31): lo and mid below 2^48,
// mid reduced to a balanced residue, then lo + rm (2^24 mod p) + C_6 (2^48
// mod p) below 2^53 with balanced weights, and a final reduction whose
// quotient can be off by one only next to +-p/2 (then one +p fixes it).
__device__ __forceinline__ uint32_t lift_recombine(const int32_t (&c)[7], double pf, double pinv, double w24,
                                                   double w48) {
    const double lo = fma((double)c[2], 65536.0, fma((double)c[1], 256.0, (double)c[0]));
    const double mid = fma((double)c[5], 65536.0, fma((double)c[4], 256.0, (double)c[3]));
    const double rm = fma(-rint(mid * pinv), pf, mid);
    const double sum = fma((double)c[6], w48, fma(rm, w24, lo));
    double r = fma(-rint(sum * pinv), pf, sum);
    r = r < 0.0 ? r + pf : r;
    return (uint32_t)r;
}

// Exact base-256 digits of 16 values x in [0, 2^26): digit fragments as in
// lift_pack, without the reduction to balanced residues.
__device__ __forceinline__ void lift_pack_exact(const uint32_t (&x)[16], v4i_l (&f)[4]) {
    uint32_t w[4][4] = {};
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        int32_t d[4];
        lift_digits((int32_t)x[e], d);
#pragma unroll
        for (int i = 0; i < 4; ++i) w[i][e >> 2] |= ((uint32_t)d[i] & 0xFFu) << (8 * (e & 3));
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) f[i] = v4i_l{(int)w[i][0], (int)w[i][1], (int)w[i][2], (int)w[i][3]};
}

// The right-hand sides of the next product as ready digit fragments: the
// 16 x 16 block of a work-group (tile[c][j] = value of column c at row
// 16 rb + j, rows past n zero) becomes lanes 16 (rb % 4) .. +15 of the four
// digit fragments of 64-row step rb / 4: exact base-256 digits of X for the
// residual update (BAL false), which needs the integer product, balanced
// digits of the balanced residue for C Rm mod p (BAL true, with p), which
// keeps that product's group sums within its bound.  One wave; its LDS
// writes precede these reads in program order.
template <bool BAL>
__device__ __forceinline__ void lift_emit_frag(const uint32_t (&tile)[16][17], int64_t rb, int lane, uint32_t p,
                                               v4i_l *__restrict__ frag) {
    if (lane >= 16) return;
    uint32_t x[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) x[j] = tile[lane][j];
    v4i_l f[4];
    if constexpr (BAL) lift_pack(x, p, f);
    else lift_pack_exact(x, f);
    const int64_t kt = rb >> 2;
    const int slot = (int)(rb & 3) * 16 + lane;
#pragma unroll
    for (int i = 0; i < 4; ++i) frag[(kt * 4 + i) * 64 + slot] = f[i];
}

// Balanced digit fragments of t <= 16 vectors v [t][ld] (entries in [0, p),
// rows past n zero; the first step's Rm for C Rm mod p): one wave per 64-row
// step, lane l taking vector l%16 and rows 16 (l/16) .. +15.
__global__ __launch_bounds__(64) void k_lift_frag(const uint32_t *__restrict__ v, int64_t n, int64_t ld, int t,
                                                  uint32_t p, v4i_l *__restrict__ frag) {
    const int kt = blockIdx.x;
    const int lane = threadIdx.x;
    const int c = lane & 15;
    const int64_t k0 = (int64_t)kt * 64 + 16 * (lane >> 4);
    uint32_t x[16];
    lift_load16(v + (int64_t)(c < t ? c : 0) * ld, k0, ld, c < t, x);
#pragma unroll
    for (int j = 0; j < 16; ++j)
        if (k0 + j >= n) x[j] = 0;
    v4i_l f[4];
    lift_pack(x, p, f);
#pragma unroll
    for (int i = 0; i < 4; ++i) frag[((int64_t)kt * 4 + i) * 64 + lane] = f[i];
}

// X[c][r] = sum_k C[r][k] Rm[c][k] mod p for one 16-row block per work-group;
// its KS waves take KS slices of the 64-column steps and add their int32
// sums in LDS.  Same step indexing as k_lift_x.
template <int KS, bool FRAG>
__global__ __launch_bounds__(64 * KS, 8 / KS) void k_lift_x_mfma(const v4i_l *__restrict__ Ct, int64_t n, int64_t ld,
                                                         int KT, const uint32_t *__restrict__ Rm0,
                                                         const uint32_t *__restrict__ Rm1, int t, uint32_t p,
                                                         uint32_t *__restrict__ Xh,
                                                         const int64_t *__restrict__ base, int off,
                                                         const v4i_l *__restrict__ Rmd, v4i_l *__restrict__ Xd,
                                                         LiftGroups gr) {
    __shared__ v4i_l part[KS][7][64];
    const int64_t rb = blockIdx.x, g = blockIdx.y;     // g: the group's own vectors and buffers
    Rm0 += g * gr.rm;
    Rm1 += g * gr.rm;
    Xh += g * gr.xh;
    Rmd += g * gr.frag;
    Xd += g * gr.frag;
    const int64_t i_step = *base + off;
    const uint32_t *__restrict__ Rm = (i_step & 1) ? Rm1 : Rm0;
    uint32_t *__restrict__ X = Xh + (i_step % gr.ring) * t * ld;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int kt0 = (int)((int64_t)KT * wave / KS), kt1 = (int)((int64_t)KT * (wave + 1) / KS);
    const int c = lane & 15;
    const bool cvalid = c < t;
    const uint32_t *rmc = Rm + (int64_t)(cvalid ? c : 0) * ld;
    const v4i_l *cf = Ct + rb * KT * 256 + lane;
    v4i_l acc[7];
#pragma unroll
    for (int g = 0; g < 7; ++g) acc[g] = v4i_l{0, 0, 0, 0};
    // Fragments of step kt+1 are loaded before the products of step kt.
    v4i_l a[4], b[4], an[4], bn[4];
    auto load = [&](int kt, v4i_l (&ar)[4], v4i_l (&br)[4]) {
#pragma unroll
        for (int i = 0; i < 4; ++i) ar[i] = cf[(int64_t)kt * 256 + i * 64];
        if constexpr (FRAG) {
#pragma unroll
            for (int i = 0; i < 4; ++i) br[i] = Rmd[((int64_t)kt * 4 + i) * 64 + lane];
        } else {
            uint32_t x[16];
            lift_load16(rmc, (int64_t)kt * 64 + 16 * (lane >> 4), ld, cvalid, x);
            lift_pack(x, p, br);
        }
    };
    if (kt0 < kt1) load(kt0, a, b);
    for (int kt = kt0; kt < kt1; ++kt) {
        if (kt + 1 < kt1) load(kt + 1, an, bn);
#pragma unroll
        for (int da = 0; da < 4; ++da)
#pragma unroll
            for (int db = 0; db < 4; ++db)
                acc[da + db] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[da], b[db], acc[da + db], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            a[i] = an[i];
            b[i] = bn[i];
        }
    }
#pragma unroll
    for (int g = 0; g < 7; ++g) part[wave][g][lane] = acc[g];
    __syncthreads();
    if (wave != 0) return;
    __shared__ uint32_t tile16[16][17];
    const double pf = (double)p, pinv = 1.0 / pf;
    const double w24 = fma(-rint(16777216.0 * pinv), pf, 16777216.0);            // 2^24 mod p, balanced
    const double w48 = fma(-rint(281474976710656.0 * pinv), pf, 281474976710656.0);   // 2^48 mod p, balanced
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        int32_t cs[7];
#pragma unroll
        for (int g = 0; g < 7; ++g) {
            int32_t sum = 0;
#pragma unroll
            for (int w = 0; w < KS; ++w) sum += part[w][g][lane][v];
            cs[g] = sum;
        }
        // 16x16x64 INT8 output layout: register v of lane l is row 4(l/16) + v, column l%16.
        const int64_t row = rb * 16 + 4 * (lane >> 4) + v;
        const uint32_t xr = lift_recombine(cs, pf, pinv, w24, w48);
        if (cvalid && row < n) X[(int64_t)c * ld + row] = xr;
        if constexpr (FRAG) tile16[c][4 * (lane >> 4) + v] = (cvalid && row < n) ? xr : 0u;
    }
    if constexpr (FRAG) lift_emit_frag<false>(tile16, rb, lane, p, Xd);
}

// The residual update on the matrix cores, for A held as int16: A splits
// exactly into two signed bytes (a = a0 + 2^8 a1, a0 and a1 in [-128, 127],
// which holds for |a| < 32640), X in [0, p) into four base-256 digits (the
// top one in [0, 4]); each of the 8 digit pairs has its own int32 sum, below
// 2^31 over k <= 65793 columns (|a_i x_j| <= 128 * 255), and
// sum S_ij 2^(8(i+j)) is the exact product sum in int64.  A's digits are tiled once per lifting (two 1 KiB
// fragments per 16-row block and 64-column step).

// One wave per (64-column step kt, 16-row block rb).
__global__ __launch_bounds__(64) void k_lift_tile_a(const int16_t *__restrict__ A, int64_t n, int64_t ld, int KT,
                                                    v4i_l *__restrict__ At) {
    const int kt = blockIdx.x;
    const int64_t rb = blockIdx.y;
    const int lane = threadIdx.x;
    const int64_t row = rb * 16 + (lane & 15);
    const int64_t k0 = (int64_t)kt * 64 + 16 * (lane >> 4);
    uint32_t w[2][4] = {};
#pragma unroll
    for (int h = 0; h < 2; ++h) {                        // 8 entries per 16-byte chunk; ld is a multiple of 8
        int4 u = {0, 0, 0, 0};
        if (row < n && k0 + 8 * h < ld) u = *reinterpret_cast<const int4 *>(A + row * ld + k0 + 8 * h);
        const int32_t q[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int32_t a = (int32_t)(int16_t)((q[e >> 1] >> (16 * (e & 1))) & 0xFFFF);
            const int32_t a0 = (int32_t)(int8_t)(a & 0xFF), a1 = (a - a0) >> 8;
            const int idx = 8 * h + e;                   // entry k0 + idx
            w[0][idx >> 2] |= ((uint32_t)a0 & 0xFFu) << (8 * (idx & 3));
            w[1][idx >> 2] |= ((uint32_t)a1 & 0xFFu) << (8 * (idx & 3));
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
        At[((rb * KT + kt) * 2 + i) * 64 + lane] = v4i_l{(int)w[i][0], (int)w[i][1], (int)w[i][2], (int)w[i][3]};
}

// R'[c][r] = (R[c][r] - sum_k A[r][k] X[c][k]) / p, Rm'[c][r] = R' mod p, for
// one 16-row block per work-group (KS waves over slices of the steps, sums
// added in LDS).  Same step indexing and error flag as k_lift_r.
template <int KS, bool FRAG>
__global__ __launch_bounds__(64 * KS, 8 / KS) void k_lift_r_mfma(const v4i_l *__restrict__ At, int64_t n,
                                                                 int64_t ld, int KT,
                                                                 const uint32_t *__restrict__ Xh,
                                                                 int64_t *__restrict__ R0, int64_t *__restrict__ R1,
                                                                 uint32_t *__restrict__ Rm0,
                                                                 uint32_t *__restrict__ Rm1, int t, uint32_t p,
                                                                 int32_t *__restrict__ err,
                                                                 const int64_t *__restrict__ base, int off,
                                                                 const v4i_l *__restrict__ Xd,
                                                                 v4i_l *__restrict__ Rmd, LiftGroups gr) {
    __shared__ v4i_l part[KS][8][64];
    const int64_t rb = blockIdx.x, g = blockIdx.y;     // g: the group's own vectors and buffers
    R0 += g * gr.r;
    R1 += g * gr.r;
    Rm0 += g * gr.rm;
    Rm1 += g * gr.rm;
    Xh += g * gr.xh;
    Xd += g * gr.frag;
    Rmd += g * gr.frag;
    const int64_t i_step = *base + off;
    const uint32_t *__restrict__ X = Xh + (i_step % gr.ring) * t * ld;
    const int64_t *__restrict__ R = (i_step & 1) ? R1 : R0;
    int64_t *__restrict__ Rn = (i_step & 1) ? R0 : R1;
    uint32_t *__restrict__ Rmn = (i_step & 1) ? Rm0 : Rm1;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int kt0 = (int)((int64_t)KT * wave / KS), kt1 = (int)((int64_t)KT * (wave + 1) / KS);
    const int c = lane & 15;
    const bool cvalid = c < t;
    const uint32_t *xc = X + (int64_t)(cvalid ? c : 0) * ld;
    const v4i_l *af = At + rb * KT * 128 + lane;
    v4i_l acc[8];                                        // acc[4 i + j]: digit pair (a_i, x_j)
#pragma unroll
    for (int g = 0; g < 8; ++g) acc[g] = v4i_l{0, 0, 0, 0};
    // Fragments of step kt+1 are loaded before the products of step kt.
    v4i_l a[2], b[4], an[2], bn[4];
    auto load = [&](int kt, v4i_l (&ar)[2], v4i_l (&br)[4]) {
#pragma unroll
        for (int i = 0; i < 2; ++i) ar[i] = af[(int64_t)kt * 128 + i * 64];
        if constexpr (FRAG) {
#pragma unroll
            for (int i = 0; i < 4; ++i) br[i] = Xd[((int64_t)kt * 4 + i) * 64 + lane];
        } else {
            uint32_t x[16];
            lift_load16(xc, (int64_t)kt * 64 + 16 * (lane >> 4), ld, cvalid, x);
            lift_pack_exact(x, br);
        }
    };
    if (kt0 < kt1) load(kt0, a, b);
    for (int kt = kt0; kt < kt1; ++kt) {
        if (kt + 1 < kt1) load(kt + 1, an, bn);
#pragma unroll
        for (int da = 0; da < 2; ++da)
#pragma unroll
            for (int db = 0; db < 4; ++db)
                acc[4 * da + db] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[da], b[db], acc[4 * da + db], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (i < 2) a[i] = an[i];
            b[i] = bn[i];
        }
    }
#pragma unroll
    for (int g = 0; g < 8; ++g) part[wave][g][lane] = acc[g];
    __syncthreads();
    if (wave != 0) return;
    __shared__ uint32_t tile16[16][17];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        int64_t sum = 0;
#pragma unroll
        for (int g = 0; g < 8; ++g) {
            int32_t sg = 0;
#pragma unroll
            for (int w = 0; w < KS; ++w) sg += part[w][g][lane][v];
            sum += (int64_t)sg << (8 * ((g >> 2) + (g & 3)));
        }
        const int64_t r = rb * 16 + 4 * (lane >> 4) + v;
        uint32_t rm = 0;
        if (cvalid && r < n) {
            const int64_t num = R[(int64_t)c * ld + r] - sum;
            int64_t qq;
            if (!LiftDiv(p).div(num, qq, rm)) atomicOr(err, 1);
            Rn[(int64_t)c * ld + r] = qq;
            Rmn[(int64_t)c * ld + r] = rm;
        }
        if constexpr (FRAG) tile16[c][4 * (lane >> 4) + v] = rm;
    }
    if constexpr (FRAG) lift_emit_frag<true>(tile16, rb, lane, p, Rmd);
}

// ------------------------------------------- grouped lifting, wide items
// The two products of a grouped step with a wider item per work-group: four
// waves, wave w taking the 16-row block 4 rbq + w against the four groups
// 4 gq .. 4 gq + 3 (64 columns) over the whole k range, so each C (or A)
// fragment loaded feeds four groups' MFMAs and no partial sums go through
// LDS.  The four groups' digit fragments of a step (16 KiB, the same for
// every wave of the work-group) are copied once into LDS with 16-byte direct
// loads, wave w copying group 4 gq + w's four, into one of two buffers:
// after a barrier each wave reads them from LDS, starts the copies of the
// next step and loads its own next C (or A) fragments into registers, then
// runs the step's MFMAs.  (Loading them from L2 into every wave's registers
// moved 2.5 times the bytes per MFMA.)  The digit fragments, shift groups,
// int32 bounds and epilogues are those of k_lift_x_mfma and k_lift_r_mfma
// (each column sum is the same sum, accumulated by one wave).  Items (4 row
// blocks x 4 groups) are dealt round-robin to the eight XCDs (work-group w
// runs on XCD w mod 8) in windows of 2 x 2 items, so that a window's C (or A)
// blocks and its groups' digit fragments are fetched into that XCD's L2 once
// and shared; the groups hold full runs of 16 vectors.
__device__ __forceinline__ bool lift_item_wide(const LiftGroups &gr, int64_t &rbq, int64_t &gq) {
    const int64_t R4 = (gr.rbs + 3) / 4, G4 = (gr.groups + 3) / 4;
    const int64_t w = blockIdx.x, xcd = w % 8, i = w / 8;
    constexpr int64_t WR = 2, WG = 2, per = WR * WG;
    const int64_t st = (i / per) * 8 + xcd;
    const int64_t wgs = (G4 + WG - 1) / WG;
    const int64_t within = i % per;
    rbq = (st / wgs) * WR + within / WG;
    gq = (st % wgs) * WG + within % WG;
    return rbq < R4 && gq < G4;
}

typedef __attribute__((address_space(3))) void lds_void_l;

__device__ __forceinline__ void lift_vm_wait_0() { __builtin_amdgcn_s_waitcnt(0x0F70); }   // vmcnt(0)

__device__ __forceinline__ void lift_barrier() {
    // The copies this barrier covers were waited for by every wave; the empty
    // asm statements keep the compiler from moving memory accesses across.
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// The k loop of a wide item: right operands (the groups' 4 digit fragments
// per step, frag_base + g * gr.frag, group 0's standing in for a group past
// the last one, whose sums are never stored) through LDS, this wave's NA
// left fragments per step (a_base, NA * 64 v4i apart per step) straight into
// registers one step ahead; `mfma(a, b)` runs one step's products.
template <int NA, class Mfma>
__device__ __forceinline__ void lift_wide_loop(const v4i_l *__restrict__ a_base, const v4i_l *__restrict__ frag_base,
                                               const LiftGroups &gr, int64_t gq, int KT, int lane, int wave,
                                               v4i_l (*bbuf)[16 * 64], Mfma &&mfma) {
    const int64_t gw = gq * 4 + wave;
    const char *bsrc = reinterpret_cast<const char *>(frag_base + (gw < gr.groups ? gw : 0) * gr.frag + lane);
    auto issue = [&](int buf, int kt) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            __builtin_amdgcn_global_load_lds((const void *)(bsrc + ((int64_t)kt * 4 + i) * 1024),
                                             (lds_void_l *)(&bbuf[buf][(wave * 4 + i) * 64]), 16, 0, 0);
    };
    v4i_l a[NA], an[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) a[i] = a_base[i * 64];
    issue(0, 0);
    for (int kt = 0; kt < KT; ++kt) {
        lift_vm_wait_0();
        lift_barrier();
        v4i_l b[4][4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int i = 0; i < 4; ++i) b[q][i] = bbuf[kt & 1][(q * 4 + i) * 64 + lane];
        if (kt + 1 < KT) {
            issue((kt + 1) & 1, kt + 1);
#pragma unroll
            for (int i = 0; i < NA; ++i) an[i] = a_base[((int64_t)kt + 1) * NA * 64 + i * 64];
        }
        mfma(a, b);
        if (kt + 1 < KT) {
#pragma unroll
            for (int i = 0; i < NA; ++i) a[i] = an[i];
        }
    }
}

__global__ __launch_bounds__(256, 2) void k_lift_x_wide(const v4i_l *__restrict__ Ct, int64_t n, int64_t ld, int KT,
                                                       int t, uint32_t p, uint32_t *__restrict__ Xh,
                                                       const int64_t *__restrict__ base, int off,
                                                       const v4i_l *__restrict__ Rmd, v4i_l *__restrict__ Xd,
                                                       LiftGroups gr) {
    __shared__ uint32_t tile16[4][16][17];
    __shared__ v4i_l bbuf[2][16 * 64];
    int64_t rbq, gq;
    if (!lift_item_wide(gr, rbq, gq)) return;            // the same for every wave of the work-group
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t rb = rbq * 4 + wave;
    // A wave past the last row block takes part in the copies and barriers
    // (on row block 0's fragments) and stores nothing.
    const bool rvalid = rb < gr.rbs;
    const int64_t i_step = *base + off;
    bool gv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) gv[q] = gq * 4 + q < gr.groups;
    const v4i_l *cf = Ct + (rvalid ? rb : 0) * KT * 256 + lane;
    v4i_l acc[4][7];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int g = 0; g < 7; ++g) acc[q][g] = v4i_l{0, 0, 0, 0};
    lift_wide_loop<4>(cf, Rmd, gr, gq, KT, lane, wave, bbuf, [&](const v4i_l (&a)[4], const v4i_l (&b)[4][4]) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int da = 0; da < 4; ++da)
#pragma unroll
                for (int db = 0; db < 4; ++db)
                    acc[q][da + db] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[da], b[q][db], acc[q][da + db], 0, 0, 0);
    });
    if (!rvalid) return;                                 // no barrier below
    const double pf = (double)p, pinv = 1.0 / pf;
    const double w24 = fma(-rint(16777216.0 * pinv), pf, 16777216.0);
    const double w48 = fma(-rint(281474976710656.0 * pinv), pf, 281474976710656.0);
    const int c = lane & 15;
    const bool cvalid = c < t;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (!gv[q]) continue;
        const int64_t g = gq * 4 + q;
        uint32_t *X = Xh + g * gr.xh + (i_step % gr.ring) * t * ld;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            int32_t cs[7];
#pragma unroll
            for (int s = 0; s < 7; ++s) cs[s] = acc[q][s][v];
            const int64_t row = rb * 16 + 4 * (lane >> 4) + v;
            const uint32_t xr = lift_recombine(cs, pf, pinv, w24, w48);
            if (cvalid && row < n) X[(int64_t)c * ld + row] = xr;
            tile16[wave][c][4 * (lane >> 4) + v] = (cvalid && row < n) ? xr : 0u;
        }
        lift_emit_frag<false>(tile16[wave], rb, lane, p, Xd + g * gr.frag);
    }
}

__global__ __launch_bounds__(256, 2) void k_lift_r_wide(const v4i_l *__restrict__ At, int64_t n, int64_t ld, int KT,
                                                       int64_t *__restrict__ R0, int64_t *__restrict__ R1,
                                                       uint32_t *__restrict__ Rm0, uint32_t *__restrict__ Rm1, int t,
                                                       uint32_t p, int32_t *__restrict__ err,
                                                       const int64_t *__restrict__ base, int off,
                                                       const v4i_l *__restrict__ Xd, v4i_l *__restrict__ Rmd,
                                                       LiftGroups gr) {
    __shared__ uint32_t tile16[4][16][17];
    __shared__ v4i_l bbuf[2][16 * 64];
    int64_t rbq, gq;
    if (!lift_item_wide(gr, rbq, gq)) return;            // the same for every wave of the work-group
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t rb = rbq * 4 + wave;
    const bool rvalid = rb < gr.rbs;                     // as in k_lift_x_wide
    const int64_t i_step = *base + off;
    bool gv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) gv[q] = gq * 4 + q < gr.groups;
    const v4i_l *af = At + (rvalid ? rb : 0) * KT * 128 + lane;
    v4i_l acc[4][8];                                     // acc[q][4 i + j]: digit pair (a_i, x_j)
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int g = 0; g < 8; ++g) acc[q][g] = v4i_l{0, 0, 0, 0};
    lift_wide_loop<2>(af, Xd, gr, gq, KT, lane, wave, bbuf, [&](const v4i_l (&a)[2], const v4i_l (&b)[4][4]) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int da = 0; da < 2; ++da)
#pragma unroll
                for (int db = 0; db < 4; ++db)
                    acc[q][4 * da + db] =
                        __builtin_amdgcn_mfma_i32_16x16x64_i8(a[da], b[q][db], acc[q][4 * da + db], 0, 0, 0);
    });
    if (!rvalid) return;                                 // no barrier below
    const int c = lane & 15;
    const bool cvalid = c < t;
    const LiftDiv ldiv(p);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (!gv[q]) continue;
        const int64_t g = gq * 4 + q;
        const int64_t *R = ((i_step & 1) ? R1 : R0) + g * gr.r;
        int64_t *Rn = ((i_step & 1) ? R0 : R1) + g * gr.r;
        uint32_t *Rmn = ((i_step & 1) ? Rm0 : Rm1) + g * gr.rm;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            int64_t sum = 0;
#pragma unroll
            for (int s = 0; s < 8; ++s) sum += (int64_t)acc[q][s][v] << (8 * ((s >> 2) + (s & 3)));
            const int64_t r = rb * 16 + 4 * (lane >> 4) + v;
            uint32_t rm = 0;
            if (cvalid && r < n) {
                const int64_t num = R[(int64_t)c * ld + r] - sum;
                int64_t qq;
                if (!ldiv.div(num, qq, rm)) atomicOr(err, 1);
                Rn[(int64_t)c * ld + r] = qq;
                Rmn[(int64_t)c * ld + r] = rm;
            }
            tile16[wave][c][4 * (lane >> 4) + v] = rm;
        }
        lift_emit_frag<true>(tile16[wave], rb, lane, p, Rmd + g * gr.frag);
    }
}

// ------------------------------- packed right operands for t <= 4 vectors
// With at most four right-hand sides, twelve of the sixteen columns of the
// right operand above would be zero.  The packed fragment puts digit d of
// vector c in column 4 d + c instead (lane l: column l%16, rows
// 16 (l/16) .. +15 of the 64-row step, one 1 KiB fragment per step), so one
// MFMA per digit of the left operand forms every digit pair, each in its
// own output column: a quarter of the products and of the fragment reads.
// Every pair sum is exact in int32 on its own (C Rm: |d_i d_j| <= 2^14 per
// column; A X: <= 128 * 255); the epilogue adds the pairs of a shift group.

// Digit d of 16 values (balanced digits of the balanced residue mod p when
// BAL, exact base-256 digits of values in [0, 2^26) otherwise).
template <bool BAL>
__device__ __forceinline__ v4i_l lift_digit_frag(const uint32_t (&x)[16], uint32_t p, int d) {
    v4i_l f[4];
    if constexpr (BAL) lift_pack(x, p, f);
    else lift_pack_exact(x, f);
    return d == 0 ? f[0] : d == 1 ? f[1] : d == 2 ? f[2] : f[3];
}

// The packed fragment of the 16 x 4 block of a work-group (tile[c][j], rows
// past n and vectors past t zero): lanes 16 (rb % 4) .. +15 of the packed
// fragment of 64-row step rb / 4.  One wave, as lift_emit_frag.
template <bool BAL>
__device__ __forceinline__ void lift_emit_frag_pk(const uint32_t (&tile)[16][17], int64_t rb, int lane, uint32_t p,
                                                  v4i_l *__restrict__ frag) {
    if (lane >= 16) return;
    uint32_t x[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) x[j] = tile[lane & 3][j];
    frag[(rb >> 2) * 64 + (rb & 3) * 16 + lane] = lift_digit_frag<BAL>(x, p, lane >> 2);
}

// Packed balanced fragments of t <= 4 vectors v [t][ld] (entries in [0, p),
// rows past n zero; the first step's Rm): one wave per 64-row step.
__global__ __launch_bounds__(64) void k_lift_frag_pk(const uint32_t *__restrict__ v, int64_t n, int64_t ld, int t,
                                                     uint32_t p, v4i_l *__restrict__ frag) {
    const int kt = blockIdx.x;
    const int lane = threadIdx.x;
    const int c = lane & 3;
    const int64_t k0 = (int64_t)kt * 64 + 16 * (lane >> 4);
    uint32_t x[16];
    lift_load16(v + (int64_t)(c < t ? c : 0) * ld, k0, ld, c < t, x);
#pragma unroll
    for (int j = 0; j < 16; ++j)
        if (k0 + j >= n) x[j] = 0;
    frag[(int64_t)kt * 64 + lane] = lift_digit_frag<true>(x, p, (lane & 15) >> 2);
}

// Sums over the KS waves of the per-wave MFMA results part[w][i][lane] into
// sums[i][row][column] (16 x 16 output layout), spread over all the threads.
template <int KS, int NI>
__device__ __forceinline__ void lift_sum_waves(const v4i_l (&part)[KS][NI][64], int32_t (&sums)[NI][16][17]) {
    for (int q = threadIdx.x; q < NI * 256; q += 64 * KS) {
        const int i = q >> 8, l = (q >> 2) & 63, v = q & 3;
        int32_t sum = 0;
#pragma unroll
        for (int w = 0; w < KS; ++w) sum += part[w][i][l][v];
        sums[i][4 * (l >> 4) + v][l & 15] = sum;
    }
}

// k_lift_x_mfma with packed fragments (t <= 4): X = C Rm mod p for one 16-row
// block per work-group, then X's packed exact fragments for the residual
// update.
template <int KS>
__global__ __launch_bounds__(64 * KS, 8 / KS) void k_lift_x_mfma_pk(const v4i_l *__restrict__ Ct, int64_t n,
                                                            int64_t ld, int KT, int t, uint32_t p,
                                                            uint32_t *__restrict__ Xh,
                                                            const int64_t *__restrict__ base, int off,
                                                            const v4i_l *__restrict__ Rmp,
                                                            v4i_l *__restrict__ Xp) {
    __shared__ v4i_l part[KS][4][64];
    __shared__ int32_t sums[4][16][17];
    __shared__ uint32_t tile16[16][17];
    const int64_t i_step = *base + off;
    uint32_t *__restrict__ X = Xh + i_step * t * ld;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t rb = blockIdx.x;
    const int kt0 = (int)((int64_t)KT * wave / KS), kt1 = (int)((int64_t)KT * (wave + 1) / KS);
    const v4i_l *cf = Ct + rb * KT * 256 + lane;
    v4i_l acc[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) acc[g] = v4i_l{0, 0, 0, 0};
    v4i_l a[4], an[4], b, bn;
    auto load = [&](int kt, v4i_l (&ar)[4], v4i_l &br) {
#pragma unroll
        for (int i = 0; i < 4; ++i) ar[i] = cf[(int64_t)kt * 256 + i * 64];
        br = Rmp[(int64_t)kt * 64 + lane];
    };
    if (kt0 < kt1) load(kt0, a, b);
    for (int kt = kt0; kt < kt1; ++kt) {
        if (kt + 1 < kt1) load(kt + 1, an, bn);
#pragma unroll
        for (int da = 0; da < 4; ++da) acc[da] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[da], b, acc[da], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = an[i];
        b = bn;
    }
#pragma unroll
    for (int g = 0; g < 4; ++g) part[wave][g][lane] = acc[g];
    __syncthreads();
    lift_sum_waves<KS, 4>(part, sums);
    __syncthreads();
    if (wave != 0) return;
    // Lane (row, c) = (lane / 4, lane % 4); column 4 d + c holds the pairs of
    // left digit i with right digit d, shift group i + d.
    const int row = lane >> 2, c = lane & 3;
    int32_t cs[7] = {0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int d = 0; d < 4; ++d) cs[i + d] += sums[i][row][4 * d + c];
    const double pf = (double)p, pinv = 1.0 / pf;
    const double w24 = fma(-rint(16777216.0 * pinv), pf, 16777216.0);            // 2^24 mod p, balanced
    const double w48 = fma(-rint(281474976710656.0 * pinv), pf, 281474976710656.0);   // 2^48 mod p, balanced
    const int64_t grow = rb * 16 + row;
    const bool ok = c < t && grow < n;
    const uint32_t xr = lift_recombine(cs, pf, pinv, w24, w48);
    if (ok) X[(int64_t)c * ld + grow] = xr;
    tile16[c][row] = ok ? xr : 0u;
    lift_emit_frag_pk<false>(tile16, rb, lane, p, Xp);
}

// k_lift_r_mfma with packed fragments (t <= 4): R' = (R - A X) / p and
// Rm' = R' mod p for one 16-row block per work-group, then Rm''s packed
// balanced fragments for the next C Rm.
template <int KS>
__global__ __launch_bounds__(64 * KS, 8 / KS) void k_lift_r_mfma_pk(const v4i_l *__restrict__ At, int64_t n,
                                                            int64_t ld, int KT, const uint32_t *__restrict__ Xh,
                                                            int64_t *__restrict__ R0, int64_t *__restrict__ R1,
                                                            uint32_t *__restrict__ Rm0,
                                                            uint32_t *__restrict__ Rm1, int t, uint32_t p,
                                                            int32_t *__restrict__ err,
                                                            const int64_t *__restrict__ base, int off,
                                                            const v4i_l *__restrict__ Xp,
                                                            v4i_l *__restrict__ Rmp) {
    __shared__ v4i_l part[KS][2][64];
    __shared__ int32_t sums[2][16][17];
    __shared__ uint32_t tile16[16][17];
    const int64_t i_step = *base + off;
    const int64_t *__restrict__ R = (i_step & 1) ? R1 : R0;
    int64_t *__restrict__ Rn = (i_step & 1) ? R0 : R1;
    uint32_t *__restrict__ Rmn = (i_step & 1) ? Rm0 : Rm1;
    (void)Xh;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t rb = blockIdx.x;
    const int kt0 = (int)((int64_t)KT * wave / KS), kt1 = (int)((int64_t)KT * (wave + 1) / KS);
    const v4i_l *af = At + rb * KT * 128 + lane;
    v4i_l acc[2] = {v4i_l{0, 0, 0, 0}, v4i_l{0, 0, 0, 0}};
    v4i_l a[2], an[2], b, bn;
    auto load = [&](int kt, v4i_l (&ar)[2], v4i_l &br) {
#pragma unroll
        for (int i = 0; i < 2; ++i) ar[i] = af[(int64_t)kt * 128 + i * 64];
        br = Xp[(int64_t)kt * 64 + lane];
    };
    if (kt0 < kt1) load(kt0, a, b);
    for (int kt = kt0; kt < kt1; ++kt) {
        if (kt + 1 < kt1) load(kt + 1, an, bn);
#pragma unroll
        for (int da = 0; da < 2; ++da) acc[da] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[da], b, acc[da], 0, 0, 0);
        a[0] = an[0];
        a[1] = an[1];
        b = bn;
    }
    part[wave][0][lane] = acc[0];
    part[wave][1][lane] = acc[1];
    __syncthreads();
    lift_sum_waves<KS, 2>(part, sums);
    __syncthreads();
    if (wave != 0) return;
    const int row = lane >> 2, c = lane & 3;
    int64_t sum = 0;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int d = 0; d < 4; ++d) sum += (int64_t)sums[i][row][4 * d + c] << (8 * (i + d));
    const int64_t grow = rb * 16 + row;
    uint32_t rm = 0;
    if (c < t && grow < n) {
        const int64_t num = R[(int64_t)c * ld + grow] - sum;
        int64_t qq;
        if (!LiftDiv(p).div(num, qq, rm)) atomicOr(err, 1);
        Rn[(int64_t)c * ld + grow] = qq;
        Rmn[(int64_t)c * ld + grow] = rm;
    }
    tile16[c][row] = rm;
    lift_emit_frag_pk<true>(tile16, rb, lane, p, Rmp);
}

// R'[c][r] = (R[c][r] - sum_k A[r][k] X[c][k]) / p and Rm'[c][r] = R' mod p.
// The host admits this form only when n max|a| p < 2^62, so every sum fits in
// an int64.  A division that is not exact (impossible for a correct C) sets
// *err instead of producing a wrong residual silently.  X beyond row n is
// never written; A's zero columns make its value irrelevant.  A is int32, or
// int16 when every |a| < 32640 (a quarter less traffic per step); either way
// one 16-byte load per lane and step of the loop.
template <typename AT>
__device__ __forceinline__ void unpack_a(const int4 raw, int32_t (&a)[16 / sizeof(AT)]) {
    if constexpr (sizeof(AT) == 4) {
        a[0] = raw.x; a[1] = raw.y; a[2] = raw.z; a[3] = raw.w;
    } else {
        const int32_t w[4] = {raw.x, raw.y, raw.z, raw.w};
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            a[2 * h] = (int32_t)(int16_t)(w[h] & 0xFFFF);
            a[2 * h + 1] = w[h] >> 16;
        }
    }
}

// One step of k_lift_r for the rows r0 .. r0+kLiftRows-1 of one work-group:
// wave w sums the columns of its quarter, the four sums meet in LDS.
template <int T, int kLiftRows, typename AT>
__global__ __launch_bounds__(256) void k_lift_r(const AT *__restrict__ A, int64_t n, int64_t ld,
                                                const uint32_t *__restrict__ Xh,
                                                int64_t *__restrict__ R0, int64_t *__restrict__ R1,
                                                uint32_t *__restrict__ Rm0, uint32_t *__restrict__ Rm1,
                                                int t, uint32_t p, int32_t *__restrict__ err,
                                                const int64_t *__restrict__ base, int off) {
    static_assert(kLiftRows * T <= 64, "one lane of wave 0 per (row, column) in the final sum");
    constexpr int kPer = 16 / (int)sizeof(AT);   // entries of A per 16-byte load
    __shared__ int64_t part[4][kLiftRows][T];
    const int64_t i_step = *base + off;
    const uint32_t *__restrict__ X = Xh + i_step * t * ld;
    const int64_t *__restrict__ R = (i_step & 1) ? R1 : R0;
    int64_t *__restrict__ Rn = (i_step & 1) ? R0 : R1;
    uint32_t *__restrict__ Rmn = (i_step & 1) ? Rm0 : Rm1;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * kLiftRows;
    if (r0 >= n) return;                                 // whole work-groups only
    const int64_t q = ld / kPer;
    const int64_t kb = q * wave / 4, ke = q * (wave + 1) / 4;
    const int4 *Ar[kLiftRows];
#pragma unroll
    for (int rr = 0; rr < kLiftRows; ++rr)
        Ar[rr] = reinterpret_cast<const int4 *>(A + (r0 + rr < n ? r0 + rr : r0) * ld);
    int64_t acc[kLiftRows][T];
#pragma unroll
    for (int rr = 0; rr < kLiftRows; ++rr)
#pragma unroll
        for (int c = 0; c < T; ++c) acc[rr][c] = 0;
#pragma unroll 2
    for (int64_t k = kb + lane; k < ke; k += 64) {
        uint32_t xv[T][kPer];
#pragma unroll
        for (int c = 0; c < T; ++c)
            if (c < t) {
#pragma unroll
                for (int h = 0; h < kPer / 4; ++h) {
                    const uint4 v = reinterpret_cast<const uint4 *>(X + (int64_t)c * ld)[k * (kPer / 4) + h];
                    xv[c][4 * h] = v.x; xv[c][4 * h + 1] = v.y; xv[c][4 * h + 2] = v.z; xv[c][4 * h + 3] = v.w;
                }
            }
#pragma unroll
        for (int rr = 0; rr < kLiftRows; ++rr) {
            int32_t av[kPer];
            unpack_a<AT>(Ar[rr][k], av);
#pragma unroll
            for (int c = 0; c < T; ++c)
                if (c < t) {
                    int64_t sum = 0;
#pragma unroll
                    for (int e = 0; e < kPer; ++e) sum += (int64_t)av[e] * xv[c][e];
                    acc[rr][c] += sum;
                }
        }
    }
#pragma unroll
    for (int rr = 0; rr < kLiftRows; ++rr)
#pragma unroll
        for (int c = 0; c < T; ++c) {
            if (c >= t) continue;
            int64_t v = acc[rr][c];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
            if (lane == 0) part[wave][rr][c] = v;
        }
    __syncthreads();
    if (wave == 0) {
        const int rr = lane / T, c = lane % T;
        const int64_t r = r0 + rr;
        if (rr < kLiftRows && c < t && r < n) {
            const int64_t v = part[0][rr][c] + part[1][rr][c] + part[2][rr][c] + part[3][rr][c];
            const int64_t num = R[(int64_t)c * ld + r] - v;
            int64_t qq;
            uint32_t rm;
            if (!LiftDiv(p).div(num, qq, rm)) atomicOr(err, 1);
            Rn[(int64_t)c * ld + r] = qq;
            Rmn[(int64_t)c * ld + r] = rm;
        }
    }
}

// *base += steps (one thread), after a run of steps.
// *flag = 1 if any of the count entries lies outside (-32640, 32640), the
// range whose entries split into two signed bytes a0 + 2^8 a1 (a plain store:
// every writer writes 1).
__global__ __launch_bounds__(256) void k_range16(const int64_t *__restrict__ A, int64_t count,
                                                 int32_t *__restrict__ flag) {
    bool out = false;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < count; e += (int64_t)gridDim.x * 256) {
        const int64_t v = A[e];
        out |= v <= -32640 || v >= 32640;
    }
    if (out) *flag = 1;
}

// The n x n int64 matrix as rows of ld entries of T (the caller has checked
// that every entry fits T), zero in the padding columns.
template <typename T>
__global__ __launch_bounds__(256) void k_pack_rows(const int64_t *__restrict__ A, int64_t n, int64_t ld,
                                                   T *__restrict__ out) {
    const int64_t total = n * ld;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t i = e / ld, j = e - i * ld;
        out[e] = j < n ? (T)A[i * n + j] : (T)0;
    }
}

__global__ void k_lift_advance(int64_t *__restrict__ base, int steps) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *base += steps;
}

// Projections of stored digits: Z[i][a][c] = sum_r Rp[a][r] Xh[i][c][r] for
// steps i in [i0, i1), a < tp, c < t, r < n (digit vectors have stride ld).
// One block per (step, column); each thread sums a strided share of the rows,
// then the block adds the shares.  |Rp| <= 2^8 and X < 2^26, so the sums
// stay far inside int64.
__global__ __launch_bounds__(256) void k_lift_proj(const uint32_t *__restrict__ Xh, int64_t n, int64_t ld,
                                                   int t, const int32_t *__restrict__ Rp, int tp,
                                                   int64_t i0, int64_t *__restrict__ Z) {
    const int64_t i = i0 + blockIdx.x / t;
    const int c = blockIdx.x % t;
    const uint32_t *x = Xh + (i * t + c) * ld;
    int64_t acc[kLiftMaxT + 2];
    for (int a = 0; a < tp; ++a) acc[a] = 0;
    for (int64_t r = threadIdx.x; r < n; r += blockDim.x) {
        const int64_t xv = x[r];
        for (int a = 0; a < tp; ++a) acc[a] += (int64_t)Rp[(int64_t)a * n + r] * xv;
    }
    __shared__ int64_t red[256];
    for (int a = 0; a < tp; ++a) {
        red[threadIdx.x] = acc[a];
        __syncthreads();
        for (int s2 = 128; s2 > 0; s2 >>= 1) {
            if ((int)threadIdx.x < s2) red[threadIdx.x] += red[threadIdx.x + s2];
            __syncthreads();
        }
        if (threadIdx.x == 0) Z[((i - i0) * tp + a) * t + c] = red[0];
        __syncthreads();
    }
}

// Multiply plane q of a residue matrix (rows x cols, leading dimension ld,
// planes plane_stride apart) by c[q] mod p_q.
__global__ __launch_bounds__(256) void k_scale(uint32_t *__restrict__ R, int64_t rows, int64_t cols,
                                               int64_t ld, int64_t plane_stride,
                                               const GjPrime *__restrict__ pr,
                                               const uint32_t *__restrict__ c) {
    const int q = blockIdx.z;
    const int64_t i = blockIdx.y;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= cols) return;
    uint32_t *x = R + q * plane_stride + i * ld + j;
    *x = mulmod_p(*x, c[q], pr[q].pf, pr[q].pinv);
}

// Residues of W-word two's-complement integers modulo L primes:
// out[j*count + e] = x_e mod p_j.  x = sum_w u_w 2^(64w) - [neg] 2^(64W);
// the value is accumulated word by word with Horner's rule in exact doubles.
// One thread per entry and prime (grid.y = prime).
__global__ __launch_bounds__(256) void k_words_mod(const uint64_t *__restrict__ x, int64_t count,
                                                   int W, const GjPrime *__restrict__ pr,
                                                   uint32_t *__restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    const uint64_t *xe = x + e * W;
    const bool neg = (xe[W - 1] >> 63) != 0;
    {
        const int j = blockIdx.y;
        const double pf = pr[j].pf, pinv = pr[j].pinv;
        double r = 0.0;
        for (int w = W - 1; w >= 0; --w) {
            const uint64_t u = xe[w];
            // r = r * 2^64 + u  (mod p) as three exact steps of 20, 22 and 22
            // bits (r < 2^26, so every intermediate stays below 2^48).
            double y = fma(r, 1048576.0, (double)(u >> 44));
            y = fma(-rint(y * pinv), pf, y);
            y = y < 0.0 ? y + pf : y;
            y = fma(y, 4194304.0, (double)((u >> 22) & 0x3FFFFF));
            y = fma(-rint(y * pinv), pf, y);
            y = y < 0.0 ? y + pf : y;
            y = fma(y, 4194304.0, (double)(u & 0x3FFFFF));
            y = fma(-rint(y * pinv), pf, y);
            r = y < 0.0 ? y + pf : y;
        }
        if (neg) {                               // subtract 2^(64W) mod p
            double y = r - pr[j].pow64w;
            r = y < 0.0 ? y + pf : y;
        }
        out[(int64_t)j * count + e] = (uint32_t)r;
    }
}

// Counts entries of the residue product P (planes [L][n][n]) that differ from
// s I modulo the plane's prime: expected s mod p on the diagonal, 0 elsewhere.
__global__ __launch_bounds__(256) void k_check_sI(const uint32_t *__restrict__ P, int64_t n,
                                                  const uint32_t *__restrict__ s_mod,
                                                  unsigned *__restrict__ mismatches) {
    const int q = blockIdx.z;
    const int64_t i = blockIdx.y;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const uint32_t want = (i == j) ? s_mod[q] : 0u;
    if (P[((int64_t)q * n + i) * n + j] != want) atomicAdd(mismatches, 1u);
}

// ------------------------------------------------ local Smith form at q --
// M: n x n uint64 entries in [0, m), m = q^e < 2^34.

__device__ __forceinline__ uint64_t mod_m(double x, double mf, double minv) {
    double r = fma(-rint(x * minv), mf, x);     // x < 2^53 -> exact, |r| <= m/2 + 1
    r = r < 0.0 ? r + mf : r;
    return (uint64_t)r;
}

__device__ __forceinline__ uint64_t mulmod_m(uint64_t a, uint64_t b, double mf, double minv) {
    const double b_ = (double)b;
    const uint64_t hi = mod_m((double)(a >> 17) * b_, mf, minv);          // < 2^51 before reduction
    return mod_m(fma((double)hi, 131072.0, (double)(a & 0x1FFFF) * b_), mf, minv);
}

// x / q and (through r) x mod q for x < 2^53: one double product with
// qinv = RN(1/q) is within 2^-19 of x / q for x < 2^34, so the truncated
// quotient is off by at most one and one correction fixes it.
__device__ __forceinline__ uint64_t divmod_q(uint64_t x, uint32_t q, double qinv, uint64_t &r) {
    int64_t t = (int64_t)((double)x * qinv);
    int64_t rr = (int64_t)x - t * (int64_t)q;
    if (rr < 0) {
        rr += q;
        --t;
    } else if (rr >= (int64_t)q) {
        rr -= q;
        ++t;
    }
    r = (uint64_t)rr;
    return (uint64_t)t;
}
__device__ __forceinline__ int valuation(uint64_t x, uint32_t q, double qinv, int e) {
    if (x == 0) return e;
    int v = 0;
    while (v < e) {
        uint64_t r;
        const uint64_t t = divmod_q(x, q, qinv, r);
        if (r) break;
        x = t;
        ++v;
    }
    return v;
}
// x / q^v for x divisible by q^v.
__device__ __forceinline__ uint64_t div_qpow(uint64_t x, uint32_t q, double qinv, int v) {
    for (int t = 0; t < v; ++t) {
        uint64_t r;
        x = divmod_q(x, q, qinv, r);
    }
    return x;
}

// X (W words per entry, two's complement) -> X mod m.
__global__ __launch_bounds__(256) void k_words_mod_m(const uint64_t *__restrict__ x, int64_t count,
                                                     int W, LocalMod lm, uint64_t *__restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    const uint64_t *xe = x + e * W;
    uint64_t r = 0;
    for (int w = W - 1; w >= 0; --w) {
        const uint64_t u = xe[w];
        // r = r * 2^64 + u mod m, in 16-bit steps (r < 2^34: r * 2^16 < 2^50)
        for (int t = 3; t >= 0; --t)
            r = mod_m(fma((double)r, 65536.0, (double)((u >> (16 * t)) & 0xFFFF)), lm.mf, lm.minv);
    }
    if ((xe[W - 1] >> 63) != 0) r = r >= lm.pow64w ? r - lm.pow64w : r + lm.m - lm.pow64w;
    out[e] = r;
}

// The F prime powers q^e of s are eliminated together: plane f of M
// ([F][n][n]) holds X mod lms[f].m, and step k of every plane runs in the
// same two launches.  The pivot of step k is the entry of least valuation in
// rows and columns k..n-1 (the smallest key (valuation << 40) | flat index);
// the keys of step k+1 are gathered by step k's elimination, which visits
// exactly that region, with one 64-bit atomicMin per block into key[f][k+1]
// (every key starts at ~0).

__device__ __forceinline__ uint64_t loc_key(uint64_t x, const LocalMod &lm, double qinv, int64_t flat) {
    return ((uint64_t)valuation(x, lm.q, qinv, lm.e) << 40) | (uint64_t)flat;
}

// Block minimum of one key per thread (every thread of the block calls it),
// then one atomicMin into *dst.
__device__ __forceinline__ void block_min_to(uint64_t key, uint64_t *dst) {
    __shared__ uint64_t red[256];
    red[threadIdx.x] = key;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s && red[threadIdx.x + s] < red[threadIdx.x]) red[threadIdx.x] = red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0 && red[0] != ~0ull)
        atomicMin(reinterpret_cast<unsigned long long *>(dst), (unsigned long long)red[0]);
}

// Keys of step 0: the whole of every plane.  Grid (blocks, F).
__global__ __launch_bounds__(256) void k_loc_init(const uint64_t *__restrict__ M, int64_t n,
                                                  const LocalMod *__restrict__ lms, uint64_t *__restrict__ key) {
    const int f = blockIdx.y;
    const LocalMod lm = lms[f];
    const uint64_t *Mf = M + (int64_t)f * n * n;
    const double qinv = 1.0 / (double)lm.q;
    uint64_t best = ~0ull;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n * n; t += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t kk = loc_key(Mf[t], lm, qinv, t);
        best = kk < best ? kk : best;
    }
    block_min_to(best, key + (int64_t)f * (n + 1));
}

__device__ uint64_t inv_unit(uint64_t u, uint64_t m) {   // u a unit mod m (m < 2^34)
    int64_t t0 = 0, t1 = 1;
    int64_t r0 = (int64_t)m, r1 = (int64_t)u;
    while (r1) {
        const int64_t qq = r0 / r1;
        int64_t tmp = r0 - qq * r1;
        r0 = r1;
        r1 = tmp;
        tmp = t0 - qq * t1;
        t0 = t1;
        t1 = tmp;
    }
    return (uint64_t)(t0 < 0 ? t0 + (int64_t)m : t0);
}

// Step k, pivot: record the valuation and swap the pivot (r, c) into (k, k),
// rows k and r and columns k and c of the whole plane, with one thread per
// index t < n: the row pair at column t (t not k or c), the column pair at
// row t (t not k or r), and thread k the four entries of rows {k, r} and
// columns {k, c} (M'[i][j] = M[sigma(i)][tau(j)] there; r = k or c = k make
// it the one swap that applies).  Each entry has one owner, which reads it
// before writing it.  Thread k, which places the pivot, also stores the
// inverse of its unit part in uinv[f]; the elimination scales row k by it as
// it reads the row.  Grid (ceil(n / 256), F).
__global__ __launch_bounds__(256) void k_loc_swap(uint64_t *__restrict__ M, int64_t n, int k,
                                                  const LocalMod *__restrict__ lms,
                                                  const uint64_t *__restrict__ keys, int32_t *__restrict__ val,
                                                  uint64_t *__restrict__ uinv) {
    const int f = blockIdx.y;
    const LocalMod lm = lms[f];
    const uint64_t key = keys[(int64_t)f * (n + 1) + k];
    const int v = key == ~0ull ? lm.e : (int)(key >> 40);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) val[(int64_t)f * n + k] = v;
    if (v >= lm.e || t >= n) return;                    // the rest is 0 mod m
    uint64_t *Mf = M + (int64_t)f * n * n;
    const int64_t flat = (int64_t)(key & ((1ull << 40) - 1));
    const int64_t r = flat / n, c = flat % n;
    if (t == k) {
        const uint64_t kk = Mf[(int64_t)k * n + k], kc = Mf[(int64_t)k * n + c];
        const uint64_t rk = Mf[r * n + k], rc = Mf[r * n + c];
        Mf[(int64_t)k * n + k] = rc;
        Mf[(int64_t)k * n + c] = rk;
        Mf[r * n + k] = kc;
        Mf[r * n + c] = kk;
        const uint64_t piv = div_qpow(rc, lm.q, 1.0 / (double)lm.q, v);   // the new M[k][k], unit part
        uinv[f] = inv_unit(piv % lm.m, lm.m);
        return;
    }
    if (r != k && t != c) {
        const uint64_t x = Mf[(int64_t)k * n + t];
        Mf[(int64_t)k * n + t] = Mf[r * n + t];
        Mf[r * n + t] = x;
    }
    if (c != k && t != r) {
        const uint64_t x = Mf[t * n + k];
        Mf[t * n + k] = Mf[t * n + c];
        Mf[t * n + c] = x;
    }
}

// Step k, elimination: rows i > k, row_i -= (M[i][k] / q^v) row_k on columns
// > k, and the keys of the updated region into key[f][k+1].  A block covers
// 256 columns of kLocRows rows.  Grid (column blocks, row groups, F).
constexpr int kLocRows = 8;

__global__ __launch_bounds__(256) void k_loc_elim(uint64_t *__restrict__ M, int64_t n, int k,
                                                  const LocalMod *__restrict__ lms, const int32_t *__restrict__ val,
                                                  const uint64_t *__restrict__ uinv, uint64_t *__restrict__ keys) {
    const int f = blockIdx.z;
    const LocalMod lm = lms[f];
    const int v = val[(int64_t)f * n + k];
    if (v >= lm.e) return;                  // uniform over the block
    uint64_t *Mf = M + (int64_t)f * n * n;
    const int64_t j = k + 1 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool colv = j < n;
    const double qinv = 1.0 / (double)lm.q;
    // Row k scaled so that the pivot is q^v.
    const uint64_t pk = colv ? mulmod_m(Mf[(int64_t)k * n + j], uinv[f], lm.mf, lm.minv) : 0;
    uint64_t best = ~0ull;
    for (int rr = 0; rr < kLocRows; ++rr) {
        const int64_t i = k + 1 + (int64_t)blockIdx.y * kLocRows + rr;
        if (i >= n || !colv) continue;
        uint64_t fct = Mf[i * n + k];
        uint64_t a = Mf[i * n + j];
        if (fct != 0) {
            fct = div_qpow(fct, lm.q, qinv, v);          // < m already
            const uint64_t d = mulmod_m(fct, pk, lm.mf, lm.minv);
            a = a >= d ? a - d : a + lm.m - d;
            Mf[i * n + j] = a;
        }
        const uint64_t kk = loc_key(a, lm, qinv, i * n + j);
        best = kk < best ? kk : best;
    }
    block_min_to(best, keys + (int64_t)f * (n + 1) + k + 1);
}

}  // namespace

// ------------------------------------------------------------- launchers --

void launch_gj_load(const int64_t *A, int64_t n, int64_t ld, uint32_t *M, const GjPrime *pr, int P,
                    hipStream_t s) {
    ProfScope trace_(tl_trace, "k_gj_load", s);
    dim3 grid((unsigned)((ld + 255) / 256), (unsigned)n, (unsigned)P);
    hipLaunchKernelGGL(k_gj_load, grid, dim3(256), 0, s, A, n, ld, M, pr);
}


// Work-groups of a grouped lifting launch: lift_item_wide's windows, padded
// to a multiple of eight windows.
unsigned lift_grid_wide(unsigned rbs, const LiftGroups &gr) {
    const int64_t r4 = (rbs + 3) / 4, g4 = (gr.groups + 3) / 4;
    const int64_t windows = (((r4 + 1) / 2) * ((g4 + 1) / 2) + 7) / 8 * 8;
    return (unsigned)(windows * 4);
}
LiftGroups lift_groups(unsigned rbs, LiftGroups gr) {
    gr.rbs = rbs;
    return gr;
}

template <int T, int RW, typename AT>
static void lift_step_t(const uint32_t *C, const AT *A, int64_t n, int64_t ld, int t, uint32_t p,
                        const LiftBufs &b, int off, hipStream_t s) {
    const unsigned blocks = (unsigned)((n + RW - 1) / RW);   // one work-group per RW rows
    // With both operands tiled the two products pass each other their right
    // operands as digit fragments (Xd, Rmd); with C alone the first product
    // splits Rm itself.
    const bool frag = b.Ct && b.At && sizeof(AT) == 2 && b.Xd && b.Rmd;
    const v4i_l *rmd = reinterpret_cast<const v4i_l *>(b.Rmd);
    v4i_l *xd = reinterpret_cast<v4i_l *>(b.Xd);
    if (frag && lift_packed(t)) {                          // both products with packed fragments
        const int KT = (int)((n + 63) / 64);
        const unsigned rbs = (unsigned)((n + 15) / 16);
        hipLaunchKernelGGL((k_lift_x_mfma_pk<8>), dim3(rbs), dim3(512), 0, s,
                           reinterpret_cast<const v4i_l *>(b.Ct), n, ld, KT, t, p, b.Xh, b.base, off, rmd, xd);
        hipLaunchKernelGGL((k_lift_r_mfma_pk<8>), dim3(rbs), dim3(512), 0, s,
                           reinterpret_cast<const v4i_l *>(b.At), n, ld, KT, b.Xh, b.R0, b.R1, b.Rm0, b.Rm1, t, p,
                           b.err, b.base, off, reinterpret_cast<const v4i_l *>(b.Xd),
                           reinterpret_cast<v4i_l *>(b.Rmd));
        return;
    }
    if (b.Ct) {
        const int KT = (int)((n + 63) / 64);
        const unsigned rbs = (unsigned)((n + 15) / 16);
        const v4i_l *ct = reinterpret_cast<const v4i_l *>(b.Ct);
        // Eight waves per 16-row block, two work-groups per CU.
        // Grouped launches: four row blocks x four groups per work-group.
        if (frag && b.grp.groups > 1)
            hipLaunchKernelGGL(k_lift_x_wide, dim3(lift_grid_wide(rbs, b.grp)), dim3(256), 0, s, ct, n, ld, KT, t, p,
                               b.Xh, b.base, off, rmd, xd, lift_groups(rbs, b.grp));
        else if (frag)
            hipLaunchKernelGGL((k_lift_x_mfma<8, true>), dim3(rbs), dim3(512), 0, s, ct, n, ld, KT, b.Rm0, b.Rm1, t,
                               p, b.Xh, b.base, off, rmd, xd, LiftGroups{});
        else
            hipLaunchKernelGGL((k_lift_x_mfma<8, false>), dim3(rbs), dim3(512), 0, s, ct, n, ld, KT, b.Rm0, b.Rm1, t,
                               p, b.Xh, b.base, off, rmd, xd, LiftGroups{});
    } else {
        hipLaunchKernelGGL((k_lift_x<T, RW>), dim3(blocks), dim3(256), 0, s, C, n, ld, b.Rm0, b.Rm1, t, p, b.Xh,
                           b.base, off);
    }
    if (b.At && sizeof(AT) == 2) {
        const int KT = (int)((n + 63) / 64);
        const unsigned rbs = (unsigned)((n + 15) / 16);
        const v4i_l *at = reinterpret_cast<const v4i_l *>(b.At);
        const v4i_l *xdc = reinterpret_cast<const v4i_l *>(b.Xd);
        v4i_l *rmdw = reinterpret_cast<v4i_l *>(b.Rmd);
        if (frag && b.grp.groups > 1)
            hipLaunchKernelGGL(k_lift_r_wide, dim3(lift_grid_wide(rbs, b.grp)), dim3(256), 0, s, at, n, ld, KT, b.R0,
                               b.R1, b.Rm0, b.Rm1, t, p, b.err, b.base, off, xdc, rmdw, lift_groups(rbs, b.grp));
        else if (frag)
            hipLaunchKernelGGL((k_lift_r_mfma<8, true>), dim3(rbs), dim3(512), 0, s, at, n, ld, KT, b.Xh, b.R0,
                               b.R1, b.Rm0, b.Rm1, t, p, b.err, b.base, off, xdc, rmdw, LiftGroups{});
        else
            hipLaunchKernelGGL((k_lift_r_mfma<8, false>), dim3(rbs), dim3(512), 0, s, at, n, ld, KT, b.Xh, b.R0,
                               b.R1, b.Rm0, b.Rm1, t, p, b.err, b.base, off, xdc, rmdw, LiftGroups{});
    } else {
        hipLaunchKernelGGL((k_lift_r<T, RW, AT>), dim3(blocks), dim3(256), 0, s, A, n, ld, b.Xh, b.R0, b.R1,
                           b.Rm0, b.Rm1, t, p, b.err, b.base, off);
    }
}

template <int T, typename AT>
static void lift_step_rw(const uint32_t *C, const AT *A, int64_t n, int64_t ld, int t, uint32_t p,
                         const LiftBufs &b, int off, hipStream_t s) {
    // Rows per work-group: more for large n, where the work-groups are many
    // anyway and each right-hand-side load then serves more rows.
    if (n >= 4 * 2048) lift_step_t<T, 4, AT>(C, A, n, ld, t, p, b, off, s);
    else if (n >= 2 * 2048) lift_step_t<T, 2, AT>(C, A, n, ld, t, p, b, off, s);
    else lift_step_t<T, 1, AT>(C, A, n, ld, t, p, b, off, s);
}

template <typename AT>
static void lift_step_at(const uint32_t *C, const AT *A, int64_t n, int64_t ld, int t, uint32_t p,
                         const LiftBufs &b, int off, hipStream_t s) {
    if (t <= 4) lift_step_rw<4, AT>(C, A, n, ld, t, p, b, off, s);
    else if (t <= 8) lift_step_rw<8, AT>(C, A, n, ld, t, p, b, off, s);
    else lift_step_rw<kLiftMaxT, AT>(C, A, n, ld, t, p, b, off, s);
}

size_t lift_tile_c_bytes(int64_t n) { return (size_t)((n + 15) / 16) * (size_t)((n + 63) / 64) * 4096; }

void launch_lift_tile_c(const uint32_t *C, int64_t n, int64_t ld, uint32_t p, char *Ct, hipStream_t s) {
    if (n <= 0) return;
    ProfScope trace_(tl_trace, "k_lift_tile_c", s);
    const int KT = (int)((n + 63) / 64);
    hipLaunchKernelGGL(k_lift_tile_c, dim3((unsigned)KT, (unsigned)((n + 15) / 16)), dim3(64), 0, s, C, n, ld, p,
                       KT, reinterpret_cast<v4i_l *>(Ct));
}

size_t lift_frag_bytes(int64_t n) { return (size_t)((n + 63) / 64) * 4096; }

void launch_lift_frag(const uint32_t *v, int64_t n, int64_t ld, int t, uint32_t p, char *frag, hipStream_t s) {
    if (n <= 0) return;
    ProfScope trace_(tl_trace, "k_lift_frag", s);
    if (lift_packed(t)) {
        hipLaunchKernelGGL(k_lift_frag_pk, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, v, n, ld, t, p,
                           reinterpret_cast<v4i_l *>(frag));
        return;
    }
    hipLaunchKernelGGL(k_lift_frag, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, v, n, ld, t, p,
                       reinterpret_cast<v4i_l *>(frag));
}

size_t lift_tile_a_bytes(int64_t n) { return (size_t)((n + 15) / 16) * (size_t)((n + 63) / 64) * 2048; }

void launch_lift_tile_a(const int16_t *A, int64_t n, int64_t ld, char *At, hipStream_t s) {
    if (n <= 0) return;
    ProfScope trace_(tl_trace, "k_lift_tile_a", s);
    const int KT = (int)((n + 63) / 64);
    hipLaunchKernelGGL(k_lift_tile_a, dim3((unsigned)KT, (unsigned)((n + 15) / 16)), dim3(64), 0, s, A, n, ld, KT,
                       reinterpret_cast<v4i_l *>(At));
}

void launch_range16(const int64_t *A, int64_t count, int32_t *flag, hipStream_t s) {
    if (count <= 0) return;
    ProfScope trace_(tl_trace, "k_range16", s);
    const int64_t blocks = std::min<int64_t>((count + 255) / 256, 4096);
    hipLaunchKernelGGL(k_range16, dim3((unsigned)blocks), dim3(256), 0, s, A, count, flag);
}

void launch_pack_rows(const int64_t *A, int64_t n, int64_t ld, int a_bytes, void *out, hipStream_t s) {
    if (n <= 0) return;
    ProfScope trace_(tl_trace, "k_pack_rows", s);
    const int64_t blocks = std::min<int64_t>((n * ld + 255) / 256, 8192);
    if (a_bytes == 2)
        hipLaunchKernelGGL(k_pack_rows<int16_t>, dim3((unsigned)blocks), dim3(256), 0, s, A, n, ld,
                           static_cast<int16_t *>(out));
    else
        hipLaunchKernelGGL(k_pack_rows<int32_t>, dim3((unsigned)blocks), dim3(256), 0, s, A, n, ld,
                           static_cast<int32_t *>(out));
}

void launch_lift_steps(const uint32_t *C, const void *A, int a_bytes, int64_t n, int64_t ld, int t, uint32_t p,
                       const LiftBufs &b, int steps, hipStream_t s) {
    ProfScope trace_(tl_trace, "k_lift_steps", s, 2 * (int64_t)steps + 1);
    for (int off = 0; off < steps; ++off) {
        if (a_bytes == 2)
            lift_step_at(C, static_cast<const int16_t *>(A), n, ld, t, p, b, off, s);
        else
            lift_step_at(C, static_cast<const int32_t *>(A), n, ld, t, p, b, off, s);
    }
    hipLaunchKernelGGL(k_lift_advance, dim3(1), dim3(64), 0, s, b.base, steps);
}

// One thread per (row i, vector c): the digits of steps step0 .. step0+cnt-1
// (slot step % ring of the vector's run) added into the entry's two 128-bit
// sums of reading 21, sum d_l B_l and sum d_l F_l with l = K - step (kept as
// (low, high) word pairs).  Consecutive rows are contiguous.
__global__ __launch_bounds__(256) void k_padic_acc(const uint32_t *__restrict__ Xh, int64_t n, int64_t ld,
                                                   int64_t cols, int64_t xh, int64_t ring, int64_t K, int64_t step0,
                                                   int cnt, const uint64_t *__restrict__ B,
                                                   const uint64_t *__restrict__ F, uint64_t *__restrict__ acc) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t c = blockIdx.y;
    if (i >= n) return;
    const uint32_t *__restrict__ d0 = Xh + (c / 16) * xh + (c % 16) * ld + i;
    const auto *Bc = cptr(B);
    const auto *Fc = cptr(F);
    uint64_t *a = acc + 4 * (c * n + i);
    unsigned __int128 sa = ((unsigned __int128)a[1] << 64) | a[0];
    unsigned __int128 sf = ((unsigned __int128)a[3] << 64) | a[2];
    for (int q = 0; q < cnt; ++q) {
        const int64_t st = step0 + q, l = K - st;
        const uint64_t d = d0[(st % ring) * 16 * ld];
        sa += (unsigned __int128)Bc[l] * d;
        sf += (unsigned __int128)Fc[l] * d;
    }
    a[0] = (uint64_t)sa;
    a[1] = (uint64_t)(sa >> 64);
    a[2] = (uint64_t)sf;
    a[3] = (uint64_t)(sf >> 64);
}

// From the sums: e = round(sum d_l F_l / 2^64), the rounding check, and
// Y[i ystride + c] = (sum d_l B_l + e B_0) mod m.
__global__ __launch_bounds__(256) void k_padic_fin(const uint64_t *__restrict__ acc, int64_t n, int64_t cols,
                                                   int64_t ystride, const uint64_t *__restrict__ B, uint64_t m,
                                                   uint64_t *__restrict__ Y, int32_t *__restrict__ bad) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t c = blockIdx.y;
    if (i >= n) return;
    const uint64_t *a = acc + 4 * (c * n + i);
    const unsigned __int128 sa = ((unsigned __int128)a[1] << 64) | a[0];
    const unsigned __int128 sf = ((unsigned __int128)a[3] << 64) | a[2];
    const uint64_t e = (uint64_t)((sf + ((unsigned __int128)1 << 63)) >> 64);
    const unsigned __int128 ee = (unsigned __int128)e << 64;
    const unsigned __int128 dist = sf > ee ? sf - ee : ee - sf;
    if (dist >= ((unsigned __int128)1 << 43)) atomicOr(bad, 1);
    const uint64_t r1 = (uint64_t)(sa % m);
    const uint64_t r2 = (uint64_t)((unsigned __int128)B[0] * (e % m) % m);
    const uint64_t r = r1 + r2;
    Y[i * ystride + c] = r >= m ? r - m : r;
}

void launch_padic_acc(const uint32_t *Xh, int64_t n, int64_t ld, int64_t cols, int64_t xh, int64_t ring, int64_t K,
                      int64_t step0, int cnt, const uint64_t *B, const uint64_t *F, uint64_t *acc, hipStream_t s) {
    if (n <= 0 || cols <= 0 || cnt <= 0) return;
    ProfScope trace_(tl_trace, "k_padic_acc", s);
    hipLaunchKernelGGL(k_padic_acc, dim3((unsigned)((n + 255) / 256), (unsigned)cols), dim3(256), 0, s, Xh, n, ld,
                       cols, xh, ring, K, step0, cnt, B, F, acc);
}

void launch_padic_fin(const uint64_t *acc, int64_t n, int64_t cols, int64_t ystride, const uint64_t *B, uint64_t m,
                      uint64_t *Y, int32_t *bad, hipStream_t s) {
    if (n <= 0 || cols <= 0) return;
    ProfScope trace_(tl_trace, "k_padic_fin", s);
    hipLaunchKernelGGL(k_padic_fin, dim3((unsigned)((n + 255) / 256), (unsigned)cols), dim3(256), 0, s, acc, n, cols,
                       ystride, B, m, Y, bad);
}

void launch_lift_proj(const uint32_t *Xh, int64_t n, int64_t ld, int t, const int32_t *Rp, int tp,
                      int64_t i0, int64_t i1, int64_t *Z, hipStream_t s) {
    if (i1 <= i0) return;
    ProfScope trace_(tl_trace, "k_lift_proj", s);
    hipLaunchKernelGGL(k_lift_proj, dim3((unsigned)((i1 - i0) * t)), dim3(256), 0, s, Xh, n, ld, t, Rp, tp,
                       i0, Z);
}

void launch_gj_blockinv(uint32_t *M, int64_t n, int64_t ld, int64_t r0, int bw, const GjPrime *pr, int P,
                        uint32_t *W, int32_t *singular, int32_t *need, uint32_t *det, hipStream_t s) {
    ProfScope trace_(tl_trace, "k_gj_blockinv", s);
    hipLaunchKernelGGL(k_gj_blockinv, dim3((unsigned)P), dim3(1024), 0, s, M, n, ld, r0, bw, pr, W, singular, need,
                       det, 0);
}

void launch_gj_pivoted(uint32_t *M, int64_t n, int64_t ld, int64_t r0, int bw, const GjPrime *pr, int P,
                       uint32_t *S, int32_t *piv, int32_t *singular, int32_t *need, uint32_t *det, uint32_t *W,
                       hipStream_t s) {
    ProfScope trace_(tl_trace, "k_gj_pivoted", s, 3);
    hipLaunchKernelGGL(k_gj_panel, dim3((unsigned)P), dim3(1024), 0, s, M, n, ld, r0, bw, pr, S, piv, singular,
                       need, det);
    hipLaunchKernelGGL(k_gj_swap, dim3((unsigned)((ld + 255) / 256), (unsigned)P), dim3(256), 0, s, M, n, ld, r0,
                       bw, piv, singular, need);
    hipLaunchKernelGGL(k_gj_blockinv, dim3((unsigned)P), dim3(1024), 0, s, M, n, ld, r0, bw, pr, W, singular, need,
                       det, 1);
}

void launch_scale(uint32_t *R, int64_t rows, int64_t cols, int64_t ld, int64_t plane_stride,
                  const GjPrime *pr, const uint32_t *c, int P, hipStream_t s) {
    ProfScope trace_(tl_trace, "k_scale", s);
    dim3 grid((unsigned)((cols + 255) / 256), (unsigned)rows, (unsigned)P);
    hipLaunchKernelGGL(k_scale, grid, dim3(256), 0, s, R, rows, cols, ld, plane_stride, pr, c);
}

void launch_words_mod(const uint64_t *x, int64_t count, int W, const GjPrime *pr, int L,
                      uint32_t *out, hipStream_t s) {
    if (count <= 0 || L <= 0) return;
    ProfScope trace_(tl_trace, "k_words_mod", s);
    hipLaunchKernelGGL(k_words_mod, dim3((unsigned)((count + 255) / 256), (unsigned)L), dim3(256), 0, s, x,
                       count, W, pr, out);
}

void launch_check_sI(const uint32_t *P, int64_t n, const uint32_t *s_mod, int L, unsigned *mism,
                     hipStream_t s) {
    ProfScope trace_(tl_trace, "k_check_sI", s);
    dim3 grid((unsigned)((n + 255) / 256), (unsigned)n, (unsigned)L);
    hipLaunchKernelGGL(k_check_sI, grid, dim3(256), 0, s, P, n, s_mod, mism);
}

void launch_words_mod_m(const uint64_t *x, int64_t count, int W, const LocalMod &lm, uint64_t *out,
                        hipStream_t s) {
    ProfScope trace_(tl_trace, "k_words_mod_m", s);
    hipLaunchKernelGGL(k_words_mod_m, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, x, count,
                       W, lm, out);
}

void launch_loc_init(const uint64_t *M, int64_t n, const LocalMod *lms, int F, uint64_t *keys, hipStream_t s) {
    ProfScope trace_(tl_trace, "k_loc_init", s);
    const int64_t blocks = std::min<int64_t>((n * n + 255) / 256, 512);
    hipLaunchKernelGGL(k_loc_init, dim3((unsigned)blocks, (unsigned)F), dim3(256), 0, s, M, n, lms, keys);
}

void launch_loc_step(uint64_t *M, int64_t n, int k, const LocalMod *lms, int F, uint64_t *keys, int32_t *val,
                     uint64_t *uinv, hipStream_t s) {
    ProfScope trace_(tl_trace, "k_loc_step", s, n - k - 1 > 0 ? 2 : 1);
    hipLaunchKernelGGL(k_loc_swap, dim3((unsigned)((n + 255) / 256), (unsigned)F), dim3(256), 0, s, M, n, k, lms,
                       keys, val, uinv);
    const int64_t w = n - k - 1;
    if (w <= 0) return;
    dim3 grid((unsigned)((w + 255) / 256), (unsigned)((w + kLocRows - 1) / kLocRows), (unsigned)F);
    hipLaunchKernelGGL(k_loc_elim, grid, dim3(256), 0, s, M, n, k, lms, val, uinv, keys);
}

}  // namespace rns
