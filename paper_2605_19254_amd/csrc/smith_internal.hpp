// Shared declarations of the Smith-form driver and its kernels.
#pragma once

#include "internal.hpp"

namespace rns {

// One prime of a batched modular computation in the driver.
struct GjPrime {
    uint32_t p;
    double pf, pinv;
    double pow64w;     // 2^(64W) mod p for the word count of the current call
};

// Modulus q^e < 2^34 of a local elimination.
struct LocalMod {
    uint32_t q;
    int e;
    uint64_t m;
    double mf, minv;
    uint64_t pow64w;   // 2^(64W) mod m
};

// [A mod p | I] (ld = 2n) or A mod p (ld = n) for P primes at once.
void launch_gj_load(const int64_t *A, int64_t n, int64_t ld, uint32_t *M, const GjPrime *pr, int P,
                    hipStream_t s);
// Blocked elimination of P planes, block at row/column r0 of width
// bw <= kGjBlock: launch_gj_blockinv inverts the unexchanged pivot block of
// every plane (need[q] = 1 where that fails); launch_gj_pivoted then handles
// the planes with need[q] = 1 (panel pivot search, row exchanges, inverse).
// The driver finishes each block with two residue products.  S: [P][n][kGjBlock]
// scratch; piv: [P][kGjBlock]; W: [P][kGjBlock][kGjBlock]; det optional.
constexpr int kGjBlock = 128;
void launch_gj_blockinv(uint32_t *M, int64_t n, int64_t ld, int64_t r0, int bw, const GjPrime *pr, int P,
                        uint32_t *W, int32_t *singular, int32_t *need, uint32_t *det, hipStream_t s);
void launch_gj_pivoted(uint32_t *M, int64_t n, int64_t ld, int64_t r0, int bw, const GjPrime *pr, int P,
                       uint32_t *S, int32_t *piv, int32_t *singular, int32_t *need, uint32_t *det, uint32_t *W,
                       hipStream_t s);
// One step of p-adic lifting for t <= 16 right-hand sides and the
// projections of stored digits.  C (n x n mod p) and A (n x n, int32 or,
// with a_bytes = 2, int16) have row stride ld, a multiple of 8, and are zero
// in columns n..ld-1; R, Rm and X hold t vectors of stride ld ([t][ld]).
constexpr int kLiftMaxCols = 16;
// Device state of a lifting run: residuals R[2] (int64) and Rm[2] (mod p),
// every step's digits Xh ([K][t][ld]), the inexact-division flag and the
// index of the next step (*base).
// Several independent liftings of kLiftMaxCols vectors each in one launch
// (blockIdx.y = group; only the unpacked matrix-core kernels with both
// operands tiled): group g's buffers start `r`, `rm`, `xh`, `frag` elements
// after group 0's.  Step i's digits go to slot i % ring of Xh.
struct LiftGroups {
    int groups = 1;
    int64_t r = 0, rm = 0, xh = 0, frag = 0;
    int64_t ring = INT64_MAX;
    int64_t rbs = 0;        // 16-row blocks (grouped launches: the work items are rbs x groups)
};
struct LiftBufs {
    int64_t *R0, *R1;
    uint32_t *Rm0, *Rm1;
    uint32_t *Xh;
    int32_t *err;
    int64_t *base;
    const char *Ct = nullptr;   // C as tiled digits (launch_lift_tile_c), or null: products on the vector units
    const char *At = nullptr;   // int16 A as tiled digits (launch_lift_tile_a), or null
    char *Xd = nullptr;         // digit fragments of the step's X and of the next Rm (each
    char *Rmd = nullptr;        // lift_frag_bytes(n)); used when Ct and At are both set
    LiftGroups grp{};
};
// One prime power m = q^e < 2^62 of a local Smith form with transforms
// (massager_kernels.hip): constants for exact division by q and for
// Montgomery products (odd m; a power of two is reduced by masking).
struct LsnfPlane {
    uint64_t m, q;
    uint64_t qinv, qmax;       // odd q: q^-1 mod 2^64, floor((2^64 - 1) / q)
    uint64_t minv, r2, rinv;   // odd m: -m^-1 mod 2^64, 2^128 mod m, 2^-64 mod m (1, 1, 1 for 2^e)
    int e, pow2;
};
// The current pivot of a plane: the minimal key (v << 42 | row << 21 |
// column), its valuation, q^v, m / q^v, the inverse of the pivot's unit part
// modulo m / q^v; done once every remaining entry is zero.
struct LsnfStep {
    uint64_t key;
    int v, done;
    uint64_t qv, mq, uinv;
};
// P (n x t, entries below s) into the F planes W_f (Montgomery form), Pf
// (plain), E_f = I (n x n) and R_f = I (t x t, stored transposed: row j of
// the buffer is column j of R_f); n, t < 2^21.
void launch_ls_load(const uint64_t *P, int64_t n, int64_t t, const LsnfPlane *pl, int F, uint64_t *W, uint64_t *Pf,
                    uint64_t *E, uint64_t *R, LsnfStep *st, hipStream_t s);
// Step c of every plane: pivot search, exchanges, pivot record (vals[f][c],
// units[f][c]), row and column elimination with E_f and R_f.
void launch_ls_step(uint64_t *W, uint64_t *E, uint64_t *R, int64_t n, int64_t t, int64_t c, const LsnfPlane *pl,
                    int F, LsnfStep *st, int32_t *vals, uint64_t *units, hipStream_t s);
// out[f][i][j] = (Pf_f R_f)[i][j] mod m_f, plain, for j < take.
void launch_ls_pr(const uint64_t *Pf, const uint64_t *R, int64_t n, int64_t t, int64_t take, const LsnfPlane *pl,
                  int F, uint64_t *out, hipStream_t s);
// Rows 0 .. rows-1 of every E_f to plain form.
void launch_ls_plain(uint64_t *E, int64_t n, int64_t rows, const LsnfPlane *pl, int F, hipStream_t s);

// Rem(s_n x, m) (m < 2^62) for the first `cols` lifted vectors (groups of
// 16) from their top L digits, in chunks: launch_padic_acc adds the digits of
// steps step0 .. step0+cnt-1 (the digit of step st of vector c, row i is
// Xh[(c / 16) xh + (st % ring) 16 ld + (c % 16) ld + i]) into per-entry
// 128-bit sums sum d_l B_l and sum d_l F_l, l = K - st, with B[l] = -a_l p^K
// mod m, F[l] = floor(frac(s_n / p^l) 2^64), B[0] = -p^K mod m as
// msg::PadicTable (acc: [cols][n][4] words, zero at first); launch_padic_fin
// writes entry (i, c) to Y[i ystride + c] and sets *bad = 1 where the
// rounding is not within 2^-21.
void launch_padic_acc(const uint32_t *Xh, int64_t n, int64_t ld, int64_t cols, int64_t xh, int64_t ring, int64_t K,
                      int64_t step0, int cnt, const uint64_t *B, const uint64_t *F, uint64_t *acc, hipStream_t s);
void launch_padic_fin(const uint64_t *acc, int64_t n, int64_t cols, int64_t ystride, const uint64_t *B, uint64_t m,
                      uint64_t *Y, int32_t *bad, hipStream_t s);
// Largest n whose lifting products run on the matrix cores (int32 sums of
// the digit products stay exact for k <= 43690).
constexpr int64_t kLiftMfmaMaxN = 43690;
// Bytes of the tiled digits of an n x n residue matrix, and their build
// (balanced digits of C mod p, 16-row blocks x 64-column steps, the matrix-
// core operand layout).
size_t lift_tile_c_bytes(int64_t n);
void launch_lift_tile_c(const uint32_t *C, int64_t n, int64_t ld, uint32_t p, char *Ct, hipStream_t s);
// With both operands tiled and t <= 4 the right operands use the packed
// fragment (digit d of vector c in MFMA column 4 d + c, 1 KiB per 64 rows).
inline bool lift_packed(int t) { return t <= 4; }
// Whether launch_lift_steps can run grouped liftings for these buffers.
inline bool lift_groups_ok(const LiftBufs &b, int a_bytes, int t) {
    return b.Ct && b.At && a_bytes == 2 && b.Xd && b.Rmd && !lift_packed(t);
}
// Digit fragments of t <= 16 vectors [t][ld] (the right operand of the
// lifting products; packed when lift_packed(t)); balanced digits of the first
// step's Rm (entries in [0, p)) for C Rm mod p.
size_t lift_frag_bytes(int64_t n);
void launch_lift_frag(const uint32_t *v, int64_t n, int64_t ld, int t, uint32_t p, char *frag, hipStream_t s);
// The same for an int16 A (two exact signed byte digits per entry).
size_t lift_tile_a_bytes(int64_t n);
void launch_lift_tile_a(const int16_t *A, int64_t n, int64_t ld, char *At, hipStream_t s);
// *flag = 1 if an entry of A (count int64 values) is outside (-32640, 32640);
// the caller clears *flag first.
void launch_range16(const int64_t *A, int64_t count, int32_t *flag, hipStream_t s);
// The n x n int64 A as int16 (a_bytes 2) or int32 rows of stride ld >= n,
// zero padded; every entry must fit the narrower type.
void launch_pack_rows(const int64_t *A, int64_t n, int64_t ld, int a_bytes, void *out, hipStream_t s);
// `steps` lifting steps (two launches each) and one launch advancing *base;
// the launches take the same arguments for every run of the same length.
void launch_lift_steps(const uint32_t *C, const void *A, int a_bytes, int64_t n, int64_t ld, int t, uint32_t p,
                       const LiftBufs &b, int steps, hipStream_t s);
void launch_lift_proj(const uint32_t *Xh, int64_t n, int64_t ld, int t, const int32_t *Rp, int tp,
                      int64_t i0, int64_t i1, int64_t *Z, hipStream_t s);
void launch_scale(uint32_t *R, int64_t rows, int64_t cols, int64_t ld, int64_t plane_stride,
                  const GjPrime *pr, const uint32_t *c, int P, hipStream_t s);
void launch_words_mod(const uint64_t *x, int64_t count, int W, const GjPrime *pr, int L,
                      uint32_t *out, hipStream_t s);
void launch_check_sI(const uint32_t *P, int64_t n, const uint32_t *s_mod, int L, unsigned *mism,
                     hipStream_t s);
void launch_words_mod_m(const uint64_t *x, int64_t count, int W, const LocalMod &lm, uint64_t *out,
                        hipStream_t s);
// Local Smith form of F planes at once (plane f modulo lms[f].m): keys
// ([F][n+1], all ~0 beforehand) of step 0, then step k of every plane
// (uinv: F words of scratch for the pivots' unit inverses).
void launch_loc_init(const uint64_t *M, int64_t n, const LocalMod *lms, int F, uint64_t *keys, hipStream_t s);
void launch_loc_step(uint64_t *M, int64_t n, int k, const LocalMod *lms, int F, uint64_t *keys, int32_t *val,
                     uint64_t *uinv, hipStream_t s);

// Unimodularity certificate (Section 2.2, Phase 3): the two residue bases of
// the double-plus-one steps.  X = p_0 ... p_{j-1} is the lifting modulus;
// the exact residues are recovered from q_0 ... q_{l-1}.  pinv[a][b] =
// p_a^-1 mod p_b (a < b), likewise qinv; phalf / qhalf are the mixed-radix
// digits of (X - 1) / 2 and (Q - 1) / 2; bound is the promised max |Z|.
constexpr int kUcMaxPrimes = 4;
struct UcBasis {
    int j, l;
    uint32_t p[kUcMaxPrimes], q[kUcMaxPrimes];
    uint32_t pinv[kUcMaxPrimes][kUcMaxPrimes], qinv[kUcMaxPrimes][kUcMaxPrimes];
    uint32_t phalf[kUcMaxPrimes], qhalf[kUcMaxPrimes];
    uint32_t x_mod_q[kUcMaxPrimes], xinv_q[kUcMaxPrimes];
    int64_t bound;
};
// Kq (l planes) <- the symmetric K given by Kp (j planes), count entries per
// plane, planes plane_stride apart.
void launch_uc_convert(const uint32_t *Kp, uint32_t *Kq, int64_t count, int64_t plane_stride, const UcBasis &b,
                       hipStream_t s);
// Z <- (residues Rq of Y - D K) X^-1 as int64; flags[0] |= some entry is
// nonzero, flags[1] |= some entry exceeds b.bound (then written as 0).
void launch_uc_tail(const uint32_t *Rq, int64_t *Z, int64_t count, int64_t plane_stride, const UcBasis &b,
                    int32_t *flags, hipStream_t s);
// Z <- I (n x n int64).
void launch_uc_identity(int64_t *Z, int64_t n, hipStream_t s);

}  // namespace rns
