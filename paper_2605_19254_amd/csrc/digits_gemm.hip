// Conversions between integers and residues as INT8 matrix-core products
// with a constant table (Section 3.1: the bullets on fast RNS base
// conversion and on precomputed RNS constants).  Each conversion is linear
// in the entry's digits, so every entry's signed base-256 digits form one row
// of a left operand D (entries x K) and a constant table G (K x N) built once
// per basis turns them into N int32 column sums T = D G on the matrix cores
// (v_mfma_i32_16x16x64_i8); a short epilogue per entry finishes exactly:
//
//  * CRT (exact, no bound needed).  y_j = r_j (M/p_j)^-1 mod p_j in balanced
//    form, S = sum_j y_j (M/p_j), x = S - a M with a = round(sum_j y_j / p_j).
//    Columns of G are the bytes of S: G[(j, i)][k] = digit k - i of M/p_j, so
//    T_k = sum over (j, i) of y_j's digit i times M/p_j's digit k - i.  The
//    epilogue forms 32-bit limbs of S and subtracts a M with signed carries.
//    sum_j y_j / p_j is exact in reals (it is S / M); its double value errs
//    by less than 2^-40 for L <= 64, so a differs from round(S / M) only
//    when S / M lies within 2^-40 of a half-integer.  There a = floor, and
//    x, then about M/2, is compared with (M-1)/2 exactly and reduced by M if
//    larger: the result is the symmetric representative in every case.
//  * Multiword reduction.  x (W two's-complement words) as 8W+1 balanced
//    digits; G[k][(b, j)] = digit b of 2^(8k) mod p_j, and
//    x mod p_j = sum_b T_(b,j) 2^(8b) mod p_j.
//  * Base conversion (the paper's Lagrange shortcut with a floating-point
//    correction).  x mod q_i = sum_j y_j (M/p_j mod q_i) - a (M mod q_i)
//    with a = round(sum_j y_j / p_j), exact when a caller bound on |x| leaves
//    the margin of the Lagrange CRT; G[(j, d)][(s, i)] = digit s - d of
//    M/p_j mod q_i, so the column sums are the seven shift groups of the
//    16 digit-pair products, recombined as in the residue products.
//
// Layout: a wave takes 16 RB consecutive entries of one matrix row (RB row
// blocks of 16); lane e builds entry e's digit row in LDS, the MFMAs read
// 16-entry row blocks from there and the table's fragments from global
// memory (L2-resident, a few KiB to tens of KiB), each fragment loaded once
// for the RB row blocks.
#include "reduce_crt.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

using namespace rns;

namespace {

typedef int v4i_d __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;             // waves per work-group
constexpr int kThreads = 64 * kWaves;
constexpr int kCrtMfmaMaxL = 64;

// Balanced base-256 digits of |r| < 2^25 (d0..d2 in [-128, 127], |d3| <= 2),
// byte i of the result holding d_i.
__device__ __forceinline__ uint32_t pack_digits(int32_t r) {
    uint32_t w = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int32_t d = (int32_t)(int8_t)(r & 0xFF);
        w |= ((uint32_t)d & 0xFFu) << (8 * i);
        r = (r - d) >> 8;
    }
    return w | (((uint32_t)r & 0xFFu) << 24);
}

// a mod p in (-p/2, p/2) for |a| < 2^52 (the quotient from the rounded
// reciprocal may be one off, which the two corrections absorb).
__device__ __forceinline__ double bal_mod(double a, double pf, double pinv) {
    double r = fma(-rint(a * pinv), pf, a);
    const double h = 0.5 * pf;
    r = r > h ? r - pf : r;
    r = r < -h ? r + pf : r;
    return r;
}

// Entry addressing shared by the kernels: chunk c of a job covers columns
// [c0, c0 + 16 RB) of row `row`.
struct Chunk {
    int64_t row, c0;
    bool any;
};

__device__ __forceinline__ Chunk chunk_of(int64_t chunk, int64_t total, int64_t col_chunks, int width) {
    Chunk c{0, 0, chunk < total};
    if (c.any) {
        c.row = chunk / col_chunks;
        c.c0 = (chunk - c.row * col_chunks) * width;
    }
    return c;
}

// Every LDS region below belongs to one wave: ordering its lanes' accesses
// needs no work-group barrier, only a wavefront-scope fence (which also keeps
// the compiler from moving LDS accesses across it), so the waves of a
// work-group run independently.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// acc[rb][cb] += D(row block rb, all k) x G(k, column block cb): D rows from
// LDS (row stride rs bytes), G fragments [NKS][NCB][64 lanes] from global.
template <int NKS, int NCB, int RB>
__device__ __forceinline__ void digits_mfma(const char *A, int rs, const v4i_d *__restrict__ G, int lane,
                                            v4i_d (&acc)[RB][NCB]) {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) acc[rb][cb] = v4i_d{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
        v4i_d a[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
            a[rb] = *reinterpret_cast<const v4i_d *>(A + (16 * rb + (lane & 15)) * rs + 64 * ks + 16 * (lane >> 4));
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            const v4i_d b = G[(ks * NCB + cb) * 64 + lane];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
                acc[rb][cb] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[rb], b, acc[rb][cb], 0, 0, 0);
        }
    }
}

// Phase A of the CRT and the conversion: balanced y_j = r_j c_j mod p_j of
// one entry, their digits into the entry's LDS row, and sum_j y_j / p_j.
// The residues are read eight planes at a time, all eight loads in flight
// before the first is used; the per-prime constants are uniform (scalar
// loads).
__device__ __forceinline__ double lagrange_digits(const uint32_t *__restrict__ res, int64_t ps, int L,
                                                  const PrimeConst *pc_, const double *cj_, uint32_t *row, int KA) {
    const auto pc = cptr(pc_);
    const auto cj = cptr(cj_);
    const auto src = gptr(res);
    double alpha = 0.0;
    for (int j0 = 0; j0 < L; j0 += 8) {
        uint32_t r[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) r[q] = src[(int64_t)min(j0 + q, L - 1) * ps];      // in bounds
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int j = j0 + q;
            if (j < L) {
                const double pf = pc[j].pf, pinv = pc[j].pinv;
                const double y = bal_mod((double)r[q] * cj[j], pf, pinv);
                alpha = fma(y, pinv, alpha);
                row[j] = pack_digits((int32_t)y);
            }
        }
    }
    for (int j = L; j < KA / 4; ++j) row[j] = 0u;
    return alpha;
}

// The same from residues already in registers (r[j], j < L <= N).
template <int N>
__device__ __forceinline__ double lagrange_digits_reg(const uint32_t (&r)[N], int L, const PrimeConst *pc_,
                                                      const double *cj_, uint32_t *row, int KA) {
    const auto pc = cptr(pc_);
    const auto cj = cptr(cj_);
    double alpha = 0.0;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        if (j < L) {
            const double pf = pc[j].pf, pinv = pc[j].pinv;
            const double y = bal_mod((double)r[j] * cj[j], pf, pinv);
            alpha = fma(y, pinv, alpha);
            row[j] = pack_digits((int32_t)y);
        }
    }
    for (int j = L; j < KA / 4; ++j) row[j] = 0u;
    return alpha;
}

// All L <= N residues of one entry into registers, every load in flight.
template <int N>
__device__ __forceinline__ void load_residues(const uint32_t *res, int64_t ps, int L, uint32_t (&r)[N]) {
    const auto src = gptr(res);
#pragma unroll
    for (int j = 0; j < N; ++j)
        if (j < L) r[j] = src[(int64_t)j * ps];
}

// ----------------------------------------------------------------- CRT --

struct CrtMfmaJob {
    const uint32_t *res;
    int64_t rows, cols, ldr, ps;
    int L, W;
    uint64_t *out;
    int64_t ldo;
    int32_t *status;
    const PrimeConst *pc;      // the range's first prime
    const double *cj;          // (M/p_j)^-1 mod p_j
    const uint32_t *mlimbs;    // M, Qp 32-bit limbs
    const uint32_t *half;      // (M-1)/2, Qp limbs
    const v4i_d *G;
};

// One wave takes EW entries per step: their digit rows (EW x RS bytes of
// LDS), products one row block of 16 at a time, each block's 32-bit limbs
// into the wave's limb rows (EW x LS words of 8 bytes, LS = QP + 1 against
// bank conflicts, at least 33 so that the same rows can stage the output
// words), then the carry chains of all EW entries at once, one per lane.
// Two waves per work-group keep that LDS within 64 KiB.
constexpr int kCrtWaves = 2;

template <int NKS, int NQB, int EW>
struct CrtShape {
    static constexpr int KA = 64 * NKS, RS = KA + 16, NCB = 4 * NQB, QP = 16 * NQB;
    static constexpr int LS = QP + 1 > 33 ? QP + 1 : 33;
    static constexpr int AREA = EW * RS + EW * LS * 8;
    static constexpr int LDS = kCrtWaves * AREA;
};

template <int NKS, int NQB, int EW, int RBP>
__global__ __launch_bounds__(64 * kCrtWaves, 3) void k_crt_mfma(CrtMfmaJob J, int64_t total_chunks,
                                                             int64_t col_chunks) {
    using Sh = CrtShape<NKS, NQB, EW>;
    constexpr int KA = Sh::KA, RS = Sh::RS, NCB = Sh::NCB, QP = Sh::QP, LS = Sh::LS;
    extern __shared__ char smem[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    char *A = smem + wave * Sh::AREA;
    int64_t *limb = reinterpret_cast<int64_t *>(A + EW * RS);
    const auto mlimbs = cptr(J.mlimbs);                       // uniform: scalar loads
    const auto half = cptr(J.half);
    const int W = J.W;
    bool over = false;
    const int64_t iters = (total_chunks + kCrtWaves - 1) / kCrtWaves;
    // Software pipelining: with L <= PRE the next step's residues are loaded
    // into registers right after this step's digits are formed, so their
    // latency passes while this step's products and carry chains run.
    constexpr int PRE = NKS <= 1 ? 16 : 1;
    const bool pipelined = J.L <= PRE && PRE > 1;
    uint32_t pre[PRE];
    auto fetch = [&](int64_t it_) {
        const Chunk c = chunk_of(it_ * kCrtWaves + wave, total_chunks, col_chunks, EW);
        const int64_t cl = c.c0 + lane;
        if (c.any && lane < EW && cl < J.cols) load_residues(J.res + c.row * J.ldr + cl, J.ps, J.L, pre);
    };
    if (pipelined && blockIdx.x < iters) fetch(blockIdx.x);
    for (int64_t it = blockIdx.x; it < iters; it += gridDim.x) {
        const Chunk ch = chunk_of(it * kCrtWaves + wave, total_chunks, col_chunks, EW);
        // Phase A: lane e < EW owns entry e of the chunk.
        const int64_t col = ch.c0 + lane;
        const bool valid = ch.any && lane < EW && col < J.cols;
        int64_t a = 0;
        bool tie = false;
        if (lane < EW) {
            uint32_t *row = reinterpret_cast<uint32_t *>(A + lane * RS);
            if (valid) {
                const double al = pipelined
                    ? lagrange_digits_reg(pre, J.L, J.pc, J.cj, row, KA)
                    : lagrange_digits(J.res + ch.row * J.ldr + col, J.ps, J.L, J.pc, J.cj, row, KA);
                const double fl = floor(al);
                tie = fabs(al - fl - 0.5) < 0x1p-40;
                a = (int64_t)(tie ? fl : rint(al));
            } else {
                for (int j = 0; j < KA / 4; ++j) row[j] = 0u;
            }
        }
        if (pipelined && it + gridDim.x < iters) fetch(it + gridDim.x);
        wave_sync();
        // Each table fragment is loaded once for RBP row blocks.
#pragma unroll 1
        for (int rb0 = 0; rb0 < EW / 16; rb0 += RBP) {
            v4i_d acc[RBP][NCB];
            digits_mfma<NKS, NCB, RBP>(A + 16 * rb0 * RS, RS, J.G, lane, acc);
            // 32-bit limb q of S (signed, below 2^47 in magnitude) from the
            // four byte columns 4q .. 4q+3; this lane holds limbs 16 qb + lane%16
            // of entries 16 rb + 4 (lane/16) + v.
#pragma unroll
            for (int r = 0; r < RBP; ++r)
#pragma unroll
                for (int v = 0; v < 4; ++v)
#pragma unroll
                    for (int qb = 0; qb < NQB; ++qb) {
                        int64_t sum = 0;
#pragma unroll
                        for (int i = 0; i < 4; ++i) sum += (int64_t)acc[r][i * NQB + qb][v] << (8 * i);
                        limb[(16 * (rb0 + r) + 4 * (lane >> 4) + v) * LS + 16 * qb + (lane & 15)] = sum;
                    }
        }
        wave_sync();
        // The carry chain of entry e in lane e, in registers: x = S - a M as
        // QP normalised 32-bit limbs.
        uint32_t xr[QP];
        uint32_t fill = 0;
        if (lane < EW) {
            const int64_t *x = limb + lane * LS;
            int64_t carry = 0;
#pragma unroll
            for (int q = 0; q < QP; ++q) {
                const int64_t v = x[q] - a * (int64_t)mlimbs[q] + carry;
                xr[q] = (uint32_t)v;
                carry = v >> 32;
            }
            fill = carry ? 0xFFFFFFFFu : 0u;                  // the sign
            if (tie && !fill) {                               // x near M/2: reduce if above (M-1)/2
                int cmp = 0;
#pragma unroll
                for (int q = QP - 1; q >= 0; --q)
                    if (cmp == 0) cmp = xr[q] > half[q] ? 1 : (xr[q] < half[q] ? -1 : 0);
                if (cmp > 0) {
                    int64_t bb = 0;
#pragma unroll
                    for (int q = 0; q < QP; ++q) {
                        const int64_t v = (int64_t)xr[q] - (int64_t)mlimbs[q] + bb;
                        xr[q] = (uint32_t)v;
                        bb = v >> 32;
                    }
                    fill = bb ? 0xFFFFFFFFu : 0u;
                }
            }
            // Fits W words: every limb from 2W up is the sign fill, and the
            // top bit of word W-1 is the sign.
            bool fits = true;
#pragma unroll
            for (int q = 0; q < QP; ++q) {
                if (q >= 2 * W) fits &= xr[q] == fill;
                if (q == 2 * W - 1) fits &= (xr[q] >> 31) == (fill & 1u);
            }
            over |= valid && !fits;
        }
        wave_sync();                                          // every limb read: the rows take the words
        if (lane < EW) {
            uint64_t *o = reinterpret_cast<uint64_t *>(limb) + lane * W;
#pragma unroll
            for (int w = 0; w < QP / 2; ++w)
                if (w < W) o[w] = (uint64_t)xr[2 * w] | ((uint64_t)xr[2 * w + 1] << 32);
            const uint64_t f64 = fill ? ~0ull : 0ull;
            for (int w = QP / 2; w < W; ++w) o[w] = f64;
        }
        wave_sync();
        // Coalesced copy of the step's valid entries (consecutive columns of
        // one row, W words each) to the output.
        {
            const int64_t ne = ch.any ? max<int64_t>(0, min<int64_t>(EW, J.cols - ch.c0)) : 0;
            const uint64_t *src = reinterpret_cast<const uint64_t *>(limb);
            uint64_t *dst = J.out + (ch.row * J.ldo + ch.c0) * W;
            for (int64_t k = lane; k < ne * W; k += 64) dst[k] = src[k];
        }
        wave_sync();
    }
    const uint64_t bad = __ballot(over);                      // one status write per wave
    if (bad && lane == __ffsll((unsigned long long)bad) - 1) atomicOr(J.status, 1);
}

// ------------------------------------------------- multiword reduction --

struct ReduceMfmaJob {
    const uint64_t *x;
    int64_t rows, cols, ldx;
    int W;
    uint32_t *res;
    int64_t ldr, ps;
    int L, groups;
    const PrimeConst *pc;
    const v4i_d *G;            // [groups][NKS][8][64]
};

constexpr int kRedGroup = 32;  // primes per product (N = 4 x 32 columns)

template <int NKS, int EW>
__global__ __launch_bounds__(kThreads, 3) void k_reduce_mw_mfma(ReduceMfmaJob J, int64_t total_chunks,
                                                             int64_t col_chunks) {
    constexpr int KA = 64 * NKS, RS = KA + 16, NCB = 8, RBP = 2;
    extern __shared__ char smem[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    char *A = smem + wave * EW * RS;
    const int64_t iters = (total_chunks + kWaves - 1) / kWaves;
    for (int64_t it = blockIdx.x; it < iters; it += gridDim.x) {
        const Chunk ch = chunk_of(it * kWaves + wave, total_chunks, col_chunks, EW);
        if (lane < EW) {
            const int64_t col = ch.c0 + lane;
            uint32_t *row = reinterpret_cast<uint32_t *>(A + lane * RS);
            int k4 = 0;                                          // next digit word of the row
            if (ch.any && col < J.cols) {
                // Balanced digits of the W-word two's-complement value: the
                // bytes with carries, the top digit (index 8W) = carry - sign;
                // two digit words per input word, eight input words in flight.
                const auto xe = gptr(J.x + (ch.row * J.ldx + col) * J.W);
                int carry = 0;
                uint64_t w = 0;
                for (int w0 = 0; w0 < J.W; w0 += 8) {
                    uint64_t u[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) u[q] = xe[min(w0 + q, J.W - 1)];
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        if (w0 + q >= J.W) break;
                        w = u[q];
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            uint32_t dw = 0;
#pragma unroll
                            for (int b = 0; b < 4; ++b) {
                                int v = (int)((w >> (32 * h + 8 * b)) & 0xFF) + carry;
                                carry = v >= 128;
                                v -= carry ? 256 : 0;
                                dw |= ((uint32_t)v & 0xFFu) << (8 * b);
                            }
                            row[k4++] = dw;
                        }
                    }
                }
                row[k4++] = (uint32_t)(carry - (int)(w >> 63)) & 0xFFu;
            }
            for (; k4 < KA / 4; ++k4) row[k4] = 0u;
        }
        wave_sync();
#pragma unroll 1
        for (int g = 0; g < J.groups; ++g) {
            const v4i_d *G = J.G + (int64_t)g * NKS * NCB * 64;
#pragma unroll 1
            for (int rb0 = 0; rb0 < EW / 16; rb0 += RBP) {
                v4i_d acc[RBP][NCB];
                digits_mfma<NKS, NCB, RBP>(A + 16 * rb0 * RS, RS, G, lane, acc);
                // Column 16 cb + lane%16 = 32 b + j (b: digit of 2^(8k) mod p_j).
#pragma unroll
                for (int r = 0; r < RBP; ++r)
#pragma unroll
                    for (int jb = 0; jb < 2; ++jb) {
                        const int j = kRedGroup * g + 16 * jb + (lane & 15);
                        if (j >= J.L) continue;
                        const double pf = J.pc[j].pf, pinv = J.pc[j].pinv;
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int64_t col = ch.c0 + 16 * (rb0 + r) + 4 * (lane >> 4) + v;
                            if (!ch.any || col >= J.cols) continue;
                            double val = 0.0;
#pragma unroll
                            for (int b = 3; b >= 0; --b) val = fma(val, 256.0, (double)acc[r][2 * b + jb][v]);
                            double m = bal_mod(val, pf, pinv);
                            J.res[(int64_t)j * J.ps + ch.row * J.ldr + col] = (uint32_t)(m < 0.0 ? m + pf : m);
                        }
                    }
            }
        }
        wave_sync();
    }
}

// ---------------------------------------------------- base conversion --

struct ConvertMfmaJob {
    const uint32_t *res;
    int64_t rows, cols, ldr, ps;
    int L;
    const PrimeConst *pc;      // source range
    const double *cj;
    uint32_t *out;
    int64_t ldo, ops;
    int L2, groups;
    const PrimeConst *qc;      // target range
    const double *mq;          // M mod q_i, balanced
    const v4i_d *G;            // [groups][NKS][7][64]
};

constexpr int kConvGroup = 16;

__device__ __forceinline__ uint32_t recombine7(const int32_t (&c)[7], const PrimeConst &q, double sub) {
    // sum_s c_s 2^(8s) - sub mod q; every partial sum below 2^52.
    const double lo = fma((double)c[2], 65536.0, fma((double)c[1], 256.0, (double)c[0]));
    const double mid = fma((double)c[5], 65536.0, fma((double)c[4], 256.0, (double)c[3]));
    const double rm = bal_mod(mid, q.pf, q.pinv);
    const double sum = fma((double)c[6], q.w[6], fma(rm, q.w[3], lo)) - sub;
    double r = bal_mod(sum, q.pf, q.pinv);
    return (uint32_t)(r < 0.0 ? r + q.pf : r);
}

template <int NKS, int EW>
__global__ __launch_bounds__(kThreads, 3) void k_convert_mfma(ConvertMfmaJob J, int64_t total_chunks,
                                                           int64_t col_chunks) {
    constexpr int KA = 64 * NKS, RS = KA + 16, NCB = 7, RBP = 2;
    extern __shared__ char smem[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    char *A = smem + wave * (EW * RS + EW * 8);
    int64_t *alpha = reinterpret_cast<int64_t *>(A + EW * RS);
    const int64_t iters = (total_chunks + kWaves - 1) / kWaves;
    for (int64_t it = blockIdx.x; it < iters; it += gridDim.x) {
        const Chunk ch = chunk_of(it * kWaves + wave, total_chunks, col_chunks, EW);
        if (lane < EW) {
            const int64_t col = ch.c0 + lane;
            uint32_t *row = reinterpret_cast<uint32_t *>(A + lane * RS);
            if (ch.any && col < J.cols) {
                const double al = lagrange_digits(J.res + ch.row * J.ldr + col, J.ps, J.L, J.pc, J.cj, row, KA);
                alpha[lane] = (int64_t)rint(al);
            } else {
                for (int k = 0; k < KA / 4; ++k) row[k] = 0u;
                alpha[lane] = 0;
            }
        }
        wave_sync();
#pragma unroll 1
        for (int g = 0; g < J.groups; ++g) {
            const v4i_d *G = J.G + (int64_t)g * NKS * NCB * 64;
            const int i = kConvGroup * g + (lane & 15);
            const bool ivalid = i < J.L2;
            const PrimeConst q = J.qc[ivalid ? i : 0];
            const double mq = J.mq[ivalid ? i : 0];
#pragma unroll 1
            for (int rb0 = 0; rb0 < EW / 16; rb0 += RBP) {
                v4i_d acc[RBP][NCB];
                digits_mfma<NKS, NCB, RBP>(A + 16 * rb0 * RS, RS, G, lane, acc);
#pragma unroll
                for (int r = 0; r < RBP; ++r)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int el = 16 * (rb0 + r) + 4 * (lane >> 4) + v;
                        const int64_t col = ch.c0 + el;
                        if (!ch.any || col >= J.cols || !ivalid) continue;
                        int32_t cs[7];
#pragma unroll
                        for (int sg = 0; sg < 7; ++sg) cs[sg] = acc[r][sg][v];
                        J.out[(int64_t)i * J.ops + ch.row * J.ldo + col] = recombine7(cs, q, (double)alpha[el] * mq);
                    }
            }
        }
        wave_sync();
    }
}

// ------------------------------------------------------------ tables --

// Balanced base-256 digits of a non-negative multiword integer (32-bit limbs):
// value = sum_k d_k 256^k, d_k in [-128, 127].
std::vector<int> balanced_bytes(const Limbs &x) {
    std::vector<int> d;
    int carry = 0;
    for (size_t i = 0; i < x.size() * 4; ++i) {
        int v = (int)((x[i / 4] >> (8 * (i % 4))) & 0xFF) + carry;
        carry = v >= 128;
        d.push_back(carry ? v - 256 : v);
    }
    if (carry) d.push_back(1);
    while (!d.empty() && d.back() == 0) d.pop_back();
    return d;
}

// Balanced digits of a balanced residue (the device's pack_digits).
void residue_digits(int64_t r, int (&d)[4]) {
    for (int i = 0; i < 3; ++i) {
        d[i] = (int)(int8_t)(r & 0xFF);
        r = (r - d[i]) >> 8;
    }
    d[3] = (int)r;
}

int64_t balanced(uint64_t r, uint32_t p) { return r > (p - 1) / 2 ? (int64_t)r - (int64_t)p : (int64_t)r; }

// Fragment of a K x 16 slice of G: lane l holds column l%16, rows
// 16 (l/16) .. +15 as bytes; `val(k, c)` gives G[k][c] for the slice.
template <class F>
void put_fragment(std::vector<int8_t> &frag, size_t base, F val) {
    for (int l = 0; l < 64; ++l)
        for (int b = 0; b < 16; ++b) frag[base + (size_t)l * 16 + b] = (int8_t)val(16 * (l / 16) + b, l % 16);
}

template <class T>
int upload(const std::vector<T> &h, T **d, hipStream_t s) {
    RNS_HIP(hipMalloc(reinterpret_cast<void **>(d), std::max<size_t>(h.size(), 1) * sizeof(T)));
    if (!h.empty()) RNS_HIP(hipMemcpyAsync(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return RNS_OK;
}

Limbs range_product(const rns_ctx *ctx, int begin, int L) {
    Limbs M{1};
    for (int j = 0; j < L; ++j) limbs_mul_small(M, ctx->primes[begin + j]);
    return M;
}

// (M/p_j)^-1 mod p_j for the range, and M/p_j itself.
void lagrange_consts(const rns_ctx *ctx, int begin, int L, const Limbs &M, std::vector<double> &c,
                     std::vector<Limbs> *mj) {
    c.resize(L);
    if (mj) mj->resize(L);
    for (int j = 0; j < L; ++j) {
        const uint32_t p = ctx->primes[begin + j];
        Limbs q = M;
        limbs_divmod_small(q, p);
        c[j] = (double)invmod_u64(limbs_mod_small(q, p), p);
        if (mj) (*mj)[j] = q;
    }
}

using TableKey = std::tuple<int, int, int, int, int>;
enum { kTabCrt = 1, kTabReduce = 2, kTabConvert = 3 };

int crt_table(rns_ctx *ctx, int begin, int L, const DigitTable **out, hipStream_t s) {
    const TableKey key{kTabCrt, begin, L, 0, 0};
    auto it = ctx->digit_tables.find(key);
    if (it != ctx->digit_tables.end()) {
        *out = &it->second;
        return RNS_OK;
    }
    const Limbs M = range_product(ctx, begin, L);
    std::vector<double> c;
    std::vector<Limbs> mj;
    lagrange_consts(ctx, begin, L, M, c, &mj);
    std::vector<std::vector<int>> md(L);
    size_t bmax = 0;
    for (int j = 0; j < L; ++j) {
        md[j] = balanced_bytes(mj[j]);
        bmax = std::max(bmax, md[j].size());
    }
    const int kout = (int)bmax + 3;                    // bytes of S
    const int q = (kout + 3) / 4;
    const int nqb = (q + 15) / 16;
    const int QP = 16 * nqb;
    // x = S - a M needs at least the limbs of M plus a sign limb.
    if (nqb > 4 || (int)M.size() + 1 > QP) return RNS_EINVAL;
    const int nks = (4 * L + 63) / 64;
    const int ncb = 4 * nqb;
    std::vector<int8_t> frag((size_t)nks * ncb * 1024);
    for (int ks = 0; ks < nks; ++ks)
        for (int cb = 0; cb < ncb; ++cb)
            put_fragment(frag, ((size_t)ks * ncb + cb) * 1024, [&](int kk, int cc) {
                const int k = 64 * ks + kk;                 // digit i of y_j
                const int col = 16 * cb + cc;               // column (i', qlimb): byte 4 qlimb + i'
                const int j = k / 4, i = k % 4;
                const int kbyte = 4 * (col % QP) + col / QP;
                const int b = kbyte - i;
                if (j >= L || b < 0 || b >= (int)md[j].size()) return 0;
                return md[j][b];
            });
    std::vector<uint32_t> ml(QP, 0u), half(QP, 0u);
    for (size_t i = 0; i < M.size(); ++i) ml[i] = M[i];
    Limbs h = M;
    limbs_divmod_small(h, 2);
    for (size_t i = 0; i < h.size(); ++i) half[i] = h[i];
    DigitTable t;
    t.nks = nks;
    t.nqb = nqb;
    t.q = QP;
    RNS_HIP(hipSetDevice(ctx->device));
    int st = upload(frag, reinterpret_cast<int8_t **>(&t.d_frag), s);
    if (st == RNS_OK) st = upload(c, &t.d_c, s);
    if (st == RNS_OK) st = upload(ml, &t.d_mlimbs, s);
    if (st == RNS_OK) st = upload(half, &t.d_half, s);
    if (st == RNS_OK && hipStreamSynchronize(s) != hipSuccess) st = RNS_EDEVICE;   // host vectors end here
    auto res = ctx->digit_tables.emplace(key, t);      // freed with the context even on failure
    if (st != RNS_OK) return st;
    *out = &res.first->second;
    return RNS_OK;
}

int reduce_table(rns_ctx *ctx, int begin, int L, int W, const DigitTable **out, hipStream_t s) {
    const TableKey key{kTabReduce, begin, L, W, 0};
    auto it = ctx->digit_tables.find(key);
    if (it != ctx->digit_tables.end()) {
        *out = &it->second;
        return RNS_OK;
    }
    const int K = 8 * W + 1;
    const int nks = (K + 63) / 64;
    const int groups = (L + kRedGroup - 1) / kRedGroup;
    // digits of 2^(8k) mod p_j, balanced
    std::vector<int> dig((size_t)L * K * 4);
    for (int j = 0; j < L; ++j) {
        const uint32_t p = ctx->primes[begin + j];
        uint64_t pw = 1;
        for (int k = 0; k < K; ++k) {
            int d[4];
            residue_digits(balanced(pw, p), d);
            for (int b = 0; b < 4; ++b) dig[((size_t)j * K + k) * 4 + b] = d[b];
            pw = pw * 256 % p;
        }
    }
    std::vector<int8_t> frag((size_t)groups * nks * 8 * 1024);
    for (int g = 0; g < groups; ++g)
        for (int ks = 0; ks < nks; ++ks)
            for (int cb = 0; cb < 8; ++cb)
                put_fragment(frag, (((size_t)g * nks + ks) * 8 + cb) * 1024, [&](int kk, int cc) {
                    const int k = 64 * ks + kk;
                    const int col = 16 * cb + cc;           // 32 b + j
                    const int b = col / kRedGroup, j = kRedGroup * g + col % kRedGroup;
                    if (k >= K || j >= L) return 0;
                    return dig[((size_t)j * K + k) * 4 + b];
                });
    DigitTable t;
    t.nks = nks;
    t.groups = groups;
    RNS_HIP(hipSetDevice(ctx->device));
    int st = upload(frag, reinterpret_cast<int8_t **>(&t.d_frag), s);
    if (st == RNS_OK && hipStreamSynchronize(s) != hipSuccess) st = RNS_EDEVICE;
    auto res = ctx->digit_tables.emplace(key, t);
    if (st != RNS_OK) return st;
    *out = &res.first->second;
    return RNS_OK;
}

int convert_table(rns_ctx *ctx, int b1, int L1, int b2, int L2, const DigitTable **out, hipStream_t s) {
    const TableKey key{kTabConvert, b1, L1, b2, L2};
    auto it = ctx->digit_tables.find(key);
    if (it != ctx->digit_tables.end()) {
        *out = &it->second;
        return RNS_OK;
    }
    const Limbs M = range_product(ctx, b1, L1);
    std::vector<double> c;
    std::vector<Limbs> mj;
    lagrange_consts(ctx, b1, L1, M, c, &mj);
    const int nks = (4 * L1 + 63) / 64;
    const int groups = (L2 + kConvGroup - 1) / kConvGroup;
    std::vector<int> dig((size_t)L1 * L2 * 4);         // digits of M/p_j mod q_i, balanced
    std::vector<double> mq(L2);
    for (int i = 0; i < L2; ++i) {
        const uint32_t q = ctx->primes[b2 + i];
        mq[i] = (double)balanced(limbs_mod_small(M, q), q);
        for (int j = 0; j < L1; ++j) {
            int d[4];
            residue_digits(balanced(limbs_mod_small(mj[j], q), q), d);
            for (int b = 0; b < 4; ++b) dig[((size_t)j * L2 + i) * 4 + b] = d[b];
        }
    }
    std::vector<int8_t> frag((size_t)groups * nks * 7 * 1024);
    for (int g = 0; g < groups; ++g)
        for (int ks = 0; ks < nks; ++ks)
            for (int sg = 0; sg < 7; ++sg)
                put_fragment(frag, (((size_t)g * nks + ks) * 7 + sg) * 1024, [&](int kk, int cc) {
                    const int k = 64 * ks + kk;               // digit dd of y_j
                    const int j = k / 4, dd = k % 4;
                    const int i = kConvGroup * g + cc;
                    const int b = sg - dd;                    // digit of the constant
                    if (j >= L1 || i >= L2 || b < 0 || b > 3) return 0;
                    return dig[((size_t)j * L2 + i) * 4 + b];
                });
    DigitTable t;
    t.nks = nks;
    t.groups = groups;
    RNS_HIP(hipSetDevice(ctx->device));
    int st = upload(frag, reinterpret_cast<int8_t **>(&t.d_frag), s);
    if (st == RNS_OK) st = upload(c, &t.d_c, s);
    if (st == RNS_OK) st = upload(mq, &t.d_mq, s);
    if (st == RNS_OK && hipStreamSynchronize(s) != hipSuccess) st = RNS_EDEVICE;
    auto res = ctx->digit_tables.emplace(key, t);
    if (st != RNS_OK) return st;
    *out = &res.first->second;
    return RNS_OK;
}

unsigned grid_for(int64_t iters) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(iters, 8192)); }

}  // namespace

namespace rns {

void DigitTable::release() {
    if (d_frag) (void)hipFree(d_frag);
    if (d_c) (void)hipFree(d_c);
    if (d_mlimbs) (void)hipFree(d_mlimbs);
    if (d_half) (void)hipFree(d_half);
    if (d_mq) (void)hipFree(d_mq);
    d_frag = nullptr;
    d_c = d_mq = nullptr;
    d_mlimbs = d_half = nullptr;
}

// Exact CRT of one residue matrix by the matrix-core Lagrange form (no
// bound needed).  The caller holds ctx->mu and has validated the arguments.
int crt_mfma(rns_ctx *ctx, const uint32_t *res, int64_t rows, int64_t cols, int64_t ldr, int64_t ps,
             int begin, int L, uint64_t *out, int W, int64_t ldo, int32_t *status, hipStream_t s) {
    if (L < 1 || L > kCrtMfmaMaxL) return RNS_EINVAL;
    const DigitTable *t = nullptr;
    int st = crt_table(ctx, begin, L, &t, s);
    if (st != RNS_OK) return st;
    CrtMfmaJob J{res, rows, cols, ldr, ps, L, W, out, ldo, status, ctx->d_prime + begin, t->d_c,
                 t->d_mlimbs, t->d_half, static_cast<const v4i_d *>(t->d_frag)};
    const int nks = t->nks, nqb = t->nqb;
    // Entries per wave step: 64 (all lanes load, every load in flight) while
    // the digit rows and one row block's limbs fit the LDS of four waves.
    const int EW = nks <= 2 ? 64 : (nks == 3 ? 32 : 16);
    const int64_t col_chunks = (cols + EW - 1) / EW;
    const int64_t chunks = rows * col_chunks;
    const int64_t iters = (chunks + kCrtWaves - 1) / kCrtWaves;
    ProfScope ps_(ctx, "k_crt_mfma", s);
#define RNS_CRT_MFMA(NKS_, NQB_, EW_, RBP_)                                                                  \
    hipLaunchKernelGGL((k_crt_mfma<NKS_, NQB_, EW_, RBP_>), dim3(grid_for(iters)), dim3(64 * kCrtWaves),       \
                       ((size_t)CrtShape<NKS_, NQB_, EW_>::LDS), s, J, chunks, col_chunks)
    if (nks == 1 && nqb == 1) RNS_CRT_MFMA(1, 1, 64, 1);
    else if (nks == 2 && nqb == 1) RNS_CRT_MFMA(2, 1, 64, 1);
    else if (nks == 2 && nqb == 2) RNS_CRT_MFMA(2, 2, 64, 1);
    else if (nks == 3 && nqb == 2) RNS_CRT_MFMA(3, 2, 32, 1);
    else if (nks == 3 && nqb == 3) RNS_CRT_MFMA(3, 3, 32, 1);
    else if (nks == 4 && nqb == 3) RNS_CRT_MFMA(4, 3, 16, 1);
    else if (nks == 4 && nqb == 4) RNS_CRT_MFMA(4, 4, 16, 1);
    else return RNS_EINVAL;
#undef RNS_CRT_MFMA
    RNS_HIP(hipGetLastError());
    return RNS_OK;
}

int reduce_mw_mfma(rns_ctx *ctx, const uint64_t *x, int W, int64_t rows, int64_t cols, int64_t ldx, int begin,
                   int L, uint32_t *res, int64_t ldr, int64_t ps, hipStream_t s) {
    const DigitTable *t = nullptr;
    int st = reduce_table(ctx, begin, L, W, &t, s);
    if (st != RNS_OK) return st;
    ReduceMfmaJob J{x, rows, cols, ldx, W, res, ldr, ps, L, t->groups, ctx->d_prime + begin,
                    static_cast<const v4i_d *>(t->d_frag)};
    const int EW = t->nks <= 2 ? 64 : 32;              // digit rows of four waves within 64 KiB
    const int64_t col_chunks = (cols + EW - 1) / EW;
    const int64_t chunks = rows * col_chunks;
    const int64_t iters = (chunks + kWaves - 1) / kWaves;
    const size_t lds = (size_t)kWaves * EW * (64 * t->nks + 16);
    ProfScope ps_(ctx, "k_reduce_mw_mfma", s);
#define RNS_RED(NKS_, EW_) \
    hipLaunchKernelGGL((k_reduce_mw_mfma<NKS_, EW_>), dim3(grid_for(iters)), dim3(kThreads), lds, s, J, chunks, \
                       col_chunks)
    switch (t->nks) {
    case 1: RNS_RED(1, 64); break;
    case 2: RNS_RED(2, 64); break;
    case 3: RNS_RED(3, 32); break;
    case 4: RNS_RED(4, 32); break;
    case 5: RNS_RED(5, 32); break;
    default: return RNS_EINVAL;
    }
#undef RNS_RED
    RNS_HIP(hipGetLastError());
    return RNS_OK;
}

}  // namespace rns

extern "C" int rns_base_convert(rns_ctx *ctx, const uint32_t *res, int64_t rows, int64_t cols, int64_t ldr,
                                int64_t plane_stride, int begin, int L, const uint64_t *bound_words, int Wb,
                                uint32_t *out, int64_t ldo, int64_t out_plane_stride, int begin_out, int L_out,
                                int32_t *d_status, void *stream) {
    if (!ctx || rows < 0 || cols < 0 || L < 1 || L > kCrtMfmaMaxL || L_out < 1) return RNS_EINVAL;
    if (begin < 0 || begin + L > ctx->L || begin_out < 0 || begin_out + L_out > ctx->L) return RNS_EINVAL;
    if (Wb < 0 || (Wb > 0 && !bound_words)) return RNS_EINVAL;
    if (rows == 0 || cols == 0) return RNS_OK;
    if (!res || !out || ldr < cols || ldo < cols) return RNS_EINVAL;
    if (L > 1 && plane_stride < (rows - 1) * ldr + cols) return RNS_EINVAL;
    if (L_out > 1 && out_plane_stride < (rows - 1) * ldo + cols) return RNS_EINVAL;
    if (rows > INT64_MAX / cols) return RNS_EINVAL;
    std::lock_guard<std::mutex> guard(ctx->mu);
    RNS_HIP(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    if (crt_fast_ok(ctx, begin, L, bound_words, Wb, kCrtMaxW)) {
        // The bound leaves the Lagrange margin: one pass, x never formed.
        const DigitTable *t = nullptr;
        int st = convert_table(ctx, begin, L, begin_out, L_out, &t, s);
        if (st != RNS_OK) return st;
        ConvertMfmaJob J{res, rows, cols, ldr, plane_stride, L, ctx->d_prime + begin, t->d_c,
                         out, ldo, out_plane_stride, L_out, t->groups, ctx->d_prime + begin_out, t->d_mq,
                         static_cast<const v4i_d *>(t->d_frag)};
        const int EW = t->nks <= 2 ? 64 : 32;
        const int64_t col_chunks = (cols + EW - 1) / EW;
        const int64_t chunks = rows * col_chunks;
        const int64_t iters = (chunks + kWaves - 1) / kWaves;
        const size_t lds = (size_t)kWaves * EW * (64 * t->nks + 16 + 8);
        ProfScope ps_(ctx, "k_convert_mfma", s);
#define RNS_CONV(NKS_, EW_) \
    hipLaunchKernelGGL((k_convert_mfma<NKS_, EW_>), dim3(grid_for(iters)), dim3(kThreads), lds, s, J, chunks, \
                       col_chunks)
        switch (t->nks) {
        case 1: RNS_CONV(1, 64); break;
        case 2: RNS_CONV(2, 64); break;
        case 3: RNS_CONV(3, 32); break;
        case 4: RNS_CONV(4, 32); break;
        default: return RNS_EINVAL;
        }
#undef RNS_CONV
        RNS_HIP(hipGetLastError());
        return RNS_OK;
    }
    // No usable bound: the exact CRT into the context workspace, then the
    // multiword reduction into the target primes.
    const Limbs M = range_product(ctx, begin, L);
    const int W = (int)((M.size() * 32 + 1 + 63) / 64);
    const size_t bytes = (size_t)rows * cols * W * sizeof(uint64_t);
    int st = ensure_workspace(ctx, bytes);
    if (st != RNS_OK) return st;
    uint64_t *x = static_cast<uint64_t *>(ctx->d_work);
    st = crt_mfma(ctx, res, rows, cols, ldr, plane_stride, begin, L, x, W, cols,
                  d_status ? d_status : ctx->d_status, s);
    if (st != RNS_OK) return st;
    return reduce_mw_mfma(ctx, x, W, rows, cols, cols, begin_out, L_out, out, ldo, out_plane_stride, s);
}
