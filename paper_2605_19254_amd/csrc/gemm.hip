// modmatmul_batched: one exact residue product per prime and per problem
// (Section 3.1: the product of two integer matrices becomes L independent
// word-size products, each exact, then reduced mod p).
//
// Two paths, both on the gfx950 matrix cores.
//
// FP64 path.  Residues are moved to the balanced range |r| <= (p-1)/2 and held
// as doubles.  v_mfma_f64_16x16x4f64 accumulates 4 products per step; after
// every 8 products the accumulator is reduced mod p with the rounded
// reciprocal (q = rint(acc/p), acc -= q*p, exact).  With p < 2^26,
//   8*((p-1)/2)^2 + (p+1)/2 < 2^53,
// so every partial sum is an integer below 2^53 and the result does not depend
// on the order of summation.  The paper's own rule bounds the whole dot
// product instead (n(p-1)^2 + (p-1) < 2^53, Section 3.1); blocking by 8 lets
// the 26-bit primes be used at any k.
//
// INT8 path.  Each balanced residue is split into four signed base-256 digits
// r = d0 + d1*2^8 + d2*2^16 + d3*2^24, d0..d2 in [-128, 127], |d3| <= 2.  The
// 16 digit-pair products are computed with v_mfma_i32_16x16x64_i8 and summed in
// int32 per shift group s = i+j (7 groups), which stays exact for k <= 43690.
// The epilogue reduces each group mod p and recombines
//   C = sum_s (C_s mod p) * (2^(8s) mod p)  (mod p)
// in exact double arithmetic.
//
// Both paths first copy the operands into a tiled layout in the context
// workspace ("prep"): one 16-row x 64-k tile of an operand becomes a
// contiguous block ordered exactly as the MFMA fragments are read, so every
// fragment load of the GEMM is one fully coalesced 1 KiB (INT8) or 512 B
// (FP64) access, and the padding to whole tiles is zero-filled.  All problems
// of a batch and all their primes are processed by one prep launch and one
// GEMM launch.
#include "internal.hpp"

#include <algorithm>
#include <cstring>
#include <vector>

using namespace rns;

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

// Work-group tiles.  INT8: 4 waves in 2x2, each 32 x 64 -> 64 x 128.
// FP64: 4 waves in 2x2, each 64 x 64 -> 128 x 128.
constexpr int kI8WaveRB = 2, kI8WaveCB = 4;
constexpr int kF64WaveRB = 4, kF64WaveCB = 4;
constexpr int kI8TileM = 2 * 16 * kI8WaveRB, kI8TileN = 2 * 16 * kI8WaveCB;
constexpr int kF64TileM = 2 * 16 * kF64WaveRB, kF64TileN = 2 * 16 * kF64WaveCB;
constexpr int kKTile = 64;   // k extent of one prep unit (both paths)

struct GemmProblem {
    const uint32_t *A, *B;
    uint32_t *C;
    int64_t lda, aps, ldb, bps, ldc, cps;
    int32_t m, n, k;
    int32_t L, prime_begin;
    int32_t RB, CB, KT;          // padded 16-row blocks of A, 16-col blocks of B, 64-k tiles
    int32_t tm, tn;              // work-group tiles along m and n
    char *At, *Bt;               // tiled operands in the workspace
    int64_t a_plane_bytes, b_plane_bytes;
    int64_t tile_begin;          // prefix over problems of L*tm*tn
    int64_t unitA_begin;         // prefix over problems of prep units (A then B)
    int64_t unitB_begin;
};

__device__ __forceinline__ int find_problem(const GemmProblem *P, int nprob, int64_t t,
                                            int64_t GemmProblem::*field) {
    int lo = 0, hi = nprob - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (P[mid].*field <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// XCD-aware remap: work-group b runs on XCD b % 8.  Give each XCD one
// contiguous range of logical tiles so that the tiles sharing operand panels
// share that XCD's L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t G) {
    const int64_t q = G / 8, r = G % 8;
    const int64_t x = b % 8, i = b / 8;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

__device__ __forceinline__ int32_t balanced(uint32_t r, uint32_t p, uint32_t half) {
    return r > half ? (int32_t)r - (int32_t)p : (int32_t)r;
}

// ------------------------------------------------------------------- prep --
// One wave converts one 16 x 64 operand tile.  "Operand rows" are the rows of
// A or the columns of B; k is the contraction index.
//   INT8 tile: 4 digit blocks of 64 lanes x 16 bytes; lane l holds operand row
//              l%16 and k = 16*(l/16) .. 16*(l/16)+15 of the tile.
//   FP64 tile: 16 fragments of 64 doubles; fragment f covers k = 4f .. 4f+3,
//              lane l holds operand row l%16 and k = 4f + l/16.

template <bool kInt8>
__global__ __launch_bounds__(256) void k_prep(const GemmProblem *__restrict__ P, int nprob,
                                              int64_t total_units,
                                              const PrimeConst *__restrict__ pc) {
    const int lane = threadIdx.x & 63;
    const int64_t unit = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (unit >= total_units) return;
    const int q = find_problem(P, nprob, unit, &GemmProblem::unitA_begin);
    const GemmProblem &g = P[q];
    const bool isB = unit >= g.unitB_begin;
    int64_t u = unit - (isB ? g.unitB_begin : g.unitA_begin);
    const int32_t nblk = isB ? g.CB : g.RB;
    const int64_t per_plane = (int64_t)nblk * g.KT;
    const int plane = (int)(u / per_plane);
    u -= (int64_t)plane * per_plane;
    const int blk = (int)(u / g.KT);
    const int kt = (int)(u - (int64_t)blk * g.KT);
    const PrimeConst &pr = pc[g.prime_begin + plane];
    const int row = blk * 16 + (lane & 15);
    const int rows_valid = isB ? g.n : g.m;
    const uint32_t *src = isB ? g.B + (int64_t)plane * g.bps : g.A + (int64_t)plane * g.aps;
    const int64_t ld = isB ? g.ldb : g.lda;
    auto fetch = [&](int kk) -> int32_t {
        if (row >= rows_valid || kk >= g.k) return 0;
        const uint32_t r = isB ? src[(int64_t)kk * ld + row] : src[(int64_t)row * ld + kk];
        return balanced(r, pr.p, pr.half);
    };
    char *dst = (isB ? g.Bt + (int64_t)plane * g.b_plane_bytes : g.At + (int64_t)plane * g.a_plane_bytes);
    if constexpr (kInt8) {
        const int k0 = kt * kKTile + (lane >> 4) * 16;
        uint32_t dig[4][4];
#pragma unroll
        for (int w = 0; w < 4; ++w) {
#pragma unroll
            for (int d = 0; d < 4; ++d) dig[d][w] = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                int32_t v = fetch(k0 + 4 * w + b);
                const int32_t d0 = (int32_t)(int8_t)(v & 0xFF);
                v = (v - d0) >> 8;
                const int32_t d1 = (int32_t)(int8_t)(v & 0xFF);
                v = (v - d1) >> 8;
                const int32_t d2 = (int32_t)(int8_t)(v & 0xFF);
                const int32_t d3 = (v - d2) >> 8;
                dig[0][w] |= ((uint32_t)d0 & 0xFF) << (8 * b);
                dig[1][w] |= ((uint32_t)d1 & 0xFF) << (8 * b);
                dig[2][w] |= ((uint32_t)d2 & 0xFF) << (8 * b);
                dig[3][w] |= ((uint32_t)d3 & 0xFF) << (8 * b);
            }
        }
        v4i *out = reinterpret_cast<v4i *>(dst) + ((int64_t)blk * g.KT + kt) * 256;
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            v4i t = {(int)dig[d][0], (int)dig[d][1], (int)dig[d][2], (int)dig[d][3]};
            out[d * 64 + lane] = t;
        }
    } else {
        double *out = reinterpret_cast<double *>(dst) + ((int64_t)blk * g.KT + kt) * 1024;
#pragma unroll
        for (int f = 0; f < 16; ++f)
            out[f * 64 + lane] = (double)fetch(kt * kKTile + 4 * f + (lane >> 4));
    }
}

// ----------------------------------------------------------- tile mapping --

struct TileCoord {
    int q, plane, tm, tn;
};

__device__ __forceinline__ TileCoord map_tile(const GemmProblem *P, int nprob, int64_t t) {
    TileCoord c;
    c.q = find_problem(P, nprob, t, &GemmProblem::tile_begin);
    const GemmProblem &g = P[c.q];
    int64_t u = t - g.tile_begin;
    const int64_t per_plane = (int64_t)g.tm * g.tn;
    c.plane = (int)(u / per_plane);
    u -= (int64_t)c.plane * per_plane;
    // Grouped raster inside a plane: 8 tile-rows at a time, column-major
    // within the group, so neighbouring work-groups share A and B panels.
    const int group = 8;
    const int64_t gsize = (int64_t)group * g.tn;
    const int gi = (int)(u / gsize);
    const int first = gi * group;
    const int rows_in = min(group, g.tm - first);
    const int64_t v = u - (int64_t)gi * gsize;
    c.tm = first + (int)(v % rows_in);
    c.tn = (int)(v / rows_in);
    return c;
}

// ------------------------------------------------------------- INT8 GEMM --

__global__ __launch_bounds__(256) void k_gemm_i8(const GemmProblem *__restrict__ P, int nprob,
                                                 int64_t total_tiles,
                                                 const PrimeConst *__restrict__ pc) {
    const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    if (t >= total_tiles) return;
    const TileCoord tc = map_tile(P, nprob, t);
    const GemmProblem &g = P[tc.q];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int rb0 = tc.tm * (2 * kI8WaveRB) + (wave >> 1) * kI8WaveRB;
    const int cb0 = tc.tn * (2 * kI8WaveCB) + (wave & 1) * kI8WaveCB;
    const int KT = g.KT;
    const v4i *Ab = reinterpret_cast<const v4i *>(g.At + (int64_t)tc.plane * g.a_plane_bytes) +
                    (int64_t)rb0 * KT * 256 + lane;
    const v4i *Bb = reinterpret_cast<const v4i *>(g.Bt + (int64_t)tc.plane * g.b_plane_bytes) +
                    (int64_t)cb0 * KT * 256 + lane;

    v4i acc[7][kI8WaveRB][kI8WaveCB];
#pragma unroll
    for (int s = 0; s < 7; ++s)
#pragma unroll
        for (int i = 0; i < kI8WaveRB; ++i)
#pragma unroll
            for (int j = 0; j < kI8WaveCB; ++j) acc[s][i][j] = v4i{0, 0, 0, 0};

    v4i a[kI8WaveRB][4], b[kI8WaveCB][4];
    v4i an[kI8WaveRB][4], bn[kI8WaveCB][4];
    auto load = [&](int kt, v4i (&ar)[kI8WaveRB][4], v4i (&br)[kI8WaveCB][4]) {
#pragma unroll
        for (int i = 0; i < kI8WaveRB; ++i)
#pragma unroll
            for (int d = 0; d < 4; ++d)
                ar[i][d] = Ab[((int64_t)i * KT + kt) * 256 + d * 64];
#pragma unroll
        for (int j = 0; j < kI8WaveCB; ++j)
#pragma unroll
            for (int d = 0; d < 4; ++d)
                br[j][d] = Bb[((int64_t)j * KT + kt) * 256 + d * 64];
    };
    load(0, a, b);
    for (int kt = 0; kt < KT; ++kt) {
        if (kt + 1 < KT) load(kt + 1, an, bn);
#pragma unroll
        for (int da = 0; da < 4; ++da)
#pragma unroll
            for (int db = 0; db < 4; ++db)
#pragma unroll
                for (int i = 0; i < kI8WaveRB; ++i)
#pragma unroll
                    for (int j = 0; j < kI8WaveCB; ++j)
                        acc[da + db][i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(
                            a[i][da], b[j][db], acc[da + db][i][j], 0, 0, 0);
        if (kt + 1 < KT) {
#pragma unroll
            for (int i = 0; i < kI8WaveRB; ++i)
#pragma unroll
                for (int d = 0; d < 4; ++d) a[i][d] = an[i][d];
#pragma unroll
            for (int j = 0; j < kI8WaveCB; ++j)
#pragma unroll
                for (int d = 0; d < 4; ++d) b[j][d] = bn[j][d];
        }
    }

    // Epilogue: C = sum_s (C_s mod p) * w_s mod p, all in exact doubles.
    const PrimeConst pr = pc[g.prime_begin + tc.plane];
    uint32_t *C = g.C + (int64_t)tc.plane * g.cps;
#pragma unroll
    for (int i = 0; i < kI8WaveRB; ++i)
#pragma unroll
        for (int j = 0; j < kI8WaveCB; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                double sum = 0.0;
#pragma unroll
                for (int s = 0; s < 7; ++s) {
                    const double cs = (double)acc[s][i][j][v];
                    const double r = fma(-rint(cs * pr.pinv), pr.pf, cs);   // |r| <= p/2
                    sum = fma(r, pr.w[s], sum);                              // |sum| < 7*2^50
                }
                double r = fma(-rint(sum * pr.pinv), pr.pf, sum);
                r = r < 0.0 ? r + pr.pf : r;
                const int row = (rb0 + i) * 16 + 4 * (lane >> 4) + v;
                const int col = (cb0 + j) * 16 + (lane & 15);
                if (row < g.m && col < g.n) C[(int64_t)row * g.ldc + col] = (uint32_t)r;
            }
}

// ------------------------------------------------- INT8 GEMM, LDS pipeline --
// Same tiles and arithmetic as k_gemm_i8, but the work-group's A and B digit
// tiles of one 64-k step (4 + 8 row/col blocks x 4 digits = 48 fragments of
// 1 KiB) are copied global -> LDS with 16-byte direct loads into two
// alternating buffers, and each wave reads its fragments from LDS.  The two
// waves that share an A (B) panel read it once from L2 instead of twice, and
// no registers hold prefetched fragments.
//
// Order inside a step: wait for this wave's copies of step kt, barrier (now
// every wave's copies of step kt are in LDS and every wave has finished
// reading step kt-1), read the fragments of step kt, start the copies of step
// kt+1 into the other buffer, then run the 128 MFMAs of step kt while those
// copies are in flight.

constexpr int kI8FragA = 2 * kI8WaveRB * 4;           // A fragments per 64-k step
constexpr int kI8FragB = 2 * kI8WaveCB * 4;           // B fragments per 64-k step
constexpr int kI8Frag = kI8FragA + kI8FragB;          // 48
constexpr int kI8FragPerWave = kI8Frag / 4;           // 12

typedef __attribute__((address_space(3))) void lds_void;

__device__ __forceinline__ void vm_wait_0() { __builtin_amdgcn_s_waitcnt(0x0F70); }   // vmcnt(0)

__device__ __forceinline__ void plain_barrier() {
    // A fenced barrier would make the compiler wait for every outstanding
    // copy; the copies this barrier must cover were already waited for.  The
    // empty asm statements keep the compiler from moving memory accesses
    // across the barrier.
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

__global__ __launch_bounds__(256) void k_gemm_i8_lds(const GemmProblem *__restrict__ P, int nprob,
                                                     int64_t total_tiles,
                                                     const PrimeConst *__restrict__ pc) {
    __shared__ v4i sbuf[2][kI8Frag * 64];
    const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    if (t >= total_tiles) return;
    const TileCoord tc = map_tile(P, nprob, t);
    const GemmProblem &g = P[tc.q];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wy = wave >> 1, wx = wave & 1;
    const int KT = g.KT;
    const char *Ag = g.At + (int64_t)tc.plane * g.a_plane_bytes +
                     (int64_t)tc.tm * (2 * kI8WaveRB) * KT * 4096 + lane * 16;
    const char *Bg = g.Bt + (int64_t)tc.plane * g.b_plane_bytes +
                     (int64_t)tc.tn * (2 * kI8WaveCB) * KT * 4096 + lane * 16;
    // Fragment f of a step: f < kI8FragA is A block f/4, digit f%4; otherwise
    // B block (f-kI8FragA)/4, digit (f-kI8FragA)%4.  Wave w copies f = 12w..12w+11.
    const char *src[kI8FragPerWave];
#pragma unroll
    for (int i = 0; i < kI8FragPerWave; ++i) {
        const int f = wave * kI8FragPerWave + i;
        src[i] = f < kI8FragA ? Ag + ((int64_t)(f >> 2) * KT) * 4096 + (f & 3) * 1024
                              : Bg + ((int64_t)((f - kI8FragA) >> 2) * KT) * 4096 + ((f - kI8FragA) & 3) * 1024;
    }
    auto issue = [&](v4i *buf, int kt) {
#pragma unroll
        for (int i = 0; i < kI8FragPerWave; ++i) {
            const int f = wave * kI8FragPerWave + i;
            __builtin_amdgcn_global_load_lds((const void *)(src[i] + (int64_t)kt * 4096),
                                             (lds_void *)(buf + f * 64), 16, 0, 0);
        }
    };

    v4i acc[7][kI8WaveRB][kI8WaveCB];
#pragma unroll
    for (int s = 0; s < 7; ++s)
#pragma unroll
        for (int i = 0; i < kI8WaveRB; ++i)
#pragma unroll
            for (int j = 0; j < kI8WaveCB; ++j) acc[s][i][j] = v4i{0, 0, 0, 0};

    issue(sbuf[0], 0);
    for (int kt = 0; kt < KT; ++kt) {
        const v4i *cur = sbuf[kt & 1];
        vm_wait_0();
        plain_barrier();
        v4i a[kI8WaveRB][4], b[kI8WaveCB][4];
#pragma unroll
        for (int i = 0; i < kI8WaveRB; ++i)
#pragma unroll
            for (int d = 0; d < 4; ++d) a[i][d] = cur[((wy * kI8WaveRB + i) * 4 + d) * 64 + lane];
#pragma unroll
        for (int j = 0; j < kI8WaveCB; ++j)
#pragma unroll
            for (int d = 0; d < 4; ++d) b[j][d] = cur[(kI8FragA + (wx * kI8WaveCB + j) * 4 + d) * 64 + lane];
        if (kt + 1 < KT) issue(sbuf[(kt + 1) & 1], kt + 1);
#pragma unroll
        for (int da = 0; da < 4; ++da)
#pragma unroll
            for (int db = 0; db < 4; ++db)
#pragma unroll
                for (int i = 0; i < kI8WaveRB; ++i)
#pragma unroll
                    for (int j = 0; j < kI8WaveCB; ++j)
                        acc[da + db][i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(
                            a[i][da], b[j][db], acc[da + db][i][j], 0, 0, 0);
    }

    const int rb0 = tc.tm * (2 * kI8WaveRB) + wy * kI8WaveRB;
    const int cb0 = tc.tn * (2 * kI8WaveCB) + wx * kI8WaveCB;
    const PrimeConst pr = pc[g.prime_begin + tc.plane];
    uint32_t *C = g.C + (int64_t)tc.plane * g.cps;
#pragma unroll
    for (int i = 0; i < kI8WaveRB; ++i)
#pragma unroll
        for (int j = 0; j < kI8WaveCB; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                double sum = 0.0;
#pragma unroll
                for (int s = 0; s < 7; ++s) {
                    const double cs = (double)acc[s][i][j][v];
                    const double r = fma(-rint(cs * pr.pinv), pr.pf, cs);
                    sum = fma(r, pr.w[s], sum);
                }
                double r = fma(-rint(sum * pr.pinv), pr.pf, sum);
                r = r < 0.0 ? r + pr.pf : r;
                const int row = (rb0 + i) * 16 + 4 * (lane >> 4) + v;
                const int col = (cb0 + j) * 16 + (lane & 15);
                if (row < g.m && col < g.n) C[(int64_t)row * g.ldc + col] = (uint32_t)r;
            }
}

// ------------------------------------------------------------- FP64 GEMM --

__global__ __launch_bounds__(256) void k_gemm_f64(const GemmProblem *__restrict__ P, int nprob,
                                                  int64_t total_tiles,
                                                  const PrimeConst *__restrict__ pc) {
    const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    if (t >= total_tiles) return;
    const TileCoord tc = map_tile(P, nprob, t);
    const GemmProblem &g = P[tc.q];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int rb0 = tc.tm * (2 * kF64WaveRB) + (wave >> 1) * kF64WaveRB;
    const int cb0 = tc.tn * (2 * kF64WaveCB) + (wave & 1) * kF64WaveCB;
    const int F = g.KT * 16;   // 4-k fragments per 16-row block
    const double *Ab = reinterpret_cast<const double *>(g.At + (int64_t)tc.plane * g.a_plane_bytes) +
                       (int64_t)rb0 * F * 64 + lane;
    const double *Bb = reinterpret_cast<const double *>(g.Bt + (int64_t)tc.plane * g.b_plane_bytes) +
                       (int64_t)cb0 * F * 64 + lane;
    const PrimeConst pr = pc[g.prime_begin + tc.plane];

    v4d acc[kF64WaveRB][kF64WaveCB];
#pragma unroll
    for (int i = 0; i < kF64WaveRB; ++i)
#pragma unroll
        for (int j = 0; j < kF64WaveCB; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

    double a[kF64WaveRB][2], b[kF64WaveCB][2], an[kF64WaveRB][2], bn[kF64WaveCB][2];
    auto load = [&](int f2, double (&ar)[kF64WaveRB][2], double (&br)[kF64WaveCB][2]) {
#pragma unroll
        for (int i = 0; i < kF64WaveRB; ++i)
#pragma unroll
            for (int s = 0; s < 2; ++s) ar[i][s] = Ab[((int64_t)i * F + 2 * f2 + s) * 64];
#pragma unroll
        for (int j = 0; j < kF64WaveCB; ++j)
#pragma unroll
            for (int s = 0; s < 2; ++s) br[j][s] = Bb[((int64_t)j * F + 2 * f2 + s) * 64];
    };
    const int F2 = F / 2;   // 8-k steps; the accumulator is reduced after each
    load(0, a, b);
    for (int f2 = 0; f2 < F2; ++f2) {
        if (f2 + 1 < F2) load(f2 + 1, an, bn);
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int i = 0; i < kF64WaveRB; ++i)
#pragma unroll
                for (int j = 0; j < kF64WaveCB; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i][s], b[j][s], acc[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < kF64WaveRB; ++i)
#pragma unroll
            for (int j = 0; j < kF64WaveCB; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const double x = acc[i][j][v];
                    acc[i][j][v] = fma(-rint(x * pr.pinv), pr.pf, x);
                }
        if (f2 + 1 < F2) {
#pragma unroll
            for (int i = 0; i < kF64WaveRB; ++i)
#pragma unroll
                for (int s = 0; s < 2; ++s) a[i][s] = an[i][s];
#pragma unroll
            for (int j = 0; j < kF64WaveCB; ++j)
#pragma unroll
                for (int s = 0; s < 2; ++s) b[j][s] = bn[j][s];
        }
    }

    uint32_t *C = g.C + (int64_t)tc.plane * g.cps;
#pragma unroll
    for (int i = 0; i < kF64WaveRB; ++i)
#pragma unroll
        for (int j = 0; j < kF64WaveCB; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                double r = acc[i][j][v];
                r = r < 0.0 ? r + pr.pf : r;
                // v_mfma_f64_16x16x4f64 returns D[4v + lane/16][lane%16] in
                // register v of lane `lane` (the INT8 form uses 4*(lane/16) + v).
                const int row = (rb0 + i) * 16 + 4 * v + (lane >> 4);
                const int col = (cb0 + j) * 16 + (lane & 15);
                if (row < g.m && col < g.n) C[(int64_t)row * g.ldc + col] = (uint32_t)r;
            }
}

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

struct Plan {
    std::vector<GemmProblem> probs;
    size_t work_bytes = 0;
    int64_t total_tiles = 0;
    int64_t total_units = 0;
};

int make_plan(rns_ctx *ctx, const rns_gemm_desc *d, int count, bool int8, Plan &plan) {
    const int TM = int8 ? kI8TileM : kF64TileM;
    const int TN = int8 ? kI8TileN : kF64TileN;
    const int64_t elem = int8 ? 4 : 8;   // bytes per operand entry in the tiled layout
    size_t off = 0;
    for (int i = 0; i < count; ++i) {
        const rns_gemm_desc &x = d[i];
        if (x.m < 0 || x.n < 0 || x.k < 0 || x.L < 0) return RNS_EINVAL;
        if (x.prime_begin < 0 || x.prime_begin + x.L > ctx->L) return RNS_EINVAL;
        if (x.m > INT32_MAX / 2 || x.n > INT32_MAX / 2 || x.k > INT32_MAX / 2) return RNS_EINVAL;
        if (x.m == 0 || x.n == 0 || x.L == 0) continue;
        if (!x.C || x.ldc < x.n) return RNS_EINVAL;
        if (x.L > 1 && x.c_plane_stride < (x.m - 1) * x.ldc + x.n) return RNS_EINVAL;
        if (x.k > 0) {
            if (!x.A || !x.B || x.lda < x.k || x.ldb < x.n) return RNS_EINVAL;
            if (x.L > 1 && (x.a_plane_stride < (x.m - 1) * x.lda + x.k ||
                            x.b_plane_stride < (x.k - 1) * x.ldb + x.n))
                return RNS_EINVAL;
        }
        if (int8 && x.k > kInt8MaxK) return RNS_EBOUND;
        GemmProblem g{};
        g.A = x.A; g.B = x.B; g.C = x.C;
        g.lda = x.lda; g.aps = x.a_plane_stride;
        g.ldb = x.ldb; g.bps = x.b_plane_stride;
        g.ldc = x.ldc; g.cps = x.c_plane_stride;
        g.m = (int32_t)x.m; g.n = (int32_t)x.n; g.k = (int32_t)x.k;
        g.L = x.L; g.prime_begin = x.prime_begin;
        const int64_t Mp = round_up(x.m, TM), Np = round_up(x.n, TN);
        const int64_t Kp = round_up(std::max<int64_t>(x.k, 1), kKTile);
        g.RB = (int32_t)(Mp / 16); g.CB = (int32_t)(Np / 16); g.KT = (int32_t)(Kp / kKTile);
        g.tm = (int32_t)(Mp / TM); g.tn = (int32_t)(Np / TN);
        g.a_plane_bytes = Mp * Kp * elem;
        g.b_plane_bytes = Np * Kp * elem;
        g.At = reinterpret_cast<char *>(off);
        off += (size_t)g.a_plane_bytes * g.L;
        g.Bt = reinterpret_cast<char *>(off);
        off += (size_t)g.b_plane_bytes * g.L;
        off = (off + 255) & ~(size_t)255;
        g.tile_begin = plan.total_tiles;
        plan.total_tiles += (int64_t)g.L * g.tm * g.tn;
        g.unitA_begin = plan.total_units;
        g.unitB_begin = g.unitA_begin + (int64_t)g.L * g.RB * g.KT;
        plan.total_units = g.unitB_begin + (int64_t)g.L * g.CB * g.KT;
        plan.probs.push_back(g);
    }
    plan.work_bytes = off;
    return RNS_OK;
}

}  // namespace

extern "C" int rns_workspace_bytes(rns_ctx *ctx, const rns_gemm_desc *descs, int count,
                                   int path, size_t *bytes) {
    if (!ctx || !bytes || count < 0 || (count > 0 && !descs)) return RNS_EINVAL;
    const bool int8 = path != RNS_PATH_FP64;
    Plan plan;
    int st = make_plan(ctx, descs, count, int8, plan);
    if (st != RNS_OK) return st;
    *bytes = plan.work_bytes;
    return RNS_OK;
}

extern "C" int modmatmul_batched(rns_ctx *ctx, const rns_gemm_desc *descs, int count,
                                 int path, void *stream) {
    if (!ctx || count < 0 || (count > 0 && !descs)) return RNS_EINVAL;
    if (path != RNS_PATH_AUTO && path != RNS_PATH_FP64 && path != RNS_PATH_INT8) return RNS_EINVAL;
    if (count == 0) return RNS_OK;
    bool int8 = path != RNS_PATH_FP64;
    std::lock_guard<std::mutex> guard(ctx->mu);
    Plan plan;
    int st = make_plan(ctx, descs, count, int8, plan);
    if (st == RNS_EBOUND && path == RNS_PATH_AUTO) {
        int8 = false;
        plan = Plan();
        st = make_plan(ctx, descs, count, int8, plan);
    }
    if (st != RNS_OK) return st;
    if (plan.probs.empty()) return RNS_OK;
    RNS_HIP(hipSetDevice(ctx->device));
    st = ensure_workspace(ctx, plan.work_bytes);
    if (st != RNS_OK) return st;
    for (auto &g : plan.probs) {
        g.At = static_cast<char *>(ctx->d_work) + reinterpret_cast<size_t>(g.At);
        g.Bt = static_cast<char *>(ctx->d_work) + reinterpret_cast<size_t>(g.Bt);
    }
    const size_t tbytes = sizeof(GemmProblem) * plan.probs.size();
    st = ensure_desc(ctx, tbytes);
    if (st != RNS_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    // The pinned staging buffer may still be read by an earlier copy on this
    // stream; wait for it before overwriting.
    RNS_HIP(hipStreamSynchronize(s));
    std::memcpy(ctx->h_desc, plan.probs.data(), tbytes);
    RNS_HIP(hipMemcpyAsync(ctx->d_desc, ctx->h_desc, tbytes, hipMemcpyHostToDevice, s));
    const GemmProblem *dP = static_cast<const GemmProblem *>(ctx->d_desc);
    const int np = (int)plan.probs.size();
    const int64_t prep_blocks = (plan.total_units + 3) / 4;
    {
    ProfScope ps(ctx, int8 ? "k_prep_i8" : "k_prep_f64", s);
    if (int8)
        hipLaunchKernelGGL(k_prep<true>, dim3((unsigned)prep_blocks), dim3(256), 0, s, dP, np,
                           plan.total_units, (const PrimeConst *)ctx->d_prime);
    else
        hipLaunchKernelGGL(k_prep<false>, dim3((unsigned)prep_blocks), dim3(256), 0, s, dP, np,
                           plan.total_units, (const PrimeConst *)ctx->d_prime);
    }
    RNS_HIP(hipGetLastError());
    {
    ProfScope ps(ctx, int8 ? "k_gemm_i8" : "k_gemm_f64", s);
    if (int8 && ctx->int8_kernel == 1)
        hipLaunchKernelGGL(k_gemm_i8, dim3((unsigned)plan.total_tiles), dim3(256), 0, s, dP, np,
                           plan.total_tiles, (const PrimeConst *)ctx->d_prime);
    else if (int8)
        hipLaunchKernelGGL(k_gemm_i8_lds, dim3((unsigned)plan.total_tiles), dim3(256), 0, s, dP, np,
                           plan.total_tiles, (const PrimeConst *)ctx->d_prime);
    else
        hipLaunchKernelGGL(k_gemm_f64, dim3((unsigned)plan.total_tiles), dim3(256), 0, s, dP, np,
                           plan.total_tiles, (const PrimeConst *)ctx->d_prime);
    }
    RNS_HIP(hipGetLastError());
    return RNS_OK;
}
