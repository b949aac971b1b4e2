// Shared pieces of the residue-product kernels: the problem table that the
// host builds for one modmatmul_batched call, the work-group tile shapes, the
// XCD-aware tile order and the balanced-residue conversion.
#pragma once

#include "internal.hpp"

namespace rns {
namespace gemm {

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
    int32_t sub;                 // 1: C := C - A B mod p
    int32_t RB, CB, KT;          // padded 16-row blocks of A, 16-col blocks of B, 64-k tiles
    int32_t tm, tn;              // work-group tiles along m and n
    char *At, *Bt;               // tiled operands in the workspace
    int64_t a_plane_bytes, b_plane_bytes;
    int64_t tile_begin;          // prefix over problems of L*tm*tn (tm*tn with the CRT fused)
    int64_t unitA_begin;         // prefix over problems of prep units (A then B)
    int64_t unitB_begin;
    // int64 operands (whole-product plans): the conversion kernel reduces them
    // straight into the tiled layouts, one unit per tile for all primes.
    const int64_t *A64, *B64;
    int64_t lda64, ldb64;
    int64_t u64A_begin, u64B_begin;   // prefix over problems of those units (A then B)
    // Plans with the CRT fused into the GEMM (at most two primes): the int64
    // result and p_0^{-1} mod p_1 of the problem's two primes.
    int64_t *C64;
    int64_t ldc64;
    uint32_t crt_inv;
};

__host__ __device__ __forceinline__ int find_problem(const GemmProblem *P, int nprob, int64_t t,
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
__host__ __device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t G) {
    const int64_t q = G / 8, r = G % 8;
    const int64_t x = b % 8, i = b / 8;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// The tile-order functions are also built for the host, where a test checks
// that they cover every tile exactly once.
//
// Windowed XCD remap, used by the GEMM kernels: XCD x (work-groups b with
// b % 8 == x) takes windows x, x+8, x+16, ... of W consecutive logical
// indices, W = the work-groups one XCD holds at a time.  The eight XCDs then
// work on neighbouring windows at the same time, inside one prime's operand
// planes (128 MB at n = 4096, which the 256 MB Infinity Cache holds), while
// each XCD's L2 still sees W neighbouring tiles.  Giving each XCD one
// contiguous range instead (xcd_remap) puts the XCDs on eight different
// primes at once; on MI355X the INT8 GEMM at n = 4096 with 24 primes ran 4 %
// slower that way.  The indices past the last full round of 8 W use
// xcd_remap.
// Work-groups one XCD of MI355X holds at a time (32 CUs) for kernels with one
// and with two work-groups per CU.
constexpr int64_t kXcdWindow1 = 32, kXcdWindow2 = 64;

__host__ __device__ __forceinline__ int64_t xcd_window_remap(int64_t b, int64_t G, int64_t W) {
    const int64_t full = G / (8 * W) * (8 * W);
    if (b >= full) return full + xcd_remap(b - full, G - full);
    const int64_t x = b % 8, i = b / 8;
    return ((i / W) * 8 + x) * W + i % W;
}

__device__ __forceinline__ int32_t balanced(uint32_t r, uint32_t p, uint32_t half) {
    return r > half ? (int32_t)r - (int32_t)p : (int32_t)r;
}

// ----------------------------------------------------------- tile mapping --

struct TileCoord {
    int q, plane, tm, tn;
};

// tile_prob (optional): the problem index of every tile, built by plans so
// that a batch of many problems needs one load instead of a search per tile.
__host__ __device__ __forceinline__ TileCoord map_tile(const GemmProblem *P, int nprob, int64_t t,
                                              const int32_t *tile_prob) {
    TileCoord c;
    c.q = tile_prob ? tile_prob[t] : find_problem(P, nprob, t, &GemmProblem::tile_begin);
    const GemmProblem &g = P[c.q];
    // A problem has fewer than 2^31 tiles (the host checks), so the index
    // arithmetic inside it is 32-bit.
    uint32_t u = (uint32_t)(t - g.tile_begin);
    const uint32_t per_plane = (uint32_t)g.tm * (uint32_t)g.tn;
    c.plane = (int)(u / per_plane);
    u -= (uint32_t)c.plane * per_plane;
    // Grouped raster inside a plane: 8 tile-rows at a time, column-major
    // within the group, so neighbouring work-groups share A and B panels.
    const uint32_t group = 8;
    const uint32_t gsize = group * (uint32_t)g.tn;
    const uint32_t gi = u / gsize;
    const uint32_t first = gi * group;
    const uint32_t rows_in = min(group, (uint32_t)g.tm - first);
    const uint32_t v = u - gi * gsize;
    c.tm = (int)(first + v % rows_in);
    c.tn = (int)(v / rows_in);
    return c;
}

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Stores one reduced product r in [0, p) at C, or C - r mod p when sub is set.
__device__ __forceinline__ void store_residue(uint32_t *C, uint32_t r, uint32_t p, int32_t sub) {
    if (sub) {
        const uint32_t c0 = *C;
        r = c0 >= r ? c0 - r : c0 + p - r;
    }
    *C = r;
}

// Launchers (one per kernel family), all asynchronous on `s`.
// INT8 GEMM variants (the autotuner chooses among them per shape class).
enum { kI8Lds = 0, kI8Direct = 1, kI8HalfPersistent = 2, kI8Wave8 = 3, kI8Half = 4, kI8NumVariants = 5 };
constexpr int kI8Default = kI8Half;

void launch_prep(bool int8, const GemmProblem *P, int nprob, int64_t units,
                 const PrimeConst *pc, unsigned *counter, hipStream_t s);
void launch_prep_i64(bool int8, const GemmProblem *P, int nprob, int64_t units,
                     const PrimeConst *pc, unsigned *counter, hipStream_t s);
void launch_gemm_i8(int variant, const GemmProblem *P, int nprob, int64_t tiles,
                    const PrimeConst *pc, const int32_t *tile_prob, unsigned *counter,
                    int num_cus, hipStream_t s);
// Both primes of each tile in one work-group, CRT to int64 in the epilogue.
void launch_gemm_i8_crt(const GemmProblem *P, int nprob, int64_t tiles, const PrimeConst *pc,
                        const int32_t *tile_prob, hipStream_t s);
void launch_gemm_f64(const GemmProblem *P, int nprob, int64_t tiles, const PrimeConst *pc,
                     const int32_t *tile_prob, hipStream_t s);

}  // namespace gemm
}  // namespace rns
