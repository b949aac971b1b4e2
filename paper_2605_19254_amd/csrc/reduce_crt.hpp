// Job descriptors of the reduction and CRT kernels, so that one launch can
// cover one matrix (job by value) or every matrix of a batched plan (job
// table in device memory).
#pragma once

#include "internal.hpp"

namespace rns {

struct ReduceJob {
    const int64_t *x;
    int64_t rows, cols, ldx;
    uint32_t *res;
    int64_t ldr, ps;
    int32_t prime_begin, L;
    int32_t vec;             // rows and planes allow 16-byte accesses of 4 entries
    int64_t col_tiles;
    int64_t tile_begin;      // prefix over jobs of rows * col_tiles
};

struct CrtJob {
    const uint32_t *res;
    int64_t rows, cols, ldr, ps;
    int32_t prime_begin, L;
    uint64_t *out;
    int64_t ldo;
    // Lagrange form (fast): per-range constants; unused by the Garner form.
    const double *lag_c;
    const uint64_t *lag_mj;
    const uint64_t *lag_m;
    // Garner form (exact): mixed-radix digits of (M-1)/2.
    const uint32_t *half;
    int32_t *status;
    int64_t col_tiles;
    int64_t tile_begin;
};

int reduce_check(const rns_ctx *ctx, const int64_t *x, int64_t rows, int64_t cols, int64_t ldx,
                 int prime_begin, int L, const uint32_t *res, int64_t ldr, int64_t plane_stride);
ReduceJob make_reduce_job(const int64_t *x, int64_t rows, int64_t cols, int64_t ldx,
                          int prime_begin, int L, uint32_t *res, int64_t ldr,
                          int64_t plane_stride, int64_t tile_begin);
int64_t reduce_tiles(const ReduceJob &j);
void launch_reduce(const ReduceJob &job0, const ReduceJob *jobs, int njobs, int64_t total_tiles,
                   const PrimeConst *pc, hipStream_t s);

// CRT: `fast` selects the Lagrange form (every job must have its tables).
// A tile covers crt_entries(fast, W, L) x 128 columns of one row; the same
// count goes to launch_crt.
int crt_entries(bool fast, int W, int L);
int64_t crt_tiles(int64_t rows, int64_t cols, int entries);
int64_t crt_col_tiles(int64_t cols, int entries);
void launch_crt(bool fast, int W, int E, const CrtJob &job0, const CrtJob *jobs, int njobs,
                int64_t total_tiles, const PrimeConst *pc, const double *garner, hipStream_t s);
// Whether a promise |x| <= B (words) lets the Lagrange form be exact for the
// primes range, and fits W output words.
bool crt_fast_ok(const rns_ctx *ctx, int begin, int L, const uint64_t *bound_words, int Wb, int W);

}  // namespace rns
