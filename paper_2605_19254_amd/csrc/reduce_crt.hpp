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

// Tiles [t0, t1) of a launch, job by job: body(J, t) for every tile t, with J
// the job that holds t (job0 when there is no table).  The job index is the
// same on every lane, so the job's fields come through scalar loads, once per
// job that the range touches.
template <class Job, class Body>
__device__ __forceinline__ void for_job_tiles(const Job &job0, const Job *__restrict__ jobs, int njobs,
                                              int64_t total_tiles, int64_t t0, int64_t t1, Body &&body) {
    if (njobs <= 0) {
        for (int64_t t = t0; t < t1; ++t) body(job0, t);
        return;
    }
    int lo = 0, hi = njobs - 1;                     // last job starting at or before t0
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].tile_begin <= t0) lo = mid; else hi = mid - 1;
    }
    int q = lo;
    int64_t t = t0;
    while (t < t1 && q < njobs) {
        q = __builtin_amdgcn_readfirstlane(q);
        const Job J = jobs[q];
        const int64_t end = q + 1 < njobs ? jobs[q + 1].tile_begin : total_tiles;
        const int64_t te = end < t1 ? end : t1;
        for (; t < te; ++t) body(J, t);
        ++q;
    }
}

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

// The matrix-core forms (digits x constant table, digits_gemm.hip); the
// caller holds ctx->mu and has validated the arguments.
int crt_mfma(rns_ctx *ctx, const uint32_t *res, int64_t rows, int64_t cols, int64_t ldr, int64_t ps,
             int begin, int L, uint64_t *out, int W, int64_t ldo, int32_t *status, hipStream_t s);
int reduce_mw_mfma(rns_ctx *ctx, const uint64_t *x, int W, int64_t rows, int64_t cols, int64_t ldx, int begin,
                   int L, uint32_t *res, int64_t ldr, int64_t ps, hipStream_t s);

}  // namespace rns
