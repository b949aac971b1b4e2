// rns_reduce: int64 matrix -> L residue planes (Section 3.1, reduction of an
// integer matrix modulo each prime; the reduction uses a floating-point
// reciprocal instead of an integer division, as in the bullet on fast modular
// reduction).
//
// x is split once into three limbs x = a2*2^42 + a1*2^21 + a0 with
// a0, a1 in [0, 2^21) and a2 in [-2^21, 2^21).  For each prime,
//   s = a2*(2^42 mod p) + a1*(2^21 mod p) + a0,   |s| < 2^48,
// is formed exactly in double arithmetic, q = rint(s/p) comes from the rounded
// reciprocal (s/p is never within 2^-27 of a half-integer because p is odd, and
// the quotient error is below 2^-29, so q is the nearest integer), and
// r = s - q*p is exact with |r| <= (p-1)/2; a negative r is moved up by p.
// HBM-bound: 8 bytes in per entry, 4*L bytes out.
//
// The same kernel serves one matrix (job passed by value) or a table of jobs
// in device memory (all matrices of a batched plan in one launch).
#include "reduce_crt.hpp"

using namespace rns;

namespace {

constexpr int kTile = 256;

// With a job table, each block takes runs of `chunk` consecutive tiles (tile =
// up to 256 entries of one row of one job); the job of the first tile is found
// by binary search and later tiles advance the job index linearly.  A single
// job uses runs of one tile.
constexpr int kChunk = 8;

__global__ __launch_bounds__(kTile) void k_reduce(ReduceJob job0, const ReduceJob *__restrict__ jobs,
                                                  int njobs, int64_t total_tiles,
                                                  const PrimeConst *__restrict__ pc_all, int chunk) {
    const int64_t nchunks = (total_tiles + chunk - 1) / chunk;
    for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const int64_t t0 = ch * chunk;
        const int64_t t1 = t0 + chunk < total_tiles ? t0 + chunk : total_tiles;
        int q = 0;
        if (njobs > 0) {
            int lo = 0, hi = njobs - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (jobs[mid].tile_begin <= t0) lo = mid; else hi = mid - 1;
            }
            q = lo;
        }
        for (int64_t t = t0; t < t1; ++t) {
            if (njobs > 0)
                while (q + 1 < njobs && jobs[q + 1].tile_begin <= t) ++q;
            q = __builtin_amdgcn_readfirstlane(q);   // uniform: scalar loads of the job
            const ReduceJob J = njobs > 0 ? jobs[q] : job0;
            const int64_t u = t - J.tile_begin;
            const int64_t i = u / J.col_tiles;
            const int64_t c = (u - i * J.col_tiles) * kTile + threadIdx.x;
            if (c >= J.cols) continue;
            const int64_t v = *gptr(J.x + i * J.ldx + c);
            const double a0 = (double)(int32_t)(v & 0x1FFFFF);
            const double a1 = (double)(int32_t)((v >> 21) & 0x1FFFFF);
            const double a2 = (double)(int32_t)(v >> 42);
            const auto dst = gptr_w(J.res + i * J.ldr + c);
            const auto pc = gptr(pc_all + J.prime_begin);
            for (int j = 0; j < J.L; ++j) {
                const auto &P = pc[j];
                const double s = fma(a2, P.c42, fma(a1, P.c21, a0));
                const double q2 = rint(s * P.pinv);
                double r = fma(-q2, P.pf, s);
                r = r < 0.0 ? r + P.pf : r;
                dst[(int64_t)j * J.ps] = (uint32_t)r;
            }
        }
    }
}

}  // namespace

namespace rns {

int reduce_check(const rns_ctx *ctx, const int64_t *x, int64_t rows, int64_t cols, int64_t ldx,
                 int prime_begin, int L, const uint32_t *res, int64_t ldr, int64_t plane_stride) {
    if (!ctx || rows < 0 || cols < 0 || L < 0) return RNS_EINVAL;
    if (prime_begin < 0 || prime_begin + L > ctx->L) return RNS_EINVAL;
    if (rows == 0 || cols == 0 || L == 0) return RNS_OK;
    if (!x || !res || ldx < cols || ldr < cols) return RNS_EINVAL;
    if (L > 1 && plane_stride < (rows - 1) * ldr + cols) return RNS_EINVAL;
    return RNS_OK;
}

ReduceJob make_reduce_job(const int64_t *x, int64_t rows, int64_t cols, int64_t ldx,
                          int prime_begin, int L, uint32_t *res, int64_t ldr,
                          int64_t plane_stride, int64_t tile_begin) {
    ReduceJob j;
    j.x = x; j.rows = rows; j.cols = cols; j.ldx = ldx;
    j.res = res; j.ldr = ldr; j.ps = plane_stride;
    j.prime_begin = prime_begin; j.L = L;
    j.col_tiles = (cols + kTile - 1) / kTile;
    j.tile_begin = tile_begin;
    return j;
}

int64_t reduce_tiles(const ReduceJob &j) { return j.rows * j.col_tiles; }

void launch_reduce(const ReduceJob &job0, const ReduceJob *jobs, int njobs, int64_t total_tiles,
                   const PrimeConst *pc, hipStream_t s) {
    const int chunk = njobs > 1 ? kChunk : 1;
    const int64_t nchunks = (total_tiles + chunk - 1) / chunk;
    const int64_t grid = nchunks < (1 << 20) ? nchunks : (1 << 20);
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)grid), dim3(kTile), 0, s, job0, jobs, njobs,
                       total_tiles, pc, chunk);
}

}  // namespace rns

extern "C" int rns_reduce(rns_ctx *ctx, const int64_t *x, int64_t rows, int64_t cols,
                          int64_t ldx, int prime_begin, int L, uint32_t *res,
                          int64_t ldr, int64_t plane_stride, void *stream) {
    int st = reduce_check(ctx, x, rows, cols, ldx, prime_begin, L, res, ldr, plane_stride);
    if (st != RNS_OK) return st;
    if (rows == 0 || cols == 0 || L == 0) return RNS_OK;
    RNS_HIP(hipSetDevice(ctx->device));
    ReduceJob j = make_reduce_job(x, rows, cols, ldx, prime_begin, L, res, ldr, plane_stride, 0);
    ProfScope ps(ctx, "k_reduce", (hipStream_t)stream);
    launch_reduce(j, nullptr, 0, reduce_tiles(j), ctx->d_prime, (hipStream_t)stream);
    RNS_HIP(hipGetLastError());
    return RNS_OK;
}
