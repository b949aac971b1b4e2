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

typedef long long v2ll __attribute__((ext_vector_type(2)));
typedef unsigned v4u __attribute__((ext_vector_type(4)));

constexpr int kTile = 256;                // threads per block
constexpr int kPer = 4;                   // consecutive entries per thread
constexpr int kTileCols = kTile * kPer;   // columns of one tile

// With a job table, each block takes runs of `chunk` consecutive tiles (tile =
// up to 1024 entries of one row of one job), job by job (for_job_tiles).  A
// single job uses runs of one tile.  Each thread reduces 4 consecutive entries,
// with 16-byte loads and stores when the job's layout allows; control flow is
// uniform except at the end of a row, so the prime constants come through
// scalar loads.
constexpr int kChunk = 8;

struct RedConst {
    double pf, pinv, c21, c42;
};

__device__ __forceinline__ uint32_t reduce_one(double a2, double a1, double a0, const RedConst &P) {
    const double s = fma(a2, P.c42, fma(a1, P.c21, a0));
    const double q2 = rint(s * P.pinv);
    double r = fma(-q2, P.pf, s);
    r = r < 0.0 ? r + P.pf : r;
    return (uint32_t)r;
}

__global__ __launch_bounds__(kTile) void k_reduce(ReduceJob job0, const ReduceJob *__restrict__ jobs,
                                                  int njobs, int64_t total_tiles,
                                                  const PrimeConst *__restrict__ pc_all, int chunk) {
    const int64_t nchunks = (total_tiles + chunk - 1) / chunk;
    for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const int64_t t0 = ch * chunk;
        const int64_t t1 = t0 + chunk < total_tiles ? t0 + chunk : total_tiles;
        for_job_tiles(job0, jobs, njobs, total_tiles, t0, t1, [&](const ReduceJob &J, int64_t t) {
            const int64_t u = t - J.tile_begin;
            const int64_t i = u / J.col_tiles;
            const int64_t c0 = (u - i * J.col_tiles) * kTileCols + kPer * threadIdx.x;
            const bool vec = J.vec && c0 + kPer <= J.cols;
            const auto src = gptr(J.x + i * J.ldx + c0);
            int64_t v[kPer];
            if (vec) {
                const auto s2 = reinterpret_cast<const __attribute__((address_space(1))) v2ll *>(src);
                const v2ll x01 = s2[0], x23 = s2[1];
                v[0] = x01.x; v[1] = x01.y; v[2] = x23.x; v[3] = x23.y;
            } else {
#pragma unroll
                for (int e = 0; e < kPer; ++e) v[e] = c0 + e < J.cols ? src[e] : 0;
            }
            double a0[kPer], a1[kPer], a2[kPer];
#pragma unroll
            for (int e = 0; e < kPer; ++e) {
                a0[e] = (double)(int32_t)(v[e] & 0x1FFFFF);
                a1[e] = (double)(int32_t)((v[e] >> 21) & 0x1FFFFF);
                a2[e] = (double)(int32_t)(v[e] >> 42);
            }
            const auto dst = gptr_w(J.res + i * J.ldr + c0);
            const auto pc = cptr(pc_all + J.prime_begin);
            for (int j = 0; j < J.L; ++j) {
                const RedConst P{pc[j].pf, pc[j].pinv, pc[j].c21, pc[j].c42};
                uint32_t r[kPer];
#pragma unroll
                for (int e = 0; e < kPer; ++e) r[e] = reduce_one(a2[e], a1[e], a0[e], P);
                const auto d = dst + (int64_t)j * J.ps;
                if (vec) {
                    *reinterpret_cast<__attribute__((address_space(1))) v4u *>(d) = v4u{r[0], r[1], r[2], r[3]};
                } else {
#pragma unroll
                    for (int e = 0; e < kPer; ++e)
                        if (c0 + e < J.cols) d[e] = r[e];
                }
            }
        });
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
    // 4-entry vectors from a column that is a multiple of 4: 16-byte aligned
    // when the bases are and the strides are even (x) or multiples of 4 (res).
    j.vec = ((uintptr_t)x % 16 == 0) && ldx % 2 == 0 && ((uintptr_t)res % 16 == 0) && ldr % 4 == 0 &&
            (L <= 1 || plane_stride % 4 == 0);
    j.col_tiles = (cols + kTileCols - 1) / kTileCols;
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

extern "C" int rns_reduce_mw(rns_ctx *ctx, const uint64_t *x, int W, int64_t rows, int64_t cols,
                             int64_t ldx, int prime_begin, int L, uint32_t *res, int64_t ldr,
                             int64_t plane_stride, void *stream) {
    if (W < 1 || W > kCrtMaxW) return RNS_EINVAL;
    int st = reduce_check(ctx, reinterpret_cast<const int64_t *>(x), rows, cols, ldx, prime_begin, L, res, ldr,
                          plane_stride);
    if (st != RNS_OK) return st;
    if (rows == 0 || cols == 0 || L == 0) return RNS_OK;
    if (rows > INT64_MAX / cols) return RNS_EINVAL;
    std::lock_guard<std::mutex> guard(ctx->mu);
    RNS_HIP(hipSetDevice(ctx->device));
    // Balanced base-256 digits of x times the table of 2^(8k) mod p_j on the
    // matrix cores (digits_gemm.hip).
    return reduce_mw_mfma(ctx, x, W, rows, cols, ldx, prime_begin, L, res, ldr, plane_stride,
                          (hipStream_t)stream);
}
