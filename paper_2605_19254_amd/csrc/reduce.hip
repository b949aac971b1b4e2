// rns_reduce: int64 matrix -> L residue planes (Section 3.1, reduction of an
// integer matrix modulo each prime; the reduction uses a floating-point
// reciprocal instead of an integer division, as in the bullet on fast modular
// reduction).
//
// x is split once into three limbs x = a2*2^42 + a1*2^21 + a0 with
// a0, a1 in [0, 2^21) and a2 in [-2^21, 2^21).  For each prime,
//   s = a2*(2^42 mod p) + a1*(2^21 mod p) + a0,   |s| < 2^48,
// is formed exactly in double arithmetic, q = rint(s/p) is taken from the
// rounded reciprocal (the quotient error is far below 1/2 at these sizes, so q
// is the nearest integer or its neighbour), and r = s - q*p is exact with
// |r| < p; a negative r is moved up by p.  HBM-bound: 8 bytes in per entry,
// 4*L bytes out.
#include "internal.hpp"

using namespace rns;

namespace {

constexpr int kTile = 256;

__global__ __launch_bounds__(kTile) void k_reduce(
    const int64_t *__restrict__ x, int64_t rows, int64_t cols, int64_t ldx,
    const PrimeConst *__restrict__ pc, int L, uint32_t *__restrict__ res,
    int64_t ldr, int64_t plane_stride, int64_t col_tiles) {
    const int64_t ntiles = rows * col_tiles;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t i = t / col_tiles;
        const int64_t c = (t - i * col_tiles) * kTile + threadIdx.x;
        if (c >= cols) continue;
        const int64_t v = x[i * ldx + c];
        const double a0 = (double)(int32_t)(v & 0x1FFFFF);
        const double a1 = (double)(int32_t)((v >> 21) & 0x1FFFFF);
        const double a2 = (double)(int32_t)(v >> 42);
        uint32_t *dst = res + i * ldr + c;
        for (int j = 0; j < L; ++j) {
            const PrimeConst &P = pc[j];
            const double s = fma(a2, P.c42, fma(a1, P.c21, a0));
            const double q = rint(s * P.pinv);
            double r = fma(-q, P.pf, s);
            r = r < 0.0 ? r + P.pf : r;
            dst[(int64_t)j * plane_stride] = (uint32_t)r;
        }
    }
}

}  // namespace

extern "C" int rns_reduce(rns_ctx *ctx, const int64_t *x, int64_t rows, int64_t cols,
                          int64_t ldx, int prime_begin, int L, uint32_t *res,
                          int64_t ldr, int64_t plane_stride, void *stream) {
    if (!ctx || rows < 0 || cols < 0 || L < 0) return RNS_EINVAL;
    if (prime_begin < 0 || prime_begin + L > ctx->L) return RNS_EINVAL;
    if (rows == 0 || cols == 0 || L == 0) return RNS_OK;
    if (!x || !res || ldx < cols || ldr < cols) return RNS_EINVAL;
    if (L > 1 && plane_stride < (rows - 1) * ldr + cols) return RNS_EINVAL;
    RNS_HIP(hipSetDevice(ctx->device));
    const int64_t col_tiles = (cols + kTile - 1) / kTile;
    const int64_t ntiles = rows * col_tiles;
    const int64_t grid = ntiles < (1 << 20) ? ntiles : (1 << 20);
    ProfScope ps(ctx, "k_reduce", (hipStream_t)stream);
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)grid), dim3(kTile), 0, (hipStream_t)stream,
                       x, rows, cols, ldx, ctx->d_prime + prime_begin, L, res, ldr,
                       plane_stride, col_tiles);
    RNS_HIP(hipGetLastError());
    return RNS_OK;
}
