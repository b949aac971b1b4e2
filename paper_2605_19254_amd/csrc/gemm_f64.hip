// FP64-MFMA residue product (Section 3.1: one exact product per prime; the
// paper computes it with an FP64 GEMM whose every partial sum stays below
// 2^53).
//
// Residues are moved to the balanced range |r| <= (p-1)/2 and held as
// doubles.  v_mfma_f64_16x16x4f64 adds 4 products per step; after every 8
// products the accumulator is reduced mod p with the rounded reciprocal
// (q = rint(acc/p), acc -= q*p, exact).  With p < 2^26,
//   8*((p-1)/2)^2 + (p+1)/2 < 2^53,
// so every partial sum is an integer below 2^53 and the result does not depend
// on the order of summation.  The paper bounds the whole dot product instead
// (n(p-1)^2 + (p-1) < 2^53); blocking by 8 lets 26-bit primes be used at any k.
//
// Work-group tile 128 x 128: four waves in 2 x 2, each 64 x 64.  Two
// work-groups per CU (the launch bound), so that the compiler keeps the 64
// accumulators per lane in ordinary VGPRs (220 registers in all) and one
// wave's reduction overlaps the other wave's MFMAs; with one work-group per
// CU the accumulators went to the accumulation registers (AGPRs), where
// FP64 MFMAs ran at half rate on MI355X.
#include "gemm_common.hpp"

namespace rns {
namespace gemm {
namespace {

// ------------------------------------------------------------- FP64 GEMM --

__global__ __launch_bounds__(256, 2) void k_gemm_f64(const GemmProblem *__restrict__ P, int nprob,
                                                  int64_t total_tiles,
                                                  const PrimeConst *__restrict__ pc,
        const int32_t *__restrict__ tile_prob) {
    const int64_t t = xcd_window_remap(blockIdx.x, gridDim.x, kXcdWindow2);
    if (t >= total_tiles) return;
    const TileCoord tc = map_tile(P, nprob, t, tile_prob);
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
                if (row < g.m && col < g.n) store_residue(C + (int64_t)row * g.ldc + col, (uint32_t)r, pr.p, g.sub);
            }
}

}  // namespace

void launch_gemm_f64(const GemmProblem *P, int nprob, int64_t tiles, const PrimeConst *pc,
                     const int32_t *tile_prob, hipStream_t s) {
    hipLaunchKernelGGL(k_gemm_f64, dim3((unsigned)tiles), dim3(256), 0, s, P, nprob, tiles, pc, tile_prob);
}

}  // namespace gemm
}  // namespace rns
