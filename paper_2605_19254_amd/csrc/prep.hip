// Operand preparation for the residue products: uint32 residues in [0, p) ->
// the tiled layouts the GEMM kernels read (balanced digits for the INT8 path,
// balanced doubles for the FP64 path).
//
// One wave converts one 16 x 64 operand tile ("operand rows" are the rows of A
// or the columns of B; k is the contraction index).
//   INT8 tile: 4 digit blocks of 64 lanes x 16 bytes; lane l holds operand row
//              l%16 and k = 16*(l/16) .. 16*(l/16)+15 of the tile.  The
//              balanced residue b is split as b = d0 + d1 2^8 + d2 2^16 + d3 2^24
//              with d0..d2 the sign-extended low bytes of the successive
//              quotients (each subtraction leaves a multiple of 256).
//   FP64 tile: 16 fragments of 64 doubles; fragment f covers k = 4f .. 4f+3,
//              lane l holds operand row l%16 and k = 4f + l/16.
// Tiles that lie inside the matrix are read without per-element bounds
// checks (row-major A with 16-byte vector loads when aligned); edge tiles
// read zeros outside the matrix, which contribute nothing to the products.
#include "gemm_common.hpp"

namespace rns {
namespace gemm {
namespace {

typedef unsigned v4u __attribute__((ext_vector_type(4)));

struct Digits {
    uint32_t d[4];
};

__device__ __forceinline__ void split_pack(int32_t v, int byte, Digits &o) {
    const int32_t d0 = (int32_t)(int8_t)(v & 0xFF);
    v = (v - d0) >> 8;
    const int32_t d1 = (int32_t)(int8_t)(v & 0xFF);
    v = (v - d1) >> 8;
    const int32_t d2 = (int32_t)(int8_t)(v & 0xFF);
    const int32_t d3 = (v - d2) >> 8;
    o.d[0] |= ((uint32_t)d0 & 0xFF) << (8 * byte);
    o.d[1] |= ((uint32_t)d1 & 0xFF) << (8 * byte);
    o.d[2] |= ((uint32_t)d2 & 0xFF) << (8 * byte);
    o.d[3] |= ((uint32_t)d3 & 0xFF) << (8 * byte);
}

template <bool kInt8>
__device__ __forceinline__ void prep_unit(const GemmProblem &g, int64_t unit, int lane,
                                          const PrimeConst *__restrict__ pc) {
    const bool isB = unit >= g.unitB_begin;
    int64_t u = unit - (isB ? g.unitB_begin : g.unitA_begin);
    const int32_t nblk = isB ? g.CB : g.RB;
    const int64_t per_plane = (int64_t)nblk * g.KT;
    const int plane = (int)(u / per_plane);
    u -= (int64_t)plane * per_plane;
    const int blk = (int)(u / g.KT);
    const int kt = (int)(u - (int64_t)blk * g.KT);
    const uint32_t p = pc[g.prime_begin + plane].p;
    const uint32_t half = (p - 1) / 2;
    const int row = blk * 16 + (lane & 15);
    const int rows_valid = isB ? g.n : g.m;
    const auto src = gptr(isB ? g.B + (int64_t)plane * g.bps : g.A + (int64_t)plane * g.aps);
    const int64_t ld = isB ? g.ldb : g.lda;
    const bool interior = (blk + 1) * 16 <= rows_valid && (kt + 1) * 64 <= g.k;
    auto bal = [&](uint32_t r) -> int32_t { return r > half ? (int32_t)r - (int32_t)p : (int32_t)r; };
    auto fetch = [&](int kk) -> int32_t {
        if (row >= rows_valid || kk >= g.k) return 0;
        return bal(isB ? src[(int64_t)kk * ld + row] : src[(int64_t)row * ld + kk]);
    };
    const auto dst = gptr_w(isB ? g.Bt + (int64_t)plane * g.b_plane_bytes : g.At + (int64_t)plane * g.a_plane_bytes);
    if constexpr (kInt8) {
        const int k0 = kt * 64 + (lane >> 4) * 16;
        int32_t v[16];
        if (interior) {
            if (!isB && (ld & 3) == 0 && ((uintptr_t)(isB ? g.B : g.A) & 15) == 0 && ((plane * (isB ? g.bps : g.aps)) & 3) == 0) {
                const auto s4 = reinterpret_cast<const __attribute__((address_space(1))) v4u *>(src + (int64_t)row * ld + k0);
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    const v4u x = s4[w];
                    v[4 * w + 0] = bal(x[0]);
                    v[4 * w + 1] = bal(x[1]);
                    v[4 * w + 2] = bal(x[2]);
                    v[4 * w + 3] = bal(x[3]);
                }
            } else if (!isB) {
                const auto s1 = src + (int64_t)row * ld + k0;
#pragma unroll
                for (int t = 0; t < 16; ++t) v[t] = bal(s1[t]);
            } else {
                const auto s1 = src + (int64_t)k0 * ld + row;
#pragma unroll
                for (int t = 0; t < 16; ++t) v[t] = bal(s1[(int64_t)t * ld]);
            }
        } else {
#pragma unroll
            for (int t = 0; t < 16; ++t) v[t] = fetch(k0 + t);
        }
        Digits dg[4];
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            dg[w].d[0] = dg[w].d[1] = dg[w].d[2] = dg[w].d[3] = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) split_pack(v[4 * w + b], b, dg[w]);
        }
        const auto out = reinterpret_cast<__attribute__((address_space(1))) v4i *>(dst) + ((int64_t)blk * g.KT + kt) * 256;
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            v4i t = {(int)dg[0].d[d], (int)dg[1].d[d], (int)dg[2].d[d], (int)dg[3].d[d]};
            out[d * 64 + lane] = t;
        }
    } else {
        const auto out = reinterpret_cast<__attribute__((address_space(1))) double *>(dst) + ((int64_t)blk * g.KT + kt) * 1024;
        const int kl = kt * 64 + (lane >> 4);
        if (interior) {
            double vals[16];
#pragma unroll
            for (int f = 0; f < 16; ++f) {
                const int kk = kl + 4 * f;
                vals[f] = (double)bal(isB ? src[(int64_t)kk * ld + row] : src[(int64_t)row * ld + kk]);
            }
#pragma unroll
            for (int f = 0; f < 16; ++f) out[f * 64 + lane] = vals[f];
        } else {
#pragma unroll
            for (int f = 0; f < 16; ++f) out[f * 64 + lane] = (double)fetch(kl + 4 * f);
        }
    }
}

// With several problems each wave converts kUnitsPerWave consecutive tiles; the
// problem of the first is found by binary search and later ones advance
// linearly.  A single problem uses one tile per wave.
constexpr int kUnitsPerWave = 4;

template <bool kInt8>
__global__ __launch_bounds__(256) void k_prep(const GemmProblem *__restrict__ P, int nprob,
                                              int64_t total_units,
                                              const PrimeConst *__restrict__ pc,
                                              unsigned *__restrict__ counter, int per_wave) {
    // Reset the work counter of a persistent GEMM launched after this kernel.
    if (counter && blockIdx.x == 0 && threadIdx.x == 0) *counter = 0u;
    const int lane = threadIdx.x & 63;
    // The wave index is uniform within a wave; saying so keeps the problem
    // table reads scalar.
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t u0 = ((int64_t)blockIdx.x * 4 + wave) * per_wave;
    if (u0 >= total_units) return;
    int q = find_problem(P, nprob, u0, &GemmProblem::unitA_begin);
    for (int r = 0; r < per_wave; ++r) {
        const int64_t unit = u0 + r;
        if (unit >= total_units) break;
        while (q + 1 < nprob && P[q + 1].unitA_begin <= unit) ++q;
        prep_unit<kInt8>(P[q], unit, lane, pc);
    }
}

}  // namespace

void launch_prep(bool int8, const GemmProblem *P, int nprob, int64_t units,
                 const PrimeConst *pc, unsigned *counter, hipStream_t s) {
    const int per_wave = nprob > 1 ? kUnitsPerWave : 1;
    const unsigned blocks = (unsigned)((units + 4 * per_wave - 1) / (4 * per_wave));
    if (int8)
        hipLaunchKernelGGL(k_prep<true>, dim3(blocks), dim3(256), 0, s, P, nprob, units, pc, counter, per_wave);
    else
        hipLaunchKernelGGL(k_prep<false>, dim3(blocks), dim3(256), 0, s, P, nprob, units, pc, counter, per_wave);
}

}  // namespace gemm
}  // namespace rns
