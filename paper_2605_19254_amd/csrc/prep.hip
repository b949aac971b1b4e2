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
typedef long long v2ll __attribute__((ext_vector_type(2)));

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
    // Fewer than 2^31 units per problem (the host checks): 32-bit indexing.
    uint32_t u = (uint32_t)(unit - (isB ? g.unitB_begin : g.unitA_begin));
    const uint32_t nblk = (uint32_t)(isB ? g.CB : g.RB);
    const uint32_t per_plane = nblk * (uint32_t)g.KT;
    const int plane = (int)(u / per_plane);
    u -= (uint32_t)plane * per_plane;
    const int blk = (int)(u / (uint32_t)g.KT);
    const int kt = (int)(u - (uint32_t)blk * (uint32_t)g.KT);
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

// int64 operands straight to the tiled layouts: one wave reads one 16 x 64
// tile of A or B once and writes it for every prime of the problem.  Each
// entry x is split into x = a2 2^42 + a1 2^21 + a0 (a0, a1 in [0, 2^21)); per
// prime, s = a2 (2^42 mod p) + a1 (2^21 mod p) + a0 is exact in doubles
// (|s| < 2^48) and r = s - rint(s/p) p, with the rounded reciprocal, is the
// balanced residue (|r| <= (p-1)/2: s/p is never within 2^-27 of a
// half-integer because p is odd, and the quotient's error is below 2^-29).
template <bool kInt8>
__device__ __forceinline__ void prep_unit_i64(const GemmProblem &g, int64_t unit, int lane,
                                              const PrimeConst *__restrict__ pc_all) {
    const bool isB = unit >= g.u64B_begin;
    const uint32_t u = (uint32_t)(unit - (isB ? g.u64B_begin : g.u64A_begin));
    const int blk = (int)(u / (uint32_t)g.KT);
    const int kt = (int)(u - (uint32_t)blk * (uint32_t)g.KT);
    const int row = blk * 16 + (lane & 15);
    const int rows_valid = isB ? g.n : g.m;
    const int64_t *base = isB ? g.B64 : g.A64;
    const auto src = gptr(base);
    const int64_t ld = isB ? g.ldb64 : g.lda64;
    const bool interior = (blk + 1) * 16 <= rows_valid && (kt + 1) * 64 <= g.k;
    // k of value t: INT8 16 consecutive k per lane; FP64 k = 4t + lane/16.
    const int kb = kt * 64 + (kInt8 ? (lane >> 4) * 16 : (lane >> 4));
    const int kstep = kInt8 ? 1 : 4;
    int64_t x[16];
    if (interior) {
        if (!isB && kInt8 && (ld & 1) == 0 && ((uintptr_t)base & 15) == 0) {
            const auto s2 = reinterpret_cast<const __attribute__((address_space(1))) v2ll *>(src + (int64_t)row * ld + kb);
#pragma unroll
            for (int w = 0; w < 8; ++w) {
                const v2ll y = s2[w];
                x[2 * w] = y.x;
                x[2 * w + 1] = y.y;
            }
        } else if (!isB) {
#pragma unroll
            for (int t = 0; t < 16; ++t) x[t] = src[(int64_t)row * ld + kb + kstep * t];
        } else {
#pragma unroll
            for (int t = 0; t < 16; ++t) x[t] = src[(int64_t)(kb + kstep * t) * ld + row];
        }
    } else {
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const int kk = kb + kstep * t;
            x[t] = (row < rows_valid && kk < g.k)
                       ? (isB ? src[(int64_t)kk * ld + row] : src[(int64_t)row * ld + kk]) : 0;
        }
    }
    double a0[16], a1[16], a2[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        a0[t] = (double)(int32_t)(x[t] & 0x1FFFFF);
        a1[t] = (double)(int32_t)((x[t] >> 21) & 0x1FFFFF);
        a2[t] = (double)(int32_t)(x[t] >> 42);
    }
    char *dst0 = isB ? g.Bt : g.At;
    const int64_t plane_bytes = isB ? g.b_plane_bytes : g.a_plane_bytes;
    const auto pc = cptr(pc_all + g.prime_begin);
    for (int plane = 0; plane < g.L; ++plane) {
        const double pf = pc[plane].pf, pinv = pc[plane].pinv, c21 = pc[plane].c21, c42 = pc[plane].c42;
        double r[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const double sv = fma(a2[t], c42, fma(a1[t], c21, a0[t]));
            r[t] = fma(-rint(sv * pinv), pf, sv);
        }
        const auto dst = gptr_w(dst0 + (int64_t)plane * plane_bytes);
        if constexpr (kInt8) {
            Digits dg[4];
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                dg[w].d[0] = dg[w].d[1] = dg[w].d[2] = dg[w].d[3] = 0;
#pragma unroll
                for (int b = 0; b < 4; ++b) split_pack((int32_t)r[4 * w + b], b, dg[w]);
            }
            const auto out = reinterpret_cast<__attribute__((address_space(1))) v4i *>(dst) + ((int64_t)blk * g.KT + kt) * 256;
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                v4i t = {(int)dg[0].d[d], (int)dg[1].d[d], (int)dg[2].d[d], (int)dg[3].d[d]};
                out[d * 64 + lane] = t;
            }
        } else {
            const auto out = reinterpret_cast<__attribute__((address_space(1))) double *>(dst) + ((int64_t)blk * g.KT + kt) * 1024;
#pragma unroll
            for (int f = 0; f < 16; ++f) out[f * 64 + lane] = r[f];
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

template <bool kInt8>
__global__ __launch_bounds__(256) void k_prep_i64(const GemmProblem *__restrict__ P, int nprob,
                                                  int64_t total_units,
                                                  const PrimeConst *__restrict__ pc,
                                                  unsigned *__restrict__ counter, int per_wave) {
    if (counter && blockIdx.x == 0 && threadIdx.x == 0) *counter = 0u;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t u0 = ((int64_t)blockIdx.x * 4 + wave) * per_wave;
    if (u0 >= total_units) return;
    int q = find_problem(P, nprob, u0, &GemmProblem::u64A_begin);
    for (int r = 0; r < per_wave; ++r) {
        const int64_t unit = u0 + r;
        if (unit >= total_units) break;
        while (q + 1 < nprob && P[q + 1].u64A_begin <= unit) ++q;
        q = __builtin_amdgcn_readfirstlane(q);
        prep_unit_i64<kInt8>(P[q], unit, lane, pc);
    }
}

}  // namespace

void launch_prep_i64(bool int8, const GemmProblem *P, int nprob, int64_t units,
                     const PrimeConst *pc, unsigned *counter, hipStream_t s) {
    const int per_wave = nprob > 1 ? kUnitsPerWave : 1;
    const unsigned blocks = (unsigned)((units + 4 * per_wave - 1) / (4 * per_wave));
    if (int8)
        hipLaunchKernelGGL(k_prep_i64<true>, dim3(blocks), dim3(256), 0, s, P, nprob, units, pc, counter, per_wave);
    else
        hipLaunchKernelGGL(k_prep_i64<false>, dim3(blocks), dim3(256), 0, s, P, nprob, units, pc, counter,
                           per_wave);
}

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
