// INT8-limb residue product (Section 3.1: one exact product per prime).
//
// Each balanced residue r (|r| <= (p-1)/2) is split into four signed base-256
// digits r = d0 + d1*2^8 + d2*2^16 + d3*2^24, d0..d2 in [-128, 127],
// |d3| <= 2 (the prep kernel does the split).  The 16 digit-pair products are
// computed with v_mfma_i32_16x16x64_i8 and summed in int32 per shift group
// s = i+j (7 groups).  The largest group sum per term is 3*2^14, so the int32
// sums are exact for k <= 43690.  The epilogue (recombine) forms
// C = sum_s C_s 2^(8s) mod p in exact doubles with one intermediate
// reduction.
//
// Every variant covers the same 64 x 128 output tiles (the host's tiling):
//   direct   four waves in 2 x 2, each 32 x 64 outputs, operands straight from
//            L2 into registers;
//   lds      the same waves, operands staged through LDS;
//   wave8    eight waves in 2 x 4, each 32 x 32 outputs, two waves per SIMD;
//   half     two independent work-groups per tile (one per 64-column half),
//            four waves of 32 x 32 each, two work-groups per CU;
//   half, persistent  the half kernel taking half-tiles from a work counter.
// Measured on MI355X: the two-waves-per-SIMD forms are faster than the
// one-wave forms (whose 224 accumulators also sit in AGPRs, where 16x16x64
// INT8 MFMAs run about a fifth slower than with VGPR accumulators); the half
// form, whose work-groups do not share a barrier, is the default.  Every form
// places its work-groups with xcd_window_remap.
#include "gemm_common.hpp"

#include <algorithm>

namespace rns {
namespace gemm {
namespace {

// Epilogue of one output: (sum_s C_s 2^(8s)) mod p in [0, p), every step an
// exact double operation.  With |C_s| < 2^31:
//   lo  = C_0 + 2^8 C_1 + 2^16 C_2 and mid = C_3 + 2^8 C_4 + 2^16 C_5 are
//         below 2^48 (exact);
//   rm  = mid mod p, balanced (quotient below 2^22, so the rounded
//         reciprocal gives it exactly);
//   C_6 = sum of e3 f3 with |e3|, |f3| <= 2 is below 4k < 2^18;
//   s   = lo + rm (2^24 mod p) + C_6 (2^48 mod p), the weights balanced:
//         |s| < 2^48 + 2^50 + 2^43 < 2^53 (exact);
//   r   = s - rint(s/p) p: the quotient can be off by one only when s mod p
//         lies next to +-p/2, and then r lands in (-p, 0) or (0, p) so that
//         adding p to a negative r still gives s mod p in [0, p).
__device__ __forceinline__ uint32_t recombine(int c0, int c1, int c2, int c3, int c4, int c5, int c6,
                                              const PrimeConst &pr) {
    const double lo = fma((double)c2, 65536.0, fma((double)c1, 256.0, (double)c0));
    const double mid = fma((double)c5, 65536.0, fma((double)c4, 256.0, (double)c3));
    const double rm = fma(-rint(mid * pr.pinv), pr.pf, mid);
    const double sum = fma((double)c6, pr.w[6], fma(rm, pr.w[3], lo));
    double r = fma(-rint(sum * pr.pinv), pr.pf, sum);
    r = r < 0.0 ? r + pr.pf : r;
    return (uint32_t)r;
}

// ------------------------------------------------------------- INT8 GEMM --

__global__ __launch_bounds__(256) void k_gemm_i8(const GemmProblem *__restrict__ P, int nprob,
                                                 int64_t total_tiles,
                                                 const PrimeConst *__restrict__ pc,
        const int32_t *__restrict__ tile_prob) {
    const int64_t t = xcd_window_remap(blockIdx.x, gridDim.x, kXcdWindow1);
    if (t >= total_tiles) return;
    const TileCoord tc = map_tile(P, nprob, t, tile_prob);
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

    const PrimeConst pr = pc[g.prime_begin + tc.plane];
    uint32_t *C = g.C + (int64_t)tc.plane * g.cps;
#pragma unroll
    for (int i = 0; i < kI8WaveRB; ++i)
#pragma unroll
        for (int j = 0; j < kI8WaveCB; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const uint32_t r = recombine(acc[0][i][j][v], acc[1][i][j][v], acc[2][i][j][v], acc[3][i][j][v],
                                             acc[4][i][j][v], acc[5][i][j][v], acc[6][i][j][v], pr);
                const int row = (rb0 + i) * 16 + 4 * (lane >> 4) + v;
                const int col = (cb0 + j) * 16 + (lane & 15);
                if (row < g.m && col < g.n) store_residue(C + (int64_t)row * g.ldc + col, r, pr.p, g.sub);
            }
}

// ------------------------------------------------- LDS-staged INT8 tiles --
// A work-group of WY x WX waves, each owning RB x CB blocks of 16 x 16
// outputs for all 7 shift groups, covers WY*RB 16-row blocks and WX*CB
// 16-column blocks.  The operand fragments of one 64-k step (A: WY*RB blocks x
// 4 digits, B: WX*CB blocks x 4 digits, 1 KiB each) are copied global -> LDS
// with 16-byte direct loads into two alternating buffers, split evenly over
// the waves, and each wave reads its own fragments from LDS.
//
// Order inside a step: wait for this wave's copies of step kt, barrier (every
// wave's copies of step kt are in LDS and every wave has finished reading
// step kt-1), read the fragments of step kt, start the copies of step kt+1
// into the other buffer, then run the MFMAs of step kt while those copies are
// in flight.  Reading before starting the next copies keeps the compiler from
// waiting for those copies before the reads.
template <int WY, int WX, int RB, int CB>
struct I8Shape {
    static constexpr int kWY = WY, kWX = WX, kRB = RB, kCB = CB;
    static constexpr int kWaves = WY * WX;
    static constexpr int kFragA = WY * RB * 4, kFragB = WX * CB * 4, kFrag = kFragA + kFragB;
    static constexpr int kFragPerWave = kFrag / kWaves;
    static_assert(kFrag % kWaves == 0, "copies split evenly over the waves");
};
using ShapeLds = I8Shape<2, 2, 2, 4>;     // 64 x 128, 4 waves of 32 x 64
using ShapeW8 = I8Shape<2, 4, 2, 2>;      // 64 x 128, 8 waves of 32 x 32
using ShapeHalf = I8Shape<2, 2, 2, 2>;    // 64 x 64, 4 waves of 32 x 32
static_assert(ShapeLds::kWY * ShapeLds::kRB * 16 == kI8TileM && ShapeLds::kWX * ShapeLds::kCB * 16 == kI8TileN,
              "tile shape");
static_assert(ShapeW8::kWY * ShapeW8::kRB * 16 == kI8TileM && ShapeW8::kWX * ShapeW8::kCB * 16 == kI8TileN,
              "tile shape");
static_assert(2 * ShapeHalf::kWX * ShapeHalf::kCB * 16 == kI8TileN, "two halves make a tile");

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

// One 64-k step of a work-group tile: wait for this wave's copies of the
// step, barrier, read this wave's fragments from `cur`, run `next` (which
// starts the copies of a later step into the other buffer, or does nothing),
// then the 16 digit-pair MFMAs per block.  (Peeling the last step off the
// loops, so that the compiler can overlap the reads with the first MFMAs
// instead of waiting for all of them at the branch join, measured 2 % slower
// on the n = 4096 product.)
template <class S, class Next>
__device__ __forceinline__ void i8_step(const v4i *cur, int lane, int wy, int wx,
                                        v4i (&acc)[7][S::kRB][S::kCB], Next &&next) {
    vm_wait_0();
    plain_barrier();
    v4i a[S::kRB][4], b[S::kCB][4];
#pragma unroll
    for (int i = 0; i < S::kRB; ++i)
#pragma unroll
        for (int d = 0; d < 4; ++d) a[i][d] = cur[((wy * S::kRB + i) * 4 + d) * 64 + lane];
#pragma unroll
    for (int j = 0; j < S::kCB; ++j)
#pragma unroll
        for (int d = 0; d < 4; ++d) b[j][d] = cur[(S::kFragA + (wx * S::kCB + j) * 4 + d) * 64 + lane];
    next();
#pragma unroll
    for (int da = 0; da < 4; ++da)
#pragma unroll
        for (int db = 0; db < 4; ++db)
#pragma unroll
            for (int i = 0; i < S::kRB; ++i)
#pragma unroll
                for (int j = 0; j < S::kCB; ++j)
                    acc[da + db][i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[i][da], b[j][db],
                                                                               acc[da + db][i][j], 0, 0, 0);
}

// One work-group tile: 16-row blocks from rblk0, 16-column blocks from cblk0.
template <class S>
__device__ __forceinline__ void i8_lds_tile(const GemmProblem &g, int plane, int rblk0, int cblk0,
                                            const PrimeConst *__restrict__ pc,
                                            v4i (*sbuf)[S::kFrag * 64]) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wy = wave / S::kWX, wx = wave % S::kWX;
    const int KT = g.KT;
    const char *Ag = g.At + (int64_t)plane * g.a_plane_bytes + (int64_t)rblk0 * KT * 4096 + lane * 16;
    const char *Bg = g.Bt + (int64_t)plane * g.b_plane_bytes + (int64_t)cblk0 * KT * 4096 + lane * 16;
    // Fragment f of a step: f < kFragA is A block f/4, digit f%4; otherwise
    // B block (f-kFragA)/4, digit (f-kFragA)%4.  Wave w copies
    // f = w*kFragPerWave .. (w+1)*kFragPerWave-1.
    const char *src[S::kFragPerWave];
#pragma unroll
    for (int i = 0; i < S::kFragPerWave; ++i) {
        const int f = wave * S::kFragPerWave + i;
        src[i] = f < S::kFragA ? Ag + ((int64_t)(f >> 2) * KT) * 4096 + (f & 3) * 1024
                               : Bg + ((int64_t)((f - S::kFragA) >> 2) * KT) * 4096 + ((f - S::kFragA) & 3) * 1024;
    }
    auto issue = [&](v4i *buf, int kt) {
#pragma unroll
        for (int i = 0; i < S::kFragPerWave; ++i) {
            const int f = wave * S::kFragPerWave + i;
            __builtin_amdgcn_global_load_lds((const void *)(src[i] + (int64_t)kt * 4096),
                                             (lds_void *)(buf + f * 64), 16, 0, 0);
        }
    };

    v4i acc[7][S::kRB][S::kCB];
#pragma unroll
    for (int s = 0; s < 7; ++s)
#pragma unroll
        for (int i = 0; i < S::kRB; ++i)
#pragma unroll
            for (int j = 0; j < S::kCB; ++j) acc[s][i][j] = v4i{0, 0, 0, 0};

    issue(sbuf[0], 0);
    for (int kt = 0; kt < KT; ++kt)
        i8_step<S>(sbuf[kt & 1], lane, wy, wx, acc, [&] {
            if (kt + 1 < KT) issue(sbuf[(kt + 1) & 1], kt + 1);
        });

    const PrimeConst pr = pc[g.prime_begin + plane];
    uint32_t *C = g.C + (int64_t)plane * g.cps;
#pragma unroll
    for (int i = 0; i < S::kRB; ++i)
#pragma unroll
        for (int j = 0; j < S::kCB; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const uint32_t r = recombine(acc[0][i][j][v], acc[1][i][j][v], acc[2][i][j][v], acc[3][i][j][v],
                                             acc[4][i][j][v], acc[5][i][j][v], acc[6][i][j][v], pr);
                const int row = (rblk0 + wy * S::kRB + i) * 16 + 4 * (lane >> 4) + v;
                const int col = (cblk0 + wx * S::kCB + j) * 16 + (lane & 15);
                if (row < g.m && col < g.n) store_residue(C + (int64_t)row * g.ldc + col, r, pr.p, g.sub);
            }
}

// ------------------------------------------ two primes, CRT in the epilogue --
// Whole-product plans whose problems have one or two primes and one output
// word.  A work-group computes its tile for both primes in turn, as one
// continuous run of k steps over the same double buffer (the copies of the
// second prime's first step overlap the first prime's last step). It keeps
// the first prime's reduced products in registers and writes the CRT of the
// pair as int64. The C residue planes and the CRT launch are not needed.
//
// The CRT of two primes (Section 3.1's reconstruction at L = 2): with
// r0 = x mod p0 and r1 = x mod p1, u = r0 + p0 t where
// t = (r1 - r0) p0^{-1} mod p1, so u is in [0, p0 p1), and x = u, or
// u - p0 p1 when u > (p0 p1 - 1)/2. Every product below is an integer
// below 2^52, exact in doubles.

// v mod p in [0, p) for an integer 0 <= v < 2^52. The rounded quotient is
// wrong by at most one, and then only next to a half-integer, so the
// remainder lands in (-p, p) and one conditional +p fixes it.
__device__ __forceinline__ double mod_nonneg(double v, const PrimeConst &pr) {
    const double r = fma(-rint(v * pr.pinv), pr.pf, v);
    return r < 0.0 ? r + pr.pf : r;
}

__device__ __forceinline__ int64_t crt_pair(uint32_t r0, uint32_t r1, const PrimeConst &p0,
                                            const PrimeConst &p1, double inv) {
    double d = (double)r1 - mod_nonneg((double)r0, p1);
    d = d < 0.0 ? d + p1.pf : d;
    const uint64_t t = (uint64_t)mod_nonneg(d * inv, p1);
    const uint64_t M = (uint64_t)p0.p * p1.p;
    const uint64_t u = (uint64_t)r0 + (uint64_t)p0.p * t;
    return u > (M - 1) / 2 ? (int64_t)u - (int64_t)M : (int64_t)u;
}

template <class S>
__device__ __forceinline__ void i8_lds_tile_crt(const GemmProblem &g, int rblk0, int cblk0,
                                                const PrimeConst *__restrict__ pc,
                                                v4i (*sbuf)[S::kFrag * 64]) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wy = wave / S::kWX, wx = wave % S::kWX;
    const int KT = g.KT;
    const int L = g.L;   // 1 or 2 (the host checks)
    const char *Ag = g.At + (int64_t)rblk0 * KT * 4096 + lane * 16;
    const char *Bg = g.Bt + (int64_t)cblk0 * KT * 4096 + lane * 16;
    // The fragments this wave copies, as in i8_lds_tile, and the distance
    // between the planes of their operand.
    const char *src[S::kFragPerWave];
    int64_t pstride[S::kFragPerWave];
#pragma unroll
    for (int i = 0; i < S::kFragPerWave; ++i) {
        const int f = wave * S::kFragPerWave + i;
        const bool isA = f < S::kFragA;
        src[i] = isA ? Ag + ((int64_t)(f >> 2) * KT) * 4096 + (f & 3) * 1024
                     : Bg + ((int64_t)((f - S::kFragA) >> 2) * KT) * 4096 + ((f - S::kFragA) & 3) * 1024;
        pstride[i] = isA ? g.a_plane_bytes : g.b_plane_bytes;
    }
    auto issue = [&](v4i *buf, int plane, int kt) {
#pragma unroll
        for (int i = 0; i < S::kFragPerWave; ++i) {
            const int f = wave * S::kFragPerWave + i;
            __builtin_amdgcn_global_load_lds((const void *)(src[i] + plane * pstride[i] + (int64_t)kt * 4096),
                                             (lds_void *)(buf + f * 64), 16, 0, 0);
        }
    };

    v4i acc[7][S::kRB][S::kCB];
    // Steps j0 .. j0 + KT - 1 of the run (buffer j & 1) for one plane; the
    // copy of its first step is already in flight.  The last step starts the
    // copy of the next plane's first step when there is one.
    auto run_plane = [&](int plane, int j0) {
#pragma unroll
        for (int s = 0; s < 7; ++s)
#pragma unroll
            for (int i = 0; i < S::kRB; ++i)
#pragma unroll
                for (int j = 0; j < S::kCB; ++j) acc[s][i][j] = v4i{0, 0, 0, 0};
        for (int kt = 0; kt < KT; ++kt)
            i8_step<S>(sbuf[(j0 + kt) & 1], lane, wy, wx, acc, [&] {
                if (kt + 1 < KT) issue(sbuf[(j0 + kt + 1) & 1], plane, kt + 1);
                else if (plane + 1 < L) issue(sbuf[(j0 + kt + 1) & 1], plane + 1, 0);
            });
    };

    issue(sbuf[0], 0, 0);
    run_plane(0, 0);
    const PrimeConst p0 = pc[g.prime_begin];
    uint32_t r0[S::kRB][S::kCB][4];
#pragma unroll
    for (int i = 0; i < S::kRB; ++i)
#pragma unroll
        for (int j = 0; j < S::kCB; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                r0[i][j][v] = recombine(acc[0][i][j][v], acc[1][i][j][v], acc[2][i][j][v], acc[3][i][j][v],
                                        acc[4][i][j][v], acc[5][i][j][v], acc[6][i][j][v], p0);
    int64_t *C = g.C64;
    if (L == 2) {
        run_plane(1, KT);
        const PrimeConst p1 = pc[g.prime_begin + 1];
        const double inv = (double)g.crt_inv;
#pragma unroll
        for (int i = 0; i < S::kRB; ++i)
#pragma unroll
            for (int j = 0; j < S::kCB; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const uint32_t r1 = recombine(acc[0][i][j][v], acc[1][i][j][v], acc[2][i][j][v],
                                                  acc[3][i][j][v], acc[4][i][j][v], acc[5][i][j][v],
                                                  acc[6][i][j][v], p1);
                    const int row = (rblk0 + wy * S::kRB + i) * 16 + 4 * (lane >> 4) + v;
                    const int col = (cblk0 + wx * S::kCB + j) * 16 + (lane & 15);
                    if (row < g.m && col < g.n) C[(int64_t)row * g.ldc64 + col] = crt_pair(r0[i][j][v], r1, p0, p1, inv);
                }
    } else {
#pragma unroll
        for (int i = 0; i < S::kRB; ++i)
#pragma unroll
            for (int j = 0; j < S::kCB; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const uint32_t r = r0[i][j][v];
                    const int row = (rblk0 + wy * S::kRB + i) * 16 + 4 * (lane >> 4) + v;
                    const int col = (cblk0 + wx * S::kCB + j) * 16 + (lane & 15);
                    if (row < g.m && col < g.n)
                        C[(int64_t)row * g.ldc64 + col] = r > p0.half ? (int64_t)r - (int64_t)p0.p : (int64_t)r;
                }
    }
}

__global__ __launch_bounds__(256, 2) void k_gemm_i8_half_crt(const GemmProblem *__restrict__ P, int nprob,
                                                             int64_t total_tiles,
                                                             const PrimeConst *__restrict__ pc,
                                                             const int32_t *__restrict__ tile_prob) {
    __shared__ v4i sbuf[2][ShapeHalf::kFrag * 64];
    const int64_t h2 = xcd_window_remap(blockIdx.x, gridDim.x, kXcdWindow2);
    if (h2 >= 2 * total_tiles) return;
    const TileCoord tc = map_tile(P, nprob, h2 >> 1, tile_prob);
    i8_lds_tile_crt<ShapeHalf>(P[tc.q], tc.tm * 4, tc.tn * 8 + (int)(h2 & 1) * 4, pc, sbuf);
}

__global__ __launch_bounds__(256) void k_gemm_i8_lds(const GemmProblem *__restrict__ P, int nprob,
                                                     int64_t total_tiles,
                                                     const PrimeConst *__restrict__ pc,
                                                     const int32_t *__restrict__ tile_prob) {
    __shared__ v4i sbuf[2][ShapeLds::kFrag * 64];
    const int64_t t = xcd_window_remap(blockIdx.x, gridDim.x, kXcdWindow1);
    if (t >= total_tiles) return;
    const TileCoord tc = map_tile(P, nprob, t, tile_prob);
    i8_lds_tile<ShapeLds>(P[tc.q], tc.plane, tc.tm * 4, tc.tn * 8, pc, sbuf);
}

__global__ __launch_bounds__(512) void k_gemm_i8_w8(const GemmProblem *__restrict__ P, int nprob,
                                                    int64_t total_tiles,
                                                    const PrimeConst *__restrict__ pc,
                                                    const int32_t *__restrict__ tile_prob) {
    __shared__ v4i sbuf[2][ShapeW8::kFrag * 64];
    const int64_t t = xcd_window_remap(blockIdx.x, gridDim.x, kXcdWindow1);
    if (t >= total_tiles) return;
    const TileCoord tc = map_tile(P, nprob, t, tile_prob);
    i8_lds_tile<ShapeW8>(P[tc.q], tc.plane, tc.tm * 4, tc.tn * 8, pc, sbuf);
}

// Half tiles: launch index h2 covers tile h2/2, column half h2%2.  The two
// halves of a tile are adjacent in launch order and so run on the same XCD,
// where they share the A panel in L2.
__global__ __launch_bounds__(256, 2) void k_gemm_i8_half(const GemmProblem *__restrict__ P, int nprob,
                                                         int64_t total_tiles,
                                                         const PrimeConst *__restrict__ pc,
                                                         const int32_t *__restrict__ tile_prob) {
    __shared__ v4i sbuf[2][ShapeHalf::kFrag * 64];
    const int64_t h2 = xcd_window_remap(blockIdx.x, gridDim.x, kXcdWindow2);
    if (h2 >= 2 * total_tiles) return;
    const TileCoord tc = map_tile(P, nprob, h2 >> 1, tile_prob);
    i8_lds_tile<ShapeHalf>(P[tc.q], tc.plane, tc.tm * 4, tc.tn * 8 + (int)(h2 & 1) * 4, pc, sbuf);
}

// Persistent form: two work-groups per CU take half-tiles from a counter in
// tile order (the host sorts problems by decreasing tile cost, so the longest
// tiles go first).  The counter is reset by the prep kernel of the same call.
__global__ __launch_bounds__(256, 2) void k_gemm_i8_half_persistent(const GemmProblem *__restrict__ P,
                                                                    int nprob, int64_t total_tiles,
                                                                    const PrimeConst *__restrict__ pc,
                                                                    const int32_t *__restrict__ tile_prob,
                                                                    unsigned *__restrict__ counter) {
    __shared__ v4i sbuf[2][ShapeHalf::kFrag * 64];
    __shared__ unsigned next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(counter, 1u);
        __syncthreads();
        const int64_t h2 = (unsigned)__builtin_amdgcn_readfirstlane((int)next);   // uniform
        __syncthreads();
        if (h2 >= 2 * total_tiles) break;
        const TileCoord tc = map_tile(P, nprob, h2 >> 1, tile_prob);
        i8_lds_tile<ShapeHalf>(P[tc.q], tc.plane, tc.tm * 4, tc.tn * 8 + (int)(h2 & 1) * 4, pc, sbuf);
    }
}

}  // namespace

void launch_gemm_i8(int variant, const GemmProblem *P, int nprob, int64_t tiles,
                    const PrimeConst *pc, const int32_t *tile_prob, unsigned *counter,
                    int num_cus, hipStream_t s) {
    if (variant == kI8Direct) {
        hipLaunchKernelGGL(k_gemm_i8, dim3((unsigned)tiles), dim3(256), 0, s, P, nprob, tiles, pc, tile_prob);
    } else if (variant == kI8Lds) {
        hipLaunchKernelGGL(k_gemm_i8_lds, dim3((unsigned)tiles), dim3(256), 0, s, P, nprob, tiles, pc, tile_prob);
    } else if (variant == kI8Wave8) {
        hipLaunchKernelGGL(k_gemm_i8_w8, dim3((unsigned)tiles), dim3(512), 0, s, P, nprob, tiles, pc, tile_prob);
    } else if (variant == kI8HalfPersistent && counter) {
        const int64_t grid = std::min<int64_t>(2 * tiles, 2 * (int64_t)num_cus);
        hipLaunchKernelGGL(k_gemm_i8_half_persistent, dim3((unsigned)grid), dim3(256), 0, s, P, nprob,
                           tiles, pc, tile_prob, counter);
    } else {
        hipLaunchKernelGGL(k_gemm_i8_half, dim3((unsigned)(2 * tiles)), dim3(256), 0, s, P, nprob, tiles,
                           pc, tile_prob);
    }
}

void launch_gemm_i8_crt(const GemmProblem *P, int nprob, int64_t tiles, const PrimeConst *pc,
                        const int32_t *tile_prob, hipStream_t s) {
    hipLaunchKernelGGL(k_gemm_i8_half_crt, dim3((unsigned)(2 * tiles)), dim3(256), 0, s, P, nprob, tiles, pc,
                       tile_prob);
}

}  // namespace gemm
}  // namespace rns
