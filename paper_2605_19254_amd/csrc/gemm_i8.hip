// INT8-limb residue product (Section 3.1: one exact product per prime).
//
// Each balanced residue r (|r| <= (p-1)/2) is split into four signed base-256
// digits r = d0 + d1*2^8 + d2*2^16 + d3*2^24, d0..d2 in [-128, 127],
// |d3| <= 2 (the prep kernel does the split).  The 16 digit-pair products are
// computed with v_mfma_i32_16x16x64_i8 and summed in int32 per shift group
// s = i+j (7 groups).  The largest group sum per term is 3*2^14, so the int32
// sums are exact for k <= 43690.  The epilogue reduces each group mod p and
// recombines C = sum_s (C_s mod p)(2^(8s) mod p) mod p in exact doubles:
// every product of two balanced residues is below 2^50 and seven of them
// stay below 2^53.
//
// Work-group tile 64 x 128: four waves in 2 x 2, each owning 32 x 64 outputs
// (2 x 4 blocks of 16 x 16) for all 7 groups, i.e. 224 accumulator registers.
#include "gemm_common.hpp"

#include <algorithm>

namespace rns {
namespace gemm {
namespace {

// ------------------------------------------------------------- INT8 GEMM --

__global__ __launch_bounds__(256) void k_gemm_i8(const GemmProblem *__restrict__ P, int nprob,
                                                 int64_t total_tiles,
                                                 const PrimeConst *__restrict__ pc,
        const int32_t *__restrict__ tile_prob) {
    const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
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

    // Epilogue: C = sum_s (C_s mod p) * w_s mod p, all in exact doubles.
    const PrimeConst pr = pc[g.prime_begin + tc.plane];
    uint32_t *C = g.C + (int64_t)tc.plane * g.cps;
#pragma unroll
    for (int i = 0; i < kI8WaveRB; ++i)
#pragma unroll
        for (int j = 0; j < kI8WaveCB; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                double sum = 0.0;
#pragma unroll
                for (int s = 0; s < 7; ++s) {
                    const double cs = (double)acc[s][i][j][v];
                    const double r = fma(-rint(cs * pr.pinv), pr.pf, cs);   // |r| <= p/2
                    sum = fma(r, pr.w[s], sum);                              // |sum| < 7*2^50
                }
                double r = fma(-rint(sum * pr.pinv), pr.pf, sum);
                r = r < 0.0 ? r + pr.pf : r;
                const int row = (rb0 + i) * 16 + 4 * (lane >> 4) + v;
                const int col = (cb0 + j) * 16 + (lane & 15);
                if (row < g.m && col < g.n) C[(int64_t)row * g.ldc + col] = (uint32_t)r;
            }
}

// ------------------------------------------------- INT8 GEMM, LDS pipeline --
// Same tiles and arithmetic as k_gemm_i8, but the work-group's A and B digit
// tiles of one 64-k step (4 + 8 row/col blocks x 4 digits = 48 fragments of
// 1 KiB) are copied global -> LDS with 16-byte direct loads into two
// alternating buffers, and each wave reads its fragments from LDS.  The two
// waves that share an A (B) panel read it once from L2 instead of twice, and
// no registers hold prefetched fragments.
//
// Order inside a step: wait for this wave's copies of step kt, barrier (now
// every wave's copies of step kt are in LDS and every wave has finished
// reading step kt-1), read the fragments of step kt, start the copies of step
// kt+1 into the other buffer, then run the 128 MFMAs of step kt while those
// copies are in flight.

constexpr int kI8FragA = 2 * kI8WaveRB * 4;           // A fragments per 64-k step
constexpr int kI8FragB = 2 * kI8WaveCB * 4;           // B fragments per 64-k step
constexpr int kI8Frag = kI8FragA + kI8FragB;          // 48
constexpr int kI8FragPerWave = kI8Frag / 4;           // 12

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

__device__ __forceinline__ void i8_lds_tile(const GemmProblem *__restrict__ P, int nprob,
                                            int64_t t, const PrimeConst *__restrict__ pc,
                                            const int32_t *__restrict__ tile_prob,
                                            v4i (*sbuf)[kI8Frag * 64]) {
    const TileCoord tc = map_tile(P, nprob, t, tile_prob);
    const GemmProblem &g = P[tc.q];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wy = wave >> 1, wx = wave & 1;
    const int KT = g.KT;
    const char *Ag = g.At + (int64_t)tc.plane * g.a_plane_bytes +
                     (int64_t)tc.tm * (2 * kI8WaveRB) * KT * 4096 + lane * 16;
    const char *Bg = g.Bt + (int64_t)tc.plane * g.b_plane_bytes +
                     (int64_t)tc.tn * (2 * kI8WaveCB) * KT * 4096 + lane * 16;
    // Fragment f of a step: f < kI8FragA is A block f/4, digit f%4; otherwise
    // B block (f-kI8FragA)/4, digit (f-kI8FragA)%4.  Wave w copies f = 12w..12w+11.
    const char *src[kI8FragPerWave];
#pragma unroll
    for (int i = 0; i < kI8FragPerWave; ++i) {
        const int f = wave * kI8FragPerWave + i;
        src[i] = f < kI8FragA ? Ag + ((int64_t)(f >> 2) * KT) * 4096 + (f & 3) * 1024
                              : Bg + ((int64_t)((f - kI8FragA) >> 2) * KT) * 4096 + ((f - kI8FragA) & 3) * 1024;
    }
    auto issue = [&](v4i *buf, int kt) {
#pragma unroll
        for (int i = 0; i < kI8FragPerWave; ++i) {
            const int f = wave * kI8FragPerWave + i;
            __builtin_amdgcn_global_load_lds((const void *)(src[i] + (int64_t)kt * 4096),
                                             (lds_void *)(buf + f * 64), 16, 0, 0);
        }
    };

    v4i acc[7][kI8WaveRB][kI8WaveCB];
#pragma unroll
    for (int s = 0; s < 7; ++s)
#pragma unroll
        for (int i = 0; i < kI8WaveRB; ++i)
#pragma unroll
            for (int j = 0; j < kI8WaveCB; ++j) acc[s][i][j] = v4i{0, 0, 0, 0};

    issue(sbuf[0], 0);
    for (int kt = 0; kt < KT; ++kt) {
        const v4i *cur = sbuf[kt & 1];
        vm_wait_0();
        plain_barrier();
        v4i a[kI8WaveRB][4], b[kI8WaveCB][4];
#pragma unroll
        for (int i = 0; i < kI8WaveRB; ++i)
#pragma unroll
            for (int d = 0; d < 4; ++d) a[i][d] = cur[((wy * kI8WaveRB + i) * 4 + d) * 64 + lane];
#pragma unroll
        for (int j = 0; j < kI8WaveCB; ++j)
#pragma unroll
            for (int d = 0; d < 4; ++d) b[j][d] = cur[(kI8FragA + (wx * kI8WaveCB + j) * 4 + d) * 64 + lane];
        if (kt + 1 < KT) issue(sbuf[(kt + 1) & 1], kt + 1);
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
    }

    const int rb0 = tc.tm * (2 * kI8WaveRB) + wy * kI8WaveRB;
    const int cb0 = tc.tn * (2 * kI8WaveCB) + wx * kI8WaveCB;
    const PrimeConst pr = pc[g.prime_begin + tc.plane];
    uint32_t *C = g.C + (int64_t)tc.plane * g.cps;
#pragma unroll
    for (int i = 0; i < kI8WaveRB; ++i)
#pragma unroll
        for (int j = 0; j < kI8WaveCB; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                double sum = 0.0;
#pragma unroll
                for (int s = 0; s < 7; ++s) {
                    const double cs = (double)acc[s][i][j][v];
                    const double r = fma(-rint(cs * pr.pinv), pr.pf, cs);
                    sum = fma(r, pr.w[s], sum);
                }
                double r = fma(-rint(sum * pr.pinv), pr.pf, sum);
                r = r < 0.0 ? r + pr.pf : r;
                const int row = (rb0 + i) * 16 + 4 * (lane >> 4) + v;
                const int col = (cb0 + j) * 16 + (lane & 15);
                if (row < g.m && col < g.n) C[(int64_t)row * g.ldc + col] = (uint32_t)r;
            }
}

// ------------------------------------------- three-stage LDS pipeline --
// As i8_lds_tile, with three LDS buffers so that the copies of two later steps
// are in flight while a step computes.  The fragments of a step are read with
// one inline-assembly block of 24 ds_read_b128 that waits for its own reads
// before it ends; the compiler therefore does not wait for the outstanding
// copies before those reads (it cannot tell the buffers apart), and the
// explicit vmcnt wait before the barrier covers exactly the copies of the
// step about to be read.

__device__ __forceinline__ void vm_wait_12() { __builtin_amdgcn_s_waitcnt(0x0F7C); }  // vmcnt(12)

__device__ __forceinline__ void lds_read_step(uint32_t a_addr, uint32_t b_addr,
                                              v4i (&a)[kI8WaveRB][4], v4i (&b)[kI8WaveCB][4]) {
    static_assert(kI8WaveRB == 2 && kI8WaveCB == 4, "read block is written for 2 x 4 blocks");
    asm volatile(
        "ds_read_b128 %0, %24\n"
        "ds_read_b128 %1, %24 offset:1024\n"
        "ds_read_b128 %2, %24 offset:2048\n"
        "ds_read_b128 %3, %24 offset:3072\n"
        "ds_read_b128 %4, %24 offset:4096\n"
        "ds_read_b128 %5, %24 offset:5120\n"
        "ds_read_b128 %6, %24 offset:6144\n"
        "ds_read_b128 %7, %24 offset:7168\n"
        "ds_read_b128 %8, %25\n"
        "ds_read_b128 %9, %25 offset:1024\n"
        "ds_read_b128 %10, %25 offset:2048\n"
        "ds_read_b128 %11, %25 offset:3072\n"
        "ds_read_b128 %12, %25 offset:4096\n"
        "ds_read_b128 %13, %25 offset:5120\n"
        "ds_read_b128 %14, %25 offset:6144\n"
        "ds_read_b128 %15, %25 offset:7168\n"
        "ds_read_b128 %16, %25 offset:8192\n"
        "ds_read_b128 %17, %25 offset:9216\n"
        "ds_read_b128 %18, %25 offset:10240\n"
        "ds_read_b128 %19, %25 offset:11264\n"
        "ds_read_b128 %20, %25 offset:12288\n"
        "ds_read_b128 %21, %25 offset:13312\n"
        "ds_read_b128 %22, %25 offset:14336\n"
        "ds_read_b128 %23, %25 offset:15360\n"
        "s_waitcnt lgkmcnt(0)\n"
        : "=&v"(a[0][0]), "=&v"(a[0][1]), "=&v"(a[0][2]), "=&v"(a[0][3]),
          "=&v"(a[1][0]), "=&v"(a[1][1]), "=&v"(a[1][2]), "=&v"(a[1][3]),
          "=&v"(b[0][0]), "=&v"(b[0][1]), "=&v"(b[0][2]), "=&v"(b[0][3]),
          "=&v"(b[1][0]), "=&v"(b[1][1]), "=&v"(b[1][2]), "=&v"(b[1][3]),
          "=&v"(b[2][0]), "=&v"(b[2][1]), "=&v"(b[2][2]), "=&v"(b[2][3]),
          "=&v"(b[3][0]), "=&v"(b[3][1]), "=&v"(b[3][2]), "=&v"(b[3][3])
        : "v"(a_addr), "v"(b_addr));
}

__device__ __forceinline__ void i8_lds3_tile(const GemmProblem *__restrict__ P, int nprob,
                                             int64_t t, const PrimeConst *__restrict__ pc,
                                             const int32_t *__restrict__ tile_prob,
                                             v4i (*sbuf)[kI8Frag * 64]) {
    const TileCoord tc = map_tile(P, nprob, t, tile_prob);
    const GemmProblem &g = P[tc.q];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wy = wave >> 1, wx = wave & 1;
    const int KT = g.KT;
    const char *Ag = g.At + (int64_t)tc.plane * g.a_plane_bytes +
                     (int64_t)tc.tm * (2 * kI8WaveRB) * KT * 4096 + lane * 16;
    const char *Bg = g.Bt + (int64_t)tc.plane * g.b_plane_bytes +
                     (int64_t)tc.tn * (2 * kI8WaveCB) * KT * 4096 + lane * 16;
    const char *src[kI8FragPerWave];
#pragma unroll
    for (int i = 0; i < kI8FragPerWave; ++i) {
        const int f = wave * kI8FragPerWave + i;
        src[i] = f < kI8FragA ? Ag + ((int64_t)(f >> 2) * KT) * 4096 + (f & 3) * 1024
                              : Bg + ((int64_t)((f - kI8FragA) >> 2) * KT) * 4096 + ((f - kI8FragA) & 3) * 1024;
    }
    auto issue = [&](v4i *buf, int kt) {
#pragma unroll
        for (int i = 0; i < kI8FragPerWave; ++i) {
            const int f = wave * kI8FragPerWave + i;
            __builtin_amdgcn_global_load_lds((const void *)(src[i] + (int64_t)kt * 4096),
                                             (lds_void *)(buf + f * 64), 16, 0, 0);
        }
    };
    // LDS byte addresses of this wave's A and B fragments in each buffer.
    uint32_t a_addr[3], b_addr[3];
#pragma unroll
    for (int u = 0; u < 3; ++u) {
        const uint32_t base = (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) v4i *)sbuf[u];
        a_addr[u] = base + (uint32_t)((wy * kI8WaveRB * 4) * 1024 + lane * 16);
        b_addr[u] = base + (uint32_t)((kI8FragA + wx * kI8WaveCB * 4) * 1024 + lane * 16);
    }

    v4i acc[7][kI8WaveRB][kI8WaveCB];
#pragma unroll
    for (int s = 0; s < 7; ++s)
#pragma unroll
        for (int i = 0; i < kI8WaveRB; ++i)
#pragma unroll
            for (int j = 0; j < kI8WaveCB; ++j) acc[s][i][j] = v4i{0, 0, 0, 0};

    issue(sbuf[0], 0);
    if (KT > 1) issue(sbuf[1], 1);
    int cur = 0;
    for (int kt = 0; kt < KT; ++kt) {
        if (kt + 1 < KT) vm_wait_12(); else vm_wait_0();
        plain_barrier();
        v4i a[kI8WaveRB][4], b[kI8WaveCB][4];
        lds_read_step(a_addr[cur], b_addr[cur], a, b);
        const int nxt2 = cur == 0 ? 2 : cur - 1;      // buffer of step kt+2 = buffer of step kt-1
        if (kt + 2 < KT) issue(sbuf[nxt2], kt + 2);
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
        cur = cur == 2 ? 0 : cur + 1;
    }

    const int rb0 = tc.tm * (2 * kI8WaveRB) + wy * kI8WaveRB;
    const int cb0 = tc.tn * (2 * kI8WaveCB) + wx * kI8WaveCB;
    const PrimeConst pr = pc[g.prime_begin + tc.plane];
    uint32_t *C = g.C + (int64_t)tc.plane * g.cps;
#pragma unroll
    for (int i = 0; i < kI8WaveRB; ++i)
#pragma unroll
        for (int j = 0; j < kI8WaveCB; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                double sum = 0.0;
#pragma unroll
                for (int s = 0; s < 7; ++s) {
                    const double cs = (double)acc[s][i][j][v];
                    const double r = fma(-rint(cs * pr.pinv), pr.pf, cs);
                    sum = fma(r, pr.w[s], sum);
                }
                double r = fma(-rint(sum * pr.pinv), pr.pf, sum);
                r = r < 0.0 ? r + pr.pf : r;
                const int row = (rb0 + i) * 16 + 4 * (lane >> 4) + v;
                const int col = (cb0 + j) * 16 + (lane & 15);
                if (row < g.m && col < g.n) C[(int64_t)row * g.ldc + col] = (uint32_t)r;
            }
}

__global__ __launch_bounds__(256) void k_gemm_i8_lds3(const GemmProblem *__restrict__ P, int nprob,
                                                      int64_t total_tiles,
                                                      const PrimeConst *__restrict__ pc,
                                                      const int32_t *__restrict__ tile_prob) {
    __shared__ v4i sbuf[3][kI8Frag * 64];
    const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    if (t >= total_tiles) return;
    i8_lds3_tile(P, nprob, t, pc, tile_prob, sbuf);
}

__global__ __launch_bounds__(256) void k_gemm_i8_lds(const GemmProblem *__restrict__ P, int nprob,
                                                     int64_t total_tiles,
                                                     const PrimeConst *__restrict__ pc,
        const int32_t *__restrict__ tile_prob) {
    __shared__ v4i sbuf[2][kI8Frag * 64];
    const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    if (t >= total_tiles) return;
    i8_lds_tile(P, nprob, t, pc, tile_prob, sbuf);
}

// Persistent form: one work-group per CU takes tiles from a counter in tile
// order (the host sorts problems by decreasing tile cost, so the longest
// tiles go first).  The counter is reset by the prep kernel of the same call.
__global__ __launch_bounds__(256) void k_gemm_i8_lds_persistent(const GemmProblem *__restrict__ P,
                                                                int nprob, int64_t total_tiles,
                                                                const PrimeConst *__restrict__ pc,
                                                                const int32_t *__restrict__ tile_prob,
                                                                unsigned *__restrict__ counter) {
    __shared__ v4i sbuf[2][kI8Frag * 64];
    __shared__ unsigned next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(counter, 1u);
        __syncthreads();
        const int64_t t = __builtin_amdgcn_readfirstlane((int)next);   // uniform tile index
        __syncthreads();
        if (t >= total_tiles) break;
        i8_lds_tile(P, nprob, t, pc, tile_prob, sbuf);
    }
}

}  // namespace

void launch_gemm_i8(int variant, const GemmProblem *P, int nprob, int64_t tiles,
                    const PrimeConst *pc, const int32_t *tile_prob, unsigned *counter,
                    int num_cus, hipStream_t s) {
    if (variant == kI8Direct) {
        hipLaunchKernelGGL(k_gemm_i8, dim3((unsigned)tiles), dim3(256), 0, s, P, nprob, tiles, pc, tile_prob);
    } else if (variant == kI8Lds3) {
        hipLaunchKernelGGL(k_gemm_i8_lds3, dim3((unsigned)tiles), dim3(256), 0, s, P, nprob, tiles, pc, tile_prob);
    } else if (variant == kI8LdsPersistent && counter) {
        const int64_t grid = std::min<int64_t>(tiles, num_cus);
        hipLaunchKernelGGL(k_gemm_i8_lds_persistent, dim3((unsigned)grid), dim3(256), 0, s, P, nprob,
                           tiles, pc, tile_prob, counter);
    } else {
        hipLaunchKernelGGL(k_gemm_i8_lds, dim3((unsigned)tiles), dim3(256), 0, s, P, nprob, tiles, pc, tile_prob);
    }
}

}  // namespace gemm
}  // namespace rns
