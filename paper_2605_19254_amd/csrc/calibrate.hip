// Measured ceilings of the matrix and vector units, so that achieved rates can
// be stated beside the published peaks.  Each probe runs independent
// accumulation chains in every wave, eight waves per CU, with its operands in
// registers: no memory traffic inside the timed loop.  With random operands the
// probe switches as many bits as real data does, which matters on a part whose
// clock falls when the matrix units draw more power.
#include "internal.hpp"

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kBlock = 256;
constexpr int kWavesPerCU = 8;
constexpr int kBlocksPerCU = kWavesPerCU * 64 / kBlock;
constexpr int kChains = 8;
// The launch bounds state the two work-groups per CU that the grid places.
// With a bound of one work-group the compiler keeps the accumulators in the
// accumulation registers (AGPRs), and 16x16x64 INT8 MFMAs with AGPR
// accumulators were measured about 20% slower on MI355X than with ordinary
// VGPR accumulators, which is where the GEMM kernels keep them.

__device__ __forceinline__ unsigned mix32(unsigned x) {
    // Integer finaliser (xor-shift / multiply rounds) for operand bits.
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

// Operand registers: kChains A and B values per lane, random or all ones.
template <class V>
__device__ __forceinline__ void fill_int(V (&a)[kChains], V (&b)[kChains], int words, bool random, unsigned seed) {
    const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
#pragma unroll
    for (int i = 0; i < kChains; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            a[i][j] = random ? (int)mix32(seed + (t * kChains + i) * 4 + j) : 0x01010101;
            b[i][j] = random ? (int)mix32(seed * 7u + 0x9e3779b9u + (t * kChains + i) * 4 + j) : 0x01010101;
        }
    (void)words;
}

// One iteration = 2 * kChains instructions (two pairings of the operands).
__global__ __launch_bounds__(kBlock, kBlocksPerCU) void k_cal_i8_16(int iters, int random, unsigned seed, int *out) {
    v4i a[kChains], b[kChains], acc[kChains];
    fill_int(a, b, 4, random != 0, seed);
#pragma unroll
    for (int i = 0; i < kChains; ++i) acc[i] = v4i{0, 0, 0, 0};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < kChains; ++i) acc[i] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[i], b[i], acc[i], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < kChains; ++i)
            acc[i] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[i], b[(i + 1) % kChains], acc[i], 0, 0, 0);
    }
    int s = 0;
#pragma unroll
    for (int i = 0; i < kChains; ++i) s += acc[i][0] ^ acc[i][1] ^ acc[i][2] ^ acc[i][3];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(kBlock, kBlocksPerCU) void k_cal_i8_32(int iters, int random, unsigned seed, int *out) {
    v4i a[kChains], b[kChains];
    v16i acc[kChains];
    fill_int(a, b, 4, random != 0, seed);
#pragma unroll
    for (int i = 0; i < kChains; ++i) acc[i] = v16i{};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < kChains; ++i) acc[i] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[i], b[i], acc[i], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < kChains; ++i)
            acc[i] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[i], b[(i + 1) % kChains], acc[i], 0, 0, 0);
    }
    int s = 0;
#pragma unroll
    for (int i = 0; i < kChains; ++i) s += acc[i][0] ^ acc[i][5] ^ acc[i][10] ^ acc[i][15];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__device__ __forceinline__ double unit_double(unsigned bits) {
    // A double in [1, 2) with random low mantissa bits (bounded products).
    return 1.0 + (double)(bits >> 8) * (1.0 / 16777216.0);
}

__global__ __launch_bounds__(kBlock, kBlocksPerCU) void k_cal_f64_mfma(int iters, int random, unsigned seed, int *out) {
    const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
    double a[kChains], b[kChains];
    v4d acc[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i) {
        a[i] = random ? unit_double(mix32(seed + t * kChains + i)) : 1.0;
        b[i] = random ? unit_double(mix32(seed * 7u + 12345u + t * kChains + i)) * 1e-300 : 1e-300;
        acc[i] = v4d{0, 0, 0, 0};
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < kChains; ++i) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[i], acc[i], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < kChains; ++i)
            acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[(i + 1) % kChains], acc[i], 0, 0, 0);
    }
    double s = 0;
#pragma unroll
    for (int i = 0; i < kChains; ++i) s += acc[i][0] + acc[i][3];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s != 0.0;
}

__global__ __launch_bounds__(kBlock, kBlocksPerCU) void k_cal_f64_fma(int iters, int random, unsigned seed, int *out) {
    const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
    double x[kChains], y[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i) {
        x[i] = random ? unit_double(mix32(seed + t * kChains + i)) : 1.0;
        y[i] = random ? 0.5 * unit_double(mix32(seed * 7u + 999u + t * kChains + i)) : 0.75;
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < kChains; ++i) x[i] = fma(x[i], y[i], 0.25);   // stays in (0.25, 1.25)
#pragma unroll
        for (int i = 0; i < kChains; ++i) x[i] = fma(x[i], y[(i + 1) % kChains], 0.25);
    }
    double s = 0;
#pragma unroll
    for (int i = 0; i < kChains; ++i) s += x[i];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s > 0.0;
}

}  // namespace

extern "C" int rns_calibrate(rns_ctx *ctx, int kind, int iters, int random_operands, void *stream,
                             double *ops_per_s, double *ms) {
    if (!ctx || !ops_per_s || !ms || iters < 1 || kind < 0 || kind > 3) return RNS_EINVAL;
    RNS_HIP(hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int grid = ctx->num_cus * kWavesPerCU * 64 / kBlock;
    // Operations per wave and iteration (2*kChains instructions).
    const double per_inst[4] = {16.0 * 16 * 64 * 2, 32.0 * 32 * 32 * 2, 16.0 * 16 * 4 * 2, 64.0 * 2};
    int *out = nullptr;
    RNS_HIP(hipMalloc(&out, (size_t)grid * kBlock * sizeof(int)));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int st = RNS_OK;
    auto launch = [&](int n) {
        switch (kind) {
        case 0: hipLaunchKernelGGL(k_cal_i8_16, dim3(grid), dim3(kBlock), 0, s, n, random_operands, 1u, out); break;
        case 1: hipLaunchKernelGGL(k_cal_i8_32, dim3(grid), dim3(kBlock), 0, s, n, random_operands, 1u, out); break;
        case 2: hipLaunchKernelGGL(k_cal_f64_mfma, dim3(grid), dim3(kBlock), 0, s, n, random_operands, 1u, out); break;
        default: hipLaunchKernelGGL(k_cal_f64_fma, dim3(grid), dim3(kBlock), 0, s, n, random_operands, 1u, out); break;
        }
    };
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) st = RNS_EDEVICE;
    if (st == RNS_OK) {
        launch(iters / 8 + 1);                                  // warm-up
        float t = 0.0f;
        if (hipEventRecord(e0, s) != hipSuccess) st = RNS_EDEVICE;
        if (st == RNS_OK) launch(iters);
        if (st == RNS_OK && (hipGetLastError() != hipSuccess || hipEventRecord(e1, s) != hipSuccess ||
                             hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess))
            st = RNS_EDEVICE;
        if (st == RNS_OK) {
            const double waves = (double)grid * (kBlock / 64);
            *ms = t;
            *ops_per_s = waves * iters * 2 * kChains * per_inst[kind] / (t * 1e-3);
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (hipFree(out) != hipSuccess && st == RNS_OK) st = RNS_EDEVICE;
    return st;
}
