// rns_lift_step: one step of Dixon's p-adic lifting (Section 3 names it as
// the solver of the method's systems) through the same kernels and the same
// set-up as the Smith-form driver's lifting, on caller-given C, A and R, so
// that the step kernels can be checked on their own at any n up to their
// exactness bound.
#include "smith_internal.hpp"

#include <algorithm>

using namespace rns;

namespace {

// Device block freed on scope exit.
template <typename T>
struct Blk {
    T *p = nullptr;
    ~Blk() {
        if (p) (void)hipFree(p);
    }
    hipError_t alloc(size_t count) { return hipMalloc(reinterpret_cast<void **>(&p), std::max<size_t>(count, 1) * sizeof(T)); }
};

// Rm[c][r] = R[c][r] mod p (floor), for t vectors of stride ld.
__global__ __launch_bounds__(256) void k_floor_mod(const int64_t *__restrict__ R, int64_t count, uint32_t p,
                                                   uint32_t *__restrict__ Rm) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= count) return;
    const int64_t m = R[i] % (int64_t)p;
    Rm[i] = (uint32_t)(m < 0 ? m + (int64_t)p : m);
}

}  // namespace

extern "C" int rns_lift_step(int device, const uint32_t *C, const int64_t *A, const int64_t *R, int64_t n,
                             int t, uint32_t p, int form, uint32_t *X, int64_t *R_next, uint32_t *Rm_next,
                             int32_t *inexact, int *kernels, void *stream) {
    if (!C || !A || !R || !X || !R_next || !Rm_next || !inexact || !kernels) return RNS_EINVAL;
    if (n < 1 || t < 1 || t > kLiftMaxCols || p < 3 || p >= kPrimeLimit || (p & 1u) == 0) return RNS_EINVAL;
    if (form != 0 && form != 1) return RNS_EINVAL;
    if (form == 1 && n > kLiftMfmaMaxN) return RNS_EBOUND;
    if (n > 65536) return RNS_EBOUND;                  // the vector kernels' 64-bit sums
    hipStream_t s = (hipStream_t)stream;
    RNS_HIP(hipSetDevice(device));
    const int64_t ld = (n + 7) / 8 * 8;
    Blk<uint32_t> Cp, Rm0, Rm1, Xh;
    Blk<int64_t> R0, R1, base;
    Blk<int32_t> err, wide;
    Blk<int16_t> A16;
    Blk<int32_t> A32;
    Blk<char> Ct, At, Xd, Rmd;
    RNS_HIP(Cp.alloc((size_t)n * ld));
    RNS_HIP(Rm0.alloc((size_t)t * ld));
    RNS_HIP(Rm1.alloc((size_t)t * ld));
    RNS_HIP(Xh.alloc((size_t)t * ld));
    RNS_HIP(R0.alloc((size_t)t * ld));
    RNS_HIP(R1.alloc((size_t)t * ld));
    RNS_HIP(base.alloc(1));
    RNS_HIP(err.alloc(1));
    RNS_HIP(wide.alloc(1));
    // C and R into rows of stride ld, zero beyond column n (the kernels read
    // whole padded rows).
    RNS_HIP(hipMemsetAsync(Cp.p, 0, sizeof(uint32_t) * n * ld, s));
    RNS_HIP(hipMemcpy2DAsync(Cp.p, sizeof(uint32_t) * ld, C, sizeof(uint32_t) * n, sizeof(uint32_t) * n, n,
                             hipMemcpyDeviceToDevice, s));
    RNS_HIP(hipMemsetAsync(R0.p, 0, sizeof(int64_t) * t * ld, s));
    RNS_HIP(hipMemcpy2DAsync(R0.p, sizeof(int64_t) * ld, R, sizeof(int64_t) * n, sizeof(int64_t) * n, t,
                             hipMemcpyDeviceToDevice, s));
    const int64_t cnt = (int64_t)t * ld;
    hipLaunchKernelGGL(k_floor_mod, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, R0.p, cnt, p, Rm0.p);
    RNS_HIP(hipGetLastError());
    RNS_HIP(hipMemsetAsync(err.p, 0, sizeof(int32_t), s));
    RNS_HIP(hipMemsetAsync(base.p, 0, sizeof(int64_t), s));
    // A as int16 when every |a| < 32640, else int32 (the driver's rule).
    RNS_HIP(hipMemsetAsync(wide.p, 0, sizeof(int32_t), s));
    launch_range16(A, n * n, wide.p, s);
    RNS_HIP(hipGetLastError());
    int32_t w = 0;
    RNS_HIP(hipMemcpyAsync(&w, wide.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    RNS_HIP(hipStreamSynchronize(s));
    const int a_bytes = w ? 4 : 2;
    void *Adev = nullptr;
    if (a_bytes == 2) {
        RNS_HIP(A16.alloc((size_t)n * ld));
        Adev = A16.p;
    } else {
        RNS_HIP(A32.alloc((size_t)n * ld));
        Adev = A32.p;
    }
    launch_pack_rows(A, n, ld, a_bytes, Adev, s);
    RNS_HIP(hipGetLastError());
    LiftBufs lb{R0.p, R1.p, Rm0.p, Rm1.p, Xh.p, err.p, base.p};
    int used = 0;
    if (form == 1) {
        RNS_HIP(Ct.alloc(lift_tile_c_bytes(n)));
        launch_lift_tile_c(Cp.p, n, ld, p, Ct.p, s);
        RNS_HIP(hipGetLastError());
        lb.Ct = Ct.p;
        used |= 1;
        if (a_bytes == 2) {
            RNS_HIP(At.alloc(lift_tile_a_bytes(n)));
            launch_lift_tile_a(A16.p, n, ld, At.p, s);
            RNS_HIP(hipGetLastError());
            RNS_HIP(Xd.alloc(lift_frag_bytes(n)));
            RNS_HIP(Rmd.alloc(lift_frag_bytes(n)));
            launch_lift_frag(Rm0.p, n, ld, t, p, Rmd.p, s);
            RNS_HIP(hipGetLastError());
            lb.At = At.p;
            lb.Xd = Xd.p;
            lb.Rmd = Rmd.p;
            used |= 2 | (lift_packed(t) ? 4 : 0);
        }
    }
    launch_lift_steps(Cp.p, Adev, a_bytes, n, ld, t, p, lb, 1, s);
    RNS_HIP(hipGetLastError());
    RNS_HIP(hipMemcpy2DAsync(X, sizeof(uint32_t) * n, Xh.p, sizeof(uint32_t) * ld, sizeof(uint32_t) * n, t,
                             hipMemcpyDeviceToDevice, s));
    RNS_HIP(hipMemcpy2DAsync(R_next, sizeof(int64_t) * n, R1.p, sizeof(int64_t) * ld, sizeof(int64_t) * n, t,
                             hipMemcpyDeviceToDevice, s));
    RNS_HIP(hipMemcpy2DAsync(Rm_next, sizeof(uint32_t) * n, Rm1.p, sizeof(uint32_t) * ld, sizeof(uint32_t) * n,
                             t, hipMemcpyDeviceToDevice, s));
    int32_t e = 0;
    RNS_HIP(hipMemcpyAsync(&e, err.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    RNS_HIP(hipStreamSynchronize(s));
    *inexact = e ? 1 : 0;
    *kernels = used | (a_bytes == 2 ? 8 : 0);
    return RNS_OK;
}
