// Internal declarations shared by the HIP translation units of librns.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/rns.h"

namespace rns {

constexpr uint32_t kPrimeLimit = 1u << 26;   // every basis prime is below 2^26
constexpr int kMaxPrimes = 4096;
constexpr int kCrtMaxL = 64;                 // primes per CRT call
constexpr int kCrtMaxW = 32;                 // output words per CRT entry
constexpr int64_t kInt8MaxK = 43690;         // int32 digit sums stay exact below
constexpr int kDescRing = 16;                // problem-table slots of modmatmul_batched

// Per-prime constants, read by every kernel (Section 3.1: precomputed once
// per basis).  All doubles hold exact integers except pinv.
struct PrimeConst {
    double pf;        // p
    double pinv;      // 1/p rounded to nearest
    double c21;       // 2^21 mod p
    double c42;       // 2^42 mod p
    double w[7];      // 2^(8s) mod p in the balanced range (-p/2, p/2), s = 0..6
    uint32_t p;
    uint32_t half;    // (p-1)/2: residues above it are negative in balanced form
};

// Pointers read from job or problem tables are generic (flat) to the
// compiler; these casts state that they point to global memory, so that
// uniform reads become scalar loads and the others global (not flat) loads.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T *gptr(const T *p) {
    return (const __attribute__((address_space(1))) T *)p;
}
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T *gptr_w(T *p) {
    return (__attribute__((address_space(1))) T *)p;
}
// Tables that no kernel writes while it reads them (prime constants, CRT
// weights): the constant address space lets uniform loads use the scalar path.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(4))) T *cptr(const T *p) {
    return (const __attribute__((address_space(4))) T *)p;
}

// Garner band: for a prime index j and a distance d in [1, kCrtMaxL),
// garner[j*kCrtMaxL + d] = p_{j-d}^{-1} mod p_j (as a double), 0 where j < d.

// Constants of the Lagrange form of the CRT for one primes range and output
// width, built on first use and kept in the context.
struct LagrangeTable {
    double *d_c = nullptr;          // L: (M/p_j)^{-1} mod p_j
    uint64_t *d_mj = nullptr;       // L x W: (M/p_j) mod 2^(64W)
    uint64_t *d_m = nullptr;        // W: M mod 2^(64W)
    std::vector<uint32_t> M;        // M as 32-bit limbs (host)
};

// Constant operand of a digits x table product on the matrix cores (CRT,
// multiword reduction, base conversion) and its per-prime constants; built on
// first use per primes range and kept in the context.
struct DigitTable {
    void *d_frag = nullptr;        // table fragments in the MFMA operand layout
    double *d_c = nullptr;         // (M/p_j)^-1 mod p_j of the source range
    uint32_t *d_mlimbs = nullptr;  // CRT: M in 32-bit limbs
    uint32_t *d_half = nullptr;    // CRT: (M-1)/2 in 32-bit limbs
    double *d_mq = nullptr;        // conversion: M mod q_i (balanced)
    int nks = 0, nqb = 0, q = 0, groups = 0;
    void release();
};

}  // namespace rns

struct rns_ctx {
    int device = 0;
    int L = 0;
    std::vector<uint32_t> primes;
    rns::PrimeConst *d_prime = nullptr;
    double *d_garner = nullptr;
    uint32_t *d_mr_half = nullptr;     // mixed-radix digits of (M_r-1)/2 per range, built lazily
    int32_t *d_status = nullptr;
    void *d_work = nullptr;
    size_t work_bytes = 0;
    // Problem tables of modmatmul_batched: a ring of kDescRing slots of
    // desc_bytes each (pinned host staging and device copy); a slot is reused
    // once the event recorded after its call's kernels has completed.
    void *d_desc = nullptr;
    size_t desc_bytes = 0;
    void *h_desc = nullptr;
    hipEvent_t desc_ev[16] = {};
    int desc_next = 0;
    std::map<std::tuple<int, int, int>, rns::LagrangeTable> lagrange;
    std::map<std::pair<int, int>, uint32_t *> mr_half;  // (begin, L) -> digits
    std::map<std::tuple<int, int, int, int, int>, rns::DigitTable> digit_tables;
    int force_cert_failures = 0;
    int smith_path = 0;               // 0 auto, 1 residues of s A^-1, 2 p-adic lifting
    bool lift_vector_only = false;    // lifting products on the vector units only (RNS_LIFT_VECTOR)
    bool crt_garner = false;          // exact CRT by the mixed-radix kernel (RNS_CRT_GARNER)
    bool separate_crt = false;        // plans never fuse the CRT into the GEMM (RNS_CTX_SEPARATE_CRT)
    int crt_form = 1;                 // exact CRT: 1 the matrix cores (k_crt_mfma), 0 Lagrange on 32-bit limbs
                                      // (k_crt_exact, RNS_CRT_FORM=limbs), 2 Garner (RNS_CRT_FORM=garner)
    int massager_r0 = 4;              // invariants taken by the first massager batch (RNS_MASSAGER_R0)
    rns_ctx *aux = nullptr;            // wide-basis context of the Smith-form driver
    // Smith-form solves on this context run on one stream, created by the
    // first, and return their device blocks of up to 64 MiB to a pool (at
    // most 512 MiB kept) that later solves allocate from.
    hipStream_t solve_stream = nullptr;
    std::multimap<size_t, void *> solve_pool;
    size_t solve_pool_bytes = 0;
    int int8_kernel = -1;              // forced INT8 GEMM variant (RNS_INT8_KERNEL), -1 = tuned
    uint64_t flags = 0;                // creation flags (RNS_CTX_PATH_*)
    int auto_path = 0;                 // what RNS_PATH_AUTO resolves to: 0 library choice, else a path
    int num_cus = 256;
    unsigned *d_counter = nullptr;     // work counter of persistent launches of modmatmul_batched
    std::map<std::string, int> tune;   // autotuned INT8 variant per shape class
    std::string tune_path;
    std::mutex mu;
    // tracing: (kernel name, start event, stop event) per launch
    bool prof = false;
    rns_ctx *prof_sink = nullptr;      // records go here instead (the driver's basis -> its owner)
    struct ProfRec {
        const char *name;
        hipEvent_t a, b;
        int64_t launches;              // kernel launches between the two events
    };
    std::vector<ProfRec> prof_recs;
    std::mutex prof_mu;
};

namespace rns {

// HIP error handling: every HIP call in the library goes through this.
#define RNS_HIP(call)                                                    \
    do {                                                                 \
        hipError_t e_ = (call);                                          \
        if (e_ != hipSuccess) return e_ == hipErrorOutOfMemory ? RNS_ENOMEM : RNS_EDEVICE; \
    } while (0)

int ensure_workspace(rns_ctx *ctx, size_t bytes);
// Address of the allocation-free entry point's static scratch on `device`
// (the device must be current); called once per device at context creation.
int scratch_init(int device);
int ensure_desc(rns_ctx *ctx, size_t bytes);

// Small host-side multiword unsigned integers (32-bit limbs, little-endian).
using Limbs = std::vector<uint32_t>;
void limbs_mul_small(Limbs &a, uint32_t m);
uint32_t limbs_divmod_small(Limbs &a, uint32_t d);     // a /= d, returns a mod d
uint32_t limbs_mod_small(const Limbs &a, uint32_t d);
int limbs_cmp(const Limbs &a, const Limbs &b);
void limbs_trim(Limbs &a);
uint64_t mulmod_u64(uint64_t a, uint64_t b, uint64_t m);
uint64_t powmod_u64(uint64_t a, uint64_t e, uint64_t m);
uint64_t invmod_u64(uint64_t a, uint64_t m);            // m prime

// Tracing helpers: bracket one kernel launch (or `launches` launches in a
// row) with events when the context traces; a null context traces nothing.
struct ProfScope {
    rns_ctx *ctx;
    const char *name;
    hipStream_t s;
    int64_t launches;
    hipEvent_t a = nullptr;
    ProfScope(rns_ctx *c, const char *n, hipStream_t st, int64_t launches = 1);
    ~ProfScope();
};
// The tracing context of the Smith-form solve running on this thread (null
// when none traces): the driver's own kernel launchers record into it.
extern thread_local rns_ctx *tl_trace;

int lagrange_table(rns_ctx *ctx, int begin, int L, int W, const LagrangeTable **out, hipStream_t s);

// A gemm plan whose operands are int64 matrices (row-major A m x k, B k x n,
// one per descriptor; the descriptors' A and B residue pointers are unused):
// its conversion kernel reduces them mod every prime of the problem straight
// into the tiled operand layouts.
struct GemmInt64Src {
    const int64_t *A;
    int64_t lda;
    const int64_t *B;
    int64_t ldb;
    // Optional int64 result (row stride ldc): when every problem of a plan has
    // one, at most two primes and the INT8 path, the GEMM launch also does the
    // CRT and writes C here (no residue planes of C).
    int64_t *C;
    int64_t ldc;
};
int gemm_plan_create_int64(rns_ctx *ctx, const rns_gemm_desc *descs, const GemmInt64Src *src, int count,
                           int path, rns_gemm_plan **out);
// Whether a plan from gemm_plan_create_int64 writes int64 results itself.
bool gemm_plan_fused_crt(const rns_gemm_plan *p);
int mixed_radix_half(rns_ctx *ctx, int begin, int L, const uint32_t **out, hipStream_t s);

}  // namespace rns
