// Smith normal form driver (Section 1 defines S; Section 2.2 describes the
// three phases this driver follows in reduced form).
//
// Phase 1 (largest invariant factor).  For two random right-hand sides b the
//   solution x = A^-1 b has a denominator dividing s_n; x is rebuilt from its
//   residues x mod q = (A^-1 mod q) b for a growing set of primes (A^-1 mod q by
//   Gauss-Jordan on the GPU, all primes at once; the products by
//   modmatmul_batched; the residues combined by crt_reconstruct) and then by
//   rational reconstruction on the host.  s = lcm of the two denominators.
// Phase 2 (the massaged matrix with J = I).  X = s A^-1 is rebuilt the same
//   way (residue planes scaled by s mod q, crt_reconstruct); A X = s I is then
//   checked exactly with modmatmul_batched on fresh primes.  Success proves
//   that X is integral, hence s_n | s.  The Smith form of X over Z/sZ is
//   diag(s/s_n, ..., s/s_1) (read with gcd(0, s) = s), so
//   s_{n+1-i} = s / g_i for its diagonal g_1 | ... | g_n.  When s factors into
//   small prime powers the diagonal comes from one elimination per prime power
//   on the GPU (minimal-valuation pivoting over Z/q^e); otherwise from gcd
//   elimination modulo s on the host.
// Phase 3 (certification).  With J = I and the exact check of A X = s I the
//   result is certified; a failed check (s too small, or too few primes for X)
//   adds primes or restarts Phase 1 with new right-hand sides (Las Vegas).
//
// p-adic lifting path, for matrices with small entries whose invariants are
// too large to rebuild s A^-1 from residues (Section 3 names Dixon's lifting
// as the solver of the integrality certification; Section 3.2 notes that its
// set-up, A^-1 mod p, costs about as much as the lifting, which is why C stays
// resident here across right-hand sides and restarts).
//   Lifting.  C = A^-1 mod p once (GPU Gauss-Jordan); for a random n x t
//     matrix J the GPU runs X_i = C R_i mod p, R_{i+1} = (R_i - A X_i) / p, so
//     that Y = A^-1 J = sum_i X_i p^i, keeping every digit X_i; the digits are
//     projected on the device by a random (t+2) x n matrix R (Z_i = R X_i) and
//     only Z_i comes to the host, where Y' = R Y mod p^K is accumulated.
//   Phase 1.  Rational reconstruction of two random combinations of Y' gives
//     denominators whose lcm s divides s_n and, with high probability, equals
//     it.  Lifting stops at the first checkpoint (32, 64, ... steps) whose s and
//     X' agree with the previous one, or at the step count that Hadamard's
//     bound guarantees.
//   Phase 2.  X' = s Y' (mod p^K, symmetric) is the integer matrix s R A^-1 J;
//     an entry that is not small shows that s misses a factor, and that
//     entry's own denominator joins s.  The Smith form of X' over Z/sZ gives
//     g_1 | ... | g_t, and s_{n+1-i} = s / g_i; while fewer than two of these
//     are 1, t doubles (up to 16) and the lifting runs again with the same C.
//   Phase 3.  prod s_i = |det A| is checked with det A / s rebuilt from
//     det A mod primes (forward elimination on the GPU, many primes at once);
//     |det A / s| <= H / s for Hadamard's bound H, so enough primes make the
//     check exact.  A failed check restarts with new random J and R.
#include "bigint.hpp"
#include "massager_host.hpp"
#include "smith_internal.hpp"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <ctime>
#include <functional>
#include <memory>
#include <new>
#include <thread>
#include <type_traits>
#include <vector>

using namespace rns;

struct rns_smith_result {
    std::vector<std::vector<uint64_t>> s;
    rns_smith_stats st{};
    // The Smith massager, when computed: row i of U and columns j of M and T,
    // each n entries of wU[i] (wM[j], wT[j]) little-endian words.
    bool massager = false;
    std::vector<std::vector<uint64_t>> U, M, T;
    std::vector<int> wU, wM, wT;
};

namespace {

constexpr int kAuxPrimes = 2048;    // basis of the driver's internal context
constexpr int kDetPanel = 512;      // columns per Schur-complement update of the determinant elimination
constexpr int kChunk = 16;          // primes added per round
constexpr int kMaxSolvePrimes = 64; // primes of one GPU CRT call
constexpr int kMaxRestarts = 4;
// Lifting path certificate: det A mod primes in chunks whose residue planes
// take at most this many bytes (and at most 64 primes).
constexpr double kCertChunkBytes = 16.0 * (1ull << 30);

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct SplitMix {
    uint64_t x;
    uint64_t next() {
        uint64_t z = (x += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
};

// f(i) for i = 0..count-1 on up to 16 host threads (independent big-integer
// work items of the lifting path).
// CPU seconds used so far by the calling thread.
double thread_cpu_s() {
    timespec ts{};
    clock_gettime(CLOCK_THREAD_CPUTIME_ID, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

// CPU seconds of the helper threads of the solve running on this thread
// (added by parallel_for; null when no solve accounts for them).
thread_local double *tl_helper_cpu = nullptr;

template <typename F>
void parallel_for(int count, F f) {
    const int hw = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    const int nt = std::min(count, hw);
    if (nt <= 1) {
        for (int i = 0; i < count; ++i) f(i);
        return;
    }
    std::atomic<int> next{0};
    std::vector<std::thread> th;
    std::vector<double> cpu((size_t)nt, 0.0);
    for (int t = 0; t < nt; ++t)
        th.emplace_back([&, t] {
            for (int i = next++; i < count; i = next++) f(i);
            cpu[(size_t)t] = thread_cpu_s();             // a fresh thread: its whole CPU time
        });
    for (auto &x : th) x.join();
    if (tl_helper_cpu)
        for (double c : cpu) *tl_helper_cpu += c;
}

// parallel_for when the items are large enough to repay starting threads,
// else the same items in order on the calling thread.
template <typename F>
void parallel_for_if(bool par, int count, F f) {
    if (par) parallel_for(count, f);
    else for (int i = 0; i < count; ++i) f(i);
}

#define DRV_HIP(call)                                                             \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess) return e_ == hipErrorOutOfMemory ? RNS_ENOMEM : RNS_EDEVICE; \
    } while (0)
#define DRV_ST(call)                     \
    do {                                 \
        int s_ = (call);                 \
        if (s_ != RNS_OK) return s_;     \
    } while (0)

// A captured run of lifting steps; destroyed with the run.
constexpr int kLiftGraphSteps = 16;
struct StepGraph {
    bool tried = false;
    hipGraph_t g = nullptr;
    hipGraphExec_t exec = nullptr;
    ~StepGraph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (g) (void)hipGraphDestroy(g);
    }
};

// The context of the Smith-form solve running on this thread (set for the
// duration of a solve): device buffers come from its pool and go back to it.
thread_local rns_ctx *t_solve_ctx = nullptr;

struct SolveScope {
    rns_ctx *prev;
    explicit SolveScope(rns_ctx *c) : prev(t_solve_ctx) { t_solve_ctx = c; }
    ~SolveScope() { t_solve_ctx = prev; }
};

// For the duration of a solve on this thread: the driver's kernel launches
// (and the products it runs on its internal basis) are traced into ctx when
// ctx traces, and the CPU time of the thread and of its helper threads is
// accounted.
struct TraceScope {
    rns_ctx *prev_trace;
    double *prev_cpu;
    double helper = 0.0, t0;
    TraceScope(rns_ctx *ctx, rns_ctx *aux) : prev_trace(tl_trace), prev_cpu(tl_helper_cpu), t0(thread_cpu_s()) {
        tl_trace = ctx->prof ? ctx : nullptr;
        if (aux) {
            aux->prof = ctx->prof;
            aux->prof_sink = ctx;
        }
        tl_helper_cpu = &helper;
    }
    double cpu_s() const { return thread_cpu_s() - t0 + helper; }
    ~TraceScope() {
        tl_trace = prev_trace;
        tl_helper_cpu = prev_cpu;
    }
};

constexpr size_t kPoolMaxBlock = size_t(64) << 20, kPoolMaxBytes = size_t(512) << 20;

// A device block of at least `bytes` (its size in `got`): the smallest pooled
// block that is not more than twice as large, else a new allocation.
void *pool_get(size_t bytes, size_t &got) {
    rns_ctx *c = t_solve_ctx;
    if (c && bytes <= kPoolMaxBlock) {
        auto it = c->solve_pool.lower_bound(bytes);
        if (it != c->solve_pool.end() && it->first <= 2 * bytes) {
            got = it->first;
            void *q = it->second;
            c->solve_pool_bytes -= it->first;
            c->solve_pool.erase(it);
            return q;
        }
    }
    bytes = (std::max<size_t>(bytes, 1) + 255) / 256 * 256;
    void *q = nullptr;
    if (hipMalloc(&q, bytes) != hipSuccess) return nullptr;
    got = bytes;
    return q;
}

// Returns a block: to the pool once the solve stream has finished with it
// (the synchronisation hipFree would do), or to the device when the pool is
// full, the block is large, or no solve is running.
void pool_put(void *q, size_t bytes) {
    rns_ctx *c = t_solve_ctx;
    if (c && c->solve_stream && bytes <= kPoolMaxBlock && c->solve_pool_bytes + bytes <= kPoolMaxBytes &&
        hipStreamSynchronize(c->solve_stream) == hipSuccess) {
        c->solve_pool.emplace(bytes, q);
        c->solve_pool_bytes += bytes;
        return;
    }
    (void)hipFree(q);
}

template <typename T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;               // elements asked for
    size_t bytes = 0;           // size of the block held
    ~DevBuf() {
        if (p) pool_put(p, bytes);
    }
    int alloc(size_t count) {
        if (count <= n) return RNS_OK;
        if (p) pool_put(p, bytes);
        p = nullptr;
        n = 0;
        bytes = 0;
        size_t got = 0;
        void *q = pool_get(std::max<size_t>(count, 1) * sizeof(T), got);
        if (!q) return RNS_ENOMEM;
        p = static_cast<T *>(q);
        n = count;
        bytes = got;
        return RNS_OK;
    }
};

// The stream of the context's solves (created by the first).
int solve_stream(rns_ctx *ctx, hipStream_t *s) {
    // Non-blocking: no implicit synchronisation with the null stream, so a
    // solve never waits for (or breaks the graph capture of) another thread.
    if (!ctx->solve_stream) RNS_HIP(hipStreamCreateWithFlags(&ctx->solve_stream, hipStreamNonBlocking));
    *s = ctx->solve_stream;
    return RNS_OK;
}

// Rational reconstruction with the coprimality check: y mod m -> num / den
// (BigInt::rat_recon gives the bounds; Lehmer's method).
bool rational_reconstruct(const BigInt &y, const BigInt &m, BigInt &num, BigInt &den) {
    if (!BigInt::rat_recon(y, m, num, den)) return false;
    return BigInt::gcd(num, den).is_one() || num.is_zero();
}

// Smith diagonal modulo s of an n x n matrix (entries reduced mod s), by
// unimodular gcd row/column operations; returns g_i = gcd(d_i, s) in
// divisibility order.  Host code for small n; the entries of one operation
// are updated in parallel when s is large.
std::vector<BigInt> snf_mod_host(std::vector<BigInt> M, int64_t n, const BigInt &s) {
    auto at = [&](int64_t i, int64_t j) -> BigInt & { return M[i * n + j]; };
    const ModReducer red(s);
    const bool par = s.bit_length() > 20000;
    auto each = [&](int64_t lo, int64_t hi, const std::function<void(int64_t)> &f) {
        if (par) parallel_for((int)(hi - lo), [&](int q) { f(lo + q); });
        else for (int64_t q = lo; q < hi; ++q) f(q);
    };
    auto op = [&](const BigInt &a, const BigInt &b, BigInt &g, BigInt &x, BigInt &y) {
        if (!a.is_zero() && mod(b, BigInt::abs(a)).is_zero()) {
            g = a;
            x = BigInt(1);
            y = BigInt(0);
        } else {
            g = BigInt::xgcd(a, b, x, y);
        }
    };
    // An operation whose pivot divides the entry (x = 1, y = 0) leaves row
    // (column) k as it is, so a run of them is independent: they are queued
    // and applied together, on host threads when the run is large, before
    // the next operation that changes row (column) k.
    std::vector<int64_t> queued;
    auto run_queued = [&](int64_t k, bool rows, std::atomic<bool> *dirty) {
        if (queued.empty()) return;
        const BigInt a = at(k, k);
        // One queued operation; its entries on host threads when s is large.
        auto one = [&](int64_t l, bool entries_par) {
            const BigInt f = rows ? at(l, k) / a : at(k, l) / a;
            auto entry = [&](int64_t q) {
                if (rows) {
                    at(l, q) = red.reduce(at(l, q) - f * at(k, q));
                } else {
                    at(q, l) = red.reduce(at(q, l) - f * at(q, k));
                    if (q > k && !at(q, k).is_zero()) *dirty = true;
                }
            };
            if (entries_par) each(k, n, entry);
            else for (int64_t q = k; q < n; ++q) entry(q);
        };
        if (par)
            for (const int64_t l : queued) one(l, true);
        else if (queued.size() >= 4 && (int64_t)queued.size() * (n - k) >= 256)
            parallel_for((int)queued.size(), [&](int q) { one(queued[(size_t)q], false); });
        else
            for (const int64_t l : queued) one(l, false);
        queued.clear();
    };
    auto divides = [](const BigInt &a, const BigInt &b) { return !a.is_zero() && mod(b, BigInt::abs(a)).is_zero(); };
    for (int64_t k = 0; k < n; ++k) {
        for (;;) {
            for (int64_t i = k + 1; i < n; ++i) {
                if (at(i, k).is_zero()) continue;
                if (divides(at(k, k), at(i, k))) {
                    queued.push_back(i);
                    continue;
                }
                run_queued(k, true, nullptr);
                BigInt g, x, y;
                const BigInt a = at(k, k), b = at(i, k);
                op(a, b, g, x, y);
                const BigInt ag = a / g, bg = b / g;
                each(k, n, [&](int64_t j) {
                    const BigInt u = at(k, j), v = at(i, j);
                    at(k, j) = red.reduce(x * u + y * v);
                    at(i, j) = red.reduce(ag * v - bg * u);
                });
            }
            run_queued(k, true, nullptr);
            std::atomic<bool> dirty{false};
            for (int64_t j = k + 1; j < n; ++j) {
                if (at(k, j).is_zero()) continue;
                if (divides(at(k, k), at(k, j))) {
                    queued.push_back(j);
                    continue;
                }
                run_queued(k, false, &dirty);
                BigInt g, x, y;
                const BigInt a = at(k, k), b = at(k, j);
                op(a, b, g, x, y);
                const BigInt ag = a / g, bg = b / g;
                each(k, n, [&](int64_t i) {
                    const BigInt u = at(i, k), v = at(i, j);
                    at(i, k) = red.reduce(x * u + y * v);
                    at(i, j) = red.reduce(ag * v - bg * u);
                    if (i > k && !at(i, k).is_zero()) dirty = true;
                });
            }
            run_queued(k, false, &dirty);
            if (!dirty) break;
        }
    }
    std::vector<BigInt> g(n);
    for (int64_t i = 0; i < n; ++i) g[i] = BigInt::gcd(at(i, i), s);   // gcd(0, s) = s
    for (int64_t i = 0; i < n; ++i)                                       // diag(a,b) ~ diag(gcd,lcm)
        for (int64_t j = i + 1; j < n; ++j) {
            const BigInt h = BigInt::gcd(g[i], g[j]);
            const BigInt l = (g[i] / h) * g[j];
            g[i] = h;
            g[j] = l;
        }
    return g;
}

struct Driver {
    rns_ctx *ctx = nullptr;     // the caller's context (stats, test hooks)
    rns_ctx *aux = nullptr;     // internal basis of kAuxPrimes primes
    int64_t n = 0;
    const int64_t *A = nullptr; // host
    uint64_t seed = 0;
    hipStream_t stream = nullptr;
    rns_smith_stats st{};
    double abits = 0;           // log2 of Hadamard's bound on |det A|
    double amax = 0;            // max |a_ij|

    DevBuf<int64_t> dA;
    DevBuf<uint32_t> dM;        // [P][n][2n] Gauss-Jordan workspace; right halves = A^-1 mod q
    DevBuf<GjPrime> dpr;
    DevBuf<int32_t> dsing;
    DevBuf<uint32_t> dtmp;
    DevBuf<uint64_t> dX;        // s A^-1, W words per entry
    DevBuf<int64_t> dB;         // right-hand sides
    DevBuf<uint32_t> dBres, dXres, dAres, dProd;
    DevBuf<uint32_t> dc;
    DevBuf<unsigned> dcount;
    DevBuf<int32_t> dstatus;
    int P = 0;                  // primes with inverses in dM
    int base = 0;               // first aux prime used for inverses
    int Wx = 1;

    ~Driver() {
        // The stream belongs to the context; the buffers (destroyed after
        // this) wait for it before they return to the pool.
    }

    GjPrime gjp(int idx, int W) const {
        GjPrime g;
        g.p = aux->primes[idx];
        g.pf = (double)g.p;
        g.pinv = 1.0 / g.pf;
        g.pow64w = (double)powmod_u64(2, 64ull * W, g.p);
        return g;
    }

    int sync() {
        DRV_HIP(hipStreamSynchronize(stream));
        return RNS_OK;
    }

    DevBuf<uint32_t> dS, dW;    // blocked elimination: panel copies, pivot-block inverses
    DevBuf<int32_t> dpiv, dneed;

    // Eliminates the P planes of M ([P][n][ld], residues mod the aux primes
    // pbeg .. pbeg+P-1, prime table dpr): Gauss-Jordan when ld = 2n (the right
    // halves become A^-1 mod p), forward elimination when ld = n (det only).
    // Blocks of kGjBlock columns: panel, swaps and pivot-block inverse on the
    // GPU (launch_gj_block), then two residue products per block through
    // modmatmul_batched: pivot rows <- P11^-1 (pivot rows), and every other
    // row (rows below only for ld = n) minus its panel times the pivot rows.
    // Both products read their operands from the tiled workspace, which the
    // product's own conversion kernel fills before the product writes C, so
    // the update in place is safe.
    // Forward elimination for the determinant (ld = n) in panels of
    // kDetPanel columns, so that the Schur complement is updated once per
    // panel with one residue product of depth kDetPanel instead of once per
    // 128 columns:
    //   A. inside the panel, 128 columns at a time: the pivot block's inverse
    //      W_j (row exchanges across whole rows where needed), its rows
    //      normalised and the rows below updated, panel columns only;
    //   B. the panel's rows outside the panel: the same steps j in order
    //      (rows of block j := W_j rows, later panel rows -= multipliers x them);
    //   C. rows below the panel, columns beyond it: -= (their panel columns,
    //      the multipliers of every step) x (the panel rows from B).
    // C is the sum of the per-block updates of the 128-column form, so the
    // result, and det, are the same.
    int eliminate_det(uint32_t *M, int P, int pbeg, uint32_t *det) {
        const int64_t ld = n;
        constexpr int kSub = kDetPanel / kGjBlock;
        DRV_ST(dS.alloc((size_t)P * n * kGjBlock));
        DRV_ST(dpiv.alloc((size_t)P * kGjBlock));
        DRV_ST(dW.alloc((size_t)P * kSub * kGjBlock * kGjBlock));
        DRV_ST(dneed.alloc((size_t)P));
        std::vector<int32_t> need(P);
        const int64_t ps = n * ld;
        const int64_t wps = (int64_t)kGjBlock * kGjBlock;
        auto prod = [&](rns_gemm_desc *d, int cnt) -> int {
            for (int i = 0; i < cnt; ++i) {
                d[i].prime_begin = pbeg;
                d[i].L = P;
                st.residue_ops += 2.0 * d[i].m * d[i].n * d[i].k * P;
            }
            DRV_ST(modmatmul_batched(aux, d, cnt, RNS_PATH_AUTO, stream));
            st.products += 1;
            return RNS_OK;
        };
        for (int64_t P0 = 0; P0 < n; P0 += kDetPanel) {
            const int64_t pend = std::min<int64_t>(n, P0 + kDetPanel);
            int j = 0;
            for (int64_t r0 = P0; r0 < pend; r0 += kGjBlock, ++j) {      // A
                const int bw = (int)std::min<int64_t>(kGjBlock, pend - r0);
                uint32_t *Wj = dW.p + (size_t)j * P * wps;
                launch_gj_blockinv(M, n, ld, r0, bw, dpr.p, P, Wj, dsing.p, dneed.p, det, stream);
                DRV_HIP(hipGetLastError());
                DRV_HIP(hipMemcpyAsync(need.data(), dneed.p, sizeof(int32_t) * P, hipMemcpyDeviceToHost, stream));
                DRV_ST(sync());
                bool any = false;
                for (int q = 0; q < P; ++q) any |= need[q] != 0;
                if (any) {
                    launch_gj_pivoted(M, n, ld, r0, bw, dpr.p, P, dS.p, dpiv.p, dsing.p, dneed.p, det, Wj, stream);
                    DRV_HIP(hipGetLastError());
                }
                rns_gemm_desc d[2]{};
                d[0].m = bw; d[0].n = pend - r0; d[0].k = bw;
                d[0].A = Wj; d[0].lda = kGjBlock; d[0].a_plane_stride = wps;
                d[0].B = M + r0 * ld + r0; d[0].ldb = ld; d[0].b_plane_stride = ps;
                d[0].C = M + r0 * ld + r0; d[0].ldc = ld; d[0].c_plane_stride = ps;
                DRV_ST(prod(d, 1));
                const int64_t cols = pend - r0 - bw, rows = n - r0 - bw;
                if (cols > 0 && rows > 0) {
                    d[1].m = rows; d[1].n = cols; d[1].k = bw;
                    d[1].A = M + (r0 + bw) * ld + r0; d[1].lda = ld; d[1].a_plane_stride = ps;
                    d[1].B = M + r0 * ld + r0 + bw; d[1].ldb = ld; d[1].b_plane_stride = ps;
                    d[1].C = M + (r0 + bw) * ld + r0 + bw; d[1].ldc = ld; d[1].c_plane_stride = ps;
                    d[1].flags = RNS_GEMM_SUBTRACT;
                    DRV_ST(prod(d + 1, 1));
                }
            }
            const int64_t beyond = ld - pend;
            if (beyond <= 0) continue;
            j = 0;
            for (int64_t r0 = P0; r0 < pend; r0 += kGjBlock, ++j) {      // B
                const int bw = (int)std::min<int64_t>(kGjBlock, pend - r0);
                rns_gemm_desc d{};
                d.m = bw; d.n = beyond; d.k = bw;
                d.A = dW.p + (size_t)j * P * wps; d.lda = kGjBlock; d.a_plane_stride = wps;
                d.B = M + r0 * ld + pend; d.ldb = ld; d.b_plane_stride = ps;
                d.C = M + r0 * ld + pend; d.ldc = ld; d.c_plane_stride = ps;
                DRV_ST(prod(&d, 1));
                const int64_t rows = pend - r0 - bw;
                if (rows > 0) {
                    rns_gemm_desc e{};
                    e.m = rows; e.n = beyond; e.k = bw;
                    e.A = M + (r0 + bw) * ld + r0; e.lda = ld; e.a_plane_stride = ps;
                    e.B = M + r0 * ld + pend; e.ldb = ld; e.b_plane_stride = ps;
                    e.C = M + (r0 + bw) * ld + pend; e.ldc = ld; e.c_plane_stride = ps;
                    e.flags = RNS_GEMM_SUBTRACT;
                    DRV_ST(prod(&e, 1));
                }
            }
            if (n - pend > 0) {                                          // C
                rns_gemm_desc d{};
                d.m = n - pend; d.n = beyond; d.k = pend - P0;
                d.A = M + pend * ld + P0; d.lda = ld; d.a_plane_stride = ps;
                d.B = M + P0 * ld + pend; d.ldb = ld; d.b_plane_stride = ps;
                d.C = M + pend * ld + pend; d.ldc = ld; d.c_plane_stride = ps;
                d.flags = RNS_GEMM_SUBTRACT;
                DRV_ST(prod(&d, 1));
            }
        }
        return RNS_OK;
    }

    int eliminate(uint32_t *M, int64_t ld, int P, int pbeg, uint32_t *det) {
        const bool full = ld == 2 * n;
        if (!full) return eliminate_det(M, P, pbeg, det);
        DRV_ST(dS.alloc((size_t)P * n * kGjBlock));
        DRV_ST(dpiv.alloc((size_t)P * kGjBlock));
        DRV_ST(dW.alloc((size_t)P * kGjBlock * kGjBlock));
        DRV_ST(dneed.alloc((size_t)P));
        std::vector<int32_t> need(P);
        const int64_t ps = n * ld;
        for (int64_t r0 = 0; r0 < n; r0 += kGjBlock) {
            const int bw = (int)std::min<int64_t>(kGjBlock, n - r0);
            launch_gj_blockinv(M, n, ld, r0, bw, dpr.p, P, dW.p, dsing.p, dneed.p, det, stream);
            DRV_HIP(hipGetLastError());
            DRV_HIP(hipMemcpyAsync(need.data(), dneed.p, sizeof(int32_t) * P, hipMemcpyDeviceToHost, stream));
            DRV_ST(sync());
            bool any = false;
            for (int q = 0; q < P; ++q) any |= need[q] != 0;
            if (any) {                               // rows must be exchanged for some planes
                launch_gj_pivoted(M, n, ld, r0, bw, dpr.p, P, dS.p, dpiv.p, dsing.p, dneed.p, det, dW.p, stream);
                DRV_HIP(hipGetLastError());
            }
            rns_gemm_desc d{};
            d.m = bw; d.n = ld - r0; d.k = bw;
            d.A = dW.p; d.lda = kGjBlock; d.a_plane_stride = (int64_t)kGjBlock * kGjBlock;
            d.B = M + r0 * ld + r0; d.ldb = ld; d.b_plane_stride = ps;
            d.C = M + r0 * ld + r0; d.ldc = ld; d.c_plane_stride = ps;
            d.prime_begin = pbeg; d.L = P;
            DRV_ST(modmatmul_batched(aux, &d, 1, RNS_PATH_AUTO, stream));
            st.products += 1;
            st.residue_ops += 2.0 * d.m * d.n * d.k * P;
            const int64_t cols = ld - r0 - bw;
            if (cols <= 0) continue;
            rns_gemm_desc u[2]{};
            int cnt = 0;
            auto add = [&](int64_t row0, int64_t rows) {
                rns_gemm_desc &e = u[cnt++];
                e.m = rows; e.n = cols; e.k = bw;
                e.A = M + row0 * ld + r0; e.lda = ld; e.a_plane_stride = ps;
                e.B = M + r0 * ld + r0 + bw; e.ldb = ld; e.b_plane_stride = ps;
                e.C = M + row0 * ld + r0 + bw; e.ldc = ld; e.c_plane_stride = ps;
                e.prime_begin = pbeg; e.L = P;
                e.flags = RNS_GEMM_SUBTRACT;
                st.residue_ops += 2.0 * rows * cols * bw * P;
            };
            if (full && r0 > 0) add(0, r0);
            if (n - r0 - bw > 0) add(r0 + bw, n - r0 - bw);
            if (cnt) {
                DRV_ST(modmatmul_batched(aux, u, cnt, RNS_PATH_AUTO, stream));
                st.products += 1;
            }
        }
        return RNS_OK;
    }

    // A^-1 mod q for the P primes aux[base .. base+P); returns the index of a
    // singular prime through *bad (-1 if none).
    int invert(int P_, int *bad) {
        P = P_;
        const int64_t per = n * 2 * n;
        DRV_ST(dM.alloc((size_t)P * per));
        DRV_ST(dpr.alloc(P));
        DRV_ST(dsing.alloc(P));
        std::vector<GjPrime> h(P);
        for (int q = 0; q < P; ++q) h[q] = gjp(base + q, 1);
        DRV_HIP(hipMemcpyAsync(dpr.p, h.data(), sizeof(GjPrime) * P, hipMemcpyHostToDevice, stream));
        DRV_HIP(hipMemsetAsync(dsing.p, 0, sizeof(int32_t) * P, stream));
        launch_gj_load(dA.p, n, 2 * n, dM.p, dpr.p, P, stream);
        DRV_HIP(hipGetLastError());
        DRV_ST(eliminate(dM.p, 2 * n, P, base, nullptr));
        std::vector<int32_t> sing(P);
        DRV_HIP(hipMemcpyAsync(sing.data(), dsing.p, sizeof(int32_t) * P, hipMemcpyDeviceToHost, stream));
        DRV_ST(sync());
        *bad = -1;
        for (int q = 0; q < P; ++q)
            if (sing[q]) {
                *bad = q;
                break;
            }
        st.lift_steps += P;
        return RNS_OK;
    }

    // CRT of residue planes res (rows x cols, ldr, plane stride) over the P
    // inverse primes into W words per entry, on the device.
    int crt(const uint32_t *res, int64_t rows, int64_t cols, int64_t ldr, int64_t ps, int W,
            uint64_t *out) {
        DRV_ST(dstatus.alloc(1));
        DRV_HIP(hipMemsetAsync(dstatus.p, 0, sizeof(int32_t), stream));
        return crt_reconstruct(aux, res, rows, cols, ldr, ps, base, P, nullptr, 0, out, W, cols,
                               dstatus.p, stream);
    }

    int gemm(const uint32_t *Ap, int64_t lda, int64_t aps, const uint32_t *Bp, int64_t ldb, int64_t bps,
             uint32_t *Cp, int64_t ldc, int64_t cps, int64_t m, int64_t nn, int64_t k, int pb, int L) {
        rns_gemm_desc d{};
        d.m = m; d.n = nn; d.k = k;
        d.A = Ap; d.lda = lda; d.a_plane_stride = aps;
        d.B = Bp; d.ldb = ldb; d.b_plane_stride = bps;
        d.C = Cp; d.ldc = ldc; d.c_plane_stride = cps;
        d.prime_begin = pb; d.L = L;
        st.products += 1;
        st.residue_ops += 2.0 * m * nn * k * L;
        return modmatmul_batched(aux, &d, 1, RNS_PATH_AUTO, stream);
    }

    // Phase 1: denominators of A^-1 b for two random b; s = their lcm.
    // Returns RNS_EBOUND when P primes are not enough yet.
    int phase1(SplitMix &rng, BigInt &s) {
        const int c = 2;
        std::vector<int64_t> b((size_t)n * c);
        for (auto &v : b) v = (int64_t)(rng.next() % 2001) - 1000;
        DRV_ST(dB.alloc((size_t)n * c));
        DRV_HIP(hipMemcpyAsync(dB.p, b.data(), sizeof(int64_t) * n * c, hipMemcpyHostToDevice, stream));
        DRV_ST(dBres.alloc((size_t)P * n * c));
        DRV_ST(rns_reduce(aux, dB.p, n, c, c, base, P, dBres.p, c, n * c, stream));
        DRV_ST(dtmp.alloc((size_t)P * n * c));
        DRV_ST(gemm(dM.p + n, 2 * n, 2 * n * n, dBres.p, c, n * c, dtmp.p, c, n * c, n, c, n, base, P));
        const int W = (int)((P * 26 + 63) / 64) + 1;
        DevBuf<uint64_t> dx;
        DRV_ST(dx.alloc((size_t)n * c * W));
        DRV_ST(crt(dtmp.p, n, c, c, n * c, W, dx.p));
        std::vector<uint64_t> hx((size_t)n * c * W);
        DRV_HIP(hipMemcpyAsync(hx.data(), dx.p, sizeof(uint64_t) * hx.size(), hipMemcpyDeviceToHost, stream));
        DRV_ST(sync());
        BigInt M(1);
        for (int q = 0; q < P; ++q) M = M.mul_small(aux->primes[base + q]);
        BigInt lcm(1);
        const BigInt B = BigInt::isqrt(M / BigInt(2));
        for (int col = 0; col < c; ++col) {
            BigInt den(1);
            for (int64_t i = 0; i < n; ++i) {
                const BigInt y = BigInt::from_twos(&hx[((size_t)i * c + col) * W], W);
                // With the current denominator the entry may already be small.
                BigInt z = mod(y * den, M);
                if (BigInt::cmp(z.shl(1), M) > 0) z = z - M;
                if (BigInt::cmp(BigInt::abs(z), B) <= 0) continue;
                BigInt num, d2;
                if (!rational_reconstruct(z, M, num, d2)) return RNS_EBOUND;
                den = den * d2;
            }
            lcm = BigInt::lcm(lcm, den);
        }
        s = lcm;
        return RNS_OK;
    }

    // Phase 2: X = s A^-1 on the device (Wx words per entry); then the exact
    // check A X = s I on fresh primes.  RNS_EBOUND: not verified.
    int phase2_build(const BigInt &s) {
        std::vector<uint32_t> sm(P);
        for (int q = 0; q < P; ++q) sm[q] = s.mod_small(aux->primes[base + q]);
        DRV_ST(dc.alloc(P));
        DRV_HIP(hipMemcpyAsync(dc.p, sm.data(), sizeof(uint32_t) * P, hipMemcpyHostToDevice, stream));
        // scale the inverse planes in place: (A^-1 mod q) * (s mod q)
        launch_scale(dM.p + n, n, n, 2 * n, 2 * n * n, dpr.p, dc.p, P, stream);
        DRV_HIP(hipGetLastError());
        Wx = (int)((P * 26 + 63) / 64) + 1;
        DRV_ST(dX.alloc((size_t)n * n * Wx));
        DRV_ST(crt(dM.p + n, n, n, 2 * n, 2 * n * n, Wx, dX.p));
        // undo the scaling is not needed: the inverse planes are not reused
        return RNS_OK;
    }

    int phase2_check(const BigInt &s, bool *ok) {
        // |X| <= (M-1)/2 < 2^(26 P), so |A X - s I| <= n max|a| 2^(26 P) + s.
        const double bits = std::max(std::log2((double)n) + std::log2(std::max(1.0, amax)) + 26.0 * P,
                                     (double)s.bit_length()) + 2.0;
        const int K = std::min(kAuxPrimes - (base + P), (int)std::ceil(bits / 25.9) + 1);
        const int cb = base + P;                // fresh primes after the inverse primes
        if (K < 1 || cb + K > kAuxPrimes || K > kMaxSolvePrimes * 4) return RNS_ENOTSUP;
        std::vector<GjPrime> h(K);
        for (int j = 0; j < K; ++j) h[j] = gjp(cb + j, Wx);
        DevBuf<GjPrime> dck;
        DRV_ST(dck.alloc(K));
        DRV_HIP(hipMemcpyAsync(dck.p, h.data(), sizeof(GjPrime) * K, hipMemcpyHostToDevice, stream));
        DRV_ST(dXres.alloc((size_t)K * n * n));
        launch_words_mod(dX.p, n * n, Wx, dck.p, K, dXres.p, stream);
        DRV_HIP(hipGetLastError());
        DRV_ST(dAres.alloc((size_t)K * n * n));
        DRV_ST(rns_reduce(aux, dA.p, n, n, n, cb, K, dAres.p, n, n * n, stream));
        DRV_ST(dProd.alloc((size_t)K * n * n));
        DRV_ST(gemm(dAres.p, n, n * n, dXres.p, n, n * n, dProd.p, n, n * n, n, n, n, cb, K));
        std::vector<uint32_t> sm(K);
        for (int j = 0; j < K; ++j) sm[j] = s.mod_small(aux->primes[cb + j]);
        DRV_ST(dc.alloc(std::max(P, K)));
        DRV_HIP(hipMemcpyAsync(dc.p, sm.data(), sizeof(uint32_t) * K, hipMemcpyHostToDevice, stream));
        DRV_ST(dcount.alloc(1));
        DRV_HIP(hipMemsetAsync(dcount.p, 0, sizeof(unsigned), stream));
        launch_check_sI(dProd.p, n, dc.p, K, dcount.p, stream);
        DRV_HIP(hipGetLastError());
        unsigned mism = 0;
        DRV_HIP(hipMemcpyAsync(&mism, dcount.p, sizeof(unsigned), hipMemcpyDeviceToHost, stream));
        DRV_ST(sync());
        st.cert_primes = K;
        *ok = mism == 0;
        return RNS_OK;
    }

    // Smith diagonal of X mod s: g_1 | ... | g_n.
    int snf(const BigInt &s, std::vector<BigInt> &g) {
        // Factor s over the primes below 2^16.
        std::vector<std::pair<uint32_t, int>> fac;
        BigInt rest = s;
        // The local Smith forms on the GPU need the factors of s, all below
        // 2^16; whether s has only such factors is one gcd with their
        // product, so trial division runs only when its result is used.
        const bool smooth = n > 24 && smooth16(s);
        // Two primes per pass over rest: one remainder modulo their product
        // (below 2^32), then each prime's own test.
        const std::vector<uint32_t> &P = small_primes();
        for (size_t i = 0; smooth && i < P.size() && !rest.is_one(); i += 2) {
            const uint32_t q1 = P[i], q2 = i + 1 < P.size() ? P[i + 1] : 1u;
            const uint32_t r = rest.mod_small(q1 * q2);
            for (const uint32_t q : {q1, q2}) {
                if (q == 1 || r % q != 0) continue;
                int e = 0;
                while (rest.mod_small(q) == 0) {
                    rest = rest / BigInt((int64_t)q);
                    ++e;
                }
                if (e) fac.push_back({q, e});
            }
        }
        bool gpu = smooth && rest.is_one();
        for (auto &f : fac) {
            double m = std::pow((double)f.first, f.second);
            if (m >= 17179869184.0) gpu = false;   // 2^34
        }
        g.assign(n, BigInt(1));
        if (gpu && !fac.empty()) {
            // Every prime power of s in one elimination: plane f is X mod q_f^e_f.
            const int F = (int)fac.size();
            DevBuf<uint64_t> dm, dkey;
            DevBuf<int32_t> dval;
            DevBuf<LocalMod> dlm;
            DevBuf<uint64_t> dinv;
            DRV_ST(dm.alloc((size_t)F * n * n));
            DRV_ST(dkey.alloc((size_t)F * (n + 1)));
            DRV_ST(dval.alloc((size_t)F * n));
            DRV_ST(dlm.alloc((size_t)F));
            DRV_ST(dinv.alloc((size_t)F));
            std::vector<LocalMod> lms(F);
            for (int f = 0; f < F; ++f) {
                LocalMod &lm = lms[f];
                lm.q = fac[f].first;
                lm.e = fac[f].second;
                lm.m = 1;
                for (int t = 0; t < lm.e; ++t) lm.m *= lm.q;
                lm.mf = (double)lm.m;
                lm.minv = 1.0 / lm.mf;
                lm.pow64w = powmod_u64(2, 64ull * Wx, lm.m);
                launch_words_mod_m(dX.p, n * n, Wx, lm, dm.p + (size_t)f * n * n, stream);
            }
            DRV_HIP(hipMemcpyAsync(dlm.p, lms.data(), sizeof(LocalMod) * F, hipMemcpyHostToDevice, stream));
            DRV_HIP(hipMemsetAsync(dkey.p, 0xFF, sizeof(uint64_t) * F * (n + 1), stream));
            launch_loc_init(dm.p, n, dlm.p, F, dkey.p, stream);
            for (int k = 0; k < n; ++k) launch_loc_step(dm.p, n, k, dlm.p, F, dkey.p, dval.p, dinv.p, stream);
            DRV_HIP(hipGetLastError());
            std::vector<int32_t> val((size_t)F * n);
            DRV_HIP(hipMemcpyAsync(val.data(), dval.p, sizeof(int32_t) * val.size(), hipMemcpyDeviceToHost, stream));
            DRV_ST(sync());
            for (int f = 0; f < F; ++f) {
                // Once the remainder is zero mod q^e the later steps record e.
                bool zero = false;
                for (int64_t i = 0; i < n; ++i) {
                    int v = zero ? lms[f].e : std::min(val[(size_t)f * n + i], lms[f].e);
                    if (v >= lms[f].e) zero = true;
                    for (int t = 0; t < v; ++t) g[i] = g[i].mul_small(lms[f].q);
                }
            }
        } else if (!gpu) {
            std::vector<uint64_t> hx((size_t)n * n * Wx);
            DRV_HIP(hipMemcpyAsync(hx.data(), dX.p, sizeof(uint64_t) * hx.size(), hipMemcpyDeviceToHost, stream));
            DRV_ST(sync());
            std::vector<BigInt> M((size_t)n * n);
            for (size_t e = 0; e < M.size(); ++e) M[e] = mod(BigInt::from_twos(&hx[e * Wx], Wx), s);
            g = snf_mod_host(std::move(M), n, s);
        }
        return RNS_OK;
    }

    int run(rns_smith_result *res) {
        const double t0 = now_s();
        st.path = 0;
        st.cert_exact = 1;
        SplitMix rng{seed ^ 0x5DEECE66Dull};
        int singular_primes = 0;
        base = 0;
        for (int attempt = 0; attempt <= kMaxRestarts; ++attempt) {
            if (attempt) st.restarts += 1;
            // Phase 1 and 2 share the inverses; grow the prime set until the
            // reconstruction of A^-1 b succeeds and X verifies.
            BigInt s;
            bool verified = false;
            double tl = now_s();
            for (int Pn = kChunk; Pn <= kMaxSolvePrimes; Pn += kChunk) {
                int bad = -1;
                if (base + Pn + 8 > kAuxPrimes) return RNS_ENOTSUP;
                DRV_ST(invert(Pn, &bad));
                if (bad >= 0) {
                    // A prime divides det A.  Enough such primes prove det A = 0.
                    singular_primes += 1;
                    if (singular_primes * 25.9 > abits + 1.0) return RNS_ESINGULAR;
                    base += bad + 1;
                    Pn -= kChunk;                    // retry with the same count
                    continue;
                }
                const double tp = now_s();
                int stp = phase1(rng, s);
                st.t_lif += now_s() - tl;
                tl = now_s();
                if (stp == RNS_EBOUND) continue;
                DRV_ST(stp);
                const double ti = now_s();
                DRV_ST(phase2_build(s));
                bool ok = false;
                const double tu = now_s();
                DRV_ST(phase2_check(s, &ok));
                st.t_uc += now_s() - tu;
                st.t_im += tu - ti;
                (void)tp;
                if (ok) {
                    verified = true;
                    break;
                }
            }
            if (!verified) continue;                 // new right-hand sides
            if (ctx->force_cert_failures > 0) {      // test hook: pretend the check failed
                ctx->force_cert_failures -= 1;
                continue;
            }
            const double ts = now_s();
            std::vector<BigInt> g;
            DRV_ST(snf(s, g));
            st.t_im += now_s() - ts;
            res->s.assign(n, {});
            for (int64_t i = 0; i < n; ++i) {
                // s_{n-i} = s / g_i (g ascending -> s_i descending)
                const BigInt v = s / g[i];
                res->s[n - 1 - i] = v.mag_words();
            }
            st.columns = (int)n;
            st.t_total = now_s() - t0;
            res->st = st;
            return RNS_OK;
        }
        return RNS_ERETRY;
    }

    // --------------------------------------------------- p-adic lifting --
    int64_t ldl = 0;            // padded row stride of the lifting operands (multiple of 8)
    DevBuf<int32_t> dA32;       // A as int32, [n][ldl], zero beyond column n
    DevBuf<int16_t> dA16;       // the same as int16 when every |a| < 32640 (then dA32 is unused)
    int a_bytes = 4;
    DevBuf<uint32_t> dG;        // [n][2n] Gauss-Jordan of the lifting prime; right half = C
    DevBuf<uint32_t> dC;        // C = A^-1 mod p, [n][ldl], zero beyond column n
    DevBuf<char> dCt;           // C as tiled digits for the matrix-core lifting products
    DevBuf<char> dAt;           // int16 A as tiled digits, the same
    DevBuf<char> dXd, dRmd;     // digit fragments passed between the two lifting products
    DevBuf<uint32_t> dXh;       // lifted digits [K][t][n]
    DevBuf<int64_t> dR0, dR1;   // residuals [t][n]
    DevBuf<uint32_t> dRm0, dRm1;
    DevBuf<int32_t> dRp;        // projection [tp][n]
    DevBuf<int64_t> dZ, dZb;    // projected digits of a checkpoint interval (two, for overlap)
    DevBuf<int32_t> derr;
    DevBuf<int32_t> dflag;      // A has an entry outside the int16 range
    DevBuf<int64_t> dstep;      // device-side index of the next lifting step
    DevBuf<uint32_t> ddet;

    // The lifting products run on the matrix cores (else on the vector units).
    bool mfma_lift() const { return n <= kLiftMfmaMaxN && !ctx->lift_vector_only; }

    // A as int16 (every |a| < 32640, two signed bytes) or int32 rows of stride ldl (zero padded)
    // for the lifting kernels, built on the device from the int64 A there
    // (lifting_applies keeps every |a| below 2^31).
    int upload_a32() {
        ldl = (n + 7) / 8 * 8;
        DRV_ST(dflag.alloc(1));
        DRV_HIP(hipMemsetAsync(dflag.p, 0, sizeof(int32_t), stream));
        launch_range16(dA.p, n * n, dflag.p, stream);
        DRV_HIP(hipGetLastError());
        int32_t wide = 0;
        DRV_HIP(hipMemcpyAsync(&wide, dflag.p, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
        DRV_ST(sync());
        a_bytes = wide ? 4 : 2;
        void *out = nullptr;
        if (a_bytes == 2) {
            DRV_ST(dA16.alloc((size_t)n * ldl));
            out = dA16.p;
        } else {
            DRV_ST(dA32.alloc((size_t)n * ldl));
            out = dA32.p;
        }
        launch_pack_rows(dA.p, n, ldl, a_bytes, out, stream);
        DRV_HIP(hipGetLastError());
        return RNS_OK;
    }

    // det A mod aux primes idx[0..count) by forward elimination, all at once.
    int det_mod_primes(const std::vector<int> &idx, std::vector<uint32_t> &det) {
        const int Pd = (int)idx.size();
        det.assign(Pd, 0);
        if (Pd == 0) return RNS_OK;
        DRV_ST(dM.alloc((size_t)Pd * n * n));
        DRV_ST(dpr.alloc(Pd));
        DRV_ST(dsing.alloc(Pd));
        DRV_ST(ddet.alloc(Pd));
        std::vector<GjPrime> h(Pd);
        for (int q = 0; q < Pd; ++q) h[q] = gjp(idx[q], 1);
        std::vector<uint32_t> ones(Pd, 1u);
        DRV_HIP(hipMemcpyAsync(dpr.p, h.data(), sizeof(GjPrime) * Pd, hipMemcpyHostToDevice, stream));
        DRV_HIP(hipMemcpyAsync(ddet.p, ones.data(), sizeof(uint32_t) * Pd, hipMemcpyHostToDevice, stream));
        DRV_HIP(hipMemsetAsync(dsing.p, 0, sizeof(int32_t) * Pd, stream));
        for (int q = 1; q < Pd; ++q)
            if (idx[q] != idx[0] + q) return RNS_EINVAL;   // the products need consecutive primes
        launch_gj_load(dA.p, n, n, dM.p, dpr.p, Pd, stream);
        DRV_HIP(hipGetLastError());
        DRV_ST(eliminate(dM.p, n, Pd, idx[0], ddet.p));
        std::vector<int32_t> sing(Pd);
        DRV_HIP(hipMemcpyAsync(det.data(), ddet.p, sizeof(uint32_t) * Pd, hipMemcpyDeviceToHost, stream));
        DRV_HIP(hipMemcpyAsync(sing.data(), dsing.p, sizeof(int32_t) * Pd, hipMemcpyDeviceToHost, stream));
        DRV_ST(sync());
        for (int q = 0; q < Pd; ++q)
            if (sing[q]) det[q] = 0;
        return RNS_OK;
    }

    // C = A^-1 mod p for the first aux prime from *pidx on that does not
    // divide det A; det A mod p through *detp.
    int lift_prime(int *pidx, uint32_t *detp) {
        int singular = 0;
        for (;;) {
            if (*pidx >= kAuxPrimes) return RNS_ENOTSUP;
            DRV_ST(dG.alloc((size_t)n * 2 * n));
            DRV_ST(dpr.alloc(1));
            DRV_ST(dsing.alloc(1));
            DRV_ST(ddet.alloc(1));
            const GjPrime h = gjp(*pidx, 1);
            const uint32_t one = 1u;
            DRV_HIP(hipMemcpyAsync(dpr.p, &h, sizeof(GjPrime), hipMemcpyHostToDevice, stream));
            DRV_HIP(hipMemcpyAsync(ddet.p, &one, sizeof(uint32_t), hipMemcpyHostToDevice, stream));
            DRV_HIP(hipMemsetAsync(dsing.p, 0, sizeof(int32_t), stream));
            launch_gj_load(dA.p, n, 2 * n, dG.p, dpr.p, 1, stream);
            DRV_HIP(hipGetLastError());
            DRV_ST(eliminate(dG.p, 2 * n, 1, *pidx, ddet.p));
            int32_t sing = 0;
            DRV_HIP(hipMemcpyAsync(&sing, dsing.p, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
            DRV_HIP(hipMemcpyAsync(detp, ddet.p, sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
            DRV_ST(sync());
            if (!sing) {
                DRV_ST(dC.alloc((size_t)n * ldl));
                DRV_HIP(hipMemsetAsync(dC.p, 0, sizeof(uint32_t) * n * ldl, stream));
                DRV_HIP(hipMemcpy2DAsync(dC.p, sizeof(uint32_t) * ldl, dG.p + n, sizeof(uint32_t) * 2 * n,
                                         sizeof(uint32_t) * n, n, hipMemcpyDeviceToDevice, stream));
                return RNS_OK;
            }
            // A prime divides det A.  Enough such primes prove det A = 0.
            singular += 1;
            if (singular * 25.9 > abits + 1.0) return RNS_ESINGULAR;
            *pidx += 1;
        }
    }

    // Lifts Y = A^-1 J for a random n x t J and returns s and X' = s R Y
    // ((t+2) x t, row-major) as described in the file comment.  RNS_EBOUND:
    // no consistent reconstruction within the guaranteed step count.
    int lift_solve(int pidx, int t, SplitMix &rng, BigInt &s_out, std::vector<BigInt> &Xp) {
        const int tp = t + 2;
        const uint32_t p = aux->primes[pidx];
        const double lp = std::log2((double)p);
        const double ln = std::log2((double)n);
        // Guaranteed step count: the combinations' numerators stay below
        // H n 2^30 t, their denominators below H; |s R A^-1 J| < H n^2 2^14.
        const int64_t Kmax = (int64_t)std::ceil((2.0 * abits + 4.0 * ln + 64.0) / lp) + 1;
        std::vector<int64_t> J((size_t)t * ldl, 0);
        std::vector<uint32_t> Jm((size_t)t * ldl, 0u);
        for (int c = 0; c < t; ++c)
            for (int64_t r = 0; r < n; ++r) {
                const int64_t v = (int64_t)(rng.next() % 257) - 128;
                J[(size_t)c * ldl + r] = v;
                Jm[(size_t)c * ldl + r] = (uint32_t)(v < 0 ? v + (int64_t)p : v);
            }
        std::vector<int32_t> Rp((size_t)tp * n);
        for (auto &v : Rp) v = (int32_t)(rng.next() % 257) - 128;
        std::vector<uint32_t> w1(t), w2(t);
        for (int c = 0; c < t; ++c) {
            w1[c] = 1 + (uint32_t)(rng.next() % 65535);
            w2[c] = 1 + (uint32_t)(rng.next() % 65535);
        }
        DRV_ST(dXh.alloc((size_t)Kmax * t * ldl));
        DRV_ST(dR0.alloc((size_t)t * ldl));
        DRV_ST(dR1.alloc((size_t)t * ldl));
        DRV_ST(dRm0.alloc((size_t)t * ldl));
        DRV_ST(dRm1.alloc((size_t)t * ldl));
        DRV_ST(dRp.alloc((size_t)tp * n));
        DRV_ST(derr.alloc(1));
        DRV_ST(dstep.alloc(1));
        DRV_HIP(hipMemcpyAsync(dR0.p, J.data(), sizeof(int64_t) * J.size(), hipMemcpyHostToDevice, stream));
        DRV_HIP(hipMemcpyAsync(dRm0.p, Jm.data(), sizeof(uint32_t) * Jm.size(), hipMemcpyHostToDevice, stream));
        DRV_HIP(hipMemcpyAsync(dRp.p, Rp.data(), sizeof(int32_t) * Rp.size(), hipMemcpyHostToDevice, stream));
        DRV_HIP(hipMemsetAsync(derr.p, 0, sizeof(int32_t), stream));
        DRV_HIP(hipMemsetAsync(dstep.p, 0, sizeof(int64_t), stream));
        LiftBufs lb{dR0.p, dR1.p, dRm0.p, dRm1.p, dXh.p, derr.p, dstep.p};
        if (mfma_lift()) {                               // C's digits, once per lifting
            DRV_ST(dCt.alloc(lift_tile_c_bytes(n)));
            launch_lift_tile_c(dC.p, n, ldl, p, dCt.p, stream);
            DRV_HIP(hipGetLastError());
            lb.Ct = dCt.p;
            if (a_bytes == 2) {
                DRV_ST(dAt.alloc(lift_tile_a_bytes(n)));
                launch_lift_tile_a(dA16.p, n, ldl, dAt.p, stream);
                DRV_HIP(hipGetLastError());
                lb.At = dAt.p;
                DRV_ST(dXd.alloc(lift_frag_bytes(n)));
                DRV_ST(dRmd.alloc(lift_frag_bytes(n)));
                launch_lift_frag(dRm0.p, n, ldl, t, p, dRmd.p, stream);   // the first step's Rm
                DRV_HIP(hipGetLastError());
                lb.Xd = dXd.p;
                lb.Rmd = dRmd.p;
            }
        }
        const void *Adev = a_bytes == 2 ? (const void *)dA16.p : (const void *)dA32.p;
        // Runs of kLiftGraphSteps steps replay one captured graph (the step
        // launches take the same arguments every time); the rest, and every
        // step if capture is not available, are launched directly.
        StepGraph graph;
        auto capture = [&]() {
            graph.tried = true;
            if (tl_trace) return;                        // traced launches are bracketed one run at a time
            if (hipStreamBeginCapture(stream, hipStreamCaptureModeRelaxed) != hipSuccess) return;
            launch_lift_steps(dC.p, Adev, a_bytes, n, ldl, t, p, lb, kLiftGraphSteps, stream);
            hipGraph_t gr = nullptr;
            if (hipStreamEndCapture(stream, &gr) != hipSuccess || !gr) {
                (void)hipGetLastError();
                return;
            }
            graph.g = gr;
            if (hipGraphInstantiate(&graph.exec, gr, nullptr, nullptr, 0) != hipSuccess) {
                graph.exec = nullptr;
                (void)hipGetLastError();
            }
        };
        const int ne = tp * t;
        std::vector<BigInt> Y(ne, BigInt(0));
        BigInt pw(1);                                    // p^K_done
        int64_t K_done = 0, K_chk = 32;
        bool have_prev = false;
        BigInt prev_s;
        std::vector<BigInt> prev_X;
        std::vector<int64_t> hz;
        // Steps k0 .. k1-1 and the projections of their digits into z.
        auto launch_interval = [&](int64_t k0, int64_t k1, DevBuf<int64_t> &z) -> int {
            int64_t i = k0;
            if (k1 - i >= kLiftGraphSteps && !graph.tried) capture();
            for (; graph.exec && k1 - i >= kLiftGraphSteps; i += kLiftGraphSteps)
                DRV_HIP(hipGraphLaunch(graph.exec, stream));
            if (i < k1) launch_lift_steps(dC.p, Adev, a_bytes, n, ldl, t, p, lb, (int)(k1 - i), stream);
            DRV_ST(z.alloc((size_t)(k1 - k0) * ne));
            launch_lift_proj(dXh.p, n, ldl, t, dRp.p, tp, k0, k1, z.p, stream);
            DRV_HIP(hipGetLastError());
            return RNS_OK;
        };
        // The interval after a checkpoint is launched before that checkpoint's
        // host work whenever the checkpoint cannot end the loop (a stable
        // result needs the previous checkpoint to have succeeded), so the
        // GPU lifts while the host reconstructs; otherwise it is launched
        // after.  zb[cur] holds the projections of the current interval.
        DevBuf<int64_t> *zb[2] = {&dZ, &dZb};
        int cur = 0;
        int64_t launched = K_done;                       // steps queued so far
        for (;;) {
            K_chk = std::min(K_chk, Kmax);
            if (launched < K_chk) {
                DRV_ST(launch_interval(K_done, K_chk, *zb[cur]));
                launched = K_chk;
            }
            const int64_t nb = K_chk - K_done;
            hz.resize((size_t)nb * ne);
            int32_t err = 0;
            DRV_HIP(hipMemcpyAsync(hz.data(), zb[cur]->p, sizeof(int64_t) * hz.size(), hipMemcpyDeviceToHost,
                                   stream));
            DRV_HIP(hipMemcpyAsync(&err, derr.p, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
            DRV_ST(sync());
            if (err) return RNS_EDEVICE;                 // an inexact division: C is not A^-1 mod p
            const int64_t K_next = std::min(2 * K_chk, Kmax);
            if (!have_prev && K_chk < Kmax) {
                DRV_ST(launch_interval(K_chk, K_next, *zb[cur ^ 1]));
                launched = K_next;
                cur ^= 1;
            }
            // Y' += (sum over the interval of Z_i p^(i - K_done)) p^K_done, the
            // inner sum by Horner's rule from the top digit.
            BigInt pnb(1);
            for (int64_t i = 0; i < nb; ++i) pnb = pnb.mul_small(p);
            // Host threads only once the numbers reach some thousand bits.
            const bool big = (double)K_chk * lp > 16384.0;
            parallel_for_if(big, ne, [&](int e) {
                BigInt v(0);
                for (int64_t i = nb - 1; i >= 0; --i) v = v.mul_small(p) + BigInt(hz[(size_t)i * ne + e]);
                Y[e] = Y[e] + v * pw;
            });
            pw = pw * pnb;
            K_done = K_chk;
            st.lift_steps = (int)K_done;
            // Phase 1 on two random combinations of the columns of rows 0, 1.
            bool ok = false;
            BigInt s;
            std::vector<BigInt> X(ne);
            {
                BigInt W1(0), W2(0);
                for (int c = 0; c < t; ++c) {
                    W1 = W1 + Y[c].mul_small(w1[c]);
                    W2 = W2 + Y[t + c].mul_small(w2[c]);
                }
                BigInt nu[2], de[2];
                bool rr[2] = {false, false};
                const BigInt *Wc[2] = {&W1, &W2};
                parallel_for_if(big, 2, [&](int i) { rr[i] = BigInt::rat_recon(mod(*Wc[i], pw), pw, nu[i], de[i]); });
                ok = rr[0] && rr[1] && de[0].mod_small(p) != 0 && de[1].mod_small(p) != 0;
                if (ok) s = BigInt::lcm(de[0], de[1]);
            }
            // Phase 2: X' = s Y' must be small; an entry that is not shows a
            // factor missing from s (its own denominator is then added).
            const size_t bb = (pw.bit_length() - 2) / 2;
            const BigInt Bnd = BigInt(1).shl(bb);
            std::unique_ptr<ModReducer> red_pw;
            if (ok) red_pw.reset(new ModReducer(pw));
            for (int pass = 0; ok && pass <= ne; ++pass) {
                std::vector<char> large(ne, 0);
                parallel_for_if(big, ne, [&](int e) {
                    BigInt x = red_pw->reduce(s * Y[e]);
                    if (BigInt::cmp(x.shl(1), pw) > 0) x = x - pw;
                    large[e] = BigInt::cmp(BigInt::abs(x), Bnd) >= 0;
                    X[e] = std::move(x);
                });
                int bad = -1;
                for (int e = 0; e < ne && bad < 0; ++e)
                    if (large[e]) bad = e;
                if (bad < 0) break;
                BigInt nu, de;
                if (!BigInt::rat_recon(mod(Y[bad], pw), pw, nu, de) || de.mod_small(p) == 0) {
                    ok = false;
                    break;
                }
                const BigInt s2 = BigInt::lcm(s, de);
                if (s2 == s) {
                    ok = false;
                    break;
                }
                s = s2;
            }
            if (ok) {
                const bool stable = have_prev && s == prev_s && X == prev_X;
                if (stable || K_done >= Kmax) {
                    s_out = s;
                    Xp = std::move(X);
                    return RNS_OK;
                }
                prev_s = s;
                prev_X = X;
                have_prev = true;
            } else {
                have_prev = false;
            }
            if (K_done >= Kmax) return RNS_EBOUND;
            K_chk = K_next;
        }
    }

    // prod of the extracted invariants == |det A|, with det A / s rebuilt from
    // det A mod primes.  s divides s_n, hence det A, and |det A / s| <= H / s
    // for Hadamard's bound H, so once the primes' product exceeds 2 H / s + 1
    // the reconstruction is det A / s itself: the check is exact (Las Vegas),
    // whatever the size.  prod = s * c for the candidate c = prod_{i<n} s_i;
    // a prime at which det A / s is neither c nor -c ends the check early.
    int lift_certify(int pidx, uint32_t detp, const BigInt &s, const BigInt &prod, bool *ok) {
        *ok = false;
        const double need = abits - (double)s.bit_length() + 3.0;     // bits of 2 H / s, generously
        const int exact_primes = std::max(1, (int)std::ceil(need / 25.9));
        const BigInt c = prod / s;
        if (!(c * s == prod)) return RNS_OK;             // |det A| is a multiple of s; prod is not
        BigInt D(0), Q(1);
        int used = 0;
        bool mismatch = false;
        auto add = [&](uint32_t q, uint32_t dq) {
            const uint32_t sq = s.mod_small(q);
            if (sq == 0) return;                         // q divides s, hence det A: no information
            // dq / sq mod q, then D <- the CRT combination of D mod Q and it mod q.
            const uint32_t sinv = (uint32_t)powmod_u64(sq, q - 2, q);
            const uint64_t target = (uint64_t)dq * sinv % q;
            const uint64_t cq = c.mod_small(q);
            if (target != cq && target != (q - cq) % q) mismatch = true;
            const uint64_t dmod = D.mod_small(q);
            const uint64_t qinv = powmod_u64(Q.mod_small(q), q - 2, q);
            const uint64_t k = (target + q - dmod) % q * qinv % q;
            D = D + Q.mul_small((uint32_t)k);
            Q = Q.mul_small(q);
            used += 1;
        };
        add(aux->primes[pidx], detp);
        int next = pidx + 1;
        const int chunk_max = (int)std::max(1.0, std::min(64.0, kCertChunkBytes / (4.0 * (double)n * (double)n)));
        while (used < exact_primes && !mismatch) {
            // one extra prime per chunk covers a prime that divides s
            const int want = std::min(chunk_max, exact_primes - used + 1);
            std::vector<int> idx;
            for (int j = 0; j < want && next < kAuxPrimes; ++j) idx.push_back(next++);
            if (idx.empty()) return RNS_ENOTSUP;        // 2 H / s exceeds the driver's basis
            std::vector<uint32_t> det;
            DRV_ST(det_mod_primes(idx, det));
            for (size_t j = 0; j < idx.size() && used < exact_primes && !mismatch; ++j)
                add(aux->primes[idx[j]], det[j]);
        }
        st.cert_primes = used;
        if (mismatch) return RNS_OK;
        BigInt Ds = D;                                   // symmetric representative
        if (BigInt::cmp(Ds.shl(1), Q) > 0) Ds = Ds - Q;
        *ok = c == BigInt::abs(Ds);
        return RNS_OK;
    }

    int run_lifting(rns_smith_result *res) {
        const double t0 = now_s();
        st.path = 1;
        DRV_ST(upload_a32());
        SplitMix rng{seed ^ 0xA0761D6478BD642Full};
        int pidx = 0;
        uint32_t detp = 0;
        double tl = now_s();
        DRV_ST(lift_prime(&pidx, &detp));
        st.t_lif += now_s() - tl;
        int t = 4;
        for (int attempt = 0; attempt <= kMaxRestarts + 3; ++attempt) {
            tl = now_s();
            BigInt s;
            std::vector<BigInt> X;
            const int stl = lift_solve(pidx, t, rng, s, X);
            st.t_lif += now_s() - tl;
            if (stl == RNS_EBOUND) {
                st.restarts += 1;
                continue;
            }
            DRV_ST(stl);
            const double ti = now_s();
            const int tp = t + 2;
            std::vector<BigInt> M((size_t)tp * tp, BigInt(0));       // padded with zero columns
            for (int a = 0; a < tp; ++a)
                for (int c = 0; c < t; ++c) M[(size_t)a * tp + c] = mod(X[(size_t)a * t + c], s);
            std::vector<BigInt> g = snf_mod_host(std::move(M), tp, s);
            int nontrivial = 0;
            for (int i = 0; i < t; ++i) nontrivial += g[i] != s;
            st.t_im += now_s() - ti;
            if (nontrivial > t - 2) {                    // more invariants may be > 1
                if (2 * t > kLiftMaxCols) return RNS_ENOTSUP;
                t *= 2;
                continue;
            }
            const double tu = now_s();
            BigInt prod(1);
            for (int i = 0; i < t; ++i) prod = prod * (s / g[i]);
            bool ok = false;
            DRV_ST(lift_certify(pidx, detp, s, prod, &ok));
            st.t_uc += now_s() - tu;
            if (ok && ctx->force_cert_failures > 0) {   // test hook: pretend the check failed
                ctx->force_cert_failures -= 1;
                ok = false;
            }
            if (!ok) {
                st.restarts += 1;
                continue;
            }
            res->s.assign(n, BigInt(1).mag_words());
            for (int i = 0; i < t; ++i) res->s[n - 1 - i] = (s / g[i]).mag_words();
            st.columns = t;
            st.cert_exact = 1;
            st.lift_a_bytes = a_bytes;
            st.lift_kernels = (mfma_lift() ? 1 : 0) | (mfma_lift() && a_bytes == 2 ? 2 | (lift_packed(t) ? 4 : 0) : 0) |
                              (a_bytes == 2 ? 8 : 0);
            st.t_total = now_s() - t0;
            res->st = st;
            return RNS_OK;
        }
        return RNS_ERETRY;
    }

    // ------------------------------------------------------- Smith massager --
    // Phase 2 of Section 2.2 with the massaged matrix B of Eq. (1), in batches
    // of index-(m, r) Smith massagers (Definition 2).  With the batches found
    // so far, (U_b, M_b) for b = 1..k (oldest first) and the modulus s (the
    // smallest invariant found, a multiple of every invariant still to come),
    // the first block row of B^-1 applied to [j; 0; 0] is, modulo integers,
    // pi(A^-1 j) with pi = (I + M_k U_k) ... (I + M_1 U_1) (block inverse of
    // Eq. (1)); s pi(A^-1 J) is integral, and P_1 = Rem(s pi(A^-1 J), s) is the
    // batch's projection.  A^-1 J is lifted p-adically on the GPU (the
    // resident C = A^-1 mod p), Rem(s_n A^-1 J, s_n) follows from the top
    // digits, the earlier batches' factors are applied modulo s_n and the
    // result divided by s_n / s.  The Smith form of P_1 over Z/sZ with its
    // transforms gives the batch: invariants s / d_j, M_j and U_j with
    // -U P_1 R = [D 0] (massager_host.hpp).  The next batch's T block against
    // the earlier ones is -U_new M_old (mod the older invariants); within a
    // batch T is I.  Batches grow with how far s fell (Section 3.2), and once
    // s fits a machine word the next batch takes every remaining invariant.
    struct MBatch {
        BigInt s;                       // the batch's modulus
        std::vector<BigInt> S;          // its invariants, ascending
        std::vector<BigInt> M;          // [r][n]: column j of M, entries mod S[j]
        std::vector<BigInt> U;          // [r][n]: row j of U, entries mod s
    };

    // Host threads in contiguous blocks once count x work (ring operations)
    // repays starting them.
    static msg::ParFor host_par() {
        return [](int64_t cnt, double work, const std::function<void(int64_t)> &f) {
            if (cnt < 2 || (double)cnt * work < 32768.0) {
                for (int64_t i = 0; i < cnt; ++i) f(i);
                return;
            }
            const int nb = (int)std::min<int64_t>(cnt, 64);
            parallel_for(nb, [&](int b) {
                for (int64_t i = cnt * b / nb; i < cnt * (b + 1) / nb; ++i) f(i);
            });
        };
    }

    // The top L of K p-adic digits of A^-1 J for the t columns of J ([t][ldl]
    // int64, host) into dig ([L][t][ldl]; l = 0 is the digit of step K - L).
    // Runs of at most kLiftMaxCols columns are independent liftings: they go
    // round-robin to kLiftLanes streams, each with its own buffers and its own
    // captured graph of the K steps (one run fills only n / 16 work-groups),
    // and copy their top digits into one device array.
    static constexpr int kLiftLanes = 4;
    struct LiftLane {
        hipStream_t s = nullptr;
        DevBuf<int64_t> R0, R1;
        DevBuf<uint32_t> Rm0, Rm1, Xh;
        DevBuf<int32_t> err;
        DevBuf<int64_t> step;
        DevBuf<char> Xd, Rmd;
        StepGraph graph;
        std::vector<uint32_t> Jm;
    };
    int lift_top(int pidx, const std::vector<int64_t> &J, int64_t t, int64_t K, int L,
                 std::vector<uint32_t> &dig) {
        const uint32_t p = aux->primes[pidx];
        const int64_t tmax = kLiftMaxCols;
        dig.assign((size_t)L * t * ldl, 0u);
        const char *Ct = nullptr, *At = nullptr;
        if (mfma_lift()) {
            DRV_ST(dCt.alloc(lift_tile_c_bytes(n)));
            launch_lift_tile_c(dC.p, n, ldl, p, dCt.p, stream);
            DRV_HIP(hipGetLastError());
            Ct = dCt.p;
            if (a_bytes == 2) {
                DRV_ST(dAt.alloc(lift_tile_a_bytes(n)));
                launch_lift_tile_a(dA16.p, n, ldl, dAt.p, stream);
                DRV_HIP(hipGetLastError());
                At = dAt.p;
            }
        }
        DevBuf<uint32_t> dtop;
        DRV_ST(dtop.alloc((size_t)L * t * ldl));
        const int64_t runs = (t + tmax - 1) / tmax;
        const int nl = (int)std::min<int64_t>(kLiftLanes, runs);
        std::vector<LiftLane> lanes((size_t)nl);
        hipEvent_t ready = nullptr;
        DRV_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
        DRV_HIP(hipEventRecord(ready, stream));
        int status = RNS_OK;
        auto fail = [&](int st_) {
            if (status == RNS_OK) status = st_;
        };
        const void *Adev = a_bytes == 2 ? (const void *)dA16.p : (const void *)dA32.p;
        std::vector<LiftBufs> lbs((size_t)nl, LiftBufs{});
        for (int k = 0; k < nl && status == RNS_OK; ++k) {
            LiftLane &ln = lanes[(size_t)k];
            if (hipStreamCreateWithFlags(&ln.s, hipStreamNonBlocking) != hipSuccess) {
                fail(RNS_EDEVICE);
                break;
            }
            if (hipStreamWaitEvent(ln.s, ready, 0) != hipSuccess) fail(RNS_EDEVICE);
            int a = ln.Xh.alloc((size_t)K * tmax * ldl);
            if (a == RNS_OK) a = ln.R0.alloc((size_t)tmax * ldl);
            if (a == RNS_OK) a = ln.R1.alloc((size_t)tmax * ldl);
            if (a == RNS_OK) a = ln.Rm0.alloc((size_t)tmax * ldl);
            if (a == RNS_OK) a = ln.Rm1.alloc((size_t)tmax * ldl);
            if (a == RNS_OK) a = ln.err.alloc(1);
            if (a == RNS_OK) a = ln.step.alloc(1);
            LiftBufs lb{ln.R0.p, ln.R1.p, ln.Rm0.p, ln.Rm1.p, ln.Xh.p, ln.err.p, ln.step.p};
            lb.Ct = Ct;
            if (a == RNS_OK && At) {
                a = ln.Xd.alloc(lift_frag_bytes(n));
                if (a == RNS_OK) a = ln.Rmd.alloc(lift_frag_bytes(n));
                lb.At = At;
                lb.Xd = ln.Xd.p;
                lb.Rmd = ln.Rmd.p;
            }
            if (a != RNS_OK) fail(a);
            if (hipMemsetAsync(ln.err.p, 0, sizeof(int32_t), ln.s) != hipSuccess) fail(RNS_EDEVICE);
            lbs[(size_t)k] = lb;
        }
        for (int64_t run = 0; run < runs && status == RNS_OK; ++run) {
            LiftLane &ln = lanes[(size_t)(run % nl)];
            const LiftBufs &lb = lbs[(size_t)(run % nl)];
            const int64_t c0 = run * tmax;
            const int tc = (int)std::min<int64_t>(tmax, t - c0);
            const size_t cnt = (size_t)tc * ldl;
            // The lane's previous run must be done with R0 before it is
            // overwritten: copies are ordered on the lane's stream, and the
            // host buffer is one per lane, so wait for that stream first.
            if (run >= nl && hipStreamSynchronize(ln.s) != hipSuccess) {
                fail(RNS_EDEVICE);
                break;
            }
            ln.Jm.assign(cnt, 0u);
            for (size_t e = 0; e < cnt; ++e) {
                const int64_t v = J[(size_t)c0 * ldl + e] % (int64_t)p;
                ln.Jm[e] = (uint32_t)(v < 0 ? v + (int64_t)p : v);
            }
            bool ok = hipMemcpyAsync(ln.R0.p, J.data() + (size_t)c0 * ldl, sizeof(int64_t) * cnt,
                                     hipMemcpyHostToDevice, ln.s) == hipSuccess;
            ok = ok && hipMemcpyAsync(ln.Rm0.p, ln.Jm.data(), sizeof(uint32_t) * cnt, hipMemcpyHostToDevice,
                                      ln.s) == hipSuccess;
            ok = ok && hipMemsetAsync(ln.step.p, 0, sizeof(int64_t), ln.s) == hipSuccess;
            if (!ok) {
                fail(RNS_EDEVICE);
                break;
            }
            if (lb.Rmd) launch_lift_frag(ln.Rm0.p, n, ldl, tc, p, ln.Rmd.p, ln.s);   // the first step's Rm
            if (tc == tmax && !ln.graph.tried && runs - run > nl) {
                ln.graph.tried = true;
                if (!tl_trace && hipStreamBeginCapture(ln.s, hipStreamCaptureModeRelaxed) == hipSuccess) {
                    launch_lift_steps(dC.p, Adev, a_bytes, n, ldl, (int)tmax, p, lb, (int)K, ln.s);
                    hipGraph_t gr = nullptr;
                    if (hipStreamEndCapture(ln.s, &gr) == hipSuccess && gr) {
                        ln.graph.g = gr;
                        if (hipGraphInstantiate(&ln.graph.exec, gr, nullptr, nullptr, 0) != hipSuccess)
                            ln.graph.exec = nullptr;
                    }
                    (void)hipGetLastError();
                }
            }
            if (tc == tmax && ln.graph.exec) {
                if (hipGraphLaunch(ln.graph.exec, ln.s) != hipSuccess) fail(RNS_EDEVICE);
            } else {
                launch_lift_steps(dC.p, Adev, a_bytes, n, ldl, tc, p, lb, (int)K, ln.s);
                if (hipGetLastError() != hipSuccess) fail(RNS_EDEVICE);
            }
            // top digits: L rows of tc x ldl words into dtop[l][c0 ..][.]
            if (hipMemcpy2DAsync(dtop.p + (size_t)c0 * ldl, sizeof(uint32_t) * (size_t)t * ldl,
                                 ln.Xh.p + (size_t)(K - L) * cnt, sizeof(uint32_t) * cnt, sizeof(uint32_t) * cnt,
                                 (size_t)L, hipMemcpyDeviceToDevice, ln.s) != hipSuccess)
                fail(RNS_EDEVICE);
            st.lift_steps += (int)K;
        }
        int32_t anyerr = 0;
        for (LiftLane &ln : lanes) {
            if (!ln.s) continue;
            int32_t e = 0;
            if (hipMemcpyAsync(&e, ln.err.p, sizeof(int32_t), hipMemcpyDeviceToHost, ln.s) != hipSuccess ||
                hipStreamSynchronize(ln.s) != hipSuccess)
                fail(RNS_EDEVICE);
            anyerr |= e;
        }
        for (LiftLane &ln : lanes)
            if (ln.s) (void)hipStreamDestroy(ln.s);
        (void)hipEventDestroy(ready);
        if (status != RNS_OK) return status;
        if (anyerr) return RNS_EDEVICE;                  // an inexact division: C is not A^-1 mod p
        DRV_HIP(hipMemcpyAsync(dig.data(), dtop.p, sizeof(uint32_t) * dig.size(), hipMemcpyDeviceToHost, stream));
        DRV_ST(sync());
        return RNS_OK;
    }

    // The first G runs of kLiftMaxCols columns of J ([t][ldl], host) lifted
    // together (one launch per product and step, blockIdx.y = run; step i's
    // digits in ring slot i % ring).  With a word table `tab` (modulus
    // m < 2^62), Y[i t + c] = Rem(s_n x, m) for those columns is computed on
    // the GPU: after the first K - L steps, the top L digits are folded into
    // per-entry sums kKeep steps at a time, so the ring holds kKeep slots (Y's
    // other columns are left for the caller); without one, the ring holds the
    // top L steps and the digits come back as dig ([L][G 16][ldl], l = 0 the
    // digit of step K - L).
    int lift_grouped(int pidx, const std::vector<int64_t> &J, int64_t t, int64_t G, int64_t K, int L,
                     const msg::PadicTable<msg::Ring64> *tab, std::vector<uint64_t> *Y, std::vector<uint32_t> *dig) {
        constexpr int kKeep = 128;
        const uint32_t p = aux->primes[pidx];
        const int64_t tc = kLiftMaxCols, cols = G * tc;
        const size_t cnt = (size_t)(cols * ldl), fb = lift_frag_bytes(n);
        const int64_t ring = tab ? std::min<int64_t>(L, kKeep) : L;
        DRV_ST(dCt.alloc(lift_tile_c_bytes(n)));
        launch_lift_tile_c(dC.p, n, ldl, p, dCt.p, stream);
        DRV_HIP(hipGetLastError());
        DRV_ST(dAt.alloc(lift_tile_a_bytes(n)));
        launch_lift_tile_a(dA16.p, n, ldl, dAt.p, stream);
        DRV_HIP(hipGetLastError());
        DevBuf<int64_t> R0, R1, step;
        DevBuf<uint32_t> Rm0, Rm1, Xh;
        DevBuf<char> Xd, Rmd;
        DevBuf<int32_t> err;
        DevBuf<uint64_t> dB, dF, dY, dacc;
        DevBuf<uint32_t> dtop;
        DRV_ST(R0.alloc(cnt));
        DRV_ST(R1.alloc(cnt));
        DRV_ST(Rm0.alloc(cnt));
        DRV_ST(Rm1.alloc(cnt));
        DRV_ST(Xh.alloc((size_t)(G * ring * tc * ldl)));
        DRV_ST(Xd.alloc((size_t)G * fb));
        DRV_ST(Rmd.alloc((size_t)G * fb));
        DRV_ST(err.alloc(2));
        DRV_ST(step.alloc(1));
        if (tab) {
            DRV_ST(dB.alloc((size_t)L + 1));
            DRV_ST(dF.alloc((size_t)L + 1));
            DRV_ST(dY.alloc((size_t)(n * t)));
            DRV_ST(dacc.alloc((size_t)(4 * cols * n)));
        }
        std::vector<uint32_t> Jm(cnt);
        for (size_t e = 0; e < cnt; ++e) {
            const int64_t v = J[e] % (int64_t)p;
            Jm[e] = (uint32_t)(v < 0 ? v + (int64_t)p : v);
        }
        DRV_HIP(hipMemcpyAsync(R0.p, J.data(), sizeof(int64_t) * cnt, hipMemcpyHostToDevice, stream));
        DRV_HIP(hipMemcpyAsync(Rm0.p, Jm.data(), sizeof(uint32_t) * cnt, hipMemcpyHostToDevice, stream));
        if (tab) {
            DRV_HIP(hipMemcpyAsync(dB.p, tab->B.data(), sizeof(uint64_t) * ((size_t)L + 1), hipMemcpyHostToDevice,
                                   stream));
            DRV_HIP(hipMemcpyAsync(dF.p, tab->frac.data(), sizeof(uint64_t) * ((size_t)L + 1),
                                   hipMemcpyHostToDevice, stream));
            DRV_HIP(hipMemsetAsync(dacc.p, 0, sizeof(uint64_t) * (size_t)(4 * cols * n), stream));
        }
        DRV_HIP(hipMemsetAsync(err.p, 0, 2 * sizeof(int32_t), stream));
        DRV_HIP(hipMemsetAsync(step.p, 0, sizeof(int64_t), stream));
        for (int64_t g = 0; g < G; ++g)                  // the first step's Rm, per run
            launch_lift_frag(Rm0.p + (size_t)(g * tc * ldl), n, ldl, (int)tc, p, Rmd.p + (size_t)g * fb, stream);
        DRV_HIP(hipGetLastError());
        LiftBufs lb{R0.p, R1.p, Rm0.p, Rm1.p, Xh.p, err.p, step.p};
        lb.Ct = dCt.p;
        lb.At = dAt.p;
        lb.Xd = Xd.p;
        lb.Rmd = Rmd.p;
        lb.grp.groups = (int)G;
        lb.grp.r = tc * ldl;
        lb.grp.rm = tc * ldl;
        lb.grp.xh = ring * tc * ldl;
        lb.grp.frag = (int64_t)(fb / 16);                // v4i_l elements
        lb.grp.ring = ring;
        if (!lift_groups_ok(lb, a_bytes, (int)tc)) return RNS_EINVAL;
        int32_t herr[2] = {0, 0};
        if (tab) {
            // K - L steps whose digits are not needed, then the top L in
            // chunks of `ring`, each folded into the sums.
            if (K > L) launch_lift_steps(dC.p, dA16.p, a_bytes, n, ldl, (int)tc, p, lb, (int)(K - L), stream);
            for (int64_t done = 0; done < L; done += ring) {
                const int chunk = (int)std::min<int64_t>(ring, L - done);
                launch_lift_steps(dC.p, dA16.p, a_bytes, n, ldl, (int)tc, p, lb, chunk, stream);
                launch_padic_acc(Xh.p, n, ldl, cols, lb.grp.xh, ring, K, K - L + done, chunk, dB.p, dF.p, dacc.p,
                                 stream);
            }
            launch_padic_fin(dacc.p, n, cols, t, dB.p, tab->F.s, dY.p, err.p + 1, stream);
            DRV_HIP(hipGetLastError());
            DRV_HIP(hipMemcpyAsync(Y->data(), dY.p, sizeof(uint64_t) * (size_t)(n * t), hipMemcpyDeviceToHost,
                                   stream));
        } else {
            launch_lift_steps(dC.p, dA16.p, a_bytes, n, ldl, (int)tc, p, lb, (int)K, stream);
            DRV_HIP(hipGetLastError());
            // plane l (step K - L + l) of every run: G blocks of 16 ldl words,
            // gathered on the device, then one contiguous copy to the host
            // (not one strided device-to-host copy per plane)
            DRV_ST(dtop.alloc((size_t)L * cnt));
            const size_t blk = sizeof(uint32_t) * (size_t)(tc * ldl);
            for (int l = 0; l < L; ++l)
                DRV_HIP(hipMemcpy2DAsync(dtop.p + (size_t)l * cnt, blk,
                                         Xh.p + (size_t)(((K - L + l) % L) * tc * ldl), sizeof(uint32_t) * lb.grp.xh,
                                         blk, (size_t)G, hipMemcpyDeviceToDevice, stream));
            dig->assign((size_t)L * cnt, 0u);
            DRV_HIP(hipMemcpyAsync(dig->data(), dtop.p, sizeof(uint32_t) * (size_t)L * cnt, hipMemcpyDeviceToHost,
                                   stream));
        }
        DRV_HIP(hipMemcpyAsync(herr, err.p, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, stream));
        DRV_ST(sync());
        if (herr[0]) return RNS_EDEVICE;                 // an inexact division: C is not A^-1 mod p
        if (herr[1]) return RNS_EBOUND;                  // s_n A^-1 J is not integral
        st.lift_steps += (int)(K * G);
        return RNS_OK;
    }

    // The largest divisor of y prime to s (repeated gcds, no factoring).
    static BigInt coprime_part(BigInt y, const BigInt &s) {
        for (;;) {
            const BigInt g = BigInt::gcd(y, s);
            if (g.is_one() || g.is_zero()) return y;
            y = y / g;
        }
    }

    // The batch's projection P_1 = Rem(s pi(A^-1 J), s) (n x t, row-major)
    // for a random J with entries in [-128, 128].  With V = s_n pi(x) (an
    // integer multiple of q = s_n / s) and P_1 = V / q mod s, only V modulo
    // M' = s_n / u matters, u the largest divisor of s_n prime to s: with
    // q = q_b u, (V mod M') / q_b = u (V / q) mod s.  So Y = s_n x and the
    // earlier batches' factors are applied modulo M' (a machine word when the
    // primes of s divide s_n only to small powers).  RNS_EBOUND when s_n A^-1 J
    // is not integral (s_n misses a factor) or V is not a multiple of q (an
    // earlier batch was not maximal).
    // Reading 21's evaluation for a multiword M' on the GPU: the dot
    // products sum_l d_l B_l of every entry are one exact residue product of
    // the 32-bit limbs of the B_l ((limbs x L) against the L digit planes, each
    // sum below L 2^58), recombined per entry on host threads; the rounding
    // term e comes from the fractions as in PadicTable::eval_block.  dig holds
    // the top L digits of tr columns ([L][tr][ldl], plane j the digit of step
    // K - L + j); Y's entries (row i, column c0 + c) are written.
    int padic_eval_big(const msg::PadicTable<msg::RingBig> &tab, const msg::RingBig &F, const std::vector<uint32_t> &dig,
                       int64_t tr, int64_t t, int64_t c0, std::vector<BigInt> &Y, bool *good) {
        const int L = tab.L;
        int64_t Wb = 1;
        for (int l = 1; l <= L; ++l) Wb = std::max<int64_t>(Wb, (int64_t)tab.B[(size_t)l].mag.size());
        const int64_t E = tr * ldl;
        std::vector<int64_t> Am((size_t)(Wb * L), 0), Bm((size_t)(L * E));
        for (int j = 0; j < L; ++j) {
            const BigInt &b = tab.B[(size_t)(L - j)];
            for (int64_t v = 0; v < (int64_t)b.mag.size(); ++v) Am[(size_t)(v * L + j)] = (int64_t)b.mag[(size_t)v];
        }
        const msg::ParFor par = host_par();
        par(L, (double)E, [&](int64_t j) {
            for (int64_t e = 0; e < E; ++e) Bm[(size_t)(j * E + e)] = (int64_t)dig[(size_t)(j * E + e)];
        });
        std::vector<uint64_t> Out;
        int Wo = 0;
        DRV_ST(exact_product(Am.data(), Wb, L, Bm.data(), E, 59.0 + std::log2((double)L), Out, Wo));
        std::atomic<bool> fine{true};
        par(tr * n, (double)Wb * 4, [&](int64_t q) {
            const int64_t c = q / n, i = q % n, e = c * ldl + i;
            unsigned __int128 fs = 0;
            for (int l = 1; l <= L; ++l) fs += (unsigned __int128)tab.frac[(size_t)l] * dig[(size_t)((L - l) * E + e)];
            const uint64_t ev = (uint64_t)((fs + ((unsigned __int128)1 << 63)) >> 64);
            const unsigned __int128 ee = (unsigned __int128)ev << 64;
            const unsigned __int128 dist = fs > ee ? fs - ee : ee - fs;
            if (dist >= ((unsigned __int128)1 << 43)) fine = false;
            std::vector<uint64_t> sl((size_t)(Wb + 4), 0);
            for (int64_t v = 0; v < Wb; ++v) {
                const uint64_t *x = Out.data() + (size_t)((v * E + e) * Wo);
                unsigned __int128 val = x[0];
                if (Wo > 1) val |= (unsigned __int128)x[1] << 64;
                for (int d = 0; d < 4 && val; ++d, val >>= 32) sl[(size_t)(v + d)] += (uint64_t)(val & 0xFFFFFFFFull);
            }
            uint64_t carry = 0;
            BigInt xb(0);
            xb.mag.resize(sl.size());
            for (size_t k = 0; k < sl.size(); ++k) {
                const uint64_t z = sl[k] + carry;
                xb.mag[k] = (uint32_t)z;
                carry = z >> 32;
            }
            while (!xb.mag.empty() && xb.mag.back() == 0) xb.mag.pop_back();
            Y[(size_t)(i * t + c0 + c)] = F.add(F.from(xb), F.mul_u64(tab.B[0], ev));
        });
        *good = fine;
        return RNS_OK;
    }

    int projection(int pidx, const BigInt &sn, const BigInt &s, const std::vector<MBatch> &B, int64_t t,
                   SplitMix &rng, std::vector<BigInt> &P1) {
        const BigInt u = coprime_part(sn, s);
        const BigInt Mp = sn / u;
        if (Mp.bit_length() <= 62) return projection_in(msg::Ring64(Mp.to_u64_mag()), sn, s, u, B, t, pidx, rng, P1);
        return projection_in(msg::RingBig(Mp), sn, s, u, B, t, pidx, rng, P1);
    }

    template <class Ring>
    int projection_in(const Ring &FM, const BigInt &sn, const BigInt &s, const BigInt &u,
                      const std::vector<MBatch> &B, int64_t t, int pidx, SplitMix &rng, std::vector<BigInt> &P1) {
        using V = typename Ring::V;
        const uint32_t p = aux->primes[pidx];
        const double lp = std::log2((double)p);
        // |s_n A^-1 J| = |adj(A) J| s_n / |det A| <= n 2^7 H s_n / |det A|, and
        // |det A| >= P, the product of the invariants found so far (the
        // earlier batches' massager is integral, so det S divides det A);
        // P includes s_n from the first batch on, so the bound only shrinks.
        // K digits leave a 2^-24 margin, L top digits resolve s_n X_K / p^K to
        // within 2^-24.
        double lpf = 0;                                  // a lower bound on log2 P
        for (const MBatch &b : B)
            for (const BigInt &o : b.S) {
                const double d = o.to_double();
                lpf += std::isfinite(d) ? std::log2(std::max(1.0, d)) - 1e-9 : (double)o.bit_length() - 1.0;
            }
        const double shrink = std::min(0.0, (double)sn.bit_length() - lpf);
        const int64_t K = (int64_t)std::ceil((abits + std::log2((double)n) + 7.0 + 24.0 + shrink) / lp) + 1;
        const int L = (int)std::min<int64_t>(K, (int64_t)std::ceil(((double)sn.bit_length() + 26.0) / lp) + 1);
        std::vector<int64_t> J((size_t)t * ldl, 0);
        for (int64_t c = 0; c < t; ++c)
            for (int64_t r = 0; r < n; ++r) J[(size_t)c * ldl + r] = (int64_t)(rng.next() % 257) - 128;
        const msg::ParFor par = host_par();
        const msg::PadicTable<Ring> tab(FM, sn, p, K, L, par);
        std::vector<V> Y((size_t)n * t);
        std::atomic<bool> ok{true};
        // With a word modulus and the matrix-core step kernels, the full runs
        // of 16 columns are lifted in one grouped run and their Y computed on
        // the GPU; the rest goes through the lanes and the host table.
        // Host evaluation of columns c0 .. c0 + tr - 1 from their digits
        // ([L][tr][ldl]), in blocks of rows of one column (the digit planes
        // are read in order).
        auto host_eval = [&](const std::vector<uint32_t> &dig, int64_t c0, int64_t tr) {
            if constexpr (std::is_same<Ring, msg::RingBig>::value) {
                if (tr * n >= 16384) {                   // the dot products on the GPU
                    bool good = true;
                    const int rc = padic_eval_big(tab, FM, dig, tr, t, c0, Y, &good);
                    if (rc != RNS_OK || !good) ok = false;
                    return;
                }
            }
            const int64_t rb = std::is_same<Ring, msg::Ring64>::value ? 1024 : 256;
            const int64_t nrb = (n + rb - 1) / rb;
            par(tr * nrb, (double)rb * L * FM.cost() / 4.0, [&](int64_t q) {
                const int64_t c = q / nrb, i0 = (q % nrb) * rb, cnt = std::min(rb, n - i0);
                if (!tab.eval_block(dig.data() + (size_t)c * ldl + i0, tr * ldl, cnt,
                                    Y.data() + (size_t)(i0 * t + c0 + c), t))
                    ok = false;
            });
        };
        int64_t tg = 0;
        const int64_t G = t / kLiftMaxCols;
        if (G >= 2 && mfma_lift() && a_bytes == 2) {
            if constexpr (std::is_same<Ring, msg::Ring64>::value) {
                DRV_ST(lift_grouped(pidx, J, t, G, K, L, &tab, &Y, nullptr));
            } else {
                std::vector<uint32_t> dig;
                DRV_ST(lift_grouped(pidx, J, t, G, K, L, nullptr, nullptr, &dig));
                host_eval(dig, 0, G * kLiftMaxCols);
            }
            tg = G * kLiftMaxCols;
        }
        if (tg < t) {
            const int64_t tr = t - tg;
            const std::vector<int64_t> Jr(J.begin() + (size_t)(tg * ldl), J.end());
            std::vector<uint32_t> dig;
            DRV_ST(lift_top(pidx, Jr, tr, K, L, dig));
            host_eval(dig, tg, tr);
        }
        if (!ok) return RNS_EBOUND;
        // Earlier batches, oldest first: Y <- Y + M_b (U_b Y) (mod M').
        for (const MBatch &b : B) {
            const int64_t r = (int64_t)b.S.size();
            std::vector<V> Ub((size_t)(r * n)), Mb((size_t)(r * n));
            par(r * n, FM.cost(), [&](int64_t e) {
                Ub[(size_t)e] = FM.from(b.U[(size_t)e]);
                Mb[(size_t)e] = FM.from(b.M[(size_t)e]);
            });
            std::vector<V> Z((size_t)(r * t));
            par(r * t, (double)n * FM.cost(), [&](int64_t e) {
                const int64_t k = e / t, c = e % t;
                V acc = FM.zero();
                for (int64_t i = 0; i < n; ++i) {
                    const V &uv = Ub[(size_t)(k * n + i)];
                    if (!FM.is_zero(uv)) acc = FM.add(acc, FM.mul(uv, Y[(size_t)(i * t + c)]));
                }
                Z[(size_t)e] = acc;
            });
            par(n, (double)(r * t) * FM.cost(), [&](int64_t i) {
                for (int64_t k = 0; k < r; ++k) {
                    const V &mv = Mb[(size_t)(k * n + i)];
                    if (FM.is_zero(mv)) continue;
                    for (int64_t c = 0; c < t; ++c)
                        Y[(size_t)(i * t + c)] = FM.add(Y[(size_t)(i * t + c)], FM.mul(mv, Z[(size_t)(k * t + c)]));
                }
            });
        }
        const BigInt Mp = FM.big(FM.s), qb = Mp / s;
        const BigInt uinv = msg::RingBig::inv(mod(u, s), s);
        P1.assign((size_t)n * t, BigInt(0));
        if constexpr (std::is_same<Ring, msg::Ring64>::value) {
            const uint64_t q64 = qb.to_u64_mag(), s64 = s.to_u64_mag(), ui64 = uinv.to_u64_mag();
            par(n * t, 2.0, [&](int64_t e) {
                const uint64_t v = Y[(size_t)e];
                if (v % q64) ok = false;
                P1[(size_t)e] = BigInt::from_u64(msg::Ring64::mulm((v / q64) % s64, ui64, s64));
            });
        } else {
            const double limbs = (double)Mp.mag.size() + 1.0;
            par(n * t, 4.0 * limbs * limbs, [&](int64_t e) {
                BigInt qq, rr;
                BigInt::divmod_trunc(FM.big(Y[(size_t)e]), qb, qq, rr);
                if (!rr.is_zero()) ok = false;
                P1[(size_t)e] = mod(qq * uinv, s);
            });
        }
        if (!ok) return RNS_EBOUND;
        st.columns += (int)t;
        return RNS_OK;
    }

    // One batch from the Smith form of P_1 over Z/sZ: the largest orders
    // s / d_j (all of them when `fin` or when at most t - extra are above 1,
    // which sets *done), with their M and U.
    template <class Ring>
    void batch_from(const Ring &F, const std::vector<BigInt> &P1, int64_t t, const BigInt &s, int64_t extra,
                    bool fin, MBatch &b, bool *done) {
        using V = typename Ring::V;
        const msg::ParFor par = host_par();
        std::vector<V> W(P1.size());
        par((int64_t)P1.size(), 2.0, [&](int64_t e) {           // entries of P_1 are already in [0, s)
            if constexpr (std::is_same<Ring, msg::Ring64>::value) W[(size_t)e] = P1[(size_t)e].to_u64_mag();
            else W[(size_t)e] = P1[(size_t)e];
        });
        // Multiword s with many rows: the Smith form of the compression
        // G P_1 ((t + 8) x t, G random with 16-bit entries) instead of P_1.
        // E' = E_G G is then a left transform of P_1 (E' P_1 R = diag(d)), so
        // -U P_1 R = [D 0] and U M = -I hold as before; G P_1 has the Smith
        // form of P_1 unless G loses rank on P_1's columns modulo a prime of
        // s (probability about 2^-8 per prime power), and a smaller batch
        // that results is caught by the projection checks or Phase 3.
        constexpr int64_t kCompressRows = 8;
        const bool compress = !std::is_same<Ring, msg::Ring64>::value && n > 4 * (t + kCompressRows);
        const int64_t nr = compress ? t + kCompressRows : n;
        std::vector<uint32_t> G;
        std::vector<V> Wc;
        if (compress) {
            SplitMix g{seed ^ 0x9E3779B97F4A7C15ull ^ ((uint64_t)t << 32) ^ (uint64_t)s.bit_length()};
            G.resize((size_t)(nr * n));
            for (auto &v : G) v = (uint32_t)(g.next() & 0xFFFF);
            Wc.assign((size_t)(nr * t), F.zero());
            par(nr * t, (double)n * 64, [&](int64_t e) {
                const int64_t r = e / t, c = e % t;
                BigInt sum(0);
                for (int64_t i = 0; i < n; ++i) {
                    const uint32_t gv = G[(size_t)(r * n + i)];
                    if (gv) sum = sum + P1[(size_t)(i * t + c)].mul_small(gv);
                }
                Wc[(size_t)e] = F.from(sum);
            });
        }
        const msg::SnfT<Ring> S = msg::snf_transform(F, compress ? Wc : W, nr, t, par);
        int64_t nontriv = 0;
        while (nontriv < t && !(F.big(S.d[(size_t)nontriv]) == s)) ++nontriv;
        *done = fin || nontriv <= t - extra;
        const int64_t take = *done ? nontriv : t - extra;
        std::vector<V> E = msg::left_rows(F, S, nr, take, par);
        if (compress) {                                      // E' = E_G G: take x n
            std::vector<V> Ef((size_t)(take * n));
            par(take * n, (double)nr * 64, [&](int64_t e) {
                const int64_t j = e / n, i = e % n;
                BigInt sum(0);
                for (int64_t r = 0; r < nr; ++r) {
                    const uint32_t gv = G[(size_t)(r * n + i)];
                    const V &ev = E[(size_t)(j * nr + r)];
                    if (gv && !F.is_zero(ev)) sum = sum + F.big(ev).mul_small(gv);
                }
                Ef[(size_t)e] = F.from(sum);
            });
            E.swap(Ef);
        }
        b.s = s;
        b.S.assign((size_t)take, BigInt(0));
        b.M.assign((size_t)(take * n), BigInt(0));
        b.U.assign((size_t)(take * n), BigInt(0));
        for (int64_t j = 0; j < take; ++j) b.S[(size_t)(take - 1 - j)] = s / F.big(S.d[(size_t)j]);
        // Word rings: sums of products in 128 bits, reduced once per `run`
        // products (each below s^2 < 2^124).
        int64_t run = 1;
        if constexpr (std::is_same<Ring, msg::Ring64>::value) {
            const unsigned __int128 sq = (unsigned __int128)F.s * F.s;
            run = (int64_t)std::min<unsigned __int128>((~(unsigned __int128)0) / (sq ? sq : 1), (unsigned __int128)1 << 30);
        }
        par(n, (double)take * t * F.cost(), [&](int64_t i) {
            for (int64_t j = 0; j < take; ++j) {
                V acc = F.zero();
                if constexpr (std::is_same<Ring, msg::Ring64>::value) {
                    unsigned __int128 a128 = 0;
                    int64_t cnt = 0;
                    for (int64_t k = 0; k < t; ++k) {
                        a128 += (unsigned __int128)W[(size_t)(i * t + k)] * S.R[(size_t)(k * t + j)];
                        if (++cnt == run) {
                            a128 %= F.s;
                            cnt = 1;
                        }
                    }
                    acc = (V)(a128 % F.s);
                } else {
                    BigInt sum(0);                           // one reduction per entry
                    for (int64_t k = 0; k < t; ++k) {
                        const V &w = W[(size_t)(i * t + k)], &rr = S.R[(size_t)(k * t + j)];
                        if (!F.is_zero(w) && !F.is_zero(rr)) sum = sum + F.big(w) * F.big(rr);
                    }
                    acc = F.from(sum);
                }
                // (P_1 R)_j = d_j L_j (mod s): the column of L, reduced mod s / d_j
                const int64_t a = take - 1 - j;
                const BigInt d = F.big(S.d[(size_t)j]);
                b.M[(size_t)(a * n + i)] = mod(F.big(acc) / d, b.S[(size_t)a]);
                b.U[(size_t)(a * n + i)] = F.big(F.neg(E[(size_t)(j * n + i)]));
            }
        });
    }

    // One batch for a word modulus s on the GPU: local Smith forms with
    // transforms over every prime power of s (massager_kernels.hip), then on
    // host threads the planes combined by the CRT: the orders s / d_j, M_j =
    // (P_1 R)_j / d_j and U_j = -(row j of E) (the same batch as batch_from).
    int gpu_batch(const std::vector<BigInt> &P1, int64_t t, const BigInt &s, int64_t extra, bool fin, MBatch &b,
                  bool *done) {
        const uint64_t s64 = s.to_u64_mag();
        if (n >= (1 << 21) || t >= (1 << 21)) return RNS_ENOTSUP;
        const auto fac = msg::factor64(s64);
        const int F = (int)fac.size();
        std::vector<LsnfPlane> pl((size_t)F);
        for (int f = 0; f < F; ++f) {
            LsnfPlane &P0 = pl[(size_t)f];
            P0.q = fac[(size_t)f].first;
            P0.e = fac[(size_t)f].second;
            P0.m = 1;
            for (int i = 0; i < P0.e; ++i) P0.m *= P0.q;
            P0.pow2 = P0.q == 2;
            P0.qinv = P0.qmax = P0.minv = 0;
            P0.r2 = P0.rinv = 1;
            if (!P0.pow2) {
                uint64_t x = P0.q;                        // Newton: q^-1 mod 2^64
                for (int i = 0; i < 6; ++i) x *= 2 - P0.q * x;
                P0.qinv = x;
                P0.qmax = ~0ull / P0.q;
                uint64_t y = P0.m;
                for (int i = 0; i < 6; ++i) y *= 2 - P0.m * y;
                P0.minv = (uint64_t)0 - y;
                const uint64_t r = (uint64_t)(((unsigned __int128)1 << 64) % P0.m);
                P0.r2 = (uint64_t)((unsigned __int128)r * r % P0.m);
                P0.rinv = msg::Ring64::inv(r, P0.m);
            }
        }
        const int64_t nt = n * t;
        DevBuf<uint64_t> dP, W, Pf, E, R, units, out;
        DevBuf<int32_t> vals;
        DevBuf<LsnfStep> dst;
        DevBuf<LsnfPlane> dpl;
        DRV_ST(dP.alloc((size_t)nt));
        DRV_ST(W.alloc((size_t)F * nt));
        DRV_ST(Pf.alloc((size_t)F * nt));
        DRV_ST(E.alloc((size_t)F * n * n));
        DRV_ST(R.alloc((size_t)F * t * t));
        DRV_ST(units.alloc((size_t)F * t));
        DRV_ST(vals.alloc((size_t)F * t));
        DRV_ST(dst.alloc((size_t)F));
        DRV_ST(dpl.alloc((size_t)F));
        std::vector<uint64_t> P64((size_t)nt);
        const msg::ParFor par = host_par();
        par(nt, 2.0, [&](int64_t e) { P64[(size_t)e] = P1[(size_t)e].to_u64_mag(); });
        DRV_HIP(hipMemcpyAsync(dP.p, P64.data(), sizeof(uint64_t) * (size_t)nt, hipMemcpyHostToDevice, stream));
        DRV_HIP(hipMemcpyAsync(dpl.p, pl.data(), sizeof(LsnfPlane) * (size_t)F, hipMemcpyHostToDevice, stream));
        launch_ls_load(dP.p, n, t, dpl.p, F, W.p, Pf.p, E.p, R.p, dst.p, stream);
        DRV_HIP(hipGetLastError());
        const int64_t steps = std::min(n, t);
        std::vector<LsnfStep> hst((size_t)F);
        int64_t c = 0;
        for (; c < steps; ++c) {
            launch_ls_step(W.p, E.p, R.p, n, t, c, dpl.p, F, dst.p, vals.p, units.p, stream);
            DRV_HIP(hipGetLastError());
            if ((c & 63) == 63) {                        // every plane finished: the rest is zero
                DRV_HIP(hipMemcpyAsync(hst.data(), dst.p, sizeof(LsnfStep) * (size_t)F, hipMemcpyDeviceToHost,
                                       stream));
                DRV_ST(sync());
                bool all = true;
                for (const LsnfStep &x : hst) all = all && x.done;
                if (all) {
                    ++c;
                    break;
                }
            }
        }
        std::vector<int32_t> hv((size_t)F * t);
        std::vector<uint64_t> hu((size_t)F * t);
        DRV_HIP(hipMemcpyAsync(hv.data(), vals.p, sizeof(int32_t) * hv.size(), hipMemcpyDeviceToHost, stream));
        DRV_HIP(hipMemcpyAsync(hu.data(), units.p, sizeof(uint64_t) * hu.size(), hipMemcpyDeviceToHost, stream));
        DRV_ST(sync());
        // Steps not run (every plane already finished) have valuation e.
        auto val = [&](int f, int64_t j) { return j < c ? hv[(size_t)(f * t + j)] : pl[(size_t)f].e; };
        std::vector<uint64_t> ord((size_t)t, 1);
        for (int64_t j = 0; j < t; ++j)
            for (int f = 0; f < F; ++f)
                for (int i = val(f, j); i < pl[(size_t)f].e; ++i) ord[(size_t)j] *= pl[(size_t)f].q;
        int64_t nontriv = 0;
        while (nontriv < t && ord[(size_t)nontriv] > 1) ++nontriv;
        *done = fin || nontriv <= t - extra;
        const int64_t take = *done ? nontriv : t - extra;
        b.s = s;
        b.S.assign((size_t)take, BigInt(0));
        b.M.assign((size_t)(take * n), BigInt(0));
        b.U.assign((size_t)(take * n), BigInt(0));
        if (take == 0) return RNS_OK;
        DRV_ST(out.alloc((size_t)F * n * take));
        launch_ls_plain(E.p, n, take, dpl.p, F, stream);
        launch_ls_pr(Pf.p, R.p, n, t, take, dpl.p, F, out.p, stream);
        DRV_HIP(hipGetLastError());
        std::vector<uint64_t> hE((size_t)F * take * n), hPR((size_t)F * n * take);
        for (int f = 0; f < F; ++f)
            DRV_HIP(hipMemcpyAsync(hE.data() + (size_t)f * take * n, E.p + (size_t)f * n * n,
                                   sizeof(uint64_t) * (size_t)(take * n), hipMemcpyDeviceToHost, stream));
        DRV_HIP(hipMemcpyAsync(hPR.data(), out.p, sizeof(uint64_t) * hPR.size(), hipMemcpyDeviceToHost, stream));
        DRV_ST(sync());
        // Per position j: the modulus of plane f for M (q^(e - v)), the inverse
        // of its unit part there, and q^v.
        std::vector<uint64_t> mm((size_t)F * take), qv((size_t)F * take), ui((size_t)F * take);
        for (int64_t j = 0; j < take; ++j) {
            b.S[(size_t)(take - 1 - j)] = BigInt::from_u64(ord[(size_t)j]);
            for (int f = 0; f < F; ++f) {
                const LsnfPlane &P0 = pl[(size_t)f];
                const int v = val(f, j);
                uint64_t a = 1, bq = 1;
                for (int i = 0; i < v; ++i) bq *= P0.q;
                for (int i = v; i < P0.e; ++i) a *= P0.q;
                const size_t k = (size_t)(f * take + j);
                mm[k] = a;
                qv[k] = bq;
                ui[k] = a > 1 ? msg::Ring64::inv(hu[(size_t)(f * t + j)] % a, a) : 0;
            }
        }
        // CRT over the planes (moduli coprime, product below 2^62).
        auto crt = [&](const uint64_t *res, const uint64_t *mod, int cnt) -> uint64_t {
            uint64_t x = 0, M = 1;
            for (int f = 0; f < cnt; ++f) {
                if (mod[f] == 1) continue;
                const uint64_t xm = x % mod[f];
                const uint64_t d = (res[f] + mod[f] - xm) % mod[f];
                const uint64_t k = msg::Ring64::mulm(d, msg::Ring64::inv(M % mod[f], mod[f]), mod[f]);
                x += M * k;
                M *= mod[f];
            }
            return x;
        };
        std::vector<uint64_t> mplane((size_t)F);
        for (int f = 0; f < F; ++f) mplane[(size_t)f] = pl[(size_t)f].m;
        par(n, (double)take * F * 8.0, [&](int64_t i) {
            std::vector<uint64_t> r((size_t)F), md((size_t)F);
            for (int64_t j = 0; j < take; ++j) {
                const int64_t a = take - 1 - j;
                for (int f = 0; f < F; ++f) {
                    const size_t k = (size_t)(f * take + j);
                    md[(size_t)f] = mm[k];
                    const uint64_t pr = hPR[(size_t)((f * n + i) * take + j)];
                    r[(size_t)f] = mm[k] > 1 ? msg::Ring64::mulm((pr / qv[k]) % mm[k], ui[k], mm[k]) : 0;
                }
                b.M[(size_t)(a * n + i)] = BigInt::from_u64(crt(r.data(), md.data(), F));
                for (int f = 0; f < F; ++f) {
                    const uint64_t e = hE[(size_t)((f * take + j) * n + i)];
                    r[(size_t)f] = e ? mplane[(size_t)f] - e : 0;
                }
                b.U[(size_t)(a * n + i)] = BigInt::from_u64(crt(r.data(), mplane.data(), F));
            }
        });
        return RNS_OK;
    }

    int massager_phase2(int pidx, const BigInt &sn, SplitMix &rng, std::vector<MBatch> &B) {
        constexpr int64_t kExtra = 8;                    // projection columns beyond the batch
        B.clear();
        int64_t m = 0, r = ctx->massager_r0;
        BigInt s = sn;
        double pbits = 0;                                // log2 of the product found, from below
        for (;;) {
            // The last batch takes every remaining invariant; it needs s and the
            // projection's modulus M' (reading 21) to fit a machine word.
            const bool word = s.bit_length() <= 62;
            const bool fin = word && (sn / coprime_part(sn, s)).bit_length() <= 62;
            const int64_t room = n - m;
            // Every invariant still to come is >= 2 and their product is at
            // most H / (product found).
            const int64_t more = (int64_t)std::max(0.0, std::floor(abits - pbits)) + 1;
            int64_t t = std::min(room, more) + kExtra;
            if (!fin) t = std::min(t, r + kExtra);
            std::vector<BigInt> P1;
            DRV_ST(projection(pidx, sn, s, B, t, rng, P1));
            MBatch b;
            bool done = false;
            if (word) {
                DRV_ST(gpu_batch(P1, t, s, kExtra, fin, b, &done));
            } else {
                batch_from(msg::RingBig(s), P1, t, s, kExtra, false, b, &done);
            }
            const int64_t take = (int64_t)b.S.size();
            for (const BigInt &o : b.S) pbits += (double)o.bit_length() - 1.0;
            m += take;
            B.push_back(std::move(b));
            st.batches += 1;
            if (done || m >= n || take == 0) return RNS_OK;
            s = B.back().S.front();                      // the smallest invariant just found
            // While s is multiword the batches double (Section 2.2's schedule);
            // once s fits a word the next batch takes every remaining invariant.
            r = std::min<int64_t>(n - m, 2 * std::max(r, take));
        }
    }

    // ------------------------------------------------ Phase 3 of the massager
    // The reduced Smith massager over the m nontrivial positions n0 .. n-1
    // (position order of the output: batches newest first, each ascending):
    // row t of U reduced mod s_t, T rebuilt from it (T_ab = -U_a M_b mod s_b
    // for a < b), and the blocks G = A M S^-1 (n x m) and V = (T + U M) S^-1
    // (m x m) of the massaged matrix B of Eq. (1).  Reducing a row of U mod
    // its own s_a keeps B integral (the change of (U M)_ab is a multiple of
    // s_a, which s_b divides for b <= a, and T absorbs it for b > a) and keeps
    // det B = det A / det S; it brings the bits of row a of B's lower half to
    // about log2(n s_a), so the whole massager takes O(n log|det A|) words.
    struct Reduced {
        int64_t m = 0, n0 = 0;
        std::vector<BigInt> s;                     // s_t
        std::vector<int> w;                        // words of s_t
        std::vector<std::vector<uint64_t>> U, M;   // row t of U, column t of M: n entries of w[t] words
        std::vector<BigInt> T, V;                  // [b][a] T_ab (a < b);  [a][b] V_ab
        std::vector<int64_t> G;                    // [i][b]
    };

    static int words_of(const BigInt &x) { return (int)std::max<size_t>(1, (x.mag.size() + 1) / 2); }

    static void put_words(uint64_t *dst, int W, const BigInt &x) {
        const size_t nl = x.mag.size();
        for (int i = 0; i < W; ++i) {
            const uint64_t lo = (size_t)(2 * i) < nl ? x.mag[(size_t)(2 * i)] : 0;
            const uint64_t hi = (size_t)(2 * i + 1) < nl ? x.mag[(size_t)(2 * i + 1)] : 0;
            dst[i] = lo | (hi << 32);
        }
    }

    static BigInt from_words(const uint64_t *x, int W) {
        BigInt r(0);
        r.mag.resize((size_t)(2 * W));
        for (int i = 0; i < W; ++i) {
            r.mag[(size_t)(2 * i)] = (uint32_t)x[i];
            r.mag[(size_t)(2 * i + 1)] = (uint32_t)(x[i] >> 32);
        }
        while (!r.mag.empty() && r.mag.back() == 0) r.mag.pop_back();
        return r;
    }

    // C (r x c, W words per entry, two's complement) = A B exactly for int64
    // A (r x k) and B (k x c), |C| < 2^lb, by residue products over the first
    // aux primes and the exact CRT.
    int exact_product(const int64_t *Ah, int64_t r, int64_t k, const int64_t *Bh, int64_t c, double lb,
                      std::vector<uint64_t> &C, int &W) {
        const int L = (int)std::ceil((lb + 2.0) / 25.9);
        W = (int)std::ceil((lb + 2.0) / 64.0);
        if (L > kMaxSolvePrimes || W > 32) return RNS_ENOTSUP;
        C.assign((size_t)(r * c * W), 0);
        if (r == 0 || c == 0) return RNS_OK;
        DevBuf<int64_t> da, db;
        DevBuf<uint32_t> ra, rb, rc;
        DevBuf<uint64_t> dc;
        DRV_ST(da.alloc((size_t)(r * k)));
        DRV_ST(db.alloc((size_t)(k * c)));
        DRV_ST(ra.alloc((size_t)(L * r * k)));
        DRV_ST(rb.alloc((size_t)(L * k * c)));
        DRV_ST(rc.alloc((size_t)(L * r * c)));
        DRV_ST(dc.alloc((size_t)(r * c * W)));
        DRV_HIP(hipMemcpyAsync(da.p, Ah, sizeof(int64_t) * r * k, hipMemcpyHostToDevice, stream));
        DRV_HIP(hipMemcpyAsync(db.p, Bh, sizeof(int64_t) * k * c, hipMemcpyHostToDevice, stream));
        DRV_ST(rns_reduce(aux, da.p, r, k, k, 0, L, ra.p, k, r * k, stream));
        DRV_ST(rns_reduce(aux, db.p, k, c, c, 0, L, rb.p, c, k * c, stream));
        DRV_ST(gemm(ra.p, k, r * k, rb.p, c, k * c, rc.p, c, r * c, r, c, k, 0, L));
        DRV_ST(dstatus.alloc(1));
        DRV_HIP(hipMemsetAsync(dstatus.p, 0, sizeof(int32_t), stream));
        DRV_ST(crt_reconstruct(aux, rc.p, r, c, c, r * c, 0, L, nullptr, 0, dc.p, W, c, dstatus.p, stream));
        DRV_HIP(hipMemcpyAsync(C.data(), dc.p, sizeof(uint64_t) * r * c * W, hipMemcpyDeviceToHost, stream));
        int32_t ovf = 0;
        DRV_HIP(hipMemcpyAsync(&ovf, dstatus.p, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
        DRV_ST(sync());
        return ovf ? RNS_EOVERFLOW : RNS_OK;
    }

    // Builds the reduced massager; *integral = false when a block of B turns
    // out not to be integral (then the massager is wrong and the solve
    // restarts).
    int massager_reduce(const std::vector<MBatch> &B, Reduced &R, bool *integral) {
        *integral = true;
        int64_t m = 0;
        for (const MBatch &b : B) m += (int64_t)b.S.size();
        R = Reduced{};
        R.m = m;
        R.n0 = n - m;
        R.s.resize((size_t)m);
        R.w.resize((size_t)m);
        R.U.resize((size_t)m);
        R.M.resize((size_t)m);
        std::vector<std::pair<int, int64_t>> src((size_t)m);
        {
            int64_t t = 0;
            for (int bi = (int)B.size() - 1; bi >= 0; --bi)
                for (int64_t a = 0; a < (int64_t)B[(size_t)bi].S.size(); ++a) src[(size_t)t++] = {bi, a};
        }
        const msg::ParFor par = host_par();
        par(m, (double)n * 64, [&](int64_t t) {
            const MBatch &b = B[(size_t)src[(size_t)t].first];
            const int64_t a = src[(size_t)t].second;
            const BigInt &sa = b.S[(size_t)a];
            const int W = words_of(sa);
            R.s[(size_t)t] = sa;
            R.w[(size_t)t] = W;
            R.U[(size_t)t].assign((size_t)(n * W), 0);
            R.M[(size_t)t].assign((size_t)(n * W), 0);
            const bool word = sa.bit_length() <= 64;
            const uint64_t sw = word ? sa.to_u64_mag() : 0;
            for (int64_t k = 0; k < n; ++k) {
                const BigInt &u = b.U[(size_t)(a * n + k)];
                if (word && u.bit_length() <= 64) {
                    R.U[(size_t)t][(size_t)k] = u.to_u64_mag() % sw;
                } else {
                    put_words(R.U[(size_t)t].data() + k * W, W, mod(u, sa));
                }
                put_words(R.M[(size_t)t].data() + k * W, W, b.M[(size_t)(a * n + k)]);
            }
        });
        if (m == 0) return RNS_OK;
        // Both products on the GPU as exact residue products of 32-bit limbs:
        // position t contributes 2 w[t] limb rows of U (limb l of every entry)
        // and 2 w[t] limb columns of M, so with Ul (rows x n) and Ml (n x
        // cols), (U M)_ab = sum_{l, l'} (Ul Ml)[a_l][b_l'] 2^(32 (l + l')) and
        // (A M)_ib = sum_l' (A Ml)[i][b_l'] 2^(32 l'); every entry of the
        // products is below n 2^64 (resp. n max|a| 2^32).
        std::vector<int64_t> off((size_t)m + 1, 0);
        for (int64_t t = 0; t < m; ++t) off[(size_t)t + 1] = off[(size_t)t] + 2 * R.w[(size_t)t];
        const int64_t C = off[(size_t)m];
        std::vector<int64_t> Ul((size_t)(C * n)), Ml((size_t)(n * C));
        par(m, (double)n * 8, [&](int64_t t) {
            const int W = R.w[(size_t)t];
            for (int l = 0; l < 2 * W; ++l) {
                const int64_t r = off[(size_t)t] + l;
                for (int64_t k = 0; k < n; ++k) {
                    const uint64_t u = R.U[(size_t)t][(size_t)(k * W + l / 2)];
                    const uint64_t v = R.M[(size_t)t][(size_t)(k * W + l / 2)];
                    Ul[(size_t)(r * n + k)] = (int64_t)((l & 1) ? u >> 32 : u & 0xFFFFFFFFull);
                    Ml[(size_t)(k * C + r)] = (int64_t)((l & 1) ? v >> 32 : v & 0xFFFFFFFFull);
                }
            }
        });
        std::vector<uint64_t> PU, PA;
        int WU = 0, WA = 0;
        DRV_ST(exact_product(Ul.data(), C, n, Ml.data(), C, 64.0 + std::log2((double)n) + 1.0, PU, WU));
        DRV_ST(exact_product(A, n, n, Ml.data(), C, std::log2(std::max(amax, 1.0) * (double)n) + 33.0, PA, WA));
        std::atomic<bool> bad{false};
        // Sum of 2-word entries shifted by 32-bit limbs into 64-bit slots of
        // 32-bit digits (each slot receives at most 3 n-independent digits per
        // term, far below 2^64), then the BigInt of the slots.
        auto slots_to_big = [](std::vector<uint64_t> &sl) {
            uint64_t carry = 0;
            for (auto &v : sl) {
                const uint64_t x = v + carry;
                v = x & 0xFFFFFFFFull;
                carry = x >> 32;
            }
            BigInt b(0);
            b.mag.assign(sl.size(), 0);
            for (size_t i = 0; i < sl.size(); ++i) b.mag[i] = (uint32_t)sl[i];
            while (!b.mag.empty() && b.mag.back() == 0) b.mag.pop_back();
            return b;
        };
        // G = A M S^-1: signed sums, positive and negative parts apart.
        R.G.assign((size_t)(n * m), 0);
        par(n, (double)C * 4, [&](int64_t i) {
            std::vector<uint64_t> pos, neg;
            for (int64_t b = 0; b < m; ++b) {
                const int Wb = R.w[(size_t)b];
                pos.assign((size_t)(2 * Wb + 4), 0);
                neg.assign((size_t)(2 * Wb + 4), 0);
                for (int l = 0; l < 2 * Wb; ++l) {
                    const uint64_t *x = PA.data() + (size_t)((i * C + off[(size_t)b] + l) * WA);
                    const bool ng = (x[WA - 1] >> 63) != 0;
                    unsigned __int128 v = 0;                    // |x| < 2^100
                    for (int w = std::min(WA, 2) - 1; w >= 0; --w) v = (v << 64) | (ng ? ~x[w] : x[w]);
                    if (ng) v += 1;
                    std::vector<uint64_t> &sl = ng ? neg : pos;
                    for (int d = 0; d < 4 && v; ++d, v >>= 32) sl[(size_t)(l + d)] += (uint64_t)(v & 0xFFFFFFFFull);
                }
                const BigInt num = slots_to_big(pos) - slots_to_big(neg);
                BigInt q, r;
                BigInt::divmod_floor(num, R.s[(size_t)b], q, r);
                if (!r.is_zero() || !q.fits_i64()) bad = true;
                R.G[(size_t)(i * m + b)] = q.to_i64();
            }
        });
        // X = U M, then T and V.
        R.T.assign((size_t)(m * m), BigInt(0));
        R.V.assign((size_t)(m * m), BigInt(0));
        auto finish = [&](int64_t a, int64_t b, const BigInt &x) {
            BigInt q, r;
            BigInt::divmod_floor(x, R.s[(size_t)b], q, r);
            if (a < b) {
                if (!r.is_zero()) {
                    R.T[(size_t)(b * m + a)] = R.s[(size_t)b] - r;
                    q = q + BigInt(1);
                }
            } else if (a == b) {
                if (!(r + BigInt(1) == R.s[(size_t)b])) bad = true;
                q = q + BigInt(1);
            } else if (!r.is_zero()) {
                bad = true;
            }
            R.V[(size_t)(a * m + b)] = q;
        };
        par(m * m, (double)C, [&](int64_t e) {
            const int64_t a = e / m, b = e % m;
            const int Wa = R.w[(size_t)a], Wb = R.w[(size_t)b];
            std::vector<uint64_t> sl((size_t)(2 * Wa + 2 * Wb + 4), 0);
            for (int la = 0; la < 2 * Wa; ++la)
                for (int lb = 0; lb < 2 * Wb; ++lb) {
                    const uint64_t *x = PU.data() + (size_t)(((off[(size_t)a] + la) * C + off[(size_t)b] + lb) * WU);
                    unsigned __int128 v = x[0];                 // < n 2^64 < 2^96
                    if (WU > 1) v |= (unsigned __int128)x[1] << 64;
                    for (int d = 0; d < 4 && v; ++d, v >>= 32) sl[(size_t)(la + lb + d)] += (uint64_t)(v & 0xFFFFFFFFull);
                }
            finish(a, b, slots_to_big(sl));
        });
        *integral = !bad;
        return RNS_OK;
    }

    // Phase 3: certifies that B (Eq. (1)) of the reduced massager is
    // unimodular.  B restricted to the nontrivial positions is
    //     B' = [ A   G ]        (n + m square; a trivial position contributes
    //          [ U'  V ]         the unit row and column e_{n+i} of B, which
    //                            do not change |det B|),
    // and its lower rows are linearized in base 2^lam (each row r becomes its
    // digit rows r_0 .. r_{k-1} and k - 1 new columns with 2^lam above and
    // -1 on the digit rows' diagonal: the same |det|, unimodular exactly when
    // B' is), so that every entry is small; lam is chosen to minimise the
    // certificate's estimated product work.
    int massager_phase3(const Reduced &R, bool *ok, int64_t *dim) {
        *ok = false;
        const int64_t m = R.m;
        std::vector<int> bits((size_t)m, 1);
        double gmax = std::max(amax, 1.0);
        for (int64_t e = 0; e < n * m; ++e) gmax = std::max(gmax, std::fabs((double)R.G[(size_t)e]));
        for (int64_t t = 0; t < m; ++t) {
            int bt = 1;
            const int W = R.w[(size_t)t];
            for (int64_t k = 0; k < n; ++k) {
                const uint64_t *u = R.U[(size_t)t].data() + k * W;
                for (int w = W - 1; w >= 0; --w)
                    if (u[w]) {
                        bt = std::max(bt, 64 * w + 64 - __builtin_clzll(u[w]));
                        break;
                    }
            }
            for (int64_t b = 0; b < m; ++b) bt = std::max(bt, (int)R.V[(size_t)(t * m + b)].bit_length());
            bits[(size_t)t] = bt;
        }
        int best = 0;
        double best_cost = INFINITY;
        for (int lam = 12; lam <= 56; lam += 4) {
            int64_t N = n;
            for (int64_t t = 0; t < m; ++t) N += (bits[(size_t)t] + lam - 1) / lam;
            const double lb = std::max(std::log2(gmax), (double)lam);
            const double lbz = lb + std::log2((double)N);
            if (lbz >= 60.0 || N > kLiftMfmaMaxN) continue;
            const double lx = lbz + std::log2((double)N) + 2.0;
            const int j = (int)std::ceil(lx / 25.99), l = (int)std::ceil((lbz + 1.0) / 25.99);
            const double lh = (double)N * (lb + 0.5 * std::log2((double)N));
            const double steps = std::ceil(std::log2(lh / (j * 25.99) + 1.0)) + 1.0;
            const double cost = (double)N * N * N * (2.0 * (j + l) * steps + 2.0 * j);
            if (cost < best_cost) {
                best_cost = cost;
                best = lam;
            }
        }
        if (!best) return RNS_ENOTSUP;
        const int lam = best;
        int64_t N = n;
        std::vector<int64_t> row0((size_t)m), ext0((size_t)m);
        int64_t extra = 0;
        for (int64_t t = 0; t < m; ++t) extra += (bits[(size_t)t] + lam - 1) / lam - 1;
        for (int64_t t = 0, r = n, c = n + m; t < m; ++t) {
            row0[(size_t)t] = r;
            ext0[(size_t)t] = c;
            const int64_t k = (bits[(size_t)t] + lam - 1) / lam;
            r += k;
            c += k - 1;
        }
        N = n + m + extra;
        *dim = N;
        std::vector<int64_t> D((size_t)(N * N), 0);
        const msg::ParFor par = host_par();
        par(n, (double)N, [&](int64_t i) {
            int64_t *row = D.data() + (size_t)(i * N);
            for (int64_t k = 0; k < n; ++k) row[k] = A[i * n + k];
            for (int64_t b = 0; b < m; ++b) row[n + b] = R.G[(size_t)(i * m + b)];
        });
        const uint64_t base = 1ull << lam, mask = base - 1;
        auto digit = [&](const uint64_t *x, int W, int l) -> int64_t {
            const int bit = l * lam, w = bit / 64, o = bit % 64;
            if (w >= W) return 0;
            uint64_t v = x[w] >> o;
            if (o && w + 1 < W) v |= x[w + 1] << (64 - o);
            return (int64_t)(v & mask);
        };
        par(m, (double)N * 8, [&](int64_t t) {
            const int64_t k = (bits[(size_t)t] + lam - 1) / lam;
            const int W = R.w[(size_t)t];
            std::vector<std::vector<uint64_t>> vw((size_t)m);
            int vwid = 1;
            for (int64_t b = 0; b < m; ++b) vwid = std::max(vwid, words_of(R.V[(size_t)(t * m + b)]));
            std::vector<uint64_t> vbuf((size_t)(m * vwid), 0);
            for (int64_t b = 0; b < m; ++b) put_words(vbuf.data() + b * vwid, vwid, R.V[(size_t)(t * m + b)]);
            for (int64_t l = 0; l < k; ++l) {
                int64_t *row = D.data() + (size_t)((row0[(size_t)t] + l) * N);
                for (int64_t c = 0; c < n; ++c) row[c] = digit(R.U[(size_t)t].data() + c * W, W, (int)l);
                for (int64_t b = 0; b < m; ++b) row[n + b] = digit(vbuf.data() + b * vwid, vwid, (int)l);
                if (l > 0) row[ext0[(size_t)t] + l - 1] = -1;
                if (l < k - 1) row[ext0[(size_t)t] + l] = (int64_t)base;
            }
        });
        Driver dd;
        dd.ctx = ctx;
        dd.aux = aux;
        dd.n = N;
        dd.A = D.data();
        dd.stream = stream;
        DRV_ST(dd.dA.alloc((size_t)(N * N)));
        DRV_HIP(hipMemcpyAsync(dd.dA.p, D.data(), sizeof(int64_t) * N * N, hipMemcpyHostToDevice, stream));
        UcInfo ui;
        const int rc = dd.uc_run(-1, nullptr, ui);
        st.products += dd.st.products;
        st.residue_ops += dd.st.residue_ops;
        DRV_ST(dd.sync());
        DRV_ST(rc);
        st.uc_steps = ui.steps;
        st.uc_dim = N;
        st.t_uc_cert = ui.seconds;
        st.uc_x_primes = ui.j;
        st.uc_lambda = lam;
        *ok = ui.verdict == 1;
        return RNS_OK;
    }

    // Assembles S, U, M, T of the reduced massager (positions: the trivial
    // invariants first, then the batches newest first, each ascending).
    void massager_output(const Reduced &R, rns_smith_result *res) {
        const int64_t m = R.m, n0 = R.n0;
        res->massager = true;
        res->s.assign((size_t)n, BigInt(1).mag_words());
        res->U.assign((size_t)n, {});
        res->M.assign((size_t)n, {});
        res->T.assign((size_t)n, {});
        res->wU.assign((size_t)n, 1);
        res->wM.assign((size_t)n, 1);
        res->wT.assign((size_t)n, 1);
        const msg::ParFor par = host_par();
        par(n, (double)n * 4, [&](int64_t j) {
            if (j < n0) {                                // s_j = 1: U row 0, M column 0, T column e_j
                res->U[(size_t)j].assign((size_t)n, 0);
                res->M[(size_t)j].assign((size_t)n, 0);
                res->T[(size_t)j].assign((size_t)n, 0);
                res->T[(size_t)j][(size_t)j] = 1;
                return;
            }
            const int64_t t = j - n0;
            const int W = R.w[(size_t)t];
            res->s[(size_t)j] = R.s[(size_t)t].mag_words();
            res->wU[(size_t)j] = W;
            res->wM[(size_t)j] = W;
            res->wT[(size_t)j] = W;
            res->U[(size_t)j] = R.U[(size_t)t];
            res->M[(size_t)j] = R.M[(size_t)t];
            std::vector<uint64_t> &T = res->T[(size_t)j];
            T.assign((size_t)(n * W), 0);
            for (int64_t a = 0; a < t; ++a) put_words(T.data() + (n0 + a) * W, W, R.T[(size_t)(t * m + a)]);
            T[(size_t)(j * W)] = 1;
        });
    }

    int run_massager(rns_smith_result *res) {
        const double t0 = now_s();
        st.path = 2;
        DRV_ST(upload_a32());
        SplitMix rng{seed ^ 0x6A09E667F3BCC909ull};
        int pidx = 0;
        uint32_t detp = 0;
        double tl = now_s();
        DRV_ST(lift_prime(&pidx, &detp));
        st.t_lif += now_s() - tl;
        for (int attempt = 0; attempt <= kMaxRestarts + 3; ++attempt) {
            if (attempt) st.restarts += 1;
            // Phase 1: s_n (Monte Carlo; a proper divisor shows up in Phase 2).
            // Eight right-hand sides: a prime power that only s_n carries is
            // missed with probability at most 2^-8 (each random vector catches
            // it with probability at least 1/2), at the cost of one lifting
            // launch of up to 16 columns per step either way.
            tl = now_s();
            BigInt sn;
            std::vector<BigInt> Xp;
            const int stl = lift_solve(pidx, 8, rng, sn, Xp);
            st.t_lif += now_s() - tl;
            if (stl == RNS_EBOUND) continue;
            DRV_ST(stl);
            const double ti = now_s();
            std::vector<MBatch> B;
            st.batches = 0;
            st.columns = 0;
            const int sp = sn.is_one() ? RNS_OK : massager_phase2(pidx, sn, rng, B);
            st.t_im += now_s() - ti;
            if (sp == RNS_EBOUND) continue;
            DRV_ST(sp);
            // Phase 3: B of the reduced massager (Eq. (1)) is unimodular,
            // certified by high-order residues; where the linearized B is
            // beyond that certificate's limits, |det A| = prod s_i exactly.
            const double tu = now_s();
            bool forced = false;
            if (ctx->force_cert_failures > 0 && !B.empty()) {
                // Test hook: drop the last batch, which leaves a valid but not
                // maximal massager for the certificate to reject.
                ctx->force_cert_failures -= 1;
                B.pop_back();
                forced = true;
            }
            Reduced R;
            bool integral = true, ok = false;
            DRV_ST(massager_reduce(B, R, &integral));
            int64_t dim = 0;
            // RNS_MASSAGER_CERT=det selects the determinant certificate (the
            // form taken beyond the residue certificate's limits).
            const char *cert_env = std::getenv("RNS_MASSAGER_CERT");
            const bool det_cert = cert_env && std::strcmp(cert_env, "det") == 0;
            const int p3 = !integral ? RNS_OK : (det_cert ? RNS_ENOTSUP : massager_phase3(R, &ok, &dim));
            if (p3 == RNS_OK) {
                st.cert_kind = 1;
                if (!ok) st.uc_rejects += 1;
            } else if (p3 == RNS_ENOTSUP || p3 == RNS_EBOUND) {   // beyond the certificate's limits
                st.cert_kind = 0;
                BigInt prod(1);
                for (const BigInt &o : R.s) prod = prod * o;
                if (sn.is_one()) {
                    const BigInt one(1);
                    DRV_ST(lift_certify(pidx, detp, one, one, &ok));
                } else {
                    DRV_ST(lift_certify(pidx, detp, sn, prod, &ok));
                }
            } else {
                return p3;
            }
            st.t_uc += now_s() - tu;
            if (ok && !forced && B.empty() && ctx->force_cert_failures > 0) {
                ctx->force_cert_failures -= 1;         // no batch to drop (A unimodular)
                ok = false;
            }
            if (!ok) continue;
            const double to = now_s();
            massager_output(R, res);
            st.t_im += now_s() - to;
            st.cert_exact = 1;
            st.lift_a_bytes = a_bytes;
            st.lift_kernels = (mfma_lift() ? 1 : 0) | (mfma_lift() && a_bytes == 2 ? 2 : 0) | (a_bytes == 2 ? 8 : 0);
            st.t_total = now_s() - t0;
            res->st = st;
            return RNS_OK;
        }
        return RNS_ERETRY;
    }

    int solve_massager(rns_smith_result *res) {
        DRV_HIP(hipSetDevice(ctx->device));
        DRV_ST(solve_stream(ctx, &stream));
        DRV_ST(bounds());
        if (!lifting_applies()) return RNS_ENOTSUP;
        DRV_ST(dA.alloc((size_t)n * n));
        DRV_HIP(hipMemcpyAsync(dA.p, A, sizeof(int64_t) * n * n, hipMemcpyHostToDevice, stream));
        return run_massager(res);
    }

    // Phase 1 alone: the largest invariant factor s_n (Monte Carlo: the lcm of
    // the denominators found divides s_n and equals it with high probability).
    int run_lif(rns_smith_result *res) {
        const double t0 = now_s();
        st.path = 1;
        DRV_ST(upload_a32());
        SplitMix rng{seed ^ 0x2545F4914F6CDD1Dull};
        int pidx = 0;
        uint32_t detp = 0;
        DRV_ST(lift_prime(&pidx, &detp));
        for (int attempt = 0; attempt <= kMaxRestarts; ++attempt) {
            BigInt s;
            std::vector<BigInt> X;
            const int stl = lift_solve(pidx, 4, rng, s, X);
            if (stl == RNS_EBOUND) {
                st.restarts += 1;
                continue;
            }
            DRV_ST(stl);
            res->s.assign(1, s.mag_words());
            st.columns = 4;
            st.cert_exact = 0;
            st.t_lif = st.t_total = now_s() - t0;
            res->st = st;
            return RNS_OK;
        }
        return RNS_ERETRY;
    }

    // Hadamard's bound (log2) and the largest entry, from the host matrix:
    // 64 fixed blocks of rows on host threads, their partial sums combined in
    // block order (the result does not depend on the thread count).
    int bounds() {
        const int nb = (int)std::min<int64_t>(n, 64);
        std::vector<double> colsq((size_t)nb * n, 0.0), rowlog(nb, 0.0), amx(nb, 0.0);
        parallel_for_if(n * n >= (1 << 20), nb, [&](int b) {
            double *cs = colsq.data() + (size_t)b * n;
            double rl = 0, am = 0;
            for (int64_t i = n * b / nb; i < n * (b + 1) / nb; ++i) {
                double r = 0;
                for (int64_t j = 0; j < n; ++j) {
                    const double v = (double)A[i * n + j];
                    r += v * v;
                    cs[j] += v * v;
                    am = std::max(am, std::fabs(v));
                }
                rl += r > 0 ? 0.5 * std::log2(r) : -1e300;
            }
            rowlog[b] = rl;
            amx[b] = am;
        });
        double rows = 0, cols = 0;
        for (int b = 0; b < nb; ++b) {
            rows += rowlog[b];
            amax = std::max(amax, amx[b]);
        }
        for (int64_t j = 0; j < n; ++j) {
            double c = 0;
            for (int b = 0; b < nb; ++b) c += colsq[(size_t)b * n + j];
            cols += c > 0 ? 0.5 * std::log2(c) : -1e300;
        }
        abits = std::min(rows, cols);
        return abits > -1e299 ? RNS_OK : RNS_ESINGULAR;   // a zero row or column
    }

    bool lifting_applies() const {
        // n max|a| < 2^36, and max|a| < 2^31 for the int32 form of A.
        return n >= 16 && amax * (double)n < 68719476736.0 && amax < 2147483648.0;
    }

    int solve_lif(rns_smith_result *res) {
        DRV_HIP(hipSetDevice(ctx->device));
        DRV_ST(solve_stream(ctx, &stream));
        DRV_ST(bounds());
        if (!lifting_applies()) return RNS_ENOTSUP;
        DRV_ST(dA.alloc((size_t)n * n));
        DRV_HIP(hipMemcpyAsync(dA.p, A, sizeof(int64_t) * n * n, hipMemcpyHostToDevice, stream));
        return run_lif(res);
    }

    // Chooses the path: residues of s A^-1 while its sizes fit the CRT of 64
    // primes, p-adic lifting beyond when the entries are small enough.
    // ---------------------------------------------- unimodularity certificate
    // Section 2.2, Phase 3: whether D = this matrix (n x n, host A, device dA)
    // is unimodular, from high-order X-adic residues computed by
    // double-plus-one steps (Z_0 = I; Z -> (Z Z - D cmod(C Z Z, X)) / X with
    // C = D^-1 mod X): Z_e = 0 at precision X^e proves D^-1 integral, and for
    // a unimodular D it holds once X^e >= 4 H, H Hadamard's bound on the
    // (n-1)-minors.  X = p_0 .. p_{j-1} >= 4 n^2 max|D| keeps |Z| <= n max|D|;
    // Z's exact value comes from l further primes with product > 2 n max|D|.
    // Every product is a residue product of n x n x n (Z Z on j + l planes,
    // C Y on j, D K on l); k_uc_convert and k_uc_tail do the rest.
    struct UcInfo {
        int verdict = -1, reason = 0, steps = 0, steps_needed = 0, j = 0, l = 0;
        uint32_t P[kUcMaxPrimes]{}, Q[kUcMaxPrimes]{};
        double log2_bound = 0, log2_x = 0, seconds = 0;
    };
    enum { kUcVanished = 0, kUcNonzero = 1, kUcSingularModX = 2, kUcZeroColumn = 3, kUcStepLimit = 4 };

    int uc_run(int max_steps, int64_t *Z_host, UcInfo &info) {
        const double t0 = now_s();
        info = UcInfo{};
        const int64_t N = n;
        if (N == 0) {
            info.verdict = 1;
            return RNS_OK;
        }
        if (N > kLiftMfmaMaxN) return RNS_ENOTSUP;
        // max|D| and the column norms.
        uint64_t dmax = 0;
        std::vector<double> col2((size_t)N, 0.0);
        for (int64_t i = 0; i < N; ++i)
            for (int64_t c = 0; c < N; ++c) {
                const int64_t v = A[i * N + c];
                if (v == INT64_MIN) return RNS_EINVAL;
                const uint64_t a = (uint64_t)(v < 0 ? -v : v);
                dmax = std::max(dmax, a);
                col2[(size_t)c] += (double)v * (double)v;
            }
        double lsum = 0, lmin = INFINITY;
        for (int64_t c = 0; c < N; ++c) {
            if (col2[(size_t)c] == 0.0) {
                info.verdict = 0;
                info.reason = kUcZeroColumn;
                return RNS_OK;
            }
            const double l2 = 0.5 * std::log2(col2[(size_t)c]);
            lsum += l2;
            lmin = std::min(lmin, l2);
        }
        // Rounding of the double sums: a relative 2^-40 per column is far more
        // than the error of n additions of squares below 2^126.
        info.log2_bound = N > 1 ? (lsum - lmin) * (1.0 + 1e-12) + 1e-6 * N : 0.0;
        using u128 = unsigned __int128;
        const u128 beta_z = (u128)dmax * (u128)N;
        if (beta_z >= ((u128)1 << 61)) return RNS_EBOUND;
        const u128 need_x = 4 * beta_z * (u128)N;
        // X and Q from the first aux primes.
        UcBasis b{};
        u128 X = 1, Qp = 1;
        int idx = 0;
        while (X < need_x) {
            if (b.j == kUcMaxPrimes) return RNS_EBOUND;
            b.p[b.j++] = aux->primes[idx++];
            X *= b.p[b.j - 1];
        }
        while (Qp <= 2 * beta_z) {
            if (b.l == kUcMaxPrimes) return RNS_EBOUND;
            b.q[b.l++] = aux->primes[idx++];
            Qp *= b.q[b.l - 1];
        }
        auto inv = [](uint64_t a, uint64_t m) { return (uint32_t)powmod_u64(a % m, m - 2, m); };
        auto digits = [](u128 v, const uint32_t *m, int k, uint32_t *d) {
            for (int i = 0; i < k; ++i) {
                d[i] = (uint32_t)(v % m[i]);
                v /= m[i];
            }
        };
        for (int a = 0; a < b.j; ++a)
            for (int c = a + 1; c < b.j; ++c) b.pinv[a][c] = inv(b.p[a], b.p[c]);
        for (int a = 0; a < b.l; ++a)
            for (int c = a + 1; c < b.l; ++c) b.qinv[a][c] = inv(b.q[a], b.q[c]);
        digits((X - 1) / 2, b.p, b.j, b.phalf);
        digits((Qp - 1) / 2, b.q, b.l, b.qhalf);
        for (int k = 0; k < b.l; ++k) {
            b.x_mod_q[k] = (uint32_t)(X % b.q[k]);
            b.xinv_q[k] = inv(b.x_mod_q[k], b.q[k]);
        }
        b.bound = (int64_t)beta_z;
        info.j = b.j;
        info.l = b.l;
        for (int i = 0; i < b.j; ++i) info.P[i] = b.p[i];
        for (int i = 0; i < b.l; ++i) info.Q[i] = b.q[i];
        info.log2_x = 0;
        for (int i = 0; i < b.j; ++i) info.log2_x += std::log2((double)b.p[i]);
        {
            const double need = (info.log2_bound + 2.0) / info.log2_x;
            int k = 0;
            while ((double)((1ll << k) - 1) < need) ++k;
            info.steps_needed = k;
        }
        const int steps = max_steps >= 0 ? max_steps : info.steps_needed;
        // C = D^-1 mod p_i (right halves of dM).
        base = 0;
        int bad = -1;
        DRV_ST(invert(b.j, &bad));
        if (bad >= 0) {
            info.verdict = 0;
            info.reason = kUcSingularModX;
            info.seconds = now_s() - t0;
            return RNS_OK;
        }
        const int L = b.j + b.l;
        const int64_t ps = N * N;
        DevBuf<int64_t> dZ;
        DevBuf<uint32_t> dZr, dYr, dKr, dDq;
        DevBuf<int32_t> dfl;
        DRV_ST(dZ.alloc((size_t)ps));
        DRV_ST(dZr.alloc((size_t)L * ps));
        DRV_ST(dYr.alloc((size_t)L * ps));
        DRV_ST(dKr.alloc((size_t)L * ps));
        DRV_ST(dDq.alloc((size_t)b.l * ps));
        DRV_ST(dfl.alloc(2));
        DRV_ST(rns_reduce(aux, dA.p, N, N, N, b.j, b.l, dDq.p, N, ps, stream));
        launch_uc_identity(dZ.p, N, stream);
        DRV_HIP(hipGetLastError());
        DRV_ST(rns_reduce(aux, dZ.p, N, N, N, 0, L, dZr.p, N, ps, stream));
        int32_t fl[2] = {1, 0};
        int run = 0;
        for (run = 0; run < steps; ++run) {
            DRV_ST(gemm(dZr.p, N, ps, dZr.p, N, ps, dYr.p, N, ps, N, N, N, 0, L));          // Y = Z Z
            DRV_ST(gemm(dM.p + N, 2 * N, 2 * N * N, dYr.p, N, ps, dKr.p, N, ps, N, N, N, 0, b.j));  // C Y mod p
            launch_uc_convert(dKr.p, dKr.p + (size_t)b.j * ps, ps, ps, b, stream);
            DRV_HIP(hipGetLastError());
            rns_gemm_desc d{};                                                             // Y - D K mod q
            d.m = N; d.n = N; d.k = N;
            d.A = dDq.p; d.lda = N; d.a_plane_stride = ps;
            d.B = dKr.p + (size_t)b.j * ps; d.ldb = N; d.b_plane_stride = ps;
            d.C = dYr.p + (size_t)b.j * ps; d.ldc = N; d.c_plane_stride = ps;
            d.prime_begin = b.j; d.L = b.l;
            d.flags = RNS_GEMM_SUBTRACT;
            DRV_ST(modmatmul_batched(aux, &d, 1, RNS_PATH_AUTO, stream));
            st.products += 1;
            st.residue_ops += 2.0 * N * N * N * b.l;
            DRV_HIP(hipMemsetAsync(dfl.p, 0, sizeof(int32_t) * 2, stream));
            launch_uc_tail(dYr.p + (size_t)b.j * ps, dZ.p, ps, ps, b, dfl.p, stream);
            DRV_HIP(hipGetLastError());
            DRV_HIP(hipMemcpyAsync(fl, dfl.p, sizeof(fl), hipMemcpyDeviceToHost, stream));
            DRV_ST(sync());
            if (fl[1]) return RNS_EBOUND;          // |Z| beyond n max|D|: the bound argument failed
            if (!fl[0]) {
                ++run;
                break;
            }
            if (run + 1 < steps) DRV_ST(rns_reduce(aux, dZ.p, N, N, N, 0, L, dZr.p, N, ps, stream));
        }
        info.steps = run;
        if (!fl[0]) {
            info.verdict = 1;
            info.reason = kUcVanished;
        } else if (run >= info.steps_needed) {
            info.verdict = 0;
            info.reason = kUcNonzero;
        } else {
            info.verdict = -1;
            info.reason = kUcStepLimit;
        }
        if (Z_host) {
            DRV_HIP(hipMemcpyAsync(Z_host, dZ.p, sizeof(int64_t) * ps, hipMemcpyDeviceToHost, stream));
            DRV_ST(sync());
        }
        info.seconds = now_s() - t0;
        return RNS_OK;
    }

    int solve(rns_smith_result *res) {
        DRV_HIP(hipSetDevice(ctx->device));
        DRV_ST(solve_stream(ctx, &stream));
        DRV_ST(bounds());
        DRV_ST(dA.alloc((size_t)n * n));
        DRV_HIP(hipMemcpyAsync(dA.p, A, sizeof(int64_t) * n * n, hipMemcpyHostToDevice, stream));
        const int mode = ctx->smith_path;
        const bool fits_residues = 2.0 * abits + std::log2((double)n) + 64.0 < kMaxSolvePrimes * 25.9;
        if (mode == 2 || (mode == 0 && !fits_residues && lifting_applies())) {
            if (!lifting_applies()) return RNS_ENOTSUP;
            return run_lifting(res);
        }
        return run(res);
    }
};

int aux_ctx(rns_ctx *ctx, rns_ctx **out) {
    std::lock_guard<std::mutex> g(ctx->mu);
    if (!ctx->aux) {
        int st = rns_ctx_create(&ctx->aux, ctx->device, nullptr, kAuxPrimes, ctx->flags);
        if (st != RNS_OK) return st;
    }
    *out = ctx->aux;
    return RNS_OK;
}

}  // namespace

extern "C" int smith_form(rns_ctx *ctx, const int64_t *A_host, int64_t n, uint64_t seed,
                          rns_smith_result **out) {
    if (!ctx || !out || n < 0 || (n > 0 && !A_host)) return RNS_EINVAL;
    *out = nullptr;
    rns_smith_result *res = new (std::nothrow) rns_smith_result;
    if (!res) return RNS_ENOMEM;
    if (n == 0) {
        *out = res;
        return RNS_OK;
    }
    if (n == 1) {
        const int64_t a = A_host[0];
        if (a == 0) {
            delete res;
            return RNS_ESINGULAR;
        }
        res->s.push_back(BigInt(a < 0 ? -a : a).mag_words());
        *out = res;
        return RNS_OK;
    }
    for (int64_t e = 0; e < n * n; ++e)
        if (A_host[e] == INT64_MIN) {         // |a| must fit in int64
            delete res;
            return RNS_EINVAL;
        }
    SolveScope scope(ctx);   // outlives the driver and its buffers
    Driver d;
    d.ctx = ctx;
    d.n = n;
    d.A = A_host;
    d.seed = seed;
    int st = aux_ctx(ctx, &d.aux);
    if (st == RNS_OK) {
        TraceScope trace(ctx, d.aux);
        st = d.solve(res);
        res->st.t_host_cpu = trace.cpu_s();
    }
    if (st != RNS_OK) {
        delete res;
        return st;
    }
    *out = res;
    return RNS_OK;
}

extern "C" int rns_largest_invariant(rns_ctx *ctx, const int64_t *A_host, int64_t n, uint64_t seed,
                                     rns_smith_result **out) {
    if (!ctx || !out || n < 0 || (n > 0 && !A_host)) return RNS_EINVAL;
    *out = nullptr;
    for (int64_t e = 0; e < n * n; ++e)
        if (A_host[e] == INT64_MIN) return RNS_EINVAL;
    rns_smith_result *res = new (std::nothrow) rns_smith_result;
    if (!res) return RNS_ENOMEM;
    SolveScope scope(ctx);
    Driver d;
    d.ctx = ctx;
    d.n = n;
    d.A = A_host;
    d.seed = seed;
    int st = aux_ctx(ctx, &d.aux);
    if (st == RNS_OK) {
        TraceScope trace(ctx, d.aux);
        st = d.solve_lif(res);
        res->st.t_host_cpu = trace.cpu_s();
    }
    if (st != RNS_OK) {
        delete res;
        return st;
    }
    *out = res;
    return RNS_OK;
}

extern "C" int rns_smith_massager(rns_ctx *ctx, const int64_t *A_host, int64_t n, uint64_t seed,
                                  rns_smith_result **out) {
    if (!ctx || !out || n < 0 || (n > 0 && !A_host)) return RNS_EINVAL;
    *out = nullptr;
    for (int64_t e = 0; e < n * n; ++e)
        if (A_host[e] == INT64_MIN) return RNS_EINVAL;
    rns_smith_result *res = new (std::nothrow) rns_smith_result;
    if (!res) return RNS_ENOMEM;
    if (n == 0) {
        res->massager = true;
        *out = res;
        return RNS_OK;
    }
    SolveScope scope(ctx);
    Driver d;
    d.ctx = ctx;
    d.n = n;
    d.A = A_host;
    d.seed = seed;
    int st = aux_ctx(ctx, &d.aux);
    if (st == RNS_OK) {
        TraceScope trace(ctx, d.aux);
        st = d.solve_massager(res);
        res->st.t_host_cpu = trace.cpu_s();
    }
    if (st != RNS_OK) {
        delete res;
        return st;
    }
    *out = res;
    return RNS_OK;
}

extern "C" int rns_unimodular_certify(rns_ctx *ctx, const int64_t *D_host, int64_t n, int max_steps,
                                      int64_t *Z_host, rns_unimod_info *info) {
    if (!ctx || !info || n < 0 || (n > 0 && !D_host)) return RNS_EINVAL;
    std::memset(info, 0, sizeof(*info));
    SolveScope scope(ctx);
    Driver d;
    d.ctx = ctx;
    d.n = n;
    d.A = D_host;
    int st = aux_ctx(ctx, &d.aux);
    Driver::UcInfo ui;
    if (st == RNS_OK) {
        TraceScope trace(ctx, d.aux);
        st = [&]() -> int {
            DRV_HIP(hipSetDevice(ctx->device));
            DRV_ST(solve_stream(ctx, &d.stream));
            if (n > 0) {
                DRV_ST(d.dA.alloc((size_t)n * n));
                DRV_HIP(hipMemcpyAsync(d.dA.p, D_host, sizeof(int64_t) * n * n, hipMemcpyHostToDevice, d.stream));
            }
            return d.uc_run(max_steps, Z_host, ui);
        }();
    }
    if (st != RNS_OK) return st;
    info->verdict = ui.verdict;
    info->reason = ui.reason;
    info->steps = ui.steps;
    info->steps_needed = ui.steps_needed;
    info->x_primes = ui.j;
    info->q_primes = ui.l;
    for (int i = 0; i < 4; ++i) {
        info->x_prime[i] = ui.P[i];
        info->q_prime[i] = ui.Q[i];
    }
    info->log2_bound = ui.log2_bound;
    info->log2_x = ui.log2_x;
    info->seconds = ui.seconds;
    info->residue_ops = d.st.residue_ops;
    info->products = d.st.products;
    return RNS_OK;
}

extern "C" int rns_smith_massager_width(const rns_smith_result *r, int which, int64_t index) {
    if (!r || !r->massager || index < 0 || index >= (int64_t)r->s.size()) return -RNS_EINVAL;
    switch (which) {
    case RNS_MASSAGER_U: return r->wU[(size_t)index];
    case RNS_MASSAGER_M: return r->wM[(size_t)index];
    case RNS_MASSAGER_T: return r->wT[(size_t)index];
    default: return -RNS_EINVAL;
    }
}

extern "C" int rns_smith_massager_vector(const rns_smith_result *r, int which, int64_t index, uint64_t *out,
                                         int W) {
    const int w = rns_smith_massager_width(r, which, index);
    if (w < 0 || !out || W < 1) return RNS_EINVAL;
    if (W < w) return RNS_EBOUND;
    const std::vector<uint64_t> &src = which == RNS_MASSAGER_U ? r->U[(size_t)index]
                                       : which == RNS_MASSAGER_M ? r->M[(size_t)index]
                                                                 : r->T[(size_t)index];
    const int64_t n = (int64_t)r->s.size();
    for (int64_t k = 0; k < n; ++k)
        for (int i = 0; i < W; ++i) out[(size_t)(k * W + i)] = i < w ? src[(size_t)(k * w + i)] : 0;
    return RNS_OK;
}

extern "C" int rns_smith_get(const rns_smith_result *r, int64_t i, const uint64_t **words,
                             int *nwords) {
    if (!r || !words || !nwords || i < 0 || i >= (int64_t)r->s.size()) return RNS_EINVAL;
    *words = r->s[i].data();
    *nwords = (int)r->s[i].size();
    return RNS_OK;
}

extern "C" int64_t rns_smith_size(const rns_smith_result *r) { return r ? (int64_t)r->s.size() : 0; }

extern "C" int rns_smith_stats_get(const rns_smith_result *r, rns_smith_stats *st) {
    if (!r || !st) return RNS_EINVAL;
    *st = r->st;
    return RNS_OK;
}

extern "C" void rns_smith_free(rns_smith_result *r) { delete r; }
