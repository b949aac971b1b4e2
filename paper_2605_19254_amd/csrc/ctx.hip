// Context, basis and precomputed constants (Section 3.1, the bullets on the
// choice of primes and on precomputed RNS constants), status codes and the
// small host-side multiword helpers the constants need.
#include "internal.hpp"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>

using namespace rns;

// ------------------------------------------------------------ host helpers --

namespace rns {

uint64_t mulmod_u64(uint64_t a, uint64_t b, uint64_t m) {
    return (uint64_t)((unsigned __int128)a * b % m);
}

uint64_t powmod_u64(uint64_t a, uint64_t e, uint64_t m) {
    uint64_t r = 1 % m;
    a %= m;
    while (e) {
        if (e & 1) r = mulmod_u64(r, a, m);
        a = mulmod_u64(a, a, m);
        e >>= 1;
    }
    return r;
}

uint64_t invmod_u64(uint64_t a, uint64_t m) {   // Fermat; m prime
    return powmod_u64(a % m, m - 2, m);
}

void limbs_trim(Limbs &a) {
    while (!a.empty() && a.back() == 0) a.pop_back();
}

void limbs_mul_small(Limbs &a, uint32_t m) {
    uint64_t carry = 0;
    for (auto &w : a) {
        uint64_t t = (uint64_t)w * m + carry;
        w = (uint32_t)t;
        carry = t >> 32;
    }
    if (carry) a.push_back((uint32_t)carry);
}

uint32_t limbs_divmod_small(Limbs &a, uint32_t d) {
    uint64_t rem = 0;
    for (size_t i = a.size(); i-- > 0;) {
        uint64_t cur = (rem << 32) | a[i];
        a[i] = (uint32_t)(cur / d);
        rem = cur % d;
    }
    limbs_trim(a);
    return (uint32_t)rem;
}

uint32_t limbs_mod_small(const Limbs &a, uint32_t d) {
    uint64_t rem = 0;
    for (size_t i = a.size(); i-- > 0;) rem = ((rem << 32) | a[i]) % d;
    return (uint32_t)rem;
}

int limbs_cmp(const Limbs &x, const Limbs &y) {
    Limbs a = x, b = y;
    limbs_trim(a);
    limbs_trim(b);
    if (a.size() != b.size()) return a.size() < b.size() ? -1 : 1;
    for (size_t i = a.size(); i-- > 0;)
        if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
    return 0;
}

}  // namespace rns

static bool is_prime_u32(uint32_t x) {
    if (x < 2) return false;
    if (x % 2 == 0) return x == 2;
    for (uint32_t d = 3; (uint64_t)d * d <= x; d += 2)
        if (x % d == 0) return false;
    return true;
}

// ------------------------------------------------------------------ status --

extern "C" const char *rns_strerror(int s) {
    switch (s) {
    case RNS_OK: return "ok";
    case RNS_EINVAL: return "invalid argument";
    case RNS_ENOMEM: return "out of memory";
    case RNS_EDEVICE: return "HIP device error";
    case RNS_EBOUND: return "exactness bound violated";
    case RNS_EOVERFLOW: return "result does not fit the output words";
    case RNS_ESINGULAR: return "matrix is singular";
    case RNS_ERETRY: return "Las Vegas restart budget exhausted";
    case RNS_ENOTSUP: return "not supported by this build";
    case RNS_EPENDING: return "request still running";
    case RNS_ESCRATCH: return "request exceeds the fixed scratch of the allocation-free entry point";
    default: return "unknown status";
    }
}

extern "C" int rns_primes_below(uint64_t bound, int count, uint32_t *out) {
    if (count < 0 || (count > 0 && !out) || bound > (1ull << 32)) return RNS_EINVAL;
    int got = 0;
    for (uint64_t x = bound; got < count;) {
        if (x <= 2) return RNS_EINVAL;
        --x;
        if (is_prime_u32((uint32_t)x)) out[got++] = (uint32_t)x;
    }
    return RNS_OK;
}

// ----------------------------------------------------------------- context --

static void fill_prime_const(uint32_t p, PrimeConst &c) {
    c.p = p;
    c.half = (p - 1) / 2;
    c.pf = (double)p;
    c.pinv = 1.0 / (double)p;
    c.c21 = (double)powmod_u64(2, 21, p);
    c.c42 = (double)powmod_u64(2, 42, p);
    for (int s = 0; s < 7; ++s) {
        uint64_t w = powmod_u64(2, 8 * s, p);
        int64_t b = (w > c.half) ? (int64_t)w - (int64_t)p : (int64_t)w;
        c.w[s] = (double)b;
    }
}

extern "C" int rns_ctx_create(rns_ctx **out, int device, const uint32_t *primes,
                              int L, uint64_t flags) {
    if (!out || L < 1 || L > kMaxPrimes) return RNS_EINVAL;
    if ((flags & ~(uint64_t)(3 | RNS_CTX_SEPARATE_CRT)) != 0 || (flags & 3) == 3) return RNS_EINVAL;
    *out = nullptr;
    std::vector<uint32_t> ps(L);
    if (primes) {
        std::copy(primes, primes + L, ps.begin());
    } else {
        int st = rns_primes_below(kPrimeLimit, L, ps.data());
        if (st != RNS_OK) return st;
    }
    {
        std::vector<uint32_t> sorted = ps;
        std::sort(sorted.begin(), sorted.end());
        for (int i = 0; i < L; ++i) {
            if (sorted[i] < 3 || sorted[i] >= kPrimeLimit || !is_prime_u32(sorted[i]))
                return RNS_EINVAL;
            if (i && sorted[i] == sorted[i - 1]) return RNS_EINVAL;
        }
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return RNS_EDEVICE;
    rns_ctx *ctx = new (std::nothrow) rns_ctx;
    if (!ctx) return RNS_ENOMEM;
    ctx->device = device;
    ctx->L = L;
    ctx->flags = flags;
    ctx->separate_crt = (flags & RNS_CTX_SEPARATE_CRT) != 0;
    ctx->auto_path = (flags & 3) == RNS_CTX_PATH_FP64 ? RNS_PATH_FP64
                   : (flags & 3) == RNS_CTX_PATH_INT8 ? RNS_PATH_INT8 : RNS_PATH_AUTO;
    if (const char *e = std::getenv("RNS_INT8_KERNEL")) ctx->int8_kernel = std::atoi(e);
    if (const char *e = std::getenv("RNS_LIFT_VECTOR")) ctx->lift_vector_only = std::atoi(e) != 0;
    if (const char *e = std::getenv("RNS_CRT_GARNER")) ctx->crt_garner = std::atoi(e) != 0;
    if (const char *e = std::getenv("RNS_CRT_FORM")) {
        const std::string f(e);
        ctx->crt_form = f == "limbs" ? 0 : (f == "garner" ? 2 : 1);
    }
    if (ctx->crt_garner) ctx->crt_form = 2;
    if (const char *e = std::getenv("RNS_MASSAGER_R0")) ctx->massager_r0 = std::max(1, std::atoi(e));
    ctx->primes = ps;

    std::vector<PrimeConst> pc(L);
    for (int j = 0; j < L; ++j) fill_prime_const(ps[j], pc[j]);
    std::vector<double> garner((size_t)L * kCrtMaxL, 0.0);
    for (int j = 0; j < L; ++j)
        for (int d = 1; d < kCrtMaxL && d <= j; ++d)
            garner[(size_t)j * kCrtMaxL + d] = (double)invmod_u64(ps[j - d] % ps[j], ps[j]);

    int st = RNS_OK;
    auto fail = [&](int s) { rns_ctx_destroy(ctx); return s; };
    if (hipSetDevice(device) != hipSuccess) return fail(RNS_EDEVICE);
    if (hipMalloc(&ctx->d_prime, sizeof(PrimeConst) * L) != hipSuccess) return fail(RNS_ENOMEM);
    if (hipMalloc(&ctx->d_garner, sizeof(double) * garner.size()) != hipSuccess) return fail(RNS_ENOMEM);
    if (hipMalloc(&ctx->d_status, sizeof(int32_t)) != hipSuccess) return fail(RNS_ENOMEM);
    if (hipMemcpy(ctx->d_prime, pc.data(), sizeof(PrimeConst) * L, hipMemcpyHostToDevice) != hipSuccess)
        return fail(RNS_EDEVICE);
    if (hipMemcpy(ctx->d_garner, garner.data(), sizeof(double) * garner.size(), hipMemcpyHostToDevice) != hipSuccess)
        return fail(RNS_EDEVICE);
    if (hipMemset(ctx->d_status, 0, sizeof(int32_t)) != hipSuccess) return fail(RNS_EDEVICE);
    if (hipMalloc(&ctx->d_counter, sizeof(unsigned)) != hipSuccess) return fail(RNS_ENOMEM);
    if (hipMemset(ctx->d_counter, 0, sizeof(unsigned)) != hipSuccess) return fail(RNS_EDEVICE);
    (void)scratch_init(device);   // modmatmul_batched_noalloc reports a failure here
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
            ctx->num_cus = prop.multiProcessorCount;
    }
    (void)st;
    *out = ctx;
    return RNS_OK;
}

extern "C" void rns_ctx_destroy(rns_ctx *ctx) {
    if (!ctx) return;
    if (ctx->aux) rns_ctx_destroy(ctx->aux);
    // Teardown is best effort: errors cannot be reported from here.
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->solve_stream) (void)hipStreamDestroy(ctx->solve_stream);
    for (auto &kv : ctx->solve_pool) (void)hipFree(kv.second);
    if (ctx->d_prime) (void)hipFree(ctx->d_prime);
    if (ctx->d_garner) (void)hipFree(ctx->d_garner);
    if (ctx->d_status) (void)hipFree(ctx->d_status);
    if (ctx->d_counter) (void)hipFree(ctx->d_counter);
    if (ctx->d_work) (void)hipFree(ctx->d_work);
    if (ctx->d_desc) (void)hipFree(ctx->d_desc);
    if (ctx->h_desc) (void)hipHostFree(ctx->h_desc);
    for (int k = 0; k < kDescRing; ++k)
        if (ctx->desc_ev[k]) (void)hipEventDestroy(ctx->desc_ev[k]);
    for (auto &kv : ctx->lagrange) {
        if (kv.second.d_c) (void)hipFree(kv.second.d_c);
        if (kv.second.d_mj) (void)hipFree(kv.second.d_mj);
        if (kv.second.d_m) (void)hipFree(kv.second.d_m);
    }
    for (auto &kv : ctx->digit_tables) kv.second.release();
    for (auto &kv : ctx->mr_half)
        if (kv.second) (void)hipFree(kv.second);
    delete ctx;
}

extern "C" int rns_ctx_num_primes(const rns_ctx *ctx) { return ctx ? ctx->L : 0; }

extern "C" int rns_ctx_primes(const rns_ctx *ctx, uint32_t *out) {
    if (!ctx || !out) return RNS_EINVAL;
    std::copy(ctx->primes.begin(), ctx->primes.end(), out);
    return RNS_OK;
}

namespace rns {

int ensure_workspace(rns_ctx *ctx, size_t bytes) {
    if (bytes <= ctx->work_bytes) return RNS_OK;
    RNS_HIP(hipSetDevice(ctx->device));
    if (ctx->d_work) {
        RNS_HIP(hipDeviceSynchronize());
        (void)hipFree(ctx->d_work);
        ctx->d_work = nullptr;
        ctx->work_bytes = 0;
    }
    size_t want = (bytes + 0xFFFFF) & ~(size_t)0xFFFFF;   // 1 MiB granules
    RNS_HIP(hipMalloc(&ctx->d_work, want));
    ctx->work_bytes = want;
    return RNS_OK;
}

int ensure_desc(rns_ctx *ctx, size_t bytes) {
    if (bytes <= ctx->desc_bytes) return RNS_OK;
    RNS_HIP(hipSetDevice(ctx->device));
    RNS_HIP(hipDeviceSynchronize());
    if (ctx->d_desc) (void)hipFree(ctx->d_desc);
    if (ctx->h_desc) (void)hipHostFree(ctx->h_desc);
    ctx->d_desc = nullptr;
    ctx->h_desc = nullptr;
    ctx->desc_bytes = 0;
    size_t want = (std::max<size_t>(bytes * 2, 4096) + 255) & ~(size_t)255;
    RNS_HIP(hipMalloc(&ctx->d_desc, want * kDescRing));
    RNS_HIP(hipHostMalloc(&ctx->h_desc, want * kDescRing, hipHostMallocDefault));
    for (int k = 0; k < kDescRing; ++k)
        if (!ctx->desc_ev[k]) RNS_HIP(hipEventCreateWithFlags(&ctx->desc_ev[k], hipEventDisableTiming));
    ctx->desc_bytes = want;
    return RNS_OK;
}

// Lagrange constants of the primes range [begin, begin+L) for W output words.
// Built on first use with copies on the caller's stream `s` (never the null
// stream, which would synchronise with other threads' streams).
int lagrange_table(rns_ctx *ctx, int begin, int L, int W, const LagrangeTable **out, hipStream_t s) {
    auto key = std::make_tuple(begin, L, W);
    auto it = ctx->lagrange.find(key);
    if (it != ctx->lagrange.end()) {
        *out = &it->second;
        return RNS_OK;
    }
    LagrangeTable t;
    Limbs M{1};
    for (int j = 0; j < L; ++j) limbs_mul_small(M, ctx->primes[begin + j]);
    t.M = M;
    std::vector<double> c(L);
    std::vector<uint64_t> mj((size_t)L * W, 0), m(W, 0);
    auto low_words = [W](const Limbs &x, uint64_t *dst) {
        for (int w = 0; w < W; ++w) {
            uint64_t lo = (size_t)(2 * w) < x.size() ? x[2 * w] : 0;
            uint64_t hi = (size_t)(2 * w + 1) < x.size() ? x[2 * w + 1] : 0;
            dst[w] = lo | (hi << 32);
        }
    };
    for (int j = 0; j < L; ++j) {
        uint32_t p = ctx->primes[begin + j];
        Limbs q = M;
        limbs_divmod_small(q, p);                       // M / p_j
        uint32_t r = limbs_mod_small(q, p);
        c[j] = (double)invmod_u64(r, p);
        low_words(q, &mj[(size_t)j * W]);
    }
    low_words(M, m.data());
    RNS_HIP(hipSetDevice(ctx->device));
    RNS_HIP(hipMalloc(&t.d_c, sizeof(double) * L));
    RNS_HIP(hipMalloc(&t.d_mj, sizeof(uint64_t) * L * W));
    RNS_HIP(hipMalloc(&t.d_m, sizeof(uint64_t) * W));
    RNS_HIP(hipMemcpyAsync(t.d_c, c.data(), sizeof(double) * L, hipMemcpyHostToDevice, s));
    RNS_HIP(hipMemcpyAsync(t.d_mj, mj.data(), sizeof(uint64_t) * L * W, hipMemcpyHostToDevice, s));
    RNS_HIP(hipMemcpyAsync(t.d_m, m.data(), sizeof(uint64_t) * W, hipMemcpyHostToDevice, s));
    RNS_HIP(hipStreamSynchronize(s));                  // the host vectors end with this call
    auto res = ctx->lagrange.emplace(key, std::move(t));
    *out = &res.first->second;
    return RNS_OK;
}

// Mixed-radix digits h_j of (M-1)/2 for the range: (M-1)/2 = sum_j h_j * prod_{i<j} p_i.
int mixed_radix_half(rns_ctx *ctx, int begin, int L, const uint32_t **out, hipStream_t s) {
    auto key = std::make_pair(begin, L);
    auto it = ctx->mr_half.find(key);
    if (it != ctx->mr_half.end()) {
        *out = it->second;
        return RNS_OK;
    }
    Limbs M{1};
    for (int j = 0; j < L; ++j) limbs_mul_small(M, ctx->primes[begin + j]);
    Limbs h = M;
    limbs_divmod_small(h, 2);                          // (M-1)/2 since M is odd
    std::vector<uint32_t> dig(L);
    for (int j = 0; j < L; ++j) dig[j] = limbs_divmod_small(h, ctx->primes[begin + j]);
    uint32_t *d = nullptr;
    RNS_HIP(hipSetDevice(ctx->device));
    RNS_HIP(hipMalloc(&d, sizeof(uint32_t) * L));
    ctx->mr_half[key] = d;
    RNS_HIP(hipMemcpyAsync(d, dig.data(), sizeof(uint32_t) * L, hipMemcpyHostToDevice, s));
    RNS_HIP(hipStreamSynchronize(s));
    *out = d;
    return RNS_OK;
}

}  // namespace rns

extern "C" int rns_ctx_reserve(rns_ctx *ctx, size_t bytes) {
    if (!ctx) return RNS_EINVAL;
    std::lock_guard<std::mutex> g(ctx->mu);
    return ensure_workspace(ctx, bytes);
}

extern "C" int rns_primes_for_bound(const rns_ctx *ctx, const uint64_t *bound_words,
                                    int W, int *L_out) {
    if (!ctx || !L_out || W < 0 || (W > 0 && !bound_words)) return RNS_EINVAL;
    Limbs twob1;
    for (int w = 0; w < W; ++w) {
        twob1.push_back((uint32_t)bound_words[w]);
        twob1.push_back((uint32_t)(bound_words[w] >> 32));
    }
    limbs_mul_small(twob1, 2);
    // + 1
    {
        size_t i = 0;
        for (;; ++i) {
            if (i == twob1.size()) { twob1.push_back(1); break; }
            if (++twob1[i] != 0) break;
        }
    }
    Limbs M{1};
    for (int j = 0; j < ctx->L; ++j) {
        limbs_mul_small(M, ctx->primes[j]);
        if (limbs_cmp(M, twob1) >= 0) {
            *L_out = j + 1;
            return RNS_OK;
        }
    }
    return RNS_EBOUND;
}

extern "C" int rns_ctx_status(rns_ctx *ctx, void *stream) {
    if (!ctx) return RNS_EINVAL;
    RNS_HIP(hipSetDevice(ctx->device));
    RNS_HIP(hipStreamSynchronize((hipStream_t)stream));
    int32_t h = 0;
    RNS_HIP(hipMemcpy(&h, ctx->d_status, sizeof(int32_t), hipMemcpyDeviceToHost));
    if (h) RNS_HIP(hipMemset(ctx->d_status, 0, sizeof(int32_t)));
    return h ? RNS_EOVERFLOW : RNS_OK;
}

extern "C" int rns_ctx_set_smith_path(rns_ctx *ctx, int path) {
    if (!ctx || path < 0 || path > 2) return RNS_EINVAL;
    ctx->smith_path = path;
    return RNS_OK;
}

extern "C" int rns_ctx_force_cert_failures(rns_ctx *ctx, int count) {
    if (!ctx || count < 0) return RNS_EINVAL;
    ctx->force_cert_failures = count;
    return RNS_OK;
}

// ----------------------------------------------------------------- tracing --

namespace rns {

thread_local rns_ctx *tl_trace = nullptr;

ProfScope::ProfScope(rns_ctx *c, const char *n, hipStream_t st, int64_t k)
    : ctx(c), name(n), s(st), launches(k) {
    if (!ctx || !ctx->prof) return;
    if (hipEventCreate(&a) != hipSuccess) { a = nullptr; return; }
    if (hipEventRecord(a, s) != hipSuccess) { (void)hipEventDestroy(a); a = nullptr; }
}

ProfScope::~ProfScope() {
    if (!a) return;
    hipEvent_t b = nullptr;
    if (hipEventCreate(&b) != hipSuccess || hipEventRecord(b, s) != hipSuccess) {
        (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
        return;
    }
    rns_ctx *sink = ctx->prof_sink ? ctx->prof_sink : ctx;
    std::lock_guard<std::mutex> g(sink->prof_mu);
    sink->prof_recs.push_back({name, a, b, launches});
}

}  // namespace rns

extern "C" int rns_ctx_profile(rns_ctx *ctx, int enable) {
    if (!ctx) return RNS_EINVAL;
    ctx->prof = enable != 0;
    return RNS_OK;
}

extern "C" int rns_ctx_profile_read(rns_ctx *ctx, const char *name, double *total_ms,
                                    int64_t *launches) {
    if (!ctx || !total_ms || !launches) return RNS_EINVAL;
    RNS_HIP(hipSetDevice(ctx->device));
    std::lock_guard<std::mutex> g(ctx->prof_mu);
    double tot = 0.0;
    int64_t cnt = 0;
    std::vector<rns_ctx::ProfRec> keep;
    int st = RNS_OK;
    for (auto &r : ctx->prof_recs) {
        const bool match = !name || !*name || std::strstr(r.name, name) != nullptr;
        if (!match) {
            keep.push_back(r);
            continue;
        }
        float ms = 0.f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess)
            st = RNS_EDEVICE;
        tot += ms;
        cnt += r.launches;
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    ctx->prof_recs.swap(keep);
    *total_ms = tot;
    *launches = cnt;
    return st;
}
