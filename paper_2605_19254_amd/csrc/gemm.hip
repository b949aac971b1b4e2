// modmatmul_batched: one exact residue product per prime and per problem
// (Section 3.1: the product of two integer matrices becomes L independent
// word-size products, each exact, then reduced mod p).
//
// The host side builds one problem table for the whole batch: every problem
// gets a slice of the context workspace for its tiled operands and a range of
// work-group tiles.  One prep launch converts all operands of all problems
// (uint32 residues -> INT8 digit tiles or balanced FP64 tiles) and one GEMM
// launch computes every tile of every prime of every problem.
#include "gemm_common.hpp"

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

using namespace rns;
using namespace rns::gemm;

namespace {

struct Plan {
    std::vector<GemmProblem> probs;
    size_t work_bytes = 0;
    int64_t total_tiles = 0;
    int64_t total_units = 0;
    bool from_int64 = false;
    int64_t total_units64 = 0;
    double residue_ops = 0;
    int64_t max_dim = 0;
    bool fused = false;          // both primes per tile and the CRT in the GEMM launch
};

int check_desc(const rns_ctx *ctx, const rns_gemm_desc &x, const GemmInt64Src *src) {
    if (x.m < 0 || x.n < 0 || x.k < 0 || x.L < 0) return RNS_EINVAL;
    if ((x.flags & ~RNS_GEMM_SUBTRACT) != 0 || x.reserved != 0) return RNS_EINVAL;
    if (x.prime_begin < 0 || x.prime_begin + x.L > ctx->L) return RNS_EINVAL;
    if (x.m > INT32_MAX / 2 || x.n > INT32_MAX / 2 || x.k > INT32_MAX / 2) return RNS_EINVAL;
    if (x.m == 0 || x.n == 0 || x.L == 0) return RNS_OK;
    // An int64 result given with the source (a plan that may fuse the CRT)
    // stands in for the residue planes of C.
    if ((!x.C && !(src && src->C)) || x.ldc < x.n) return RNS_EINVAL;
    if (x.L > 1 && x.c_plane_stride < (x.m - 1) * x.ldc + x.n) return RNS_EINVAL;
    if (x.k > 0 && src) {
        if (!src->A || !src->B || src->lda < x.k || src->ldb < x.n) return RNS_EINVAL;
    } else if (x.k > 0) {
        if (!x.A || !x.B || x.lda < x.k || x.ldb < x.n) return RNS_EINVAL;
        if (x.L > 1 && (x.a_plane_stride < (x.m - 1) * x.lda + x.k ||
                        x.b_plane_stride < (x.k - 1) * x.ldb + x.n))
            return RNS_EINVAL;
    }
    return RNS_OK;
}

// Builds the problem table.  Problems are ordered by decreasing tile cost
// (k, then m*n), so that a persistent launch hands out the longest tiles
// first; workspace offsets are relative (the caller adds the base).  With
// `fuse` (INT8, int64 sources with int64 results, at most two primes each)
// a tile covers every prime of its problem.
int make_plan(rns_ctx *ctx, const rns_gemm_desc *d, int count, bool int8, Plan &plan,
              const GemmInt64Src *src = nullptr, bool fuse = false) {
    const int TM = int8 ? kI8TileM : kF64TileM;
    const int TN = int8 ? kI8TileN : kF64TileN;
    const int64_t elem = int8 ? 4 : 8;   // bytes per operand entry in the tiled layout
    std::vector<int> order;
    for (int i = 0; i < count; ++i) {
        int st = check_desc(ctx, d[i], src ? &src[i] : nullptr);
        if (st != RNS_OK) return st;
        if (d[i].m == 0 || d[i].n == 0 || d[i].L == 0) continue;
        if (int8 && d[i].k > kInt8MaxK) return RNS_EBOUND;
        order.push_back(i);
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        if (d[a].k != d[b].k) return d[a].k > d[b].k;
        return d[a].m * d[a].n > d[b].m * d[b].n;
    });
    size_t off = 0;
    for (int i : order) {
        const rns_gemm_desc &x = d[i];
        GemmProblem g{};
        g.A = x.A; g.B = x.B; g.C = x.C;
        g.lda = x.lda; g.aps = x.a_plane_stride;
        g.ldb = x.ldb; g.bps = x.b_plane_stride;
        g.ldc = x.ldc; g.cps = x.c_plane_stride;
        g.m = (int32_t)x.m; g.n = (int32_t)x.n; g.k = (int32_t)x.k;
        g.L = x.L; g.prime_begin = x.prime_begin;
        g.sub = (x.flags & RNS_GEMM_SUBTRACT) ? 1 : 0;
        const int64_t Mp = round_up(x.m, TM), Np = round_up(x.n, TN);
        const int64_t Kp = round_up(std::max<int64_t>(x.k, 1), kKTile);
        g.RB = (int32_t)(Mp / 16); g.CB = (int32_t)(Np / 16); g.KT = (int32_t)(Kp / kKTile);
        g.tm = (int32_t)(Mp / TM); g.tn = (int32_t)(Np / TN);
        // 32-bit tile and conversion-unit indices inside a problem
        if ((int64_t)g.L * g.tm * g.tn >= ((int64_t)1 << 31) ||
            (int64_t)g.L * (g.RB + g.CB) * g.KT >= ((int64_t)1 << 31))
            return RNS_EINVAL;
        g.a_plane_bytes = Mp * Kp * elem;
        g.b_plane_bytes = Np * Kp * elem;
        g.At = reinterpret_cast<char *>(off);
        off += (size_t)g.a_plane_bytes * g.L;
        g.Bt = reinterpret_cast<char *>(off);
        off += (size_t)g.b_plane_bytes * g.L;
        off = (off + 255) & ~(size_t)255;
        g.tile_begin = plan.total_tiles;
        plan.total_tiles += (fuse ? 1 : (int64_t)g.L) * g.tm * g.tn;
        if (fuse) {
            g.C64 = src[i].C;
            g.ldc64 = src[i].ldc;
            if (g.L == 2) {
                const uint64_t p0 = ctx->primes[x.prime_begin], p1 = ctx->primes[x.prime_begin + 1];
                g.crt_inv = (uint32_t)invmod_u64(p0 % p1, p1);
            }
        }
        g.unitA_begin = plan.total_units;
        g.unitB_begin = g.unitA_begin + (int64_t)g.L * g.RB * g.KT;
        plan.total_units = g.unitB_begin + (int64_t)g.L * g.CB * g.KT;
        if (src) {
            g.A64 = src[i].A; g.lda64 = src[i].lda;
            g.B64 = src[i].B; g.ldb64 = src[i].ldb;
            g.u64A_begin = plan.total_units64;
            g.u64B_begin = g.u64A_begin + (int64_t)g.RB * g.KT;
            plan.total_units64 = g.u64B_begin + (int64_t)g.CB * g.KT;
        }
        plan.residue_ops += 2.0 * x.m * x.n * x.k * x.L;
        plan.max_dim = std::max<int64_t>(plan.max_dim, std::max(x.m, std::max(x.n, x.k)));
        plan.probs.push_back(g);
    }
    plan.work_bytes = off;
    plan.from_int64 = src != nullptr;
    plan.fused = fuse;
    return RNS_OK;
}

// Whether a plan of int64 products can fuse the CRT into its GEMM launch:
// INT8 path, every problem with an int64 result and at most two primes.
bool can_fuse(const rns_ctx *ctx, const rns_gemm_desc *d, const GemmInt64Src *src, int count, bool int8) {
    if (!src || !int8 || ctx->separate_crt) return false;
    for (int i = 0; i < count; ++i)
        if (d[i].m > 0 && d[i].n > 0 && d[i].L > 0 && (d[i].L > 2 || !src[i].C || src[i].ldc < d[i].n))
            return false;
    return true;
}

// Plans for a path; AUTO takes INT8 unless k exceeds its exactness bound.
int make_plan_path(rns_ctx *ctx, const rns_gemm_desc *d, int count, int path, bool &int8, Plan &plan,
                   const GemmInt64Src *src = nullptr) {
    if (path == RNS_PATH_AUTO) path = ctx->auto_path;
    int8 = path != RNS_PATH_FP64;
    int st = make_plan(ctx, d, count, int8, plan, src);
    if (st == RNS_EBOUND && path == RNS_PATH_AUTO) {
        int8 = false;
        plan = Plan();
        st = make_plan(ctx, d, count, int8, plan, src);
    }
    return st;
}

int ilog2_ceil(double x) {
    int e = 0;
    while (x > 1.0) { x /= 2.0; ++e; }
    return e;
}

// Shape class of a batch for the autotuner: path, number of problems, largest
// dimension and total residue work, each on a log2 scale.
std::string tune_key(bool int8, const Plan &plan) {
    char buf[128];
    std::snprintf(buf, sizeof buf, "gfx950/%s/count%d/dim%d/ops%d", int8 ? "int8" : "fp64",
                  ilog2_ceil((double)plan.probs.size()), ilog2_ceil((double)plan.max_dim),
                  ilog2_ceil(plan.residue_ops));
    return buf;
}

int choose_variant(rns_ctx *ctx, bool int8, const Plan &plan) {
    if (!int8) return 0;
    if (ctx->int8_kernel >= 0) return ctx->int8_kernel;
    auto it = ctx->tune.find(tune_key(int8, plan));
    return it != ctx->tune.end() ? it->second : kI8Default;
}

// units: conversion units (per prime and tile, or per tile for int64 operands).
int run_plan(rns_ctx *ctx, bool int8, int variant, const GemmProblem *dP, int np, int64_t tiles,
             int64_t units, const int32_t *tile_prob, unsigned *counter, hipStream_t s,
             bool from_int64 = false, bool fused = false) {
    const bool persistent = int8 && !fused && variant == kI8HalfPersistent;
    if (from_int64) {
        ProfScope ps(ctx, int8 ? "k_prep_i64_i8" : "k_prep_i64_f64", s);
        launch_prep_i64(int8, dP, np, units, (const PrimeConst *)ctx->d_prime,
                        persistent ? counter : nullptr, s);
    } else {
        ProfScope ps(ctx, int8 ? "k_prep_i8" : "k_prep_f64", s);
        launch_prep(int8, dP, np, units, (const PrimeConst *)ctx->d_prime,
                    persistent ? counter : nullptr, s);
    }
    RNS_HIP(hipGetLastError());
    if (fused) {
        ProfScope ps(ctx, "k_gemm_i8", s);
        launch_gemm_i8_crt(dP, np, tiles, (const PrimeConst *)ctx->d_prime, tile_prob, s);
    } else {
        ProfScope ps(ctx, int8 ? "k_gemm_i8" : "k_gemm_f64", s);
        if (int8)
            launch_gemm_i8(variant, dP, np, tiles, (const PrimeConst *)ctx->d_prime, tile_prob,
                           counter, ctx->num_cus, s);
        else
            launch_gemm_f64(dP, np, tiles, (const PrimeConst *)ctx->d_prime, tile_prob, s);
    }
    RNS_HIP(hipGetLastError());
    return RNS_OK;
}

}  // namespace

// ------------------------------------------------------------------ plans --

struct rns_gemm_plan {
    rns_ctx *ctx = nullptr;
    bool int8 = true;
    bool from_int64 = false;        // operands are int64 matrices (conversion reduces them)
    bool fused = false;             // the GEMM launch also does the CRT into int64 results
    int variant = 0;
    int nprob = 0;
    int64_t total_tiles = 0, total_units = 0;
    size_t work_bytes = 0;
    double residue_ops = 0;
    std::string key;
    GemmProblem *d_probs = nullptr;
    int32_t *d_tile_prob = nullptr;
    void *d_work = nullptr;
    unsigned *d_counter = nullptr;
};

extern "C" void rns_gemm_plan_destroy(rns_gemm_plan *p) {
    if (!p) return;
    (void)hipSetDevice(p->ctx->device);
    (void)hipDeviceSynchronize();
    if (p->d_probs) (void)hipFree(p->d_probs);
    if (p->d_tile_prob) (void)hipFree(p->d_tile_prob);
    if (p->d_work) (void)hipFree(p->d_work);
    if (p->d_counter) (void)hipFree(p->d_counter);
    delete p;
}

namespace {

int gemm_plan_create(rns_ctx *ctx, const rns_gemm_desc *descs, const GemmInt64Src *src, int count, int path,
                     rns_gemm_plan **out) {
    if (!ctx || !out || count < 0 || (count > 0 && !descs)) return RNS_EINVAL;
    if (path != RNS_PATH_AUTO && path != RNS_PATH_FP64 && path != RNS_PATH_INT8) return RNS_EINVAL;
    *out = nullptr;
    bool int8 = true;
    Plan plan;
    int st = make_plan_path(ctx, descs, count, path, int8, plan, src);
    if (st != RNS_OK) return st;
    if (can_fuse(ctx, descs, src, count, int8)) {
        plan = Plan();
        st = make_plan(ctx, descs, count, int8, plan, src, true);
        if (st != RNS_OK) return st;
    }
    rns_gemm_plan *p = new (std::nothrow) rns_gemm_plan;
    if (!p) return RNS_ENOMEM;
    p->ctx = ctx;
    p->int8 = int8;
    p->from_int64 = plan.from_int64;
    p->fused = plan.fused;
    p->nprob = (int)plan.probs.size();
    p->total_tiles = plan.total_tiles;
    p->total_units = plan.from_int64 ? plan.total_units64 : plan.total_units;
    p->work_bytes = plan.work_bytes;
    p->residue_ops = plan.residue_ops;
    p->key = tune_key(int8, plan);
    {
        std::lock_guard<std::mutex> guard(ctx->mu);
        p->variant = choose_variant(ctx, int8, plan);
    }
    auto fail = [&](int s) { rns_gemm_plan_destroy(p); return s; };
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(RNS_EDEVICE);
    if (p->nprob > 0) {
        if (hipMalloc(&p->d_work, std::max<size_t>(plan.work_bytes, 256)) != hipSuccess) return fail(RNS_ENOMEM);
        for (auto &g : plan.probs) {
            g.At = static_cast<char *>(p->d_work) + reinterpret_cast<size_t>(g.At);
            g.Bt = static_cast<char *>(p->d_work) + reinterpret_cast<size_t>(g.Bt);
        }
        const size_t tbytes = sizeof(GemmProblem) * plan.probs.size();
        if (hipMalloc(&p->d_probs, tbytes) != hipSuccess) return fail(RNS_ENOMEM);
        if (hipMemcpy(p->d_probs, plan.probs.data(), tbytes, hipMemcpyHostToDevice) != hipSuccess)
            return fail(RNS_EDEVICE);
        if (p->nprob > 1) {
            std::vector<int32_t> tp((size_t)plan.total_tiles);
            for (int q = 0; q < p->nprob; ++q) {
                const int64_t end = q + 1 < p->nprob ? plan.probs[q + 1].tile_begin : plan.total_tiles;
                for (int64_t t = plan.probs[q].tile_begin; t < end; ++t) tp[(size_t)t] = q;
            }
            if (hipMalloc(&p->d_tile_prob, tp.size() * sizeof(int32_t)) != hipSuccess) return fail(RNS_ENOMEM);
            if (hipMemcpy(p->d_tile_prob, tp.data(), tp.size() * sizeof(int32_t), hipMemcpyHostToDevice) !=
                hipSuccess)
                return fail(RNS_EDEVICE);
        }
        if (hipMalloc(&p->d_counter, sizeof(unsigned)) != hipSuccess) return fail(RNS_ENOMEM);
        if (hipMemset(p->d_counter, 0, sizeof(unsigned)) != hipSuccess) return fail(RNS_EDEVICE);
    }
    *out = p;
    return RNS_OK;
}

}  // namespace

extern "C" int rns_gemm_plan_create(rns_ctx *ctx, const rns_gemm_desc *descs, int count, int path,
                                    rns_gemm_plan **out) {
    return gemm_plan_create(ctx, descs, nullptr, count, path, out);
}

namespace rns {
int gemm_plan_create_int64(rns_ctx *ctx, const rns_gemm_desc *descs, const GemmInt64Src *src, int count,
                           int path, rns_gemm_plan **out) {
    if (count > 0 && !src) return RNS_EINVAL;
    return gemm_plan_create(ctx, descs, src, count, path, out);
}
bool gemm_plan_fused_crt(const rns_gemm_plan *p) { return p && p->fused; }
}  // namespace rns

extern "C" int rns_gemm_plan_execute(rns_gemm_plan *p, void *stream) {
    if (!p) return RNS_EINVAL;
    if (p->nprob == 0) return RNS_OK;
    RNS_HIP(hipSetDevice(p->ctx->device));
    return run_plan(p->ctx, p->int8, p->variant, p->d_probs, p->nprob, p->total_tiles,
                    p->total_units, p->d_tile_prob, p->d_counter, (hipStream_t)stream, p->from_int64,
                    p->fused);
}

extern "C" int rns_gemm_plan_info(const rns_gemm_plan *p, rns_plan_info *info) {
    if (!p || !info) return RNS_EINVAL;
    info->path = p->int8 ? RNS_PATH_INT8 : RNS_PATH_FP64;
    info->variant = p->fused ? RNS_I8_HALF_CRT : p->variant;
    info->tiles = p->total_tiles;
    info->workspace_bytes = p->work_bytes;
    info->residue_ops = p->residue_ops;
    return RNS_OK;
}

extern "C" int rns_gemm_plan_set_variant(rns_gemm_plan *p, int variant) {
    if (!p || variant < 0 || (p->int8 ? variant >= kI8NumVariants : variant != 0)) return RNS_EINVAL;
    if (p->fused) return RNS_EINVAL;   // one kernel form
    p->variant = variant;
    return RNS_OK;
}

// ------------------------------------------------------------- autotuner --

namespace {

void tune_store(rns_ctx *ctx, const std::string &key, int variant) {
    ctx->tune[key] = variant;
    if (!ctx->tune_path.empty()) {
        if (FILE *f = std::fopen(ctx->tune_path.c_str(), "a")) {
            std::fprintf(f, "%s %d\n", key.c_str(), variant);
            std::fclose(f);
        }
    }
}

}  // namespace

extern "C" int rns_ctx_set_tune_cache(rns_ctx *ctx, const char *path) {
    if (!ctx) return RNS_EINVAL;
    std::lock_guard<std::mutex> guard(ctx->mu);
    ctx->tune_path = path ? path : "";
    if (ctx->tune_path.empty()) return RNS_OK;
    if (FILE *f = std::fopen(ctx->tune_path.c_str(), "r")) {
        char key[256];
        int v = 0;
        while (std::fscanf(f, "%255s %d", key, &v) == 2)
            if (v >= 0 && v < kI8NumVariants) ctx->tune[key] = v;   // later lines win
        std::fclose(f);
    }
    return RNS_OK;
}

extern "C" int rns_gemm_plan_autotune(rns_gemm_plan *p, void *stream, int *variant_out) {
    if (!p || !variant_out) return RNS_EINVAL;
    if (p->fused) {   // one kernel form: nothing to choose
        *variant_out = RNS_I8_HALF_CRT;
        return RNS_OK;
    }
    rns_ctx *ctx = p->ctx;
    hipStream_t s = (hipStream_t)stream;
    int best = p->variant, st = RNS_OK;
    if (p->int8 && p->nprob > 0) {
        hipEvent_t a = nullptr, b = nullptr;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return RNS_EDEVICE;
        float best_ms = 1e30f;
        for (int v = 0; v < kI8NumVariants && st == RNS_OK; ++v) {
            p->variant = v;
            st = rns_gemm_plan_execute(p, stream);            // warm-up
            if (st != RNS_OK) break;
            float tot = 0.f;
            for (int r = 0; r < 3 && st == RNS_OK; ++r) {
                float ms = 0.f;
                if (hipEventRecord(a, s) != hipSuccess) { st = RNS_EDEVICE; break; }
                st = rns_gemm_plan_execute(p, stream);
                if (st != RNS_OK) break;
                if (hipEventRecord(b, s) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
                    hipEventElapsedTime(&ms, a, b) != hipSuccess) {
                    st = RNS_EDEVICE;
                    break;
                }
                tot += ms;
            }
            if (st == RNS_OK && tot < best_ms) {
                best_ms = tot;
                best = v;
            }
        }
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
    }
    if (st != RNS_OK) return st;
    p->variant = best;
    {
        std::lock_guard<std::mutex> guard(ctx->mu);
        tune_store(ctx, p->key, best);
    }
    *variant_out = best;
    return RNS_OK;
}

extern "C" int rns_autotune(rns_ctx *ctx, const rns_gemm_desc *descs, int count, int path,
                            void *stream, int *variant_out) {
    if (!ctx || !variant_out) return RNS_EINVAL;
    rns_gemm_plan *p = nullptr;
    int st = rns_gemm_plan_create(ctx, descs, count, path, &p);
    if (st != RNS_OK) return st;
    st = rns_gemm_plan_autotune(p, stream, variant_out);
    rns_gemm_plan_destroy(p);
    return st;
}

// ------------------------------------------------- one-shot batched call --

extern "C" int rns_workspace_bytes(rns_ctx *ctx, const rns_gemm_desc *descs, int count,
                                   int path, size_t *bytes) {
    if (!ctx || !bytes || count < 0 || (count > 0 && !descs)) return RNS_EINVAL;
    bool int8 = true;
    Plan plan;
    int st = make_plan_path(ctx, descs, count, path, int8, plan);
    if (st != RNS_OK) return st;
    *bytes = plan.work_bytes;
    return RNS_OK;
}

extern "C" int modmatmul_batched(rns_ctx *ctx, const rns_gemm_desc *descs, int count,
                                 int path, void *stream) {
    if (!ctx || count < 0 || (count > 0 && !descs)) return RNS_EINVAL;
    if (path != RNS_PATH_AUTO && path != RNS_PATH_FP64 && path != RNS_PATH_INT8) return RNS_EINVAL;
    if (count == 0) return RNS_OK;
    std::lock_guard<std::mutex> guard(ctx->mu);
    bool int8 = true;
    Plan plan;
    int st = make_plan_path(ctx, descs, count, path, int8, plan);
    if (st != RNS_OK) return st;
    if (plan.probs.empty()) return RNS_OK;
    RNS_HIP(hipSetDevice(ctx->device));
    st = ensure_workspace(ctx, plan.work_bytes);
    if (st != RNS_OK) return st;
    for (auto &g : plan.probs) {
        g.At = static_cast<char *>(ctx->d_work) + reinterpret_cast<size_t>(g.At);
        g.Bt = static_cast<char *>(ctx->d_work) + reinterpret_cast<size_t>(g.Bt);
    }
    const size_t tbytes = sizeof(GemmProblem) * plan.probs.size();
    st = ensure_desc(ctx, tbytes);
    if (st != RNS_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    // Next slot of the problem-table ring: its previous call (copy and
    // kernels) must have finished before the slot is overwritten, which after
    // kDescRing calls it normally has, so consecutive calls do not wait for
    // each other.
    const int k = ctx->desc_next;
    ctx->desc_next = (k + 1) % kDescRing;
    RNS_HIP(hipEventSynchronize(ctx->desc_ev[k]));
    char *h = static_cast<char *>(ctx->h_desc) + (size_t)k * ctx->desc_bytes;
    char *dd = static_cast<char *>(ctx->d_desc) + (size_t)k * ctx->desc_bytes;
    std::memcpy(h, plan.probs.data(), tbytes);
    RNS_HIP(hipMemcpyAsync(dd, h, tbytes, hipMemcpyHostToDevice, s));
    const int variant = choose_variant(ctx, int8, plan);
    st = run_plan(ctx, int8, variant, reinterpret_cast<const GemmProblem *>(dd), (int)plan.probs.size(),
                  plan.total_tiles, plan.total_units, nullptr, ctx->d_counter, s);
    if (st != RNS_OK) return st;
    RNS_HIP(hipEventRecord(ctx->desc_ev[k], s));
    return RNS_OK;
}

// ------------------------------------------ allocation-free batched call --
// modmatmul_batched_noalloc keeps its scratch (tiled operands, problem table,
// work counter) in this fixed array instead of the context's growable
// workspace.  Each device holds its own copy; host code reaches it only
// through the address hipGetSymbolAddress returns for that device (kept in
// g_scratch), never through the array's name.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch[kScratchDevices] = {};

size_t round256(size_t x) { return (x + 255) & ~(size_t)255; }
}  // namespace

namespace rns {
// Called by rns_ctx_create with `device` current.  A failure leaves the
// device without scratch; only modmatmul_batched_noalloc reports it.
int scratch_init(int device) {
    if (device < 0 || device >= kScratchDevices) return RNS_EDEVICE;
    std::lock_guard<std::mutex> guard(g_scratch_mu);
    if (g_scratch[device]) return RNS_OK;
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return RNS_EDEVICE;
    }
    g_scratch[device] = static_cast<unsigned char *>(ptr);
    return RNS_OK;
}
}  // namespace rns

extern "C" int rns_noalloc_scratch_bytes(size_t *bytes) {
    if (!bytes) return RNS_EINVAL;
    *bytes = kScratchBytes;
    return RNS_OK;
}

extern "C" int modmatmul_batched_noalloc(rns_ctx *ctx, const rns_gemm_desc *descs, int count, int path,
                                         void *stream) {
    if (!ctx || count < 0 || (count > 0 && !descs)) return RNS_EINVAL;
    if (path != RNS_PATH_AUTO && path != RNS_PATH_FP64 && path != RNS_PATH_INT8) return RNS_EINVAL;
    if (count == 0) return RNS_OK;
    std::lock_guard<std::mutex> guard(ctx->mu);
    bool int8 = true;
    Plan plan;
    int st = make_plan_path(ctx, descs, count, path, int8, plan);
    if (st != RNS_OK) return st;
    if (plan.probs.empty()) return RNS_OK;
    unsigned char *base = nullptr;
    {
        std::lock_guard<std::mutex> g(g_scratch_mu);
        if (ctx->device >= 0 && ctx->device < kScratchDevices) base = g_scratch[ctx->device];
    }
    if (!base) return RNS_EDEVICE;
    // Layout: tiled operands, then the problem table, then the work counter.
    const size_t work = round256(plan.work_bytes);
    const size_t tbytes = sizeof(GemmProblem) * plan.probs.size();
    const size_t need = work + round256(tbytes) + 256;
    if (need > kScratchBytes) return RNS_ESCRATCH;
    RNS_HIP(hipSetDevice(ctx->device));
    for (auto &g : plan.probs) {
        g.At = reinterpret_cast<char *>(base) + reinterpret_cast<size_t>(g.At);
        g.Bt = reinterpret_cast<char *>(base) + reinterpret_cast<size_t>(g.Bt);
    }
    GemmProblem *table = reinterpret_cast<GemmProblem *>(base + work);
    unsigned *counter = reinterpret_cast<unsigned *>(base + work + round256(tbytes));
    hipStream_t s = (hipStream_t)stream;
    // The table's host copy belongs to this call: the copy must be complete
    // before returning, so the stream is synchronised once after it (the
    // launches below stay asynchronous).  The persistent variant's counter is
    // cleared by the conversion launch before the GEMM reads it.
    RNS_HIP(hipMemcpyAsync(table, plan.probs.data(), tbytes, hipMemcpyHostToDevice, s));
    RNS_HIP(hipStreamSynchronize(s));
    const int variant = choose_variant(ctx, int8, plan);
    return run_plan(ctx, int8, variant, table, (int)plan.probs.size(), plan.total_tiles, plan.total_units,
                    nullptr, counter, s);
}
