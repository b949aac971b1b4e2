// Whole-product plans: int64 A and B -> per-prime products -> CRT for a batch
// of independent integer products (Section 3.1 end to end).  The conversion
// kernel of the plan's gemm plan reduces A and B straight into the tiled
// operand layouts (no residue planes of A and B are written); the residue
// planes of every C stay resident in a plan-owned buffer for the CRT.  Plans
// of one-word results with at most two primes per problem instead let the
// GEMM launch do the CRT (no C planes, two launches per execution).
#include "reduce_crt.hpp"

#include <algorithm>
#include <new>
#include <vector>

using namespace rns;

struct rns_matmul_plan {
    rns_ctx *ctx = nullptr;
    int W = 1;
    int crt_E = 1;              // CRT entries per thread (the same for every job)
    bool fast_crt = false;
    bool fused = false;         // the gemm plan writes C itself
    void *d_planes = nullptr;
    CrtJob *d_cjobs = nullptr;
    int nc = 0;
    int64_t ctiles = 0;
    rns_gemm_plan *gemm = nullptr;
};

extern "C" void rns_matmul_plan_destroy(rns_matmul_plan *p) {
    if (!p) return;
    (void)hipSetDevice(p->ctx->device);
    (void)hipDeviceSynchronize();
    if (p->gemm) rns_gemm_plan_destroy(p->gemm);
    if (p->d_planes) (void)hipFree(p->d_planes);
    if (p->d_cjobs) (void)hipFree(p->d_cjobs);
    delete p;
}

extern "C" int rns_matmul_plan_create(rns_ctx *ctx, const rns_matmul_desc *d, int count, int path,
                                      int W, rns_matmul_plan **out) {
    if (!ctx || !out || count < 0 || (count > 0 && !d)) return RNS_EINVAL;
    if (W < 1 || W > kCrtMaxW) return RNS_EINVAL;
    *out = nullptr;
    // Validate and lay out the resident C planes.
    std::vector<size_t> offC(count);
    size_t off = 0;
    bool all_fast = count > 0;
    int max_L = 1;
    for (int i = 0; i < count; ++i) {
        const rns_matmul_desc &x = d[i];
        if (x.m < 0 || x.n < 0 || x.k < 0) return RNS_EINVAL;
        if (x.L < 1 || x.L > kCrtMaxL || x.prime_begin < 0 || x.prime_begin + x.L > ctx->L)
            return RNS_EINVAL;
        if (x.m > 0 && x.n > 0) {
            if (!x.C || x.ldc < x.n) return RNS_EINVAL;
            if (x.k > 0 && (!x.A || !x.B || x.lda < x.k || x.ldb < x.n)) return RNS_EINVAL;
        }
        offC[i] = off;
        off += ((size_t)x.L * x.m * x.n * sizeof(uint32_t) + 255) & ~(size_t)255;
        if (!(x.bound > 0 && crt_fast_ok(ctx, x.prime_begin, x.L, &x.bound, 1, W))) all_fast = false;
        max_L = std::max(max_L, x.L);
    }
    rns_matmul_plan *p = new (std::nothrow) rns_matmul_plan;
    if (!p) return RNS_ENOMEM;
    p->ctx = ctx;
    p->W = W;
    if (W == 1 && max_L <= 2 && path != RNS_PATH_FP64 && !ctx->separate_crt) {
        // The gemm plan fuses the CRT when its path resolves to INT8.
        std::vector<rns_gemm_desc> gd;
        std::vector<GemmInt64Src> src;
        for (int i = 0; i < count; ++i) {
            const rns_matmul_desc &x = d[i];
            if (x.m == 0 || x.n == 0) continue;
            rns_gemm_desc g{};
            g.m = x.m; g.n = x.n; g.k = x.k;
            g.prime_begin = x.prime_begin; g.L = x.L;
            g.ldc = x.n; g.c_plane_stride = x.m * x.n;   // no residue planes: the int64 C below
            gd.push_back(g);
            src.push_back(GemmInt64Src{x.A, x.lda, x.B, x.ldb, reinterpret_cast<int64_t *>(x.C), x.ldc});
        }
        int st = gemm_plan_create_int64(ctx, gd.data(), src.data(), (int)gd.size(), path, &p->gemm);
        if (st != RNS_OK) { delete p; return st; }
        if (gemm_plan_fused_crt(p->gemm) || gd.empty()) {
            p->fused = true;
            *out = p;
            return RNS_OK;
        }
        rns_gemm_plan_destroy(p->gemm);
        p->gemm = nullptr;
    }
    p->fast_crt = all_fast;
    p->crt_E = crt_entries(all_fast, W, max_L);
    auto fail = [&](int s) { rns_matmul_plan_destroy(p); return s; };
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(RNS_EDEVICE);
    if (hipMalloc(&p->d_planes, std::max<size_t>(off, 256)) != hipSuccess) return fail(RNS_ENOMEM);
    char *base = static_cast<char *>(p->d_planes);

    std::vector<rns_gemm_desc> gd;
    std::vector<GemmInt64Src> src;
    std::vector<CrtJob> cj;
    int64_t ct = 0;
    for (int i = 0; i < count; ++i) {
        const rns_matmul_desc &x = d[i];
        if (x.m == 0 || x.n == 0) continue;
        uint32_t *C = reinterpret_cast<uint32_t *>(base + offC[i]);
        rns_gemm_desc g{};
        g.m = x.m; g.n = x.n; g.k = x.k;
        g.C = C; g.ldc = x.n; g.c_plane_stride = x.m * x.n;
        g.prime_begin = x.prime_begin; g.L = x.L;
        gd.push_back(g);
        src.push_back(GemmInt64Src{x.A, x.lda, x.B, x.ldb, nullptr, 0});
        // A contiguous C is one row of m*n entries for the CRT, so that
        // small problems fill whole tiles.
        CrtJob c{};
        const bool cflat = x.ldc == x.n;
        c.res = C; c.rows = cflat ? 1 : x.m; c.cols = cflat ? x.m * x.n : x.n;
        c.ldr = c.cols; c.ps = x.m * x.n;
        c.prime_begin = x.prime_begin; c.L = x.L; c.out = x.C; c.ldo = cflat ? c.cols : x.ldc;
        c.status = ctx->d_status;
        const int E = p->crt_E;
        c.col_tiles = crt_col_tiles(c.cols, E);
        c.tile_begin = ct;
        ct += crt_tiles(c.rows, c.cols, E);
        {
            std::lock_guard<std::mutex> guard(ctx->mu);
            if (all_fast) {
                const LagrangeTable *lt = nullptr;
                int st = lagrange_table(ctx, x.prime_begin, x.L, W, &lt, nullptr);
                if (st != RNS_OK) return fail(st);
                c.lag_c = lt->d_c; c.lag_mj = lt->d_mj; c.lag_m = lt->d_m;
            } else {
                int st = mixed_radix_half(ctx, x.prime_begin, x.L, &c.half, nullptr);
                if (st != RNS_OK) return fail(st);
            }
        }
        cj.push_back(c);
    }
    int st = gemm_plan_create_int64(ctx, gd.data(), src.data(), (int)gd.size(), path, &p->gemm);
    if (st != RNS_OK) return fail(st);
    p->nc = (int)cj.size();
    p->ctiles = ct;
    if (p->nc) {
        if (hipMalloc(&p->d_cjobs, sizeof(CrtJob) * p->nc) != hipSuccess) return fail(RNS_ENOMEM);
        if (hipMemcpy(p->d_cjobs, cj.data(), sizeof(CrtJob) * p->nc, hipMemcpyHostToDevice) != hipSuccess)
            return fail(RNS_EDEVICE);
    }
    *out = p;
    return RNS_OK;
}

extern "C" int rns_matmul_plan_execute(rns_matmul_plan *p, void *stream) {
    if (!p) return RNS_EINVAL;
    rns_ctx *ctx = p->ctx;
    hipStream_t s = (hipStream_t)stream;
    RNS_HIP(hipSetDevice(ctx->device));
    int st = rns_gemm_plan_execute(p->gemm, stream);
    if (st != RNS_OK) return st;
    if (p->nc) {
        ProfScope ps(ctx, p->fast_crt ? "k_crt_lagrange" : "k_crt_garner", s);
        launch_crt(p->fast_crt, p->W, p->crt_E, CrtJob{}, p->d_cjobs, p->nc, p->ctiles, ctx->d_prime,
                   ctx->d_garner, s);
    }
    RNS_HIP(hipGetLastError());
    return RNS_OK;
}

extern "C" int rns_matmul_plan_info(const rns_matmul_plan *p, rns_plan_info *info) {
    if (!p || !info) return RNS_EINVAL;
    return rns_gemm_plan_info(p->gemm, info);
}

extern "C" rns_gemm_plan *rns_matmul_plan_gemm(rns_matmul_plan *p) { return p ? p->gemm : nullptr; }
