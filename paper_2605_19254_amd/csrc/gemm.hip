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
#include <cstring>
#include <vector>

using namespace rns;
using namespace rns::gemm;

namespace {

struct Plan {
    std::vector<GemmProblem> probs;
    size_t work_bytes = 0;
    int64_t total_tiles = 0;
    int64_t total_units = 0;
};

int make_plan(rns_ctx *ctx, const rns_gemm_desc *d, int count, bool int8, Plan &plan) {
    const int TM = int8 ? kI8TileM : kF64TileM;
    const int TN = int8 ? kI8TileN : kF64TileN;
    const int64_t elem = int8 ? 4 : 8;   // bytes per operand entry in the tiled layout
    size_t off = 0;
    for (int i = 0; i < count; ++i) {
        const rns_gemm_desc &x = d[i];
        if (x.m < 0 || x.n < 0 || x.k < 0 || x.L < 0) return RNS_EINVAL;
        if (x.prime_begin < 0 || x.prime_begin + x.L > ctx->L) return RNS_EINVAL;
        if (x.m > INT32_MAX / 2 || x.n > INT32_MAX / 2 || x.k > INT32_MAX / 2) return RNS_EINVAL;
        if (x.m == 0 || x.n == 0 || x.L == 0) continue;
        if (!x.C || x.ldc < x.n) return RNS_EINVAL;
        if (x.L > 1 && x.c_plane_stride < (x.m - 1) * x.ldc + x.n) return RNS_EINVAL;
        if (x.k > 0) {
            if (!x.A || !x.B || x.lda < x.k || x.ldb < x.n) return RNS_EINVAL;
            if (x.L > 1 && (x.a_plane_stride < (x.m - 1) * x.lda + x.k ||
                            x.b_plane_stride < (x.k - 1) * x.ldb + x.n))
                return RNS_EINVAL;
        }
        if (int8 && x.k > kInt8MaxK) return RNS_EBOUND;
        GemmProblem g{};
        g.A = x.A; g.B = x.B; g.C = x.C;
        g.lda = x.lda; g.aps = x.a_plane_stride;
        g.ldb = x.ldb; g.bps = x.b_plane_stride;
        g.ldc = x.ldc; g.cps = x.c_plane_stride;
        g.m = (int32_t)x.m; g.n = (int32_t)x.n; g.k = (int32_t)x.k;
        g.L = x.L; g.prime_begin = x.prime_begin;
        const int64_t Mp = round_up(x.m, TM), Np = round_up(x.n, TN);
        const int64_t Kp = round_up(std::max<int64_t>(x.k, 1), kKTile);
        g.RB = (int32_t)(Mp / 16); g.CB = (int32_t)(Np / 16); g.KT = (int32_t)(Kp / kKTile);
        g.tm = (int32_t)(Mp / TM); g.tn = (int32_t)(Np / TN);
        g.a_plane_bytes = Mp * Kp * elem;
        g.b_plane_bytes = Np * Kp * elem;
        g.At = reinterpret_cast<char *>(off);
        off += (size_t)g.a_plane_bytes * g.L;
        g.Bt = reinterpret_cast<char *>(off);
        off += (size_t)g.b_plane_bytes * g.L;
        off = (off + 255) & ~(size_t)255;
        g.tile_begin = plan.total_tiles;
        plan.total_tiles += (int64_t)g.L * g.tm * g.tn;
        g.unitA_begin = plan.total_units;
        g.unitB_begin = g.unitA_begin + (int64_t)g.L * g.RB * g.KT;
        plan.total_units = g.unitB_begin + (int64_t)g.L * g.CB * g.KT;
        plan.probs.push_back(g);
    }
    plan.work_bytes = off;
    return RNS_OK;
}

}  // namespace

extern "C" int rns_workspace_bytes(rns_ctx *ctx, const rns_gemm_desc *descs, int count,
                                   int path, size_t *bytes) {
    if (!ctx || !bytes || count < 0 || (count > 0 && !descs)) return RNS_EINVAL;
    const bool int8 = path != RNS_PATH_FP64;
    Plan plan;
    int st = make_plan(ctx, descs, count, int8, plan);
    if (st != RNS_OK) return st;
    *bytes = plan.work_bytes;
    return RNS_OK;
}

extern "C" int modmatmul_batched(rns_ctx *ctx, const rns_gemm_desc *descs, int count,
                                 int path, void *stream) {
    if (!ctx || count < 0 || (count > 0 && !descs)) return RNS_EINVAL;
    if (path != RNS_PATH_AUTO && path != RNS_PATH_FP64 && path != RNS_PATH_INT8) return RNS_EINVAL;
    if (count == 0) return RNS_OK;
    bool int8 = path != RNS_PATH_FP64;
    std::lock_guard<std::mutex> guard(ctx->mu);
    Plan plan;
    int st = make_plan(ctx, descs, count, int8, plan);
    if (st == RNS_EBOUND && path == RNS_PATH_AUTO) {
        int8 = false;
        plan = Plan();
        st = make_plan(ctx, descs, count, int8, plan);
    }
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
    // The pinned staging buffer may still be read by an earlier copy on this
    // stream; wait for it before overwriting.
    RNS_HIP(hipStreamSynchronize(s));
    std::memcpy(ctx->h_desc, plan.probs.data(), tbytes);
    RNS_HIP(hipMemcpyAsync(ctx->d_desc, ctx->h_desc, tbytes, hipMemcpyHostToDevice, s));
    const GemmProblem *dP = static_cast<const GemmProblem *>(ctx->d_desc);
    const int np = (int)plan.probs.size();
    {
    ProfScope ps(ctx, int8 ? "k_prep_i8" : "k_prep_f64", s);
    launch_prep(int8, dP, np, plan.total_units, (const PrimeConst *)ctx->d_prime, s);
    }
    RNS_HIP(hipGetLastError());
    {
    ProfScope ps(ctx, int8 ? "k_gemm_i8" : "k_gemm_f64", s);
    if (int8)
        launch_gemm_i8(ctx->int8_kernel, dP, np, plan.total_tiles, (const PrimeConst *)ctx->d_prime, s);
    else
        launch_gemm_f64(dP, np, plan.total_tiles, (const PrimeConst *)ctx->d_prime, s);
    }
    RNS_HIP(hipGetLastError());
    return RNS_OK;
}
