// Smith normal form driver (Section 2.2).  Placeholder until the driver lands.
#include "internal.hpp"

struct rns_smith_result {
    std::vector<std::vector<uint64_t>> s;
    rns_smith_stats st{};
};

extern "C" int smith_form(rns_ctx *ctx, const int64_t *A, int64_t n, uint64_t seed,
                          rns_smith_result **out) {
    (void)ctx; (void)A; (void)n; (void)seed;
    if (out) *out = nullptr;
    return RNS_ENOTSUP;
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
