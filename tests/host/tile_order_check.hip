// Host check of the GEMM tile order: the windowed XCD placement is a
// bijection of [0, G) for every grid size, and map_tile visits every
// (problem, prime, tile-row, tile-column) of a ragged problem table exactly
// once.  Built with hipcc and run on the host by tests/test_host_tile_order.py
// (no device code runs).
#include "../../paper_2605_19254_amd/csrc/gemm_common.hpp"

#include <cstdio>
#include <set>
#include <tuple>
#include <vector>

using namespace rns::gemm;

int main() {
    int bad = 0;
    // 1. Placements are bijections, including grids that are not a multiple
    //    of 8 windows and grids smaller than one window.
    const int64_t sizes[] = {1, 2, 7, 8, 9, 31, 63, 64, 65, 255, 256, 257, 511, 512, 513, 1000, 4095, 4096,
                             4097, 8191, 98304, 98304 + 17, 51228};
    for (int64_t G : sizes)
        for (int64_t W : {int64_t(1), int64_t(32), int64_t(64), int64_t(128)}) {
            std::vector<char> seen((size_t)G, 0);
            for (int64_t b = 0; b < G; ++b) {
                const int64_t h = xcd_window_remap(b, G, W);
                if (h < 0 || h >= G || seen[(size_t)h]) {
                    ++bad;
                    printf("window remap G=%lld W=%lld b=%lld -> %lld\n", (long long)G, (long long)W,
                           (long long)b, (long long)h);
                    break;
                }
                seen[(size_t)h] = 1;
            }
            // Full rounds: work-groups of one XCD (b % 8) get whole windows.
            const int64_t full = G / (8 * W) * (8 * W);
            for (int64_t b = 0; b < full; ++b)
                if ((xcd_window_remap(b, G, W) / W) % 8 != b % 8) {
                    ++bad;
                    printf("window owner G=%lld W=%lld b=%lld\n", (long long)G, (long long)W, (long long)b);
                    break;
                }
        }
    // 2. map_tile over a ragged table: problems with different tile grids and
    //    prime counts, tile_begin as the prefix of L * tm * tn.
    struct Shape { int tm, tn, L; };
    const Shape shapes[] = {{1, 1, 1}, {3, 5, 2}, {9, 2, 3}, {17, 4, 1}, {8, 32, 2}, {64, 32, 1}, {5, 9, 4}};
    std::vector<GemmProblem> P;
    int64_t total = 0;
    for (const Shape &sh : shapes) {
        GemmProblem g{};
        g.tm = sh.tm;
        g.tn = sh.tn;
        g.L = sh.L;
        g.tile_begin = total;
        total += (int64_t)sh.L * sh.tm * sh.tn;
        P.push_back(g);
    }
    std::vector<int32_t> tile_prob((size_t)total);
    for (int q = 0; q < (int)P.size(); ++q) {
        const int64_t end = q + 1 < (int)P.size() ? P[q + 1].tile_begin : total;
        for (int64_t t = P[q].tile_begin; t < end; ++t) tile_prob[(size_t)t] = q;
    }
    for (int use_table = 0; use_table < 2; ++use_table) {
        std::set<std::tuple<int, int, int, int>> seen;
        for (int64_t t = 0; t < total; ++t) {
            const TileCoord c = map_tile(P.data(), (int)P.size(), t, use_table ? tile_prob.data() : nullptr);
            const GemmProblem &g = P[c.q];
            if (c.plane < 0 || c.plane >= g.L || c.tm < 0 || c.tm >= g.tm || c.tn < 0 || c.tn >= g.tn ||
                !seen.insert(std::make_tuple(c.q, c.plane, c.tm, c.tn)).second) {
                ++bad;
                printf("map_tile t=%lld -> q=%d plane=%d tm=%d tn=%d\n", (long long)t, c.q, c.plane, c.tm, c.tn);
                break;
            }
        }
        if ((int64_t)seen.size() != total) {
            ++bad;
            printf("map_tile covered %zu of %lld tiles\n", seen.size(), (long long)total);
        }
    }
    printf("tiles=%lld bad=%d\n", (long long)total, bad);
    return bad != 0;
}
