// Host check of the Smith massager path's algebra (massager_host.hpp): the
// modular Smith form with transforms over Z/sZ against determinantal
// divisors of the integer matrix (brute force on tiny inputs), the identity
// E P R = diag(d), the batch conditions -U P R = [D 0] and U M = -I modulo
// the orders, agreement of the word and big-integer rings, and the p-adic
// top-digit conversion against a direct computation.
// Built and run by tests/test_host_massager.py.
#include "../../paper_2605_19254_amd/csrc/massager_host.hpp"

#include <cstdio>
#include <random>

using namespace rns;
using namespace rns::msg;

static int bad = 0;
#define CHECK(c, ...)                  \
    do {                               \
        if (!(c)) {                    \
            ++bad;                     \
            printf(__VA_ARGS__);       \
            printf("\n");              \
        }                              \
    } while (0)

// Integer determinant by cofactor expansion (tiny k).
static BigInt det_int(const std::vector<BigInt> &m, int k) {
    if (k == 1) return m[0];
    BigInt r(0);
    for (int c = 0; c < k; ++c) {
        std::vector<BigInt> sub;
        for (int i = 1; i < k; ++i)
            for (int j = 0; j < k; ++j)
                if (j != c) sub.push_back(m[(size_t)(i * k + j)]);
        const BigInt v = m[(size_t)c] * det_int(sub, k - 1);
        r = (c % 2) ? r - v : r + v;
    }
    return r;
}

// gcd of all k x k minors of the n x t integer matrix P.
static BigInt minors_gcd(const std::vector<BigInt> &P, int n, int t, int k) {
    BigInt g(0);
    std::vector<int> ri(k), ci(k);
    std::function<void(int, int)> rows, cols;
    rows = [&](int pos, int from) {
        if (pos == k) {
            cols(0, 0);
            return;
        }
        for (int i = from; i < n; ++i) {
            ri[pos] = i;
            rows(pos + 1, i + 1);
        }
    };
    cols = [&](int pos, int from) {
        if (pos == k) {
            std::vector<BigInt> m;
            for (int a = 0; a < k; ++a)
                for (int b = 0; b < k; ++b) m.push_back(P[(size_t)(ri[a] * t + ci[b])]);
            g = BigInt::gcd(g, det_int(m, k));
            return;
        }
        for (int j = from; j < t; ++j) {
            ci[pos] = j;
            cols(pos + 1, j + 1);
        }
    };
    rows(0, 0);
    return g;
}

// Checks one Smith form with transforms of P (n x t, entries in [0, s)).
template <class Ring>
static std::vector<BigInt> check_one(const Ring &F, const std::vector<BigInt> &Pb, int n, int t, const char *tag) {
    using V = typename Ring::V;
    const BigInt s = F.big(F.s);
    std::vector<V> P(Pb.size());
    for (size_t e = 0; e < Pb.size(); ++e) P[e] = F.from(Pb[e]);
    const SnfT<Ring> S = snf_transform(F, P, n, t);
    std::vector<BigInt> d(t);
    for (int j = 0; j < t; ++j) d[j] = F.big(S.d[j]);
    for (int j = 0; j < t; ++j) {
        CHECK(mod(s, d[j]).is_zero(), "%s: d_%d does not divide s", tag, j);
        if (j + 1 < t) CHECK(mod(d[j + 1], d[j]).is_zero(), "%s: chain broken at %d", tag, j);
    }
    // E P: the operations applied to P in order; then times R.
    std::vector<BigInt> EP = Pb;
    for (const auto &o : S.ops) {
        if (o.kind == 0) {
            for (int j = 0; j < t; ++j) std::swap(EP[(size_t)(o.a * t + j)], EP[(size_t)(o.b * t + j)]);
        } else {
            const BigInt x = F.big(o.x);
            for (int j = 0; j < t; ++j) EP[(size_t)(o.a * t + j)] = mod(EP[(size_t)(o.a * t + j)] + x * EP[(size_t)(o.b * t + j)], s);
        }
    }
    std::vector<BigInt> PR((size_t)n * t, BigInt(0));
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < t; ++j) {
            BigInt e(0), f(0);
            for (int k = 0; k < t; ++k) {
                e = e + EP[(size_t)(i * t + k)] * F.big(S.R[(size_t)(k * t + j)]);
                f = f + Pb[(size_t)(i * t + k)] * F.big(S.R[(size_t)(k * t + j)]);
            }
            e = mod(e, s);
            PR[(size_t)(i * t + j)] = mod(f, s);
            const BigInt want = (i == j && i < t) ? mod(d[j], s) : BigInt(0);
            CHECK(e == want, "%s: (E P R)[%d][%d] wrong", tag, i, j);
        }
    // Batch columns and rows for every j with order s / d_j > 1.
    int r = 0;
    while (r < t && !(d[r] == s)) ++r;
    const std::vector<V> E = left_rows(F, S, n, r);
    for (int j = 0; j < r; ++j) {
        const BigInt o = s / d[j];
        for (int i2 = 0; i2 < r; ++i2) {
            // (U M)[i2][j] = -(row i2 of E) . M_j  = -delta (mod o)
            BigInt um(0);
            for (int i = 0; i < n; ++i) um = um + F.big(E[(size_t)(i2 * n + i)]) * mod(PR[(size_t)(i * t + j)] / d[j], o);
            const BigInt want = i2 == j ? BigInt(1) : BigInt(0);
            CHECK(mod(um - want, o).is_zero(), "%s: U M != -I at (%d,%d)", tag, i2, j);
        }
        for (int jj = 0; jj < t; ++jj) {
            // -U P R = [D 0] (mod s): (E P R)[j][jj]
            BigInt v(0);
            for (int i = 0; i < n; ++i) v = v + F.big(E[(size_t)(j * n + i)]) * PR[(size_t)(i * t + jj)];
            const BigInt want = jj == j ? d[j] : BigInt(0);
            CHECK(mod(v - want, s).is_zero(), "%s: U P R row %d col %d", tag, j, jj);
        }
    }
    return d;
}

static std::vector<BigInt> brute_d(const std::vector<BigInt> &Pb, int n, int t, const BigInt &s) {
    // Integer Smith form from determinantal divisors, then gcd with s.
    std::vector<BigInt> out;
    BigInt prev(1);
    const int k = std::min(n, t);
    for (int j = 1; j <= k; ++j) {
        const BigInt g = minors_gcd(Pb, n, t, j);
        if (g.is_zero()) {
            while ((int)out.size() < t) out.push_back(s);
            return out;
        }
        out.push_back(BigInt::gcd(g / prev, s));
        prev = g;
    }
    while ((int)out.size() < t) out.push_back(s);
    return out;
}

int main() {
    std::mt19937_64 g(7);
    // Tiny matrices: brute-force Smith form over Z, both rings.
    const uint64_t small_s[] = {6, 12, 30, 64, 81, 360, 2310, 4096 * 27, 97, 1};
    for (const uint64_t sv : small_s) {
        if (sv == 1) continue;
        for (int it = 0; it < 60; ++it) {
            const int n = 1 + g() % 4, t = 1 + g() % 3;
            std::vector<BigInt> Pb((size_t)n * t);
            for (auto &v : Pb) {
                const uint64_t mode = g() % 4;
                const uint64_t x = mode == 0 ? 0 : (mode == 1 ? (sv / (1 + g() % 6)) * (g() % 4) : g());
                v = BigInt::from_u64(x % sv);
            }
            const BigInt s = BigInt::from_u64(sv);
            const std::vector<BigInt> d64 = check_one(Ring64(sv), Pb, n, t, "ring64 tiny");
            const std::vector<BigInt> dbg = check_one(RingBig(s), Pb, n, t, "ringbig tiny");
            const std::vector<BigInt> ref = brute_d(Pb, n, t, s);
            for (int j = 0; j < t; ++j) {
                CHECK(d64[j] == ref[j], "tiny s=%llu n=%d t=%d: d_%d differs from minors", (unsigned long long)sv, n, t, j);
                CHECK(dbg[j] == ref[j], "tiny big s=%llu: d_%d differs", (unsigned long long)sv, j);
            }
        }
    }
    // Larger: word moduli near 2^62 and a multiword modulus; structured rows.
    const uint64_t words[] = {(1ull << 62) - 57, 2ull * 3 * 5 * 7 * 11 * 13 * 17 * 19 * 23 * 29 * 31 * 37 * 41 * 43 * 47,
                              (1ull << 40) * 3 * 3 * 3 * 5, 4611686018427387847ull};
    for (const uint64_t sv : words) {
        for (int it = 0; it < 6; ++it) {
            const int n = 5 + g() % 20, t = 1 + g() % 9;
            std::vector<BigInt> Pb((size_t)n * t);
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < t; ++j) {
                    uint64_t x = g() % sv;
                    if (it % 2) x = (x % 5) * (sv / 7 + 1) % sv;          // many shared factors
                    if (j == 1 && t > 2) x = 0;                         // a zero column
                    Pb[(size_t)(i * t + j)] = BigInt::from_u64(x);
                }
            const BigInt s = BigInt::from_u64(sv);
            const auto a = check_one(Ring64(sv), Pb, n, t, "ring64");
            const auto b = check_one(RingBig(s), Pb, n, t, "ringbig");
            for (int j = 0; j < t; ++j) CHECK(a[j] == b[j], "rings differ s=%llu d_%d", (unsigned long long)sv, j);
        }
    }
    {
        // s = 2^70 3^30 q (q a 61-bit prime): big ring only.
        BigInt s = BigInt(1).shl(70);
        for (int i = 0; i < 30; ++i) s = s.mul_small(3);
        s = s * BigInt::from_u64(2305843009213693951ull);
        for (int it = 0; it < 4; ++it) {
            const int n = 8 + g() % 10, t = 2 + g() % 6;
            std::vector<BigInt> Pb((size_t)n * t);
            for (auto &v : Pb) {
                BigInt x(0);
                for (int w = 0; w < 5; ++w) x = x.shl(32) + BigInt((int64_t)(g() & 0xFFFFFFFF));
                if (it % 2) x = x.shl(60 + g() % 20);
                v = mod(x, s);
            }
            check_one(RingBig(s), Pb, n, t, "ringbig multiword");
        }
    }
    // p-adic top digits: x = N / s_n with |N| small; digits of x mod p^K; the
    // table gives N mod s_n (big ring) and N mod M' for a word-size divisor
    // M' of s_n (word ring), and refuses x = N / (3 s_n).
    {
        const uint32_t p = 67108859u;
        for (int it = 0; it < 40; ++it) {
            const uint64_t Mw = (g() % ((1ull << 62) - 3)) + 2;       // word-size factor of s_n
            BigInt sn = BigInt::from_u64(Mw);
            for (int w = 0; w < 1 + (int)(g() % 6); ++w) sn = sn.shl(32) + BigInt((int64_t)(g() & 0xFFFFFFFF));
            sn = sn - mod(sn, BigInt::from_u64(Mw));                  // a multiple of Mw
            if (sn.is_zero() || BigInt::gcd(sn, BigInt((int64_t)p)) != BigInt(1)) continue;
            const int K = 30;
            BigInt pK(1);
            for (int k = 0; k < K; ++k) pK = pK.mul_small(p);
            BigInt N(0);
            for (int w = 0; w < 4; ++w) N = N.shl(32) + BigInt((int64_t)(g() & 0xFFFFFFFF));
            if (g() & 1) N = -N;
            auto digits = [&](const BigInt &den, std::vector<uint32_t> &dig) {
                BigInt xi, yi;
                BigInt::xgcd(mod(den, pK), pK, xi, yi);
                BigInt xK = mod(N * xi, pK);
                dig.assign(K, 0u);
                for (int k = 0; k < K; ++k) {
                    dig[k] = xK.mod_small(p);
                    xK = xK / BigInt((int64_t)p);
                }
            };
            std::vector<uint32_t> dig;
            digits(sn, dig);
            const int L = (int)((sn.bit_length() + 24) / 25) + 1;
            const RingBig FB(sn);
            const PadicTable<RingBig> TB(FB, sn, p, K, L);
            BigInt out;
            const bool ok = TB.eval(dig.data() + (K - L), 1, out);
            CHECK(ok && out == mod(N, sn), "padic table (big) wrong at %d", it);
            const Ring64 FW(Mw);
            const PadicTable<Ring64> TW(FW, sn, p, K, L);
            uint64_t ow = 0;
            const bool okw = TW.eval(dig.data() + (K - L), 1, ow);
            CHECK(okw && BigInt::from_u64(ow) == mod(N, BigInt::from_u64(Mw)), "padic table (word) wrong at %d", it);
            // The block form over several entries (digit planes of stride 3,
            // the entry's digits at offset 1) agrees with the single form.
            {
                // entries N, N + 1, -N, 0 side by side (stride 4), outputs at stride 2
                const BigInt Ns[4] = {N, N + BigInt(1), -N, BigInt(0)};
                std::vector<uint32_t> planes((size_t)K * 4, 0u);
                for (int j = 0; j < 4; ++j) {
                    BigInt xi, yi;
                    BigInt::xgcd(mod(sn, pK), pK, xi, yi);
                    BigInt xK = mod(Ns[j] * xi, pK);
                    for (int k = 0; k < K; ++k) {
                        planes[(size_t)k * 4 + j] = xK.mod_small(p);
                        xK = xK / BigInt((int64_t)p);
                    }
                }
                BigInt ob[8];
                uint64_t owb[8] = {0};
                const bool okb = TB.eval_block(planes.data() + (size_t)(K - L) * 4, 4, 4, ob, 2);
                const bool okw2 = TW.eval_block(planes.data() + (size_t)(K - L) * 4, 4, 4, owb, 2);
                for (int j = 0; j < 4; ++j) {
                    CHECK(okb && ob[2 * j] == mod(Ns[j], sn), "padic block (big) entry %d at %d", j, it);
                    CHECK(okw2 && BigInt::from_u64(owb[2 * j]) == mod(Ns[j], BigInt::from_u64(Mw)),
                          "padic block (word) entry %d at %d", j, it);
                }
            }
            // x = N / (3 s_n) with 3 not dividing N: s_n x is not an integer.
            if (mod(N, BigInt(3)).is_zero()) N = N + BigInt(1);
            digits(sn.mul_small(3), dig);
            CHECK(!TB.eval(dig.data() + (K - L), 1, out), "padic table accepted a non-integer at %d", it);
        }
    }
    // Word factorisation: the product of the prime powers gives n back, every
    // factor passes trial division (below 2^32) or is checked against a known
    // prime; semiprimes of two 31-bit primes and prime powers included.
    {
        auto tdiv_prime = [](uint64_t q) {
            if (q < 2) return false;
            for (uint64_t d = 2; d * d <= q; ++d)
                if (q % d == 0) return false;
            return true;
        };
        const uint64_t cases[] = {1, 2, 97, 1ull << 61, 3486784401ull /* 3^20 */, 2147483647ull * 2147483629ull,
                                  2305843009213693951ull /* 2^61 - 1 */, 999999937ull * 999999929ull,
                                  (1ull << 8) * 27 * 5 * 49 * 13 * 19, 614889782588491410ull};
        for (uint64_t nv : cases) {
            const auto f = factor64(nv);
            unsigned __int128 prod = 1;
            for (auto &pe : f) {
                for (int e = 0; e < pe.second; ++e) prod *= pe.first;
                const bool ok = pe.first < (1ull << 32) ? tdiv_prime(pe.first)
                                                        : (pe.first == 2305843009213693951ull);
                CHECK(ok, "factor64(%llu): %llu is not prime", (unsigned long long)nv, (unsigned long long)pe.first);
            }
            CHECK(prod == nv, "factor64(%llu): product differs", (unsigned long long)nv);
        }
        for (int it = 0; it < 200; ++it) {
            const uint64_t nv = (g() >> 2) | 1;
            const auto f = factor64(nv);
            unsigned __int128 prod = 1;
            for (auto &pe : f) {
                for (int e = 0; e < pe.second; ++e) prod *= pe.first;
                if (pe.first < (1ull << 32)) CHECK(tdiv_prime(pe.first), "random factor not prime");
                else CHECK(is_prime64(pe.first), "random large factor not prime");
            }
            CHECK(prod == nv, "random factor64 product differs");
        }
    }
    printf("bad=%d\n", bad);
    return bad != 0;
}
