// Host check of the driver's big-integer routines (Karatsuba products, Barrett
// reduction, 2^16-smoothness, Lehmer gcd, extended gcd, rational
// reconstruction) against schoolbook products, long division, trial division
// and plain Euclid on random inputs.
// Built and run by tests/test_host_bigint.py.
#include "../../paper_2605_19254_amd/csrc/bigint.hpp"
#include <chrono>
#include <cstdio>
#include <random>
using namespace rns;
// Reference: plain Euclid.
static BigInt gcd_ref(BigInt a, BigInt b) { a.neg=b.neg=false; while(!b.is_zero()){BigInt q,r; BigInt::divmod_trunc(a,b,q,r); a=std::move(b); b=std::move(r);} return a; }
static BigInt rnd(std::mt19937_64 &g, int limbs, bool sgn) {
    BigInt x(0);
    for (int i = 0; i < limbs; ++i) x = x.shl(32) + BigInt((int64_t)(g() & 0xFFFFFFFFu));
    if (sgn && (g() & 1)) x = -x;
    return x;
}
// Reference: schoolbook product, one limb of b at a time.
static BigInt mul_ref(const BigInt &a, const BigInt &b) {
    BigInt r(0);
    for (size_t j = b.mag.size(); j-- > 0;) r = r.shl(32) + BigInt::abs(a).mul_small(b.mag[j]);
    if (a.neg != b.neg && !r.is_zero()) r = -r;
    return r;
}
// Limbs of all ones (carry paths) or random.
static BigInt limbs(std::mt19937_64 &g, int n, bool ones) {
    BigInt x(0);
    for (int i = 0; i < n; ++i) x = x.shl(32) + BigInt((int64_t)(ones ? 0xFFFFFFFFu : (g() & 0xFFFFFFFFu)));
    return x;
}
int main() {
    std::mt19937_64 g(5);
    int bad = 0;
    // Products across the Karatsuba threshold: balanced, unbalanced, all-ones.
    for (int it = 0; it < 400; ++it) {
        const int la = 1 + g() % 300, lb = (it % 5 == 0) ? la : 1 + g() % 300;
        const bool ones = it % 9 == 0;
        BigInt a = limbs(g, la, ones), b = limbs(g, lb, ones);
        if (g() & 1) a = -a;
        if (it % 17 == 0) b = BigInt(0);
        if (a * b != mul_ref(a, b)) { ++bad; printf("mul mismatch %d (%d x %d)\n", it, la, lb); }
    }
    // Barrett reduction against long division, up to the 2k-limb limit and past it.
    for (int it = 0; it < 400; ++it) {
        const int lm = 1 + g() % 160;
        BigInt m = limbs(g, lm, it % 11 == 0);
        if (m.is_zero()) m = BigInt(7);
        const ModReducer R(m);
        for (int j = 0; j < 4; ++j) {
            const int lx = j == 3 ? 2 * lm + 1 + (int)(g() % 3) : (int)(g() % (2 * lm + 1));
            BigInt x = limbs(g, lx, it % 13 == 0);
            if (g() & 1) x = -x;
            if (j == 0) x = m * limbs(g, 1 + g() % lm, false);       // multiples of m
            if (R.reduce(x) != mod(x, m)) { ++bad; printf("barrett mismatch %d/%d\n", it, j); }
        }
    }
    // 2^16-smoothness by the primorial gcd against trial division: products
    // of primes around the bound (65521 is the largest below, 65537 the
    // first above) and of random small factors.
    for (int it = 0; it < 600; ++it) {
        BigInt s(1);
        const int k = 1 + g() % 10;
        for (int j = 0; j < k; ++j) {
            uint64_t f = (it % 3 == 0) ? small_primes()[g() % small_primes().size()]
                                       : 2 + g() % ((it % 3 == 1) ? 70000 : 200);
            if (it % 17 == 0 && j == 0) f = 65537;
            if (it % 19 == 0 && j == 0) f = 65521;
            s = s.mul_small((uint32_t)f);
        }
        BigInt r = s;
        for (uint32_t q : small_primes())
            while (r.mod_small(q) == 0) r = r / BigInt((int64_t)q);
        if (smooth16(s) != r.is_one()) { ++bad; printf("smooth16 mismatch %d\n", it); }
    }
    if (bad) {                 // the gcd checks below rely on the products
        printf("bad=%d\n", bad);
        return 1;
    }
    for (int it = 0; it < 3000; ++it) {
        int la = 1 + g() % 40, lb = 1 + g() % 40;
        if (it % 7 == 0) lb = la;
        BigInt a = rnd(g, la, true), b = rnd(g, lb, true);
        BigInt f = rnd(g, 1 + g() % 12, false);
        if (it % 3 == 0) { a = a * f; b = b * f; }
        if (it % 11 == 0) b = BigInt(0);
        if (it % 13 == 0) a = BigInt(0);
        BigInt gg = BigInt::gcd(a, b), gr = gcd_ref(a, b);
        if (gg != gr) { ++bad; printf("gcd mismatch %d\n", it); }
        BigInt x, y;
        BigInt g2 = BigInt::xgcd(a, b, x, y);
        if (g2 != gr || x * a + y * b != g2) { ++bad; printf("xgcd mismatch %d\n", it); }
    }
    // rational reconstruction round trips
    for (int it = 0; it < 300; ++it) {
        BigInt m(1);
        int K = 2 + g() % 300;
        for (int i = 0; i < K; ++i) m = m.mul_small(67108859u);
        int bits = (int)(m.bit_length() - 2) / 2 - 3;
        BigInt N = rnd(g, bits / 32, true), D = rnd(g, bits / 32, false);
        if (D.is_zero()) D = BigInt(1);
        if (D.mod_small(67108859u) == 0) D = D + BigInt(1);
        BigInt gnd = BigInt::gcd(N, D);
        if (!gnd.is_zero()) { N = N / gnd; D = D / gnd; }
        BigInt x, y;
        BigInt::xgcd(D, m, x, y);
        BigInt v = mod(N * x, m), num, den;
        bool ok = BigInt::rat_recon(v, m, num, den);
        if (!ok || num != N || den != D) { ++bad; printf("rr mismatch %d ok=%d\n", it, ok); }
    }
    printf("bad=%d\n", bad);
    return bad != 0;
}
