// Host check of the driver's big-integer routines (Lehmer gcd, extended gcd,
// rational reconstruction) against plain Euclid on random inputs.  Built and
// run by tests/test_host_bigint.py.
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
int main() {
    std::mt19937_64 g(5);
    int bad = 0;
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
