// Host algebra of the Smith massager path: the modular Smith form of an
// n x t projection over Z/sZ with the transforms that give the batch's U and
// M (Section 2.2, Phase 2, item 2), and the conversion of the top p-adic
// digits of A^-1 J into Rem(s A^-1 J, s).
//
// Notation (Section 2.2, Phase 2): P_1 is n x t over Z/sZ.  The elimination
// finds unimodular (mod s) E (n x n, kept as its list of row operations) and
// R (t x t, kept explicitly) with E P_1 R = diag(d_0, ..., d_{t-1}) padded by
// zero rows, d_0 | d_1 | ... | s, each d_j a divisor of s (d_j = s for a zero
// entry).  With L = E^-1 this is P_1 R = L [D; 0]; the batch's massager
// columns are M_j = L_j (the columns of P_1 R divided by d_j, determined
// modulo s / d_j) and its rows are U_j = -(row j of E), so that
// -U P_1 R = [D 0] and U M = -I modulo the orders s / d_j.
#pragma once

#include <algorithm>
#include <cstdint>
#include <functional>
#include <type_traits>
#include <utility>
#include <vector>

#include "bigint.hpp"

namespace rns {
namespace msg {

// Z/sZ on machine words, s < 2^63.
struct Ring64 {
    using V = uint64_t;
    uint64_t s;
    explicit Ring64(uint64_t m) : s(m) {}
    V zero() const { return 0; }
    V one() const { return s == 1 ? 0 : 1; }
    bool is_zero(V a) const { return a == 0; }
    bool is_one(V a) const { return a == 1; }
    V from(const BigInt &x) const {
        const BigInt r = mod(x, BigInt::from_u64(s));
        return r.to_u64_mag();
    }
    BigInt big(V a) const { return BigInt::from_u64(a); }
    V mul(V a, V b) const { return (V)((unsigned __int128)a * b % s); }
    V add(V a, V b) const {
        const V r = a + b;
        return r >= s ? r - s : r;
    }
    V neg(V a) const { return a ? s - a : 0; }
    static uint64_t gcd(uint64_t a, uint64_t b) {
        while (b) {
            const uint64_t t = a % b;
            a = b;
            b = t;
        }
        return a;
    }
    V gcd_s(V a) const { return gcd(a, s); }
    bool divides(V g, V b) const { return b % g == 0; }
    // a^-1 mod m for a prime to m (0 when m = 1), by the extended Euclidean
    // algorithm on signed 128-bit cofactors.
    static uint64_t inv(uint64_t a, uint64_t m) {
        if (m == 1) return 0;
        __int128 r0 = m, r1 = a % m, t0 = 0, t1 = 1;
        while (r1) {
            const __int128 q = r0 / r1;
            __int128 x = r0 - q * r1;
            r0 = r1;
            r1 = x;
            x = t0 - q * t1;
            t0 = t1;
            t1 = x;
        }
        if (t0 < 0) t0 += m;
        return (uint64_t)t0;
    }
    static uint64_t mulm(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((unsigned __int128)a * b % m); }
    double cost() const { return 1.0; }               // ring operations, relative to a word product
    // f with b - f a = 0 (mod s), where g = gcd(a, s) divides b: a = g a',
    // b = g b', a' prime to s/g, f = b' a'^-1 mod s/g; quot_inv(a, g) is the
    // part that depends on a alone.
    V quot_inv(V a, V g) const {
        const uint64_t m = s / g;
        return inv((a / g) % m, m);
    }
    V quot_by(V b, V g, V ainv) const {
        const uint64_t m = s / g;
        return mulm((b / g) % m, ainv, m);
    }
    V quot(V b, V a, V g) const { return quot_by(b, g, quot_inv(a, g)); }
    // sum over l = 1..L of dig[(L - l) stride] B[l], mod s (digits < 2^32,
    // L < 2^30: the 128-bit sum does not overflow).
    V dot_digits(const std::vector<V> &B, const uint32_t *dig, int64_t stride, int L) const {
        unsigned __int128 acc = 0;
        for (int l = 1; l <= L; ++l) acc += (unsigned __int128)B[(size_t)l] * dig[(size_t)(L - l) * stride];
        return (V)(acc % s);
    }
    V mul_u64(V a, uint64_t e) const { return mulm(a, e % s, s); }
    // x with gcd(a + x b, s) = gcd(a, b, s): with g that gcd, x is the
    // largest divisor of s/g prime to a/g (then every prime of s/g divides
    // exactly one of a/g and x b/g).
    V stab(V a, V b) const {
        const uint64_t g = gcd(gcd(a, b), s);
        const uint64_t N = s / g, ap = (a / g) % N;
        uint64_t d = N, h;
        while ((h = gcd(d, ap)) > 1) d /= h;
        return d % s;
    }
    // u^-1 mod s for a = g u with u a unit mod s (g = gcd(a, s)).
    V unit_inv(V a, V g) const {
        const uint64_t N = s / g, u0 = (a / g) % N;
        const uint64_t k = stab(u0 % s, N % s);
        const uint64_t u = (u0 + mulm(k, N, s)) % s;
        return inv(u, s);
    }
    // gcd h of divisors a, b of s with h = x a + y b; x, y mod s.
    void xgcd(V a, V b, V &h, V &x, V &y) const {
        __int128 r0 = a, r1 = b, s0 = 1, s1 = 0, t0 = 0, t1 = 1;
        while (r1) {
            const __int128 q = r0 / r1;
            __int128 v = r0 - q * r1;
            r0 = r1;
            r1 = v;
            v = s0 - q * s1;
            s0 = s1;
            s1 = v;
            v = t0 - q * t1;
            t0 = t1;
            t1 = v;
        }
        h = (V)r0;
        s0 %= (__int128)s;
        t0 %= (__int128)s;
        x = (V)(s0 < 0 ? s0 + s : s0);
        y = (V)(t0 < 0 ? t0 + s : t0);
    }
    V divexact(V a, V b) const { return a / b; }
    V mulexact(V a, V b) const { return a * b; }   // a b divides s here
    // Elimination updates: words are always reduced.
    static constexpr bool kLazy = false;
    V fma_lazy(V acc, V f, V b) const { return add(acc, mul(f, b)); }
    V reduce(V a) const { return a; }
};

// Z/sZ for any s > 1 on big integers.
struct RingBig {
    using V = BigInt;
    BigInt s;
    ModReducer red;
    explicit RingBig(const BigInt &m) : s(m), red(m) {}
    V zero() const { return BigInt(0); }
    V one() const { return s.is_one() ? BigInt(0) : BigInt(1); }
    bool is_zero(const V &a) const { return a.is_zero(); }
    bool is_one(const V &a) const { return a.is_one(); }
    V from(const BigInt &x) const { return red.reduce(x); }
    BigInt big(const V &a) const { return a; }
    V mul(const V &a, const V &b) const { return red.reduce(a * b); }
    V add(const V &a, const V &b) const {
        BigInt r = a + b;
        if (BigInt::cmp(r, s) >= 0) r = r - s;
        return r;
    }
    V neg(const V &a) const { return a.is_zero() ? a : s - a; }
    V gcd_s(const V &a) const { return a.is_zero() ? s : BigInt::gcd(a, s); }
    bool divides(const V &g, const V &b) const { return mod(b, g).is_zero(); }
    static BigInt inv(const BigInt &a, const BigInt &m) {
        if (m.is_one()) return BigInt(0);
        BigInt x, y;
        BigInt::xgcd(mod(a, m), m, x, y);
        return mod(x, m);
    }
    double cost() const {
        const double k = (double)s.mag.size();
        return 4.0 + 3.0 * k * k;
    }
    V quot_inv(const V &a, const V &g) const {
        const BigInt m = s / g;
        return inv(a / g, m);
    }
    V quot_by(const V &b, const V &g, const V &ainv) const {
        const BigInt m = s / g;
        return mod((b / g) * ainv, m);
    }
    V quot(const V &b, const V &a, const V &g) const { return quot_by(b, g, quot_inv(a, g)); }
    V dot_digits(const std::vector<V> &B, const uint32_t *dig, int64_t stride, int L) const {
        BigInt acc(0);
        for (int l = 1; l <= L; ++l) acc = acc + B[(size_t)l].mul_small(dig[(size_t)(L - l) * stride]);
        return red.reduce(acc);
    }
    V mul_u64(const V &a, uint64_t e) const { return red.reduce(a * BigInt::from_u64(e)); }
    V stab(const V &a, const V &b) const {
        const BigInt g = BigInt::gcd(BigInt::gcd(a, b), s);
        const BigInt N = s / g, ap = mod(a / g, N);
        BigInt d = N, h;
        while (!(h = BigInt::gcd(d, ap)).is_one() && !h.is_zero()) d = d / h;
        return mod(d, s);
    }
    V unit_inv(const V &a, const V &g) const {
        const BigInt N = s / g, u0 = mod(a / g, N);
        const BigInt k = stab(mod(u0, s), mod(N, s));
        return inv(mod(u0 + k * N, s), s);
    }
    void xgcd(const V &a, const V &b, V &h, V &x, V &y) const {
        BigInt xx, yy;
        h = BigInt::xgcd(a, b, xx, yy);
        x = mod(xx, s);
        y = mod(yy, s);
    }
    V divexact(const V &a, const V &b) const { return a / b; }
    V mulexact(const V &a, const V &b) const { return a * b; }
    // Elimination updates without reduction (an entry grows by one product
    // per update; entries are reduced before they are read as a pivot column
    // or row).
    static constexpr bool kLazy = true;
    V fma_lazy(const V &acc, const V &f, const V &b) const { return acc + f * b; }
    V reduce(const V &a) const { return red.reduce(a); }
};

// One row operation of the elimination, as a left factor of E:
// kind 0 exchanges rows a and b; kind 1 adds x times row b to row a.
template <class V>
struct RowOp {
    int kind;
    int64_t a, b;
    V x;
};

template <class Ring>
struct SnfT {
    using V = typename Ring::V;
    std::vector<V> d;                 // t diagonal entries (divisors of s, divisibility order)
    std::vector<V> R;                 // t x t, row-major
    std::vector<RowOp<V>> ops;        // E = E_last ... E_first
    int64_t rank = 0;                 // nonzero diagonal entries
};

// A loop over [0, count) that may run on host threads; `work` is the cost of
// one item in ring operations (a hint for whether threads pay off).
using ParFor = std::function<void(int64_t count, double work, const std::function<void(int64_t)> &)>;
inline void seq_for(int64_t count, double, const std::function<void(int64_t)> &f) {
    for (int64_t i = 0; i < count; ++i) f(i);
}

// Smith form of W (n x t over Z/sZ, row-major, entries reduced) with its
// transforms.  Each step takes a nonzero pivot and makes it divide its column
// and row (adding a multiple of another row or column chosen so that the
// pivot's gcd with s becomes that of the pair), clears both, and scales the
// pivot to the divisor gcd(pivot, s); a last pass puts the diagonal in
// divisibility order by 2 x 2 operations that turn (a, b) into
// (gcd(a, b), lcm(a, b)).
template <class Ring>
SnfT<Ring> snf_transform(const Ring &F, std::vector<typename Ring::V> W, int64_t n, int64_t t,
                         const ParFor &par = seq_for) {
    using V = typename Ring::V;
    SnfT<Ring> out;
    out.R.assign((size_t)(t * t), F.zero());
    for (int64_t j = 0; j < t; ++j) out.R[(size_t)(j * t + j)] = F.one();
    auto at = [&](int64_t i, int64_t j) -> V & { return W[(size_t)(i * t + j)]; };
    auto Rat = [&](int64_t i, int64_t j) -> V & { return out.R[(size_t)(i * t + j)]; };
    auto rowswap = [&](int64_t a, int64_t b) {
        if (a == b) return;
        for (int64_t j = 0; j < t; ++j) std::swap(at(a, j), at(b, j));
        out.ops.push_back({0, a, b, F.zero()});
    };
    auto colswap = [&](int64_t a, int64_t b) {
        if (a == b) return;
        for (int64_t i = 0; i < n; ++i) std::swap(at(i, a), at(i, b));
        for (int64_t i = 0; i < t; ++i) std::swap(Rat(i, a), Rat(i, b));
    };
    auto rowadd = [&](int64_t a, int64_t b, const V &x) {     // row a += x row b
        for (int64_t j = 0; j < t; ++j) at(a, j) = F.add(at(a, j), F.mul(x, at(b, j)));
        out.ops.push_back({1, a, b, x});
    };
    auto coladd = [&](int64_t a, int64_t b, const V &x) {     // col a += x col b
        for (int64_t i = 0; i < n; ++i) at(i, a) = F.add(at(i, a), F.mul(x, at(i, b)));
        for (int64_t i = 0; i < t; ++i) Rat(i, a) = F.add(Rat(i, a), F.mul(x, Rat(i, b)));
    };
    const int64_t steps = std::min(n, t);
    int64_t c = 0;
    // Big rings: column c and row c are reduced before they are read (after
    // any exchange that brings other entries there).
    auto normalise = [&]() {
        if constexpr (Ring::kLazy) {
            par(n - c, F.cost(), [&](int64_t k) { at(c + k, c) = F.reduce(at(c + k, c)); });
            for (int64_t j = c + 1; j < t; ++j) at(c, j) = F.reduce(at(c, j));
        }
    };
    for (; c < steps; ++c) {
        normalise();
        if (F.is_zero(at(c, c))) {
            bool found = false;
            for (int64_t i = c + 1; i < n && !found; ++i)
                if (!F.is_zero(at(i, c))) {
                    rowswap(c, i);
                    found = true;
                }
            for (int64_t j = c + 1; j < t && !found; ++j)
                if (!F.is_zero(at(c, j))) {
                    colswap(c, j);
                    found = true;
                }
            for (int64_t i = c + 1; i < n && !found; ++i)
                for (int64_t j = c + 1; j < t && !found; ++j)
                    if (!F.is_zero(at(i, j) = F.reduce(at(i, j)))) {
                        rowswap(c, i);
                        colswap(c, j);
                        found = true;
                    }
            if (!found) break;                    // the rest is zero
            normalise();
        }
        // The pivot's gcd with s only decreases (in the divisor order), so
        // the loop ends.
        std::vector<char> nd;
        for (;;) {
            V a = at(c, c), g = F.gcd_s(a);
            // Rows whose entry in column c the pivot does not divide (none
            // when the pivot is a unit); the flags are computed in parallel
            // and rechecked after each change of the pivot.
            if (!F.is_one(g)) {
                nd.assign((size_t)n, 0);
                par(n - c - 1, F.cost(), [&](int64_t k) {
                    const V &b = at(c + 1 + k, c);
                    nd[(size_t)(c + 1 + k)] = !F.is_zero(b) && !F.divides(g, b);
                });
                for (int64_t i = c + 1; i < n && !F.is_one(g); ++i) {
                    if (!nd[(size_t)i]) continue;
                    const V b = at(i, c);
                    if (F.divides(g, b)) continue;
                    rowadd(c, i, F.stab(a, b));
                    a = at(c, c);
                    g = F.gcd_s(a);
                }
            }
            bool col_changed = false;
            for (int64_t j = c + 1; j < t; ++j) {
                const V b = at(c, j);
                if (!F.is_zero(b) && !F.divides(g, b)) {
                    coladd(c, j, F.stab(a, b));
                    a = at(c, c);
                    g = F.gcd_s(a);
                    col_changed = true;
                }
            }
            if (!col_changed) break;
        }
        const V a = at(c, c), g = F.gcd_s(a), ainv = F.quot_inv(a, g);
        // Column c below the pivot: row i += f_i row c, rows independent.
        std::vector<int64_t> rows;
        for (int64_t i = c + 1; i < n; ++i)
            if (!F.is_zero(at(i, c))) rows.push_back(i);
        std::vector<V> fs(rows.size());
        const bool unit = F.is_one(g);                   // then f = -b a^-1 (no division by g)
        par((int64_t)rows.size(), F.cost(), [&](int64_t k) {
            const V &b = at(rows[(size_t)k], c);
            fs[(size_t)k] = F.neg(unit ? F.mul(b, ainv) : F.quot_by(b, g, ainv));
        });
        par((int64_t)rows.size(), (double)(t - c) * F.cost(), [&](int64_t k) {
            const int64_t i = rows[(size_t)k];
            const V &f = fs[(size_t)k];
            at(i, c) = F.zero();                         // = b + f a = 0 (mod s)
            for (int64_t j = c + 1; j < t; ++j) at(i, j) = F.fma_lazy(at(i, j), f, at(c, j));
        });
        for (size_t k = 0; k < rows.size(); ++k) out.ops.push_back({1, rows[k], c, fs[k]});
        // Row c right of the pivot: column j += f_j column c; column c is zero
        // off the pivot, so in W only entry (c, j) changes.  R's rows are
        // independent.
        std::vector<int64_t> cols;
        std::vector<V> gs;
        for (int64_t j = c + 1; j < t; ++j) {
            if (F.is_zero(at(c, j))) continue;
            cols.push_back(j);
            gs.push_back(F.neg(unit ? F.mul(at(c, j), ainv) : F.quot_by(at(c, j), g, ainv)));
            at(c, j) = F.zero();
        }
        if (!cols.empty())
            par(t, (double)cols.size() * F.cost(), [&](int64_t i) {
                const V rc = Rat(i, c);
                if (F.is_zero(rc)) return;
                for (size_t k = 0; k < cols.size(); ++k) Rat(i, cols[k]) = F.add(Rat(i, cols[k]), F.mul(gs[k], rc));
            });
        // The pivot a = g u (u a unit): column c times u^-1 makes it g.
        const V ui = F.unit_inv(a, g);
        for (int64_t i = 0; i < t; ++i) Rat(i, c) = F.mul(Rat(i, c), ui);
        at(c, c) = F.from(F.big(g));
    }
    out.rank = c;
    out.d.assign((size_t)t, F.s);
    for (int64_t j = 0; j < c; ++j) out.d[(size_t)j] = F.gcd_s(at(j, j));
    // Divisibility order among the nonzero entries (the zeros, s, are last
    // and every d_j divides s).
    for (int64_t i = 0; i < c; ++i)
        for (int64_t j = i + 1; j < c; ++j) {
            const V di = out.d[(size_t)i], dj = out.d[(size_t)j];
            if (F.divides(di, dj)) continue;
            V h, x, y;
            F.xgcd(di, dj, h, x, y);
            const V l = F.mulexact(F.divexact(di, h), dj);   // lcm, a divisor of s
            // row i += row j: (d_i, d_j / 0, d_j)
            out.ops.push_back({1, i, j, F.one()});
            // columns (i, j) <- (i, j) [[x, -d_j/h], [y, d_i/h]]: row i -> (h, 0),
            // row j -> (y d_j, l)
            const V a11 = x, a12 = F.neg(F.from(F.big(F.divexact(dj, h)))), a21 = y,
                    a22 = F.from(F.big(F.divexact(di, h)));
            for (int64_t k = 0; k < t; ++k) {
                const V ci = Rat(k, i), cj = Rat(k, j);
                Rat(k, i) = F.add(F.mul(ci, a11), F.mul(cj, a21));
                Rat(k, j) = F.add(F.mul(ci, a12), F.mul(cj, a22));
            }
            // row j -= (y d_j / h) row i
            const V f = F.neg(F.mul(y, F.from(F.big(F.divexact(dj, h)))));
            out.ops.push_back({1, j, i, f});
            out.d[(size_t)i] = h;
            out.d[(size_t)j] = l;
        }
    return out;
}

// Rows 0..r-1 of E (r x n, row-major): the unit rows multiplied on the right
// by the recorded operations, last to first.
template <class Ring>
std::vector<typename Ring::V> left_rows(const Ring &F, const SnfT<Ring> &S, int64_t n, int64_t r,
                                        const ParFor &par = seq_for) {
    using V = typename Ring::V;
    std::vector<V> v((size_t)(r * n), F.zero());
    par(r, (double)S.ops.size() * F.cost(), [&](int64_t k) {
        V *row = v.data() + (size_t)(k * n);
        row[k] = F.one();
        for (size_t q = S.ops.size(); q-- > 0;) {
            const RowOp<V> &o = S.ops[q];
            if (o.kind == 0) {
                std::swap(row[o.a], row[o.b]);
            } else if (!F.is_zero(row[o.a])) {      // E_op = I + x e_a e_b^T
                row[o.b] = F.add(row[o.b], F.mul(o.x, row[o.a]));
            }
        }
    });
    return v;
}

// Rem(s_n x, M') for x = A^-1 j known by the top L of its K p-adic digits,
// where M' divides s_n (the ring's modulus).  With d_l the digit of step
// K - l (l = 1..L) and s_n / p^l = a_l + f_l (a_l an integer, 0 <= f_l < 1):
// s_n X_K / p^K = sum d_l a_l + sum d_l f_l + (the lower digits' share, below
// s_n p^-L).  Y = s_n x is an integer with |Y| < p^K 2^-24 and
// s_n X_K = Y + c p^K, so c = round(s_n X_K / p^K) = sum d_l a_l + e with
// e = round(sum d_l f_l), and Y = -c p^K (mod s_n).  Hence
//     Y mod M' = sum d_l B_l + e B_0 (mod M'),  B_l = -a_l p^K, B_0 = -p^K.
// The f_l are kept as 64-bit fractions; eval fails when sum d_l f_l is not
// within 2^-21 of an integer (then s_n x is not an integer).
template <class Ring>
struct PadicTable {
    using V = typename Ring::V;
    const Ring &F;
    int L;
    std::vector<V> B;                 // B[0] = B_0, B[l] = B_l
    std::vector<uint64_t> frac;       // frac[l] = floor(f_l 2^64), l = 1..L
    // a_l = floor(s_n / p^l) by repeated division by p, whose remainders d_l
    // give the fractional parts by f_l = (d_l + f_{l-1}) / p (in 64-bit fixed
    // point: each step adds less than one unit of error and divides the
    // previous error by p, so frac[l] is within one unit of floor(2^64 f_l));
    // B_l = -a_l (p^K mod s) mod s, the products independent (par).
    PadicTable(const Ring &ring, const BigInt &sn, uint32_t p, int64_t K, int Ltop, const ParFor &par = seq_for)
        : F(ring), L(Ltop) {
        BigInt pK(1);
        for (int64_t k = 0; k < K; ++k) pK = pK.mul_small(p);
        B.assign((size_t)L + 1, F.zero());
        frac.assign((size_t)L + 1, 0);
        const V pKm = F.from(pK);
        B[0] = F.neg(pKm);
        std::vector<BigInt> a((size_t)L + 1);
        a[0] = sn;
        uint64_t fprev = 0;
        for (int l = 1; l <= L; ++l) {
            const uint32_t d = a[(size_t)l - 1].mod_small(p);
            a[(size_t)l] = a[(size_t)l - 1].div_small(p);
            frac[(size_t)l] = (uint64_t)((((unsigned __int128)d << 64) + fprev) / p);
            fprev = frac[(size_t)l];
        }
        par(L, 8.0 * F.cost(), [&](int64_t l) {
            B[(size_t)l + 1] = F.neg(F.mul(F.from(a[(size_t)l + 1]), pKm));
        });
    }
    // eval for cnt entries whose digit planes are contiguous (entry k's digit
    // of step K - l at dig[(L - l) stride + k]); out[k ostride].  The digit
    // index is the outer loop, so every plane is read in order.
    bool eval_block(const uint32_t *dig, int64_t stride, int64_t cnt, V *out, int64_t ostride) const {
        std::vector<unsigned __int128> fs((size_t)cnt, 0);
        for (int l = 1; l <= L; ++l) {
            const uint32_t *d = dig + (size_t)(L - l) * stride;
            const uint64_t f = frac[(size_t)l];
            for (int64_t k = 0; k < cnt; ++k) fs[(size_t)k] += (unsigned __int128)f * d[k];
        }
        std::vector<uint64_t> ev((size_t)cnt);
        for (int64_t k = 0; k < cnt; ++k) {
            const uint64_t e = (uint64_t)((fs[(size_t)k] + ((unsigned __int128)1 << 63)) >> 64);
            const unsigned __int128 ee = (unsigned __int128)e << 64;
            const unsigned __int128 dist = fs[(size_t)k] > ee ? fs[(size_t)k] - ee : ee - fs[(size_t)k];
            if (dist >= ((unsigned __int128)1 << 43)) return false;
            ev[(size_t)k] = e;
        }
        if constexpr (std::is_same<Ring, Ring64>::value) {
            std::vector<unsigned __int128> acc((size_t)cnt, 0);
            for (int l = 1; l <= L; ++l) {
                const uint32_t *d = dig + (size_t)(L - l) * stride;
                const uint64_t b = B[(size_t)l];
                for (int64_t k = 0; k < cnt; ++k) acc[(size_t)k] += (unsigned __int128)b * d[k];
            }
            for (int64_t k = 0; k < cnt; ++k)
                out[(size_t)(k * ostride)] = F.add((V)(acc[(size_t)k] % F.s), F.mul_u64(B[0], ev[(size_t)k]));
        } else {
            // 64-bit words of the B_l, and a word accumulator per entry
            // (sum of L products below 2^(64 W + 32 + log2 L)).
            size_t W = 1;
            for (int l = 1; l <= L; ++l) W = std::max(W, B[(size_t)l].mag_words().size());
            std::vector<uint64_t> bw((size_t)(L + 1) * W, 0);
            for (int l = 1; l <= L; ++l) {
                const std::vector<uint64_t> w = B[(size_t)l].mag_words();
                std::copy(w.begin(), w.end(), bw.begin() + (size_t)l * W);
            }
            const size_t AW = W + 2;
            std::vector<uint64_t> acc((size_t)cnt * AW, 0);
            for (int l = 1; l <= L; ++l) {
                const uint32_t *d = dig + (size_t)(L - l) * stride;
                const uint64_t *b = bw.data() + (size_t)l * W;
                for (int64_t k = 0; k < cnt; ++k) {
                    const uint64_t dk = d[k];
                    if (!dk) continue;
                    uint64_t *a = acc.data() + (size_t)k * AW;
                    unsigned __int128 carry = 0;
                    for (size_t w = 0; w < W; ++w) {
                        const unsigned __int128 v = (unsigned __int128)b[w] * dk + a[w] + carry;
                        a[w] = (uint64_t)v;
                        carry = v >> 64;
                    }
                    for (size_t w = W; carry && w < AW; ++w) {
                        const unsigned __int128 v = (unsigned __int128)a[w] + carry;
                        a[w] = (uint64_t)v;
                        carry = v >> 64;
                    }
                }
            }
            for (int64_t k = 0; k < cnt; ++k) {
                const uint64_t *a = acc.data() + (size_t)k * AW;
                BigInt x;
                x.mag.resize(2 * AW);
                for (size_t w = 0; w < AW; ++w) {
                    x.mag[2 * w] = (uint32_t)a[w];
                    x.mag[2 * w + 1] = (uint32_t)(a[w] >> 32);
                }
                while (!x.mag.empty() && x.mag.back() == 0) x.mag.pop_back();
                out[(size_t)(k * ostride)] = F.add(F.from(x), F.mul_u64(B[0], ev[(size_t)k]));
            }
        }
        return true;
    }
    bool eval(const uint32_t *dig, int64_t stride, V &out) const {
        unsigned __int128 fs = 0;
        for (int l = 1; l <= L; ++l) fs += (unsigned __int128)frac[(size_t)l] * dig[(size_t)(L - l) * stride];
        const uint64_t e = (uint64_t)((fs + ((unsigned __int128)1 << 63)) >> 64);
        const unsigned __int128 ee = (unsigned __int128)e << 64;
        const unsigned __int128 dist = fs > ee ? fs - ee : ee - fs;
        if (dist >= ((unsigned __int128)1 << 43)) return false;
        out = F.add(F.dot_digits(B, dig, stride, L), F.mul_u64(B[0], e));
        return true;
    }
};

// Prime factorisation of a word n < 2^63 (the modulus of a word-size batch,
// split into prime powers for the local Smith forms): trial division by the
// primes below 2^10, then Miller-Rabin with the first twelve prime bases
// (deterministic below 2^64) and Pollard's rho with Brent's cycle search.
inline uint64_t mulmod64(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((unsigned __int128)a * b % m); }
inline uint64_t powmod64(uint64_t a, uint64_t e, uint64_t m) {
    uint64_t r = 1 % m;
    a %= m;
    for (; e; e >>= 1) {
        if (e & 1) r = mulmod64(r, a, m);
        a = mulmod64(a, a, m);
    }
    return r;
}
inline bool is_prime64(uint64_t n) {
    if (n < 2) return false;
    static const uint64_t small[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    for (uint64_t q : small)
        if (n % q == 0) return n == q;
    uint64_t d = n - 1;
    int r = 0;
    while ((d & 1) == 0) {
        d >>= 1;
        ++r;
    }
    for (uint64_t a : small) {
        uint64_t x = powmod64(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool comp = true;
        for (int i = 1; i < r && comp; ++i) {
            x = mulmod64(x, x, n);
            if (x == n - 1) comp = false;
        }
        if (comp) return false;
    }
    return true;
}
// A nontrivial factor of an odd composite n (Brent's variant, batched gcds).
inline uint64_t rho64(uint64_t n) {
    for (uint64_t c = 1;; ++c) {
        auto f = [&](uint64_t x) { return (mulmod64(x, x, n) + c) % n; };
        uint64_t y = 2, g = 1, q = 1, x = 0, ys = 0;
        const uint64_t m = 128;
        for (uint64_t r = 1; g == 1; r <<= 1) {
            x = y;
            for (uint64_t i = 0; i < r; ++i) y = f(y);
            for (uint64_t k = 0; k < r && g == 1; k += m) {
                ys = y;
                for (uint64_t i = 0; i < std::min(m, r - k); ++i) {
                    y = f(y);
                    q = mulmod64(q, x > y ? x - y : y - x, n);
                }
                g = Ring64::gcd(q, n);
            }
        }
        if (g == n) {
            do {
                ys = f(ys);
                g = Ring64::gcd(x > ys ? x - ys : ys - x, n);
            } while (g == 1);
        }
        if (g != n) return g;
    }
}
inline void factor_rec(uint64_t n, std::vector<uint64_t> &out) {
    if (n == 1) return;
    if (is_prime64(n)) {
        out.push_back(n);
        return;
    }
    const uint64_t d = rho64(n);
    factor_rec(d, out);
    factor_rec(n / d, out);
}
inline std::vector<std::pair<uint64_t, int>> factor64(uint64_t n) {
    std::vector<uint64_t> ps;
    for (uint64_t q = 2; q < 1024 && q * q <= n; ++q)
        while (n % q == 0) {
            ps.push_back(q);
            n /= q;
        }
    factor_rec(n, ps);
    std::sort(ps.begin(), ps.end());
    std::vector<std::pair<uint64_t, int>> out;
    for (uint64_t q : ps) {
        if (!out.empty() && out.back().first == q) ++out.back().second;
        else out.push_back({q, 1});
    }
    return out;
}

}  // namespace msg
}  // namespace rns
