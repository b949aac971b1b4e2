// Host-side arbitrary-precision signed integers for the Smith-form driver
// (the big numbers of Section 2: the largest invariant factor s, p-adic
// lifting sums, rational reconstruction).  Sign and magnitude, 32-bit limbs,
// Karatsuba products, Knuth's long division and Barrett reduction for a fixed
// modulus; sizes here reach some ten thousand limbs.
#pragma once

#include <algorithm>
#include <cstdint>
#include <string>
#include <utility>
#include <vector>

namespace rns {

class BigInt {
public:
    bool neg = false;
    std::vector<uint32_t> mag;   // little-endian, no leading zero limbs; empty = 0

    BigInt() = default;
    BigInt(int64_t v) { set_i64(v); }   // NOLINT: implicit by design
    static BigInt from_u64(uint64_t v) {
        BigInt r;
        if (v) {
            r.mag.push_back((uint32_t)v);
            if (v >> 32) r.mag.push_back((uint32_t)(v >> 32));
        }
        return r;
    }
    void set_i64(int64_t v) {
        mag.clear();
        neg = v < 0;
        uint64_t u = neg ? (uint64_t)0 - (uint64_t)v : (uint64_t)v;
        while (u) {
            mag.push_back((uint32_t)u);
            u >>= 32;
        }
    }
    bool is_zero() const { return mag.empty(); }
    bool is_one() const { return !neg && mag.size() == 1 && mag[0] == 1; }
    int sign() const { return is_zero() ? 0 : (neg ? -1 : 1); }
    size_t bit_length() const {
        if (mag.empty()) return 0;
        return 32 * (mag.size() - 1) + (32 - __builtin_clz(mag.back()));
    }
    bool fits_i64() const {
        if (mag.size() > 2) return false;
        const uint64_t u = to_u64_mag();
        return neg ? u <= (1ull << 63) : u < (1ull << 63);
    }
    uint64_t to_u64_mag() const {
        uint64_t u = 0;
        if (mag.size() > 0) u |= mag[0];
        if (mag.size() > 1) u |= (uint64_t)mag[1] << 32;
        return u;
    }
    int64_t to_i64() const {
        const uint64_t u = to_u64_mag();
        return neg ? (int64_t)((uint64_t)0 - u) : (int64_t)u;
    }
    double to_double() const {
        double r = 0;
        for (size_t i = mag.size(); i-- > 0;) r = r * 4294967296.0 + mag[i];
        return neg ? -r : r;
    }
    // Little-endian 64-bit words of the magnitude.
    std::vector<uint64_t> mag_words() const {
        std::vector<uint64_t> w((mag.size() + 1) / 2, 0);
        for (size_t i = 0; i < mag.size(); ++i) w[i / 2] |= (uint64_t)mag[i] << (32 * (i % 2));
        if (w.empty()) w.push_back(0);
        return w;
    }
    // From W little-endian two's-complement words.
    static BigInt from_twos(const uint64_t *w, int W) {
        BigInt r;
        const bool negv = (w[W - 1] >> 63) != 0;
        std::vector<uint64_t> u(w, w + W);
        if (negv) {                      // magnitude = ~u + 1
            uint64_t c = 1;
            for (int i = 0; i < W; ++i) {
                const uint64_t x = ~u[i];
                u[i] = x + c;
                c = (u[i] < x) ? 1 : 0;
            }
        }
        for (int i = 0; i < W; ++i) {
            r.mag.push_back((uint32_t)u[i]);
            r.mag.push_back((uint32_t)(u[i] >> 32));
        }
        r.trim();
        r.neg = negv && !r.is_zero();
        return r;
    }
    void trim() {
        while (!mag.empty() && mag.back() == 0) mag.pop_back();
        if (mag.empty()) neg = false;
    }

    // ---- magnitude helpers
    static int cmp_mag(const std::vector<uint32_t> &a, const std::vector<uint32_t> &b) {
        if (a.size() != b.size()) return a.size() < b.size() ? -1 : 1;
        for (size_t i = a.size(); i-- > 0;)
            if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
        return 0;
    }
    static std::vector<uint32_t> add_mag(const std::vector<uint32_t> &a, const std::vector<uint32_t> &b) {
        const std::vector<uint32_t> &x = a.size() >= b.size() ? a : b;
        const std::vector<uint32_t> &y = a.size() >= b.size() ? b : a;
        std::vector<uint32_t> r(x.size() + 1);
        uint64_t c = 0;
        for (size_t i = 0; i < x.size(); ++i) {
            c += (uint64_t)x[i] + (i < y.size() ? y[i] : 0);
            r[i] = (uint32_t)c;
            c >>= 32;
        }
        r[x.size()] = (uint32_t)c;
        while (!r.empty() && r.back() == 0) r.pop_back();
        return r;
    }
    // |a| >= |b|
    static std::vector<uint32_t> sub_mag(const std::vector<uint32_t> &a, const std::vector<uint32_t> &b) {
        std::vector<uint32_t> r(a.size());
        int64_t br = 0;
        for (size_t i = 0; i < a.size(); ++i) {
            int64_t t = (int64_t)a[i] - (i < b.size() ? (int64_t)b[i] : 0) - br;
            br = t < 0;
            r[i] = (uint32_t)(t + (br ? (1ll << 32) : 0));
        }
        while (!r.empty() && r.back() == 0) r.pop_back();
        return r;
    }
    // ---- products: schoolbook below kKaraLimbs limbs, Karatsuba above.
    static constexpr size_t kKaraLimbs = 40;

    // r[0 .. na+nb) = a b (r is overwritten).
    static void mul_school(const uint32_t *a, size_t na, const uint32_t *b, size_t nb, uint32_t *r) {
        std::fill(r, r + na + nb, 0u);
        for (size_t j = 0; j < nb; ++j) {
            const uint64_t bj = b[j];
            uint64_t c = 0;
            if (bj)
                for (size_t i = 0; i < na; ++i) {
                    c += a[i] * bj + r[i + j];
                    r[i + j] = (uint32_t)c;
                    c >>= 32;
                }
            r[j + na] = (uint32_t)c;
        }
    }
    // r[0 .. n) += a[0 .. na), na <= n; returns the carry out of r[n-1].
    static uint32_t add_into(uint32_t *r, size_t n, const uint32_t *a, size_t na) {
        uint64_t c = 0;
        size_t i = 0;
        for (; i < na; ++i) {
            c += (uint64_t)r[i] + a[i];
            r[i] = (uint32_t)c;
            c >>= 32;
        }
        for (; c && i < n; ++i) {
            c += r[i];
            r[i] = (uint32_t)c;
            c >>= 32;
        }
        return (uint32_t)c;
    }
    // r[0 .. n) -= a[0 .. na), na <= n; returns the borrow out of r[n-1].
    static uint32_t sub_into(uint32_t *r, size_t n, const uint32_t *a, size_t na) {
        int64_t br = 0;
        size_t i = 0;
        for (; i < na; ++i) {
            const int64_t t = (int64_t)r[i] - a[i] - br;
            br = t < 0;
            r[i] = (uint32_t)t;
        }
        for (; br && i < n; ++i) {
            const int64_t t = (int64_t)r[i] - br;
            br = t < 0;
            r[i] = (uint32_t)t;
        }
        return (uint32_t)br;
    }
    // Scratch limbs that kara needs for n-limb operands.
    static size_t kara_scratch(size_t n) {
        return n < kKaraLimbs ? 0 : 4 * (n - n / 2 + 1) + kara_scratch(n - n / 2 + 1);
    }
    // r[0 .. 2n) = a b for two n-limb operands (Karatsuba: with a = a0 + a1 B^h,
    // b likewise, a b = z0 + (z1 - z0 - z2) B^h + z2 B^2h for z0 = a0 b0,
    // z2 = a1 b1, z1 = (a0 + a1)(b0 + b1)).  w: kara_scratch(n) limbs.
    static void kara(const uint32_t *a, const uint32_t *b, size_t n, uint32_t *r, uint32_t *w) {
        if (n < kKaraLimbs) {
            mul_school(a, n, b, n, r);
            return;
        }
        const size_t lo = n / 2, hi = n - lo;
        kara(a, b, lo, r, w);                            // z0 -> r[0, 2 lo)
        kara(a + lo, b + lo, hi, r + 2 * lo, w);         // z2 -> r[2 lo, 2 n)
        uint32_t *sa = w, *sb = w + hi + 1, *z1 = w + 2 * (hi + 1);
        std::copy(a + lo, a + n, sa);
        sa[hi] = add_into(sa, hi, a, lo);
        std::copy(b + lo, b + n, sb);
        sb[hi] = add_into(sb, hi, b, lo);
        kara(sa, sb, hi + 1, z1, w + 4 * (hi + 1));
        sub_into(z1, 2 * hi + 2, r, 2 * lo);
        sub_into(z1, 2 * hi + 2, r + 2 * lo, 2 * hi);
        // z1 - z0 - z2 = a0 b1 + a1 b0 < 2 B^n: its limbs above n are zero.
        add_into(r + lo, 2 * n - lo, z1, std::min(2 * hi + 2, 2 * n - lo));
    }
    // r[0 .. na+nb) = a b for any sizes: Karatsuba on equal pieces of the
    // longer operand, each the length of the shorter.
    static void mul_into(const uint32_t *a, size_t na, const uint32_t *b, size_t nb, uint32_t *r) {
        if (na < nb) {
            std::swap(a, b);
            std::swap(na, nb);
        }
        if (nb < kKaraLimbs) {
            mul_school(a, na, b, nb, r);
            return;
        }
        const size_t ws = kara_scratch(nb);
        std::vector<uint32_t> w(ws + (na == nb ? 0 : 2 * nb));
        if (na == nb) {
            kara(a, b, nb, r, w.data());
            return;
        }
        uint32_t *t = w.data() + ws;
        std::fill(r, r + na + nb, 0u);
        for (size_t off = 0; off < na; off += nb) {
            const size_t len = std::min(nb, na - off);
            if (len == nb)
                kara(a + off, b, nb, t, w.data());
            else
                mul_into(a + off, len, b, nb, t);
            add_into(r + off, na + nb - off, t, len + nb);
        }
    }
    // ---- the same products on 64-bit limbs (128-bit partial products), which
    // take a quarter of the limb products; mul_mag packs pairs of 32-bit limbs
    // into them for operands of kMul64Limbs 32-bit limbs and more.
    static constexpr size_t kKara64Limbs = 48, kMul64Limbs = 16;
    static void mul_school64(const uint64_t *a, size_t na, const uint64_t *b, size_t nb, uint64_t *r) {
        std::fill(r, r + na + nb, (uint64_t)0);
        for (size_t j = 0; j < nb; ++j) {
            const unsigned __int128 bj = b[j];
            unsigned __int128 c = 0;
            if (bj)
                for (size_t i = 0; i < na; ++i) {
                    c += a[i] * bj + r[i + j];
                    r[i + j] = (uint64_t)c;
                    c >>= 64;
                }
            r[j + na] = (uint64_t)c;
        }
    }
    static uint64_t add_into64(uint64_t *r, size_t n, const uint64_t *a, size_t na) {
        unsigned __int128 c = 0;
        size_t i = 0;
        for (; i < na; ++i) {
            c += (unsigned __int128)r[i] + a[i];
            r[i] = (uint64_t)c;
            c >>= 64;
        }
        for (; c && i < n; ++i) {
            c += r[i];
            r[i] = (uint64_t)c;
            c >>= 64;
        }
        return (uint64_t)c;
    }
    static uint64_t sub_into64(uint64_t *r, size_t n, const uint64_t *a, size_t na) {
        uint64_t br = 0;
        size_t i = 0;
        for (; i < na; ++i) {
            const uint64_t x = r[i], y = a[i];
            const uint64_t d = x - y - br;
            br = (x < y) || (x == y && br) ? 1 : 0;
            r[i] = d;
        }
        for (; br && i < n; ++i) {
            br = r[i] == 0 ? 1 : 0;
            r[i] -= 1;
        }
        return br;
    }
    static size_t kara64_scratch(size_t n) {
        return n < kKara64Limbs ? 0 : 4 * (n - n / 2 + 1) + kara64_scratch(n - n / 2 + 1);
    }
    // As kara, on 64-bit limbs.
    static void kara64(const uint64_t *a, const uint64_t *b, size_t n, uint64_t *r, uint64_t *w) {
        if (n < kKara64Limbs) {
            mul_school64(a, n, b, n, r);
            return;
        }
        const size_t lo = n / 2, hi = n - lo;
        kara64(a, b, lo, r, w);
        kara64(a + lo, b + lo, hi, r + 2 * lo, w);
        uint64_t *sa = w, *sb = w + hi + 1, *z1 = w + 2 * (hi + 1);
        std::copy(a + lo, a + n, sa);
        sa[hi] = add_into64(sa, hi, a, lo);
        std::copy(b + lo, b + n, sb);
        sb[hi] = add_into64(sb, hi, b, lo);
        kara64(sa, sb, hi + 1, z1, w + 4 * (hi + 1));
        sub_into64(z1, 2 * hi + 2, r, 2 * lo);
        sub_into64(z1, 2 * hi + 2, r + 2 * lo, 2 * hi);
        add_into64(r + lo, 2 * n - lo, z1, std::min(2 * hi + 2, 2 * n - lo));
    }
    static void mul_into64(const uint64_t *a, size_t na, const uint64_t *b, size_t nb, uint64_t *r) {
        if (na < nb) {
            std::swap(a, b);
            std::swap(na, nb);
        }
        if (nb < kKara64Limbs) {
            mul_school64(a, na, b, nb, r);
            return;
        }
        const size_t ws = kara64_scratch(nb);
        std::vector<uint64_t> w(ws + (na == nb ? 0 : 2 * nb));
        if (na == nb) {
            kara64(a, b, nb, r, w.data());
            return;
        }
        uint64_t *t = w.data() + ws;
        std::fill(r, r + na + nb, (uint64_t)0);
        for (size_t off = 0; off < na; off += nb) {
            const size_t len = std::min(nb, na - off);
            if (len == nb)
                kara64(a + off, b, nb, t, w.data());
            else
                mul_into64(a + off, len, b, nb, t);
            add_into64(r + off, na + nb - off, t, len + nb);
        }
    }
    static std::vector<uint32_t> mul_mag(const std::vector<uint32_t> &a, const std::vector<uint32_t> &b) {
        if (a.empty() || b.empty()) return {};
        std::vector<uint32_t> r(a.size() + b.size());
        if (std::min(a.size(), b.size()) < kMul64Limbs) {
            mul_into(a.data(), a.size(), b.data(), b.size(), r.data());
        } else {
            const size_t na = (a.size() + 1) / 2, nb = (b.size() + 1) / 2;
            std::vector<uint64_t> buf(na + nb + na + nb);
            uint64_t *a64 = buf.data(), *b64 = a64 + na, *r64 = b64 + nb;
            for (size_t i = 0; i < na; ++i)
                a64[i] = a[2 * i] | ((2 * i + 1 < a.size() ? (uint64_t)a[2 * i + 1] : 0) << 32);
            for (size_t i = 0; i < nb; ++i)
                b64[i] = b[2 * i] | ((2 * i + 1 < b.size() ? (uint64_t)b[2 * i + 1] : 0) << 32);
            mul_into64(a64, na, b64, nb, r64);
            for (size_t i = 0; i < r.size(); ++i) r[i] = (uint32_t)(r64[i / 2] >> (32 * (i % 2)));
        }
        while (!r.empty() && r.back() == 0) r.pop_back();
        return r;
    }
    // Knuth, TAOCP vol. 2, 4.3.1 Algorithm D: q = a / b, r = a mod b (magnitudes).
    static void divmod_mag(const std::vector<uint32_t> &a, const std::vector<uint32_t> &b,
                           std::vector<uint32_t> &q, std::vector<uint32_t> &r) {
        if (cmp_mag(a, b) < 0) {
            q.clear();
            r = a;
            return;
        }
        if (b.size() == 1) {
            q.assign(a.size(), 0);
            uint64_t rem = 0;
            for (size_t i = a.size(); i-- > 0;) {
                const uint64_t cur = (rem << 32) | a[i];
                q[i] = (uint32_t)(cur / b[0]);
                rem = cur % b[0];
            }
            while (!q.empty() && q.back() == 0) q.pop_back();
            r.clear();
            if (rem) r.push_back((uint32_t)rem);
            return;
        }
        const int s = __builtin_clz(b.back());
        std::vector<uint32_t> v(b.size()), u(a.size() + 1);
        for (size_t i = b.size(); i-- > 0;)
            v[i] = (b[i] << s) | (s && i ? (uint32_t)((uint64_t)b[i - 1] >> (32 - s)) : 0);
        u[a.size()] = s ? (uint32_t)((uint64_t)a.back() >> (32 - s)) : 0;
        for (size_t i = a.size(); i-- > 0;)
            u[i] = (a[i] << s) | (s && i ? (uint32_t)((uint64_t)a[i - 1] >> (32 - s)) : 0);
        const size_t n = v.size(), m = a.size() - n;
        q.assign(m + 1, 0);
        for (size_t j = m + 1; j-- > 0;) {
            const uint64_t num = ((uint64_t)u[j + n] << 32) | u[j + n - 1];
            uint64_t qh = num / v[n - 1];
            uint64_t rh = num % v[n - 1];
            while (qh >= (1ull << 32) || qh * v[n - 2] > ((rh << 32) | u[j + n - 2])) {
                --qh;
                rh += v[n - 1];
                if (rh >= (1ull << 32)) break;
            }
            int64_t borrow = 0;
            uint64_t carry = 0;
            for (size_t i = 0; i < n; ++i) {
                const uint64_t p = qh * v[i] + carry;
                carry = p >> 32;
                const int64_t t = (int64_t)u[i + j] - (int64_t)(uint32_t)p - borrow;
                u[i + j] = (uint32_t)t;
                borrow = t < 0 ? 1 : 0;
            }
            const int64_t t = (int64_t)u[j + n] - (int64_t)carry - borrow;
            u[j + n] = (uint32_t)t;
            if (t < 0) {                 // add back
                --qh;
                uint64_t c = 0;
                for (size_t i = 0; i < n; ++i) {
                    c += (uint64_t)u[i + j] + v[i];
                    u[i + j] = (uint32_t)c;
                    c >>= 32;
                }
                u[j + n] += (uint32_t)c;
            }
            q[j] = (uint32_t)qh;
        }
        while (!q.empty() && q.back() == 0) q.pop_back();
        r.assign(n, 0);
        for (size_t i = 0; i < n; ++i)
            r[i] = (u[i] >> s) | (s ? (uint32_t)((uint64_t)u[i + 1] << (32 - s)) : 0);
        while (!r.empty() && r.back() == 0) r.pop_back();
    }

    // ---- signed arithmetic
    friend BigInt operator+(const BigInt &a, const BigInt &b) {
        BigInt r;
        if (a.neg == b.neg) {
            r.mag = add_mag(a.mag, b.mag);
            r.neg = a.neg;
        } else if (cmp_mag(a.mag, b.mag) >= 0) {
            r.mag = sub_mag(a.mag, b.mag);
            r.neg = a.neg;
        } else {
            r.mag = sub_mag(b.mag, a.mag);
            r.neg = b.neg;
        }
        r.trim();
        return r;
    }
    BigInt operator-() const {
        BigInt r = *this;
        if (!r.is_zero()) r.neg = !r.neg;
        return r;
    }
    friend BigInt operator-(const BigInt &a, const BigInt &b) { return a + (-b); }
    friend BigInt operator*(const BigInt &a, const BigInt &b) {
        BigInt r;
        r.mag = mul_mag(a.mag, b.mag);
        r.neg = !r.mag.empty() && (a.neg != b.neg);
        return r;
    }
    // Truncating division (like C): q = trunc(a/b), r = a - q*b.
    static void divmod_trunc(const BigInt &a, const BigInt &b, BigInt &q, BigInt &r) {
        divmod_mag(a.mag, b.mag, q.mag, r.mag);
        q.neg = !q.mag.empty() && (a.neg != b.neg);
        r.neg = !r.mag.empty() && a.neg;
    }
    // Floor division with non-negative remainder for b > 0.
    static void divmod_floor(const BigInt &a, const BigInt &b, BigInt &q, BigInt &r) {
        divmod_trunc(a, b, q, r);
        if (r.neg) {
            r = r + abs(b);
            q = q - BigInt(b.neg ? -1 : 1);
        }
    }
    friend BigInt operator/(const BigInt &a, const BigInt &b) {
        BigInt q, r;
        divmod_trunc(a, b, q, r);
        return q;
    }
    // Non-negative residue for m > 0.
    friend BigInt mod(const BigInt &a, const BigInt &m) {
        BigInt q, r;
        divmod_floor(a, m, q, r);
        return r;
    }
    static BigInt abs(const BigInt &a) {
        BigInt r = a;
        r.neg = false;
        return r;
    }
    // floor(|x| / p) for p > 0 (the magnitude; the caller's values are
    // non-negative).
    BigInt div_small(uint32_t p) const {
        BigInt q;
        q.mag.resize(mag.size());
        uint64_t rem = 0;
        for (size_t i = mag.size(); i-- > 0;) {
            const uint64_t cur = (rem << 32) | mag[i];
            q.mag[i] = (uint32_t)(cur / p);
            rem = cur % p;
        }
        while (!q.mag.empty() && q.mag.back() == 0) q.mag.pop_back();
        return q;
    }
    uint32_t mod_small(uint32_t p) const {   // non-negative residue
        uint64_t rem = 0;
        for (size_t i = mag.size(); i-- > 0;) rem = ((rem << 32) | mag[i]) % p;
        if (neg && rem) rem = p - rem;
        return (uint32_t)rem;
    }
    BigInt mul_small(uint32_t m) const {
        BigInt r;
        r.neg = neg;
        r.mag.resize(mag.size() + 1);
        uint64_t c = 0;
        for (size_t i = 0; i < mag.size(); ++i) {
            c += (uint64_t)mag[i] * m;
            r.mag[i] = (uint32_t)c;
            c >>= 32;
        }
        r.mag[mag.size()] = (uint32_t)c;
        r.trim();
        return r;
    }
    friend bool operator==(const BigInt &a, const BigInt &b) { return a.neg == b.neg && a.mag == b.mag; }
    friend bool operator!=(const BigInt &a, const BigInt &b) { return !(a == b); }
    static int cmp(const BigInt &a, const BigInt &b) {
        if (a.neg != b.neg) return a.neg ? -1 : 1;
        const int c = cmp_mag(a.mag, b.mag);
        return a.neg ? -c : c;
    }
    friend bool operator<(const BigInt &a, const BigInt &b) { return cmp(a, b) < 0; }
    friend bool operator<=(const BigInt &a, const BigInt &b) { return cmp(a, b) <= 0; }
    friend bool operator>(const BigInt &a, const BigInt &b) { return cmp(a, b) > 0; }

    // ---- Euclid's algorithm, Lehmer's way (Knuth TAOCP 4.5.2, Algorithm L):
    // far from the end, runs of quotients are found from the leading 124 bits
    // of the two remainders (128-bit arithmetic, so that a run goes on until
    // its matrix entries near 2^62) and applied to the full numbers as one
    // 2 x 2 matrix; the cofactor sequence (t0, t1) follows the same matrices.

    // One exact step: (r0, r1) <- (r1, r0 - q r1), (t0, t1) <- (t1, t0 - q t1).
    static void euclid_step(BigInt &r0, BigInt &r1, BigInt &t0, BigInt &t1, bool track) {
        BigInt q, r;
        divmod_trunc(r0, r1, q, r);
        r0 = std::move(r1);
        r1 = std::move(r);
        if (track) {
            BigInt t = t0 - q * t1;
            t0 = std::move(t1);
            t1 = std::move(t);
        }
    }
    // floor(|x| / 2^shift) mod 2^128.
    static unsigned __int128 shifted_u128(const BigInt &x, size_t shift) {
        const size_t w = shift / 32, b = shift % 32;
        unsigned __int128 v = 0;
        for (int i = 3; i >= 0; --i) {
            const size_t idx = w + (size_t)i;
            v = (v << 32) | (idx < x.mag.size() ? x.mag[idx] : 0u);
        }
        const size_t top = w + 4;                        // the bits above the four limbs
        const uint32_t hi = top < x.mag.size() ? x.mag[top] : 0u;
        return b ? (v >> b) | ((unsigned __int128)hi << (128 - b)) : v;
    }
    // a x - b y for magnitudes when the result is >= 0 (a, b < 2^63).
    static std::vector<uint32_t> lin_sub_mag(const std::vector<uint32_t> &x, uint64_t a,
                                             const std::vector<uint32_t> &y, uint64_t b) {
        const size_t n = std::max(x.size(), y.size()) + 2;
        std::vector<uint32_t> r(n);
        __int128 carry = 0;
        for (size_t i = 0; i < n; ++i) {
            const __int128 t = (__int128)(i < x.size() ? x[i] : 0u) * a -
                               (__int128)(i < y.size() ? y[i] : 0u) * b + carry;
            const uint32_t lo = (uint32_t)(uint64_t)t;
            r[i] = lo;
            carry = (t - (__int128)lo) >> 32;            // exact: t - lo is a multiple of 2^32
        }
        while (!r.empty() && r.back() == 0) r.pop_back();
        return r;
    }
    // a x + b y for magnitudes.
    static std::vector<uint32_t> lin_add_mag(const std::vector<uint32_t> &x, uint64_t a,
                                             const std::vector<uint32_t> &y, uint64_t b) {
        const size_t n = std::max(x.size(), y.size()) + 3;
        std::vector<uint32_t> r(n);
        unsigned __int128 carry = 0;
        for (size_t i = 0; i < n; ++i) {
            const unsigned __int128 t = (unsigned __int128)(i < x.size() ? x[i] : 0u) * a +
                                        (unsigned __int128)(i < y.size() ? y[i] : 0u) * b + carry;
            r[i] = (uint32_t)t;
            carry = t >> 32;
        }
        while (!r.empty() && r.back() == 0) r.pop_back();
        return r;
    }
    // Advances r0 >= r1 >= 0 (and the cofactors when track) by Lehmer runs
    // while r1 has more than stop_bits + 130 bits; the caller finishes with
    // euclid_step.
    static void lehmer_run(BigInt &r0, BigInt &r1, BigInt &t0, BigInt &t1, size_t stop_bits, bool track) {
        // |A|, |B|, |C|, |D| < lim; the leading digits are below 2^124, so
        // every sum, product and quotient below fits a signed 128-bit word.
        const __int128 lim = (__int128)1 << 62;
        while (!r1.is_zero() && r1.bit_length() > stop_bits + 130) {
            const size_t shift = r0.bit_length() - 124;
            __int128 uh = (__int128)shifted_u128(r0, shift), vh = (__int128)shifted_u128(r1, shift);
            int64_t A = 1, B = 0, C = 0, D = 1;
            for (;;) {
                const __int128 dc = vh + C, dd = vh + D;
                if (dc <= 0 || dd <= 0) break;
                const __int128 q1 = (uh + A) / dc, q2 = (uh + B) / dd;
                if (q1 != q2 || q1 < 1 || q1 >= lim) break;
                const __int128 nC = (__int128)A - q1 * C, nD = (__int128)B - q1 * D;
                if (nC >= lim || nC <= -lim || nD >= lim || nD <= -lim) break;
                A = C; C = (int64_t)nC;
                B = D; D = (int64_t)nD;
                const __int128 nv = uh - q1 * vh;
                uh = vh; vh = nv;
            }
            if (B == 0) {                                 // no run found: one exact step
                euclid_step(r0, r1, t0, t1, track);
                continue;
            }
            // Each matrix row (a, b) has entries of opposite signs (or a zero):
            // a r0 + b r1 is a difference of magnitudes (the result is a
            // remainder, >= 0); the cofactors alternate in sign, so a t0 + b t1
            // is a sum of magnitudes with the sign of its nonzero terms.
            auto rem = [&](int64_t a, int64_t b) {
                BigInt r;
                r.mag = b <= 0 ? lin_sub_mag(r0.mag, (uint64_t)a, r1.mag, (uint64_t)(-b))
                               : lin_sub_mag(r1.mag, (uint64_t)b, r0.mag, (uint64_t)(-a));
                return r;
            };
            auto cof = [&](int64_t a, int64_t b) {
                BigInt r;
                const uint64_t ua = (uint64_t)(a < 0 ? -a : a), ub = (uint64_t)(b < 0 ? -b : b);
                r.mag = lin_add_mag(t0.mag, ua, t1.mag, ub);
                const bool neg_ = (a != 0 && !t0.is_zero()) ? ((a < 0) != t0.neg) : ((b < 0) != t1.neg);
                r.neg = neg_ && !r.mag.empty();
                return r;
            };
            BigInt n0 = rem(A, B), n1 = rem(C, D);
            if (track) {
                BigInt s0 = cof(A, B), s1 = cof(C, D);
                t0 = std::move(s0);
                t1 = std::move(s1);
            }
            r0 = std::move(n0);
            r1 = std::move(n1);
        }
    }

    static BigInt gcd(BigInt a, BigInt b) {
        a.neg = b.neg = false;
        if (cmp_mag(a.mag, b.mag) < 0) std::swap(a, b);
        BigInt t0, t1;
        lehmer_run(a, b, t0, t1, 0, false);
        while (!b.is_zero()) euclid_step(a, b, t0, t1, false);
        return a;
    }
    static BigInt lcm(const BigInt &a, const BigInt &b) {
        if (a.is_zero() || b.is_zero()) return BigInt(0);
        return abs(a) / gcd(a, b) * abs(b);
    }
    // g = gcd(a, b) >= 0 with x*a + y*b = g.
    static BigInt xgcd(const BigInt &a0, const BigInt &b0, BigInt &x, BigInt &y) {
        if (b0.is_zero()) {
            x = BigInt(a0.neg ? -1 : (a0.is_zero() ? 0 : 1));
            y = BigInt(0);
            return abs(a0);
        }
        BigInt r0 = abs(a0), r1 = abs(b0), t0(1), t1(0);     // t: cofactor of |a0|
        if (cmp_mag(r0.mag, r1.mag) < 0) euclid_step(r0, r1, t0, t1, true);
        lehmer_run(r0, r1, t0, t1, 0, true);
        while (!r1.is_zero()) euclid_step(r0, r1, t0, t1, true);
        // t0 |a0| = r0 (mod |b0|): the cofactor of |b0| follows exactly.
        const BigInt yb = (r0 - t0 * abs(a0)) / abs(b0);
        x = a0.neg ? -t0 : t0;
        y = b0.neg ? -yb : yb;
        return r0;
    }
    // Rational reconstruction: y mod m -> (num, den) with |num| < B, 0 < den < B
    // and num = den y (mod m), for B = 2^floor((bits(m) - 2) / 2), so that
    // 2 B^2 < m and such a fraction is unique.  False if none exists.  The
    // caller checks that den is prime to m where that matters.
    static bool rat_recon(const BigInt &y, const BigInt &m, BigInt &num, BigInt &den) {
        const size_t bb = (m.bit_length() - 2) / 2;
        const BigInt Bnd = BigInt(1).shl(bb);
        BigInt r0 = m, r1 = mod(y, m), t0(0), t1(1);
        lehmer_run(r0, r1, t0, t1, bb, true);
        while (cmp(r1, Bnd) >= 0) euclid_step(r0, r1, t0, t1, true);
        if (t1.is_zero() || cmp(abs(t1), Bnd) >= 0) return false;
        num = t1.neg ? -r1 : r1;
        den = abs(t1);
        return true;
    }
    BigInt shl(size_t bits) const {
        BigInt r;
        if (is_zero()) return r;
        const size_t w = bits / 32, b = bits % 32;
        r.mag.assign(mag.size() + w + 1, 0);
        for (size_t i = 0; i < mag.size(); ++i) {
            r.mag[i + w] |= mag[i] << b;
            if (b) r.mag[i + w + 1] |= (uint32_t)((uint64_t)mag[i] >> (32 - b));
        }
        r.neg = neg;
        r.trim();
        return r;
    }
    // Integer square root of a non-negative value (floor).
    static BigInt isqrt(const BigInt &a) {
        if (a.is_zero()) return BigInt(0);
        BigInt x = BigInt(1).shl((a.bit_length() + 1) / 2 + 1);
        while (true) {
            const BigInt y = x + a / x;
            BigInt q, r;
            divmod_trunc(y, BigInt(2), q, r);
            if (!(q < x)) return x;
            x = q;
        }
    }
};

// Reduction modulo one fixed m > 0 by Barrett's method (Handbook of Applied
// Cryptography, Algorithm 14.42): with B = 2^32, k the limbs of m and
// mu = floor(B^2k / m) found once, x < B^2k costs two products and at most
// two subtractions instead of a long division.  Larger x fall back to mod.
class ModReducer {
public:
    explicit ModReducer(const BigInt &m) : m_(BigInt::abs(m)), k_(m_.mag.size()) {
        if (k_ == 0) return;
        std::vector<uint32_t> p(2 * k_ + 1, 0u), r;
        p[2 * k_] = 1;
        BigInt::divmod_mag(p, m_.mag, mu_, r);
    }
    const BigInt &modulus() const { return m_; }
    // The non-negative residue of x.
    BigInt reduce(const BigInt &x) const {
        if (x.mag.size() > 2 * k_ || k_ < 2) return mod(x, m_);
        BigInt r;
        if (x.mag.size() < k_) {
            r.mag = x.mag;                                   // |x| < m already
        } else {
            const std::vector<uint32_t> q1(x.mag.begin() + (k_ - 1), x.mag.end());
            const std::vector<uint32_t> q2 = BigInt::mul_mag(q1, mu_);
            if (q2.size() > k_ + 1) {
                const std::vector<uint32_t> q3(q2.begin() + (k_ + 1), q2.end());
                r.mag = BigInt::sub_mag(x.mag, BigInt::mul_mag(q3, m_.mag));   // q3 <= floor(|x| / m)
            } else {
                r.mag = x.mag;
            }
            while (BigInt::cmp_mag(r.mag, m_.mag) >= 0) r.mag = BigInt::sub_mag(r.mag, m_.mag);
        }
        if (x.neg && !r.mag.empty()) r.mag = BigInt::sub_mag(m_.mag, r.mag);
        return r;
    }

private:
    BigInt m_;
    size_t k_;
    std::vector<uint32_t> mu_;
};

// The primes below 2^16 (sieve of Eratosthenes, built once).
inline const std::vector<uint32_t> &small_primes() {
    static const std::vector<uint32_t> primes = [] {
        std::vector<char> comp(65536, 0);
        std::vector<uint32_t> v;
        for (uint32_t q = 2; q < 65536; ++q) {
            if (comp[q]) continue;
            v.push_back(q);
            for (uint32_t m = q * q; m < 65536; m += q) comp[m] = 1;
        }
        return v;
    }();
    return primes;
}

// True when every prime factor of s > 0 is below 2^16: s is divided by its
// gcd with the product of those primes (built once) until the gcd is 1.
inline bool smooth16(const BigInt &s) {
    static const BigInt primorial = [] {
        BigInt q(1);
        for (uint32_t p : small_primes()) q = q.mul_small(p);
        return q;
    }();
    BigInt rest = BigInt::abs(s);
    while (!rest.is_one() && !rest.is_zero()) {
        const BigInt g = BigInt::gcd(primorial, rest);
        if (g.is_one()) return false;
        rest = rest / g;
    }
    return rest.is_one();
}

}  // namespace rns
