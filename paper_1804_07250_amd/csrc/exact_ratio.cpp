// Exact rational thresholds (see exact_ratio.hpp).
#include "exact_ratio.hpp"

#include <math.h>

#include <algorithm>

namespace tl {

BigU::BigU(uint64_t v)
{
    while (v) {
        d_.push_back((uint32_t)v);
        v >>= 32;
    }
}

void BigU::trim()
{
    while (!d_.empty() && d_.back() == 0u) d_.pop_back();
}

BigU BigU::operator*(const BigU &o) const
{
    BigU r;
    if (zero() || o.zero()) return r;
    r.d_.assign(d_.size() + o.d_.size(), 0u);
    for (size_t i = 0; i < d_.size(); ++i) {
        uint64_t carry = 0;
        for (size_t j = 0; j < o.d_.size(); ++j) {
            const uint64_t t = (uint64_t)d_[i] * o.d_[j] + r.d_[i + j] + carry;
            r.d_[i + j] = (uint32_t)t;
            carry = t >> 32;
        }
        size_t k = i + o.d_.size();
        while (carry) {
            const uint64_t t = (uint64_t)r.d_[k] + carry;
            r.d_[k++] = (uint32_t)t;
            carry = t >> 32;
        }
    }
    r.trim();
    return r;
}

BigU BigU::operator+(const BigU &o) const
{
    BigU r;
    const size_t n = std::max(d_.size(), o.d_.size());
    r.d_.assign(n + 1, 0u);
    uint64_t carry = 0;
    for (size_t i = 0; i < n; ++i) {
        const uint64_t t = (uint64_t)(i < d_.size() ? d_[i] : 0u) + (i < o.d_.size() ? o.d_[i] : 0u) + carry;
        r.d_[i] = (uint32_t)t;
        carry = t >> 32;
    }
    r.d_[n] = (uint32_t)carry;
    r.trim();
    return r;
}

BigU BigU::shl(uint32_t bits) const
{
    BigU r;
    if (zero()) return r;
    const uint32_t limbs = bits / 32u, sh = bits % 32u;
    r.d_.assign(d_.size() + limbs + 1, 0u);
    for (size_t i = 0; i < d_.size(); ++i) {
        const uint64_t v = (uint64_t)d_[i] << sh;
        r.d_[i + limbs] |= (uint32_t)v;
        r.d_[i + limbs + 1] |= (uint32_t)(v >> 32);
    }
    r.trim();
    return r;
}

int BigU::cmp(const BigU &o) const
{
    if (d_.size() != o.d_.size()) return d_.size() < o.d_.size() ? -1 : 1;
    for (size_t i = d_.size(); i-- > 0;)
        if (d_[i] != o.d_[i]) return d_[i] < o.d_[i] ? -1 : 1;
    return 0;
}

uint64_t BigU::small_quotient(const BigU &o) const
{
    // the largest q < 2^33 with q * o <= *this, bit by bit from the top
    uint64_t q = 0;
    for (int b = 32; b >= 0; --b) {
        const uint64_t c = q | (1ull << b);
        if ((o * BigU(c)).cmp(*this) <= 0) q = c;
    }
    return q;
}

Ratio Ratio::of(double v)
{
    // v = m 2^e with m a 53-bit integer
    int e = 0;
    const double f = frexp(v, &e);
    const uint64_t m = (uint64_t)ldexp(f, 53);
    e -= 53;
    Ratio r;
    r.num = BigU(m);
    r.den = BigU(1);
    if (e >= 0) r.num = r.num.shl((uint32_t)e);
    else r.den = r.den.shl((uint32_t)-e);
    return r;
}

Ratio Ratio::operator*(const Ratio &o) const { return Ratio{num * o.num, den * o.den}; }

Ratio Ratio::operator/(const Ratio &o) const { return Ratio{num * o.den, den * o.num}; }

Ratio Ratio::pow(int e) const
{
    Ratio r;
    const Ratio b = e >= 0 ? *this : inv();
    for (int i = 0; i < (e >= 0 ? e : -e); ++i) r = r * b;
    return r;
}

bool exact_thresholds(const std::vector<Ratio> &R, bool metropolis, std::vector<uint32_t> &out)
{
    out.clear();
    for (const Ratio &r : R) {
        if (!metropolis) {
            // floor(2^32 N / (N + D)) < 2^32
            out.push_back((uint32_t)r.num.shl(32).small_quotient(r.num + r.den));
        } else {
            // current down: floor(2^31 min(1, N / D))
            const uint64_t dn = r.num.cmp(r.den) >= 0 ? (1ull << 31) : r.num.shl(31).small_quotient(r.den);
            // current up: 2^32 - floor(2^31 min(1, D / N))
            const uint64_t f = r.den.cmp(r.num) >= 0 ? (1ull << 31) : r.den.shl(31).small_quotient(r.num);
            if (f == 0) return false;
            out.push_back((uint32_t)dn);
            out.push_back((uint32_t)((1ull << 32) - f));
        }
    }
    return true;
}

}  // namespace tl
