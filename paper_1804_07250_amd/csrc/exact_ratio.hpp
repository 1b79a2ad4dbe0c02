// Exact positive rationals for the acceptance thresholds (host only).
//
// Every finite double is an exact dyadic rational m 2^e, so the weight ratios
// W_up / W_down the tables are built from (products and quotients of the
// weights the caller passes) are exact rationals N / D of unbounded integers,
// and T = floor(2^32 p) is computed without rounding: heat-bath
// p = N / (N + D), lazy Metropolis min(1, R) / 2 and 1 - min(1, 1/R) / 2.
#pragma once
#include <stdint.h>

#include <vector>

namespace tl {

// Unsigned integer of any size: 32-bit limbs, least significant first, no
// leading zero limbs (zero is the empty vector).
class BigU {
public:
    BigU() = default;
    explicit BigU(uint64_t v);
    bool zero() const { return d_.empty(); }
    BigU operator*(const BigU &o) const;
    BigU operator+(const BigU &o) const;
    BigU shl(uint32_t bits) const;
    // -1, 0, 1 as *this <, ==, > o
    int cmp(const BigU &o) const;
    // floor(*this / o) when that quotient is below 2^33 (o != 0)
    uint64_t small_quotient(const BigU &o) const;

private:
    void trim();
    std::vector<uint32_t> d_;
};

// A positive rational N / D.
struct Ratio {
    BigU num{1}, den{1};
    // Exact value of a positive finite double.
    static Ratio of(double v);
    Ratio operator*(const Ratio &o) const;
    Ratio operator/(const Ratio &o) const;
    Ratio inv() const { return Ratio{den, num}; }
    Ratio pow(int e) const;   // any integer exponent
};

// Threshold tables from exact up/down weight ratios R (heat-bath: one entry
// per context; lazy Metropolis: the pair [current down, current up] per
// context).  Returns false when a Metropolis "up" entry would need 2^32
// (R above 2^31: the state would never leave up), which a 32-bit table
// cannot hold.
bool exact_thresholds(const std::vector<Ratio> &R, bool metropolis, std::vector<uint32_t> &out);

}  // namespace tl
