// Host-side configuration of an emulated-DGEMM plan: modulus set, CRT
// constants, exactness caps and kept-bit rules (Sec. III-A, III-C, V).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "ozemu_internal.hpp"

namespace ozemu {

// Unsigned multiword integer, little-endian 32-bit digits, fixed capacity.
struct BigU {
    uint32_t d[kMaxDigits + 2] = {};
    static constexpr int cap = kMaxDigits + 2;
    static BigU from_u64(uint64_t v);
    BigU& mul_small(uint32_t f);           // *= f (f < 2^32); overflow is a bug
    uint32_t div_small(uint32_t f);         // /= f, returns remainder
    uint32_t mod_small(uint32_t f) const;   // remainder only
    BigU& sub(const BigU& o);               // -= o, requires *this >= o
    BigU& add_small(uint32_t v);
    BigU& shr1();
    int bit_length() const;
    int cmp(const BigU& o) const;
    bool is_zero() const;
    double log2() const;
};

struct Plan {
    int format = 0;
    int scaling = 0;
    int n = 0;
    std::vector<int> moduli;  // descending
    BigU P;
    int p_bits = 0;
    int64_t kappa_acc = 0;    // Lambda_INT32 / max radius^2
    ModConsts mod{};
    CrtConsts crt{};
};

// Largest-product pairwise-coprime set of `count` integers in [2, limit]
// (ties: lexicographically largest descending list). Empty on failure.
std::vector<int> best_coprime_set(int count, int limit);

// Builds constants; returns an empty string or an error message.
std::string build_plan(Plan& p, int format, const std::vector<int>& moduli, int scaling);

// floor(log2((P - 1) / (2 k))) for k >= 1, or -1 if (P - 1) / (2k) < 1.
int window_bits(const Plan& p, int64_t k);

// True when P > 2 k (2^ba - 1)(2^bb - 1) (CRT window, eq. "ov-crtgen").
bool window_holds(const Plan& p, int64_t k, int ba, int bb);

// floor(log2((P - 1) / 2)): the L of the bound-adaptive mode.
int half_window_bits(const Plan& p);

}  // namespace ozemu
