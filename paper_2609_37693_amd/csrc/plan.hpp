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

// One limb channel: modulus, rank (1 one-limb, 3 two-limb Toom), base.
struct FpChannel {
    int m = 0, rank = 0, base = 0;
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
    // float-alphabet plans (format != 0)
    int64_t k_slab = 0;                 // terms per accumulation slab
    std::vector<FpChannel> chans;
    FpConsts fp{};
    std::vector<uint8_t> tables;        // code tables of all channels
    uint8_t* pinned_tables = nullptr;   // pinned copy for uploads (first call)
};

// Float-alphabet plan (format 1 E4M3, 3 E2M1): the channel pool at slab
// length k_slab (one-limb and two-limb Toom channels within the radius
// floor(sqrt(2^24 / k_slab))), then the coprime selection: within `gemms`
// GEMMs the largest product, or for gemms == 0 the least GEMM count whose
// product exceeds k_slab * 2^107. Builds the code tables and constants.
std::string build_plan_fp(Plan& p, int format, int gemms, int64_t k_slab, int scaling);

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
