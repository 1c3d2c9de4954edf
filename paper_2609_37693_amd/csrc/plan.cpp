// Host configuration build for libozemu (Sec. V: a configuration is built
// once from its moduli; building checks the accumulator bound and the CRT
// window and refuses k above the reconstruction cap).
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <map>
#include <numeric>

namespace ozemu {

BigU BigU::from_u64(uint64_t v) {
    BigU r;
    r.d[0] = (uint32_t)v;
    r.d[1] = (uint32_t)(v >> 32);
    return r;
}

BigU& BigU::mul_small(uint32_t f) {
    uint64_t carry = 0;
    for (int i = 0; i < cap; ++i) {
        uint64_t t = (uint64_t)d[i] * f + carry;
        d[i] = (uint32_t)t;
        carry = t >> 32;
    }
    return *this;
}

uint32_t BigU::div_small(uint32_t f) {
    uint64_t rem = 0;
    for (int i = cap - 1; i >= 0; --i) {
        uint64_t cur = (rem << 32) | d[i];
        d[i] = (uint32_t)(cur / f);
        rem = cur % f;
    }
    return (uint32_t)rem;
}

uint32_t BigU::mod_small(uint32_t f) const {
    uint64_t rem = 0;
    for (int i = cap - 1; i >= 0; --i) rem = ((rem << 32) | d[i]) % f;
    return (uint32_t)rem;
}

BigU& BigU::sub(const BigU& o) {
    int64_t borrow = 0;
    for (int i = 0; i < cap; ++i) {
        int64_t t = (int64_t)d[i] - o.d[i] - borrow;
        borrow = t < 0;
        d[i] = (uint32_t)(t + (borrow ? (1ll << 32) : 0));
    }
    return *this;
}

BigU& BigU::add_small(uint32_t v) {
    uint64_t carry = v;
    for (int i = 0; i < cap && carry; ++i) {
        uint64_t t = (uint64_t)d[i] + carry;
        d[i] = (uint32_t)t;
        carry = t >> 32;
    }
    return *this;
}

BigU& BigU::shr1() {
    for (int i = 0; i < cap; ++i) {
        uint32_t hi = (i + 1 < cap) ? d[i + 1] : 0;
        d[i] = (d[i] >> 1) | (hi << 31);
    }
    return *this;
}

int BigU::bit_length() const {
    for (int i = cap - 1; i >= 0; --i)
        if (d[i]) return 32 * i + (32 - __builtin_clz(d[i]));
    return 0;
}

int BigU::cmp(const BigU& o) const {
    for (int i = cap - 1; i >= 0; --i)
        if (d[i] != o.d[i]) return d[i] < o.d[i] ? -1 : 1;
    return 0;
}

bool BigU::is_zero() const {
    for (int i = 0; i < cap; ++i)
        if (d[i]) return false;
    return true;
}

double BigU::log2() const {
    double v = 0;
    for (int i = cap - 1; i >= 0; --i) v = v * 4294967296.0 + d[i];
    return std::log2(v);
}

namespace {

struct Cand {
    BigU prod;
    std::vector<int> members;  // descending
    bool valid = false;
};

// a better than b: larger product, then lexicographically larger members.
bool better(const Cand& a, const Cand& b) {
    if (!b.valid) return a.valid;
    if (!a.valid) return false;
    int c = a.prod.cmp(b.prod);
    if (c != 0) return c > 0;
    return std::lexicographical_compare(b.members.begin(), b.members.end(), a.members.begin(),
                                        a.members.end());
}

bool is_prime(int v) {
    if (v < 2) return false;
    for (int q = 2; q * q <= v; ++q)
        if (v % q == 0) return false;
    return true;
}

}  // namespace

std::vector<int> best_coprime_set(int count, int limit) {
    if (count < 1 || limit < 2) return {};
    // Every integer <= limit has at most one prime factor p with p*p > limit.
    std::vector<int> small;
    for (int p = 2; p * p <= limit; ++p)
        if (is_prime(p)) small.push_back(p);
    if (small.size() > 20) return {};
    // items: each either one number (no large factor) or all numbers sharing
    // one large prime (choose at most one).
    std::map<int, std::vector<std::pair<int, uint32_t>>> by_large;
    std::vector<std::vector<std::pair<int, uint32_t>>> items;
    for (int v = 2; v <= limit; ++v) {
        int r = v;
        uint32_t mask = 0;
        for (size_t i = 0; i < small.size(); ++i) {
            if (r % small[i] == 0) {
                mask |= 1u << i;
                while (r % small[i] == 0) r /= small[i];
            }
        }
        if (r == 1)
            items.push_back({{v, mask}});
        else
            by_large[r].push_back({v, mask});
    }
    for (auto& kv : by_large) items.push_back(kv.second);

    const int masks = 1 << small.size();
    auto idx = [&](uint32_t mask, int size) { return (size_t)size * masks + mask; };
    std::vector<Cand> best((size_t)(count + 1) * masks);
    best[idx(0, 0)].valid = true;
    best[idx(0, 0)].prod = BigU::from_u64(1);
    for (const auto& group : items) {
        std::vector<Cand> next = best;
        for (int size = 0; size < count; ++size) {
            for (int mask = 0; mask < masks; ++mask) {
                const Cand& c = best[idx(mask, size)];
                if (!c.valid) continue;
                for (const auto& it : group) {
                    if (it.second & (uint32_t)mask) continue;
                    Cand n;
                    n.valid = true;
                    n.prod = c.prod;
                    n.prod.mul_small((uint32_t)it.first);
                    n.members = c.members;
                    n.members.push_back(it.first);
                    std::sort(n.members.rbegin(), n.members.rend());
                    Cand& slot = next[idx(mask | it.second, size + 1)];
                    if (better(n, slot)) slot = n;
                }
            }
        }
        best.swap(next);
    }
    Cand win;
    for (int mask = 0; mask < masks; ++mask)
        if (better(best[idx(mask, count)], win)) win = best[idx(mask, count)];
    return win.valid ? win.members : std::vector<int>{};
}

std::string build_plan(Plan& p, int format, const std::vector<int>& moduli_in, int scaling) {
    if (format != 0) return "unsupported format";
    if (scaling < 0 || scaling > 2) return "unknown scaling mode";
    int n = (int)moduli_in.size();
    if (n < 2 || n > kMaxModuli) return "number of moduli must be in [2, 32]";
    std::vector<int> ms = moduli_in;
    std::sort(ms.rbegin(), ms.rend());
    for (int i = 0; i < n; ++i) {
        if (ms[i] < 2 || ms[i] > 256) return "INT8 moduli must lie in [2, 256]";
        for (int j = i + 1; j < n; ++j)
            if (std::gcd(ms[i], ms[j]) != 1) return "moduli must be pairwise coprime";
    }
    p.format = format;
    p.scaling = scaling;
    p.n = n;
    p.moduli = ms;
    p.P = BigU::from_u64(1);
    for (int m : ms) p.P.mul_small((uint32_t)m);
    p.p_bits = p.P.bit_length();
    int rmax = 0;
    for (int m : ms) rmax = std::max(rmax, m / 2);
    p.kappa_acc = (int64_t)((2147483647ll) / ((int64_t)rmax * rmax));

    p.mod.n = n;
    p.crt.n = n;
    // digits: N * P < 2^(p_bits + 5) plus a sign bit
    int digits = (p.p_bits + 6 + 31) / 32;
    if (digits > kMaxDigits) return "modulus product too large";
    p.crt.d = digits;
    for (int l = 0; l < n; ++l) {
        uint32_t m = (uint32_t)ms[l];
        uint32_t mu = (uint32_t)((1ull << 32) / m);
        p.mod.m[l] = m;
        p.mod.mu[l] = mu;
        p.mod.c32[l] = (uint32_t)((1ull << 32) % m);
        p.mod.c16[l] = (uint32_t)((1ull << 16) % m);
        p.mod.rcp[l] = 1.0f / (float)m;
        for (int i = 0; i < 6; ++i) {
            uint64_t w = 1 % m;
            for (int b = 0; b < 12 * i; ++b) w = (w * 2) % m;
            p.mod.w12[l][i] = (uint16_t)w;
        }
        p.crt.m[l] = m;
        p.crt.mu[l] = mu;
        p.crt.rcp[l] = 1.0 / (double)m;
        BigU Ml = p.P;
        uint32_t rem = Ml.div_small(m);
        if (rem != 0) return "internal: P not divisible";
        uint32_t Mm = Ml.mod_small(m);
        uint32_t inv = 0;
        for (uint32_t c = 1; c < m; ++c)
            if ((Mm * c) % m == 1) { inv = c; break; }
        if (m == 1 || inv == 0) return "internal: no inverse";
        p.crt.inv[l] = inv;
        for (int i = 0; i < kMaxDigits; ++i) p.crt.Ml[l][i] = Ml.d[i];
    }
    BigU half = p.P;
    BigU one = BigU::from_u64(1);
    half.sub(one).shr1();
    for (int i = 0; i < kMaxDigits; ++i) {
        p.crt.P[i] = p.P.d[i];
        p.crt.half[i] = half.d[i];
    }
    return "";
}

int window_bits(const Plan& p, int64_t k) {
    if (k < 1) k = 1;
    if (k > 0x7FFFFFFFll) return -1;
    BigU q = p.P;
    q.sub(BigU::from_u64(1));
    q.div_small((uint32_t)(2 * k));  // 2k < 2^32
    if (q.is_zero()) return -1;
    return q.bit_length() - 1;
}

bool window_holds(const Plan& p, int64_t k, int ba, int bb) {
    // 2 k (2^ba - 1)(2^bb - 1) < P  <=>  rhs computed exactly and compared.
    if (ba < 0 || bb < 0) return false;
    if (ba == 0 || bb == 0) return true;
    BigU r = BigU::from_u64(2ull * (uint64_t)k);
    int total = ba + bb + 1 + 64;
    if (total > 32 * BigU::cap - 8) return false;
    // multiply by (2^ba - 1): r*2^ba - r
    auto mul_pow2m1 = [](BigU& x, int b) {
        BigU y = x;
        for (int i = 0; i < b; ++i) {
            uint32_t carry = 0;
            for (int j = 0; j < BigU::cap; ++j) {
                uint32_t nc = x.d[j] >> 31;
                x.d[j] = (x.d[j] << 1) | carry;
                carry = nc;
            }
        }
        x.sub(y);
    };
    mul_pow2m1(r, ba);
    mul_pow2m1(r, bb);
    return r.cmp(p.P) < 0;
}

int half_window_bits(const Plan& p) {
    BigU h = p.P;
    h.sub(BigU::from_u64(1)).shr1();
    return h.bit_length() - 1;
}

}  // namespace ozemu
