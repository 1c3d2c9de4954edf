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

std::string fill_moduli(Plan& p, const std::vector<int>& ms);

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
    return fill_moduli(p, ms);
}

// Bits [cb c, cb c + cb) of a big integer.
static uint64_t chunk_of(const BigU& x, int c, int cb) {
    uint64_t v = 0;
    for (int b = 0; b < cb; ++b) {
        const int bit = cb * c + b;
        if (bit / 32 < BigU::cap && ((x.d[bit / 32] >> (bit % 32)) & 1u)) v |= 1ull << b;
    }
    return v;
}

// P, caps, Barrett, digit-weight and CRT constants of a sorted modulus set.
std::string fill_moduli(Plan& p, const std::vector<int>& ms) {
    const int n = (int)ms.size();
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
        {
            // strictly above 1/m: the next FP32 value up when 1/m is exact
            float r = 1.0f / (float)m;
            if ((double)r * (double)m <= 1.0) r = std::nextafter(r, 1.0f);  // exact test
            p.mod.rcp_up[l] = r;
            const uint64_t c = (uint64_t)((((unsigned __int128)1) << 64) % m);
            p.mod.c64n[l] = (uint32_t)((m - c) % m);
        }
        p.mod.km[l] = m * (((1u << 17) + m - 1) / m);
        p.mod.s8[l][0] = p.mod.s8[l][1] = 0;
        p.mod.w8[l][0] = p.mod.w8[l][1] = 0;
        if (m <= 256)
            for (int i = 0; i < 8; ++i) {
                uint64_t w = 1 % m;
                for (int b = 0; b < 8 * i; ++b) w = (w * 2) % m;
                p.mod.w8[l][i / 4] |= (uint32_t)w << (8 * (i % 4));
                const int64_t bal = (int64_t)w > (int64_t)m / 2 ? (int64_t)w - m : (int64_t)w;
                p.mod.s8[l][i / 4] |= (uint32_t)(uint8_t)(int8_t)bal << (8 * (i % 4));
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
        // N_l = inv_l M_l < m_l M_l = P, in chunks of cb bits
        BigU Nl = Ml;
        Nl.mul_small(inv);
        const int cb = p.format == 0 ? kChunkBits : kChunkBitsFp;
        for (int c = 0; c < kMaxChunks; ++c) p.crt.N40[l][c] = (double)chunk_of(Nl, c, cb);
    }
    p.crt.cb = p.format == 0 ? kChunkBits : kChunkBitsFp;  // INT8 plans: format 0
    p.crt.kc = (p.p_bits + 2 + p.crt.cb - 1) / p.crt.cb;
    if (p.crt.kc > kMaxChunks) {
        if (p.format == 0) return "modulus product too large";
        p.crt.kc = 0;  // float channels: 32-bit digits instead
    }
    {
        double Pd = 0;  // P to within a few ulps
        for (int i = BigU::cap - 1; i >= 0; --i) Pd = Pd * 4294967296.0 + p.P.d[i];
        for (int c = 0; c < kMaxChunks; ++c) {
            p.crt.P40[c] = (double)chunk_of(p.P, c, p.crt.cb);
            p.crt.R40[c] = std::ldexp(1.0 / Pd, p.crt.cb * c);
        }
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

// ---- Float alphabets ----

namespace {

constexpr int64_t kLambdaFp32 = 1ll << 24;

// Integer alphabet of a format (finite values times 2^es) with the code of
// each value: exponent/mantissa fields of the OCP formats; E4M3 has no
// infinities and one NaN pattern per sign (exponent and mantissa all ones).
struct Alphabet {
    int es = 0;
    std::map<int, uint8_t> code;  // value -> code (non-negative zero for 0)
};

bool alphabet_of(int format, Alphabet& a) {
    int E, M;
    bool fn;
    if (format == 1) {  // E4M3
        E = 4, M = 3, fn = true, a.es = 9;
    } else if (format == 2) {  // E2M3 (FP6: no infinities or NaN)
        E = 2, M = 3, fn = false, a.es = 3;
    } else if (format == 3) {  // E2M1
        E = 2, M = 1, fn = false, a.es = 1;
    } else {
        return false;
    }
    const int bias = (1 << (E - 1)) - 1;
    for (int sgn = 1; sgn >= 0; --sgn)  // positive codes last, so +0 wins
        for (int ex = 0; ex < (1 << E); ++ex)
            for (int mt = 0; mt < (1 << M); ++mt) {
                if (fn && ex == (1 << E) - 1 && mt == (1 << M) - 1) continue;
                // value * 2^es: subnormal mt * 2^(1 - bias - M + es), normal
                // (2^M + mt) * 2^(ex - bias - M + es)
                const int sh = (ex == 0 ? 1 : ex) - bias - M + a.es;
                const int mag = (ex == 0 ? mt : ((1 << M) + mt));
                if (sh < 0) return false;  // es is the least making all integral
                const int v = mag << sh;
                a.code[sgn ? -v : v] = (uint8_t)((sgn << (E + M)) | (ex << M) | mt);
            }
    return true;
}

bool covers(const std::vector<int>& vals, int m) {
    std::vector<char> hit(m, 0);
    int cnt = 0;
    for (int v : vals) {
        int r = ((v % m) + m) % m;
        if (!hit[r]) hit[r] = 1, ++cnt;
    }
    return cnt == m;
}

// L(m): log2 m with 32 fraction bits, repeated squaring in 62-bit fixed
// point truncated after each square.
int64_t fixed_log2(int64_t m) {
    int e = 63 - __builtin_clzll((uint64_t)m);
    unsigned __int128 x = ((unsigned __int128)m << 62) >> e;
    int64_t out = e;
    const unsigned __int128 two = (unsigned __int128)2 << 62;
    for (int i = 0; i < 32; ++i) {
        x = (x * x) >> 62;
        out <<= 1;
        if (x >= two) {
            x >>= 1;
            out |= 1;
        }
    }
    return out;
}

std::vector<int> prime_factors(int n) {
    std::vector<int> out;
    for (int q = 2; (int64_t)q * q <= n; ++q)
        if (n % q == 0) {
            out.push_back(q);
            while (n % q == 0) n /= q;
        }
    if (n > 1) out.push_back(n);
    return out;
}

int isqrt64(int64_t v) {
    int64_t r = (int64_t)std::sqrt((double)v);
    while (r * r > v) --r;
    while ((r + 1) * (r + 1) <= v) ++r;
    return (int)r;
}

}  // namespace

std::string build_plan_fp(Plan& p, int format, int gemms, int64_t k_slab, int scaling) {
    Alphabet al;
    if (!alphabet_of(format, al)) return "unsupported float format";
    if (scaling != 0 && scaling != 1) return "float plans support F53 and WINDOW";
    if (k_slab < 128 || k_slab % 128 != 0 || k_slab > kLambdaFp32)
        return "k_slab must be a positive multiple of 128 up to 2^24";
    if (gemms < 0 || gemms > 3 * kMaxModuli) return "gemms out of range";
    const int r1 = isqrt64(kLambdaFp32 / k_slab);
    std::vector<int> Sr;
    for (auto& kv : al.code)
        if (std::abs(kv.first) <= r1) Sr.push_back(kv.first);
    std::vector<char> inS(2 * r1 + 1, 0);
    for (int v : Sr) inS[v + r1] = 1;
    auto in_sr = [&](int v) { return v >= -r1 && v <= r1 && inS[v + r1]; };
    // Toom-2 value sets per base
    const int bmax = 4 * r1 + 1;
    std::vector<std::vector<int>> tv(bmax + 1);
    size_t mmax = 0;
    for (int b = 2; b <= bmax; ++b) {
        std::vector<int>& v = tv[b];
        for (int c0 : Sr)
            for (int c1 : Sr)
                if (in_sr(c0 + c1)) v.push_back(c0 + b * c1);
        std::sort(v.begin(), v.end());
        v.erase(std::unique(v.begin(), v.end()), v.end());
        mmax = std::max(mmax, v.size());
    }
    // pool
    std::vector<FpChannel> pool;
    for (int m = 2; m <= (int)mmax; ++m) {
        if (covers(Sr, m)) {
            pool.push_back({m, 1, 0});
            continue;
        }
        for (int b = 2; b <= bmax; ++b) {
            if ((int)tv[b].size() < m || !covers(tv[b], m)) continue;
            const int64_t l0 = (((int64_t)(1 - b) % m) + m) % m, l1 = b % m,
                          l2 = ((((int64_t)b * b - b) % m) + m) % m;
            if (std::max<int64_t>(2 * m, (int64_t)(m - 1) * (l0 + l1 + l2)) <= kLambdaFp32) {
                pool.push_back({m, 3, b});
                break;
            }
        }
    }
    if (pool.empty()) return "empty channel pool";
    // selection: DP over (rank spent, small-prime mask), one member per large prime
    const int M = pool.back().m;
    const int tau = isqrt64(M);
    std::vector<int> small;
    for (int q = 2; q <= tau; ++q) {
        bool pr = true;
        for (int d = 2; d * d <= q; ++d)
            if (q % d == 0) pr = false;
        if (pr) small.push_back(q);
    }
    if (small.size() > 20) return "channel pool too wide";
    struct Item {
        int idx;
        uint32_t mask;
    };
    std::vector<std::vector<Item>> items;
    std::map<int, std::vector<Item>> by_large;
    for (int i = 0; i < (int)pool.size(); ++i) {
        uint32_t mask = 0;
        int large = 0;
        for (int f : prime_factors(pool[i].m)) {
            auto it = std::find(small.begin(), small.end(), f);
            if (it != small.end())
                mask |= 1u << (it - small.begin());
            else
                large = f;
        }
        if (large == 0)
            items.push_back({{i, mask}});
        else
            by_large[large].push_back({i, mask});
    }
    for (auto& kv : by_large) items.push_back(kv.second);
    const int qmax = gemms > 0 ? gemms : 3 * kMaxModuli;
    const int NM = 1 << small.size();
    const int64_t NEG = INT64_MIN / 4;
    std::vector<int64_t> best((size_t)(qmax + 1) * NM, NEG);
    best[0] = 0;
    struct Choice {
        int gi;
        int src;
    };
    std::vector<std::vector<Choice>> trail;  // per item group, dense (q, mask)
    for (const auto& grp : items) {
        std::vector<int64_t> nb = best;
        std::vector<Choice> ch((size_t)(qmax + 1) * NM, Choice{-1, 0});
        for (int gi = 0; gi < (int)grp.size(); ++gi) {
            const FpChannel& mb = pool[grp[gi].idx];
            const uint32_t mk = grp[gi].mask;
            const int64_t L = fixed_log2(mb.m);
            for (int q = 0; q + mb.rank <= qmax; ++q)
                for (int src = 0; src < NM; ++src) {
                    if (src & mk) continue;
                    const int64_t v = best[(size_t)q * NM + src];
                    if (v <= NEG) continue;
                    const size_t dst = (size_t)(q + mb.rank) * NM + (src | mk);
                    if (v + L > nb[dst]) {
                        nb[dst] = v + L;
                        ch[dst] = Choice{gi, src};
                    }
                }
        }
        trail.push_back(std::move(ch));
        best.swap(nb);
    }
    auto rebuild = [&](int q, int mask) {
        std::vector<FpChannel> out;
        for (int g = (int)items.size() - 1; g >= 0; --g) {
            const Choice c = trail[g][(size_t)q * NM + mask];
            if (c.gi >= 0) {
                const FpChannel& mb = pool[items[g][c.gi].idx];
                out.push_back(mb);
                q -= mb.rank;
                mask = c.src;
            }
        }
        std::sort(out.begin(), out.end(), [](const FpChannel& a, const FpChannel& b) { return a.m > b.m; });
        return out;
    };
    std::vector<FpChannel> chosen;
    if (gemms > 0) {
        size_t arg = 0;
        for (size_t i = 1; i < best.size(); ++i)
            if (best[i] > best[arg]) arg = i;  // first maximum: least q, then least mask
        chosen = rebuild((int)(arg / NM), (int)(arg % NM));
    } else {
        // least q whose product exceeds k_slab * 2^107, exactly
        BigU target = BigU::from_u64((uint64_t)k_slab);
        for (int i = 0; i < 107; ++i) target.mul_small(2);
        const int64_t lt = fixed_log2(k_slab) + (107ll << 32);
        const int64_t slack = 64 * ((int64_t)pool.size() + 1);
        for (int q = 0; q <= qmax && chosen.empty(); ++q) {
            std::vector<int> order;
            for (int mk = 0; mk < NM; ++mk)
                if (best[(size_t)q * NM + mk] >= lt - slack) order.push_back(mk);
            std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
                return best[(size_t)q * NM + a] > best[(size_t)q * NM + b];
            });
            for (int mk : order) {
                std::vector<FpChannel> c = rebuild(q, mk);
                BigU P = BigU::from_u64(1);
                for (const FpChannel& x : c) P.mul_small((uint32_t)x.m);
                if (P.cmp(target) > 0) {
                    chosen = c;
                    break;
                }
            }
        }
        if (chosen.empty()) return "no channel set of this alphabet reaches the window";
    }
    if (chosen.size() < 2 || (int)chosen.size() > kMaxModuli) return "channel count out of range";
    // constants and moduli
    std::vector<int> ms;
    for (const FpChannel& c : chosen) ms.push_back(c.m);
    p.format = format;
    p.scaling = scaling;
    std::string err = fill_moduli(p, ms);
    if (!err.empty()) return err;
    // each slab of k_slab terms is exact at radius r1; longer k runs in slabs
    p.kappa_acc = 1ll << 30;
    p.k_slab = k_slab;
    p.chans = chosen;
    // tables: per class the representing tuple of least (largest plane
    // magnitude, sum of limb magnitudes, reversed tuple) whose planes lie in S_r
    FpConsts& f = p.fp;
    f = FpConsts{};
    f.n = (int)chosen.size();
    f.fmt = format == 1 ? 0 : format == 2 ? 2 : 4;  // MFMA operand format codes
    f.es = al.es;
    p.tables.clear();
    int plane = 0;
    for (int c = 0; c < f.n; ++c) {
        const FpChannel& ch = chosen[c];
        const int m = ch.m;
        f.m[c] = (uint32_t)m;
        f.mu[c] = (uint32_t)((1ull << 32) / (uint32_t)m);
        f.rank[c] = ch.rank;
        f.plane0[c] = plane;
        f.toff[c] = (int32_t)p.tables.size();
        plane += ch.rank;
        for (int i = 0; i < 6; ++i) {
            uint64_t w = 1 % m;
            for (int b = 0; b < 12 * i; ++b) w = (w * 2) % m;
            f.w12[c][i] = (uint16_t)w;
        }
        if (ch.rank == 1) {
            f.lbar[c][0] = 1 % m;
            for (int t = 0; t < m; ++t) {
                int bestv = 0;
                bool have = false;
                for (int v : Sr) {
                    if (((v % m) + m) % m != t) continue;
                    // key (|v|, |v|, v): least magnitude, then the smaller value
                    if (!have || std::abs(v) < std::abs(bestv) ||
                        (std::abs(v) == std::abs(bestv) && v < bestv))
                        bestv = v, have = true;
                }
                if (!have) return "internal: class without a one-limb value";
                p.tables.push_back(al.code[bestv]);
            }
        } else {
            const int b = ch.base;
            f.lbar[c][0] = (uint32_t)((((int64_t)(1 - b) % m) + m) % m);
            f.lbar[c][1] = (uint32_t)(b % m);
            f.lbar[c][2] = (uint32_t)((((int64_t)b * b - b) % m + m) % m);
            struct Key {
                int mx, sum, c1, c0;
            };
            std::vector<Key> bk(m, Key{INT32_MAX, 0, 0, 0});
            for (int c0 : Sr)
                for (int c1 : Sr) {
                    if (!in_sr(c0 + c1)) continue;
                    const int t = (int)((((int64_t)c0 + (int64_t)b * c1) % m + m) % m);
                    const Key k{std::max(std::max(std::abs(c0), std::abs(c1)), std::abs(c0 + c1)),
                                std::abs(c0) + std::abs(c1), c1, c0};
                    const Key& o = bk[t];
                    const bool better = k.mx != o.mx ? k.mx < o.mx
                                       : k.sum != o.sum ? k.sum < o.sum
                                       : k.c1 != o.c1 ? k.c1 < o.c1
                                                      : k.c0 < o.c0;
                    if (better) bk[t] = k;
                }
            for (int t = 0; t < m; ++t) {
                if (bk[t].mx == INT32_MAX) return "internal: class without a Toom tuple";
                // planes at points 0, 1, infinity: c0, c0 + c1, c1
                p.tables.push_back(al.code[bk[t].c0]);
                p.tables.push_back(al.code[bk[t].c0 + bk[t].c1]);
                p.tables.push_back(al.code[bk[t].c1]);
            }
        }
    }
    f.planes = plane;
    // the encode kernels hold every table in LDS
    if (p.tables.size() > 65536) return "channel tables exceed 64 KiB";
    return "";
}

}  // namespace ozemu
