// Reconstruct (Sec. V-A phase 5, Sec. V-D "Reconstruct"): for each output
// entry, the balanced CRT solution X of its residues, then one rounding of
// X 2^-(s_i + t_j) into FP64.
//
// CRT sum in digits whose sums stay exact. With INT8 moduli the residues
// z_l enter directly: S = sum_l z_l N_l with N_l = inv_l M_l (below P,
// inv_l = M_l^-1 mod m_l) is congruent to X modulo P and S / P = sum_l z_l
// inv_l / m_l exactly. With float-channel moduli u_l = (z_l inv_l) mod m_l
// comes first and S = sum_l u_l M_l. Either way one FP64 estimate q of the
// nearest integer to S / P gives X = S - q P, exact in the same digits. When
// the estimate is off by one (only possible when |X| is within a few ulps of
// P / 2), |X| exceeds (P - 1) / 2 and the exact fallback replaces |X| by
// P - |X| with the sign flipped. The magnitude is then rounded once, to
// nearest even, at the bit that lands on 2^-1074 or on the 53rd significant
// bit, whichever is higher, and scaled by an exact ldexp; overflow gives an
// infinity.
#include "ozemu_internal.hpp"

namespace ozemu {

namespace {

constexpr int kThreads = 256;
constexpr int kPerThread = 4;  // consecutive output columns per thread

// Finishes one entry from its digit sums acc = sum_l u_l M_l and the
// estimate f = sum_l u_l / m_l.
template <int D>
__device__ __forceinline__ double finish_one(const CrtConsts& cc, int64_t* acc, double f, int sc) {
    const int64_t q = (int64_t)rint(f);
#pragma unroll
    for (int d = 0; d < D; ++d) acc[d] -= q * (int64_t)cc.P[d];
    // carry-normalize into two's complement digits
    uint32_t x[D];
    int64_t carry = 0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const int64_t v = acc[d] + carry;
        x[d] = (uint32_t)v;
        carry = v >> 32;  // arithmetic shift
    }
    bool neg = carry < 0;
    if (neg) {  // magnitude = -X
        uint64_t c = 1;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const uint64_t v = (uint64_t)(~x[d]) + c;
            x[d] = (uint32_t)v;
            c = v >> 32;
        }
    }
    // exact fallback: |X| > (P - 1) / 2  =>  |X| <- P - |X|, sign flipped
    int cmp = 0;
#pragma unroll
    for (int d = D - 1; d >= 0; --d)
        if (cmp == 0 && x[d] != cc.half[d]) cmp = (x[d] > cc.half[d]) ? 1 : -1;
    if (cmp > 0) {
        int64_t b = 0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int64_t v = (int64_t)cc.P[d] - (int64_t)x[d] - b;
            b = v < 0;
            x[d] = (uint32_t)(v + (b ? (1ll << 32) : 0));
        }
        neg = !neg;
    }
    // bit length
    int L = 0;
#pragma unroll
    for (int d = 0; d < D; ++d)
        if (x[d] != 0) L = 32 * d + 32 - __clz(x[d]);
    if (L == 0) return 0.0;
    int rb = L - 53;
    if (sc - 1074 > rb) rb = sc - 1074;
    double r;
    if (rb <= 0) {
        const uint64_t t = (uint64_t)x[0] | ((uint64_t)x[1] << 32);  // L <= 53
        r = ldexp((double)t, -sc);
    } else {
        uint64_t t = 0;
        bool half = false, sticky = false;
        const int hb = rb - 1;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int off = 32 * d - rb;
            const uint64_t v = x[d];
            if (off >= 0 && off < 64)
                t |= v << off;
            else if (off < 0 && off > -32)
                t |= v >> (-off);
            const int lo = 32 * d;
            if (hb >= lo && hb < lo + 32) half = (x[d] >> (hb - lo)) & 1u;
            if (lo + 32 <= hb)
                sticky |= (x[d] != 0);
            else if (lo < hb)
                sticky |= (x[d] & ((1u << (hb - lo)) - 1u)) != 0;
        }
        if (half && (sticky || (t & 1))) t += 1;
        r = ldexp((double)t, rb - sc);
    }
    return neg ? -r : r;
}

// Finishes one entry from its CRT sum S = sum_l z_l N_l held as KC
// FP64 chunks s_k (S = sum_k s_k 2^(40 k), each s_k an integer below
// 2^53) with INT8 moduli. f = sum_k s_k 2^(40 k) / P is within 2^-34 of
// S / P and q = rint(f). When e = f - q is at least 2^-30 from 0 and from
// +-1/2 (nearly always), q is the nearest integer to S / P and X = S - q P
// has the sign of e: sg X is formed chunk by chunk (exact) and carried
// into 40-bit chunks in [0, 2^40), which give the 32-bit words of |X|.
// Otherwise X itself is formed, its last carry (-1 or 0) is the sign, the
// words are complemented when negative, and the exact fallback of
// finish_one applies. On the fast path the rounding is done in FP64 from
// the leading digits (below), except at an exact tie of the first 53 bits
// or for results below 2^-1021. The exact rounding position is
// rb = max(L - 53, sc - 1074)
// for the bit length L of |X|: the 64 bits of |X| from p = max(rb - 2, 0)
// up, the bits below p folded into the lowest (they are only a sticky
// bit), are rounded at rb to nearest even in integer arithmetic and scaled
// exactly.
template <int D, int KC, int CB>
__device__ __forceinline__ double finish_chunks(const CrtConsts& cc, const double* s, int sc) {
    // f is within 2^-34 of S / P for INT8 moduli (S / P < 2^13) and within
    // 2^-26 for float channels (S / P < 2^21); the fast path keeps clear of
    // that by a factor of 16 or more
    constexpr double kTau = CB == kChunkBits ? 0x1p-30 : 0x1p-20;
    constexpr double kUnit = (double)(1ull << CB), kInvUnit = 1.0 / kUnit;
    double f = 0.0;
#pragma unroll
    for (int k = 0; k < KC; ++k) f = __builtin_fma(s[k], cc.R40[k], f);
    const double q = rint(f);
    const double e = f - q;
    const bool fast = fabs(e) >= kTau && fabs(e) <= 0.5 - kTau;
    const double sg = (fast && e < 0.0) ? -1.0 : 1.0;
    const double qs = q * sg;
    double dg[KC];
    double carry = 0.0;
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        // |t| < 2^53: exact
        const double t = __builtin_fma(-qs, cc.P40[k], s[k] * sg) + carry;
        carry = floor(t * kInvUnit);
        dg[k] = __builtin_fma(-carry, kUnit, t);  // [0, 2^CB)
    }
    if (fast) {
        // |X| = sum_k dg_k 2^(CB k) >= 0 (nonzero: |X| > tau P). With j its
        // top nonzero digit, V = top 2^CB + nxt holds its leading 2 CB (if
        // dg_j >= 2^(53 - CB)) or 3 CB bits (else top = dg_j 2^CB + dg_j-1,
        // exact below 2^53), at unit 2^unit; V >= 2^53, so hi = RN(V) has
        // an ulp of at least 2 and its exact remainder e1 (Fast2Sum) is an
        // integer. Unless |e1| is exactly half an ulp, the digits below V
        // (worth less than one unit) cannot move the rounding: hi 2^unit
        // is |X| rounded to 53 bits, and scaling it is exact while the
        // result stays at or above 2^-1021 (the binade above the smallest
        // normal, so that no rounding at the subnormal spacing differs) or
        // overflows to infinity. Ties and tiny results take the exact path.
        double a = 0.0, b = 0.0, c = 0.0;
        int j = -1;
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            const bool nz = dg[k] != 0.0;
            j = nz ? k : j;
            a = nz ? dg[k] : a;
            b = nz ? (k >= 1 ? dg[k >= 1 ? k - 1 : 0] : 0.0) : b;
            c = nz ? (k >= 2 ? dg[k >= 2 ? k - 2 : 0] : 0.0) : c;
        }
        const bool low = a < (double)(1ull << (53 - CB));
        const double top = low ? __builtin_fma(a, kUnit, b) : a;
        const double nxt = low ? c : b;
        const int unit = CB * (low ? j - 2 : j - 1);
        const double big = top * kUnit;
        const double hi = big + nxt;
        const double e1 = nxt - (hi - big);
        const int eh = __builtin_amdgcn_frexp_exp(hi);  // hi = m 2^eh, m in [1/2, 1)
        const bool tie = fabs(e1) == ldexp(1.0, eh - 54);
        if (j >= 0 && !tie && eh + unit - sc >= -1020) {
            const double r = ldexp(hi, unit - sc);
            return sg < 0.0 ? -r : r;
        }
    }
    uint64_t ch[KC + 1];
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        const double hi = floor(dg[k] * 0x1p-32);
        const double lo = __builtin_fma(-hi, 0x1p32, dg[k]);
        ch[k] = ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
    }
    bool neg = carry < 0.0;  // false on the fast path
    ch[KC] = neg ? (1ull << CB) - 1ull : 0ull;  // sign extension of the chunk form
    // 32-bit words of sg X (two's complement over 32 D bits)
    uint32_t x[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const int k0 = (32 * j) / CB, o = 32 * j - CB * k0;
        uint64_t v = ch[k0] >> o;
        if (CB - o < 32) v |= ch[k0 + 1] << (CB - o);
        if (CB - o + CB < 32) v |= ch[k0 + 2] << (CB - o + CB);
        x[j] = (uint32_t)v;
    }
    if (fast) {
        neg = sg < 0.0;
    } else {
        // |X|: complement and add one when negative
        const uint32_t m = neg ? 0xFFFFFFFFu : 0u;
        uint64_t c = neg ? 1u : 0u;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const uint64_t v = (uint64_t)(x[j] ^ m) + c;
            x[j] = (uint32_t)v;
            c = v >> 32;
        }
        // fallback: |X| > (P - 1) / 2  =>  |X| <- P - |X|, sign flipped
        int64_t b = 0;  // borrow of half - |X|
#pragma unroll
        for (int j = 0; j < D; ++j) b = ((int64_t)cc.half[j] - (int64_t)x[j] + b) >> 32;
        const bool over = b < 0;
        int64_t br = 0;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const int64_t v = (int64_t)cc.P[j] - (int64_t)x[j] + br;
            x[j] = over ? (uint32_t)v : x[j];
            br = v >> 32;
        }
        neg = neg != over;
    }
    int L = 0;
#pragma unroll
    for (int j = 0; j < D; ++j) L = x[j] ? 32 * j + 32 - (int)__clz(x[j]) : L;
    const int rb = max(L - 53, sc - 1074);
    const int p = max(rb - 2, 0);
    const int g = rb - p;  // bits to round off: 0, 1 or 2 (none when rb <= 0)
    const int dw = p >> 5, sh = p & 31;
    uint32_t a = 0, b = 0, c = 0, below = 0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const bool at = j == dw;
        a = at ? x[j] : a;
        b = at ? (j + 1 < D ? x[j + 1] : 0u) : b;
        c = at ? (j + 2 < D ? x[j + 2] : 0u) : c;
        below |= (j < dw) ? x[j] : 0u;
    }
    const uint32_t sticky = (below | (a & ((1u << sh) - 1u))) != 0u;
    const uint32_t lo = __builtin_amdgcn_alignbit(b, a, sh) | sticky;
    const uint32_t hi = __builtin_amdgcn_alignbit(c, b, sh);
    const uint64_t w = ((uint64_t)hi << 32) | lo;
    uint64_t t = w >> (g > 0 ? g : 0);
    if (g > 0) {
        const uint64_t rem = w & ((1ull << g) - 1ull), half = 1ull << (g - 1);
        t += (rem > half || (rem == half && (t & 1ull))) ? 1ull : 0ull;
    }
    const double r = ldexp((double)t, (rb > 0 ? rb : 0) - sc);  // t <= 2^53: exact
    return neg ? -r : r;
}

// Thread g of the output: row g / ceil(n / 4), four consecutive columns.
// Residues are uint8 (INT8 moduli) or uint16 (float-channel moduli).
template <int D, typename R = uint8_t>
__device__ __forceinline__ void reconstruct_body(const CrtConsts& cc, int64_t m, int64_t n,
                                                 int64_t m_pad, int64_t n_pad,
                                                 const R* __restrict__ Z,
                                                 const int32_t* __restrict__ sa,
                                                 const int32_t* __restrict__ sb,
                                                 double* __restrict__ C, int64_t ldc, int64_t g) {
    const int64_t per_row = (n + kPerThread - 1) / kPerThread;
    if (g >= m * per_row) return;
    const int64_t i = g / per_row;
    const int64_t j0 = (g % per_row) * kPerThread;
    const int64_t plane = m_pad * n_pad;
    // shifts first (clamped indices, unconditional loads), so that their
    // latency hides behind the residue loop
    const int32_t si = sa[i];
    int32_t tj[kPerThread];
#pragma unroll
    for (int c = 0; c < kPerThread; ++c) tj[c] = sb[(j0 + c < n) ? j0 + c : n - 1];
    const R* zp = Z + i * n_pad + j0;
    double out[kPerThread];
    if constexpr (sizeof(R) == 1) {
        // INT8 moduli: S = sum_l z_l N_l with N_l = inv_l M_l, congruent to
        // the CRT sum modulo P, so no per-residue reduction is needed. S is
        // summed in 40-bit chunks, each exactly in FP64: a product z_l
        // N_l,k is below 2^48 and a chunk's sum over at most 32 moduli below
        // 2^53. The residues of up to kBatch moduli are loaded before any is
        // used, so that each wave keeps that many loads in flight (loads
        // past the last modulus re-read the last plane and count as zeros).
        constexpr int KC = (32 * D + kChunkBits - 1) / kChunkBits;
        constexpr int kBatch = 16;
        double sk[kPerThread][KC];
#pragma unroll
        for (int c = 0; c < kPerThread; ++c)
#pragma unroll
            for (int k = 0; k < KC; ++k) sk[c][k] = 0.0;
        for (int l0 = 0; l0 < cc.n; l0 += kBatch) {
            uint32_t word[kBatch];
#pragma unroll
            for (int b = 0; b < kBatch; ++b) {
                const int l = (l0 + b < cc.n) ? l0 + b : cc.n - 1;
                word[b] = __builtin_nontemporal_load(
                    reinterpret_cast<const uint32_t*>(zp + (int64_t)l * plane));
            }
#pragma unroll
            for (int b = 0; b < kBatch; ++b) {
                const bool live = l0 + b < cc.n;
                const int l = live ? l0 + b : cc.n - 1;
                const uint32_t wb = live ? word[b] : 0u;
#pragma unroll
                for (int c = 0; c < kPerThread; ++c) {
                    const double z = (double)((wb >> (8 * c)) & 0xFFu);
#pragma unroll
                    for (int k = 0; k < KC; ++k) sk[c][k] = __builtin_fma(z, cc.N40[l][k], sk[c][k]);
                }
            }
        }
#pragma unroll
        for (int c = 0; c < kPerThread; ++c) {
            out[c] = 0.0;
            if (j0 + c >= n) continue;
            if (si == kShiftNonFinite || tj[c] == kShiftNonFinite)
                out[c] = __builtin_nan("");
            else
                out[c] = finish_chunks<D, KC, kChunkBits>(cc, sk[c], si + tj[c]);
        }
    } else {
        constexpr int KC = (32 * D + kChunkBitsFp - 1) / kChunkBitsFp;
        bool done = false;
        if constexpr (KC <= kMaxChunks) {
            if (cc.kc > 0) {
                // float-channel moduli (below 2^16): S = sum_l z_l N_l in
                // 30-bit chunks, exact in FP64 (a product is below 2^46, a
                // chunk's sum over at most 32 channels below 2^51); loads as
                // in the INT8 form
                constexpr int kBatch = 16;
                double sk[kPerThread][KC];
#pragma unroll
                for (int c = 0; c < kPerThread; ++c)
#pragma unroll
                    for (int k = 0; k < KC; ++k) sk[c][k] = 0.0;
                for (int l0 = 0; l0 < cc.n; l0 += kBatch) {
                    uint2 word[kBatch];
#pragma unroll
                    for (int b = 0; b < kBatch; ++b) {
                        const int l = (l0 + b < cc.n) ? l0 + b : cc.n - 1;
                        word[b] = *reinterpret_cast<const uint2*>(zp + (int64_t)l * plane);
                    }
#pragma unroll
                    for (int b = 0; b < kBatch; ++b) {
                        const bool live = l0 + b < cc.n;
                        const int l = live ? l0 + b : cc.n - 1;
                        const uint32_t w0 = live ? word[b].x : 0u, w1 = live ? word[b].y : 0u;
                        const double z[kPerThread] = {(double)(w0 & 0xFFFFu), (double)(w0 >> 16),
                                                      (double)(w1 & 0xFFFFu), (double)(w1 >> 16)};
#pragma unroll
                        for (int c = 0; c < kPerThread; ++c)
#pragma unroll
                            for (int k = 0; k < KC; ++k)
                                sk[c][k] = __builtin_fma(z[c], cc.N40[l][k], sk[c][k]);
                    }
                }
#pragma unroll
                for (int c = 0; c < kPerThread; ++c) {
                    out[c] = 0.0;
                    if (j0 + c >= n) continue;
                    if (si == kShiftNonFinite || tj[c] == kShiftNonFinite)
                        out[c] = __builtin_nan("");
                    else
                        out[c] = finish_chunks<D, KC, kChunkBitsFp>(cc, sk[c], si + tj[c]);
                }
                done = true;
            }
        }
        if (!done) {
            // too many chunks: u_l = (z_l inv_l) mod m_l and S = sum_l u_l M_l
            // in 32-bit digits, each term below 2^48
            int64_t acc[kPerThread][D];
            double f[kPerThread];
#pragma unroll
            for (int c = 0; c < kPerThread; ++c) f[c] = 0.0;
#pragma unroll
            for (int c = 0; c < kPerThread; ++c)
#pragma unroll
                for (int d = 0; d < D; ++d) acc[c][d] = 0;
            for (int l = 0; l < cc.n; ++l) {
                uint32_t zv[kPerThread];
                const uint2 w2 = *reinterpret_cast<const uint2*>(zp + (int64_t)l * plane);
                zv[0] = w2.x & 0xFFFFu;
                zv[1] = w2.x >> 16;
                zv[2] = w2.y & 0xFFFFu;
                zv[3] = w2.y >> 16;
                const uint32_t ml = cc.m[l], mu = cc.mu[l], inv = cc.inv[l];
                const double rcp = cc.rcp[l];
#pragma unroll
                for (int c = 0; c < kPerThread; ++c) {
                    const uint64_t u = barrett32(zv[c] * inv, ml, mu);
                    f[c] += (double)u * rcp;
#pragma unroll
                    for (int d = 0; d < D; ++d) acc[c][d] += (int64_t)(u * cc.Ml[l][d]);
                }
            }
#pragma unroll
            for (int c = 0; c < kPerThread; ++c) {
                out[c] = 0.0;
                if (j0 + c >= n) continue;
                if (si == kShiftNonFinite || tj[c] == kShiftNonFinite)
                    out[c] = __builtin_nan("");
                else
                    out[c] = finish_one<D>(cc, acc[c], f[c], si + tj[c]);
            }
        }
    }
    double* crow = C + i * ldc + j0;
    if (j0 + kPerThread <= n && ((reinterpret_cast<uintptr_t>(crow) & 15) == 0)) {
        reinterpret_cast<double2*>(crow)[0] = make_double2(out[0], out[1]);
        reinterpret_cast<double2*>(crow)[1] = make_double2(out[2], out[3]);
    } else {
        for (int c = 0; c < kPerThread; ++c)
            if (j0 + c < n) crow[c] = out[c];
    }
}

// Five waves per SIMD (at most 96 VGPRs) where that needs no spills: more
// residue loads in flight per CU, about 2% faster at 16 moduli.
template <int D, typename R>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(
    (sizeof(R) == 1 ? D <= 8 : D <= 7) ? 5 : 1))) void reconstruct_kernel(CrtConsts cc, int64_t m, int64_t n,
                                                               int64_t m_pad, int64_t n_pad,
                                                               const R* __restrict__ Z,
                                                               const int32_t* __restrict__ sa,
                                                               const int32_t* __restrict__ sb,
                                                               double* __restrict__ C, int64_t ldc) {
    reconstruct_body<D, R>(cc, m, n, m_pad, n_pad, Z, sa, sb, C, ldc,
                        (int64_t)blockIdx.x * kThreads + threadIdx.x);
}

__global__ void zero_c_kernel(int64_t m, int64_t n, double* C, int64_t ldc) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= m * n) return;
    C[(g / n) * ldc + g % n] = 0.0;
}

// Grouped Reconstruct; a problem with k = 0 gets zeros.
template <int D>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(D <= 8 ? 5 : 1)))
void group_reconstruct_kernel(GroupArgs g) {
    const int32_t* pre = g.prefix + kGCrt * (g.count + 1);
    const int p = group_find(pre, g.count, blockIdx.x);
    const GProblem& P = g.probs[p];
    const int64_t t = (int64_t)(blockIdx.x - pre[p]) * kThreads + threadIdx.x;
    if (P.k == 0) {
        const int64_t per_row = (P.n + kPerThread - 1) / kPerThread;
        if (t >= P.m * per_row) return;
        const int64_t i = t / per_row, j0 = (t % per_row) * kPerThread;
        for (int c = 0; c < kPerThread; ++c)
            if (j0 + c < P.n) P.C[i * P.ldc + j0 + c] = 0.0;
        return;
    }
    reconstruct_body<D>(g.crts[P.plan], P.m, P.n, P.m_pad, P.n_pad,
                        reinterpret_cast<const uint8_t*>(g.ws + P.off_z),
                        reinterpret_cast<const int32_t*>(g.ws + P.off_sa),
                        reinterpret_cast<const int32_t*>(g.ws + P.off_sb), P.C, P.ldc, t);
}

template <int D>
hipError_t launch_group_d(hipStream_t st, const GroupArgs& g, int32_t blocks) {
    group_reconstruct_kernel<D><<<dim3((unsigned)blocks), dim3(kThreads), 0, st>>>(g);
    return hipGetLastError();
}

template <int D, typename R>
hipError_t launch_d(hipStream_t st, const CrtConsts& cc, int64_t m, int64_t n, int64_t m_pad,
                    int64_t n_pad, const R* Z, const int32_t* sa, const int32_t* sb,
                    double* C, int64_t ldc) {
    const int64_t threads = m * ((n + kPerThread - 1) / kPerThread);
    const int64_t blocks = (threads + kThreads - 1) / kThreads;
    reconstruct_kernel<D, R><<<dim3((unsigned)blocks), dim3(kThreads), 0, st>>>(
        cc, m, n, m_pad, n_pad, Z, sa, sb, C, ldc);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_any(hipStream_t st, const CrtConsts& cc, int64_t m, int64_t n, int64_t m_pad,
                      int64_t n_pad, const R* Z, const int32_t* sa, const int32_t* sb, double* C,
                      int64_t ldc) {
    if (m <= 0 || n <= 0) return hipSuccess;
    switch (cc.d) {
        case 2: return launch_d<2, R>(st, cc, m, n, m_pad, n_pad, Z, sa, sb, C, ldc);
        case 3: return launch_d<3, R>(st, cc, m, n, m_pad, n_pad, Z, sa, sb, C, ldc);
        case 4: return launch_d<4, R>(st, cc, m, n, m_pad, n_pad, Z, sa, sb, C, ldc);
        case 5: return launch_d<5, R>(st, cc, m, n, m_pad, n_pad, Z, sa, sb, C, ldc);
        case 6: return launch_d<6, R>(st, cc, m, n, m_pad, n_pad, Z, sa, sb, C, ldc);
        case 7: return launch_d<7, R>(st, cc, m, n, m_pad, n_pad, Z, sa, sb, C, ldc);
        case 8: return launch_d<8, R>(st, cc, m, n, m_pad, n_pad, Z, sa, sb, C, ldc);
        case 9: return launch_d<9, R>(st, cc, m, n, m_pad, n_pad, Z, sa, sb, C, ldc);
        case 10: return launch_d<10, R>(st, cc, m, n, m_pad, n_pad, Z, sa, sb, C, ldc);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_reconstruct(hipStream_t st, const CrtConsts& cc, int64_t m, int64_t n,
                              int64_t m_pad, int64_t n_pad, const uint8_t* residues,
                              const int32_t* shift_a, const int32_t* shift_b, double* C,
                              int64_t ldc) {
    return launch_any<uint8_t>(st, cc, m, n, m_pad, n_pad, residues, shift_a, shift_b, C, ldc);
}

hipError_t launch_reconstruct16(hipStream_t st, const CrtConsts& cc, int64_t m, int64_t n,
                                int64_t m_pad, int64_t n_pad, const uint16_t* residues,
                                const int32_t* shift_a, const int32_t* shift_b, double* C,
                                int64_t ldc) {
    return launch_any<uint16_t>(st, cc, m, n, m_pad, n_pad, residues, shift_a, shift_b, C, ldc);
}

hipError_t launch_group_reconstruct(hipStream_t st, const GroupArgs& g, int32_t blocks, int dmax) {
    if (blocks <= 0) return hipSuccess;
    switch (dmax) {
        case 2: return launch_group_d<2>(st, g, blocks);
        case 3: return launch_group_d<3>(st, g, blocks);
        case 4: return launch_group_d<4>(st, g, blocks);
        case 5: return launch_group_d<5>(st, g, blocks);
        case 6: return launch_group_d<6>(st, g, blocks);
        case 7: return launch_group_d<7>(st, g, blocks);
        case 8: return launch_group_d<8>(st, g, blocks);
        case 9: return launch_group_d<9>(st, g, blocks);
        case 10: return launch_group_d<10>(st, g, blocks);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_zero_c(hipStream_t st, int64_t m, int64_t n, double* C, int64_t ldc) {
    if (m <= 0 || n <= 0) return hipSuccess;
    const int64_t total = m * n;
    zero_c_kernel<<<dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st>>>(m, n, C, ldc);
    return hipGetLastError();
}

}  // namespace ozemu
