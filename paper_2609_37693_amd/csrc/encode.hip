// Reduce phase (Sec. V-A phase 2, Sec. V-D "Reduce"): applies Scale's shifts,
// truncates each entry (eq. "convert") without storing A' or B', and writes
// its balanced residue modulo every modulus of the plan as int8 (two's
// complement) into the residue planes. Each FP64 entry is read once; all
// moduli are produced from registers.
//
// Planes of A hold row i of A' K-contiguously and planes of B column j of B'
// (a transpose, done through LDS), both in the blocked GEMM order of
// plane_offset, so the GEMM reads each K step of a tile as one block.
//
// Three forms of an entry, by the plan's kept bits: at most 62, A' as eight
// signed base-256 digits and two byte dot products per modulus; above 62
// (the exact form), twelve signed digits and three dot products while every
// entry of the workgroup is below 2^94, else the bytes of the significand
// and a factor 2^s mod m from an LDS table.
#include "ozemu_internal.hpp"

namespace ozemu {

namespace {

constexpr int kEncThreads = 256;
constexpr int kEncVec = 16;   // consecutive k entries per thread (one 16-byte store per modulus)
constexpr int kMaxShift = 80; // largest left shift of a significand: kBetaCap - 53 < 80

// |A'| of one entry: the significand scaled by 2^(exponent + shift),
// truncated toward zero (eq. "convert"), with its sign. Branch-free: every
// lane of a wave takes the same instructions whatever its entry's class.
// With kBig false the kept bits are at most 63 and |A'| = mant 2^sh (or
// mant >> -sh) fits in 64 bits, stored as two 32-bit words. With kBig true
// only mant >> max(-sh, 0) is stored and a positive sh is applied per
// modulus as a factor 2^sh mod m. Non-finite entries and the marker shift
// give zero.
struct Entry {
    uint32_t lo, hi;
    int sh;    // > 0 only in the kBig form
    bool neg;
};

template <bool kBig>
__device__ __forceinline__ Entry make_entry(double x, int32_t shift) {
    Entry e;
    const uint64_t bits = (uint64_t)__double_as_longlong(x);
    const uint64_t a = bits & 0x7FFFFFFFFFFFFFFFull;
    const bool keep = a < 0x7FF0000000000000ull && shift != kShiftNonFinite;
    const uint32_t be = (uint32_t)(a >> 52);
    const uint64_t mant = keep ? ((a & 0x000FFFFFFFFFFFFFull) | ((uint64_t)(be != 0) << 52)) : 0;
    // exponent of the significand's unit: be - 1075, or -1074 for subnormals
    const int sh = keep ? (int)(be > 1u ? be : 1u) - 1075 + shift : 0;
    const int down = sh < 0 ? (-sh < 63 ? -sh : 63) : 0;  // mant < 2^53: >> 63 gives 0
    uint64_t v = mant >> down;
    if (!kBig) v = sh > 0 ? mant << sh : v;  // sh <= 10 here: below 2^63
    e.lo = (uint32_t)v;
    e.hi = (uint32_t)(v >> 32);
    e.sh = (kBig && sh > 0) ? sh : 0;
    e.neg = (bits >> 63) != 0;
    return e;
}

// An entry in the form the INT8 residues use. With kBig false (at most 62
// kept bits, |A'| < 2^62): A' as eight signed base-256 digits d_i in
// [-128, 127], A' = sum_i d_i 2^(8 i): the bytes of A' + 0x8080...80 (two's
// complement, no wrap since |A'| < 2^62) with their top bits flipped. With
// kBig true: the bytes of |A'| (of 2^64 - |A'| when A' < 0) and a mask that
// adds (-2^64) mod m per modulus for negative entries; sh > 0 is applied per
// modulus.
struct Entry8 {
    uint32_t lo, hi;
    uint32_t negm;  // kBig: all ones if A' < 0
    int sh;
};

template <bool kBig>
__device__ __forceinline__ Entry8 make_entry8(double x, int32_t shift) {
    const Entry e = make_entry<kBig>(x, shift);
    const uint64_t v = ((uint64_t)e.hi << 32) | e.lo;
    const bool neg = e.neg && v != 0;
    const uint64_t w = neg ? (uint64_t)0 - v : v;
    Entry8 r;
    r.sh = e.sh;
    if constexpr (kBig) {
        r.lo = (uint32_t)w;
        r.hi = (uint32_t)(w >> 32);
        r.negm = neg ? 0xFFFFFFFFu : 0u;
    } else {
        const uint64_t y = w + 0x8080808080808080ull;
        r.lo = (uint32_t)y ^ 0x80808080u;
        r.hi = (uint32_t)(y >> 32) ^ 0x80808080u;
        r.negm = 0u;
    }
    return r;
}

// Balanced residue t - m floor(t/m + 1/2), in [-floor(m/2), ceil(m/2) - 1],
// of t < 2^19, returned in the low byte of the result (two's complement;
// the upper bytes are not part of the value). With rcp_up strictly above
// 1/m (by at most one FP32 ulp), t rcp_up exceeds t/m by less than
// 2^19 2^-23 / m = 1/(16 m), while t/m lies at least 1/(2m) from every
// half-integer it is not equal to, and above t/m a tie t/m = k + 1/2 moves
// up: fma(t, rcp_up, 1.5 2^23), rounded once to the unit grid of
// [2^23, 2^24), is 1.5 2^23 + q with q = floor(t/m + 1/2). Its low 24 bits
// are 2^22 + q (bit 23 is the exponent's low bit, 0), so one 24-bit
// multiply-add gives t - q m - 2^22 m, whose low byte is that of t - q m
// (2^22 m is a multiple of 256). Checked on the CPU for every m <= 256 and
// every t < 2^19.
__device__ __forceinline__ int32_t balanced19(uint32_t t, uint32_t m, float rcp_up) {
    const float x = __builtin_fmaf((float)t, rcp_up, 12582912.0f);
    return (int32_t)t + __mul24(__builtin_bit_cast(int32_t, x), -(int32_t)m);
}

// Balanced residue of the entry modulo m_l, in the low byte of the int32; p2
// is the LDS table of 2^s mod m_l (kBig only). kBig false: two signed byte
// dot products with the balanced weights 2^(8 i) mod m (|sum| <= 8 128 127
// < 2^17) on top of km = a multiple of m in [2^17, 2^17 + m), so t lies in
// [0, 2^19). kBig true: two unsigned byte dot products sum at most
// 8 255 255 + 255 < 2^19.
template <bool kBig>
__device__ __forceinline__ int32_t entry_residue(const Entry8& e, const ModConsts& mc, int l,
                                                 const uint8_t* p2) {
    const uint32_t m = mc.m[l];
    uint32_t t;
    if constexpr (kBig) {
        t = __builtin_amdgcn_udot4(e.lo, mc.w8[l][0], e.negm & mc.c64n[l], false);
        t = __builtin_amdgcn_udot4(e.hi, mc.w8[l][1], t, false);
        if (e.sh > 0) t = mod24(t, m, mc.rcp[l]) * p2[e.sh];  // below 2^16
    } else {
        // weights in VGPRs (copied once per modulus) and km as the scalar
        // addend of a three-operand dot product: no per-entry copy of km
        int32_t w0, w1, u;
        asm("v_mov_b32 %0, %1" : "=v"(w0) : "s"(mc.s8[l][0]));
        asm("v_mov_b32 %0, %1" : "=v"(w1) : "s"(mc.s8[l][1]));
        asm("v_dot4_i32_i8 %0, %1, %2, %3" : "=v"(u) : "v"(e.lo), "v"(w0), "s"(mc.km[l]));
        u = __builtin_amdgcn_sdot4((int32_t)e.hi, w1, u, false);
        t = (uint32_t)u;
    }
    return balanced19(t, m, mc.rcp_up[l]);
}

// Low bytes of four values, a in byte 0.
__device__ __forceinline__ uint32_t pack4(int32_t a, int32_t b, int32_t c, int32_t d) {
    const uint32_t ab = __builtin_amdgcn_perm((uint32_t)b, (uint32_t)a, 0x0c0c0400u);
    const uint32_t cd = __builtin_amdgcn_perm((uint32_t)d, (uint32_t)c, 0x0c0c0400u);
    return __builtin_amdgcn_perm(cd, ab, 0x05040100u);
}

// Sixteen residues of one modulus as one 16-byte word, entry q in byte q.
template <bool kBig>
__device__ __forceinline__ uint4 residues16(const Entry8* ent, const ModConsts& mc, int l,
                                            const uint8_t* p2) {
    int32_t r[kEncVec];
#pragma unroll
    for (int q = 0; q < kEncVec; ++q) r[q] = entry_residue<kBig>(ent[q], mc, l, p2);
    return make_uint4(pack4(r[0], r[1], r[2], r[3]), pack4(r[4], r[5], r[6], r[7]),
                      pack4(r[8], r[9], r[10], r[11]), pack4(r[12], r[13], r[14], r[15]));
}

// The exact form's entries when every |A'| of a wave is below 2^94
// (positive shift at most kMidShift): A' as twelve signed base-256 digits
// (the bytes of A' + 0x80...80 over 96 bits, top bits flipped), written over
// the entry's own registers (lo, hi, negm = digit words 0, 1, 2), and per
// modulus three signed byte dot products with the balanced weights
// 2^(8 i) mod m (bytes 8..11 from MidConsts) on top of 2 km, a multiple of m
// in [2^18, 2^18 + 2m): |sum| <= 12 128 128 < 2^18 keeps t in [0, 2^19).
// No shift table and no per-modulus multiply.
constexpr int kMidShift = 41;  // |A'| = mant 2^sh < 2^53 2^41

struct MidConsts {
    int32_t s8c[kMaxModuli];  // balanced 2^(64 + 8 i) mod m_l, i = 0..3, as signed bytes
    int on;                   // 0: the exact form only
};

__device__ __forceinline__ bool mid_fits(const Entry8& e) { return e.sh <= kMidShift; }

__device__ __forceinline__ void to_mid(Entry8& e) {
    const bool neg = e.negm != 0u;
    const uint64_t w = ((uint64_t)e.hi << 32) | e.lo;
    const uint64_t v = neg ? (uint64_t)0 - w : w;  // |A'| 2^-sh, below 2^53
    const int sh = e.sh;                           // 0 .. kMidShift
    const uint64_t lo = v << sh;
    const uint32_t hi = sh > 0 ? (uint32_t)(v >> (64 - sh)) : 0u;
    const uint64_t nlo = neg ? (uint64_t)0 - lo : lo;  // two's complement over 96 bits
    const uint32_t nhi = neg ? ~hi + (lo == 0 ? 1u : 0u) : hi;
    const uint64_t y0 = nlo + 0x8080808080808080ull;
    const uint32_t y1 = nhi + 0x80808080u + (y0 < nlo ? 1u : 0u);
    e.lo = (uint32_t)y0 ^ 0x80808080u;
    e.hi = (uint32_t)(y0 >> 32) ^ 0x80808080u;
    e.negm = y1 ^ 0x80808080u;
    e.sh = 0;
}

__device__ __forceinline__ int32_t mid_residue(const Entry8& e, const ModConsts& mc,
                                               const MidConsts& md, int l) {
    int32_t w0, w1, w2, u;
    asm("v_mov_b32 %0, %1" : "=v"(w0) : "s"(mc.s8[l][0]));
    asm("v_mov_b32 %0, %1" : "=v"(w1) : "s"(mc.s8[l][1]));
    asm("v_mov_b32 %0, %1" : "=v"(w2) : "s"(md.s8c[l]));
    asm("v_dot4_i32_i8 %0, %1, %2, %3" : "=v"(u) : "v"(e.lo), "v"(w0), "s"(2u * mc.km[l]));
    u = __builtin_amdgcn_sdot4((int32_t)e.hi, w1, u, false);
    u = __builtin_amdgcn_sdot4((int32_t)e.negm, w2, u, false);
    return balanced19((uint32_t)u, mc.m[l], mc.rcp_up[l]);
}

__device__ __forceinline__ uint4 mid_residues16(const Entry8* ent, const ModConsts& mc,
                                                const MidConsts& md, int l) {
    int32_t r[kEncVec];
#pragma unroll
    for (int q = 0; q < kEncVec; ++q) r[q] = mid_residue(ent[q], mc, md, l);
    return make_uint4(pack4(r[0], r[1], r[2], r[3]), pack4(r[4], r[5], r[6], r[7]),
                      pack4(r[8], r[9], r[10], r[11]), pack4(r[12], r[13], r[14], r[15]));
}

// True in every thread of the workgroup when every entry of the workgroup
// fits the 96-bit form (kBig kernels given the constants). A block-wide
// vote: every thread of the workgroup must call it.
template <bool kBig>
__device__ __forceinline__ bool block_mid(const Entry8* ent, const MidConsts* md) {
    if constexpr (!kBig) {
        return false;
    } else {
        if (md == nullptr || !md->on) return false;
        bool fits = true;
#pragma unroll
        for (int q = 0; q < kEncVec; ++q) fits = fits && mid_fits(ent[q]);
        return __syncthreads_and(fits) != 0;
    }
}

// Shift of an entry whose row (or column) shift is s and whose inner index
// carries the fold f: s - f, the marker if either is the marker.
template <bool kFold>
__device__ __forceinline__ int32_t entry_shift(int32_t s, const int32_t* fold, int64_t h) {
    if constexpr (!kFold) {
        return s;
    } else {
        const int32_t f = fold[h];
        return (s == kShiftNonFinite || f == kShiftNonFinite) ? kShiftNonFinite : s - f;
    }
}

// Table of 2^s mod m_l for s < kMaxShift in LDS (kBig only).
template <bool kBig>
__device__ __forceinline__ void fill_p2(const ModConsts& mc, uint8_t* p2) {
    if constexpr (kBig) {
        for (int e = threadIdx.x; e < mc.n * kMaxShift; e += kEncThreads) {
            const int l = e / kMaxShift, sft = e % kMaxShift;
            p2[e] = (uint8_t)pow2mod(sft, mc.m[l], mc.mu[l]);
        }
        __syncthreads();
    }
}

// encode_a works on 16-entry chunks of the plane's rows, k_pad / 16 per
// row, 256 consecutive chunks per workgroup (crossing rows when k_pad is
// short), so every thread has work for any K.
constexpr int64_t kChunksPerBlock = kEncThreads;
static_assert(kChunksPerBlock == 256 && kEncVec == 16 && kPlaneK == 64, "encode_a tile map");

// Chunk c of the A planes (16 entries of a row): groups of 256 chunks (one
// workgroup) cover tiles of 64 rows x 64 columns, k_pad / 64 tiles per band
// of 64 rows; chunk t of a group is row t / 4 of its tile, columns
// 16 (t % 4) .. + 15. A 64-row slice of a plane block is 4 KB in one piece
// (plane_offset), so each modulus' stores of a workgroup fill one
// contiguous 4 KB region. Padding rows and columns get zeros without
// residue work. p2: LDS table (kBig only).
template <bool kBig, bool kFold>
__device__ __forceinline__ void encode_a_body(const ModConsts& mc, int64_t m, int64_t k,
                                              const double* A, int64_t lda,
                                              const int32_t* shift_a, const int32_t* fold,
                                              int64_t m_pad, int64_t k_pad, int8_t* planes,
                                              int64_t c, uint8_t* p2,
                                              const MidConsts* md = nullptr) {
    const int64_t tiles_k = k_pad / kPlaneK;
    const int64_t tile = c >> 8;
    const int t = (int)(c & 255);
    const int64_t i = (tile / tiles_k) * 64 + (t >> 2);
    const int64_t h = (tile % tiles_k) * kPlaneK + (t & 3) * kEncVec;
    const bool live = i < m && h < k;
    Entry8 ent[kEncVec];
    if (live) {
        const int32_t s = shift_a[i];
        const double* row = A + i * lda;
        if (h + kEncVec <= k && ((reinterpret_cast<uintptr_t>(row + h) & 15) == 0)) {
            const double2* p2v = reinterpret_cast<const double2*>(row + h);
#pragma unroll
            for (int q = 0; q < kEncVec / 2; ++q) {
                double2 v = p2v[q];
                ent[2 * q] = make_entry8<kBig>(v.x, entry_shift<kFold>(s, fold, h + 2 * q));
                ent[2 * q + 1] =
                    make_entry8<kBig>(v.y, entry_shift<kFold>(s, fold, h + 2 * q + 1));
            }
        } else {
#pragma unroll
            for (int q = 0; q < kEncVec; ++q) {
                const bool in = h + q < k;
                double v = in ? row[h + q] : 0.0;
                ent[q] = make_entry8<kBig>(v, in ? entry_shift<kFold>(s, fold, h + q) : 0);
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < kEncVec; ++q) ent[q] = Entry8{0u, 0u, 0u, 0};
    }
    // every thread votes before any leaves: the 96-bit form for the whole
    // workgroup, else the shift table
    const bool use_mid = block_mid<kBig>(ent, md);
    if (!use_mid) fill_p2<kBig>(mc, p2);
    if (i >= m_pad) return;
    const int64_t plane_stride = m_pad * k_pad;
    int8_t* out = planes + plane_offset(i, h, k_pad);
    if (!live) {
        for (int l = 0; l < mc.n; ++l)
            *reinterpret_cast<uint4*>(out + (int64_t)l * plane_stride) = make_uint4(0, 0, 0, 0);
        return;
    }
    if (use_mid) {
#pragma unroll
        for (int q = 0; q < kEncVec; ++q) to_mid(ent[q]);
        for (int l = 0; l < mc.n; ++l)
            *reinterpret_cast<uint4*>(out + (int64_t)l * plane_stride) =
                mid_residues16(ent, mc, *md, l);
        return;
    }
    for (int l = 0; l < mc.n; ++l)
        *reinterpret_cast<uint4*>(out + (int64_t)l * plane_stride) =
            residues16<kBig>(ent, mc, l, p2 + l * kMaxShift);
}

// grid: ceil(m_pad * k_pad / 16 / 256).
template <bool kBig, bool kFold>
__global__ __launch_bounds__(kEncThreads) void encode_a_kernel(ModConsts mc, int64_t m, int64_t k,
                                                               const double* A, int64_t lda,
                                                               const int32_t* shift_a,
                                                               const int32_t* fold,
                                                               int64_t m_pad, int64_t k_pad,
                                                               int8_t* planes, MidConsts md) {
    __shared__ uint8_t p2[kBig ? kMaxModuli * kMaxShift : 1];
    encode_a_body<kBig, kFold>(mc, m, k, A, lda, shift_a, fold, m_pad, k_pad, planes,
                               (int64_t)blockIdx.x * kChunksPerBlock + threadIdx.x, p2, &md);
}

// Workgroup (bx, by) of encode_b: a 64 (k) x 64 (n) tile of B. Thread t
// reads column j = t % 64 at rows 16 * (t / 64) .. + 15 (coalesced along j),
// builds the 16 residues of that column segment per modulus, stores them as
// one 16-byte word into LDS row j, and the tile is written out row by row
// (64 K-contiguous bytes per column of B).
constexpr int kTB = 64;
constexpr int kLdsRow = kTB + 16;  // bytes; padding spreads rows over banks

template <bool kBig, bool kFold>
__device__ __forceinline__ void encode_b_body(const ModConsts& mc, int64_t k, int64_t n,
                                              const double* B, int64_t ldb,
                                              const int32_t* shift_b, const int32_t* fold,
                                              int64_t n_pad, int64_t k_pad, int8_t* planes,
                                              int64_t bx, int64_t by, int8_t* tile, uint8_t* p2,
                                              const MidConsts* md = nullptr) {
    const int64_t j0 = bx * kTB;
    const int64_t h0 = by * kTB;
    const int64_t plane_stride = n_pad * k_pad;
    const int orow = threadIdx.x >> 2;    // output column of B (row of the plane)
    const int ochunk = threadIdx.x & 3;   // 16-byte chunk of K
    if (j0 >= n || h0 >= k) {  // a tile of padding: zeros, no residue work
        for (int l = 0; l < mc.n; ++l)
            *reinterpret_cast<uint4*>(planes + (int64_t)l * plane_stride +
                                      plane_offset(j0 + orow, h0 + ochunk * kEncVec, k_pad)) =
                make_uint4(0, 0, 0, 0);
        return;
    }
    const int tj = threadIdx.x & 63;
    const int hq = threadIdx.x >> 6;  // 0..3
    const int64_t j = j0 + tj;
    const int32_t s = (j < n) ? shift_b[j] : 0;
    Entry8 ent[kEncVec];
#pragma unroll
    for (int q = 0; q < kEncVec; ++q) {
        const int64_t h = h0 + hq * kEncVec + q;
        const bool in = j < n && h < k;
        double v = in ? B[h * ldb + j] : 0.0;
        ent[q] = make_entry8<kBig>(v, in ? entry_shift<kFold>(s, fold, h) : 0);
    }
    const bool use_mid = block_mid<kBig>(ent, md);  // uniform in the workgroup
    if (!use_mid) fill_p2<kBig>(mc, p2);
    if (use_mid) {
#pragma unroll
        for (int q = 0; q < kEncVec; ++q) to_mid(ent[q]);
    }
    for (int l = 0; l < mc.n; ++l) {
        const uint4 w = use_mid ? mid_residues16(ent, mc, *md, l)
                                : residues16<kBig>(ent, mc, l, p2 + l * kMaxShift);
        if (l > 0) __syncthreads();  // previous modulus fully copied out
        *reinterpret_cast<uint4*>(tile + tj * kLdsRow + hq * kEncVec) = w;
        __syncthreads();
        uint4 o = *reinterpret_cast<const uint4*>(tile + orow * kLdsRow + ochunk * kEncVec);
        *reinterpret_cast<uint4*>(planes + (int64_t)l * plane_stride +
                                  plane_offset(j0 + orow, h0 + ochunk * kEncVec, k_pad)) = o;
    }
}

// grid: (n_pad / 64, k_pad / 64).
template <bool kBig, bool kFold>
__global__ __launch_bounds__(kEncThreads) void encode_b_kernel(ModConsts mc, int64_t k, int64_t n,
                                                               const double* B, int64_t ldb,
                                                               const int32_t* shift_b,
                                                               const int32_t* fold,
                                                               int64_t n_pad, int64_t k_pad,
                                                               int8_t* planes, MidConsts md) {
    __shared__ __align__(16) int8_t tile[kTB * kLdsRow];
    __shared__ uint8_t p2[kBig ? kMaxModuli * kMaxShift : 1];
    encode_b_body<kBig, kFold>(mc, k, n, B, ldb, shift_b, fold, n_pad, k_pad, planes, blockIdx.x,
                               blockIdx.y, tile, p2, &md);
}

// ---- Reduce for float-alphabet channels ----
// Each entry's class modulo every channel (12-bit digit sums and a Barrett
// step, m < 2^16), then the format codes of the class's plane values from
// the channel's table (in LDS) into every plane: one byte per entry for
// FP8, one nibble for FP4 (entry h in nibble h % 2 of byte h / 2, low
// first). Planes use the block order of plane_offset over the planes' byte
// extent kb_pad (k_pad for FP8, k_pad / 2 for FP4).

__device__ __forceinline__ uint32_t fp_class(const Digits12& g, bool neg, const FpConsts& fc,
                                             int c) {
    // 12-bit digits: float-channel moduli exceed a byte
    const uint16_t* w = fc.w12[c];
    uint32_t t = g.d[0];
    t = __umul24(g.d[1], w[1]) + t;
    t = __umul24(g.d[2], w[2]) + t;
    t = __umul24(g.d[3], w[3]) + t;
    t = __umul24(g.d[4], w[4]) + t;
    t = __umul24(g.d[5], w[5]) + t;
    const uint32_t m = fc.m[c];
    uint32_t r = barrett32(t, m, fc.mu[c]);
    return (neg && r) ? m - r : r;
}

__device__ __forceinline__ void load_tables(const uint8_t* tables, int bytes, uint8_t* lds) {
    for (int i = threadIdx.x * 4; i < bytes; i += kEncThreads * 4) {
        if (i + 4 <= bytes) {
            *reinterpret_cast<uint32_t*>(lds + i) = *reinterpret_cast<const uint32_t*>(tables + i);
        } else {
            for (int q = i; q < bytes; ++q) lds[q] = tables[q];
        }
    }
    __syncthreads();
}

// Codes of 16 consecutive entries (h a multiple of 16) into plane p at
// (row, h): 16 bytes (FP8), 8 bytes (FP4, two codes per byte) or 12 bytes
// (FP6, packed: code i of a 32-code half at bits [6 i, 6 i + 6) of its 24
// bytes, units placed by plane_offset6; kb_pad is then the padded K in
// codes). The first 16 codes of a half fill its unit 0 and the low half of
// unit 1, the second 16 the high half of unit 1 and unit 2.
template <int kBits>
__device__ __forceinline__ void store_codes(int8_t* plane, int64_t row, int64_t h, int64_t kb_pad,
                                            const uint8_t* code) {
    if constexpr (kBits == 8) {
        uint4 w;
        w.x = code[0] | (code[1] << 8) | (code[2] << 16) | ((uint32_t)code[3] << 24);
        w.y = code[4] | (code[5] << 8) | (code[6] << 16) | ((uint32_t)code[7] << 24);
        w.z = code[8] | (code[9] << 8) | (code[10] << 16) | ((uint32_t)code[11] << 24);
        w.w = code[12] | (code[13] << 8) | (code[14] << 16) | ((uint32_t)code[15] << 24);
        *reinterpret_cast<uint4*>(plane + plane_offset(row, h, kb_pad)) = w;
    } else if constexpr (kBits == 6) {
        uint32_t d[3] = {0u, 0u, 0u};
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const uint32_t c = code[q] & 63u;
            const int bit = 6 * q, w = bit / 32, o = bit % 32;
            d[w] |= c << o;
            if (o > 26) d[w + 1] |= c >> (32 - o);
        }
        const int64_t s = h >> 6;
        const int u0 = 3 * (int)((h >> 5) & 1);
        if ((h & 16) == 0) {
            *reinterpret_cast<uint2*>(plane + plane_offset6(row, s, u0, kb_pad)) =
                make_uint2(d[0], d[1]);
            *reinterpret_cast<uint32_t*>(plane + plane_offset6(row, s, u0 + 1, kb_pad)) = d[2];
        } else {
            *reinterpret_cast<uint32_t*>(plane + plane_offset6(row, s, u0 + 1, kb_pad) + 4) = d[0];
            *reinterpret_cast<uint2*>(plane + plane_offset6(row, s, u0 + 2, kb_pad)) =
                make_uint2(d[1], d[2]);
        }
    } else {
        uint32_t lo = 0, hi = 0;
#pragma unroll
        for (int q = 0; q < 8; ++q) lo |= (uint32_t)(code[q] & 15u) << (4 * q);
#pragma unroll
        for (int q = 0; q < 8; ++q) hi |= (uint32_t)(code[8 + q] & 15u) << (4 * q);
        *reinterpret_cast<uint2*>(plane + plane_offset(row, h / 2, kb_pad)) = make_uint2(lo, hi);
    }
}

// A side: thread handles a 16-entry chunk of a row (chunks cross rows as in
// encode_a). Dynamic LDS: the table blob.
template <int kBits>
__global__ __launch_bounds__(kEncThreads) void encode_fp_a_kernel(
    FpConsts fc, const uint8_t* tables, int table_bytes, int64_t m, int64_t k, const double* A,
    int64_t lda, const int32_t* shift_a, int64_t m_pad, int64_t k_pad, int8_t* planes) {
    extern __shared__ uint8_t tab[];
    load_tables(tables, table_bytes, tab);
    // row argument of store_codes (bytes, or codes for FP6) and plane bytes
    const int64_t kb_pad = kBits == 4 ? k_pad / 2 : k_pad;
    const int64_t plane_stride = m_pad * (kBits == 6 ? k_pad / 4 * 3 : kb_pad);
    // a workgroup covers a tile of 64 rows x 64 codes (FP4: 32 rows x 128
    // codes), so each plane's stores fill one contiguous region of its block
    // (4 KB of FP8, 3 KB of FP6, 2 KB of FP4), as in encode_a
    constexpr int kTileCodes = kBits == 4 ? 128 : 64;
    constexpr int kTpr = kTileCodes / kEncVec;  // threads per tile row
    constexpr int kTileRows = kEncThreads / kTpr;
    const int64_t c = (int64_t)blockIdx.x * kChunksPerBlock + threadIdx.x;
    const int64_t tiles_k = k_pad / kTileCodes;
    const int64_t tile = c >> 8;
    const int t = (int)(c & 255);
    const int64_t i = (tile / tiles_k) * kTileRows + t / kTpr;
    const int64_t h = (tile % tiles_k) * kTileCodes + (t % kTpr) * kEncVec;
    if (i >= m_pad) return;
    uint8_t code[kEncVec];
    if (i >= m || h >= k) {  // padding: code 0 is +0 in both formats
        for (int q = 0; q < kEncVec; ++q) code[q] = 0;
        for (int p = 0; p < fc.planes; ++p) store_codes<kBits>(planes + p * plane_stride, i, h, kb_pad, code);
        return;
    }
    Entry ent[kEncVec];
    const int32_t s = shift_a[i];
    const double* row = A + i * lda;
#pragma unroll
    for (int q = 0; q < kEncVec; ++q) {
        const bool in = h + q < k;
        ent[q] = make_entry<false>(in ? row[h + q] : 0.0, in ? s : 0);
    }
    Digits12 g[kEncVec];
#pragma unroll
    for (int q = 0; q < kEncVec; ++q) g[q] = digits12(((uint64_t)ent[q].hi << 32) | ent[q].lo);
    for (int ch = 0; ch < fc.n; ++ch) {
        uint32_t cls[kEncVec];
#pragma unroll
        for (int q = 0; q < kEncVec; ++q) cls[q] = fp_class(g[q], ent[q].neg, fc, ch);
        const int rank = fc.rank[ch];
        const uint8_t* t = tab + fc.toff[ch];
        for (int r = 0; r < rank; ++r) {
#pragma unroll
            for (int q = 0; q < kEncVec; ++q) code[q] = t[cls[q] * rank + r];
            store_codes<kBits>(planes + (fc.plane0[ch] + r) * plane_stride, i, h, kb_pad, code);
        }
    }
}

// B side: workgroup (bx, by) covers columns 64 bx .. + 63 and K rows
// 64 by .. + 63; thread t takes column t % 64 over 16 consecutive K.
template <int kBits>
__global__ __launch_bounds__(kEncThreads) void encode_fp_b_kernel(
    FpConsts fc, const uint8_t* tables, int table_bytes, int64_t k, int64_t n, const double* B,
    int64_t ldb, const int32_t* shift_b, int64_t n_pad, int64_t k_pad, int8_t* planes) {
    extern __shared__ uint8_t tab[];
    load_tables(tables, table_bytes, tab);
    const int64_t kb_pad = kBits == 4 ? k_pad / 2 : k_pad;
    const int64_t plane_stride = n_pad * (kBits == 6 ? k_pad / 4 * 3 : kb_pad);
    const int64_t j = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
    const int64_t h = (int64_t)blockIdx.y * 64 + (threadIdx.x >> 6) * kEncVec;
    uint8_t code[kEncVec];
    if (j >= n || h >= k) {
        for (int q = 0; q < kEncVec; ++q) code[q] = 0;
        for (int p = 0; p < fc.planes; ++p) store_codes<kBits>(planes + p * plane_stride, j, h, kb_pad, code);
        return;
    }
    Entry ent[kEncVec];
    const int32_t s = shift_b[j];
#pragma unroll
    for (int q = 0; q < kEncVec; ++q) {
        const bool in = h + q < k;
        ent[q] = make_entry<false>(in ? B[(h + q) * ldb + j] : 0.0, in ? s : 0);
    }
    Digits12 g[kEncVec];
#pragma unroll
    for (int q = 0; q < kEncVec; ++q) g[q] = digits12(((uint64_t)ent[q].hi << 32) | ent[q].lo);
    for (int ch = 0; ch < fc.n; ++ch) {
        uint32_t cls[kEncVec];
#pragma unroll
        for (int q = 0; q < kEncVec; ++q) cls[q] = fp_class(g[q], ent[q].neg, fc, ch);
        const int rank = fc.rank[ch];
        const uint8_t* t = tab + fc.toff[ch];
        for (int r = 0; r < rank; ++r) {
#pragma unroll
            for (int q = 0; q < kEncVec; ++q) code[q] = t[cls[q] * rank + r];
            store_codes<kBits>(planes + (fc.plane0[ch] + r) * plane_stride, j, h, kb_pad, code);
        }
    }
}

// ---- Grouped Reduce ----
// kBig is chosen for the whole group (the form for kept bits above 62 is
// exact for any shift, only slower).

template <bool kBig>
__global__ __launch_bounds__(kEncThreads) void group_encode_a_kernel(GroupArgs g) {
    __shared__ uint8_t p2[kBig ? kMaxModuli * kMaxShift : 1];
    const int32_t* pre = g.prefix + kGEncA * (g.count + 1);
    const int p = group_find(pre, g.count, blockIdx.x);
    const GProblem& P = g.probs[p];
    encode_a_body<kBig, false>(g.mods[P.plan], P.m, P.k, P.A, P.lda,
                               reinterpret_cast<const int32_t*>(g.ws + P.off_sa), nullptr, P.m_pad,
                               P.k_pad, reinterpret_cast<int8_t*>(g.ws + P.off_pa),
                               (int64_t)(blockIdx.x - pre[p]) * kChunksPerBlock + threadIdx.x, p2);
}

template <bool kBig>
__global__ __launch_bounds__(kEncThreads) void group_encode_b_kernel(GroupArgs g) {
    __shared__ __align__(16) int8_t tile[kTB * kLdsRow];
    __shared__ uint8_t p2[kBig ? kMaxModuli * kMaxShift : 1];
    const int32_t* pre = g.prefix + kGEncB * (g.count + 1);
    const int p = group_find(pre, g.count, blockIdx.x);
    const GProblem& P = g.probs[p];
    const int64_t lb = blockIdx.x - pre[p];
    const int64_t gx = P.n_pad / kTB;
    encode_b_body<kBig, false>(g.mods[P.plan], P.k, P.n, P.B, P.ldb,
                               reinterpret_cast<const int32_t*>(g.ws + P.off_sb), nullptr, P.n_pad,
                               P.k_pad, reinterpret_cast<int8_t*>(g.ws + P.off_pb), lb % gx, lb / gx,
                               tile, p2);
}

}  // namespace

hipError_t launch_group_encode(hipStream_t st, const GroupArgs& g, int32_t enc_a, int32_t enc_b,
                               bool big) {
    if (enc_a > 0) {
        if (big)
            group_encode_a_kernel<true><<<dim3((unsigned)enc_a), dim3(kEncThreads), 0, st>>>(g);
        else
            group_encode_a_kernel<false><<<dim3((unsigned)enc_a), dim3(kEncThreads), 0, st>>>(g);
    }
    if (enc_b > 0) {
        if (big)
            group_encode_b_kernel<true><<<dim3((unsigned)enc_b), dim3(kEncThreads), 0, st>>>(g);
        else
            group_encode_b_kernel<false><<<dim3((unsigned)enc_b), dim3(kEncThreads), 0, st>>>(g);
    }
    return hipGetLastError();
}

hipError_t launch_encode_fp(hipStream_t st, const FpConsts& fc, const uint8_t* tables,
                            int table_bytes, int64_t m, int64_t n, int64_t k, const double* A,
                            int64_t lda, const double* B, int64_t ldb, const int32_t* shift_a,
                            const int32_t* shift_b, int64_t m_pad, int64_t n_pad, int64_t k_pad,
                            int8_t* planes_a, int8_t* planes_b) {
    const size_t lds = (size_t)table_bytes;
    auto run = [&](auto bits_tag) {
        constexpr int kBits = decltype(bits_tag)::value;
        if (m_pad > 0 && k_pad > 0) {
            dim3 grid((unsigned)((m_pad * (k_pad / kEncVec) + kChunksPerBlock - 1) /
                                 kChunksPerBlock));
            encode_fp_a_kernel<kBits><<<grid, dim3(kEncThreads), lds, st>>>(
                fc, tables, table_bytes, m, k, A, lda, shift_a, m_pad, k_pad, planes_a);
        }
        if (n_pad > 0 && k_pad > 0) {
            dim3 grid((unsigned)(n_pad / 64), (unsigned)(k_pad / 64));
            encode_fp_b_kernel<kBits><<<grid, dim3(kEncThreads), lds, st>>>(
                fc, tables, table_bytes, k, n, B, ldb, shift_b, n_pad, k_pad, planes_b);
        }
    };
    if (fc.fmt == 4)
        run(std::integral_constant<int, 4>{});
    else if (fc.fmt == 2)
        run(std::integral_constant<int, 6>{});
    else
        run(std::integral_constant<int, 8>{});
    return hipGetLastError();
}

namespace {

// Host: the weights of bytes 8..11 for the 96-bit form of the exact form.
MidConsts mid_consts(const ModConsts& mc, bool big) {
    MidConsts md{};
    md.on = big ? 1 : 0;
    for (int l = 0; l < mc.n && l < kMaxModuli; ++l) {
        const uint32_t m = mc.m[l];
        uint32_t w = 1 % m;
        for (int b = 0; b < 64; ++b) w = (w * 2u) % m;  // 2^64 mod m
        uint32_t packed = 0;
        for (int i = 0; i < 4; ++i) {
            const int32_t v = w >= (m + 1) / 2 ? (int32_t)w - (int32_t)m : (int32_t)w;
            packed |= (uint32_t)(uint8_t)(int8_t)v << (8 * i);
            w = (w * 256u) % m;
        }
        md.s8c[l] = (int32_t)packed;
    }
    return md;
}

}  // namespace

hipError_t launch_encode_a(hipStream_t st, const ModConsts& mc, int64_t m, int64_t k,
                           const double* A, int64_t lda, const int32_t* shift_a, int64_t m_pad,
                           int64_t k_pad, int8_t* planes_a, bool big, const int32_t* fold) {
    if (m_pad <= 0 || k_pad <= 0) return hipSuccess;
    dim3 grid((unsigned)((m_pad * (k_pad / kEncVec) + kChunksPerBlock - 1) / kChunksPerBlock));
    const MidConsts md = mid_consts(mc, big);
    auto go = [&](auto kernel) {
        kernel<<<grid, dim3(kEncThreads), 0, st>>>(mc, m, k, A, lda, shift_a, fold, m_pad, k_pad,
                                                   planes_a, md);
    };
    if (big)
        fold ? go(encode_a_kernel<true, true>) : go(encode_a_kernel<true, false>);
    else
        fold ? go(encode_a_kernel<false, true>) : go(encode_a_kernel<false, false>);
    return hipGetLastError();
}

hipError_t launch_encode_b(hipStream_t st, const ModConsts& mc, int64_t k, int64_t n,
                           const double* B, int64_t ldb, const int32_t* shift_b, int64_t n_pad,
                           int64_t k_pad, int8_t* planes_b, bool big, const int32_t* fold) {
    if (n_pad <= 0 || k_pad <= 0) return hipSuccess;
    dim3 grid((unsigned)(n_pad / kTB), (unsigned)(k_pad / kTB));
    const MidConsts md = mid_consts(mc, big);
    auto go = [&](auto kernel) {
        kernel<<<grid, dim3(kEncThreads), 0, st>>>(mc, k, n, B, ldb, shift_b, fold, n_pad, k_pad,
                                                   planes_b, md);
    };
    if (big)
        fold ? go(encode_b_kernel<true, true>) : go(encode_b_kernel<true, false>);
    else
        fold ? go(encode_b_kernel<false, true>) : go(encode_b_kernel<false, false>);
    return hipGetLastError();
}

}  // namespace ozemu
