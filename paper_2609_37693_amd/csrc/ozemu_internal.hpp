// Internal definitions shared by the host plan code and the HIP kernels of
// libozemu: launch-argument structs, tile sizes, and the integer helpers the
// kernels use (Barrett reduction, IEEE-754 field extraction).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ozemu {

constexpr int kMaxModuli = 32;  // moduli per plan
constexpr int kMaxDigits = 10;  // 32-bit digits of CRT sums: N * P < 2^(8*32 + 5)
constexpr int kChunkBits = 40;    // FP64 chunks of CRT sums with INT8 moduli
constexpr int kChunkBitsFp = 30;  // ... and with float-channel moduli (below 2^16)
constexpr int kMaxChunks = 7;   // 40-bit chunks of P + 2 bits for at most 32 moduli of <= 2^8
constexpr int kBetaCap = 127;   // largest kept-bit count of any mode
constexpr int kSmallBits = 62;  // kept bits up to which Reduce takes signed base-256 digits

// Residue GEMM tiling. Planes are padded to whole tiles, so the GEMM kernel
// needs no bounds checks; padding entries are zero.
constexpr int kTileM = 256;
constexpr int kTileN = 256;
constexpr int kTileK = 64;

// Residue planes (and the bound planes) are stored in the order the GEMM
// reads them: blocks of 256 rows x 64 K-bytes (16 KB), block (row tile tr,
// K step ks) at byte ((tr * (k_pad / 64)) + ks) * 16384 of the plane; inside
// a block row r takes 64 bytes and its 16-byte chunk c sits at chunk
// position c ^ ((r >> 2) & 3). One K step of a tile is then one contiguous
// 16 KB block, copied unchanged into LDS, where the chunk swizzle spreads
// the MFMA operand reads of 16 consecutive rows over distinct LDS banks.
constexpr int kPlaneRows = 256;
constexpr int kPlaneK = 64;
__host__ __device__ __forceinline__ int64_t plane_offset(int64_t row, int64_t h, int64_t k_pad) {
    const int64_t tr = row >> 8, r = row & 255, ks = h >> 6, c = (h >> 4) & 3;
    return ((tr * (k_pad >> 6) + ks) * 256 + r) * 64 + ((c ^ ((r >> 2) & 3)) << 4) + (h & 15);
}

// Packed FP6 planes: a K step of 64 codes is 48 bytes of a row, six 8-byte
// units; the block of (row tile, step) is 256 rows x 48 bytes at
// ((tile * steps) + step) * 12288, row r at 48 r in it, and unit u at
// position (u + rot(r)) mod 6 with rot(r) = ((r >> 3) ^ (r >> 4)) & 1, so
// that the 8-byte fragment reads of 32 consecutive rows spread over the LDS
// banks. Byte offset of unit u (0..5) of step s of a row; k_pad in codes.
constexpr int kF6StepBytes = 48;
__host__ __device__ __forceinline__ int64_t plane_offset6(int64_t row, int64_t s, int u,
                                                        int64_t k_pad) {
    const int64_t tr = row >> 8;
    const int r = (int)(row & 255);
    const int rot = ((r >> 3) ^ (r >> 4)) & 1;
    const int pos = (u + rot) % 6;
    return ((tr * (k_pad >> 6) + s) * 256 + r) * kF6StepBytes + 8 * pos;
}

// Row/column key for the exponent scan: frexp exponent of the largest
// magnitude, or these sentinels.
constexpr int32_t kKeyZero = INT32_MIN + 1;
constexpr int32_t kKeyNonFinite = INT32_MAX;
constexpr int32_t kShiftNonFinite = INT32_MIN;

// Per-modulus constants for reduction (Barrett with mu = floor(2^32 / m),
// one correction step) passed by value as a kernel argument.
struct ModConsts {
    int n;
    uint32_t m[kMaxModuli];
    uint32_t mu[kMaxModuli];
    uint32_t c32[kMaxModuli];  // 2^32 mod m
    uint32_t c16[kMaxModuli];  // 2^16 mod m
    float rcp[kMaxModuli];     // 1 / m rounded to FP32
    uint16_t w12[kMaxModuli][6];  // 2^(12 i) mod m, i = 0..5
    uint32_t w8[kMaxModuli][2];   // bytes 2^(8 i) mod m, i = 0..3 and 4..7 (m <= 256)
    float rcp_up[kMaxModuli];     // 1 / m rounded up to FP32
    uint32_t c64n[kMaxModuli];    // (-2^64) mod m
    uint32_t s8[kMaxModuli][2];   // signed bytes: balanced 2^(8 i) mod m, i = 0..7
    uint32_t km[kMaxModuli];      // m ceil(2^17 / m)
};

// t mod m for t < 2^24 and 2 <= m <= 256: t is exact in FP32 and t * rcp
// is within 1/m < 1/2 of t / m, so the truncated quotient is off by at most
// one and a single correction in either direction finishes.
__host__ __device__ __forceinline__ uint32_t mod24(uint32_t t, uint32_t m, float rcp) {
    const uint32_t q = (uint32_t)((float)t * rcp);
#if defined(__HIP_DEVICE_COMPILE__)
    int32_t r = (int32_t)t - (int32_t)__umul24(q, m);
#else
    int32_t r = (int32_t)t - (int32_t)(q * m);
#endif
    r += (r < 0) ? (int32_t)m : 0;
    r -= (r >= (int32_t)m) ? (int32_t)m : 0;
    return (uint32_t)r;
}

// 12-bit digits of a value below 2^72 (six digits).
struct Digits12 {
    uint32_t d[6];
};
__host__ __device__ __forceinline__ Digits12 digits12(uint64_t v) {
    const uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    Digits12 g;
    g.d[0] = lo & 0xFFFu;
    g.d[1] = (lo >> 12) & 0xFFFu;
    g.d[2] = (lo >> 24) | ((hi & 0xFu) << 8);
    g.d[3] = (hi >> 4) & 0xFFFu;
    g.d[4] = (hi >> 16) & 0xFFFu;
    g.d[5] = hi >> 28;
    return g;
}

// v mod m from its digits: sum_i d_i (2^(12 i) mod m) < 6 * 2^12 * 2^8 < 2^23.
__host__ __device__ __forceinline__ uint32_t digits_mod(const Digits12& g, const uint16_t* w,
                                                       uint32_t m, float rcp) {
#if defined(__HIP_DEVICE_COMPILE__)
    uint32_t t = g.d[0];
    t = __umul24(g.d[1], w[1]) + t;
    t = __umul24(g.d[2], w[2]) + t;
    t = __umul24(g.d[3], w[3]) + t;
    t = __umul24(g.d[4], w[4]) + t;
    t = __umul24(g.d[5], w[5]) + t;
#else
    uint32_t t = g.d[0] + g.d[1] * w[1] + g.d[2] * w[2] + g.d[3] * w[3] + g.d[4] * w[4] +
                 g.d[5] * w[5];
#endif
    return mod24(t, m, rcp);
}

// CRT constants: X = sum_l u_l M_l - q P with u_l = (z_l * inv_l) mod m_l,
// M_l = P / m_l, inv_l = M_l^-1 mod m_l; digits little-endian, 32 bits each.
struct CrtConsts {
    int n;
    int d;  // digits used
    uint32_t m[kMaxModuli];
    uint32_t mu[kMaxModuli];
    uint32_t inv[kMaxModuli];
    double rcp[kMaxModuli];  // 1 / m_l rounded to FP64
    uint32_t Ml[kMaxModuli][kMaxDigits];
    uint32_t P[kMaxDigits];
    uint32_t half[kMaxDigits];  // floor((P - 1) / 2)
    // N_l = inv_l M_l (below P) and P in chunks of cb bits (kChunkBits for
    // INT8 moduli, kChunkBitsFp for float channels) held exactly in FP64,
    // and 2^(cb k) / P rounded to FP64; kc chunks (0: too many for the
    // chunk form, float channels then take 32-bit digits)
    int kc;
    int cb;
    double N40[kMaxModuli][kMaxChunks];
    double P40[kMaxChunks];
    double R40[kMaxChunks];
};
static_assert(sizeof(CrtConsts) + 128 <= 4096, "CRT constants travel as a kernel argument");

// x mod m for x < 2^32, m in [2, 2^16]; mu = floor(2^32 / m).
__host__ __device__ __forceinline__ uint32_t barrett32(uint32_t x, uint32_t m, uint32_t mu) {
#if defined(__HIP_DEVICE_COMPILE__)
    uint32_t q = __umulhi(x, mu);
#else
    uint32_t q = (uint32_t)(((uint64_t)x * mu) >> 32);
#endif
    uint32_t r = x - q * m;
    return r >= m ? r - m : r;
}

// v mod m for v < 2^53, m <= 256: with v = a 2^32 + b 2^16 + c the sum
// a (2^32 mod m) + b (2^16 mod m) + c is below 2^21 2^8 + 2^16 2^8 + 2^16
// < 2^30, so one Barrett step finishes the reduction.
__host__ __device__ __forceinline__ uint32_t mod53(uint64_t v, uint32_t m, uint32_t mu, uint32_t c32,
                                                  uint32_t c16) {
    uint32_t a = (uint32_t)(v >> 32);  // < 2^21
    uint32_t lo = (uint32_t)v;
    uint32_t t = a * c32 + (lo >> 16) * c16 + (lo & 0xFFFFu);
    return barrett32(t, m, mu);
}

// 2^e mod m for 0 <= e, by square and multiply (values < 2^16).
__host__ __device__ __forceinline__ uint32_t pow2mod(int e, uint32_t m, uint32_t mu) {
    uint32_t r = 1 % m, b = 2 % m;
    while (e > 0) {
        if (e & 1) r = barrett32(r * b, m, mu);
        b = barrett32(b * b, m, mu);
        e >>= 1;
    }
    return r;
}

// Magnitude of a finite double as integer significand times a power of two:
// |x| = mant * 2^ex, mant < 2^53 (0 for zero).
__host__ __device__ __forceinline__ void split_double(uint64_t bits, uint64_t& mant, int& ex) {
    uint32_t be = (uint32_t)((bits >> 52) & 0x7FF);
    uint64_t frac = bits & 0x000FFFFFFFFFFFFFull;
    if (be == 0) {
        mant = frac;
        ex = -1074;
    } else {
        mant = frac | (1ull << 52);
        ex = (int)be - 1075;
    }
}

// frexp exponent e of a finite nonzero magnitude: 2^(e-1) <= |x| < 2^e.
__host__ __device__ __forceinline__ int frexp_exponent(uint64_t absbits) {
    uint32_t be = (uint32_t)(absbits >> 52);
    if (be != 0) return (int)be - 1022;
#if defined(__HIP_DEVICE_COMPILE__)
    int lz = __clzll((long long)absbits);
#else
    int lz = __builtin_clzll(absbits);
#endif
    return (64 - lz) - 1074;
}

// Row/column key of one entry (see kKeyZero, kKeyNonFinite).
__host__ __device__ __forceinline__ int32_t entry_key(uint64_t bits) {
    uint64_t a = bits & 0x7FFFFFFFFFFFFFFFull;
    if (a >= 0x7FF0000000000000ull) return kKeyNonFinite;
    if (a == 0) return kKeyZero;
    return frexp_exponent(a);
}

// Balanced residue in two's complement int8 of the integer sign * |v| where
// r = |v| mod m: representatives [-floor(m/2), ceil(m/2) - 1].
__host__ __device__ __forceinline__ int8_t balanced_i8(uint32_t r, bool neg, uint32_t m) {
    if (neg && r != 0) r = m - r;
    int32_t v = (r >= (m + 1) / 2) ? (int32_t)r - (int32_t)m : (int32_t)r;
    return (int8_t)v;
}

// Residue of trunc(x * 2^s) modulo m for a finite double x, in [0, m), with
// the sign returned separately. Writing |x| = mant * 2^ex, the truncated
// magnitude is mant >> (-(ex + s)) when ex + s <= 0 (a 53-bit integer), else
// mant * 2^(ex + s), whose residue is (mant mod m)(2^(ex+s) mod m) mod m.
__host__ __device__ __forceinline__ uint32_t trunc_residue(uint64_t mant, int sh, uint32_t m,
                                                          uint32_t mu, uint32_t c32, uint32_t c16) {
    if (sh <= 0) {
        uint64_t v = (sh <= -64) ? 0 : (mant >> (-sh));
        return mod53(v, m, mu, c32, c16);
    }
    uint32_t r0 = mod53(mant, m, mu, c32, c16);
    return barrett32(r0 * pow2mod(sh, m, mu), m, mu);
}

// Limb channels of a float alphabet (FP8 E4M3, FP4 E2M1) for the kernels:
// channel c has modulus m[c], rank[c] planes (1: one limb; 3: two-limb Toom
// form at points 0, 1, infinity) starting at plane plane0[c], weights
// lbar[c][k] (the form's weights reduced into [0, m)), the 12-bit digit
// weights 2^(12 i) mod m, and its code table at byte toff[c] of the table
// blob: m * rank bytes, the format codes of the plane values of each class.
struct FpConsts {
    int n;       // channels
    int planes;  // sum of ranks
    int fmt;     // MFMA operand format: 0 FP8 E4M3, 2 FP6 E2M3, 4 FP4 E2M1
    int es;      // plane value v is stored as v * 2^-es
    uint32_t m[kMaxModuli];
    uint32_t mu[kMaxModuli];
    int32_t rank[kMaxModuli];
    int32_t plane0[kMaxModuli];
    int32_t toff[kMaxModuli];
    uint32_t lbar[kMaxModuli][3];
    uint16_t w12[kMaxModuli][6];
};

// One plane round of the float-channel products over one slab (kernel
// argument): items c < count, each tiles of one channel's plane; K bytes
// [kb_begin, kb_begin + kb_len) of planes whose rows hold kb_pad bytes.
struct FpGemmArgs {
    int count;
    int first;        // the residues start at zero (first plane of the first slab)
    float scale;      // 2^(2 es): accumulator to integer
    int64_t start[kMaxModuli + 1];  // first workgroup of each item
    int32_t plane[kMaxModuli];
    int32_t chan[kMaxModuli];
    uint32_t m[kMaxModuli], mu[kMaxModuli], lbar[kMaxModuli];
    int64_t m_pad, n_pad, kb_pad, kb_begin, kb_len;
    const int8_t* pa;
    const int8_t* pb;
    uint16_t* z;
};

// ---- Grouped launches: many independent products in one set of launches.
// The work of each phase is a list of workgroups, problem after problem:
// prefix[kind * (count + 1) + p] is the first workgroup of problem p and
// prefix[kind * (count + 1) + count] the total. The GEMM's work items
// (modulus, tile) are split into one list per XCD (kind kGTiles + x): each
// (problem, modulus) gives every XCD a contiguous eighth of its tiles in
// band order, so the workgroups of one XCD share operand strips in its L2.
// The lists follow the problems in `order` (descending K), so the longest
// tiles are taken first.
constexpr int kMaxGroup = 4096;  // problems per group (two 64-wide ballots)
constexpr int kXcds = 8;
enum GKind : int {
    kGColInit = 0, kGRows, kGCols, kGShifts, kGEncA, kGEncB, kGCrt, kGTiles,
    kGKinds = kGTiles + kXcds
};

// Moduli that XCD x takes, with every tile of each, for the q-th problem
// in GEMM order: l = first, first + 8, ... (count of them). The XCD's
// workgroups then run the tiles of one modulus together, so that the
// operand strips they share stay in that XCD's L2; the residue rotates with
// q so that remainders spread over the XCDs.
__host__ __device__ __forceinline__ void xcd_moduli(int N, int x, int q, int& first, int& count) {
    first = (x + q) & (kXcds - 1);
    count = first < N ? (N - 1 - first) / kXcds + 1 : 0;
}

struct GProblem {
    int64_t m, n, k, m_pad, n_pad, k_pad;
    const double* A;
    const double* B;
    double* C;
    int64_t lda, ldb, ldc;
    int64_t off_sa, off_sb, off_pa, off_pb, off_z;  // byte offsets into the workspace
    int32_t plan, beta_a, beta_b, big;
};

// Kernel argument of every grouped launch (tables live in the workspace).
struct GroupArgs {
    const GProblem* probs;
    const ModConsts* mods;
    const CrtConsts* crts;
    const int32_t* prefix;  // [kGKinds][count + 1]
    const int32_t* order;   // problems in GEMM work order
    char* ws;
    int32_t* counter;       // persistent GEMM work counters, one per XCD
    int32_t count;
};

#if defined(__HIPCC__)
// Problem p with prefix[p] <= b < prefix[p + 1] (empty problems skipped);
// the whole wave must be active. Two ballots: over every stride-th entry,
// then inside the chosen stride (count <= 64 * 64).
__device__ __forceinline__ int group_find(const int32_t* prefix, int count, int32_t b) {
    const int lane = threadIdx.x & 63;
    const int stride = (count + 63) >> 6;
    const int i1 = lane * stride;
    const unsigned long long m1 = __ballot(i1 < count && prefix[i1] <= b);
    const int base = (63 - __clzll((long long)m1)) * stride;
    const int i2 = base + lane;
    const unsigned long long m2 = __ballot(lane < stride && i2 < count && prefix[i2] <= b);
    return __builtin_amdgcn_readfirstlane(base + 63 - __clzll((long long)m2));
}
#endif

// Launchers (defined in the .hip files). All take the caller's stream and
// return hipSuccess or the launch error.
// Row / column keys. A non-null `fold` (k entries) counts entry (i, h) of
// A as A_ih 2^-fold[h] (rows), entry (h, j) of B as B_hj 2^-fold[h]
// (columns): the power-of-two fold of cached shifts used by the backward.
hipError_t launch_scale_rows(hipStream_t st, int64_t m, int64_t k, const double* A, int64_t lda,
                             int32_t* key_a, const int32_t* fold = nullptr);
hipError_t launch_scale_cols(hipStream_t st, int64_t k, int64_t n, const double* B, int64_t ldb,
                             int32_t* key_b, const int32_t* fold = nullptr);
hipError_t launch_keys_to_shifts(hipStream_t st, int64_t count, int32_t* key_to_shift, int beta,
                                 const int32_t* beta_per_entry);
// Encode: `big` selects the form for kept bits above 63 (left shifts of
// more than 10 bits), required for the bound-adaptive mode. A non-null
// `fold` (k entries) subtracts fold[h] from the shift of every entry with
// inner index h, as in launch_scale_rows / launch_scale_cols.
hipError_t launch_encode_a(hipStream_t st, const ModConsts& mc, int64_t m, int64_t k,
                           const double* A, int64_t lda, const int32_t* shift_a, int64_t m_pad,
                           int64_t k_pad, int8_t* planes_a, bool big,
                           const int32_t* fold = nullptr);
hipError_t launch_encode_b(hipStream_t st, const ModConsts& mc, int64_t k, int64_t n,
                           const double* B, int64_t ldb, const int32_t* shift_b, int64_t n_pad,
                           int64_t k_pad, int8_t* planes_b, bool big,
                           const int32_t* fold = nullptr);
// Transpose block-ordered planes: `in` holds `planes` planes of
// in_rows_pad x in_k_pad, `out` gets out_rows_pad x in_rows_pad with
// out(r, h) = in(h, r); rows r >= in_k_pad are zero. out_rows_pad is a
// multiple of 256 not below in_k_pad.
hipError_t launch_transpose_planes(hipStream_t st, int planes, int64_t in_rows_pad,
                                   int64_t in_k_pad, int64_t out_rows_pad, const int8_t* in,
                                   int8_t* out);
hipError_t launch_residue_gemm(hipStream_t st, const ModConsts& mc, int64_t m_pad, int64_t n_pad,
                               int64_t k_pad, const int8_t* planes_a, const int8_t* planes_b,
                               uint8_t* residues);
hipError_t launch_bound_gemm(hipStream_t st, int64_t m_pad, int64_t n_pad, int64_t k_pad,
                             const int8_t* bar_a, const int8_t* bar_b, int32_t* gmax_a,
                             int32_t* gmax_b);
hipError_t launch_bound_planes_a(hipStream_t st, int64_t m, int64_t k, const double* A,
                                 int64_t lda, const int32_t* key_a, int64_t m_pad, int64_t k_pad,
                                 int8_t* bar_a);
hipError_t launch_bound_planes_b(hipStream_t st, int64_t k, int64_t n, const double* B,
                                 int64_t ldb, const int32_t* key_b, int64_t n_pad, int64_t k_pad,
                                 int8_t* bar_b);
hipError_t launch_bound_shifts(hipStream_t st, int64_t count, const int32_t* key,
                               const int32_t* gmax, int L, int32_t* shift);
hipError_t launch_fill_i32(hipStream_t st, int64_t count, int32_t value, int32_t* out);
hipError_t launch_reconstruct(hipStream_t st, const CrtConsts& cc, int64_t m, int64_t n,
                              int64_t m_pad, int64_t n_pad, const uint8_t* residues,
                              const int32_t* shift_a, const int32_t* shift_b, double* C,
                              int64_t ldc);
hipError_t launch_zero_c(hipStream_t st, int64_t m, int64_t n, double* C, int64_t ldc);

// Float channels: Reduce (codes of every plane), one plane round of the
// residue GEMMs, Reconstruct from uint16 residues.
hipError_t launch_encode_fp(hipStream_t st, const FpConsts& fc, const uint8_t* tables,
                            int table_bytes, int64_t m, int64_t n, int64_t k, const double* A,
                            int64_t lda, const double* B, int64_t ldb, const int32_t* shift_a,
                            const int32_t* shift_b, int64_t m_pad, int64_t n_pad, int64_t k_pad,
                            int8_t* planes_a, int8_t* planes_b);
hipError_t launch_fp_gemm(hipStream_t st, const FpGemmArgs& g, int fmt);
hipError_t launch_reconstruct16(hipStream_t st, const CrtConsts& cc, int64_t m, int64_t n,
                                int64_t m_pad, int64_t n_pad, const uint16_t* residues,
                                const int32_t* shift_a, const int32_t* shift_b, double* C,
                                int64_t ldc);

// Grouped phases; `total` is the phase's workgroup count (prefix total).
hipError_t launch_group_init(hipStream_t st, const GroupArgs& g, int32_t total);
hipError_t launch_group_scale(hipStream_t st, const GroupArgs& g, int32_t rows, int32_t cols,
                              int32_t shifts);
hipError_t launch_group_encode(hipStream_t st, const GroupArgs& g, int32_t enc_a, int32_t enc_b,
                               bool big);
hipError_t launch_group_gemm(hipStream_t st, const GroupArgs& g, const int32_t* tiles_per_xcd,
                             int32_t workers);
hipError_t launch_group_reconstruct(hipStream_t st, const GroupArgs& g, int32_t blocks, int dmax);

}  // namespace ozemu
