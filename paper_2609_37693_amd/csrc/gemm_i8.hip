// Residue GEMMs with the fused epilogue (Sec. V-A phases 3-4, Sec. V-C):
// for every modulus m_l, W = R_A[l] R_B[l]^T in exact INT32 on the gfx950
// INT8 matrix cores (v_mfma_i32_32x32x32_i8), then Z = W mod m_l in [0, m_l)
// stored as uint8. One launch covers all moduli and output tiles.
//
// Exactness: |W| <= k floor(m/2)^2 <= 2^31 - 1 is checked by the host before
// launch (eq. "ov-accgen"), so INT32 accumulation never wraps, in any order.
//
// Tiling: 256 x 256 output tile per workgroup of 4 waves (2 x 2), each wave
// 128 x 128 as 4 x 4 MFMA blocks of 32 x 32 with INT32 accumulators (256
// accumulation registers per lane, one wave per SIMD). The MFMA's first
// operand takes the B-plane rows (output columns j) and its second the
// A-plane rows (output rows i), so each lane ends with 4 consecutive j of
// one i and the epilogue packs them into one 32-bit word.
//
// The same kernel with a max epilogue serves the bound-adaptive scaling
// mode: it computes Gbar = abar bbar^T and reduces row and column maxima.
#include <type_traits>

#include "ozemu_internal.hpp"

namespace ozemu {

namespace {

typedef int v2i __attribute__((ext_vector_type(2)));
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int kThreads = 256;
constexpr int kBM = kTileM;  // rows i per tile
constexpr int kBN = kTileN;  // columns j per tile
constexpr int kWaveM = 128, kWaveN = 128;
constexpr int kFM = kWaveM / 32, kFN = kWaveN / 32;  // MFMA blocks per wave
constexpr int kGroup = 8;  // tile rows per band of the tile order

// Output staging for the residue epilogue reuses the operand LDS. Row stride
// of 66 dwords: the 32 rows a store instruction touches land on even banks
// and the two lane halves on even/odd banks.
constexpr int kOutRow = 264;
// uint16 staging of half a tile (128 rows x 256 residues) for the float
// channels' epilogue: 528-byte rows.
constexpr int kOutRow16 = 528;

enum class Epi { kMod, kMax, kRmw };

// Band order inside one modulus: bands of kGroup tile rows, column by
// column, so consecutive tiles share operand strips.
__device__ __forceinline__ void band_tile(int64_t t, int tiles_m, int tiles_n, int& tm, int& tn) {
    const int64_t in_group = (int64_t)kGroup * tiles_n;
    const int first_m = (int)(t / in_group) * kGroup;
    const int gsize = min(tiles_m - first_m, kGroup);
    const int64_t r = t % in_group;
    tm = first_m + (int)(r % gsize);
    tn = (int)(r / gsize);
}

// Tile order: all XCDs on one modulus at a time (the hardware dispatches
// workgroup b to XCD b % 8), each XCD on a contiguous band-ordered eighth of
// that modulus's tiles, so operand strips are shared inside one L2.
__device__ __forceinline__ void tile_of(int64_t bid, int tiles_m, int tiles_n, int& l, int& tm,
                                        int& tn) {
    const int64_t T = (int64_t)tiles_m * tiles_n;
    int64_t t;
    if ((T & 7) == 0) {
        const int64_t x = bid & 7, u = bid >> 3, per = T >> 3;
        l = (int)(u / per);
        t = x * per + (u % per);
    } else {
        l = (int)(bid / T);
        t = bid % T;
    }
    band_tile(t, tiles_m, tiles_n, tm, tn);
}

// K pipeline: K steps of 64 bytes in four LDS stages, filled by
// global_load_lds_dwordx4 (each lane moves 16 bytes from global memory
// straight into LDS, with no VGPR staging and no LDS store instructions)
// three steps ahead of their use. A K step of a tile is one contiguous 16 KB
// block of each plane (plane_offset), so every wave-level load copies 1 KB
// of whole cache lines unchanged into LDS, chunk swizzle included. One
// barrier per step, preceded by the wait for the loads of step t+2 only; the
// barrier has no memory fence, so the loads of step t+3 stay in flight
// across it. MFMA operands are read one 32-byte slice ahead, across step
// boundaries.
constexpr int kDBK = 64;
// Ring depth: four K steps (128 KiB). A fifth (the 160 KiB limit) measured
// slower at 8192^3, so every kernel uses four.
constexpr int kDStages = 4;
constexpr int kDStagesMax = 5;
constexpr int kDStage = (kBM + kBN) * kDBK;          // 32 KB
constexpr int kDLoads = (kBM + kBN) * kDBK / 1024 / 4;  // 1 KB wave loads per wave per step
static_assert(kDLoads == 8, "load split");
static_assert(kBM * kOutRow <= kDStages * kDStage, "output staging fits");
static_assert(128 * kOutRow16 <= kDStages * kDStage, "float-channel staging fits");

// s_waitcnt immediate: vmcnt(v) and lgkmcnt(l), expcnt untouched.
#define OZ_WAITCNT(v, l) (((v) & 15) | (((v) >> 4) << 14) | (7 << 4) | ((l) << 8))

typedef __attribute__((address_space(3))) void* lds_ptr_t;

__device__ __forceinline__ void barrier_no_fence() {
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
}

// One 256 x 256 output tile (tm, tn) over K = k_pad (a positive multiple of
// 64): gA and gB point at the first block of the tile's row strip in the A
// and B planes of one modulus (plane_offset order), gZ at the tile's first
// residue (row stride n_pad). Modulus m (kMod; mu is the Barrett constant
// of the float-channel epilogue);
// row/column maxima into gmax_a/gmax_b (kMax). `lds` holds
// S * kDStage bytes (a ring of S K steps, loads issued S - 1 steps ahead);
// the caller synchronizes before reusing it.
// Operand format of gemm_tile: INT8 (v_mfma_i32_32x32x32_i8, INT32
// accumulators) or the float alphabets through v_mfma_f32_32x32x64_f8f6f4
// with FP32 accumulators: FP8 E4M3 (32 bytes per lane, one instruction per
// 64-byte K step) and FP4 E2M1 (16 bytes per lane, two per step, read as
// INT8 is).
enum Fmt : int { kI8 = 0, kF8 = 1, kF4 = 2, kF6 = 3 };
// FP6 E2M3 uses the FP8 tile and K pipeline over packed planes (48 bytes of
// a row per K step of 64 codes, plane_offset6): a lane's 32 values are 24
// bytes of 6-bit codes (value i at bits [6 i, 6 i + 6) of the first six
// dwords of the operand; the last two are not read).
template <int F>
constexpr int mfma_fmt() { return F == kF4 ? 4 : F == kF6 ? 2 : 0; }

// Epilogue of a float-channel product: residues z (uint16, row stride
// n_pad) of the tile receive (z + lbar (W mod m)) mod m, or that value
// alone when `first`; W = accumulator * scale (exact integers).
struct FpEpi {
    uint16_t* z = nullptr;
    uint32_t lbar = 0;
    int first = 0;
    float scale = 1.0f;
};

template <Epi E, int F = kI8, int S = kDStages>
__device__ __forceinline__ void gemm_tile(uint32_t m, uint32_t mu, int64_t k_pad, int64_t n_pad,
                                          const int8_t* __restrict__ gA,
                                          const int8_t* __restrict__ gB, uint8_t* __restrict__ gZ,
                                          int32_t* __restrict__ gmax_a,
                                          int32_t* __restrict__ gmax_b, int tm, int tn,
                                          int8_t* lds, FpEpi fe = FpEpi{}) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wi = wave >> 1;
    const int wj = wave & 1;
    static_assert(S >= 4 && S <= kDStagesMax, "ring depth");
    auto ring = [](int t) {
        if constexpr ((S & (S - 1)) == 0)
            return t & (S - 1);
        else
            return (int)((unsigned)t % (unsigned)S);
    };

    // Bytes of a row of one K step (48 for packed FP6, else 64), of one
    // operand's block of a step, and 1 KB wave loads per wave per step.
    constexpr int kRowB = (F == kF6) ? kF6StepBytes : kDBK;
    constexpr int kOpB = kPlaneRows * kRowB;
    constexpr int kPerSide = kOpB / 1024;
    constexpr int kLoads = 2 * kPerSide / 4;
    static_assert(kLoads * 4 * 1024 == 2 * kOpB, "load split");
    // Loads: wave-load R = wave * kLoads + p copies kilobyte R % kPerSide of
    // operand R / kPerSide's block for the step; lane L moves bytes
    // [16 L, 16 L + 16).
    // The LDS destination of a wave-level load is uniform: its offsets are
    // made scalar once, outside the K loop, so each load's M0 comes from
    // scalar arithmetic only.
    const int8_t* gsrc[kLoads];
    int lds_off[kLoads];
    const int wave_s = __builtin_amdgcn_readfirstlane(wave);
#pragma unroll
    for (int p = 0; p < kLoads; ++p) {
        const int R = wave_s * kLoads + p;
        const int side = R / kPerSide, rk = R % kPerSide;
        gsrc[p] = (side ? gB : gA) + rk * 1024 + lane * 16;
        lds_off[p] = side * kOpB + rk * 1024;
    }
    auto dma = [&](int t) {
        int8_t* stage = lds + ring(t) * kDStage;
#pragma unroll
        for (int p = 0; p < kLoads; ++p)
            __builtin_amdgcn_global_load_lds(
                (const void*)(gsrc[p] + (int64_t)t * kOpB),
                (lds_ptr_t)(stage + lds_off[p]), 16, 0, 0);
    };

    using Acc = std::conditional_t<F == kI8, v16i, v16f>;
    Acc acc[kFM][kFN];
#pragma unroll
    for (int a = 0; a < kFM; ++a)
#pragma unroll
        for (int b = 0; b < kFN; ++b) acc[a][b] = (Acc){0};

    // Fragment reads: row (lane & 31) of a 32-row block; logical chunk
    // 2 * kk + (lane >> 5), stored at its xor with (row >> 2) & 3, which is
    // (lane & 15) >> 2 because the block rows start at multiples of 16.
    const int fr = lane & 31;
    const int fsw = (lane & 15) >> 2;
    const int offA = (wi * kWaveM + fr) * kDBK;
    const int offB = kBM * kDBK + (wj * kWaveN + fr) * kDBK;
    const int cofs0 = ((0 + (lane >> 5)) ^ fsw) * 16;
    const int cofs1 = ((2 + (lane >> 5)) ^ fsw) * 16;
    const int nk = (int)(k_pad / kRowB);
    const int pre = nk < S - 1 ? nk : S - 1;
    // waits: at the end of step t stage t + 2 must be in LDS; the loads of
    // the stages issued after it may stay in flight
    auto wait_prologue = [&]() {
        if (pre >= 4)
            __builtin_amdgcn_s_waitcnt(OZ_WAITCNT(2 * kLoads, 0));
        else if (pre == 3)
            __builtin_amdgcn_s_waitcnt(OZ_WAITCNT(kLoads, 0));
        else
            __builtin_amdgcn_s_waitcnt(OZ_WAITCNT(0, 0));
    };
    auto wait_stages = [&](auto n_tag) {
        constexpr int n = decltype(n_tag)::value;
        __builtin_amdgcn_s_waitcnt(OZ_WAITCNT(n * kLoads, 0));
    };
    using w0 = std::integral_constant<int, 0>;
    using w1 = std::integral_constant<int, 1>;
    using wL = std::integral_constant<int, S - 3>;
    using yes = std::integral_constant<bool, true>;
    using no = std::integral_constant<bool, false>;

    if constexpr (F != kF8 && F != kF6) {
    v4i xa[2][kFN], yb[2][kFM];
    auto read_frags = [&](int buf, int t, int kk) {
        const int8_t* stage = lds + ring(t) * kDStage;
        const int c = kk ? cofs1 : cofs0;
#pragma unroll
        for (int b = 0; b < kFN; ++b)
            xa[buf][b] = *reinterpret_cast<const v4i*>(stage + offB + b * 32 * kDBK + c);
#pragma unroll
        for (int a = 0; a < kFM; ++a)
            yb[buf][a] = *reinterpret_cast<const v4i*>(stage + offA + a * 32 * kDBK + c);
    };
    auto mfma_slice = [&](int buf) {
#pragma unroll
        for (int a = 0; a < kFM; ++a)
#pragma unroll
            for (int b = 0; b < kFN; ++b) {
                if constexpr (F == kI8) {
                    acc[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(xa[buf][b], yb[buf][a],
                                                                      acc[a][b], 0, 0, 0);
                } else {
                    const v4i x = xa[buf][b], y = yb[buf][a];
                    const v8i x8 = {x[0], x[1], x[2], x[3], 0, 0, 0, 0};
                    const v8i y8 = {y[0], y[1], y[2], y[3], 0, 0, 0, 0};
                    acc[a][b] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                        x8, y8, acc[a][b], 4, 4, 0, 0, 0, 0);
                }
            }
    };

    for (int t = 0; t < pre; ++t) dma(t);
    // steps 0 and 1 in LDS (step 2 may stay in flight)
    wait_prologue();
    barrier_no_fence();
    read_frags(0, 0, 0);

    // One step: kLoad issues the loads of step t+3; kNext reads the first
    // operands of step t+1 during the second slice. Ends with the wait for
    // step t+2's loads and the barrier that publishes them.
    auto step = [&](int t, auto load_tag, auto next_tag, auto wait_tag) {
        constexpr bool kLoad = decltype(load_tag)::value;
        constexpr bool kNext = decltype(next_tag)::value;
        if constexpr (kLoad) dma(t + S - 1);
        read_frags(1, t, 1);
        mfma_slice(0);
        if constexpr (kLoad) {
#pragma unroll
            for (int i = 0; i < kLoads; ++i) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
                __builtin_amdgcn_sched_group_barrier(0x010, 1, 0);  // global load to LDS
            }
        }
#pragma unroll
        for (int i = 0; i < kFM + kFN; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // LDS read
        }
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (kNext) read_frags(0, t + 1, 0);
        mfma_slice(1);
        if constexpr (kNext) {
#pragma unroll
            for (int i = 0; i < kFM + kFN; ++i) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // LDS read
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        wait_stages(wait_tag);
        barrier_no_fence();
    };
    int t = 0;
    for (; t + S - 1 < nk; ++t) step(t, yes{}, yes{}, wL{});
    if (S == 5 && t + 4 == nk) {  // stage t + 3 = nk - 1 may stay in flight
        step(t, no{}, yes{}, w1{});
        ++t;
    }
    for (; t + 1 < nk; ++t) step(t, no{}, yes{}, w0{});
    step(t, no{}, no{}, w0{});
    } else {
    // FP8: a fragment is 32 bytes, logical chunks 2h and 2h + 1 (h = lane >> 5).
    // One register set per fragment: B fragment b of step t+1 is read as
    // soon as the four MFMAs of step t that use it have issued, the A
    // fragments after the last MFMA of the step.
    const int c8lo = ((2 * (lane >> 5)) ^ fsw) * 16;
    const int c8hi = ((2 * (lane >> 5) + 1) ^ fsw) * 16;
    // FP6 (packed): the 24 bytes of a lane's 32 codes are units 3h .. 3h + 2
    // of its row, unit u at position (u + rot) mod 6 (plane_offset6; the
    // rows of a 32-row block start at multiples of 32, so rot depends on
    // lane & 31 only); three 8-byte reads.
    const int f6rot = ((fr >> 3) ^ (fr >> 4)) & 1;
    const int u6 = 3 * (lane >> 5);
    const int p6a = ((u6 + f6rot) % 6) * 8, p6b = ((u6 + 1 + f6rot) % 6) * 8,
              p6c = ((u6 + 2 + f6rot) % 6) * 8;
    const int offA8 = (wi * kWaveM + fr) * kRowB;
    const int offB8 = kOpB + (wj * kWaveN + fr) * kRowB;
    v8i xa[kFN], yb[kFM];
    auto frag8 = [&](const int8_t* base) {
        if constexpr (F == kF6) {
            const v2i a = *reinterpret_cast<const v2i*>(base + p6a);
            const v2i b = *reinterpret_cast<const v2i*>(base + p6b);
            const v2i c = *reinterpret_cast<const v2i*>(base + p6c);
            return (v8i){a[0], a[1], b[0], b[1], c[0], c[1], 0, 0};
        } else {
            const v4i lo = *reinterpret_cast<const v4i*>(base + c8lo);
            const v4i hi = *reinterpret_cast<const v4i*>(base + c8hi);
            return (v8i){lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
        }
    };
    auto stage_of = [&](int t) { return lds + ring(t) * kDStage; };
    for (int t = 0; t < pre; ++t) dma(t);
    wait_prologue();
    barrier_no_fence();
#pragma unroll
    for (int b = 0; b < kFN; ++b) xa[b] = frag8(stage_of(0) + offB8 + b * 32 * kRowB);
#pragma unroll
    for (int a = 0; a < kFM; ++a) yb[a] = frag8(stage_of(0) + offA8 + a * 32 * kRowB);
    auto step8 = [&](int t, auto load_tag, auto next_tag, auto wait_tag) {
        constexpr bool kLoad = decltype(load_tag)::value;
        constexpr bool kNext = decltype(next_tag)::value;
        if constexpr (kLoad) dma(t + S - 1);
        const int8_t* nxt = stage_of(t + 1);
#pragma unroll
        for (int b = 0; b < kFN; ++b) {
#pragma unroll
            for (int a = 0; a < kFM; ++a)
                acc[a][b] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                    xa[b], yb[a], acc[a][b], mfma_fmt<F>(), mfma_fmt<F>(), 0, 0, 0, 0);
            if constexpr (kNext) xa[b] = frag8(nxt + offB8 + b * 32 * kRowB);
        }
        if constexpr (kNext) {
#pragma unroll
            for (int a = 0; a < kFM; ++a) yb[a] = frag8(nxt + offA8 + a * 32 * kRowB);
        }
        if constexpr (kLoad) {
#pragma unroll
            for (int i = 0; i < kLoads; ++i) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
                __builtin_amdgcn_sched_group_barrier(0x010, 1, 0);  // global load to LDS
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        wait_stages(wait_tag);
        barrier_no_fence();
    };
    int t = 0;
    for (; t + S - 1 < nk; ++t) step8(t, yes{}, yes{}, wL{});
    if (S == 5 && t + 4 == nk) {
        step8(t, no{}, yes{}, w1{});
        ++t;
    }
    for (; t + 1 < nk; ++t) step8(t, no{}, yes{}, w0{});
    step8(t, no{}, no{}, w0{});
    }

    const int li = lane & 31;
    const int lj = (lane >> 5) * 4;
    if constexpr (E == Epi::kRmw) {
        // two passes of 128 rows: the waves of that half stage
        // lbar (W mod m) as uint16 in LDS, then every thread adds its
        // 16-byte pieces into the residues with coalesced reads and writes
        uint8_t* sO = reinterpret_cast<uint8_t*>(lds);
        for (int half = 0; half < 2; ++half) {
            if (wi == half) {
#pragma unroll
                for (int a = 0; a < kFM; ++a)
#pragma unroll
                    for (int b = 0; b < kFN; ++b)
#pragma unroll
                        for (int g = 0; g < 4; ++g) {
                            uint32_t v[4];
#pragma unroll
                            for (int q = 0; q < 4; ++q) {
                                const int32_t w = (int32_t)(acc[a][b][4 * g + q] * fe.scale);
                                const uint32_t aw = (uint32_t)(w < 0 ? -w : w);
                                uint32_t r = barrett32(aw, m, mu);
                                if (w < 0 && r != 0) r = m - r;
                                v[q] = barrett32(fe.lbar * r, m, mu);
                            }
                            const int i = a * 32 + li;  // row inside this half
                            const int j = wj * kWaveN + b * 32 + 8 * g + lj;
                            *reinterpret_cast<uint2*>(sO + i * kOutRow16 + j * 2) =
                                make_uint2(v[0] | (v[1] << 16), v[2] | (v[3] << 16));
                        }
            }
            __syncthreads();
            uint16_t* zt = fe.z + (int64_t)(half * 128) * n_pad;
            for (int c = tid; c < 128 * (kBN / 8); c += kThreads) {
                const int row = c / (kBN / 8), col = (c % (kBN / 8)) * 8;
                const uint4 add = *reinterpret_cast<const uint4*>(sO + row * kOutRow16 + col * 2);
                uint4* dst = reinterpret_cast<uint4*>(zt + (int64_t)row * n_pad + col);
                if (fe.first) {
                    *dst = add;
                } else {
                    const uint4 old = *dst;
                    const uint32_t* pa = reinterpret_cast<const uint32_t*>(&add);
                    const uint32_t* po = reinterpret_cast<const uint32_t*>(&old);
                    uint32_t o[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        uint32_t lo = (pa[q] & 0xFFFFu) + (po[q] & 0xFFFFu);
                        uint32_t hi = (pa[q] >> 16) + (po[q] >> 16);
                        lo -= (lo >= m) ? m : 0u;
                        hi -= (hi >= m) ? m : 0u;
                        o[q] = lo | (hi << 16);
                    }
                    *dst = make_uint4(o[0], o[1], o[2], o[3]);
                }
            }
            __syncthreads();
        }
    } else if constexpr (E == Epi::kMod) {
        uint8_t* sO = reinterpret_cast<uint8_t*>(lds);
        // w mod m in [0, m) for any INT32 w. x = fma(w, rcp64, 1.5 2^52)
        // (rcp64 = 1/m in FP64, w rcp64 within 2^-22 / m of w / m) holds
        // 1.5 2^52 + q, q a nearest integer to w / m, in its low mantissa
        // bits: its low 32 bits are q in two's complement. One 24-bit
        // multiply-add w + q24 (2^16 - m) (q24 = the low 24 bits of q) has
        // the low 16 bits of r = w - q m in [-m/2, m/2]. Pairs of r then take
        // two unsigned-min steps in packed 16-bit arithmetic into [0, m).
        // Checked on the CPU for every m <= 256 on the INT32 extremes and a
        // sample of w.
        const double rcp64 = 1.0 / (double)m;
        const uint32_t negm16 = 65536u - m;
        using u16x2 = unsigned short __attribute__((ext_vector_type(2)));
        const u16x2 m2 = {(unsigned short)m, (unsigned short)m};
        auto r16 = [&](int32_t w) -> uint32_t {
            const double x = __builtin_fma((double)w, rcp64, 6755399441055744.0);
            const uint32_t q = (uint32_t)__builtin_bit_cast(uint64_t, x);
            return __umul24(q, negm16) + (uint32_t)w;
        };
        auto fix2 = [&](uint32_t lo, uint32_t hi) -> u16x2 {
            u16x2 v = __builtin_bit_cast(u16x2, __builtin_amdgcn_perm(hi, lo, 0x05040100u));
            v = __builtin_elementwise_min(v, v + m2);
            return __builtin_elementwise_min(v, v - m2);
        };
#pragma unroll
        for (int a = 0; a < kFM; ++a) {
#pragma unroll
            for (int b = 0; b < kFN; ++b) {
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const int32_t* w = reinterpret_cast<const int32_t*>(&acc[a][b]) + 4 * g;
                    const u16x2 v01 = fix2(r16(w[0]), r16(w[1]));
                    const u16x2 v23 = fix2(r16(w[2]), r16(w[3]));
                    const uint32_t packed = __builtin_amdgcn_perm(
                        __builtin_bit_cast(uint32_t, v23), __builtin_bit_cast(uint32_t, v01), 0x06040200u);
                    const int i = wi * kWaveM + a * 32 + li;
                    const int j = wj * kWaveN + b * 32 + 8 * g + lj;
                    *reinterpret_cast<uint32_t*>(sO + i * kOutRow + j) = packed;
                }
            }
        }
        __syncthreads();
#pragma unroll 4
        for (int c = tid; c < kBM * (kBN / 8); c += kThreads) {
            const int row = c / (kBN / 8), col = (c % (kBN / 8)) * 8;
            const uint2 v = *reinterpret_cast<const uint2*>(sO + row * kOutRow + col);
            *reinterpret_cast<uint2*>(gZ + (int64_t)row * n_pad + col) = v;
        }
    } else {
#pragma unroll
        for (int a = 0; a < kFM; ++a) {
            int32_t rmax = 0;
#pragma unroll
            for (int b = 0; b < kFN; ++b)
#pragma unroll
                for (int q = 0; q < 16; ++q) rmax = max(rmax, acc[a][b][q]);
            rmax = max(rmax, __shfl_xor(rmax, 32, 64));
            if (lane < 32) atomicMax(gmax_a + (int64_t)tm * kBM + wi * kWaveM + a * 32 + li, rmax);
        }
#pragma unroll
        for (int b = 0; b < kFN; ++b) {
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                int32_t cmax = 0;
#pragma unroll
                for (int a = 0; a < kFM; ++a) cmax = max(cmax, acc[a][b][q]);
#pragma unroll
                for (int off = 16; off > 0; off >>= 1) cmax = max(cmax, __shfl_xor(cmax, off, 64));
                if (li == 0) {
                    const int j = wj * kWaveN + b * 32 + 8 * (q / 4) + lj + (q % 4);
                    atomicMax(gmax_b + (int64_t)tn * kBN + j, cmax);
                }
            }
        }
    }
}

template <Epi E>
__global__ __launch_bounds__(kThreads) void residue_gemm_kernel(ModConsts mc, int tiles_m, int tiles_n,
                                                             int64_t k_pad, int64_t plane_a,
                                                             int64_t plane_b, int64_t plane_z,
                                                             int64_t n_pad,
                                                             const int8_t* __restrict__ RA,
                                                             const int8_t* __restrict__ RB,
                                                             uint8_t* __restrict__ Z,
                                                             int32_t* __restrict__ gmax_a,
                                                             int32_t* __restrict__ gmax_b) {
    __shared__ __align__(1024) int8_t lds[kDStages * kDStage];
    int l, tm, tn;
    tile_of(blockIdx.x, tiles_m, tiles_n, l, tm, tn);
    const int8_t* gA = RA + (int64_t)l * plane_a + (int64_t)tm * kBM * k_pad;
    const int8_t* gB = RB + (int64_t)l * plane_b + (int64_t)tn * kBN * k_pad;
    uint8_t* gZ = (E == Epi::kMod)
                      ? Z + (int64_t)l * plane_z + (int64_t)tm * kBM * n_pad + (int64_t)tn * kBN
                      : nullptr;
    gemm_tile<E, kI8, kDStages>(E == Epi::kMod ? mc.m[l] : 0u, E == Epi::kMod ? mc.mu[l] : 0u,
                                   k_pad, n_pad, gA, gB, gZ, gmax_a, gmax_b, tm, tn, lds);
}

// Float-channel products of one plane round over one slab: work item b
// is a tile of channel item c (start[c] <= b < start[c + 1]), A plane
// plane[c] times B plane plane[c] over K bytes [kb_begin, kb_begin + kb_len),
// epilogue into the residues of channel chan[c] with weight lbar[c].
template <int F>
__global__ __launch_bounds__(kThreads) void fp_gemm_kernel(FpGemmArgs g) {
    __shared__ __align__(1024) int8_t lds[kDStages * kDStage];
    const int64_t bid = blockIdx.x;
    int c = 0;
    while (c + 1 < g.count && bid >= g.start[c + 1]) ++c;
    const int tiles_m = (int)(g.m_pad / kBM), tiles_n = (int)(g.n_pad / kBN);
    const int64_t T = (int64_t)tiles_m * tiles_n;
    const int64_t local = bid - g.start[c];
    // XCD-aware: workgroup b runs on XCD b % 8; give each XCD a contiguous
    // eighth of the channel's tiles in band order when the start allows
    int64_t t = local;
    if ((T & 7) == 0 && (g.start[c] & 7) == 0) t = (local & 7) * (T >> 3) + (local >> 3);
    int tm, tn;
    band_tile(t, tiles_m, tiles_n, tm, tn);
    const int64_t pl = g.plane[c];
    const int8_t* gA = g.pa + pl * g.m_pad * g.kb_pad + (int64_t)tm * kBM * g.kb_pad +
                       g.kb_begin * kPlaneRows;
    const int8_t* gB = g.pb + pl * g.n_pad * g.kb_pad + (int64_t)tn * kBN * g.kb_pad +
                       g.kb_begin * kPlaneRows;
    FpEpi fe;
    fe.z = g.z + (int64_t)g.chan[c] * g.m_pad * g.n_pad + (int64_t)tm * kBM * g.n_pad +
           (int64_t)tn * kBN;
    fe.lbar = g.lbar[c];
    fe.first = g.first;
    fe.scale = g.scale;
    gemm_tile<Epi::kRmw, F, kDStages>(g.m[c], g.mu[c], g.kb_len, g.n_pad, gA, gB, nullptr,
                                         nullptr, nullptr, tm, tn, lds, fe);
}

// Grouped residue GEMM, persistent: workgroup b starts on the list of its
// XCD (b % 8, the hardware's round-robin placement) and takes work items
// (problem, modulus, tile) from that list's counter; when it is exhausted
// it helps the other XCDs' lists in turn. An XCD's list holds whole moduli
// of each problem (every tile, in band order), so its workgroups share the
// operand strips of one modulus in their L2. Every wave of a workgroup sees
// the same item, so all waves leave the loops together.
__global__ __launch_bounds__(kThreads) void group_gemm_kernel(GroupArgs g) {
    __shared__ __align__(1024) int8_t lds[kDStages * kDStage];
    __shared__ int32_t next;
    const int x0 = blockIdx.x & (kXcds - 1);
    for (int d = 0; d < kXcds; ++d) {
        const int x = (x0 + d) & (kXcds - 1);
        const int32_t* pre = g.prefix + (kGTiles + x) * (g.count + 1);
        const int32_t total = pre[g.count];
        if (threadIdx.x == 0) next = atomicAdd(g.counter + x, 1);
        __syncthreads();
        int32_t w = __builtin_amdgcn_readfirstlane(next);
        __syncthreads();
        // The problem of the previous item, kept while the items stay in it
        // (they come in runs of whole moduli), so that most items need no
        // table reads before their tile starts.
        int q = -1, first = 0, tiles_m = 1, tiles_n = 1;
        int32_t qlo = 0, qhi = 0, T = 1;
        int64_t m_pad = 0, n_pad = 0, k_pad = 0;
        const int8_t* pa = nullptr;
        const int8_t* pb = nullptr;
        uint8_t* pz = nullptr;
        const ModConsts* mc = nullptr;
        while (w < total) {
            if (q < 0 || w >= qhi) {
                q = group_find(pre, g.count, w);
                qlo = pre[q];
                qhi = pre[q + 1];
                const GProblem& P = g.probs[g.order[q]];
                m_pad = P.m_pad;
                n_pad = P.n_pad;
                k_pad = P.k_pad;
                tiles_m = (int)(m_pad / kBM);
                tiles_n = (int)(n_pad / kBN);
                T = tiles_m * tiles_n;
                pa = reinterpret_cast<const int8_t*>(g.ws + P.off_pa);
                pb = reinterpret_cast<const int8_t*>(g.ws + P.off_pb);
                pz = reinterpret_cast<uint8_t*>(g.ws + P.off_z);
                mc = g.mods + P.plan;
                int cnt;
                xcd_moduli(mc->n, x, q, first, cnt);
            }
            // the next item's index is fetched while this one runs
            int32_t nxt = 0;
            if (threadIdx.x == 0) nxt = atomicAdd(g.counter + x, 1);
            const int32_t local = w - qlo;  // < cnt * T
            const int l = first + kXcds * (local / T);
            int tm, tn;
            band_tile(local % T, tiles_m, tiles_n, tm, tn);
            const int8_t* gA = pa + (int64_t)l * m_pad * k_pad + (int64_t)tm * kBM * k_pad;
            const int8_t* gB = pb + (int64_t)l * n_pad * k_pad + (int64_t)tn * kBN * k_pad;
            uint8_t* gZ = pz + (int64_t)l * m_pad * n_pad + (int64_t)tm * kBM * n_pad +
                          (int64_t)tn * kBN;
            gemm_tile<Epi::kMod>(mc->m[l], mc->mu[l], k_pad, n_pad, gA, gB, gZ, nullptr, nullptr,
                                 tm, tn, lds);
            if (threadIdx.x == 0) next = nxt;
            __syncthreads();
            w = __builtin_amdgcn_readfirstlane(next);
            __syncthreads();
        }
    }
}

}  // namespace

hipError_t launch_group_gemm(hipStream_t st, const GroupArgs& g, const int32_t* tiles_per_xcd,
                             int32_t workers) {
    int64_t tiles = 0;
    for (int x = 0; x < kXcds; ++x) tiles += tiles_per_xcd[x];
    if (tiles <= 0) return hipSuccess;
    const int32_t grid = workers < tiles ? workers : (int32_t)tiles;
    group_gemm_kernel<<<dim3((unsigned)grid), dim3(kThreads), 0, st>>>(g);
    return hipGetLastError();
}

hipError_t launch_fp_gemm(hipStream_t st, const FpGemmArgs& g, int fmt) {
    const int64_t blocks = g.start[g.count];
    if (blocks <= 0) return hipSuccess;
    if (fmt == 4)
        fp_gemm_kernel<kF4><<<dim3((unsigned)blocks), dim3(kThreads), 0, st>>>(g);
    else if (fmt == 2)
        fp_gemm_kernel<kF6><<<dim3((unsigned)blocks), dim3(kThreads), 0, st>>>(g);
    else
        fp_gemm_kernel<kF8><<<dim3((unsigned)blocks), dim3(kThreads), 0, st>>>(g);
    return hipGetLastError();
}

hipError_t launch_residue_gemm(hipStream_t st, const ModConsts& mc, int64_t m_pad, int64_t n_pad,
                               int64_t k_pad, const int8_t* planes_a, const int8_t* planes_b,
                               uint8_t* residues) {
    if (m_pad <= 0 || n_pad <= 0) return hipSuccess;
    const int tiles_m = (int)(m_pad / kBM), tiles_n = (int)(n_pad / kBN);
    const int64_t blocks = (int64_t)tiles_m * tiles_n * mc.n;
    residue_gemm_kernel<Epi::kMod><<<dim3((unsigned)blocks), dim3(kThreads), 0, st>>>(
        mc, tiles_m, tiles_n, k_pad, m_pad * k_pad, n_pad * k_pad, m_pad * n_pad, n_pad, planes_a,
        planes_b, residues, nullptr, nullptr);
    return hipGetLastError();
}

hipError_t launch_bound_gemm(hipStream_t st, int64_t m_pad, int64_t n_pad, int64_t k_pad,
                             const int8_t* bar_a, const int8_t* bar_b, int32_t* gmax_a,
                             int32_t* gmax_b) {
    if (m_pad <= 0 || n_pad <= 0) return hipSuccess;
    hipError_t e = launch_fill_i32(st, m_pad, 0, gmax_a);
    if (e == hipSuccess) e = launch_fill_i32(st, n_pad, 0, gmax_b);
    if (e != hipSuccess) return e;
    ModConsts one{};
    one.n = 1;
    const int tiles_m = (int)(m_pad / kBM), tiles_n = (int)(n_pad / kBN);
    const int64_t blocks = (int64_t)tiles_m * tiles_n;
    residue_gemm_kernel<Epi::kMax><<<dim3((unsigned)blocks), dim3(kThreads), 0, st>>>(
        one, tiles_m, tiles_n, k_pad, 0, 0, 0, n_pad, bar_a, bar_b, nullptr, gmax_a, gmax_b);
    return hipGetLastError();
}

}  // namespace ozemu
