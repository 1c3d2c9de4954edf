// Residue GEMMs with the fused epilogue (Sec. V-A phases 3-4, Sec. V-C):
// for every modulus m_l, W = R_A[l] R_B[l]^T in exact INT32 on the gfx950
// INT8 matrix cores (v_mfma_i32_32x32x32_i8), then Z = W mod m_l in [0, m_l)
// stored as uint8. One launch covers all moduli and output tiles.
//
// Exactness: |W| <= k floor(m/2)^2 <= 2^31 - 1 is checked by the host before
// launch (eq. "ov-accgen"), so INT32 accumulation never wraps, in any order.
//
// Tiling: 256 x 256 output tile per workgroup of 4 waves (2 x 2), each wave
// 128 x 128 as 4 x 4 MFMA blocks of 32 x 32 with INT32 accumulators. K is
// staged through LDS in steps of kBK bytes, double-buffered: the global
// loads of step t+1 are in flight while step t's MFMAs run. Rows in LDS are
// padded by 16 bytes so the 16-byte fragment reads of 16 consecutive rows
// fall in distinct banks. The MFMA's first operand takes the B-plane rows
// (output columns j) and its second the A-plane rows (output rows i), so
// each lane ends with 4 consecutive j of one i and the epilogue packs them.
//
// The same kernel with a max epilogue serves the bound-adaptive scaling
// mode: it computes Gbar = abar bbar^T and reduces row and column maxima.
#include "ozemu_internal.hpp"

namespace ozemu {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kThreads = 256;
constexpr int kBM = kTileM;  // rows i per tile
constexpr int kBN = kTileN;  // columns j per tile
constexpr int kBK = 64;       // K bytes per stage (variant 0)
constexpr int kRowBytes = kBK + 16;
constexpr int kStageBytes = (kBM + kBN) * kRowBytes;
constexpr int kWaveM = 128, kWaveN = 128;
constexpr int kFM = kWaveM / 32, kFN = kWaveN / 32;  // MFMA blocks per wave
constexpr int kChunksPerRow = kBK / 16;
constexpr int kLoadsA = kBM * kChunksPerRow / kThreads;  // 16-byte loads per thread
constexpr int kLoadsB = kBN * kChunksPerRow / kThreads;
constexpr int kGroup = 8;  // tile rows per band of the tile order

static_assert(kLoadsA * kThreads == kBM * kChunksPerRow, "A tile load split");
static_assert(kLoadsB * kThreads == kBN * kChunksPerRow, "B tile load split");

// Output staging for the residue epilogue reuses the operand LDS. Row stride
// of 66 dwords: the 32 rows a store instruction touches land on even banks
// and the two lane halves on even/odd banks.
constexpr int kOutRow = 264;
static_assert(kBM * kOutRow <= 2 * kStageBytes, "output staging fits");

enum class Epi { kMod, kMax };

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
    const int64_t in_group = (int64_t)kGroup * tiles_n;
    const int first_m = (int)(t / in_group) * kGroup;
    const int gsize = min(tiles_m - first_m, kGroup);
    const int64_t r = t % in_group;
    tm = first_m + (int)(r % gsize);
    tn = (int)(r / gsize);
}

template <Epi E>
__global__ __launch_bounds__(kThreads) void residue_gemm_kernel(ModConsts mc, int tiles_m,
                                                                int tiles_n, int64_t k_pad,
                                                                int64_t plane_a, int64_t plane_b,
                                                                int64_t plane_z, int64_t n_pad,
                                                                const int8_t* __restrict__ RA,
                                                                const int8_t* __restrict__ RB,
                                                                uint8_t* __restrict__ Z,
                                                                int32_t* __restrict__ gmax_a,
                                                                int32_t* __restrict__ gmax_b) {
    __shared__ __align__(16) int8_t lds[2 * kStageBytes];
    int l, tm, tn;
    tile_of(blockIdx.x, tiles_m, tiles_n, l, tm, tn);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wi = wave >> 1;  // wave row (i)
    const int wj = wave & 1;   // wave column (j)

    const int8_t* gA = RA + (int64_t)l * plane_a + (int64_t)tm * kBM * k_pad;
    const int8_t* gB = RB + (int64_t)l * plane_b + (int64_t)tn * kBN * k_pad;

    // global -> register staging for one K step
    v4i ra[kLoadsA], rb[kLoadsB];
    auto gload = [&](int64_t k0) {
#pragma unroll
        for (int p = 0; p < kLoadsA; ++p) {
            const int c = tid + p * kThreads;
            const int row = c / kChunksPerRow, col = c % kChunksPerRow;
            ra[p] = *reinterpret_cast<const v4i*>(gA + (int64_t)row * k_pad + k0 + col * 16);
        }
#pragma unroll
        for (int p = 0; p < kLoadsB; ++p) {
            const int c = tid + p * kThreads;
            const int row = c / kChunksPerRow, col = c % kChunksPerRow;
            rb[p] = *reinterpret_cast<const v4i*>(gB + (int64_t)row * k_pad + k0 + col * 16);
        }
    };
    auto sstore = [&](int buf) {
        int8_t* sA = lds + buf * kStageBytes;
        int8_t* sB = sA + kBM * kRowBytes;
#pragma unroll
        for (int p = 0; p < kLoadsA; ++p) {
            const int c = tid + p * kThreads;
            const int row = c / kChunksPerRow, col = c % kChunksPerRow;
            *reinterpret_cast<v4i*>(sA + row * kRowBytes + col * 16) = ra[p];
        }
#pragma unroll
        for (int p = 0; p < kLoadsB; ++p) {
            const int c = tid + p * kThreads;
            const int row = c / kChunksPerRow, col = c % kChunksPerRow;
            *reinterpret_cast<v4i*>(sB + row * kRowBytes + col * 16) = rb[p];
        }
    };

    v16i acc[kFM][kFN];
#pragma unroll
    for (int a = 0; a < kFM; ++a)
#pragma unroll
        for (int b = 0; b < kFN; ++b) acc[a][b] = (v16i){0};

    const int nk = (int)(k_pad / kBK);
    gload(0);
    sstore(0);
    __syncthreads();
    const int frag_row = lane & 31;
    const int frag_k = (lane >> 5) * 16;
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) gload((int64_t)(kt + 1) * kBK);
        const int8_t* sA = lds + cur * kStageBytes;
        const int8_t* sB = sA + kBM * kRowBytes;
#pragma unroll
        for (int kk = 0; kk < kBK; kk += 32) {
            v4i xa[kFN], yb[kFM];
#pragma unroll
            for (int b = 0; b < kFN; ++b)
                xa[b] = *reinterpret_cast<const v4i*>(
                    sB + (wj * kWaveN + b * 32 + frag_row) * kRowBytes + kk + frag_k);
#pragma unroll
            for (int a = 0; a < kFM; ++a)
                yb[a] = *reinterpret_cast<const v4i*>(
                    sA + (wi * kWaveM + a * 32 + frag_row) * kRowBytes + kk + frag_k);
#pragma unroll
            for (int a = 0; a < kFM; ++a)
#pragma unroll
                for (int b = 0; b < kFN; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(xa[b], yb[a], acc[a][b], 0, 0, 0);
        }
        if (kt + 1 < nk) sstore(cur ^ 1);
        __syncthreads();
    }

    // acc[a][b][q] holds W[i][j] with i = tile row wi*128 + a*32 + lane%32 and
    // j = wj*128 + b*32 + 8*(q/4) + 4*(lane/32) + q%4.
    const int li = lane & 31;
    const int lj = (lane >> 5) * 4;
    if constexpr (E == Epi::kMod) {
        const uint32_t m = mc.m[l], mu = mc.mu[l];
        uint8_t* sO = reinterpret_cast<uint8_t*>(lds);
#pragma unroll
        for (int a = 0; a < kFM; ++a) {
#pragma unroll
            for (int b = 0; b < kFN; ++b) {
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    uint32_t packed = 0;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int32_t w = acc[a][b][4 * g + q];
                        const uint32_t aw = (uint32_t)(w < 0 ? -w : w);
                        uint32_t r = barrett32(aw, m, mu);
                        if (w < 0 && r != 0) r = m - r;
                        packed |= r << (8 * q);
                    }
                    const int i = wi * kWaveM + a * 32 + li;
                    const int j = wj * kWaveN + b * 32 + 8 * g + lj;
                    *reinterpret_cast<uint32_t*>(sO + i * kOutRow + j) = packed;
                }
            }
        }
        __syncthreads();
        // 256 rows x 256 bytes: 8 bytes per lane, 32 lanes per row.
        uint8_t* gZ = Z + (int64_t)l * plane_z + (int64_t)tm * kBM * n_pad + (int64_t)tn * kBN;
#pragma unroll 4
        for (int c = tid; c < kBM * (kBN / 8); c += kThreads) {
            const int row = c / (kBN / 8), col = (c % (kBN / 8)) * 8;
            const uint2 v = *reinterpret_cast<const uint2*>(sO + row * kOutRow + col);
            *reinterpret_cast<uint2*>(gZ + (int64_t)row * n_pad + col) = v;
        }
    } else {
        // Row maxima over this tile's columns and column maxima over its rows.
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


// Pipelined variant: K steps of 128 bytes, two LDS stages and one register
// stage, so the global loads of step t+2 and the LDS stores of step t+1
// overlap the MFMAs of step t; MFMA fragments are double-buffered inside a
// step. The loop is peeled so the steady-state body has no branches.
constexpr int kPBK = 128;
constexpr int kPRow = kPBK + 16;  // 36 dwords: 16 consecutive rows hit distinct banks
constexpr int kPStage = (kBM + kBN) * kPRow;
constexpr int kPChunks = kPBK / 16;
constexpr int kPLoadsA = kBM * kPChunks / kThreads;
constexpr int kPLoadsB = kBN * kPChunks / kThreads;
static_assert(kBM * kOutRow <= 2 * kPStage, "output staging fits");

template <Epi E>
__global__ __launch_bounds__(kThreads) void residue_gemm_pipelined(ModConsts mc, int tiles_m,
                                                                   int tiles_n, int64_t k_pad,
                                                                   int64_t plane_a, int64_t plane_b,
                                                                   int64_t plane_z, int64_t n_pad,
                                                                   const int8_t* __restrict__ RA,
                                                                   const int8_t* __restrict__ RB,
                                                                   uint8_t* __restrict__ Z,
                                                                   int32_t* __restrict__ gmax_a,
                                                                   int32_t* __restrict__ gmax_b) {
    __shared__ __align__(16) int8_t lds[2 * kPStage];
    int l, tm, tn;
    tile_of(blockIdx.x, tiles_m, tiles_n, l, tm, tn);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wi = wave >> 1;
    const int wj = wave & 1;
    const int8_t* gA = RA + (int64_t)l * plane_a + (int64_t)tm * kBM * k_pad;
    const int8_t* gB = RB + (int64_t)l * plane_b + (int64_t)tn * kBN * k_pad;

    v4i ra[kPLoadsA], rb[kPLoadsB];
    auto gload = [&](int64_t k0) {
#pragma unroll
        for (int p = 0; p < kPLoadsA; ++p) {
            const int c = tid + p * kThreads;
            ra[p] = *reinterpret_cast<const v4i*>(gA + (int64_t)(c / kPChunks) * k_pad + k0 +
                                                  (c % kPChunks) * 16);
        }
#pragma unroll
        for (int p = 0; p < kPLoadsB; ++p) {
            const int c = tid + p * kThreads;
            rb[p] = *reinterpret_cast<const v4i*>(gB + (int64_t)(c / kPChunks) * k_pad + k0 +
                                                  (c % kPChunks) * 16);
        }
    };
    auto sstore = [&](int buf) {
        int8_t* sA = lds + buf * kPStage;
        int8_t* sB = sA + kBM * kPRow;
#pragma unroll
        for (int p = 0; p < kPLoadsA; ++p) {
            const int c = tid + p * kThreads;
            *reinterpret_cast<v4i*>(sA + (c / kPChunks) * kPRow + (c % kPChunks) * 16) = ra[p];
        }
#pragma unroll
        for (int p = 0; p < kPLoadsB; ++p) {
            const int c = tid + p * kThreads;
            *reinterpret_cast<v4i*>(sB + (c / kPChunks) * kPRow + (c % kPChunks) * 16) = rb[p];
        }
    };

    v16i acc[kFM][kFN];
#pragma unroll
    for (int a = 0; a < kFM; ++a)
#pragma unroll
        for (int b = 0; b < kFN; ++b) acc[a][b] = (v16i){0};

    const int frag_row = lane & 31;
    const int frag_k = (lane >> 5) * 16;
    const int offB = (wj * kWaveN + frag_row) * kPRow + frag_k;
    const int offA = (wi * kWaveM + frag_row) * kPRow + frag_k;

    // One K step from LDS stage `cur`; optionally stores the register stage
    // into the other LDS stage and refills the registers from global memory.
    auto step = [&](int cur, bool store_next, bool load_next2, int64_t k_next2) {
        const int8_t* sA = lds + cur * kPStage;
        const int8_t* sB = sA + kBM * kPRow;
        v4i xa[2][kFN], yb[2][kFM];
#pragma unroll
        for (int b = 0; b < kFN; ++b)
            xa[0][b] = *reinterpret_cast<const v4i*>(sB + offB + b * 32 * kPRow);
#pragma unroll
        for (int a = 0; a < kFM; ++a)
            yb[0][a] = *reinterpret_cast<const v4i*>(sA + offA + a * 32 * kPRow);
#pragma unroll
        for (int kk = 0; kk < kPBK / 32; ++kk) {
            const int f = kk & 1;
            if (kk + 1 < kPBK / 32) {
#pragma unroll
                for (int b = 0; b < kFN; ++b)
                    xa[f ^ 1][b] = *reinterpret_cast<const v4i*>(sB + offB + b * 32 * kPRow +
                                                                 (kk + 1) * 32);
#pragma unroll
                for (int a = 0; a < kFM; ++a)
                    yb[f ^ 1][a] = *reinterpret_cast<const v4i*>(sA + offA + a * 32 * kPRow +
                                                                 (kk + 1) * 32);
            }
            if (kk == 1 && store_next) sstore(cur ^ 1);
            if (kk == 2 && load_next2) gload(k_next2);
#pragma unroll
            for (int a = 0; a < kFM; ++a)
#pragma unroll
                for (int b = 0; b < kFN; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(xa[f][b], yb[f][a], acc[a][b],
                                                                      0, 0, 0);
        }
        __syncthreads();
    };

    const int nk = (int)(k_pad / kPBK);
    gload(0);
    sstore(0);
    if (nk > 1) gload(kPBK);
    __syncthreads();
    int kt = 0;
    for (; kt + 2 < nk; ++kt) step(kt & 1, true, true, (int64_t)(kt + 2) * kPBK);
    if (kt + 1 < nk) {
        step(kt & 1, true, false, 0);
        ++kt;
    }
    step(kt & 1, false, false, 0);

    const int li = lane & 31;
    const int lj = (lane >> 5) * 4;
    if constexpr (E == Epi::kMod) {
        const uint32_t m = mc.m[l], mu = mc.mu[l];
        uint8_t* sO = reinterpret_cast<uint8_t*>(lds);
#pragma unroll
        for (int a = 0; a < kFM; ++a) {
#pragma unroll
            for (int b = 0; b < kFN; ++b) {
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    uint32_t packed = 0;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int32_t w = acc[a][b][4 * g + q];
                        const uint32_t aw = (uint32_t)(w < 0 ? -w : w);
                        uint32_t r = barrett32(aw, m, mu);
                        if (w < 0 && r != 0) r = m - r;
                        packed |= r << (8 * q);
                    }
                    const int i = wi * kWaveM + a * 32 + li;
                    const int j = wj * kWaveN + b * 32 + 8 * g + lj;
                    *reinterpret_cast<uint32_t*>(sO + i * kOutRow + j) = packed;
                }
            }
        }
        __syncthreads();
        uint8_t* gZ = Z + (int64_t)l * plane_z + (int64_t)tm * kBM * n_pad + (int64_t)tn * kBN;
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

}  // namespace

hipError_t launch_residue_gemm(hipStream_t st, const ModConsts& mc, int64_t m_pad, int64_t n_pad,
                               int64_t k_pad, const int8_t* planes_a, const int8_t* planes_b,
                               uint8_t* residues, int variant) {
    if (m_pad <= 0 || n_pad <= 0) return hipSuccess;
    const int tiles_m = (int)(m_pad / kBM), tiles_n = (int)(n_pad / kBN);
    const int64_t blocks = (int64_t)tiles_m * tiles_n * mc.n;
    if (variant == 1) {
        residue_gemm_pipelined<Epi::kMod><<<dim3((unsigned)blocks), dim3(kThreads), 0, st>>>(
            mc, tiles_m, tiles_n, k_pad, m_pad * k_pad, n_pad * k_pad, m_pad * n_pad, n_pad,
            planes_a, planes_b, residues, nullptr, nullptr);
    } else {
        residue_gemm_kernel<Epi::kMod><<<dim3((unsigned)blocks), dim3(kThreads), 0, st>>>(
            mc, tiles_m, tiles_n, k_pad, m_pad * k_pad, n_pad * k_pad, m_pad * n_pad, n_pad,
            planes_a, planes_b, residues, nullptr, nullptr);
    }
    return hipGetLastError();
}

hipError_t launch_bound_gemm(hipStream_t st, int64_t m_pad, int64_t n_pad, int64_t k_pad,
                             const int8_t* bar_a, const int8_t* bar_b, int32_t* gmax_a,
                             int32_t* gmax_b, int variant) {
    if (m_pad <= 0 || n_pad <= 0) return hipSuccess;
    hipError_t e = launch_fill_i32(st, m_pad, 0, gmax_a);
    if (e == hipSuccess) e = launch_fill_i32(st, n_pad, 0, gmax_b);
    if (e != hipSuccess) return e;
    ModConsts one{};
    one.n = 1;
    const int tiles_m = (int)(m_pad / kBM), tiles_n = (int)(n_pad / kBN);
    const int64_t blocks = (int64_t)tiles_m * tiles_n;
    if (variant == 1)
        residue_gemm_pipelined<Epi::kMax><<<dim3((unsigned)blocks), dim3(kThreads), 0, st>>>(
            one, tiles_m, tiles_n, k_pad, 0, 0, 0, n_pad, bar_a, bar_b, nullptr, gmax_a, gmax_b);
    else
        residue_gemm_kernel<Epi::kMax><<<dim3((unsigned)blocks), dim3(kThreads), 0, st>>>(
            one, tiles_m, tiles_n, k_pad, 0, 0, 0, n_pad, bar_a, bar_b, nullptr, gmax_a, gmax_b);
    return hipGetLastError();
}

}  // namespace ozemu
