// Scale phase (Sec. V-A phase 1; Sec. II-A): one exponent per row of A and
// per column of B. HBM-bound: every entry is read once, as its IEEE bits.
//
// The key of a row is the frexp exponent of its largest magnitude, which is
// the largest frexp exponent of its entries, so rows reduce with an integer
// max (kKeyZero for a zero row, kKeyNonFinite if a NaN or infinity occurs).
// Columns of the row-major B are reduced over slabs of rows with an atomic
// max on the key, so the launch fills the chip for any shape.
#include "ozemu_internal.hpp"

namespace ozemu {

namespace {

constexpr int kScaleThreads = 256;

__device__ __forceinline__ int32_t wave_max(int32_t v) {
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    return v;
}

// Key of x * 2^-fold: the frexp exponent drops by fold exactly; a fold
// holding the non-finite marker makes the entry non-finite.
template <bool kFold>
__device__ __forceinline__ int32_t folded_key(double x, const int32_t* fold, int64_t idx) {
    const int32_t key = entry_key(__double_as_longlong(x));
    if constexpr (!kFold) {
        return key;
    } else {
        const int32_t f = fold[idx];
        if (f == kShiftNonFinite) return kKeyNonFinite;
        return (key == kKeyZero || key == kKeyNonFinite) ? key : key - f;
    }
}

// Key of one row, computed by a whole workgroup; each thread strides the
// row with 16-byte loads. With kFold, entry h counts as A_ih * 2^-fold[h]
// (a power-of-two column scaling applied without rounding).
template <bool kFold>
__device__ __forceinline__ void scale_row_body(int64_t k, const double* row, const int32_t* fold,
                                               int32_t* key_out) {
    int32_t key = kKeyZero;
    const bool vec = ((reinterpret_cast<uintptr_t>(row) & 15) == 0);
    if (vec) {
        const int64_t k2 = k / 2;
        const double2* r2 = reinterpret_cast<const double2*>(row);
        for (int64_t h = threadIdx.x; h < k2; h += kScaleThreads) {
            double2 v = r2[h];
            key = max(key, folded_key<kFold>(v.x, fold, 2 * h));
            key = max(key, folded_key<kFold>(v.y, fold, 2 * h + 1));
        }
        if ((k & 1) && threadIdx.x == 0) key = max(key, folded_key<kFold>(row[k - 1], fold, k - 1));
    } else {
        for (int64_t h = threadIdx.x; h < k; h += kScaleThreads)
            key = max(key, folded_key<kFold>(row[h], fold, h));
    }
    key = wave_max(key);
    __shared__ int32_t part[kScaleThreads / 64];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = key;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t r = part[0];
        for (int w = 1; w < kScaleThreads / 64; ++w) r = max(r, part[w]);
        *key_out = r;
    }
}

// One workgroup per row.
template <bool kFold>
__global__ __launch_bounds__(kScaleThreads) void scale_rows_kernel(int64_t k, const double* A,
                                                                   int64_t lda, const int32_t* fold,
                                                                   int32_t* key_a) {
    const int64_t i = blockIdx.x;
    scale_row_body<kFold>(k, A + i * lda, fold, key_a + i);
}

constexpr int kColRows = 64;  // rows of B per workgroup slab

// Workgroup (bx, by) of the column scan: columns 256 bx .. + 255 over rows
// kColRows by .. + kColRows - 1; key_b pre-filled with kKeyZero. With
// kFold, entry (h, j) counts as B_hj * 2^-fold[h].
template <bool kFold>
__device__ __forceinline__ void scale_cols_body(int64_t k, int64_t n, const double* B, int64_t ldb,
                                                const int32_t* fold, int32_t* key_b, int64_t bx,
                                                int64_t by) {
    const int64_t j = bx * kScaleThreads + threadIdx.x;
    if (j >= n) return;
    const int64_t h0 = by * kColRows;
    const int64_t h1 = min(k, h0 + kColRows);
    int32_t key = kKeyZero;
    for (int64_t h = h0; h < h1; ++h) key = max(key, folded_key<kFold>(B[h * ldb + j], fold, h));
    if (key != kKeyZero) atomicMax(key_b + j, key);
}

// grid: (ceil(n / 256), ceil(k / kColRows)).
template <bool kFold>
__global__ __launch_bounds__(kScaleThreads) void scale_cols_kernel(int64_t k, int64_t n,
                                                                   const double* B, int64_t ldb,
                                                                   const int32_t* fold,
                                                                   int32_t* key_b) {
    scale_cols_body<kFold>(k, n, B, ldb, fold, key_b, blockIdx.x, blockIdx.y);
}

__global__ void fill_i32_kernel(int64_t count, int32_t value, int32_t* out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) out[i] = value;
}

// shift = beta - e for a nonzero row, 0 for a zero row, the non-finite
// marker otherwise.
__device__ __forceinline__ int32_t key_to_shift(int32_t key, int32_t beta) {
    if (key == kKeyNonFinite) return kShiftNonFinite;
    if (key == kKeyZero) return 0;
    return beta - key;
}

// beta is per entry when beta_per_entry is given.
__global__ void keys_to_shifts_kernel(int64_t count, int32_t* io, int beta,
                                      const int32_t* beta_per_entry) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    io[i] = key_to_shift(io[i], beta_per_entry ? beta_per_entry[i] : beta);
}

// Bound-adaptive mode: abar = ceil(|x| 2^(6 - e)) in [0, 64]. The scaling
// by a power of two is exact in FP64 unless it underflows to zero, which
// only happens for a nonzero x whose exact scaled value lies in (0, 1),
// whose ceiling is 1. Rows (A) and transposed columns (B) are written into
// zero-padded planes in the blocked order of the residue planes.
__device__ __forceinline__ int8_t bound_value(double x, int32_t key) {
    const double a = fabs(x);
    if (!(a > 0.0) || !isfinite(a) || key == kKeyNonFinite || key == kKeyZero) return 0;
    const double c = ceil(ldexp(a, 6 - key));
    return (int8_t)(c > 0.0 ? (int)c : 1);
}

__global__ void bound_planes_a_kernel(int64_t m, int64_t k, const double* A, int64_t lda,
                                      const int32_t* key_a, int64_t k_pad, int8_t* bar_a) {
    const int64_t i = blockIdx.x;
    const int64_t h = ((int64_t)blockIdx.y * blockDim.x + threadIdx.x);
    if (h >= k_pad) return;
    int8_t v = 0;
    if (i < m && h < k) v = bound_value(A[i * lda + h], key_a[i]);
    bar_a[plane_offset(i, h, k_pad)] = v;
}

// grid (ceil(n_pad/64), ceil(k_pad/64)); transpose through LDS.
__global__ __launch_bounds__(256) void bound_planes_b_kernel(int64_t k, int64_t n, const double* B,
                                                            int64_t ldb, const int32_t* key_b,
                                                            int64_t n_pad, int64_t k_pad,
                                                            int8_t* bar_b) {
    __shared__ int8_t tile[64][65];
    const int64_t j0 = (int64_t)blockIdx.x * 64, h0 = (int64_t)blockIdx.y * 64;
    const int tj = threadIdx.x & 63, th = threadIdx.x >> 6;
    for (int r = th; r < 64; r += 4) {
        int64_t h = h0 + r, j = j0 + tj;
        int8_t v = 0;
        if (h < k && j < n) v = bound_value(B[h * ldb + j], key_b[j]);
        tile[tj][r] = v;
    }
    __syncthreads();
    for (int r = th; r < 64; r += 4) {
        int64_t j = j0 + r, h = h0 + tj;
        if (j < n_pad && h < k_pad) bar_b[plane_offset(j, h, k_pad)] = tile[r][tj];
    }
}

// sigma = min(cap, floor((L + 12 - ceil(log2 gmax)) / 2)), cap when gmax = 0;
// the shift is sigma - e (0 for a zero row, the marker for a non-finite one).
__global__ void bound_shifts_kernel(int64_t count, const int32_t* key, const int32_t* gmax, int L,
                                    int32_t* shift) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    int32_t kk = key[i];
    int32_t g = gmax[i];
    int32_t sigma;
    if (g <= 0) {
        sigma = kBetaCap;
    } else {
        int c = (g == 1) ? 0 : 32 - __clz((uint32_t)(g - 1));
        int v = L + 12 - c;
        sigma = (v >= 0) ? v / 2 : -((-v + 1) / 2);
        if (sigma > kBetaCap) sigma = kBetaCap;
    }
    int32_t s;
    if (kk == kKeyNonFinite)
        s = kShiftNonFinite;
    else if (kk == kKeyZero)
        s = 0;
    else
        s = sigma - kk;
    shift[i] = s;
}

// ---- Grouped Scale ----

// Column keys of every problem pre-filled with kKeyZero (256 per
// workgroup); workgroup 0 also zeroes the GEMM work counters.
__global__ __launch_bounds__(kScaleThreads) void group_init_kernel(GroupArgs g, int32_t total) {
    if (blockIdx.x == 0 && threadIdx.x < kXcds) g.counter[threadIdx.x] = 0;
    if ((int32_t)blockIdx.x >= total) return;
    const int32_t* pre = g.prefix + kGColInit * (g.count + 1);
    const int p = group_find(pre, g.count, blockIdx.x);
    const GProblem& P = g.probs[p];
    const int64_t j = (int64_t)(blockIdx.x - pre[p]) * kScaleThreads + threadIdx.x;
    if (j < P.n) reinterpret_cast<int32_t*>(g.ws + P.off_sb)[j] = kKeyZero;
}

__global__ __launch_bounds__(kScaleThreads) void group_scale_rows_kernel(GroupArgs g) {
    const int32_t* pre = g.prefix + kGRows * (g.count + 1);
    const int p = group_find(pre, g.count, blockIdx.x);
    const GProblem& P = g.probs[p];
    const int64_t i = blockIdx.x - pre[p];
    scale_row_body<false>(P.k, P.A + i * P.lda, nullptr,
                          reinterpret_cast<int32_t*>(g.ws + P.off_sa) + i);
}

__global__ __launch_bounds__(kScaleThreads) void group_scale_cols_kernel(GroupArgs g) {
    const int32_t* pre = g.prefix + kGCols * (g.count + 1);
    const int p = group_find(pre, g.count, blockIdx.x);
    const GProblem& P = g.probs[p];
    const int64_t lb = blockIdx.x - pre[p];
    const int64_t gx = (P.n + kScaleThreads - 1) / kScaleThreads;
    scale_cols_body<false>(P.k, P.n, P.B, P.ldb, nullptr,
                           reinterpret_cast<int32_t*>(g.ws + P.off_sb), lb % gx, lb / gx);
}

// Keys to shifts: thread t < m handles row t, then the n columns.
__global__ __launch_bounds__(kScaleThreads) void group_shifts_kernel(GroupArgs g) {
    const int32_t* pre = g.prefix + kGShifts * (g.count + 1);
    const int p = group_find(pre, g.count, blockIdx.x);
    const GProblem& P = g.probs[p];
    const int64_t t = (int64_t)(blockIdx.x - pre[p]) * kScaleThreads + threadIdx.x;
    if (t < P.m) {
        int32_t* sa = reinterpret_cast<int32_t*>(g.ws + P.off_sa);
        sa[t] = key_to_shift(sa[t], P.beta_a);
    } else if (t < P.m + P.n) {
        int32_t* sb = reinterpret_cast<int32_t*>(g.ws + P.off_sb);
        sb[t - P.m] = key_to_shift(sb[t - P.m], P.beta_b);
    }
}

}  // namespace

hipError_t launch_group_init(hipStream_t st, const GroupArgs& g, int32_t total) {
    group_init_kernel<<<dim3((unsigned)(total > 0 ? total : 1)), dim3(kScaleThreads), 0, st>>>(g,
                                                                                              total);
    return hipGetLastError();
}

hipError_t launch_group_scale(hipStream_t st, const GroupArgs& g, int32_t rows, int32_t cols,
                              int32_t shifts) {
    if (rows > 0) group_scale_rows_kernel<<<dim3((unsigned)rows), dim3(kScaleThreads), 0, st>>>(g);
    if (cols > 0) group_scale_cols_kernel<<<dim3((unsigned)cols), dim3(kScaleThreads), 0, st>>>(g);
    if (shifts > 0) group_shifts_kernel<<<dim3((unsigned)shifts), dim3(kScaleThreads), 0, st>>>(g);
    return hipGetLastError();
}

hipError_t launch_scale_rows(hipStream_t st, int64_t m, int64_t k, const double* A, int64_t lda,
                             int32_t* key_a, const int32_t* fold) {
    if (m <= 0) return hipSuccess;
    if (fold)
        scale_rows_kernel<true><<<dim3((unsigned)m), dim3(kScaleThreads), 0, st>>>(k, A, lda, fold,
                                                                                   key_a);
    else
        scale_rows_kernel<false><<<dim3((unsigned)m), dim3(kScaleThreads), 0, st>>>(k, A, lda,
                                                                                    nullptr, key_a);
    return hipGetLastError();
}

hipError_t launch_fill_i32(hipStream_t st, int64_t count, int32_t value, int32_t* out) {
    if (count <= 0) return hipSuccess;
    fill_i32_kernel<<<dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st>>>(count, value, out);
    return hipGetLastError();
}

hipError_t launch_scale_cols(hipStream_t st, int64_t k, int64_t n, const double* B, int64_t ldb,
                             int32_t* key_b, const int32_t* fold) {
    if (n <= 0) return hipSuccess;
    hipError_t e = launch_fill_i32(st, n, kKeyZero, key_b);
    if (e != hipSuccess || k <= 0) return e;
    dim3 grid((unsigned)((n + kScaleThreads - 1) / kScaleThreads),
              (unsigned)((k + kColRows - 1) / kColRows));
    if (fold)
        scale_cols_kernel<true><<<grid, dim3(kScaleThreads), 0, st>>>(k, n, B, ldb, fold, key_b);
    else
        scale_cols_kernel<false><<<grid, dim3(kScaleThreads), 0, st>>>(k, n, B, ldb, nullptr, key_b);
    return hipGetLastError();
}

hipError_t launch_keys_to_shifts(hipStream_t st, int64_t count, int32_t* io, int beta,
                                 const int32_t* beta_per_entry) {
    if (count <= 0) return hipSuccess;
    keys_to_shifts_kernel<<<dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st>>>(
        count, io, beta, beta_per_entry);
    return hipGetLastError();
}

hipError_t launch_bound_planes_a(hipStream_t st, int64_t m, int64_t k, const double* A,
                                 int64_t lda, const int32_t* key_a, int64_t m_pad, int64_t k_pad,
                                 int8_t* bar_a) {
    dim3 grid((unsigned)m_pad, (unsigned)((k_pad + 255) / 256));
    bound_planes_a_kernel<<<grid, dim3(256), 0, st>>>(m, k, A, lda, key_a, k_pad, bar_a);
    return hipGetLastError();
}

hipError_t launch_bound_planes_b(hipStream_t st, int64_t k, int64_t n, const double* B,
                                 int64_t ldb, const int32_t* key_b, int64_t n_pad, int64_t k_pad,
                                 int8_t* bar_b) {
    dim3 grid((unsigned)((n_pad + 63) / 64), (unsigned)((k_pad + 63) / 64));
    bound_planes_b_kernel<<<grid, dim3(256), 0, st>>>(k, n, B, ldb, key_b, n_pad, k_pad, bar_b);
    return hipGetLastError();
}

hipError_t launch_bound_shifts(hipStream_t st, int64_t count, const int32_t* key,
                               const int32_t* gmax, int L, int32_t* shift) {
    if (count <= 0) return hipSuccess;
    bound_shifts_kernel<<<dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st>>>(count, key,
                                                                                   gmax, L, shift);
    return hipGetLastError();
}

}  // namespace ozemu
