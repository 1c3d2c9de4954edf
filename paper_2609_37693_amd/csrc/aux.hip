// Transpose of block-ordered residue planes, used by the backward products
// that reuse a forward's cached planes: the cached B planes (columns of W',
// K = rows of W) become the B operand of dX = dY W^T (columns of W'^T), and
// the cached A planes (rows of X') the A operand of dW = X^T dY.
#include "ozemu_internal.hpp"

namespace ozemu {

namespace {

// Transpose of block-ordered planes: out(r, h) = in(h, r) for r < in_k_pad
// (rows of `out` at or above in_k_pad are zero). `in` has in_rows_pad rows and
// K extent in_k_pad (a multiple of 64); `out` has out_rows_pad rows
// (a multiple of 256, >= in_k_pad) and K extent in_rows_pad.
// grid: (out_rows_pad / 64, in_rows_pad / 64, planes), 256 threads.
__global__ __launch_bounds__(256) void transpose_planes_kernel(int64_t in_rows_pad,
                                                               int64_t in_k_pad,
                                                               int64_t out_rows_pad,
                                                               const int8_t* in, int8_t* out) {
    __shared__ int8_t tile[64][65];
    const int64_t l = blockIdx.z;
    const int64_t r0 = (int64_t)blockIdx.x * 64;  // output rows = input K index
    const int64_t h0 = (int64_t)blockIdx.y * 64;  // output K index = input rows
    const int8_t* src = in + l * in_rows_pad * in_k_pad;
    int8_t* dst = out + l * out_rows_pad * in_rows_pad;
    const int row = threadIdx.x >> 2, chunk = threadIdx.x & 3;
    // load input rows h0 + row, K bytes r0 + 16 chunk .. + 15
    if (r0 < in_k_pad) {
        const uint4 v =
            *reinterpret_cast<const uint4*>(src + plane_offset(h0 + row, r0 + chunk * 16, in_k_pad));
        const int8_t* b = reinterpret_cast<const int8_t*>(&v);
#pragma unroll
        for (int q = 0; q < 16; ++q) tile[row][chunk * 16 + q] = b[q];
    } else {
#pragma unroll
        for (int q = 0; q < 16; ++q) tile[row][chunk * 16 + q] = 0;
    }
    __syncthreads();
    // write output row r0 + row, K bytes h0 + 16 chunk .. + 15
    uint32_t w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
        w[q] = (uint32_t)(uint8_t)tile[chunk * 16 + 4 * q][row] |
               ((uint32_t)(uint8_t)tile[chunk * 16 + 4 * q + 1][row] << 8) |
               ((uint32_t)(uint8_t)tile[chunk * 16 + 4 * q + 2][row] << 16) |
               ((uint32_t)(uint8_t)tile[chunk * 16 + 4 * q + 3][row] << 24);
    *reinterpret_cast<uint4*>(dst + plane_offset(r0 + row, h0 + chunk * 16, in_rows_pad)) =
        make_uint4(w[0], w[1], w[2], w[3]);
}

}  // namespace

hipError_t launch_transpose_planes(hipStream_t st, int planes, int64_t in_rows_pad,
                                   int64_t in_k_pad, int64_t out_rows_pad, const int8_t* in,
                                   int8_t* out) {
    if (planes <= 0 || in_rows_pad <= 0 || out_rows_pad <= 0) return hipSuccess;
    dim3 grid((unsigned)(out_rows_pad / 64), (unsigned)(in_rows_pad / 64), (unsigned)planes);
    transpose_planes_kernel<<<grid, dim3(256), 0, st>>>(in_rows_pad, in_k_pad, out_rows_pad, in,
                                                        out);
    return hipGetLastError();
}

}  // namespace ozemu
