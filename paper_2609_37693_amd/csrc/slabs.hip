// Running residues of the blocked call (Sec. V-B, "Slabs"): the inner
// dimension is cut into slabs, each slab's residue GEMMs are accumulated on
// their own (the INT32 cap holds per slab) and their residues W mod m_l are
// added into the running residue of every output entry, (z + w) mod m_l,
// which is exact: residues of a sum are sums of residues.
#include "slabs.hpp"

namespace ozemu {

namespace {

// Thread g adds 16 bytes: vector g of the buffers, in plane g / plane_vec.
__global__ __launch_bounds__(256) void add_residues_kernel(ModConsts mc, int64_t plane_vec,
                                                          int64_t total_vec, uint8_t* z,
                                                          const uint8_t* w) {
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= total_vec) return;
    const uint32_t m = mc.m[g / plane_vec];
    uint4 a = reinterpret_cast<const uint4*>(z)[g];
    const uint4 b = reinterpret_cast<const uint4*>(w)[g];
    uint32_t* pa = reinterpret_cast<uint32_t*>(&a);
    const uint32_t* pb = reinterpret_cast<const uint32_t*>(&b);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        uint32_t o = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            uint32_t s = ((pa[q] >> (8 * i)) & 0xFFu) + ((pb[q] >> (8 * i)) & 0xFFu);  // < 2m
            s -= (s >= m) ? m : 0u;
            o |= s << (8 * i);
        }
        pa[q] = o;
    }
    reinterpret_cast<uint4*>(z)[g] = a;
}

}  // namespace

hipError_t launch_add_residues(hipStream_t st, const ModConsts& mc, int planes,
                               int64_t plane_bytes, uint8_t* z, const uint8_t* w) {
    const int64_t plane_vec = plane_bytes / 16;
    const int64_t total = plane_vec * planes;
    if (total <= 0) return hipSuccess;
    add_residues_kernel<<<dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st>>>(
        mc, plane_vec, total, z, w);
    return hipGetLastError();
}

}  // namespace ozemu
