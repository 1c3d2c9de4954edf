// Running residues of the blocked call (Sec. V-B, "Slabs").
#pragma once

#include "ozemu_internal.hpp"

namespace ozemu {

// z_l <- (z_l + w_l) mod m_l for `planes` residue planes of plane_bytes bytes
// each (plane l at l * plane_bytes; plane_bytes a multiple of 16, both
// buffers 16-byte aligned), every byte below m_l on entry.
hipError_t launch_add_residues(hipStream_t st, const ModConsts& mc, int planes,
                               int64_t plane_bytes, uint8_t* z, const uint8_t* w);

}  // namespace ozemu
