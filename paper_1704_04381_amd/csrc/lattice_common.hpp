// Shared pieces of the lattice growth kernels: the canonical move table.
//
// Candidate codes c = 0..6 without 3 stand for the neighbour directions
// -z, -y, -x, +x, +y, +z (dQ = c - 3 with Q = x + 2y + 3z); this is also the
// canonical order in which free candidates are numbered.
#pragma once

#include "rsaw_device.hpp"

namespace rsaw {

// LUT[mask * 8 + r]: the move to the r-th free candidate of the 7-bit mask,
// packed as (coordinate delta in bytes 1..3) | (dQ mod 256 in byte 0).
__device__ __forceinline__ uint32_t lattice_move(uint32_t idx)
{
    const uint32_t mask = idx >> 3, r = idx & 7u;
    uint32_t seen = 0;
    for (uint32_t c = 0; c < 7; ++c) {
        if (c == 3 || !((mask >> c) & 1u)) continue;
        if (seen == r) {
            const int dq = (int)c - 3;
            const int axis = dq < 0 ? -dq : dq; // 1 = x, 2 = y, 3 = z
            const int32_t dcoord = (dq < 0 ? -1 : 1) * (int32_t)(1u << (8 * axis));
            return ((uint32_t)dcoord & 0xFFFFFF00u) | ((uint32_t)dq & 0xFFu);
        }
        ++seen;
    }
    return 0;
}

constexpr int kLutSize = 120 * 8; // masks up to 0x77

} // namespace rsaw
