// hsgn_persist.hpp -- launcher of the persistent window-stage kernel
// k_win_persist (defined in hsgn_window.hpp, built in hsgn_persist.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "hsgn_window.hpp"

namespace hsgn {

constexpr int kPersistRows = 8;  // rows per thread of the persistent kernels

// Resident workgroups per CU of k_win_persist<nt, kPersistRows, bed, stage>
// (nt 256 or 512, stage 1 or 2) in *occ.
hipError_t win_persist_occupancy(int nt, bool bed, int stage, int* occ);

// Launch k_win_persist<nt, kPersistRows, bed, stage> with `grid` workgroups
// (a positive multiple of 8) on stream s; w.queue points to 9 zeroed counters.
hipError_t launch_win_persist(int nt, bool bed, int stage, int grid, hipStream_t s,
                              const WinArgs& w);

}  // namespace hsgn
