// hsgn_persist.hip -- the persistent window-stage kernels and their launcher.
//
// Built as a translation unit of its own, with the compiler's machine-level
// loop-invariant code motion off: the window loop of k_win_persist would
// otherwise hoist per-window constants and addresses out of the loop and
// keep them live across the whole window body, which spills registers.
#include "hsgn_persist.hpp"

namespace hsgn {

namespace {

template <int NT, bool BED, int STAGE>
const void* persist_fn() {
  return reinterpret_cast<const void*>(k_win_persist<NT, kPersistRows, BED, STAGE>);
}

const void* pick(int nt, bool bed, int stage) {
  if (nt == 512) {
    if (bed) return stage == 1 ? persist_fn<512, true, 1>() : persist_fn<512, true, 2>();
    return stage == 1 ? persist_fn<512, false, 1>() : persist_fn<512, false, 2>();
  }
  if (bed) return stage == 1 ? persist_fn<256, true, 1>() : persist_fn<256, true, 2>();
  return stage == 1 ? persist_fn<256, false, 1>() : persist_fn<256, false, 2>();
}

}  // namespace

hipError_t win_persist_occupancy(int nt, bool bed, int stage, int* occ) {
  if ((nt != 256 && nt != 512) || (stage != 1 && stage != 2)) return hipErrorInvalidValue;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, pick(nt, bed, stage), nt, 0);
}

hipError_t launch_win_persist(int nt, bool bed, int stage, int grid, hipStream_t s,
                              const WinArgs& w) {
  if ((nt != 256 && nt != 512) || (stage != 1 && stage != 2) || grid < 8 || grid % 8 != 0 ||
      !w.queue)
    return hipErrorInvalidValue;
  WinArgs a = w;
  void* args[] = {&a};
  return hipLaunchKernel(pick(nt, bed, stage), dim3(grid), dim3(nt), args, 0, s);
}

}  // namespace hsgn
