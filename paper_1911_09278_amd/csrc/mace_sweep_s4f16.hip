// Instantiation unit: super-voxel side 4, FP16 records.
#include "mace_sweep.h"

namespace mace {
hipError_t launch_sv_s4f16(const SvArgs& a, int mode, int slots, int grid, size_t lds,
                          hipStream_t st) {
  return launch_s<4, true>(a, mode, slots, grid, lds, st);
}
}  // namespace mace
