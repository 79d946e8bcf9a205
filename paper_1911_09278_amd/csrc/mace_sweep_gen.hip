// Instantiation unit: the sweep for general records, super-voxel sides 4-32.
#include "mace_sweep_gen.h"

namespace mace {
hipError_t launch_sv_gen(const SvArgs& a, int mode, int grid, size_t lds, hipStream_t st) {
  switch (a.S) {
    case 4: return launch_gen_s<4>(a, mode, grid, lds, st);
    case 8: return launch_gen_s<8>(a, mode, grid, lds, st);
    case 16: return launch_gen_s<16>(a, mode, grid, lds, st);
    case 32: return launch_gen_s<32>(a, mode, grid, lds, st);
    default: return hipErrorInvalidValue;
  }
}
}  // namespace mace
