// 3D space-time slab operator (placeholder until the 3D kernel lands).
#include <stdexcept>
#include "kernels.h"
namespace bt {
template <typename T> void launch_apply3d(const ApplyArgs&, const void*, void*, int) {
  throw std::runtime_error("3D apply not built yet");
}
template void launch_apply3d<double>(const ApplyArgs&, const void*, void*, int);
template void launch_apply3d<float>(const ApplyArgs&, const void*, void*, int);
int apply3d_tile_cells_xy() { return 7; }
int apply3d_tile_cells_z() { return 8; }
}  // namespace bt
