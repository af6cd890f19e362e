// 3D space-time slab operator (placeholder until the 3D kernel lands).
#include <stdexcept>
#include "kernels.h"
#include "prec.h"
namespace bt {
template <typename T> void launch_apply3d(const ApplyArgs&, const void*, void*, int) {
  throw std::runtime_error("3D apply not built yet");
}
template void launch_apply3d<double>(const ApplyArgs&, const void*, void*, int);
template void launch_apply3d<float>(const ApplyArgs&, const void*, void*, int);
template <typename T>
void launch_uapply3d(const UGridSeg*, const int4*, int, int, int, const T*, const T*, T*, hipStream_t) {
  throw std::runtime_error("3D elasticity apply not built yet");
}
template void launch_uapply3d<double>(const UGridSeg*, const int4*, int, int, int, const double*, const double*,
                                      double*, hipStream_t);
template void launch_uapply3d<float>(const UGridSeg*, const int4*, int, int, int, const float*, const float*, float*,
                                     hipStream_t);
int apply3d_tile_cells_xy() { return 7; }
int apply3d_tile_cells_z() { return 8; }
}  // namespace bt
