// Internal launcher interface between the runtime and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include "common.h"

namespace bt {

struct ApplyArgs {
  const InstDev* inst;   // device
  const int4* work;      // device work list (instance, tile x, tile y, tile z)
  int nwork;
  int nl;                // r + 1
  const TimeMat* tm;     // host copy, passed by value to kernels
  const void* kinv;      // device per-cell eta/K (double or float, matching dtype)
  const void* emat;      // device element matrices (2D), matching dtype
  int variant;           // tile variant (2D: tile edge; 3D: z-chunk) of the work list
  int count;             // instances
  long long maxN;        // largest spatial level size
  long long maxc;        // largest cell count
  hipStream_t stream;
};

template <typename T> void launch_apply2d(const ApplyArgs& a, const void* x, void* y, int transpose);
template <typename T> void launch_apply3d(const ApplyArgs& a, const void* x, void* y, int transpose);
int apply2d_variants();
int apply2d_tile_cells(int variant);
int apply3d_variants();
int apply3d_tile_cells_xy();
int apply3d_tile_cells_z(int variant);

}  // namespace bt
