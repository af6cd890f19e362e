// Internal runtime state behind the opaque biot_problem handle.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/biotst.h"
#include "common.h"
#include "temporal.h"

namespace bt {

// work list reordered so that each XCD processes one contiguous run of tiles
std::vector<int4> xcd_ordered(const std::vector<int4>& w);

// workspace layout builder: the same code sizes and carves the workspace
struct Layout {
  size_t off = 0;
  char* base = nullptr;
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

struct BiotError {
  biot_status st;
  std::string msg;
};

void set_error(const std::string& m);
void hip_check(hipError_t e, const char* what);

struct MgLevel;     // preconditioner data (precond.h)
struct PrecData;

}  // namespace bt

struct biot_problem_s {
  int count = 0, dim = 0, r = 0, nl = 0;
  std::vector<biot_problem_desc> descs;
  std::vector<bt::InstDev> inst;       // host copies
  bt::TemporalConstants tc;
  bt::TimeMat tm;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  long long slab_len = 0, state_len = 0, ncells = 0;
  // device arrays (carved from ws)
  bt::InstDev* d_inst = nullptr;
  // operator-apply work lists, one per tile variant; variant[dtype] is the one in use
  static constexpr int kMaxVariants = 3;
  int nvariants = 1;
  int4* d_work_apply[kMaxVariants] = {nullptr, nullptr, nullptr};
  int nwork_apply[kMaxVariants] = {0, 0, 0};
  int variant[2] = {0, 0};
  double* d_kinv64 = nullptr;
  float* d_kinv32 = nullptr;
  double* d_theta = nullptr;
  double* d_emat64 = nullptr;          // element matrices per instance (tau*A_e, E_e)
  float* d_emat32 = nullptr;
  long long emat_len = 0;
  bt::PrecData* prec = nullptr;        // owned (host struct with device pointers)
};
