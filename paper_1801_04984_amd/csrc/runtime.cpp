// C ABI of the space-time Biot slab library: handle life cycle, validation,
// workspace carving and the operator apply.  Solver entry points live in
// solver.cpp.
#include "runtime.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <sstream>

#include "element.h"
#include "kernels.h"
#include "solver.h"

namespace bt {

static thread_local std::string g_last_error;

void set_error(const std::string& m) { g_last_error = m; }

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    std::ostringstream os;
    os << what << ": " << hipGetErrorString(e);
    throw BiotError{BIOT_ERR_DEVICE, os.str()};
  }
}

static void arg_fail(const std::string& m) { throw BiotError{BIOT_ERR_ARG, m}; }

static void validate_desc(const biot_problem_desc& d, int idx) {
  std::ostringstream os;
  os << "instance " << idx << ": ";
  auto fin = [](double v) { return std::isfinite(v); };
  if (d.dim != 2 && d.dim != 3) arg_fail(os.str() + "dim must be 2 or 3");
  for (int e = 0; e < d.dim; ++e) {
    if (d.n[e] < 1) arg_fail(os.str() + "n must be >= 1 on every axis");
    if (d.n[e] > 4096) arg_fail(os.str() + "n must be <= 4096 on every axis");
    if (!fin(d.length[e]) || d.length[e] <= 0) arg_fail(os.str() + "box lengths must be > 0");
  }
  if (d.r < 0 || d.r > 3) arg_fail(os.str() + "dG order r must be in 0..3");
  {
    // kernels index within one instance's slab with 32-bit integers
    double nu = 1, np = 1, nq = 0;
    for (int e = 0; e < d.dim; ++e) { nu *= 2.0 * d.n[e] + 1; np *= 2.0 * d.n[e]; }
    for (int c = 0; c < d.dim; ++c) {
      double t = 1;
      for (int e = 0; e < d.dim; ++e) t *= (e == c) ? 2.0 * d.n[e] + 1 : 2.0 * d.n[e];
      nq += t;
    }
    if ((d.r + 1) * (d.dim * nu + nq + np) >= 2147483647.0)
      arg_fail(os.str() + "one instance's slab must hold fewer than 2^31 unknowns");
  }
  if (!fin(d.tau) || d.tau <= 0) arg_fail(os.str() + "tau must be > 0");
  if (!fin(d.mu) || d.mu <= 0) arg_fail(os.str() + "mu must be > 0");
  if (!fin(d.lambda) || d.lambda + 2.0 * d.mu / d.dim <= 0) arg_fail(os.str() + "lambda + 2 mu / dim must be > 0");
  if (!fin(d.b) || d.b <= 0 || d.b >= 1) arg_fail(os.str() + "Biot coefficient b must lie in (0, 1)");
  if (!fin(d.M) || d.M <= 0) arg_fail(os.str() + "Biot modulus M must be > 0");
  if (!fin(d.eta) || d.eta <= 0) arg_fail(os.str() + "viscosity eta must be > 0");
  if (!fin(d.L_fs)) arg_fail(os.str() + "L_fs must be finite");
  if (d.pair_mode < BIOT_PAIR_AUTO || d.pair_mode > BIOT_PAIR_SHIFT)
    arg_fail(os.str() + "unknown pair_mode");
  if (d.load_kind != BIOT_LOAD_STEP && d.load_kind != BIOT_LOAD_RAMP) arg_fail(os.str() + "unknown load_kind");
  if (!fin(d.load_s0)) arg_fail(os.str() + "load_s0 must be finite");
  if (d.load_kind == BIOT_LOAD_RAMP && (!fin(d.load_t_ramp) || d.load_t_ramp <= 0))
    arg_fail(os.str() + "load_t_ramp must be > 0 for a ramp load");
}

// 2D: tau A_e (18 x 18) followed by E_e (18 x 4); 3D: matrix-core fragments of [tau A_e | E_e]
static long long emat_per_instance(int d) { return d == 2 ? 18 * 18 + 18 * 4 : 6 * 23 * 64; }

static InstDev make_inst(const biot_problem_desc& d) {
  InstDev I;
  std::memset(&I, 0, sizeof(I));
  I.dim = d.dim;
  for (int e = 0; e < 3; ++e) {
    I.n[e] = e < d.dim ? d.n[e] : 1;
    I.su[e] = e < d.dim ? 2 * d.n[e] + 1 : 1;
    I.sp[e] = e < d.dim ? 2 * d.n[e] : 1;
    I.h[e] = e < d.dim ? d.length[e] / d.n[e] : 1.0;
  }
  for (int c = 0; c < 3; ++c)
    for (int e = 0; e < 3; ++e) I.sq[c][e] = (e == c) ? I.su[e] : I.sp[e];
  long long nu1 = (long long)I.su[0] * I.su[1] * I.su[2];
  long long o = 0;
  for (int c = 0; c < d.dim; ++c) { I.off_u[c] = o; o += nu1; }
  for (int c = 0; c < d.dim; ++c) {
    I.off_q[c] = o;
    o += (long long)I.sq[c][0] * I.sq[c][1] * I.sq[c][2];
  }
  I.off_p = o;
  o += (long long)I.sp[0] * I.sp[1] * I.sp[2];
  I.N = o;
  I.tau = d.tau; I.lam = d.lambda; I.mu = d.mu; I.b = d.b; I.Minv = 1.0 / d.M; I.eta = d.eta;
  I.Lfs = d.L_fs > 0 ? d.L_fs : d.b * d.b / (d.lambda + 2.0 * d.mu / d.dim);
  I.s0 = d.load_s0; I.t_ramp = d.load_t_ramp; I.load_kind = d.load_kind;
  I.ncells = (long long)I.n[0] * I.n[1] * I.n[2];
  return I;
}

// work list reordered so that each XCD processes one contiguous run of tiles
std::vector<int4> xcd_ordered(const std::vector<int4>& w) {
  const long long n = (long long)w.size();
  std::vector<int4> o(w.size());
  for (long long b = 0; b < n; ++b) o[b] = w[xcd_tile(b, n)];
  return o;
}

static std::vector<int4> make_work(const biot_problem_s* h, int variant) {
  std::vector<int4> w;
  for (int k = 0; k < h->count; ++k) {
    const InstDev& I = h->inst[k];
    if (h->dim == 2) {
      int t = apply2d_tile_cells(variant);
      for (int ty = 0; ty < (I.n[1] + t - 1) / t; ++ty)
        for (int tx = 0; tx < (I.n[0] + t - 1) / t; ++tx) w.push_back(make_int4(k, tx, ty, 0));
    } else {
      int t = apply3d_tile_cells_xy(), tz = apply3d_tile_cells_z(variant);
      for (int z = 0; z < (I.n[2] + tz - 1) / tz; ++z)
        for (int ty = 0; ty < (I.n[1] + t - 1) / t; ++ty)
          for (int tx = 0; tx < (I.n[0] + t - 1) / t; ++tx) w.push_back(make_int4(k, tx, ty, z));
    }
  }
  return xcd_ordered(w);
}

// layout of everything the handle keeps on the device
static void plan_layout(biot_problem_s* h, Layout& L, bool carve) {
  auto* d_inst = L.take<InstDev>(h->count);
  int4* d_work[biot_problem_s::kMaxVariants] = {nullptr, nullptr, nullptr};
  for (int v = 0; v < h->nvariants; ++v) d_work[v] = L.take<int4>(h->nwork_apply[v]);
  auto* kinv64 = L.take<double>(h->ncells);
  auto* kinv32 = L.take<float>(h->ncells);
  auto* theta = L.take<double>(h->ncells);
  auto* em64 = L.take<double>(std::max(1LL, h->emat_len));
  auto* em32 = L.take<float>(std::max(1LL, h->emat_len));
  if (carve) {
    h->d_inst = d_inst; h->d_kinv64 = kinv64; h->d_kinv32 = kinv32;
    for (int v = 0; v < h->nvariants; ++v) h->d_work_apply[v] = d_work[v];
    h->d_theta = theta; h->d_emat64 = em64; h->d_emat32 = em32;
  }
  plan_solver_layout(h, L, carve);
}

static void build_host_state(biot_problem_s* h, const biot_problem_desc* descs, int count) {
  h->count = count;
  h->dim = descs[0].dim;
  h->r = descs[0].r;
  h->nl = h->r + 1;
  h->descs.assign(descs, descs + count);
  h->inst.clear();
  long long xo = 0, so = 0, co = 0;
  for (int k = 0; k < count; ++k) {
    InstDev I = make_inst(descs[k]);
    I.x_off = xo; I.state_off = so; I.cell_off = co;
    I.emat_off = (long long)k * emat_per_instance(descs[0].dim);
    xo += I.N * h->nl; so += I.N; co += I.ncells;
    h->inst.push_back(I);
  }
  h->emat_len = (long long)count * emat_per_instance(descs[0].dim);
  h->slab_len = xo; h->state_len = so; h->ncells = co;
  // apply work lists (one per tile variant)
  h->nvariants = h->dim == 2 ? apply2d_variants() : apply3d_variants();
  for (int v = 0; v < h->nvariants; ++v) h->nwork_apply[v] = (int)make_work(h, v).size();
  h->tc = make_temporal(h->r);
  std::memset(&h->tm, 0, sizeof(h->tm));
  for (int k = 0; k < 16; ++k) { h->tm.T[k] = h->tc.T[k]; h->tm.Q[k] = h->tc.Q[k]; h->tm.Qi[k] = h->tc.Qi[k]; }
  for (int k = 0; k < 4; ++k) { h->tm.g[k] = h->tc.g[k]; h->tm.s[k] = h->tc.s[k]; h->tm.alpha[k] = h->tc.alpha[k]; }
}

static void check_batch(const biot_problem_desc* descs, int count) {
  if (!descs) arg_fail("descs is null");
  if (count < 1) arg_fail("count must be >= 1");
  for (int k = 0; k < count; ++k) validate_desc(descs[k], k);
  for (int k = 1; k < count; ++k) {
    if (descs[k].dim != descs[0].dim) arg_fail("all instances of a batch must share dim");
    if (descs[k].r != descs[0].r) arg_fail("all instances of a batch must share r");
    // step() and adjoint_sweep() advance the whole batch on one clock
    if (descs[k].tau != descs[0].tau) arg_fail("all instances of a batch must share tau");
    if (descs[k].pair_mode != descs[0].pair_mode) arg_fail("all instances of a batch must share pair_mode");
  }
}

static void upload_log_k(biot_problem_s* h, const double* const* log_k, hipStream_t s) {
  if (!log_k) arg_fail("log_k is null");
  std::vector<double> th(h->ncells), k64(h->ncells);
  std::vector<float> k32(h->ncells);
  for (int k = 0; k < h->count; ++k) {
    const InstDev& I = h->inst[k];
    if (!log_k[k]) arg_fail("log_k[" + std::to_string(k) + "] is null");
    for (long long c = 0; c < I.ncells; ++c) {
      double v = log_k[k][c];
      if (!std::isfinite(v)) arg_fail("log_k of instance " + std::to_string(k) + " is not finite");
      th[I.cell_off + c] = v;
      k64[I.cell_off + c] = I.eta * std::exp(-v);
      k32[I.cell_off + c] = (float)k64[I.cell_off + c];
    }
  }
  hip_check(hipMemcpyAsync(h->d_theta, th.data(), th.size() * 8, hipMemcpyHostToDevice, s), "upload theta");
  hip_check(hipMemcpyAsync(h->d_kinv64, k64.data(), k64.size() * 8, hipMemcpyHostToDevice, s), "upload K");
  hip_check(hipMemcpyAsync(h->d_kinv32, k32.data(), k32.size() * 4, hipMemcpyHostToDevice, s), "upload K");
  hip_check(hipStreamSynchronize(s), "upload sync");
}

ApplyArgs apply_args(const biot_problem_s* h, int dtype, hipStream_t s) {
  ApplyArgs a;
  a.inst = h->d_inst;
  a.variant = h->variant[dtype ? 1 : 0];
  a.work = h->d_work_apply[a.variant];
  a.nwork = h->nwork_apply[a.variant];
  a.nl = h->nl;
  a.tm = &h->tm;
  a.kinv = dtype ? (const void*)h->d_kinv32 : (const void*)h->d_kinv64;
  a.emat = dtype ? (const void*)h->d_emat32 : (const void*)h->d_emat64;
  a.count = h->count;
  a.maxN = 0;
  a.maxc = 0;
  for (auto& I : h->inst) { a.maxN = std::max(a.maxN, I.N); a.maxc = std::max(a.maxc, I.ncells); }
  a.stream = s;
  return a;
}

void launch_apply(const biot_problem_s* h, const void* x, void* y, int transpose, int dtype, hipStream_t s) {
  ApplyArgs a = apply_args(h, dtype, s);
  if (h->dim == 2) {
    if (dtype) launch_apply2d<float>(a, x, y, transpose);
    else launch_apply2d<double>(a, x, y, transpose);
  } else {
    if (dtype) launch_apply3d<float>(a, x, y, transpose);
    else launch_apply3d<double>(a, x, y, transpose);
  }
  hip_check(hipGetLastError(), "apply launch");
}

}  // namespace bt

using namespace bt;

#define BIOT_TRY try {
#define BIOT_CATCH                                     \
  }                                                    \
  catch (const BiotError& e) {                         \
    set_error(e.msg);                                  \
    return e.st;                                       \
  }                                                    \
  catch (const std::exception& e) {                    \
    set_error(std::string("internal error: ") + e.what()); \
    return BIOT_ERR_ARG;                               \
  }                                                    \
  return BIOT_OK;

extern "C" {

const char* biot_last_error(void) { return bt::g_last_error.c_str(); }

biot_status biot_workspace_bytes(const biot_problem_desc* descs, int32_t count, size_t* bytes) {
  BIOT_TRY
  if (!bytes) arg_fail("bytes is null");
  check_batch(descs, count);
  biot_problem_s tmp;
  build_host_state(&tmp, descs, count);
  Layout L;
  plan_layout(&tmp, L, false);
  destroy_solver(&tmp);
  *bytes = L.off + 256;
  BIOT_CATCH
}

biot_status create_slab_problem(const biot_problem_desc* descs, int32_t count, const double* const* log_k,
                                void* workspace, size_t ws_bytes, void* stream, biot_problem* out) {
  biot_problem_s* h = nullptr;
  try {
    if (!out) arg_fail("out is null");
    *out = nullptr;
    check_batch(descs, count);
    if (!log_k) arg_fail("log_k is null");
    for (int k = 0; k < count; ++k) {
      if (!log_k[k]) arg_fail("log_k[" + std::to_string(k) + "] is null");
      long long nc = 1;
      for (int e = 0; e < descs[k].dim; ++e) nc *= descs[k].n[e];
      for (long long c = 0; c < nc; ++c)
        if (!std::isfinite(log_k[k][c])) arg_fail("log_k of instance " + std::to_string(k) + " is not finite");
    }
    h = new biot_problem_s();
    build_host_state(h, descs, count);
    Layout L;
    plan_layout(h, L, false);
    size_t need = L.off + 256;
    if (!workspace) throw BiotError{BIOT_ERR_WORKSPACE, "workspace is null"};
    if (ws_bytes < need) {
      throw BiotError{BIOT_ERR_WORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes, got " +
                                              std::to_string(ws_bytes)};
    }
    uintptr_t base = ((uintptr_t)workspace + 255) & ~uintptr_t(255);
    h->ws = (char*)workspace;
    h->ws_bytes = ws_bytes;
    Layout C;
    C.base = (char*)base;
    plan_layout(h, C, true);
    hipStream_t s = (hipStream_t)stream;
    // look up this device's copy of the static scratch of biot_misfit_noalloc once, here
    (void)scratch_ptr();
    // the workspace starts defined: no buffer of the handle ever holds stale caller data
    hip_check(hipMemsetAsync((void*)base, 0, C.off, s), "workspace clear");
    hip_check(hipMemcpyAsync(h->d_inst, h->inst.data(), sizeof(InstDev) * h->count, hipMemcpyHostToDevice, s),
              "upload instances");
    std::vector<std::vector<int4>> works;
    for (int v = 0; v < h->nvariants; ++v) {
      works.push_back(make_work(h, v));
      hip_check(hipMemcpyAsync(h->d_work_apply[v], works.back().data(), sizeof(int4) * works.back().size(),
                               hipMemcpyHostToDevice, s),
                "upload work list");
    }
    upload_log_k(h, log_k, s);
    if (h->emat_len > 0) {
      std::vector<double> em(h->emat_len);
      std::vector<float> em32(h->emat_len);
      for (int k = 0; k < h->count; ++k) {
        const auto& D = h->descs[k];
        const double hh[3] = {h->inst[k].h[0], h->inst[k].h[1], h->inst[k].h[2]};
        auto A = elast_element(h->dim, hh, D.lambda, D.mu, D.tau);
        auto E = coupling_element(h->dim, hh);
        if (h->dim == 3) {
          auto F = elast_fragments3d(A, &E);
          std::copy(F.begin(), F.end(), em.begin() + h->inst[k].emat_off);
        } else {
          std::copy(A.begin(), A.end(), em.begin() + h->inst[k].emat_off);
          std::copy(E.begin(), E.end(), em.begin() + h->inst[k].emat_off + (long long)A.size());
        }
      }
      for (long long q = 0; q < h->emat_len; ++q) em32[q] = (float)em[q];
      hip_check(hipMemcpyAsync(h->d_emat64, em.data(), 8 * em.size(), hipMemcpyHostToDevice, s), "emat");
      hip_check(hipMemcpyAsync(h->d_emat32, em32.data(), 4 * em32.size(), hipMemcpyHostToDevice, s), "emat");
      hip_check(hipStreamSynchronize(s), "emat sync");
    }
    setup_solver(h, s);
    hip_check(hipStreamSynchronize(s), "create sync");
    *out = h;
  } catch (const BiotError& e) {
    set_error(e.msg);
    if (h) { destroy_solver(h); delete h; }
    return e.st;
  } catch (const std::exception& e) {
    set_error(std::string("internal error: ") + e.what());
    if (h) { destroy_solver(h); delete h; }
    return BIOT_ERR_ARG;
  }
  return BIOT_OK;
}

biot_status destroy_slab_problem(biot_problem h) {
  BIOT_TRY
  if (!h) arg_fail("handle is null");
  destroy_solver(h);
  delete h;
  BIOT_CATCH
}

biot_status biot_set_log_k(biot_problem h, const double* const* log_k, void* stream) {
  BIOT_TRY
  if (!h) arg_fail("handle is null");
  upload_log_k(h, log_k, (hipStream_t)stream);
  refresh_solver(h, (hipStream_t)stream);
  hip_check(hipStreamSynchronize((hipStream_t)stream), "set_log_k sync");
  BIOT_CATCH
}

biot_status biot_sizes(biot_problem h, int32_t instance, int64_t* level_dofs, int64_t* slab_offset,
                       int64_t* state_offset) {
  BIOT_TRY
  if (!h) arg_fail("handle is null");
  if (instance < 0 || instance >= h->count) arg_fail("instance out of range");
  if (level_dofs) *level_dofs = h->inst[instance].N;
  if (slab_offset) *slab_offset = h->inst[instance].x_off;
  if (state_offset) *state_offset = h->inst[instance].state_off;
  BIOT_CATCH
}

biot_status biot_totals(biot_problem h, int64_t* slab_len, int64_t* state_len) {
  BIOT_TRY
  if (!h) arg_fail("handle is null");
  if (slab_len) *slab_len = h->slab_len;
  if (state_len) *state_len = h->state_len;
  BIOT_CATCH
}

biot_status apply_operator(biot_problem h, const void* x, void* y, int32_t transpose, int32_t dtype, void* stream) {
  BIOT_TRY
  if (!h) arg_fail("handle is null");
  if (!x || !y) arg_fail("x and y must be device pointers");
  if (x == y) arg_fail("x and y must not alias");
  if (transpose != 0 && transpose != 1) arg_fail("transpose must be 0 or 1");
  if (dtype != 0 && dtype != 1) arg_fail("dtype must be 0 (double) or 1 (float)");
  launch_apply(h, x, y, transpose, dtype, (hipStream_t)stream);
  BIOT_CATCH
}

}  // extern "C"
