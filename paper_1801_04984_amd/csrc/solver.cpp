// Slab solver (host orchestration): preconditioner hierarchy set-up, the
// level-blockwise fixed-stress preconditioner, restarted GMRES (FP64, or FP32
// inner solves inside FP64 iterative refinement), slab marching and the
// discrete adjoint sweep.
//
// Sections "Monolithic Approach" and "Preconditioning technology": the slab
// matrix A = T kron M_t + tau I kron K_s is preconditioned in the real block
// eigenbasis of T, where it is block diagonal up to the +-beta M_t couplings of
// complex eigenvalue pairs.  A pair's coupled 2x2 block is solved by the
// preconditioned square-block factorisation (two level solves with the shift
// alpha + beta, pairs.hip), or its couplings are dropped ("diagonal
// blockwise"), per biot_pair_mode; every dG(0)-type level solve
// (alpha M_t + tau K_s)^-1 is approximated by one truncated fixed-stress sweep.
#include "solver.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <random>
#include <string>
#include <type_traits>
#include <vector>

#include "kernels.h"
#include "element.h"
#include "kernels_aux.h"
#include "prec.h"
#include "vec.h"

namespace bt {

constexpr int kMaxRestart = 64;
// coarse-correction over-relaxation of the aggregation multigrid (2^d cells per
// aggregate; measured best on the 2D 128^2 / 3D 48^3 workloads: 2.1 / 2.1)
inline double omega_p(int) { return 2.1; }
// Chebyshev smoothing degree on the DG pressure level: 3 in 2D, 4 in 3D (measured
// on 32^3 and 48^3: degree 3 costs more slab iterations than it saves per
// iteration, degree 5 saves none)
inline int pdeg(int dim) { return dim == 2 ? 3 : 4; }
// degree on the aggregated cell levels below it: 3 in both dimensions (in 3D,
// degree 5 there saves at most one slab iteration in forty, less than it costs)
inline int pcdeg(int) { return 3; }
// Chebyshev smoothing intervals [lo, hi] in units of the power-iteration estimate of
// lambda_max(D^-1 A).  A degree-2 smoother damps a narrow upper band far better than a
// wide one: on the 3D elasticity levels lo = 1/15 cost 48 slab iterations at 48^3 dG(2)
// (the V-cycle barely contracts; lo = 1/20 stagnates), lo = 1/6 cost 31; 1/4 to 1/10 are
// alike.  hi = 1.3 leaves room for an underestimated lambda_max.
constexpr double kPLo = 1.0 / 3.0, kPHi = 1.1;
// Chebyshev degrees of the elasticity smoother before and after the coarse correction.
// In 2D one pre-smoothing step does as well as two (the same slab iteration counts on
// 128^2 and on the 64-instance batch, 5% less time); in 3D one step before or after
// costs iterations at 32^3.
inline int udeg_pre(int dim) { return dim == 2 ? 1 : 2; }
inline int udeg_post(int) { return 2; }
constexpr double kULo = 1.0 / 6.0, kUHi = 1.3;
constexpr double kQLo = 0.25, kQHi = 1.75;  // Gershgorin interval of Dq^-1 Mq
constexpr long long kLineSolveMinLines = 16384;   // automatic flux-block choice
constexpr int kQDegDefault = 8;                     // Chebyshev degree when line solves are not used
// Coarsest multigrid levels: coarsening stops once the largest instance is
// small, or once the dense inverses of the whole batch fit a byte budget that
// keeps one dense coarse product cheaper than another level of the cycle
// (the inverses stay resident in the last-level cache).
constexpr long long kPCoarseCells = 256;
constexpr long long kUCoarseDofs = 1100;
// 2D elasticity levels with fewer 16x16 tiles (times levels j) than this use 8x8 tiles
constexpr long long kUTile16MinTiles = 1024;
constexpr long long kPCoarseBytes = 96LL << 20;   // sum over instances and levels j
constexpr long long kUCoarseBytes = 48LL << 20;   // sum over instances (shared by the levels)

template <typename T>
struct PrecBufs {
  T* V = nullptr;
  T *w = nullptr, *t = nullptr, *r = nullptr;
  T *Wr = nullptr, *Wz = nullptr, *Wf = nullptr, *T1 = nullptr, *T2 = nullptr, *T3 = nullptr, *T4 = nullptr;
  T* Ws = nullptr;   // complex-pair blocks solved with their couplings: w (first level of each pair)
  T* dqinv = nullptr;
  T* pdg_dinv = nullptr;
  std::vector<T*> pc_x, pc_b, pc_r, pc_d0, pc_d1, pc_coef, pc_dinv;
  std::vector<T*> u_x, u_b, u_r, u_d0, u_d1, u_y, u_dinv, u_t1, u_t2;
  T* kinv = nullptr;
  T *xin = nullptr, *bin = nullptr;   // mixed precision: inner solution / right-hand side
  T* pin = nullptr;                   // fixed input of the captured preconditioner graph
};

struct PrecData {
  int nl = 1, dim = 2, count = 1;
  // complex-pair level blocks (biot_pair_mode) and the pairs of the real block form
  int pair_mode = BIOT_PAIR_DROP;   // resolved (never BIOT_PAIR_AUTO)
  PairSet pairs{};
  // preconditioner level k is column lperm[k] of the real block eigenbasis, with its
  // alpha and beta (square-block factorisation: pair firsts, real levels, pair seconds;
  // otherwise the eigenbasis order)
  int lperm[4] = {0, 1, 2, 3};
  double lalpha[4] = {0, 0, 0, 0}, lbeta[4] = {0, 0, 0, 0};
  // pressure hierarchy
  int npl = 0;
  std::vector<PDgSeg> pdg;
  PDgSeg* d_pdg = nullptr;
  long long pdg_total = 0, pdg_max = 0;
  std::vector<std::vector<PCellSeg>> pc;
  std::vector<PCellSeg*> d_pc;
  std::vector<long long> pc_total, pc_max;
  // elasticity hierarchy
  int nul = 0;
  std::vector<std::vector<UGridSeg>> ug;        // level 0: slab layout
  std::vector<UGridSeg*> d_ug;
  std::vector<UGridSeg> ug0c;                   // level 0 compact layout (set-up)
  UGridSeg* d_ug0c = nullptr;
  std::vector<long long> u_total, u_max;
  // elasticity operator work lists and tile variants per u level l and number of time
  // levels nj of a launch (index uvar(l, nj)): 2D tile edge variant, 3D z-chunk
  std::vector<std::vector<int4>> uwork;
  std::vector<int> utile;
  std::vector<int4*> d_uwork;
  std::vector<std::vector<std::vector<RPass>>> rp;   // [transition][pass][inst]
  std::vector<std::vector<RPass*>> d_rp;
  std::vector<std::vector<long long>> rp_max;
  std::vector<long long> t1_total, t2_total;
  std::vector<std::vector<UProl>> up;
  std::vector<UProl*> d_up;
  std::vector<std::vector<LSeg>> ul;            // Chebyshev segments per u level (level 0 slab layout)
  std::vector<LSeg*> d_ul;
  std::vector<LSeg> ul0c;
  LSeg* d_ul0c = nullptr;
  std::vector<double> utab_h;
  double* d_utab = nullptr;
  long long uemat_len = 0;
  double* d_uemat64 = nullptr;
  float* d_uemat32 = nullptr;
  // coarse dense solves
  std::vector<DSeg> ud, pd;
  DSeg *d_ud = nullptr, *d_pd = nullptr;
  double *uAinv = nullptr, *pAinv = nullptr;
  int u_maxn = 0, p_maxn = 0;
  long long uAinv_len = 0, pAinv_len = 0;
  // their in-place inversion on the device (one matrix per instance for u, per
  // instance and level j for p)
  std::vector<GJMat> gju, gjp;
  GJMat *d_gju = nullptr, *d_gjp = nullptr;
  double* gj_snap = nullptr;
  long long gj_snap_len = 0;
  int* gj_bad = nullptr;
  // GMRES segments
  std::vector<VSeg> gseg;
  VSeg* d_gseg = nullptr;
  long long gmax = 0;
  // scalars
  double *partial = nullptr, *dot1 = nullptr, *dot2 = nullptr, *dot3 = nullptr, *coef = nullptr, *scal = nullptr;
  // adjoint helpers
  double *lam = nullptr, *lam_next = nullptr, *xfwd = nullptr, *arhs = nullptr, *sres = nullptr, *sobs = nullptr;
  // march predictor: xfwd holds the slab solved last by step(), ending at prev_tend
  bool have_prev = false;
  double prev_tend = 0.0;
  Mat4 pred;
  SensorW* sw = nullptr;
  int max_sens = 256;
  PrecBufs<double> b64;
  PrecBufs<float> b32;
  Mat4 Q, Qi;     // real block eigenbasis of T and its inverse
  Mat4 Qt, Qit;   // their transposes (the eigenbasis of T^T is Q^-T)
  // captured preconditioner graphs (per precision and flux Chebyshev degree)
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec[12] = {};   // [precision + 2 * transpose + 4 * sub-system]
  int gdeg[12] = {};
  // captured Arnoldi steps (preconditioner, operator, CGS2, normalisation), one
  // per Krylov index and variant; their dot products land in pinned host memory
  std::map<long long, hipGraphExec_t> arnoldi;
  double* hdots = nullptr;   // 3 x count x 64: V^T w of the two Gram-Schmidt passes, |w|^2
  long long maxN = 0, maxcells = 0, maxlines = 0;
  int maxcells_line = 0;   // most cells along any axis of any instance
};

template <typename T>
PrecBufs<T>& bufs(PrecData* P);
template <typename T>
const T* uemat(PrecData* P);
template <>
PrecBufs<double>& bufs<double>(PrecData* P) { return P->b64; }
template <>
PrecBufs<float>& bufs<float>(PrecData* P) { return P->b32; }
template <>
const double* uemat<double>(PrecData* P) { return P->d_uemat64; }
template <>
const float* uemat<float>(PrecData* P) { return P->d_uemat32; }

// ---------------------------------------------------------------------------
// hierarchy description (host), identical for sizing and carving
// ---------------------------------------------------------------------------
static int half(int n) { return (n + 1) / 2; }

// 1D interpolation of the coarse Q2 basis (nc cells) at the fine Q2 nodes (nf cells), both on [0, L]
static void interp_table(int nf, int nc, std::vector<double>& prol, std::vector<std::vector<std::pair<int, double>>>& rows) {
  const double L = 1.0;
  const double hf = L / nf, hc = L / nc;
  prol.assign(4 * (2 * nf + 1), 0.0);
  rows.assign(2 * nc + 1, {});
  for (int m = 0; m < 2 * nf + 1; ++m) {
    const double x = m * hf / 2.0;
    int C = (int)std::floor(x / hc + 1e-12);
    if (C > nc - 1) C = nc - 1;
    if (C < 0) C = 0;
    double s = x / hc - C;
    if (std::fabs(s) < 1e-13) s = 0.0;
    if (std::fabs(s - 1.0) < 1e-13) s = 1.0;
    prol[4 * m] = C;
    for (int a = 0; a < 3; ++a) {
      double w = phi(a, s);
      if (std::fabs(w) < 1e-14) w = 0.0;
      prol[4 * m + 1 + a] = w;
      if (w != 0.0) rows[2 * C + a].push_back({m, w});
    }
  }
}

// work-list index of u level l for launches over nj time levels (1..4)
static inline int uvar(int l, int nj) { return 4 * l + nj - 1; }

// z-chunk (cell layers per block) of the 3D elasticity kernel for a launch over nj
// time levels.  A block (an xy tile of a chunk of one level) holds a whole CU, so a
// launch takes ceil(blocks / CUs) rounds, each of about chunk + halo layer + one
// layer's worth of set-up; the chunk with the fewest such layer steps is taken
// (ties: the longer chunk).  At 48^3 this gives 16 layers for three levels, 10 for
// one or two; the small levels, which are bound by the latency of the serial layer
// march, get chunks of one or two layers.
static int zchunk3d(const std::vector<UGridSeg>& segs, int nj) {
  const int t = apply3d_tile_cells_xy();
  int nzmax = 1;
  for (const auto& g : segs) nzmax = std::max(nzmax, g.n[2]);
  int best = 1;
  long long bestc = -1;
  for (int zc = 1; zc <= 16; ++zc) {
    long long blocks = 0;
    for (const auto& g : segs)
      blocks += (long long)((g.n[0] + t - 1) / t) * ((g.n[1] + t - 1) / t) * ((g.n[2] + zc - 1) / zc);
    const long long rounds = (blocks * nj + kCus - 1) / kCus;
    const long long c = rounds * (std::min(zc, nzmax) + (nzmax > zc ? 1 : 0) + 1);
    if (bestc < 0 || c <= bestc) { bestc = c; best = zc; }
  }
  return best;
}

static void build_hierarchy(biot_problem_s* h, PrecData* P) {
  const int d = h->dim, nl = h->nl, cnt = h->count;
  P->nl = nl; P->dim = d; P->count = cnt;
  P->maxN = 0; P->maxcells = 0; P->maxlines = 0; P->maxcells_line = 0;
  for (auto& I : h->inst) {
    P->maxN = std::max(P->maxN, I.N);
    P->maxcells = std::max(P->maxcells, I.ncells);
    long long lines = 0;   // lines of flux nodes: per component, the product of the open sizes across
    for (int e = 0; e < d; ++e) {
      long long c = 1;
      for (int f = 0; f < d; ++f)
        if (f != e) c *= I.sp[f];
      lines += c;
    }
    P->maxlines = std::max(P->maxlines, lines);
    for (int e = 0; e < d; ++e) P->maxcells_line = std::max(P->maxcells_line, I.n[e]);
  }
  // ---- pressure: DG level segments
  P->pdg.clear();
  long long off = 0;
  P->pdg_max = 0;
  for (int k = 0; k < cnt; ++k) {
    const InstDev& I = h->inst[k];
    const auto& D = h->descs[k];
    PDgSeg s;
    std::memset(&s, 0, sizeof(s));
    s.inst = k;
    s.I = I;
    s.voff = I.x_off + I.off_p;
    s.vjstride = I.N;
    s.dqoff = I.state_off;
    const long long np = (long long)I.sp[0] * I.sp[1] * I.sp[2];
    s.doff = off;
    s.djstride = np;
    off += nl * np;
    const double kdr = D.lambda + 2.0 * D.mu / d;
    const double L = D.L_fs > 0 ? D.L_fs : D.b * D.b / kdr;
    // level shift: alpha_j, or alpha_j + |beta_j| on complex-pair levels unless their couplings are dropped
    for (int j = 0; j < 4; ++j) {
      const double sh = P->lalpha[j] + (P->pair_mode == BIOT_PAIR_DROP ? 0.0 : std::fabs(P->lbeta[j]));
      s.cm[j] = (j < nl) ? sh * (1.0 / D.M + L) : 0.0;
    }
    P->pdg.push_back(s);
    P->pdg_max = std::max(P->pdg_max, np);
  }
  P->pdg_total = off;
  // ---- pressure cell levels (uniform depth across the batch)
  std::vector<std::array<int, 3>> n(cnt);
  for (int k = 0; k < cnt; ++k) n[k] = {h->inst[k].n[0], h->inst[k].n[1], h->inst[k].n[2]};
  P->pc.clear(); P->pc_total.clear(); P->pc_max.clear();
  while (true) {
    std::vector<PCellSeg> lev;
    long long voff = 0, coff = 0, doff = 0, mx = 0;
    for (int k = 0; k < cnt; ++k) {
      PCellSeg s;
      std::memset(&s, 0, sizeof(s));
      s.dim = d;
      for (int e = 0; e < 3; ++e) s.n[e] = e < d ? n[k][e] : 1;
      s.ncells = (long long)s.n[0] * s.n[1] * s.n[2];
      s.voff = voff; s.vjstride = s.ncells; voff += nl * s.ncells;
      s.coff = coff; coff += 5 * s.ncells;
      s.doff = doff; s.djstride = s.ncells; doff += nl * s.ncells;
      for (int j = 0; j < 4; ++j) s.cm[j] = P->pdg[k].cm[j];
      lev.push_back(s);
      mx = std::max(mx, s.ncells);
    }
    P->pc.push_back(lev);
    P->pc_total.push_back(voff / nl);
    P->pc_max.push_back(mx);
    long long dbytes = 0;
    for (const auto& c : lev) dbytes += 8LL * nl * c.ncells * c.ncells;
    if (mx <= kPCoarseCells || dbytes <= kPCoarseBytes) break;
    for (int k = 0; k < cnt; ++k)
      for (int e = 0; e < d; ++e) n[k][e] = half(n[k][e]);
  }
  P->npl = (int)P->pc.size();
  // ---- elasticity levels
  for (int k = 0; k < cnt; ++k) n[k] = {h->inst[k].n[0], h->inst[k].n[1], h->inst[k].n[2]};
  P->ug.clear(); P->u_total.clear(); P->u_max.clear(); P->ul.clear();
  P->ug0c.clear(); P->ul0c.clear();
  int level = 0;
  long long dinv_off = 0;
  long long uemat_off = 0;
  std::vector<long long> dinv_base;
  while (true) {
    std::vector<UGridSeg> lev;
    std::vector<LSeg> ls;
    long long voff = 0, mx = 0, lvtot = 0;
    for (int k = 0; k < cnt; ++k) {
      const auto& D = h->descs[k];
      UGridSeg g;
      std::memset(&g, 0, sizeof(g));
      g.dim = d;
      for (int e = 0; e < 3; ++e) {
        g.n[e] = e < d ? n[k][e] : 1;
        g.su[e] = e < d ? 2 * n[k][e] + 1 : 1;
        g.h[e] = e < d ? D.length[e] / n[k][e] : 1.0;
      }
      g.tau = D.tau; g.lam = D.lambda; g.mu = D.mu;
      g.nu = (long long)d * g.su[0] * g.su[1] * g.su[2];
      g.emat_off = uemat_off;
      uemat_off += d == 2 ? 18 * 18 : 6 * 21 * 64;
      g.doff = dinv_off + lvtot;
      if (level == 0) { g.voff = h->inst[k].x_off + h->inst[k].off_u[0]; g.vjstride = h->inst[k].N; }
      else { g.voff = voff; g.vjstride = g.nu; voff += nl * g.nu; }
      lev.push_back(g);
      LSeg l;
      l.off = g.voff; l.jstride = g.vjstride; l.len = g.nu; l.doff = g.doff; l.djstride = 0;
      ls.push_back(l);
      if (level == 0) {
        UGridSeg gc = g;
        gc.voff = lvtot; gc.vjstride = g.nu;
        P->ug0c.push_back(gc);
        LSeg lc = l;
        lc.off = gc.voff; lc.jstride = gc.vjstride;
        P->ul0c.push_back(lc);
      }
      lvtot += g.nu;
      mx = std::max(mx, g.nu);
    }
    dinv_base.push_back(dinv_off);
    dinv_off += lvtot;
    P->ug.push_back(lev);
    P->ul.push_back(ls);
    P->u_total.push_back(lvtot);
    P->u_max.push_back(mx);
    ++level;
    long long dbytes = 0;
    for (const auto& g : lev) dbytes += 8LL * g.nu * g.nu;
    if (mx <= kUCoarseDofs || dbytes <= kUCoarseBytes) break;
    for (int k = 0; k < cnt; ++k)
      for (int e = 0; e < d; ++e) n[k][e] = half(n[k][e]);
  }
  P->nul = (int)P->ug.size();
  P->uemat_len = uemat_off;
  // work lists per u level and launch width nj; 2D levels with few 16x16 tiles use 8x8 tiles
  P->uwork.assign(P->nul * 4, {});
  P->utile.assign(P->nul * 4, 0);
  for (int l = 0; l < P->nul; ++l)
    for (int nj = 1; nj <= nl; ++nj) {
      const int v = uvar(l, nj);
      if (d == 3) {
        P->utile[v] = zchunk3d(P->ug[l], nj);
      } else {
        long long t16 = 0;
        for (const auto& g : P->ug[l]) t16 += (long long)((g.n[0] + 14) / 15) * ((g.n[1] + 14) / 15);
        P->utile[v] = t16 * nj < kUTile16MinTiles ? 1 : 0;
      }
      for (int k = 0; k < cnt; ++k) {
        const UGridSeg& g = P->ug[l][k];
        if (d == 2) {
          const int t = uapply_tile(d, P->utile[v]);
          for (int ty = 0; ty < (g.n[1] + t - 1) / t; ++ty)
            for (int tx = 0; tx < (g.n[0] + t - 1) / t; ++tx) P->uwork[v].push_back(make_int4(k, tx, ty, 0));
        } else {
          const int txy = apply3d_tile_cells_xy(), tz = P->utile[v];
          for (int z = 0; z < (g.n[2] + tz - 1) / tz; ++z)
            for (int ty = 0; ty < (g.n[1] + txy - 1) / txy; ++ty)
              for (int tx = 0; tx < (g.n[0] + txy - 1) / txy; ++tx)
                P->uwork[v].push_back(make_int4(k, tx, ty, z));
        }
      }
      P->uwork[v] = xcd_ordered(P->uwork[v]);
    }
  // transfers per transition l -> l+1
  P->utab_h.clear();
  P->rp.assign(std::max(0, P->nul - 1), {});
  P->rp_max.assign(std::max(0, P->nul - 1), {});
  P->up.assign(std::max(0, P->nul - 1), {});
  P->t1_total.assign(std::max(0, P->nul - 1), 0);
  P->t2_total.assign(std::max(0, P->nul - 1), 0);
  for (int l = 0; l + 1 < P->nul; ++l) {
    P->rp[l].assign(d, {});
    P->rp_max[l].assign(d, 0);
    long long t1o = 0, t2o = 0;
    for (int k = 0; k < cnt; ++k) {
      const UGridSeg& F = P->ug[l][k];
      const UGridSeg& C = P->ug[l + 1][k];
      long long tabp[3] = {0, 0, 0}, tabr[3] = {0, 0, 0};
      int width[3] = {1, 1, 1};
      for (int e = 0; e < d; ++e) {
        std::vector<double> prol;
        std::vector<std::vector<std::pair<int, double>>> rows;
        interp_table(F.n[e], C.n[e], prol, rows);
        tabp[e] = (long long)P->utab_h.size();
        P->utab_h.insert(P->utab_h.end(), prol.begin(), prol.end());
        int w = 1;
        for (auto& rw : rows) w = std::max(w, (int)rw.size());
        width[e] = w;
        tabr[e] = (long long)P->utab_h.size();
        for (auto& rw : rows) {
          for (int q = 0; q < w; ++q) {
            if (q < (int)rw.size()) { P->utab_h.push_back(rw[q].first); P->utab_h.push_back(rw[q].second); }
            else { P->utab_h.push_back(0.0); P->utab_h.push_back(0.0); }
          }
        }
      }
      UProl pr;
      std::memset(&pr, 0, sizeof(pr));
      pr.dim = d;
      for (int e = 0; e < 3; ++e) { pr.sf[e] = F.su[e]; pr.sc[e] = C.su[e]; pr.tab[e] = tabp[e]; }
      pr.foff = F.voff; pr.fjstride = F.vjstride; pr.coff = C.voff; pr.cjstride = C.vjstride;
      P->up[l].push_back(pr);
      // separable restriction passes: axis 0 -> t1, axis 1 -> t2 (3D) / coarse (2D), axis 2 -> coarse
      int cur[3] = {F.su[0], F.su[1], F.su[2]};
      for (int pass = 0; pass < d; ++pass) {
        RPass rp;
        std::memset(&rp, 0, sizeof(rp));
        rp.dim = d;
        rp.axis = pass;
        rp.width = width[pass];
        rp.last = pass == d - 1;
        for (int e = 0; e < 3; ++e) rp.din[e] = cur[e];
        cur[pass] = C.su[pass];
        for (int e = 0; e < 3; ++e) rp.dout[e] = cur[e];
        rp.tab = tabr[pass];
        const long long nout = (long long)d * cur[0] * cur[1] * cur[2];
        P->rp_max[l][pass] = std::max(P->rp_max[l][pass], nout);
        // input
        if (pass == 0) { rp.ioff = F.voff; rp.ijstride = F.vjstride; }
        else {
          const auto& prev = P->rp[l][pass - 1].back();
          rp.ioff = prev.ooff; rp.ijstride = prev.ojstride;
        }
        // output
        if (rp.last) { rp.ooff = C.voff; rp.ojstride = C.vjstride; }
        else if (pass == 0) { rp.ooff = t1o; rp.ojstride = nout; t1o += nl * nout; }
        else { rp.ooff = t2o; rp.ojstride = nout; t2o += nl * nout; }
        P->rp[l][pass].push_back(rp);
      }
    }
    P->t1_total[l] = t1o;
    P->t2_total[l] = t2o;
  }
  // dense coarse segments
  P->ud.clear(); P->pd.clear();
  P->u_maxn = 0; P->p_maxn = 0;
  long long mo = 0;
  for (int k = 0; k < cnt; ++k) {
    const UGridSeg& g = P->ug[P->nul - 1][k];
    DSeg s;
    std::memset(&s, 0, sizeof(s));
    s.off = g.voff; s.jstride = g.vjstride; s.n = (int)g.nu; s.moff = mo; s.mjstride = 0;
    mo += g.nu * g.nu;
    P->ud.push_back(s);
    P->u_maxn = std::max(P->u_maxn, s.n);
  }
  P->uAinv_len = mo;
  P->gju.clear();
  long long so = 0;
  for (const auto& d : P->ud) {
    P->gju.push_back(GJMat{d.moff, so, d.n, 0});
    so += 4LL * d.n;
  }
  P->gj_snap_len = so;
  mo = 0;
  for (int k = 0; k < cnt; ++k) {
    const PCellSeg& c = P->pc[P->npl - 1][k];
    DSeg s;
    std::memset(&s, 0, sizeof(s));
    s.off = c.voff; s.jstride = c.vjstride; s.n = (int)c.ncells; s.moff = mo; s.mjstride = c.ncells * c.ncells;
    mo += nl * c.ncells * c.ncells;
    P->pd.push_back(s);
    P->p_maxn = std::max(P->p_maxn, s.n);
  }
  P->pAinv_len = mo;
  P->gjp.clear();
  so = 0;
  for (const auto& d : P->pd)
    for (int j = 0; j < nl; ++j) {
      P->gjp.push_back(GJMat{d.moff + j * d.mjstride, so, d.n, 0});
      so += 4LL * d.n;
    }
  P->gj_snap_len = std::max(P->gj_snap_len, so);
  if (P->u_maxn > 65535 || P->p_maxn > 65535) throw BiotError{BIOT_ERR_ARG, "coarse level too large"};
  // GMRES segments
  P->gseg.clear();
  P->gmax = 0;
  for (auto& I : h->inst) {
    VSeg s{I.x_off, I.N * nl};
    P->gseg.push_back(s);
    P->gmax = std::max(P->gmax, s.len);
  }
}

template <typename T>
static void carve_bufs(biot_problem_s* h, PrecData* P, PrecBufs<T>& B, Layout& L, bool fp32) {
  const long long S = h->slab_len;
  B.V = L.take<T>((size_t)(kMaxRestart + 1) * S);
  B.w = L.take<T>(S); B.t = L.take<T>(S); B.r = L.take<T>(S);
  B.xin = L.take<T>(S); B.bin = L.take<T>(S); B.pin = L.take<T>(S);
  B.Wr = L.take<T>(S); B.Wz = L.take<T>(S); B.Wf = L.take<T>(S);
  B.T1 = L.take<T>(S); B.T2 = L.take<T>(S); B.T3 = L.take<T>(S); B.T4 = L.take<T>(S);
  if (P->pair_mode == BIOT_PAIR_PRESB && P->pairs.n > 0) B.Ws = L.take<T>(S);
  B.dqinv = L.take<T>(h->state_len);
  B.pdg_dinv = L.take<T>(P->pdg_total);
  const int nl = h->nl;
  B.pc_x.assign(P->npl, nullptr); B.pc_b = B.pc_x; B.pc_r = B.pc_x; B.pc_d0 = B.pc_x; B.pc_d1 = B.pc_x;
  B.pc_coef = B.pc_x; B.pc_dinv = B.pc_x;
  for (int l = 0; l < P->npl; ++l) {
    const long long n = P->pc_total[l];
    B.pc_x[l] = L.take<T>(nl * n); B.pc_b[l] = L.take<T>(nl * n); B.pc_r[l] = L.take<T>(nl * n);
    B.pc_d0[l] = L.take<T>(nl * n); B.pc_d1[l] = L.take<T>(nl * n);
    B.pc_coef[l] = L.take<T>(5 * n); B.pc_dinv[l] = L.take<T>(nl * n);
  }
  B.u_x.assign(P->nul, nullptr); B.u_b = B.u_x; B.u_r = B.u_x; B.u_d0 = B.u_x; B.u_d1 = B.u_x; B.u_y = B.u_x;
  B.u_dinv = B.u_x; B.u_t1 = B.u_x; B.u_t2 = B.u_x;
  long long dtot = 0;
  for (int l = 0; l < P->nul; ++l) dtot += P->u_total[l];
  T* dall = L.take<T>(dtot);
  for (int l = 0; l < P->nul; ++l) {
    B.u_dinv[l] = dall;   // every level's segments carry absolute offsets into this array
    if (l == 0) continue;
    const long long n = P->u_total[l];
    B.u_x[l] = L.take<T>(nl * n); B.u_b[l] = L.take<T>(nl * n); B.u_r[l] = L.take<T>(nl * n);
    B.u_d0[l] = L.take<T>(nl * n); B.u_d1[l] = L.take<T>(nl * n); B.u_y[l] = L.take<T>(nl * n);
  }
  for (int l = 0; l + 1 < P->nul; ++l) {
    B.u_t1[l] = L.take<T>(std::max(1LL, P->t1_total[l]));
    B.u_t2[l] = L.take<T>(std::max(1LL, P->t2_total[l]));
  }
  (void)fp32;
}

void plan_solver_layout(biot_problem_s* h, Layout& L, bool carve) {
  PrecData* P = h->prec;
  if (!P) {
    P = new PrecData();
    h->prec = P;
  }
  // BIOT_PAIR_AUTO: the square-block factorisation where its second pass of level solves
  // costs less than the iterations it saves (3D, r >= 2)
  P->pair_mode = h->descs[0].pair_mode;
  if (P->pair_mode == BIOT_PAIR_AUTO) P->pair_mode = (h->dim == 3 && h->r >= 2) ? BIOT_PAIR_PRESB : BIOT_PAIR_DROP;
  const LevelOrder lo = level_order(h->tc, P->pair_mode == BIOT_PAIR_PRESB);
  P->pairs = PairSet{};
  P->pairs.n = lo.npairs;
  for (int i = 0; i < lo.npairs; ++i) {
    P->pairs.j[i] = lo.first[i];
    P->pairs.j2[i] = lo.second[i];
    P->pairs.beta[i] = lo.beta[i];
  }
  for (int k = 0; k < 4; ++k) {
    P->lperm[k] = lo.perm[k];
    P->lalpha[k] = h->tc.alpha[lo.perm[k]];
    P->lbeta[k] = h->tc.beta[lo.perm[k]];
  }
  build_hierarchy(h, P);
  carve_bufs<double>(h, P, P->b64, L, false);
  carve_bufs<float>(h, P, P->b32, L, true);
  P->b64.kinv = nullptr;
  P->b32.kinv = nullptr;
  P->d_pdg = L.take<PDgSeg>(P->pdg.size());
  P->d_pc.assign(P->npl, nullptr);
  for (int l = 0; l < P->npl; ++l) P->d_pc[l] = L.take<PCellSeg>(P->pc[l].size());
  P->d_ug.assign(P->nul, nullptr);
  P->d_uwork.assign(P->uwork.size(), nullptr);
  P->d_ul.assign(P->nul, nullptr);
  for (int l = 0; l < P->nul; ++l) {
    P->d_ug[l] = L.take<UGridSeg>(P->ug[l].size());
    P->d_ul[l] = L.take<LSeg>(P->ul[l].size());
  }
  for (size_t v = 0; v < P->uwork.size(); ++v)
    if (!P->uwork[v].empty()) P->d_uwork[v] = L.take<int4>(P->uwork[v].size());
  P->d_ug0c = L.take<UGridSeg>(P->ug0c.size());
  P->d_ul0c = L.take<LSeg>(P->ul0c.size());
  P->d_rp.assign(std::max(0, P->nul - 1), {});
  P->d_up.assign(std::max(0, P->nul - 1), nullptr);
  for (int l = 0; l + 1 < P->nul; ++l) {
    for (int pass = 0; pass < P->dim; ++pass) P->d_rp[l].push_back(L.take<RPass>(P->rp[l][pass].size()));
    P->d_up[l] = L.take<UProl>(P->up[l].size());
  }
  P->d_utab = L.take<double>(std::max<size_t>(1, P->utab_h.size()));
  P->d_uemat64 = L.take<double>(std::max(1LL, P->uemat_len));
  P->d_uemat32 = L.take<float>(std::max(1LL, P->uemat_len));
  P->d_ud = L.take<DSeg>(P->ud.size());
  P->d_pd = L.take<DSeg>(P->pd.size());
  P->uAinv = L.take<double>(P->uAinv_len);
  P->pAinv = L.take<double>(P->pAinv_len);
  P->d_gju = L.take<GJMat>(P->gju.size());
  P->d_gjp = L.take<GJMat>(P->gjp.size());
  P->gj_snap = L.take<double>(std::max(1LL, P->gj_snap_len));
  P->gj_bad = L.take<int>(1);
  P->d_gseg = L.take<VSeg>(P->gseg.size());
  const size_t nsc = (size_t)std::max(h->count * h->nl, h->count) * 64;
  P->partial = L.take<double>((size_t)std::max(h->count * h->nl, h->count) * kMaxChunks * 64);
  P->dot1 = L.take<double>(nsc); P->dot2 = L.take<double>(nsc); P->dot3 = L.take<double>(nsc);
  P->coef = L.take<double>(nsc); P->scal = L.take<double>(nsc);
  P->lam = L.take<double>(h->slab_len);
  P->lam_next = L.take<double>(h->slab_len);
  P->xfwd = L.take<double>(h->slab_len);
  P->arhs = L.take<double>(h->slab_len);
  P->sres = L.take<double>((size_t)h->count * P->max_sens);
  P->sobs = L.take<double>((size_t)h->count * P->max_sens);
  P->sw = L.take<SensorW>((size_t)h->count * P->max_sens);
  if (!carve) {
    // sizing pass only: forget device pointers
    P->b64 = PrecBufs<double>();
    P->b32 = PrecBufs<float>();
  }
}

// ---------------------------------------------------------------------------
// host dense helpers
// ---------------------------------------------------------------------------
// assembled tau A of the coarsest elasticity level, essential rows and columns
// replaced by the identity (inverted on the device)
static std::vector<double> coarse_elast_matrix(const UGridSeg& g) {
  const int d = g.dim;
  const int n = (int)g.nu;
  const long long nn = (long long)g.su[0] * g.su[1] * g.su[2];
  std::vector<double> A((size_t)n * n, 0.0);
  auto Ke = elast_element(d, g.h, g.lam, g.mu, g.tau);
  const int nnl = d == 2 ? 9 : 27, nloc = d * nnl;
  std::vector<long long> gidx(nloc);
  for (int k = 0; k < g.n[2]; ++k)
    for (int j = 0; j < g.n[1]; ++j)
      for (int i = 0; i < g.n[0]; ++i) {
        for (int c = 0; c < d; ++c)
          for (int a = 0; a < nnl; ++a) {
            const int ax = a % 3, ay = (a / 3) % 3, az = d == 3 ? a / 9 : 0;
            gidx[c * nnl + a] = c * nn + (2 * i + ax) + (long long)g.su[0] * ((2 * j + ay) + (long long)g.su[1] * (2 * k + az));
          }
        for (int r = 0; r < nloc; ++r)
          for (int c = 0; c < nloc; ++c) A[(size_t)gidx[r] * n + gidx[c]] += Ke[(size_t)r * nloc + c];
      }
  for (int c = 0; c < d; ++c)
    for (long long t = 0; t < nn; ++t) {
      const int mx = t % g.su[0], my = (t / g.su[0]) % g.su[1], mz = (int)(t / ((long long)g.su[0] * g.su[1]));
      if (!ugrid_fixed(d, g.su, c, mx, my, mz)) continue;
      const long long row = c * nn + t;
      for (int q = 0; q < n; ++q) { A[(size_t)row * n + q] = 0.0; A[(size_t)q * n + row] = 0.0; }
      A[(size_t)row * n + row] = 1.0;
    }
  return A;
}

// diag of tau*A on a level (host), 1 on essential rows
static std::vector<double> elast_diag(const UGridSeg& g) {
  const int d = g.dim;
  const long long nn = (long long)g.su[0] * g.su[1] * g.su[2];
  std::vector<double> D(d * nn, 0.0);
  auto Ke = elast_element(d, g.h, g.lam, g.mu, g.tau);
  const int nnl = d == 2 ? 9 : 27, nloc = d * nnl;
  for (int c = 0; c < d; ++c)
    for (long long t = 0; t < nn; ++t) {
      const int m[3] = {(int)(t % g.su[0]), (int)((t / g.su[0]) % g.su[1]), (int)(t / ((long long)g.su[0] * g.su[1]))};
      if (ugrid_fixed(d, g.su, c, m[0], m[1], m[2])) { D[c * nn + t] = 1.0; continue; }
      // cells containing the node: local index per axis
      double s = 0.0;
      int cl[3][2], al[3][2], ncl[3];
      for (int e = 0; e < 3; ++e) {
        ncl[e] = 0;
        if (e >= d) { cl[e][0] = 0; al[e][0] = 0; ncl[e] = 1; continue; }
        if (m[e] & 1) { cl[e][0] = (m[e] - 1) / 2; al[e][0] = 1; ncl[e] = 1; }
        else {
          if (m[e] / 2 - 1 >= 0) { cl[e][ncl[e]] = m[e] / 2 - 1; al[e][ncl[e]] = 2; ++ncl[e]; }
          if (m[e] / 2 < g.n[e]) { cl[e][ncl[e]] = m[e] / 2; al[e][ncl[e]] = 0; ++ncl[e]; }
        }
      }
      for (int iz = 0; iz < ncl[2]; ++iz)
        for (int iy = 0; iy < ncl[1]; ++iy)
          for (int ix = 0; ix < ncl[0]; ++ix) {
            const int a = al[0][ix] + 3 * al[1][iy] + 9 * al[2][iz];
            s += Ke[(size_t)(c * nnl + a) * nloc + (c * nnl + a)];
          }
      D[c * nn + t] = 1.0 / s;
    }
  return D;
}

// ---------------------------------------------------------------------------
// set-up
// ---------------------------------------------------------------------------
struct ChebSeq {
  double s0;
  std::vector<std::pair<double, double>> steps;   // (rho, sig) for step k
};
static ChebSeq cheb_seq(double lo, double hi, int deg) {
  ChebSeq c;
  const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
  double rho = 1.0 / sigma;
  c.s0 = 1.0 / theta;
  for (int k = 0; k < deg; ++k) {
    const double rn = 1.0 / (2.0 * sigma - rho);
    c.steps.push_back({rn * rho, 2.0 * rn / delta});
    rho = rn;
  }
  return c;
}

// host -> device copy of a host vector; waits, so the host buffer may go away afterwards
template <typename X>
static void upload(const std::vector<X>& v, X* d, hipStream_t s) {
  if (v.empty()) return;
  hip_check(hipMemcpyAsync(d, v.data(), sizeof(X) * v.size(), hipMemcpyHostToDevice, s), "upload");
  hip_check(hipStreamSynchronize(s), "upload sync");
}

// invert the uploaded coarse matrices in place and fail on a zero pivot
static void invert_on_device(PrecData* P, const GJMat* mats, int nmats, int maxn, double* A, hipStream_t s) {
  hip_check(hipMemsetAsync(P->gj_bad, 0, sizeof(int), s), "gj flag clear");
  dense_invert(mats, nmats, maxn, A, P->gj_snap, P->gj_bad, s);
  int bad = 0;
  hip_check(hipMemcpyAsync(&bad, P->gj_bad, sizeof(int), hipMemcpyDeviceToHost, s), "gj flag read");
  hip_check(hipStreamSynchronize(s), "gj sync");
  if (bad) throw BiotError{BIOT_ERR_ARG, "singular coarse matrix"};
}

// power iteration for lambda_max(Dinv S) per segment; apply(x, y) computes y = Dinv S x
template <typename F>
static std::vector<double> power_max(PrecData* P, F apply, double* x, double* y, const std::vector<VSeg>& segs,
                                     hipStream_t s, int iters = 14) {
  const int ns = (int)segs.size();
  VSeg* dsegs = (VSeg*)P->scal;   // reuse a scalar block for the segment list (small)
  static_assert(sizeof(VSeg) == 16, "VSeg layout");
  if ((size_t)ns * sizeof(VSeg) > (size_t)std::max(P->count * P->nl, P->count) * 64 * sizeof(double))
    throw BiotError{BIOT_ERR_ARG, "too many power-iteration segments"};
  upload(segs, dsegs, s);
  // the start vector covers every segment (segments need not be packed)
  long long span = 0;
  for (auto& sg : segs) span = std::max(span, sg.off + sg.len);
  std::vector<double> hx(span);
  std::mt19937_64 rng(12345);
  std::uniform_real_distribution<double> U(0.5, 1.5);
  for (auto& v : hx) v = U(rng);
  hip_check(hipMemcpyAsync(x, hx.data(), 8 * span, hipMemcpyHostToDevice, s), "power init");
  hip_check(hipStreamSynchronize(s), "power init sync");
  long long mx = 0;
  for (auto& sg : segs) mx = std::max(mx, sg.len);
  std::vector<double> nrm(ns * 64), lam(ns, 1.0);
  for (int it = 0; it < iters; ++it) {
    seg_mdot<double, double>(x, 0, 1, x, dsegs, ns, 8, P->partial, P->dot1, s);
    seg_scale<double, double>(x, x, P->dot1, 0, 2, dsegs, ns, mx, s);   // x / ||x||
    apply(x, y);
    seg_mdot<double, double>(y, 0, 1, y, dsegs, ns, 8, P->partial, P->dot1, s);
    hip_check(hipMemcpyAsync(nrm.data(), P->dot1, 8 * ns * 64, hipMemcpyDeviceToHost, s), "power norm");
    hip_check(hipStreamSynchronize(s), "power sync");
    for (int q = 0; q < ns; ++q) lam[q] = std::sqrt(std::max(nrm[q * 64], 0.0));
    std::swap(x, y);
  }
  return lam;
}

// scale dinv segments by 1/lambda
static void scale_dinv(PrecData* P, double* dinv, const std::vector<VSeg>& dsegs, const std::vector<double>& lam,
                       hipStream_t s) {
  const int ns = (int)dsegs.size();
  std::vector<double> fac(ns * 64, 0.0);
  for (int q = 0; q < ns; ++q) fac[q * 64] = 1.0 / lam[q];
  VSeg* d = (VSeg*)P->scal;
  upload(dsegs, d, s);
  upload(fac, P->dot2, s);
  long long mx = 0;
  for (auto& v : dsegs) mx = std::max(mx, v.len);
  seg_scale<double, double>(dinv, dinv, P->dot2, 0, 0, d, ns, mx, s);
}

static void cast_to_f32(const double* a, float* b, long long n, hipStream_t s) { vcast(a, b, n, s); }

// pressure coefficients, diagonals, spectral normalisation and coarse inverses (depend on K)
static void setup_pressure(biot_problem_s* h, hipStream_t s) {
  PrecData* P = h->prec;
  auto& B = P->b64;
  const int nl = h->nl, cnt = h->count, d = h->dim;
  launch_dq(h->d_inst, cnt, P->maxN, h->d_kinv64, B.dqinv, s);
  launch_pdg_diag(d, h->d_inst, P->d_pdg, cnt, nl, P->pdg_max, B.dqinv, B.pdg_dinv, s);
  launch_pcoef_first(h->d_inst, P->d_pdg, P->d_pc[0], cnt, P->pc_max[0], B.dqinv, B.pc_coef[0], s);
  for (int l = 0; l + 1 < P->npl; ++l)
    launch_pcoef_coarsen(P->d_pc[l], P->d_pc[l + 1], cnt, P->pc_max[l + 1], B.pc_coef[l], B.pc_coef[l + 1], s);
  for (int l = 0; l < P->npl; ++l) launch_pcell_diag(P->d_pc[l], cnt, nl, P->pc_max[l], B.pc_coef[l], B.pc_dinv[l], s);
  // power iterations: DG level per (instance, level j)
  {
    std::vector<VSeg> segs, dsegs;
    for (int k = 0; k < cnt; ++k)
      for (int j = 0; j < nl; ++j) {
        const PDgSeg& g = P->pdg[k];
        const long long np = (long long)h->inst[k].sp[0] * h->inst[k].sp[1] * h->inst[k].sp[2];
        segs.push_back({g.voff + j * g.vjstride, np});
        dsegs.push_back({g.doff + j * g.djstride, np});
      }
    auto apply = [&](double* x, double* y) {
      launch_pdg<double>(d, h->d_inst, P->d_pdg, cnt, nl, P->pdg_max, kApplyDinv, ChebCoef{0, 0, 0, 1}, B.dqinv,
                         B.pdg_dinv, nullptr, nullptr, nullptr, x, y, s);
    };
    auto lam = power_max(P, apply, B.T1, B.T2, segs, s);
    scale_dinv(P, B.pdg_dinv, dsegs, lam, s);
  }
  for (int l = 0; l < P->npl; ++l) {
    std::vector<VSeg> segs;
    for (int k = 0; k < cnt; ++k)
      for (int j = 0; j < nl; ++j) {
        const PCellSeg& c = P->pc[l][k];
        segs.push_back({c.voff + j * c.vjstride, c.ncells});
      }
    auto apply = [&](double* x, double* y) {
      launch_pcell<double>(P->d_pc[l], cnt, nl, P->pc_max[l], kApplyDinv, ChebCoef{0, 0, 0, 1}, B.pc_coef[l],
                           B.pc_dinv[l], nullptr, nullptr, nullptr, x, y, s);
    };
    auto lam = power_max(P, apply, B.pc_x[l], B.pc_r[l], segs, s);
    std::vector<VSeg> dsegs;
    for (int k = 0; k < cnt; ++k)
      for (int j = 0; j < nl; ++j) dsegs.push_back({P->pc[l][k].doff + j * P->pc[l][k].djstride, P->pc[l][k].ncells});
    scale_dinv(P, B.pc_dinv[l], dsegs, lam, s);
  }
  // coarse dense inverses per (instance, level j) from the coarsest coefficients
  {
    const int l = P->npl - 1;
    std::vector<double> coef(5 * P->pc_total[l]);
    hip_check(hipMemcpyAsync(coef.data(), B.pc_coef[l], 8 * coef.size(), hipMemcpyDeviceToHost, s), "coef read");
    hip_check(hipStreamSynchronize(s), "coef sync");
    std::vector<double> all(P->pAinv_len);
    for (int k = 0; k < cnt; ++k) {
      const PCellSeg& c = P->pc[l][k];
      const long long nc = c.ncells;
      const double* C = coef.data() + c.coff;
      for (int j = 0; j < nl; ++j) {
        std::vector<double> A(nc * nc, 0.0);
        const long long str[3] = {1, (long long)c.n[0], (long long)c.n[0] * c.n[1]};
        for (long long q = 0; q < nc; ++q) {
          const int ce[3] = {(int)(q % c.n[0]), (int)((q / c.n[0]) % c.n[1]), (int)(q / ((long long)c.n[0] * c.n[1]))};
          double dg = c.cm[j] * C[4 * nc + q] + C[3 * nc + q];
          for (int e = 0; e < d; ++e) {
            if (ce[e] > 0) { const double t = C[e * nc + q]; dg += t; A[q * nc + q - str[e]] -= t; }
            if (ce[e] + 1 < c.n[e]) { const double t = C[e * nc + q + str[e]]; dg += t; A[q * nc + q + str[e]] -= t; }
          }
          A[q * nc + q] += dg;
        }
        std::copy(A.begin(), A.end(), all.begin() + P->pd[k].moff + j * P->pd[k].mjstride);
      }
    }
    upload(all, P->pAinv, s);
    invert_on_device(P, P->d_gjp, (int)P->gjp.size(), P->p_maxn, P->pAinv, s);
  }
  // FP32 copies
  auto& F = P->b32;
  cast_to_f32(B.dqinv, F.dqinv, h->state_len, s);
  cast_to_f32(B.pdg_dinv, F.pdg_dinv, P->pdg_total, s);
  for (int l = 0; l < P->npl; ++l) {
    cast_to_f32(B.pc_coef[l], F.pc_coef[l], 5 * P->pc_total[l], s);
    cast_to_f32(B.pc_dinv[l], F.pc_dinv[l], nl * P->pc_total[l], s);
  }
}

static void setup_elasticity(biot_problem_s* h, hipStream_t s) {
  PrecData* P = h->prec;
  auto& B = P->b64;
  const int cnt = h->count, d = h->dim;
  {
    std::vector<double> em(P->uemat_len);
    for (int l = 0; l < P->nul; ++l)
      for (int k = 0; k < cnt; ++k) {
        const UGridSeg& g = P->ug[l][k];
        auto A = elast_element(d, g.h, g.lam, g.mu, g.tau);
        if (d == 3) A = elast_fragments3d(A, nullptr);
        std::copy(A.begin(), A.end(), em.begin() + g.emat_off);
      }
    upload(em, P->d_uemat64, s);
    std::vector<float> e32(em.begin(), em.end());
    upload(e32, P->d_uemat32, s);
  }
  // diagonals (host), all levels into one array
  long long dtot = 0;
  for (int l = 0; l < P->nul; ++l) dtot += P->u_total[l];
  std::vector<double> diag(dtot);
  for (int l = 0; l < P->nul; ++l)
    for (int k = 0; k < cnt; ++k) {
      auto D = elast_diag(P->ug[l][k]);
      std::copy(D.begin(), D.end(), diag.begin() + P->ug[l][k].doff);
    }
  upload(diag, B.u_dinv[0], s);
  // power iterations per level (compact layout, one time level)
  for (int l = 0; l < P->nul - 1; ++l) {
    std::vector<VSeg> segs;
    const UGridSeg* dseg;
    const LSeg* dls;
    double *x, *y;
    if (l == 0) {
      for (auto& g : P->ug0c) segs.push_back({g.voff, g.nu});
      dseg = P->d_ug0c; dls = P->d_ul0c; x = B.T1; y = B.T2;
    } else {
      for (auto& g : P->ug[l]) segs.push_back({g.voff, g.nu});
      dseg = P->d_ug[l]; dls = P->d_ul[l]; x = B.u_x[l]; y = B.u_y[l];
    }
    const int uv = uvar(l, 1);
    const int4* work = P->d_uwork[uv];
    const int nwork = (int)P->uwork[uv].size();
    const long long mx = P->u_max[l];
    auto apply = [&](double* xx, double* yy) {
      launch_uapply<double>(d, dseg, work, nwork, 1, 0, xx, nullptr, yy, P->d_uemat64, s, P->utile[uv]);
      launch_mul_dinv<double>(dls, cnt, 1, mx, B.u_dinv[0], yy, yy, s);
    };
    auto lam = power_max(P, apply, x, y, segs, s);
    std::vector<VSeg> dsegs;
    for (auto& g : P->ug[l]) dsegs.push_back({g.doff, g.nu});
    scale_dinv(P, B.u_dinv[0], dsegs, lam, s);
  }
  // coarse dense inverses
  std::vector<double> all(P->uAinv_len);
  for (int k = 0; k < cnt; ++k) {
    auto A = coarse_elast_matrix(P->ug[P->nul - 1][k]);
    std::copy(A.begin(), A.end(), all.begin() + P->ud[k].moff);
  }
  upload(all, P->uAinv, s);
  invert_on_device(P, P->d_gju, (int)P->gju.size(), P->u_maxn, P->uAinv, s);
  long long dt = 0;
  for (int l = 0; l < P->nul; ++l) dt += P->u_total[l];
  cast_to_f32(B.u_dinv[0], P->b32.u_dinv[0], dt, s);
}

void setup_solver(biot_problem_s* h, hipStream_t s) {
  PrecData* P = h->prec;
  if (!P->hdots)
    hip_check(hipHostMalloc((void**)&P->hdots, sizeof(double) * 3 * 64 * h->count, hipHostMallocDefault),
              "pinned dot buffer");
  // descriptors
  upload(P->pdg, P->d_pdg, s);
  for (int l = 0; l < P->npl; ++l) upload(P->pc[l], P->d_pc[l], s);
  for (int l = 0; l < P->nul; ++l) {
    upload(P->ug[l], P->d_ug[l], s);
    upload(P->ul[l], P->d_ul[l], s);
  }
  for (size_t v = 0; v < P->uwork.size(); ++v)
    if (!P->uwork[v].empty()) upload(P->uwork[v], P->d_uwork[v], s);
  upload(P->ug0c, P->d_ug0c, s);
  upload(P->ul0c, P->d_ul0c, s);
  for (int l = 0; l + 1 < P->nul; ++l) {
    for (int pass = 0; pass < P->dim; ++pass) upload(P->rp[l][pass], P->d_rp[l][pass], s);
    upload(P->up[l], P->d_up[l], s);
  }
  upload(P->utab_h, P->d_utab, s);
  upload(P->ud, P->d_ud, s);
  upload(P->pd, P->d_pd, s);
  upload(P->gju, P->d_gju, s);
  upload(P->gjp, P->d_gjp, s);
  upload(P->gseg, P->d_gseg, s);
  // level k = eigenbasis column lperm[k]: Q's columns and Q^-1's rows in level order
  for (int i = 0; i < 4; ++i)
    for (int k = 0; k < 4; ++k) {
      P->Q.m[i * 4 + k] = h->tc.Q[i * 4 + P->lperm[k]];
      P->Qi.m[k * 4 + i] = h->tc.Qi[P->lperm[k] * 4 + i];
    }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) { P->Qt.m[i * 4 + j] = P->Q.m[j * 4 + i]; P->Qit.m[i * 4 + j] = P->Qi.m[j * 4 + i]; }
  // initial guess of the next slab: the previous slab's solution extrapolated
  // linearly in time through its last two Radau levels (r >= 1), or its end
  // value (r = 0), evaluated at the next slab's levels 1 + s_i (units of tau)
  std::memset(&P->pred, 0, sizeof(P->pred));
  {
    const int r = h->r;
    for (int i = 0; i <= r; ++i) {
      if (r == 0) { P->pred.m[0] = 1.0; break; }
      const double s1 = h->tc.s[r], s0 = h->tc.s[r - 1];
      const double f = (1.0 + h->tc.s[i] - s1) / (s1 - s0);
      P->pred.m[i * 4 + r] = 1.0 + f;
      P->pred.m[i * 4 + r - 1] = -f;
    }
  }
  P->b64.kinv = h->d_kinv64;
  P->b32.kinv = h->d_kinv32;
  setup_elasticity(h, s);
  setup_pressure(h, s);
  hip_check(hipStreamSynchronize(s), "solver setup");
}

void refresh_solver(biot_problem_s* h, hipStream_t s) {
  h->prec->have_prev = false;
  setup_pressure(h, s);
  hip_check(hipStreamSynchronize(s), "solver refresh");
}

void destroy_solver(biot_problem_s* h) {
  PrecData* P = h->prec;
  if (P) {
    for (int q = 0; q < 12; ++q)
      if (P->gexec[q]) (void)hipGraphExecDestroy(P->gexec[q]);
    for (auto& kv : P->arnoldi) (void)hipGraphExecDestroy(kv.second);
    if (P->cap_stream) (void)hipStreamDestroy(P->cap_stream);
    if (P->hdots) (void)hipHostFree(P->hdots);
  }
  delete h->prec;
  h->prec = nullptr;
}

// ---------------------------------------------------------------------------
// the preconditioner  z = P^-1 r  (vectors of type T)
// ---------------------------------------------------------------------------
template <typename T>
static void p_vcycle(biot_problem_s* h, int l, int nl, hipStream_t s) {
  PrecData* P = h->prec;
  auto& B = bufs<T>(P);
  const int cnt = h->count;
  const int pd = pcdeg(h->dim);
  const ChebSeq cs = cheb_seq(kPLo, kPHi, pd);
  if (l == P->npl - 1) {
    dense_solve<T>(P->d_pd, cnt, nl, P->p_maxn, false, P->pAinv, B.pc_b[l], B.pc_x[l], s);
    return;
  }
  const PCellSeg* sg = P->d_pc[l];
  const long long mx = P->pc_max[l];
  T *x = B.pc_x[l], *b = B.pc_b[l], *r = B.pc_r[l], *d0 = B.pc_d0[l], *d1 = B.pc_d1[l];
  launch_pcell<T>(sg, cnt, nl, mx, kResInitZero, ChebCoef{cs.s0, 0, 0, 1}, B.pc_coef[l], B.pc_dinv[l], b, x, r,
                  nullptr, d0, s);
  for (int k = 0; k < pd; ++k) {
    launch_pcell<T>(sg, cnt, nl, mx, kStep, ChebCoef{0, cs.steps[k].first, cs.steps[k].second, 1}, B.pc_coef[l],
                    B.pc_dinv[l], b, x, r, (k & 1) ? d1 : d0, (k & 1) ? d0 : d1, s);
  }
  launch_p_restrict_cell<T>(sg, P->d_pc[l + 1], cnt, nl, P->pc_max[l + 1], r, B.pc_b[l + 1], s);
  p_vcycle<T>(h, l + 1, nl, s);
  launch_p_prolong_cell<T>(sg, P->d_pc[l + 1], cnt, nl, mx, omega_p(h->dim), B.pc_x[l + 1], x, s);
  launch_pcell<T>(sg, cnt, nl, mx, kResInit, ChebCoef{cs.s0, 0, 0, 1}, B.pc_coef[l], B.pc_dinv[l], b, x, r, nullptr,
                  d0, s);
  for (int k = 0; k < pd; ++k) {
    launch_pcell<T>(sg, cnt, nl, mx, kStep, ChebCoef{0, cs.steps[k].first, cs.steps[k].second, 1}, B.pc_coef[l],
                    B.pc_dinv[l], b, x, r, (k & 1) ? d1 : d0, (k & 1) ? d0 : d1, s);
  }
}

// S_j y = bsign * b on the DG level (x, b: slab layout p-blocks), levels j < nl
template <typename T>
static void p_solve(biot_problem_s* h, const T* b, T* x, int nl, hipStream_t s) {
  PrecData* P = h->prec;
  auto& B = bufs<T>(P);
  const int cnt = h->count, d = h->dim;
  const int pd = pdeg(h->dim);
  const ChebSeq cs = cheb_seq(kPLo, kPHi, pd);
  T *r = B.T1, *d0 = B.T2, *d1 = B.T3;
  launch_pdg<T>(d, h->d_inst, P->d_pdg, cnt, nl, P->pdg_max, kResInitZero, ChebCoef{cs.s0, 0, 0, -1}, B.dqinv,
                B.pdg_dinv, b, x, r, nullptr, d0, s);
  for (int k = 0; k < pd; ++k)
    launch_pdg<T>(d, h->d_inst, P->d_pdg, cnt, nl, P->pdg_max, kStep,
                  ChebCoef{0, cs.steps[k].first, cs.steps[k].second, -1}, B.dqinv, B.pdg_dinv, b, x, r,
                  (k & 1) ? d1 : d0, (k & 1) ? d0 : d1, s);
  launch_p_restrict_dg<T>(h->d_inst, P->d_pdg, P->d_pc[0], cnt, nl, P->pc_max[0], r, B.pc_b[0], s);
  p_vcycle<T>(h, 0, nl, s);
  launch_p_prolong_dg<T>(h->d_inst, P->d_pdg, P->d_pc[0], cnt, nl, P->pdg_max, omega_p(h->dim), B.pc_x[0], x, s);
  launch_pdg<T>(d, h->d_inst, P->d_pdg, cnt, nl, P->pdg_max, kResInit, ChebCoef{cs.s0, 0, 0, -1}, B.dqinv,
                B.pdg_dinv, b, x, r, nullptr, d0, s);
  for (int k = 0; k < pd; ++k)
    launch_pdg<T>(d, h->d_inst, P->d_pdg, cnt, nl, P->pdg_max, kStep,
                  ChebCoef{0, cs.steps[k].first, cs.steps[k].second, -1}, B.dqinv, B.pdg_dinv, b, x, r,
                  (k & 1) ? d1 : d0, (k & 1) ? d0 : d1, s);
}

// one V-cycle for tau A_l x = b at u level l (level 0: slab layout buffers given),
// time levels j < nl
template <typename T>
static void u_vcycle(biot_problem_s* h, int l, int nl, T* x, const T* b, T* r, T* d0, T* y, hipStream_t s) {
  PrecData* P = h->prec;
  auto& B = bufs<T>(P);
  const int cnt = h->count, d = h->dim;
  const int upre = udeg_pre(d), upost = udeg_post(d);
  const ChebSeq cs_pre = cheb_seq(kULo, kUHi, upre), cs_post = cheb_seq(kULo, kUHi, upost);
  if (l == P->nul - 1) {
    dense_solve<T>(P->d_ud, cnt, nl, P->u_maxn, true, P->uAinv, b, x, s);
    return;
  }
  const LSeg* ls = P->d_ul[l];
  const long long mx = P->u_max[l];
  const UGridSeg* gs = P->d_ug[l];
  const int uv = uvar(l, nl);
  const int4* work = P->d_uwork[uv];
  const int nwork = (int)P->uwork[uv].size();
  const T* dinv = B.u_dinv[0];
  // the ud Chebyshev steps from the direction in d0 (3D: the operator product and the
  // update in one sweep, the direction alternating between d0 and y)
  auto cheb_steps = [&](const ChebSeq& cs, int ud) {
    if (d == 3) {
      T *din = d0, *dout = y;
      for (int k = 0; k < ud; ++k) {
        launch_uapply3d_cheb<T>(gs, work, nwork, nl, P->utile[uv], din, x, r, dout, dinv, cs.steps[k].first,
                                cs.steps[k].second, uemat<T>(P), s);
        std::swap(din, dout);
      }
      return;
    }
    for (int k = 0; k < ud; ++k) {
      launch_uapply<T>(d, gs, work, nwork, nl, 0, d0, nullptr, y, uemat<T>(P), s, P->utile[uv]);
      cheb_update<T>(ls, cnt, nl, mx, 1, cs.steps[k].first, cs.steps[k].second, x, r, d0, y, dinv, nullptr, s);
    }
  };
  // pre-smoothing from x = 0
  cheb_update<T>(ls, cnt, nl, mx, 2, 0.0, cs_pre.s0, x, r, d0, nullptr, dinv, b, s);
  cheb_steps(cs_pre, upre);
  // restriction of r
  const T* in = r;
  for (int pass = 0; pass < d; ++pass) {
    T* out = (pass == d - 1) ? B.u_b[l + 1] : (pass == 0 ? B.u_t1[l] : B.u_t2[l]);
    launch_rpass<T>(P->d_rp[l][pass], cnt, nl, P->rp_max[l][pass], P->d_utab, in, out, s);
    in = out;
  }
  u_vcycle<T>(h, l + 1, nl, B.u_x[l + 1], B.u_b[l + 1], B.u_r[l + 1], B.u_d0[l + 1], B.u_y[l + 1], s);
  launch_uprolong<T>(P->d_up[l], cnt, nl, mx, P->d_utab, B.u_x[l + 1], x, s);
  // post-smoothing
  launch_uapply<T>(d, gs, work, nwork, nl, 1, x, b, r, uemat<T>(P), s, P->utile[uv]);
  cheb_update<T>(ls, cnt, nl, mx, 0, 0.0, cs_post.s0, x, r, d0, nullptr, dinv, nullptr, s);
  cheb_steps(cs_post, upost);
}

// the fixed-stress level solves of the levels j < nl at once: B.Wr -> B.Wz (B.Wr is read only).
// transpose: the blocks L_j^T.  Their pressure Schur complement (with the
// fixed-stress term) is that of L_j, and the sweep differs only in the
// displacement right-hand side, r_u + c_j b E p with c_j = the level shift
// instead of tau (the u-p couplings of L_j^T carry the coefficients of L_j's
// p-u couplings).
template <typename T>
static void level_solves(biot_problem_s* h, int nl, int qdeg, int transpose, hipStream_t s,
                         bool flow_only = false) {
  PrecData* P = h->prec;
  auto& B = bufs<T>(P);
  const int cnt = h->count, d = h->dim;
  // 1) pressure: S_j p = -r_p
  p_solve<T>(h, B.Wr, B.Wz, nl, s);
  // 2) coupling right-hand sides
  LevelCoef cu{};
  for (int j = 0; j < 4; ++j)
    cu.c[j] = transpose ? P->lalpha[j] + (P->pair_mode == BIOT_PAIR_DROP ? 0.0 : std::fabs(P->lbeta[j]))
                        : h->descs[0].tau;
  launch_coupling<T>(d, h->d_inst, cnt, nl, P->maxN, cu, B.Wr, B.Wz, B.Wf, B.Wf, s);
  // 3) flux: tau Mq q = f_q  (exact line solves, or Chebyshev-Jacobi of degree qdeg on the Gershgorin interval)
  if (qdeg == 0) {
    launch_mq_lines<T>(d, h->d_inst, cnt, nl, P->maxlines, P->maxcells_line, B.kinv, B.Wf, B.Wz, B.T1, s);
  } else {
    const ChebSeq cs = cheb_seq(kQLo, kQHi, qdeg);
    launch_mq<T>(d, h->d_inst, cnt, nl, P->maxN, kResInitZero, ChebCoef{cs.s0, 0, 0, 1}, B.kinv, nullptr, B.Wf, B.Wz,
                 B.T1, nullptr, B.T2, s);
    for (int k = 0; k < qdeg; ++k)
      launch_mq<T>(d, h->d_inst, cnt, nl, P->maxN, kStep, ChebCoef{0, cs.steps[k].first, cs.steps[k].second, 1},
                   B.kinv, nullptr, B.Wf, B.Wz, B.T1, (k & 1) ? B.T3 : B.T2, (k & 1) ? B.T2 : B.T3, s);
  }
  // 4) mechanics: tau A u = f_u  (one V-cycle)
  if (!flow_only) u_vcycle<T>(h, 0, nl, B.Wz, B.Wf, B.T1, B.T2, B.T4, s);
}

// Sub-systems of the fixed-stress iterative coupling (fixed_stress.hip): 0 = the slab
// system, 1 = the flow sub-system on (q, p), 2 = the mechanics sub-system tau A on u.
enum SubSystem { kSysSlab = 0, kSysFlow = 1, kSysMech = 2 };

// z = P^-1 r for the slab operator (transpose = 0) or its transpose (1).
// Forward: P^-1 = (Q kron I) blockdiag(L_j^-1) (Q^-1 kron I), T = Q Lambda_R Q^-1.
// Transposed: T^T = Q^-T Lambda_R^T Q^T, so P^-1 = (Q^-T kron I) blockdiag(L_j^-T) (Q^T kron I),
// and a pair block carries -beta where the forward one carries beta.
template <typename T>
static void apply_prec(biot_problem_s* h, const T* rin, T* z, int qdeg, int transpose, hipStream_t s,
                       int sys = kSysSlab) {
  PrecData* P = h->prec;
  auto& B = bufs<T>(P);
  const int nl = h->nl, cnt = h->count, d = h->dim;
  if (sys == kSysMech) {
    // one V-cycle per level on the u-rows (essential rows pass through, q and p rows zero)
    vfill<T>(B.Wz, T(0), h->slab_len, s);
    LevelCoef cu{};
    launch_coupling<T>(d, h->d_inst, cnt, nl, P->maxN, cu, rin, B.Wz, B.Wf, B.Wf, s);   // f_u: essential rows 0
    u_vcycle<T>(h, 0, nl, B.Wz, B.Wf, B.T1, B.T2, B.T4, s);
    Mat4 id{};
    for (int i = 0; i < 4; ++i) id.m[i * 5] = 1.0;
    launch_prec_finalize<T>(h->d_inst, cnt, P->maxN, nl, id, B.Wz, rin, z, s);
    launch_zero_rows<T>(h->d_inst, cnt, P->maxN, nl, 1, z, s);
    return;
  }
  // into the real block eigenbasis of T (of T^T)
  time_transform<T>(h->d_inst, cnt, P->maxN, nl, transpose ? P->Qt : P->Qi, rin, B.Wr, s);
  if (sys == kSysFlow) {
    // the flow part of every level solve (pressure Schur cycle, then the flux lines); the
    // pair couplings are dropped
    level_solves<T>(h, nl, qdeg, transpose, s, true);
    launch_prec_finalize<T>(h->d_inst, cnt, P->maxN, nl, P->Q, B.Wz, rin, z, s);
    launch_zero_rows<T>(h->d_inst, cnt, P->maxN, nl, 0, z, s);
    return;
  }
  if (P->pair_mode == BIOT_PAIR_PRESB && P->pairs.n > 0) {
    // pair blocks with their couplings (square-block factorisation), forward:
    // w = H^-1 (f - g), y = H^-1 (g + beta M_t w), x = (w + y, y); transposed:
    // w = H^-T (f + g), y = H^-T (g - beta M_t^T w), x = (w - y, y).  The levels
    // are ordered pair firsts, real levels, pair seconds: the first pass solves
    // the w of every pair with the real levels, the second the y of every pair
    // in the pair firsts' slots (same shift alpha + beta).
    const int np = P->pairs.n;
    launch_pair_split<T>(h->d_inst, cnt, P->maxN, P->pairs, transpose, B.Wr, s);
    level_solves<T>(h, nl - np, qdeg, transpose, s);
    launch_pair_couple<T>(d, h->d_inst, cnt, P->maxN, P->pairs, transpose, B.Wz, B.Ws, B.Wr, s);
    level_solves<T>(h, np, qdeg, transpose, s);
    launch_pair_join<T>(h->d_inst, cnt, P->maxN, P->pairs, transpose, B.Ws, B.Wz, s);
  } else {
    level_solves<T>(h, nl, qdeg, transpose, s);
  }
  // back to the nodal time basis; essential rows pass through
  launch_prec_finalize<T>(h->d_inst, cnt, P->maxN, nl, transpose ? P->Qit : P->Q, B.Wz, rin, z, s);
}

// z = P^-1 r through a captured graph: r is staged in a fixed buffer, the
// graph (captured once on a private stream, replayed on the caller's stream)
// runs the whole preconditioner and writes B.t.
template <typename T>
static void apply_prec_graph(biot_problem_s* h, const T* rin, T* z, int qdeg, int transpose, bool use_graph,
                             hipStream_t s, int sys = kSysSlab) {
  PrecData* P = h->prec;
  auto& B = bufs<T>(P);
  if (!use_graph || z != B.t) {
    apply_prec<T>(h, rin, z, qdeg, transpose, s, sys);
    return;
  }
  const int q = (std::is_same<T, float>::value ? 1 : 0) + (transpose ? 2 : 0) + 4 * sys;
  if (P->gexec[q] && P->gdeg[q] != qdeg) {
    hip_check(hipGraphExecDestroy(P->gexec[q]), "graph destroy");
    P->gexec[q] = nullptr;
  }
  if (!P->gexec[q]) {
    if (!P->cap_stream) hip_check(hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking), "capture stream");
    hip_check(hipStreamSynchronize(s), "pre-capture sync");
    hipGraph_t g;
    hip_check(hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeRelaxed), "begin capture");
    apply_prec<T>(h, B.pin, B.t, qdeg, transpose, P->cap_stream, sys);
    hip_check(hipStreamEndCapture(P->cap_stream, &g), "end capture");
    hip_check(hipGraphInstantiate(&P->gexec[q], g, nullptr, nullptr, 0), "graph instantiate");
    hip_check(hipGraphDestroy(g), "graph destroy");
    P->gdeg[q] = qdeg;
  }
  hip_check(hipMemcpyAsync(B.pin, rin, sizeof(T) * h->slab_len, hipMemcpyDeviceToDevice, s), "graph input");
  hip_check(hipGraphLaunch(P->gexec[q], s), "graph launch");
}

// ---------------------------------------------------------------------------
// GMRES (right preconditioned, restarted, CGS2), batched over instances
// ---------------------------------------------------------------------------
struct SolveCtl {
  double rtol;
  int maxit, restart, qdeg;
  bool graph;
  bool flex32 = false;   // FP64 flexible GMRES with the preconditioner applied in FP32
  int sys = kSysSlab;    // the system solved (SubSystem)
  bool lowsync = false;  // Gram-Schmidt with delayed reorthogonalisation (set by gmres)
};

// y = A x for the slab system or a fixed-stress sub-system (x zero outside the
// sub-system's rows; y zero there)
template <typename T>
static void sys_apply(biot_problem_s* h, const T* x, T* y, int transpose, int sys, hipStream_t s) {
  const int dt = std::is_same<T, float>::value ? 1 : 0;
  PrecData* P = h->prec;
  if (sys == kSysMech) {
    const int uv = uvar(0, h->nl);
    launch_uapply<T>(h->dim, P->d_ug[0], P->d_uwork[uv], (int)P->uwork[uv].size(), h->nl, 0, x, nullptr, y,
                     uemat<T>(P), s, P->utile[uv]);
    launch_zero_rows<T>(h->d_inst, h->count, P->maxN, h->nl, 1, y, s);
    return;
  }
  launch_apply(h, x, y, transpose, dt, s);
  if (sys == kSysFlow) launch_fs_flow_fix<T>(h->d_inst, h->count, P->maxN, h->nl, h->tm, x, y, s);
}

// y = b - A x into r (type T)
template <typename T>
static void residual(biot_problem_s* h, const T* b, const T* x, T* r, int transpose, hipStream_t s,
                     int sys = kSysSlab) {
  sys_apply<T>(h, x, r, transpose, sys, s);
  vaxpby<T>(1.0, b, -1.0, r, h->slab_len, s);
}

template <typename T>
static void seg_norms(PrecData* P, const T* v, int cnt, hipStream_t s, std::vector<double>& out) {
  seg_mdot<T, T>(v, 0, 1, v, P->d_gseg, cnt, dot_chunks(P->gmax), P->partial, P->dot3, s);
  std::vector<double> tmp(cnt * 64);
  hip_check(hipMemcpyAsync(tmp.data(), P->dot3, 8 * cnt * 64, hipMemcpyDeviceToHost, s), "norm read");
  hip_check(hipStreamSynchronize(s), "norm sync");
  out.resize(cnt);
  for (int k = 0; k < cnt; ++k) out[k] = std::sqrt(std::max(tmp[k * 64], 0.0));
}

// Dot-product sets hold 64 values per instance: the combined second pass (jj + 2
// values) fits up to Krylov index 62; the last index of a 64-step cycle takes a
// separate norm pass.
static inline bool pythagorean_norm(int jj) { return jj + 2 <= 64; }

// One Arnoldi step at Krylov index jj: w = A P^-1 v_jj, two classical
// Gram-Schmidt passes against v_0..v_jj, v_{jj+1} = w / ||w||.  The three dot
// product sets are also written to P->hdots for the host's Givens update.
template <typename T>
static void arnoldi_step(biot_problem_s* h, int jj, int transpose, const SolveCtl& ctl, hipStream_t s) {
  PrecData* P = h->prec;
  auto& B = bufs<T>(P);
  const int cnt = h->count;
  const long long S = h->slab_len;
  T* vj = B.V + (long long)jj * S;
  T* vn = B.V + (long long)(jj + 1) * S;
  bool done_prec = false;
  if constexpr (std::is_same<T, double>::value) {
    if (ctl.flex32) {
      // z_j = P32(v_j), kept in FP32 (the FP32 Krylov basis is unused in this mode);
      // the Arnoldi relation uses exactly these values, so x += Z y stays consistent
      auto& F = P->b32;
      float* zj = F.V + (long long)jj * S;
      vcast(vj, F.w, S, s);
      apply_prec<float>(h, F.w, F.t, ctl.qdeg, transpose, s);
      vcopy<float>(F.t, zj, S, s);
      vcast(zj, B.t, S, s);
      done_prec = true;
    }
  }
  if (!done_prec) apply_prec<T>(h, vj, B.t, ctl.qdeg, transpose, s, ctl.sys);
  sys_apply<T>(h, B.t, vn, transpose, ctl.sys, s);
  const int nch = dot_chunks(P->gmax);
  double* hd = P->hdots;
  if (ctl.lowsync) {
    // slot jj held the candidate (its operator image is in slot jj+1): one reduction
    // and one update sweep make slot jj final and slot jj+1 the next candidate
    dcgs_step<T>(B.V, S, jj, P->d_gseg, cnt, nch, P->partial, P->dot1, P->dot2, s, hd, hd + 64 * cnt);
    return;
  }
  seg_mdot<T, T>(B.V, S, jj + 1, vn, P->d_gseg, cnt, nch, P->partial, P->dot1, s, hd);
  if (jj + 1 <= kFuseK) {
    // the same two passes with three sweeps over the basis: the update of pass 1
    // fused with the dot products of pass 2 (which also give |w|^2), then the update
    // of pass 2 fused with the normalisation (norm by Pythagoras, as below)
    gs_update_dot<T, T>(B.V, S, jj + 1, P->dot1, vn, P->d_gseg, cnt, nch, P->partial, P->dot2, s, hd + 64 * cnt);
    gs_update_scale<T, T>(B.V, S, jj + 1, P->dot2, vn, P->d_gseg, cnt, P->gmax, s);
  } else if (pythagorean_norm(jj)) {
    seg_maxpy<T, T>(B.V, S, jj + 1, P->dot1, -1.0, vn, P->d_gseg, cnt, P->gmax, s);
    // second pass; w itself is basis slot jj+1, so the same pass gives |w|^2, and
    // the norm after the update follows by Pythagoras (the second-pass components
    // are at rounding level, so no cancellation)
    seg_mdot<T, T>(B.V, S, jj + 2, vn, P->d_gseg, cnt, nch, P->partial, P->dot2, s, hd + 64 * cnt);
    seg_maxpy<T, T>(B.V, S, jj + 1, P->dot2, -1.0, vn, P->d_gseg, cnt, P->gmax, s);
    seg_scale<T, T>(vn, vn, P->dot2, jj + 1, 3, P->d_gseg, cnt, P->gmax, s);   // 0 for a zero norm
  } else {
    seg_maxpy<T, T>(B.V, S, jj + 1, P->dot1, -1.0, vn, P->d_gseg, cnt, P->gmax, s);
    seg_mdot<T, T>(B.V, S, jj + 1, vn, P->d_gseg, cnt, nch, P->partial, P->dot2, s, hd + 64 * cnt);
    seg_maxpy<T, T>(B.V, S, jj + 1, P->dot2, -1.0, vn, P->d_gseg, cnt, P->gmax, s);
    seg_mdot<T, T>(vn, 0, 1, vn, P->d_gseg, cnt, nch, P->partial, P->dot3, s, hd + 128 * cnt);
    seg_scale<T, T>(vn, vn, P->dot3, 0, 2, P->d_gseg, cnt, P->gmax, s);
  }
}

// the Arnoldi step through a graph captured once per (index, variant), replayed on s
template <typename T>
static void arnoldi_step_graph(biot_problem_s* h, int jj, int transpose, const SolveCtl& ctl, hipStream_t s) {
  PrecData* P = h->prec;
  if (!ctl.graph) {
    arnoldi_step<T>(h, jj, transpose, ctl, s);
    return;
  }
  const long long key =
      ((((((long long)jj * 2 + (transpose ? 1 : 0)) * 2 + (ctl.flex32 ? 1 : 0)) * 2 +
         (std::is_same<T, float>::value ? 1 : 0)) * 128 + ctl.qdeg) * 3 + ctl.sys) * 2 + (ctl.lowsync ? 1 : 0);
  auto it = P->arnoldi.find(key);
  if (it == P->arnoldi.end()) {
    if (!P->cap_stream) hip_check(hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking), "capture stream");
    hip_check(hipStreamSynchronize(s), "pre-capture sync");
    hipGraph_t g;
    hip_check(hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeRelaxed), "begin capture");
    arnoldi_step<T>(h, jj, transpose, ctl, P->cap_stream);
    hip_check(hipStreamEndCapture(P->cap_stream, &g), "end capture");
    hipGraphExec_t ge;
    hip_check(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0), "graph instantiate");
    hip_check(hipGraphDestroy(g), "graph destroy");
    it = P->arnoldi.emplace(key, ge).first;
  }
  hip_check(hipGraphLaunch(it->second, s), "graph launch");
}

// wait for the stream by polling (the host has nothing else to do, and the
// Arnoldi loop waits once per iteration)
static void spin_wait(hipStream_t s) {
  hipError_t e;
  while ((e = hipStreamQuery(s)) == hipErrorNotReady) {
  }
  hip_check(e, "stream wait");
}

template <typename T>
static void gmres(biot_problem_s* h, const T* b, T* x, int transpose, const SolveCtl& ctl, std::vector<int>& its,
                  std::vector<int>& rst, std::vector<double>& relres, std::vector<int>& status, hipStream_t s) {
  PrecData* P = h->prec;
  auto& B = bufs<T>(P);
  const int cnt = h->count;
  const long long S = h->slab_len;
  const int m = std::min(std::max(ctl.restart, 1), kMaxRestart);
  its.assign(cnt, 0); rst.assign(cnt, 0); relres.assign(cnt, 0.0); status.assign(cnt, BIOT_OK);
  std::vector<double> bn, beta;
  seg_norms<T>(P, b, cnt, s, bn);
  for (int k = 0; k < cnt; ++k)
    if (!std::isfinite(bn[k])) throw BiotError{BIOT_ERR_NONFINITE, "right-hand side is not finite"};
  residual<T>(h, b, x, B.r, transpose, s, ctl.sys);
  seg_norms<T>(P, B.r, cnt, s, beta);
  std::vector<char> done(cnt, 0);
  for (int k = 0; k < cnt; ++k) {
    relres[k] = bn[k] > 0 ? beta[k] / bn[k] : 0.0;
    if (bn[k] == 0.0 || beta[k] <= ctl.rtol * bn[k]) done[k] = 1;
  }
  std::vector<double> H((size_t)cnt * (kMaxRestart + 1) * kMaxRestart), cs(cnt * kMaxRestart), sn(cnt * kMaxRestart),
      g(cnt * (kMaxRestart + 1));
  std::vector<double> coef(cnt * 64);
  std::vector<int> stall(cnt, 0);
  int total = 0;
  // Gram-Schmidt with delayed reorthogonalisation (dcgs_step) for restart lengths whose
  // dot sets fit the 64 slots per instance.  The operator is applied to the candidate
  // u_j of each slot: right preconditioning reconstructs A P^-1 of the final vector (the
  // columns below); the flexible mode keeps z_j = P(u_j) itself, whose image
  // w = V b + e v + nu_j u_{j+1} gives its column directly.
  SolveCtl c = ctl;
  c.lowsync = m <= kLowSyncMax;
  const bool flex = ctl.flex32;
  // delayed mode: unrotated Hessenberg columns, the provisional column of the last step,
  // and whether a column was already completed by an early check of convergence
  std::vector<double> Hr(c.lowsync ? (size_t)cnt * (kMaxRestart + 1) * kMaxRestart : 0),
      hp(c.lowsync ? (size_t)cnt * (kMaxRestart + 1) : 0);
  std::vector<char> early(cnt, 0);
  std::vector<double> nuc(cnt, 1.0);   // flexible mode: nu of the candidate whose column is provisional
  while (true) {
    bool all = true;
    for (int k = 0; k < cnt; ++k) all = all && done[k];
    if (all || total >= ctl.maxit) break;
    // v0 = r / ||r||  (dot3 still holds ||r||^2 per instance from seg_norms)
    seg_scale<T, T>(B.r, B.V, P->dot3, 0, 2, P->d_gseg, cnt, P->gmax, s);
    std::vector<int> jk(cnt, 0);
    std::vector<char> act(cnt);
    for (int k = 0; k < cnt; ++k) {
      act[k] = !done[k];
      g[k * (kMaxRestart + 1)] = beta[k];
      ++rst[k];
    }
    int jj = 0;
    // column cc of instance k from its unrotated entries raw[0..cc+1]: stored, rotated,
    // the residual estimate updated; the instance stops when it has converged
    auto complete_column = [&](int k, int cc, const double* raw) {
      double* Hk = &H[(size_t)k * (kMaxRestart + 1) * kMaxRestart];
      double* Hrk = &Hr[(size_t)k * (kMaxRestart + 1) * kMaxRestart];
      double col[kMaxRestart + 1];
      for (int i = 0; i <= cc + 1; ++i) {
        Hrk[i * kMaxRestart + cc] = raw[i];
        col[i] = raw[i];
      }
      for (int i = 0; i < cc; ++i) {
        const double cr = cs[k * kMaxRestart + i], sv = sn[k * kMaxRestart + i];
        const double t0 = cr * col[i] + sv * col[i + 1];
        col[i + 1] = -sv * col[i] + cr * col[i + 1];
        col[i] = t0;
      }
      const double den = std::hypot(col[cc], col[cc + 1]);
      const double cr = den > 0 ? col[cc] / den : 1.0, sv = den > 0 ? col[cc + 1] / den : 0.0;
      cs[k * kMaxRestart + cc] = cr;
      sn[k * kMaxRestart + cc] = sv;
      col[cc] = den;
      for (int i = 0; i <= cc; ++i) Hk[i * kMaxRestart + cc] = col[i];
      double* gk = &g[k * (kMaxRestart + 1)];
      gk[cc + 1] = -sv * gk[cc];
      gk[cc] = cr * gk[cc];
      jk[k] = cc + 1;
      ++its[k];
      if (std::fabs(gk[cc + 1]) <= ctl.rtol * bn[k] || raw[cc + 1] == 0.0) act[k] = 0;
    };
    for (int k = 0; k < cnt; ++k) early[k] = 0;
    for (; c.lowsync && jj < m && total < ctl.maxit; ++jj) {
      // slot jj becomes final, which completes column jj - 1; column jj is provisional
      arnoldi_step_graph<T>(h, jj, transpose, c, s);
      spin_wait(s);
      bool check = false;
      for (int k = 0; k < cnt; ++k) {
        const double* d = P->hdots + k * 64;
        const double* a = d;
        const double* bb = d + jj;
        double n2 = d[2 * jj], ab = 0.0;
        for (int i = 0; i < jj; ++i) {
          n2 -= a[i] * a[i];
          ab += a[i] * bb[i];
        }
        const double nu = std::sqrt(std::max(n2, 0.0));
        const double un2 = P->hdots[64 * cnt + k * 64];
        if (!std::isfinite(nu) || !std::isfinite(un2)) throw BiotError{BIOT_ERR_NONFINITE, "non-finite Krylov vector"};
        if (!act[k]) continue;
        double* hpk = &hp[(size_t)k * (kMaxRestart + 1)];
        if (jj == 0) {
          g[k * (kMaxRestart + 1)] *= nu;   // v0 / nu is the final first vector
        } else if (!early[k]) {
          // completed with the second-pass coefficients a of the candidate (flexible
          // mode: scaled by the previous candidate's nu, as that candidate was)
          const double sc = flex ? nuc[k] : 1.0;
          double raw[kMaxRestart + 1];
          for (int i = 0; i < jj; ++i) raw[i] = hpk[i] + sc * a[i];
          raw[jj] = sc * nu;
          complete_column(k, jj - 1, raw);
        }
        early[k] = 0;
        if (!act[k] || nu == 0.0) continue;
        // provisional column jj: ([V^T w; v.w] - Hbar a) / nu (unrotated Hbar = columns
        // 0..jj-1); flexible mode: [V^T w; v.w]
        const double* Hrk = &Hr[(size_t)k * (kMaxRestart + 1) * kMaxRestart];
        for (int i = 0; i <= jj; ++i) {
          const double wi = i < jj ? bb[i] : (d[2 * jj + 1] - ab) / nu;
          if (flex) {
            hpk[i] = wi;
            continue;
          }
          double ha = 0.0;
          for (int cc = std::max(i - 1, 0); cc < jj; ++cc) ha += Hrk[i * kMaxRestart + cc] * a[cc];
          hpk[i] = (wi - ha) / nu;
        }
        nuc[k] = nu;
        // predicted estimate with |u_{jj+1}| for the subdiagonal (an upper bound)
        double col[kMaxRestart + 1];
        for (int i = 0; i <= jj; ++i) col[i] = hpk[i];
        col[jj + 1] = (flex ? nu : 1.0) * std::sqrt(std::max(un2, 0.0));
        for (int i = 0; i < jj; ++i) {
          const double cr = cs[k * kMaxRestart + i], sv = sn[k * kMaxRestart + i];
          const double t0 = cr * col[i] + sv * col[i + 1];
          col[i + 1] = -sv * col[i] + cr * col[i + 1];
          col[i] = t0;
        }
        const double den = std::hypot(col[jj], col[jj + 1]);
        const double est = den > 0 ? std::fabs(g[k * (kMaxRestart + 1) + jj]) * col[jj + 1] / den : 0.0;
        if (est <= ctl.rtol * bn[k]) check = true;
      }
      ++total;
      bool any = false;
      for (int k = 0; k < cnt; ++k) any = any || act[k];
      if (!any) break;
      if (check || jj == m - 1 || total >= ctl.maxit) {
        // complete column jj now: the second-pass coefficients of the candidate in slot jj+1
        const int nch = dot_chunks(P->gmax);
        seg_mdot<T, T>(B.V, S, jj + 2, B.V + (long long)(jj + 1) * S, P->d_gseg, cnt, nch, P->partial, P->dot3, s,
                       P->hdots + 128 * cnt);
        spin_wait(s);
        for (int k = 0; k < cnt; ++k) {
          if (!act[k]) continue;
          const double* d = P->hdots + 128 * cnt + k * 64;
          const double* hpk = &hp[(size_t)k * (kMaxRestart + 1)];
          const double sc = flex ? nuc[k] : 1.0;
          double raw[kMaxRestart + 1], n2 = d[jj + 1];
          for (int i = 0; i <= jj; ++i) {
            raw[i] = hpk[i] + sc * d[i];
            n2 -= d[i] * d[i];
          }
          raw[jj + 1] = sc * std::sqrt(std::max(n2, 0.0));
          complete_column(k, jj, raw);
          early[k] = 1;
        }
        any = false;
        for (int k = 0; k < cnt; ++k) any = any || act[k];
        if (!any) { ++jj; break; }
      }
    }
    for (; !c.lowsync && jj < m && total < ctl.maxit; ++jj) {
      arnoldi_step_graph<T>(h, jj, transpose, c, s);
      spin_wait(s);
      const double* h1 = P->hdots;
      const double* h2 = P->hdots + 64 * cnt;
      const double* hn = P->hdots + 128 * cnt;
      for (int k = 0; k < cnt; ++k) {
        double n2;
        if (pythagorean_norm(jj)) {
          n2 = h2[k * 64 + jj + 1];
          for (int i = 0; i <= jj; ++i) n2 -= h2[k * 64 + i] * h2[k * 64 + i];
        } else {
          n2 = hn[k * 64];
        }
        const double nrm = std::sqrt(std::max(n2, 0.0));
        if (!std::isfinite(nrm)) throw BiotError{BIOT_ERR_NONFINITE, "non-finite Krylov vector"};
        if (!act[k]) continue;
        double* Hk = &H[(size_t)k * (kMaxRestart + 1) * kMaxRestart];
        double col[kMaxRestart + 1];
        for (int i = 0; i <= jj; ++i) col[i] = h1[k * 64 + i] + h2[k * 64 + i];
        col[jj + 1] = nrm;
        // previous rotations
        for (int i = 0; i < jj; ++i) {
          const double c = cs[k * kMaxRestart + i], sv = sn[k * kMaxRestart + i];
          const double t0 = c * col[i] + sv * col[i + 1];
          col[i + 1] = -sv * col[i] + c * col[i + 1];
          col[i] = t0;
        }
        const double den = std::hypot(col[jj], col[jj + 1]);
        const double c = den > 0 ? col[jj] / den : 1.0, sv = den > 0 ? col[jj + 1] / den : 0.0;
        cs[k * kMaxRestart + jj] = c;
        sn[k * kMaxRestart + jj] = sv;
        col[jj] = den;
        col[jj + 1] = 0.0;
        for (int i = 0; i <= jj; ++i) Hk[i * kMaxRestart + jj] = col[i];
        double* gk = &g[k * (kMaxRestart + 1)];
        gk[jj + 1] = -sv * gk[jj];
        gk[jj] = c * gk[jj];
        jk[k] = jj + 1;
        ++its[k];
        const double est = std::fabs(gk[jj + 1]);
        if (est <= ctl.rtol * bn[k] || nrm == 0.0) act[k] = 0;
      }
      ++total;
      bool any = false;
      for (int k = 0; k < cnt; ++k) any = any || act[k];
      if (!any) { ++jj; break; }
    }
    // x += P^-1 (V y)
    std::fill(coef.begin(), coef.end(), 0.0);
    int kmax = 0;
    for (int k = 0; k < cnt; ++k) {
      if (jk[k] == 0) continue;
      const double* Hk = &H[(size_t)k * (kMaxRestart + 1) * kMaxRestart];
      const double* gk = &g[k * (kMaxRestart + 1)];
      const int n = jk[k];
      std::vector<double> y(n);
      for (int i = n - 1; i >= 0; --i) {
        double v = gk[i];
        for (int q = i + 1; q < n; ++q) v -= Hk[i * kMaxRestart + q] * y[q];
        y[i] = v / Hk[i * kMaxRestart + i];
      }
      for (int i = 0; i < n; ++i) coef[k * 64 + i] = y[i];
      kmax = std::max(kmax, n);
    }
    if (kmax > 0) {
      upload(coef, P->coef, s);
      bool done_update = false;
      if constexpr (std::is_same<T, double>::value) {
        if (ctl.flex32) {      // x += Z y
          seg_maxpy<float, double>(P->b32.V, S, kmax, P->coef, 1.0, x, P->d_gseg, cnt, P->gmax, s);
          done_update = true;
        }
      }
      if (!done_update) {
        hip_check(hipMemsetAsync(B.w, 0, sizeof(T) * S, s), "zero");
        seg_maxpy<T, T>(B.V, S, kmax, P->coef, 1.0, B.w, P->d_gseg, cnt, P->gmax, s);
        apply_prec_graph<T>(h, B.w, B.t, ctl.qdeg, transpose, ctl.graph, s, ctl.sys);
        vaxpby<T>(1.0, B.t, 1.0, x, S, s);
      }
    }
    std::vector<double> prev = beta;
    residual<T>(h, b, x, B.r, transpose, s, ctl.sys);
    seg_norms<T>(P, B.r, cnt, s, beta);
    for (int k = 0; k < cnt; ++k) {
      if (!std::isfinite(beta[k])) throw BiotError{BIOT_ERR_NONFINITE, "non-finite residual"};
      relres[k] = bn[k] > 0 ? beta[k] / bn[k] : 0.0;
      if (bn[k] == 0.0 || beta[k] <= ctl.rtol * bn[k]) { done[k] = 1; continue; }
      // rounding floor of b - A x: two restart cycles in a row that do not halve the true residual
      if (!done[k] && jk[k] > 0) {
        stall[k] = (beta[k] > 0.5 * prev[k]) ? stall[k] + 1 : 0;
        if (stall[k] >= 2) { done[k] = 2; }
      }
    }
  }
  for (int k = 0; k < cnt; ++k) {
    if (done[k] == 1) status[k] = BIOT_OK;
    else if (done[k] == 2) status[k] = (relres[k] <= 100.0 * ctl.rtol) ? BIOT_OK : BIOT_ERR_NOCONV;
    else status[k] = BIOT_ERR_NOCONV;
  }
}



// FP64 or mixed solve of A x = b (device double vectors)
static void solve_impl(biot_problem_s* h, const double* b, double* x, int transpose, const biot_solve_opts* o,
                       biot_solve_info* info, hipStream_t s) {
  biot_solve_opts opts;
  opts.rtol = 1e-12; opts.maxit = 1000; opts.restart = 30; opts.precision = BIOT_FP64;
  opts.inner_rtol = 1e-2; opts.max_refine = 30; opts.cheb_degree = -1; opts.graph = 1;
  if (o) opts = *o;
  if (!(opts.rtol > 0) || !std::isfinite(opts.rtol)) throw BiotError{BIOT_ERR_ARG, "rtol must be > 0"};
  if (opts.maxit < 1) throw BiotError{BIOT_ERR_ARG, "maxit must be >= 1"};
  if (opts.restart < 1 || opts.restart > kMaxRestart) throw BiotError{BIOT_ERR_ARG, "restart must be in 1..64"};
  if (opts.precision != BIOT_FP64 && opts.precision != BIOT_MIXED && opts.precision != BIOT_FP32_PREC)
    throw BiotError{BIOT_ERR_ARG, "unknown precision"};
  if (opts.cheb_degree < -1 || opts.cheb_degree > 64) throw BiotError{BIOT_ERR_ARG, "cheb_degree must be in -1..64"};
  if (opts.cheb_degree == -1) {
    // exact line solves: one wavefront per line up to kPcrMaxCells cells per line;
    // longer lines take one thread each, which pays only when the lines of all
    // instances and time levels fill the device (Chebyshev-Jacobi otherwise)
    const long long lines = (long long)h->count * h->nl * h->prec->maxlines;
    const bool wave_lines = h->prec->maxcells_line <= kPcrMaxCells;
    opts.cheb_degree = (wave_lines || lines >= kLineSolveMinLines) ? 0 : kQDegDefault;
  }
  const int cnt = h->count;
  std::vector<int> its, rst, st;
  std::vector<double> rr;
  if (opts.precision == BIOT_FP64 || opts.precision == BIOT_FP32_PREC) {
    SolveCtl ctl{opts.rtol, opts.maxit, opts.restart, opts.cheb_degree, opts.graph != 0,
                 opts.precision == BIOT_FP32_PREC};
    gmres<double>(h, b, x, transpose, ctl, its, rst, rr, st, s);
    for (int k = 0; k < cnt; ++k) {
      info[k].iterations = its[k]; info[k].restarts = rst[k]; info[k].ir_sweeps = 0;
      info[k].status = st[k]; info[k].rel_residual = rr[k];
    }
  } else {
    if (!(opts.inner_rtol > 0) || opts.max_refine < 1) throw BiotError{BIOT_ERR_ARG, "bad mixed-precision controls"};
    PrecData* P = h->prec;
    auto& B64 = P->b64;
    auto& B32 = P->b32;
    std::vector<double> bn, rn;
    seg_norms<double>(P, b, cnt, s, bn);
    std::vector<int> tot(cnt, 0), totr(cnt, 0), sweeps(cnt, 0);
    std::vector<char> done(cnt, 0);
    std::vector<double> rprev(cnt, 1e300);
    for (int sw = 0; sw <= opts.max_refine; ++sw) {
      residual<double>(h, b, x, B64.r, transpose, s);
      seg_norms<double>(P, B64.r, cnt, s, rn);
      bool all = true;
      for (int k = 0; k < cnt; ++k) {
        if (!std::isfinite(rn[k])) throw BiotError{BIOT_ERR_NONFINITE, "non-finite residual"};
        if (bn[k] == 0.0 || rn[k] <= opts.rtol * bn[k]) done[k] = 1;
        // refinement no longer reduces the FP64 residual: rounding floor reached
        if (!done[k] && rn[k] > 0.5 * rprev[k] && rn[k] <= 100.0 * opts.rtol * bn[k]) done[k] = 1;
        rprev[k] = rn[k];
        all = all && done[k];
      }
      if (all || sw == opts.max_refine) break;
      vcast(B64.r, B32.bin, h->slab_len, s);
      hip_check(hipMemsetAsync(B32.xin, 0, sizeof(float) * h->slab_len, s), "zero");
      SolveCtl ctl{opts.inner_rtol, opts.maxit, opts.restart, opts.cheb_degree, opts.graph != 0};
      float* d32 = B32.xin;
      gmres<float>(h, B32.bin, d32, transpose, ctl, its, rst, rr, st, s);
      vacc(d32, x, h->slab_len, s);
      for (int k = 0; k < cnt; ++k) { tot[k] += its[k]; totr[k] += rst[k]; if (!done[k]) ++sweeps[k]; }
    }
    for (int k = 0; k < cnt; ++k) {
      info[k].iterations = tot[k]; info[k].restarts = totr[k]; info[k].ir_sweeps = sweeps[k];
      info[k].status = done[k] ? BIOT_OK : BIOT_ERR_NOCONV;
      info[k].rel_residual = bn[k] > 0 ? rn[k] / bn[k] : 0.0;
    }
  }
}

// Fixed-stress iterative coupling of one slab system (section "Iterative Coupling
// Approach"), as a stationary iteration on the slab residual:
//   flow:      solve the flow sub-system (fixed-stress term L Mp in the mass rows) for
//              the (q, p) correction of the current residual,
//   mechanics: solve tau A u_i = (b - A x)_u per level with the new pressure,
// until ||b - A x|| <= rtol ||b||.  Each sub-system is solved by restarted GMRES
// preconditioned with its part of the level solves (flow: pressure Schur cycle and
// flux lines in the eigenbasis of T; mechanics: one V-cycle per level).
static void fixed_stress_impl(biot_problem_s* h, const double* b, double* x, const biot_fs_opts* o,
                              biot_fs_info* info, hipStream_t s) {
  biot_fs_opts opts;
  opts.rtol = 1e-12; opts.max_outer = 1000; opts.inner_rtol = 1e-4; opts.inner_maxit = 500;
  if (o) opts = *o;
  if (!(opts.rtol > 0) || !std::isfinite(opts.rtol)) throw BiotError{BIOT_ERR_ARG, "rtol must be > 0"};
  if (!(opts.inner_rtol > 0) || !(opts.inner_rtol < 1)) throw BiotError{BIOT_ERR_ARG, "inner_rtol must be in (0, 1)"};
  if (opts.max_outer < 1 || opts.inner_maxit < 1) throw BiotError{BIOT_ERR_ARG, "iteration limits must be >= 1"};
  PrecData* P = h->prec;
  auto& B = P->b64;
  const int cnt = h->count, nl = h->nl;
  const long long S = h->slab_len;
  double* R = B.bin;   // outer residual / sub-system right-hand side
  double* D = B.xin;   // sub-system correction
  const long long lines = (long long)cnt * nl * P->maxlines;
  const int qdeg = (P->maxcells_line <= kPcrMaxCells || lines >= kLineSolveMinLines) ? 0 : kQDegDefault;
  std::vector<double> bn, rn;
  seg_norms<double>(P, b, cnt, s, bn);
  for (int k = 0; k < cnt; ++k)
    if (!std::isfinite(bn[k])) throw BiotError{BIOT_ERR_NONFINITE, "right-hand side is not finite"};
  std::vector<int> its, rst, st, fl(cnt, 0), me(cnt, 0), outer(cnt, 0);
  std::vector<double> rr;
  std::vector<char> done(cnt, 0);
  for (int it = 0;; ++it) {
    residual<double>(h, b, x, R, 0, s);
    seg_norms<double>(P, R, cnt, s, rn);
    bool all = true;
    for (int k = 0; k < cnt; ++k) {
      if (!std::isfinite(rn[k])) throw BiotError{BIOT_ERR_NONFINITE, "non-finite residual"};
      if (bn[k] == 0.0 || rn[k] <= opts.rtol * bn[k]) done[k] = 1;
      all = all && done[k];
    }
    if (all || it == opts.max_outer) break;
    for (int k = 0; k < cnt; ++k) if (!done[k]) ++outer[k];
    for (int sys : {kSysFlow, kSysMech}) {
      if (sys == kSysMech) residual<double>(h, b, x, R, 0, s);
      launch_zero_rows<double>(h->d_inst, cnt, P->maxN, nl, sys == kSysFlow ? 0 : 1, R, s);
      vfill<double>(D, 0.0, S, s);
      SolveCtl ctl{opts.inner_rtol, opts.inner_maxit, 30, qdeg, true};
      ctl.sys = sys;
      gmres<double>(h, R, D, 0, ctl, its, rst, rr, st, s);
      for (int k = 0; k < cnt; ++k) (sys == kSysFlow ? fl : me)[k] += its[k];
      vaxpby<double>(1.0, D, 1.0, x, S, s);
    }
  }
  for (int k = 0; k < cnt; ++k) {
    info[k].outer = outer[k]; info[k].flow_iterations = fl[k]; info[k].mech_iterations = me[k];
    info[k].rel_residual = bn[k] > 0 ? rn[k] / bn[k] : 0.0;
    info[k].status = done[k] ? BIOT_OK : BIOT_ERR_NOCONV;
  }
}

static long long max_cells(const biot_problem_s* h) {
  long long m = 0;
  for (auto& I : h->inst) m = I.ncells > m ? I.ncells : m;
  return m;
}

void launch_slab_rhs(const biot_problem_s* h, const double* state, double t_start, double* rhs, hipStream_t s) {
  hip_check(hipMemsetAsync(rhs, 0, sizeof(double) * h->slab_len, s), "rhs clear");
  launch_rhs(h->d_inst, h->count, max_cells(h), h->tm, h->nl, t_start, state, rhs, s);
  hip_check(hipGetLastError(), "rhs launch");
}

// ---------------------------------------------------------------------------
// Static scratch of biot_misfit_noalloc: the sensor weights and residuals that
// biot_misfit keeps in the handle's workspace live here instead.  One copy per
// GPU, held until the process ends; host code reaches it only through the
// per-device address from hipGetSymbolAddress (the array's name is a host-side
// stand-in, not a device address).
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = size_t(4) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// address of this device's copy of the scratch array (looked up once per
// device, with that device current)
void* scratch_ptr() {
  int dev = 0;
  hip_check(hipGetDevice(&dev), "current device");
  if (dev < 0 || dev >= kMaxDevices) throw BiotError{BIOT_ERR_DEVICE, "device index beyond the scratch table"};
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "scratch symbol address");
    if (!p) throw BiotError{BIOT_ERR_DEVICE, "scratch symbol has no device address"};
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

static size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

// sensor weights (host): containing cell (floor, clipped), DG-Q1 Lagrange weights
static std::vector<SensorW> sensor_weights(biot_problem_s* h, const double* sensors_xyz, int nsens) {
  const int cnt = h->count, d = h->dim;
  std::vector<SensorW> sw((size_t)cnt * nsens);
  for (int k = 0; k < cnt; ++k) {
    const InstDev& I = h->inst[k];
    for (int q = 0; q < nsens; ++q) {
      SensorW w;
      std::memset(&w, 0, sizeof(w));
      int ce[3] = {0, 0, 0};
      double sl[3] = {0, 0, 0};
      for (int e = 0; e < d; ++e) {
        const double xv = sensors_xyz[q * d + e];
        if (!std::isfinite(xv)) throw BiotError{BIOT_ERR_ARG, "sensor coordinates must be finite"};
        int c = (int)std::floor(xv / I.h[e]);
        c = std::min(std::max(c, 0), I.n[e] - 1);
        ce[e] = c;
        sl[e] = xv / I.h[e] - c;
      }
      for (int g = 0; g < (d == 3 ? 8 : 4); ++g) {
        const int gg[3] = {g & 1, (g >> 1) & 1, (g >> 2) & 1};
        double wt = 1.0;
        for (int e = 0; e < d; ++e) wt *= psi(gg[e], sl[e]);
        w.idx[g] = (2 * ce[0] + gg[0]) + (long long)I.sp[0] * ((2 * ce[1] + gg[1]) + (long long)I.sp[1] * (d == 3 ? 2 * ce[2] + gg[2] : 0));
        w.w[g] = wt;
      }
      sw[(size_t)k * nsens + q] = w;
    }
  }
  return sw;
}

}  // namespace bt

using namespace bt;

#define BIOT_TRY try {
#define BIOT_CATCH                                         \
  }                                                        \
  catch (const BiotError& e) {                             \
    set_error(e.msg);                                      \
    return e.st;                                           \
  }                                                        \
  catch (const std::exception& e) {                        \
    set_error(std::string("internal error: ") + e.what()); \
    return BIOT_ERR_ARG;                                   \
  }                                                        \
  return BIOT_OK;

static void need(bool c, const char* m) {
  if (!c) throw BiotError{BIOT_ERR_ARG, m};
}

static biot_status worst(const biot_solve_info* info, int n) {
  int st = BIOT_OK;
  for (int k = 0; k < n; ++k)
    if (info[k].status != BIOT_OK) st = info[k].status;
  return (biot_status)st;
}

extern "C" {

biot_status biot_get_tuning(biot_problem h, biot_tuning* out) {
  BIOT_TRY
  need(h && out, "handle and out must be non-null");
  std::memset(out, 0, sizeof(*out));
  out->apply_variant[0] = h->variant[0];
  out->apply_variant[1] = h->variant[1];
  out->n_variants = h->nvariants;
  BIOT_CATCH
}

// captured Arnoldi steps hold the operator kernel of the tile variant in use
// when they were captured: drop them when the selection changes (every solve
// has completed by then: the solver waits on its stream before returning)
static void drop_arnoldi_graphs(PrecData* P) {
  for (auto& kv : P->arnoldi) (void)hipGraphExecDestroy(kv.second);
  P->arnoldi.clear();
}

biot_status biot_set_tuning(biot_problem h, const biot_tuning* t) {
  BIOT_TRY
  need(h && t, "handle and tuning must be non-null");
  for (int q = 0; q < 2; ++q)
    need(t->apply_variant[q] >= 0 && t->apply_variant[q] < h->nvariants, "apply_variant out of range");
  if (h->variant[0] != t->apply_variant[0] || h->variant[1] != t->apply_variant[1]) drop_arnoldi_graphs(h->prec);
  h->variant[0] = t->apply_variant[0];
  h->variant[1] = t->apply_variant[1];
  BIOT_CATCH
}

biot_status biot_autotune(biot_problem h, int32_t reps, biot_tuning* out, void* stream) {
  BIOT_TRY
  need(h, "handle is null");
  need(reps >= 1 && reps <= 1000, "reps must be in 1..1000");
  hipStream_t s = (hipStream_t)stream;
  PrecData* P = h->prec;
  biot_tuning res;
  std::memset(&res, 0, sizeof(res));
  res.n_variants = h->nvariants;
  hipEvent_t e0, e1;
  hip_check(hipEventCreate(&e0), "event");
  hip_check(hipEventCreate(&e1), "event");
  const int saved[2] = {h->variant[0], h->variant[1]};
  for (int dt = 0; dt < 2; ++dt) {
    const void* x = dt ? (const void*)P->b32.T1 : (const void*)P->b64.T1;
    void* y = dt ? (void*)P->b32.T2 : (void*)P->b64.T2;
    if (dt) vfill<float>(P->b32.T1, 0.5f, h->slab_len, s);
    else vfill<double>(P->b64.T1, 0.5, h->slab_len, s);
    int best = saved[dt];
    double best_us = 0.0;
    for (int v = 0; v < h->nvariants; ++v) {
      h->variant[dt] = v;
      launch_apply(h, x, y, 0, dt, s);     // warm-up
      hip_check(hipEventRecord(e0, s), "event record");
      for (int q = 0; q < reps; ++q) launch_apply(h, x, y, 0, dt, s);
      hip_check(hipEventRecord(e1, s), "event record");
      hip_check(hipEventSynchronize(e1), "event sync");
      float ms = 0.0f;
      hip_check(hipEventElapsedTime(&ms, e0, e1), "event time");
      const double us = 1e3 * ms / reps;
      res.apply_us[dt][v] = us;
      if (v == 0 || us < best_us) { best_us = us; best = v; }
    }
    h->variant[dt] = best;
    res.apply_variant[dt] = best;
  }
  hip_check(hipEventDestroy(e0), "event");
  hip_check(hipEventDestroy(e1), "event");
  if (h->variant[0] != saved[0] || h->variant[1] != saved[1]) drop_arnoldi_graphs(P);
  if (out) *out = res;
  BIOT_CATCH
}

biot_status biot_elasticity_apply(biot_problem h, const void* x, void* y, int32_t dtype, void* stream) {
  try {
    need(h, "handle is null");
    need(x && y, "x and y must be device pointers");
    need(x != y, "x and y must not alias");
    need(dtype == 0 || dtype == 1, "dtype must be 0 (double) or 1 (float)");
    PrecData* P = h->prec;
    hipStream_t s = (hipStream_t)stream;
    const int uv = uvar(0, h->nl);
    const int nwork = (int)P->uwork[uv].size();
    if (dtype == 0)
      launch_uapply<double>(h->dim, P->d_ug[0], P->d_uwork[uv], nwork, h->nl, 0, (const double*)x, nullptr,
                            (double*)y, uemat<double>(P), s, P->utile[uv]);
    else
      launch_uapply<float>(h->dim, P->d_ug[0], P->d_uwork[uv], nwork, h->nl, 0, (const float*)x, nullptr,
                           (float*)y, uemat<float>(P), s, P->utile[uv]);
    hip_check(hipGetLastError(), "elasticity apply launch");
    return BIOT_OK;
  } catch (const BiotError& e) {
    set_error(e.msg);
    return e.st;
  } catch (const std::exception& e) {
    set_error(std::string("internal error: ") + e.what());
    return BIOT_ERR_ARG;
  }
}

biot_status slab_rhs(biot_problem h, const double* state, double t_start, double* rhs, void* stream) {
  BIOT_TRY
  need(h, "handle is null");
  need(state && rhs, "state and rhs must be device pointers");
  need(std::isfinite(t_start), "t_start must be finite");
  launch_slab_rhs(h, state, t_start, rhs, (hipStream_t)stream);
  BIOT_CATCH
}

static biot_status solve_common(biot_problem h, const double* rhs, double* x, int transpose,
                                const biot_solve_opts* opts, biot_solve_info* info, void* stream) {
  try {
    need(h, "handle is null");
    need(rhs && x, "rhs and x must be device pointers");
    need(info, "info is null");
    need((const void*)rhs != (const void*)x, "rhs and x must not alias");
    solve_impl(h, rhs, x, transpose, opts, info, (hipStream_t)stream);
    biot_status st = worst(info, h->count);
    if (st != BIOT_OK) set_error("GMRES did not reach the tolerance within maxit");
    return st;
  } catch (const BiotError& e) {
    set_error(e.msg);
    return e.st;
  } catch (const std::exception& e) {
    set_error(std::string("internal error: ") + e.what());
    return BIOT_ERR_ARG;
  }
}

biot_status solve_slab(biot_problem h, const double* rhs, double* x, const biot_solve_opts* opts,
                       biot_solve_info* info, void* stream) {
  return solve_common(h, rhs, x, 0, opts, info, stream);
}

biot_status solve_slab_fixed_stress(biot_problem h, const double* rhs, double* x, const biot_fs_opts* opts,
                                    biot_fs_info* info, void* stream) {
  try {
    need(h, "handle is null");
    need(rhs && x, "rhs and x must be device pointers");
    need(info, "info is null");
    h->prec->have_prev = false;
    fixed_stress_impl(h, rhs, x, opts, info, (hipStream_t)stream);
    hip_check(hipStreamSynchronize((hipStream_t)stream), "fixed-stress sync");
    biot_status w = BIOT_OK;
    for (int k = 0; k < h->count; ++k)
      if (info[k].status != BIOT_OK) w = (biot_status)info[k].status;
    if (w != BIOT_OK) set_error("the fixed-stress iteration did not reach the tolerance");
    return w;
  } catch (const BiotError& e) {
    set_error(e.msg);
    return e.st;
  } catch (const std::exception& e) {
    set_error(std::string("internal error: ") + e.what());
    return BIOT_ERR_ARG;
  }
}

biot_status solve_slab_transposed(biot_problem h, const double* rhs, double* x, const biot_solve_opts* opts,
                                  biot_solve_info* info, void* stream) {
  return solve_common(h, rhs, x, 1, opts, info, stream);
}

biot_status step(biot_problem h, int32_t nslabs, double t_start, double* state, double* slabs_out,
                 double* checkpoints, const biot_solve_opts* opts, biot_solve_info* infos, void* stream) {
  try {
    need(h, "handle is null");
    need(nslabs >= 0, "nslabs must be >= 0");
    need(state, "state must be a device pointer");
    need(infos || nslabs == 0, "infos is null");
    need(std::isfinite(t_start), "t_start must be finite");
    hipStream_t s = (hipStream_t)stream;
    PrecData* P = h->prec;
    double* rhs = P->arhs;
    double* x = P->xfwd;
    biot_status worst_st = BIOT_OK;
    const double tau = h->descs[0].tau;
    // continue from the slab solved last (still in x) when this call picks up where it ended.
    // With checkpoints every slab starts from its entering state broadcast to all levels, the
    // start adjoint_sweep takes when it recomputes the slab, so the recomputed forward slabs
    // are bitwise the ones marched here.
    bool prev = !checkpoints && P->have_prev && std::fabs(t_start - P->prev_tend) <= 1e-9 * tau;
    P->have_prev = false;
    for (int n = 0; n < nslabs; ++n) {
      if (checkpoints)
        hip_check(hipMemcpyAsync(checkpoints + (long long)n * h->state_len, state, 8 * h->state_len,
                                 hipMemcpyDeviceToDevice, s), "checkpoint");
      const double tn = t_start + n * tau;
      launch_slab_rhs(h, state, tn, rhs, s);
      if (prev) {
        time_transform<double>(h->d_inst, h->count, P->maxN, h->nl, P->pred, x, P->b64.T1, s);
        hip_check(hipMemcpyAsync(x, P->b64.T1, 8 * h->slab_len, hipMemcpyDeviceToDevice, s), "predictor");
      } else {
        launch_bcast(h->d_inst, h->count, P->maxN, h->nl, state, x, s);
      }
      prev = !checkpoints;
      solve_impl(h, rhs, x, 0, opts, infos + (long long)n * h->count, s);
      biot_status st = worst(infos + (long long)n * h->count, h->count);
      if (st != BIOT_OK) worst_st = st;
      if (slabs_out)
        hip_check(hipMemcpyAsync(slabs_out + (long long)n * h->slab_len, x, 8 * h->slab_len, hipMemcpyDeviceToDevice,
                                 s), "slab out");
      launch_extract(h->d_inst, h->count, P->maxN, h->nl - 1, x, state, s);
    }
    hip_check(hipStreamSynchronize(s), "step sync");
    P->have_prev = nslabs > 0;
    P->prev_tend = t_start + nslabs * tau;
    if (worst_st != BIOT_OK) set_error("a slab solve did not reach the tolerance");
    return worst_st;
  } catch (const BiotError& e) {
    set_error(e.msg);
    return e.st;
  } catch (const std::exception& e) {
    set_error(std::string("internal error: ") + e.what());
    return BIOT_ERR_ARG;
  }
}

biot_status biot_misfit(biot_problem h, int32_t nslabs, const double* states, const double* sensors_xyz,
                        int32_t nsens, const double* p_obs, double* J, void* stream) {
  try {
    need(h, "handle is null");
    need(nslabs >= 1, "nslabs must be >= 1");
    need(states && p_obs, "states and p_obs must be device pointers");
    need(sensors_xyz && J, "sensors_xyz and J must be host pointers");
    PrecData* P = h->prec;
    P->have_prev = false;   // the forward slab buffer is reused below
    need(nsens >= 1 && nsens <= P->max_sens, "nsens must be in 1..256");
    hipStream_t s = (hipStream_t)stream;
    const int cnt = h->count;
    auto sw = sensor_weights(h, sensors_xyz, nsens);
    upload(sw, P->sw, s);
    std::vector<double> Jk(cnt, 0.0), res((size_t)cnt * nsens);
    for (int n = 0; n < nslabs; ++n) {
      // states are spatial vectors; view state n as level 0 of a slab-shaped buffer
      launch_bcast(h->d_inst, cnt, P->maxN, 1, states + (long long)n * h->state_len, P->xfwd, s);
      for (int k = 0; k < cnt; ++k)
        hip_check(hipMemcpyAsync(P->sobs + (long long)k * nsens, p_obs + ((long long)k * nslabs + n) * nsens,
                                 8 * nsens, hipMemcpyDeviceToDevice, s), "obs gather");
      launch_sensor(h->d_inst, cnt, 0, nsens, P->sw, P->xfwd, P->sobs, P->sres, s);
      hip_check(hipMemcpyAsync(res.data(), P->sres, 8 * res.size(), hipMemcpyDeviceToHost, s), "res read");
      hip_check(hipStreamSynchronize(s), "misfit sync");
      for (int k = 0; k < cnt; ++k)
        for (int q = 0; q < nsens; ++q) Jk[k] += 0.5 * res[(size_t)k * nsens + q] * res[(size_t)k * nsens + q];
    }
    for (int k = 0; k < cnt; ++k) J[k] = Jk[k];
    return BIOT_OK;
  } catch (const BiotError& e) {
    set_error(e.msg);
    return e.st;
  } catch (const std::exception& e) {
    set_error(std::string("internal error: ") + e.what());
    return BIOT_ERR_ARG;
  }
}

biot_status biot_misfit_noalloc(biot_problem h, int32_t nslabs, const double* states, const double* sensors_xyz,
                                int32_t nsens, const double* p_obs, double* J, void* stream) {
  try {
    need(h, "handle is null");
    need(nslabs >= 1, "nslabs must be >= 1");
    need(states && p_obs, "states and p_obs must be device pointers");
    need(sensors_xyz && J, "sensors_xyz and J must be host pointers");
    need(nsens >= 1, "nsens must be >= 1");
    const int cnt = h->count;
    const size_t wbytes = align256(sizeof(SensorW) * (size_t)cnt * nsens);
    const size_t need_bytes = wbytes + sizeof(double) * (size_t)cnt * nsens;
    if (need_bytes > kScratchBytes)
      throw BiotError{BIOT_ERR_ARG, "instances x sensors needs " + std::to_string(need_bytes) +
                                        " bytes of scratch; the static scratch holds " +
                                        std::to_string(kScratchBytes)};
    hipStream_t s = (hipStream_t)stream;
    char* base = (char*)scratch_ptr();
    SensorW* sw_d = (SensorW*)base;
    double* res_d = (double*)(base + wbytes);
    auto sw = sensor_weights(h, sensors_xyz, nsens);
    hip_check(hipMemcpyAsync(sw_d, sw.data(), sizeof(SensorW) * sw.size(), hipMemcpyHostToDevice, s), "weights");
    std::vector<double> Jk(cnt, 0.0), res((size_t)cnt * nsens);
    for (int n = 0; n < nslabs; ++n) {
      launch_sensor_state(h->d_inst, cnt, n, nslabs, nsens, sw_d, states + (long long)n * h->state_len, p_obs, res_d,
                          s);
      hip_check(hipMemcpyAsync(res.data(), res_d, 8 * res.size(), hipMemcpyDeviceToHost, s), "res read");
      hip_check(hipStreamSynchronize(s), "misfit sync");
      for (int k = 0; k < cnt; ++k)
        for (int q = 0; q < nsens; ++q) Jk[k] += 0.5 * res[(size_t)k * nsens + q] * res[(size_t)k * nsens + q];
    }
    for (int k = 0; k < cnt; ++k) J[k] = Jk[k];
    return BIOT_OK;
  } catch (const BiotError& e) {
    set_error(e.msg);
    return e.st;
  } catch (const std::exception& e) {
    set_error(std::string("internal error: ") + e.what());
    return BIOT_ERR_ARG;
  }
}

biot_status adjoint_sweep(biot_problem h, int32_t nslabs, double t_start, const double* checkpoints,
                          const double* sensors_xyz, int32_t nsens, const double* p_obs, const biot_solve_opts* opts,
                          double* J, double* grad_log_k, void* stream) {
  try {
    need(h, "handle is null");
    need(nslabs >= 1, "nslabs must be >= 1");
    need(checkpoints && p_obs && grad_log_k, "checkpoints, p_obs and grad_log_k must be device pointers");
    need(sensors_xyz && J, "sensors_xyz and J must be host pointers");
    PrecData* P = h->prec;
    P->have_prev = false;   // the forward slab buffer is reused below
    need(nsens >= 1 && nsens <= P->max_sens, "nsens must be in 1..256");
    hipStream_t s = (hipStream_t)stream;
    const int cnt = h->count, d = h->dim, nl = h->nl;
    auto sw = sensor_weights(h, sensors_xyz, nsens);
    upload(sw, P->sw, s);
    hip_check(hipMemsetAsync(grad_log_k, 0, 8 * h->ncells, s), "grad clear");
    std::vector<double> Jk(cnt, 0.0), res((size_t)cnt * nsens);
    std::vector<biot_solve_info> info(cnt);
    // p_obs is instance-major [k][n][s]: gather slab n into a compact [k][s] block
    for (int n = nslabs - 1; n >= 0; --n) {
      const double* st = checkpoints + (long long)n * h->state_len;
      const double tn = t_start + n * h->descs[0].tau;
      // recompute the forward slab from its checkpoint
      launch_slab_rhs(h, st, tn, P->arhs, s);
      launch_bcast(h->d_inst, cnt, P->maxN, nl, st, P->xfwd, s);
      solve_impl(h, P->arhs, P->xfwd, 0, opts, info.data(), s);
      for (int k = 0; k < cnt; ++k)
        if (info[k].status != BIOT_OK) throw BiotError{(biot_status)info[k].status, "forward recompute did not converge"};
      for (int k = 0; k < cnt; ++k)
        hip_check(hipMemcpyAsync(P->sobs + (long long)k * nsens, p_obs + ((long long)k * nslabs + n) * nsens,
                                 8 * nsens, hipMemcpyDeviceToDevice, s), "obs gather");
      launch_sensor(h->d_inst, cnt, nl - 1, nsens, P->sw, P->xfwd, P->sobs, P->sres, s);
      hip_check(hipMemcpyAsync(res.data(), P->sres, 8 * res.size(), hipMemcpyDeviceToHost, s), "res read");
      hip_check(hipStreamSynchronize(s), "adjoint sync");
      for (int k = 0; k < cnt; ++k)
        for (int q = 0; q < nsens; ++q) Jk[k] += 0.5 * res[(size_t)k * nsens + q] * res[(size_t)k * nsens + q];
      launch_adjrhs(h->d_inst, cnt, P->maxN, h->tm, nl, n < nslabs - 1, P->lam_next, nsens, P->sw, P->sres, P->arhs,
                    s);
      hip_check(hipMemsetAsync(P->lam, 0, 8 * h->slab_len, s), "lam clear");
      solve_impl(h, P->arhs, P->lam, 1, opts, info.data(), s);
      for (int k = 0; k < cnt; ++k)
        if (info[k].status != BIOT_OK) throw BiotError{(biot_status)info[k].status, "adjoint solve did not converge"};
      launch_grad(h->d_inst, cnt, P->maxcells, nl, h->d_kinv64, P->lam, P->xfwd, grad_log_k, s);
      std::swap(P->lam, P->lam_next);
    }
    hip_check(hipStreamSynchronize(s), "adjoint end");
    for (int k = 0; k < cnt; ++k) J[k] = Jk[k];
    return BIOT_OK;
  } catch (const BiotError& e) {
    set_error(e.msg);
    return e.st;
  } catch (const std::exception& e) {
    set_error(std::string("internal error: ") + e.what());
    return BIOT_ERR_ARG;
  }
}

}  // extern "C"
