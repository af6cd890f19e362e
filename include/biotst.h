/*
 * biotst -- space-time Biot slab operator and solver for MI355X (gfx950).
 *
 * C ABI.  Koecher, "Space-Time-Parallel Poroelasticity Simulation":
 *   - section "Poroelasticity": the fully coupled (u, q, p) Biot system;
 *   - section "Discretisation in Time": dG(r) slabs I_n = (t_{n-1}, t_n),
 *     marched one after the other;
 *   - section "Discretisation in Space": RT1 flux / DG-Q1 pressure mixed
 *     element; the displacement here is continuous Q2;
 *   - section "Monolithic Approach": the (r+1)-level slab block system;
 *   - section "Preconditioning technology": GMRES with a fixed-stress,
 *     level-blockwise (L_j) preconditioner.
 *
 * Discretisation contract (shared with the FP64 CPU oracle in oracle/):
 *   Mesh: box [0,L_0] x .. x [0,L_{d-1}], n_e uniform cells per axis, cells
 *   lexicographic x fastest.  1D bases: closed = quadratic Lagrange on
 *   {0, 1/2, 1}; open = linear Lagrange on the two Gauss points.
 *   u_c: closed in every axis, array (2n_0+1) x .. ; q_c: closed along axis c,
 *   open along the others; p: open in every axis, array (2n_0) x .. .
 *   Spatial level vector = [u_0..u_{d-1}, q_0..q_{d-1}, p], each block x-fastest.
 *   Slab vector = levels j = 0..r outermost (Lagrange coefficients on the
 *   right Gauss-Radau points of [0,1]; level r is the end-of-slab value).
 *   Operator (W^-1-scaled dG(r) system, essential rows = identity):
 *     Y_i = sum_j T_ij M_t X_j + tau K_s X_i,   T = W^-1 D  (Radau),
 *     K_s = [[A,0,-bE],[0,Mq,B],[0,B^T,0]],  M_t = [[0,0,0],[0,0,0],[-bE^T,0,-Mp/M]],
 *     a(u,v) = (2 mu eps(u), eps(v)) + (lam div u, div v), E_ij = (psi_j, div phi_i),
 *     Mq_ij = (eta K^-1 w_j, w_i), B_ij = -(psi_j, div w_i), Mp_ij = (psi_j, psi_i).
 *   Boundary: bottom (x_{d-1}=0) u = 0, q.n = 0; lateral faces u.n = 0,
 *   q.n = 0; top: compressive traction sigma(t) and drained p = 0.
 *   Slab right-hand side: tau F(t_{n-1} + tau s_i) + g_i M_t X^-_{n-1},
 *   g = W^-1 phi(0).
 *
 * Ownership: every buffer is the caller's.  Device pointers must stay valid
 * for the duration of a call; `workspace` must outlive the handle.  The
 * library allocates no device memory: everything it keeps on the device is
 * carved from the caller's workspace.  Host pointers are only read during
 * the call.  Handles are not thread-safe.
 *
 * Errors: every call returns biot_status.  Argument checks run on the host
 * before any launch and leave no side effect.  biot_last_error() returns a
 * thread-local message for the last non-OK status.  Device faults surface at
 * the next synchronising call as BIOT_ERR_DEVICE.
 *
 * Streams: `stream` is a hipStream_t passed as void* (0 = null stream).
 */
#ifndef BIOTST_H
#define BIOTST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct biot_problem_s* biot_problem;

typedef enum {
  BIOT_OK = 0,
  BIOT_ERR_ARG = 1,        /* invalid argument (checked on the host)             */
  BIOT_ERR_WORKSPACE = 2,  /* workspace missing or smaller than required         */
  BIOT_ERR_DEVICE = 3,     /* a HIP call failed                                  */
  BIOT_ERR_NOCONV = 4,     /* iteration limit reached; x holds the last iterate  */
  BIOT_ERR_BREAKDOWN = 5,  /* Krylov breakdown with an unconverged residual      */
  BIOT_ERR_NONFINITE = 6   /* NaN/Inf met in a residual norm                     */
} biot_status;

/* BIOT_FP64: everything in FP64.
 * BIOT_MIXED: FP32 GMRES (FP32 operator apply and preconditioner, FP64 dot
 *   accumulation, Hessenberg and coarse/diagonal inverses) as the inner solve of
 *   FP64 iterative refinement on the FP64 residual.
 * BIOT_FP32_PREC: FP64 flexible GMRES (FP64 apply and orthogonalisation) with
 *   the whole preconditioner applied in FP32; one Krylov space, no refinement. */
typedef enum { BIOT_FP64 = 0, BIOT_MIXED = 1, BIOT_FP32_PREC = 2 } biot_precision;
typedef enum { BIOT_LOAD_STEP = 0, BIOT_LOAD_RAMP = 1 } biot_load_kind;

/* Complex-pair level blocks of the preconditioner (section "Monolithic
 * Approach": a complex eigenvalue alpha +- i beta of the temporal matrix gives
 * a 2x2 level block [[L, beta M_t], [-beta M_t, L]], L = alpha M_t + tau K_s,
 * whose off-diagonal blocks are the paper's C^+-).
 * BIOT_PAIR_AUTO (default): BIOT_PAIR_PRESB for dim == 3 and r >= 2, else
 *   BIOT_PAIR_DROP (the faster of the two in every measured case: in 3D at
 *   dG(2) and dG(3) the kept couplings save 15-30% of the iterations for a
 *   second, serial pass of level solves; in 2D and at dG(1) that pass costs
 *   more than the iterations it saves).
 * BIOT_PAIR_DROP: couplings dropped, each level solved with the shift alpha
 *   ("diagonal blockwise").
 * BIOT_PAIR_PRESB: couplings kept; the block is solved by the preconditioned
 *   square-block factorisation, two level solves with the shift alpha + beta
 *   one after the other, and one M_t product.  The preconditioner still costs
 *   one level solve per level, in two passes: the first solves of the pairs
 *   with the real levels, then the second solves of the pairs.
 * BIOT_PAIR_SHIFT: couplings dropped, each level solved with the shift
 *   alpha + beta.
 * Real eigenvalues always give one level solve with their own shift.  The
 * mode changes iteration counts, never the solution.  Transposed solves use
 * the transposed blocks in the eigenbasis of T^T. */
typedef enum {
  BIOT_PAIR_AUTO = 0,
  BIOT_PAIR_DROP = 1,
  BIOT_PAIR_PRESB = 2,
  BIOT_PAIR_SHIFT = 3
} biot_pair_mode;

/* One problem instance.  Section "Poroelasticity": isotropic C (lambda, mu),
 * Biot coefficient 0 < b < 1, Biot modulus M > 0, viscosity eta; cellwise
 * permeability K = exp(log_k). */
typedef struct {
  int32_t dim;          /* 2 or 3                                                    */
  int32_t n[3];         /* cells per axis (1..4096); n[2] ignored for dim == 2;      *
                         * one instance's slab must hold < 2^31 unknowns             */
  double length[3];     /* box edge lengths                                          */
  int32_t r;            /* dG(r) order, 0..3; all instances of a batch share it      */
  double tau;           /* slab length > 0; all instances of a batch share it (the   *
                         * batch is marched on one clock), else BIOT_ERR_ARG         */
  double lambda, mu;    /* Lame parameters: mu > 0, lambda + 2 mu / dim > 0          */
  double b;             /* Biot coefficient in (0, 1)                                */
  double M;             /* Biot modulus > 0                                          */
  double eta;           /* fluid viscosity > 0                                       */
  double L_fs;          /* fixed-stress parameter; <= 0 selects b^2 / K_dr           */
  int32_t load_kind;    /* biot_load_kind                                            */
  double load_s0;       /* top compressive traction magnitude                        */
  double load_t_ramp;   /* ramp time (> 0 for BIOT_LOAD_RAMP)                        */
  int32_t pair_mode;    /* biot_pair_mode; all instances of a batch share it         */
} biot_problem_desc;

/* Solver controls (nullable: defaults in brackets). */
typedef struct {
  double rtol;          /* stop when ||b - A x|| <= rtol ||b||          [1e-12]   */
  int32_t maxit;        /* total GMRES iterations                         [1000]   */
  int32_t restart;      /* GMRES(m) restart length, <= 64                   [30]   */
  int32_t precision;    /* biot_precision                                [FP64]   */
  double inner_rtol;    /* mixed: inner FP32 solve tolerance              [1e-2]   */
  int32_t max_refine;   /* mixed: outer refinement sweeps                   [30]   */
  int32_t cheb_degree;  /* flux-mass block: 0 = exact line solves, k = 1..64 [-1]
                           Chebyshev-Jacobi of degree k, -1 = line solves
                           when every line has <= 511 cells (one wavefront
                           per line) or instances x levels x flux lines
                           >= 16384 (one thread per line), else degree 8  */
  int32_t graph;        /* 1: replay the preconditioner as a captured      [1]
                           hipGraph (captured on first use); 0: eager     */
} biot_solve_opts;

typedef struct {
  int32_t iterations;   /* GMRES iterations (inner iterations summed when mixed)   */
  int32_t restarts;
  int32_t ir_sweeps;    /* mixed precision refinement sweeps (0 for FP64)          */
  int32_t status;       /* biot_status of this solve                               */
  double rel_residual;  /* final true relative residual ||b - A x|| / ||b||        */
} biot_solve_info;

/* Bytes of device workspace needed for `count` instances. */
biot_status biot_workspace_bytes(const biot_problem_desc* descs, int32_t count,
                                 size_t* bytes);

/* Create a handle for `count` instances (count > 1 = batched; instances are
 * concatenated in every vector argument, each one a full slab vector).
 * log_k[i]: host array of prod(n) cellwise log K values of instance i.
 * Validates every descriptor and log_k (finite) before touching the device;
 * clears the workspace and uploads constants into it; returns after
 * `stream` drains. */
biot_status create_slab_problem(const biot_problem_desc* descs, int32_t count,
                                const double* const* log_k, void* workspace,
                                size_t ws_bytes, void* stream, biot_problem* out);

biot_status destroy_slab_problem(biot_problem h);

/* Replace the log-permeability fields (host arrays as in create). */
biot_status biot_set_log_k(biot_problem h, const double* const* log_k, void* stream);

/* Sizes: spatial DoFs per level and slab-vector offset of instance i. */
biot_status biot_sizes(biot_problem h, int32_t instance, int64_t* level_dofs,
                       int64_t* slab_offset, int64_t* state_offset);
/* Totals over all instances: slab-vector length and state length. */
biot_status biot_totals(biot_problem h, int64_t* slab_len, int64_t* state_len);

/* y = A x (transpose = 0) or y = A^T x (transpose = 1) on device slab vectors
 * (section "Monolithic Approach" block system; A^T = T^T kron M_t^T +
 * tau I kron K_s^T with the same identity rows).  dtype 0: double x, y;
 * dtype 1: float x, y.  x and y must not alias.  Asynchronous on stream. */
biot_status apply_operator(biot_problem h, const void* x, void* y, int32_t transpose,
                           int32_t dtype, void* stream);

/* The elasticity block of the slab operator, y_u = tau A x_u (section
 * "Monolithic Approach": the tau-scaled displacement block of every L_j), on
 * the u-blocks of every time level and instance of device slab vectors, with
 * the essential u DoFs eliminated: x at essential DoFs is ignored and the
 * essential rows of y are 0; the q and p entries of y are not written.  This
 * is the fine-level operator of the preconditioner's elasticity multigrid.
 * dtype 0: double, 1: float.  x and y must not alias.  Asynchronous. */
biot_status biot_elasticity_apply(biot_problem h, const void* x, void* y, int32_t dtype, void* stream);

/* Tile shapes of the operator apply.  Every variant computes bitwise the same
 * y; they differ only in the work decomposition (2D: 0 = 16x16-thread tiles,
 * 1 = 8x8, 2 = 8x8 with one thread layer per time level, the levels in
 * parallel; 3D: z-chunk of 0 = 8, 1 = 4, 2 = 16 cell layers per block).
 * apply_variant[0] is used for FP64 applies, [1] for FP32.  Changing the
 * selection drops the solver's captured Arnoldi-step graphs (they are
 * captured again on the next solve). */
typedef struct {
  int32_t apply_variant[2];
  int32_t n_variants;        /* out: variants available for the handle's dimension */
  double apply_us[2][4];     /* out of biot_autotune: average apply time per variant,
                                microseconds (0 for variants beyond n_variants)    */
} biot_tuning;

/* In-project autotuner: times `reps` (1..1000) operator applies per variant
 * and precision on `stream` (HIP events; workspace buffers as operands),
 * selects the fastest for each precision and reports the timings in `out`
 * (nullable).  Synchronises `stream`. */
biot_status biot_autotune(biot_problem h, int32_t reps, biot_tuning* out, void* stream);
/* Current selection (n_variants filled, apply_us zero). */
biot_status biot_get_tuning(biot_problem h, biot_tuning* out);
/* Select variants (e.g. from a cache of earlier biot_autotune results);
 * BIOT_ERR_ARG for an index outside 0..n_variants-1. */
biot_status biot_set_tuning(biot_problem h, const biot_tuning* t);

/* Slab right-hand side (device): rhs = tau F(t_start + tau s_i) + g_i M_t state,
 * essential rows zero.  state: device, one spatial level per instance. */
biot_status slab_rhs(biot_problem h, const double* state, double t_start, double* rhs,
                     void* stream);

/* Solve A x = rhs (device vectors; x: initial guess in, solution out) with
 * right-preconditioned restarted GMRES and the level-blockwise fixed-stress
 * preconditioner (section "Preconditioning technology").  Stops per instance
 * when the true relative residual is <= rtol, or when two restart cycles in a
 * row fail to halve it (the FP64 rounding floor of b - A x); the latter counts
 * as converged if the residual is within 100 rtol, else BIOT_ERR_NOCONV.
 * Synchronises `stream` once per iteration.  info: host, one per instance. */
biot_status solve_slab(biot_problem h, const double* rhs, double* x,
                       const biot_solve_opts* opts, biot_solve_info* info, void* stream);

/* Transposed solve A^T x = rhs (adjoint slab), same preconditioner family. */
biot_status solve_slab_transposed(biot_problem h, const double* rhs, double* x,
                                  const biot_solve_opts* opts, biot_solve_info* info,
                                  void* stream);

/* The paper's alternative to the monolithic solve (section "Iterative Coupling
 * Approach"): the fixed-stress iterative coupling of flow and mechanics, here on
 * the whole slab system.  Each outer iteration solves the flow sub-system for the
 * (q, p) correction of the current residual, with the displacement's response to
 * the pressure replaced by the fixed-stress term L Mp in the mass rows (L = the
 * descriptor's L_fs, default b^2 / K_dr), then the mechanics sub-system
 * tau A u = (b - A x)_u per time level with the new pressure.  The sub-systems
 * are solved by GMRES preconditioned with the flow and mechanics parts of the
 * level solves.  The fixed point is the slab solution of solve_slab; the
 * iteration converges linearly, at a rate set by L.  x: initial guess in,
 * solution out (device); info: host, one per instance; FP64 only. */
typedef struct {
  double rtol;          /* outer: ||b - A x|| <= rtol ||b||               [1e-12] */
  int32_t max_outer;    /* outer fixed-stress iterations                   [1000] */
  double inner_rtol;    /* relative tolerance of each sub-system solve     [1e-4] */
  int32_t inner_maxit;  /* GMRES iterations per sub-system solve            [500] */
} biot_fs_opts;
typedef struct {
  int32_t outer;            /* outer iterations                                    */
  int32_t flow_iterations;  /* GMRES iterations of all flow solves                 */
  int32_t mech_iterations;  /* GMRES iterations of all mechanics solves            */
  int32_t status;           /* BIOT_OK, or BIOT_ERR_NOCONV after max_outer           */
  double rel_residual;      /* final ||b - A x|| / ||b||                           */
} biot_fs_info;
biot_status solve_slab_fixed_stress(biot_problem h, const double* rhs, double* x, const biot_fs_opts* opts,
                                    biot_fs_info* info, void* stream);

/* March nslabs slabs from t_start (section "Discretisation in Time"):
 * state (device, in/out) = X^- per instance; slabs_out (device, nullable)
 * receives nslabs slab vectors; checkpoints (device, nullable) receives the
 * state entering each slab.  infos: host, nslabs * count entries.
 * Initial guess of each slab solve: the previous slab extrapolated in time;
 * with checkpoints, the entering state broadcast to all levels instead, so
 * that adjoint_sweep (same opts) recomputes bitwise the same slabs. */
biot_status step(biot_problem h, int32_t nslabs, double t_start, double* state,
                 double* slabs_out, double* checkpoints, const biot_solve_opts* opts,
                 biot_solve_info* infos, void* stream);

/* Discrete adjoint of J = 1/2 sum_n sum_s (p_h(x_s, t_n) - p_obs[n][s])^2 with
 * respect to cellwise log K.  checkpoints: device, nslabs states as written by
 * step (the forward slabs are recomputed from them); sensors_xyz: host,
 * nsens * dim coordinates (shared by all instances); p_obs: device,
 * count * nslabs * nsens values (instance-major); J: host, count values;
 * grad_log_k: device, concatenated prod(n) per instance (overwritten). */
biot_status adjoint_sweep(biot_problem h, int32_t nslabs, double t_start,
                          const double* checkpoints, const double* sensors_xyz,
                          int32_t nsens, const double* p_obs, const biot_solve_opts* opts,
                          double* J, double* grad_log_k, void* stream);

/* Pressure misfit of a forward march: J[k] = 1/2 sum_n sum_s (p_h(x_s) - p_obs)^2
 * with p_h the DG-Q1 pressure of the state after slab n (end of slab n, the
 * last Radau level).  states: device, nslabs states (one spatial level per
 * instance each, e.g. the checkpoints written by step shifted by one slab plus
 * the final state, stored contiguously); sensors_xyz: host, nsens * dim;
 * p_obs: device, count * nslabs * nsens (instance-major); J: host, count. */
biot_status biot_misfit(biot_problem h, int32_t nslabs, const double* states, const double* sensors_xyz,
                        int32_t nsens, const double* p_obs, double* J, void* stream);

/* biot_misfit for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same J, with the sensor weights and residuals kept in a static device
 * scratch of 4 MiB instead of the handle's workspace, and the states and
 * p_obs read in place.  It calls no hipMalloc/hipFree and allocates nothing
 * on the device.  Needs 256-byte-aligned count * nsens * 128 bytes +
 * count * nsens * 8 bytes <= 4 MiB, else BIOT_ERR_ARG (no side effect); no
 * other limit on nsens.  Every call on one GPU shares that GPU's scratch
 * (held until the process ends): calls that overlap on one GPU (other
 * streams, other threads, other handles) race and must be serialised by the
 * caller.  Arguments and result as biot_misfit; synchronises `stream`. */
biot_status biot_misfit_noalloc(biot_problem h, int32_t nslabs, const double* states,
                                const double* sensors_xyz, int32_t nsens, const double* p_obs,
                                double* J, void* stream);

/* Thread-local message describing the last non-OK status. */
const char* biot_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BIOTST_H */
