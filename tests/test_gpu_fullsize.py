"""Parity at the benchmark sizes, in the launch configuration the benchmark
times (autotuned tile variants, graph-replayed preconditioner):

* 2D 128x128 dG(1): every output of the FP64 and FP32 apply (all tile
  variants) against the oracle's assembled slab matrix, and one slab solve
  whose residual is evaluated with the oracle's matrix and right-hand side;
* 3D 48^3 dG(2): sampled rows of the apply (random rows plus the first and
  last rows of every block and level) against rows built from the oracle's
  per-cell matrices, and the adjoint identity z.(A x) = x.(A^T z) at full size;
* the 64-instance batch: every instance of the batched apply bitwise equal to
  the same instance applied alone.
"""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import field_rel, torch_cuda

pytestmark = pytest.mark.gpu


def _handle(wls):
    from paper_1801_04984_amd import BiotSlab
    return BiotSlab(wls, [w.log_k() for w in wls])


def test_apply_2d_128_every_output():
    torch = torch_cuda()
    from oracle import slab
    wl = W.c2_hetero2d()
    prob = slab.problem_from_workload(wl)
    h = _handle([wl])
    x = np.random.default_rng(11).standard_normal(h.slab_len)
    for tr in (False, True):
        ref = prob.apply(x, transpose=tr)
        tol = 1e-12 * np.abs(ref).max()
        for v in range(h.get_tuning()["n_variants"]):
            h.set_tuning([v, v])
            got = h.apply(torch.tensor(x, device="cuda"), transpose=tr).cpu().numpy()
            bad = np.abs(got - ref) > tol
            assert not bad.any(), (tr, v, int(bad.sum()), np.abs(got - ref).max(), tol)
            x32 = x.astype(np.float32)
            got32 = h.apply(torch.tensor(x32, device="cuda"), transpose=tr).double().cpu().numpy()
            ref32 = prob.apply(x32.astype(np.float64), transpose=tr)
            err = field_rel(prob, got32, ref32)
            assert max(err.values()) < 2e-5, (tr, v, err)
    h.close()


def test_solve_2d_128_residual_with_oracle_matrix():
    """One slab of the benchmark march (t = 0.02 .. 0.04 after one slab from
    rest), solved on the GPU at the default tolerance; the residual of the
    GPU solution is taken with the oracle's slab matrix and right-hand side."""
    torch = torch_cuda()
    from oracle import slab
    wl = W.c2_hetero2d()
    prob = slab.problem_from_workload(wl)
    h = _handle([wl])
    state = h.zeros_state()
    infos, st = h.step(1, 0.0, state)
    assert st == 0, infos
    s_host = state.cpu().numpy()
    rhs_o = prob.rhs(wl.tau, s_host)
    rhs_g = h.rhs(state, wl.tau).cpu().numpy()
    assert np.abs(rhs_g - rhs_o).max() <= 1e-12 * np.abs(rhs_o).max()
    x, info, st = h.solve(torch.tensor(rhs_o, device="cuda"))
    assert st == 0 and info[0]["rel_residual"] <= 1e-10, info
    r = rhs_o - prob.apply(x.cpu().numpy())
    assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(rhs_o)
    h.close()


def _march_vs_lu(n, nslabs=2):
    """The first slabs of the benchmark march (2D heterogeneous workload, dG(1),
    tau 0.02, ramp load) on an n x n mesh: the GPU march at its default
    tolerance, autotuned, against the oracle's nested-dissection LU march, per
    field (relative l2 over all levels of a slab) <= 1e-10."""
    torch = torch_cuda()
    from oracle import slab
    from paper_1801_04984_amd import tuning
    wl = W.c2_hetero2d().scaled(n)
    theta = wl.log_k()
    h = _handle([wl])
    tuning.tune(h, path=None)
    state = h.zeros_state()
    slabs = torch.zeros(nslabs * h.slab_len, dtype=torch.float64, device="cuda")
    infos, st = h.step(nslabs, 0.0, state, slabs_out=slabs)
    assert st == 0, infos
    sv = slabs.cpu().numpy().reshape(nslabs, -1)
    h.close()
    prob = slab.problem_from_workload(wl, theta=theta)
    ref = prob.march(nslabs)
    errs = [field_rel(prob, sv[k], ref[k]) for k in range(nslabs)]
    print(f"{n}: per-field errors {errs}; iterations {[i['iterations'] for i in infos]}")
    for k in range(nslabs):
        assert max(errs[k].values()) <= 1e-10, (k, errs[k])


def test_march_2d_64_matches_oracle_lu():
    _march_vs_lu((64, 64))


@pytest.mark.timeout(900)
def test_march_2d_128_matches_oracle_lu():
    """At the benchmark mesh itself (658,436 slab unknowns; the oracle's LU
    factorisation takes a few minutes on one host core)."""
    _march_vs_lu((128, 128))


class _RowOracle:
    """Rows of the slab operator from the oracle's per-cell matrices: for a
    free row g of level l, y = sum_j T_lj (M_t xm_j)[g] + tau (K_s xm_l)[g]
    with xm = x with essential entries zeroed; essential rows copy x."""

    def __init__(self, wl):
        from oracle import fe, temporal
        self.mesh = fe.Mesh(tuple(wl.n), wl.length)
        self.mat = fe.Material(wl.lam, wl.mu, wl.b, wl.M, wl.eta)
        self.Ks, self.Mq, self.Mt = fe.cell_matrices(self.mesh, self.mat)
        self.G = fe.global_map(self.mesh)
        self.mask = fe.constrained_mask(self.mesh)
        self.kinv = np.exp(-wl.log_k())
        self.T = temporal.dg_matrices(wl.r)[3]
        self.tau = wl.tau
        flat = self.G.ravel()
        self.order = np.argsort(flat, kind="stable")
        self.sorted = flat[self.order]
        self.N = self.mesh.N

    def masked(self, x):
        L = self.T.shape[0]
        return [np.where(self.mask, 0.0, x[j * self.N:(j + 1) * self.N]) for j in range(L)]

    def row(self, xm, x, l, g):
        """(value, scale): scale = sum of the magnitudes of the summed terms."""
        if self.mask[g]:
            v = x[l * self.N + g]
            return v, abs(v)
        a, b = np.searchsorted(self.sorted, [g, g + 1])
        y, sc = 0.0, 0.0
        for pos in self.order[a:b]:
            cell, loc = divmod(int(pos), self.G.shape[1])
            cols = self.G[cell]
            kc = self.tau * (self.Ks[loc] + self.kinv[cell] * self.Mq[loc])
            t = kc * xm[l][cols]
            y += t.sum()
            sc += np.abs(t).sum()
            for j in range(len(xm)):
                t = self.T[l, j] * self.Mt[loc] * xm[j][cols]
                y += t.sum()
                sc += np.abs(t).sum()
        return y, sc


def test_apply_3d_48_dg2_sampled_rows_and_adjoint():
    torch = torch_cuda()
    from paper_1801_04984_amd import tuning
    wl = W.c4_adjoint3d()
    h = _handle([wl])
    tuning.tune(h, path=None)
    N, L = h.level_dofs[0], wl.r + 1
    rng = np.random.default_rng(17)
    x = rng.standard_normal(h.slab_len)
    y = h.apply(torch.tensor(x, device="cuda")).cpu().numpy()
    ro = _RowOracle(wl)
    m = ro.mesh
    starts = [m.off_u[c] for c in range(3)] + [m.off_q[c] for c in range(3)] + [m.off_p, N]
    rows = set()
    for l in range(L):
        for k in range(len(starts) - 1):
            for g in list(range(starts[k], starts[k] + 6)) + list(range(starts[k + 1] - 6, starts[k + 1])):
                rows.add((l, g))
    for _ in range(240):
        rows.add((int(rng.integers(L)), int(rng.integers(N))))
    xm = ro.masked(x)
    for l, g in sorted(rows):
        ref, scale = ro.row(xm, x, l, g)
        got = y[l * N + g]
        assert abs(got - ref) <= 1e-12 * scale + 1e-300, (l, g, got, ref, scale)
    # adjoint identity z.(A x) = x.(A^T z) at full size
    z = rng.standard_normal(h.slab_len)
    yt = h.apply(torch.tensor(z, device="cuda"), transpose=True).cpu().numpy()
    lhs, rhs = float(z @ y), float(x @ yt)
    assert abs(lhs - rhs) <= 1e-11 * (np.linalg.norm(z) * np.linalg.norm(y)), (lhs, rhs)
    h.close()


def test_batch_64_instances_match_single_handles():
    torch = torch_cuda()
    from paper_1801_04984_amd import tuning
    wls = W.c5_batch()
    h = _handle(wls)
    tuning.tune(h, path=None)
    x = torch.tensor(np.random.default_rng(23).standard_normal(h.slab_len), device="cuda")
    y = h.apply(x)
    for k in range(0, len(wls), 9):
        g = _handle([wls[k]])
        g.set_tuning(h.get_tuning()["apply_variant"])
        xs = h.instance_slab(x, k).contiguous()
        ys = g.apply(xs)
        assert torch.equal(ys, h.instance_slab(y, k)), k
        g.close()
    h.close()


@pytest.mark.timeout(900)
def test_adjoint_3d_48_dg2_mixed_matches_fd_20_directions():
    """The 3D 48^3 dG(2) adjoint workload: the gradient of J = 1/2 sum (p_h - p_obs)^2
    at 64 sensors with respect to all 110,592 cellwise log K values, computed by
    adjoint_sweep with the slab solves in mixed precision (FP32 inner solves in
    FP64 refinement), against central FP64 finite differences of the forward map
    along 20 random unit directions (eps = 1e-4), on the first two slabs."""
    torch = torch_cuda()
    from paper_1801_04984_amd import tuning
    wl = W.c4_adjoint3d()
    theta = wl.log_k()
    h = _handle([wl])
    tuning.tune(h, path=None)
    ns = 2
    sens = W.sensors(W.C4_NSENS, 3, W.C4_SENSOR_SEED)
    # p_obs: the FP64 forward of the K field of the next seed
    obs_wl = wl.scaled(wl.n, k_seed=W.C4_OBS_K_SEED)
    h.set_log_k([obs_wl.log_k()])
    st = h.zeros_state()
    chk = torch.zeros(ns * h.state_len, dtype=torch.float64, device="cuda")
    infos, s0 = h.step(ns, 0.0, st, checkpoints=chk, rtol=1e-13)
    assert s0 == 0, infos
    ends = torch.cat([chk[h.state_len:], st])
    # the observations: that field's pressure at the sensors after each slab
    from oracle import fe
    P = fe.pressure_point_matrix(fe.Mesh(tuple(wl.n), wl.length), sens)
    pe = ends.view(ns, h.level_dofs[0]).cpu().numpy()
    p_obs = torch.tensor(np.concatenate([P @ pe[k] for k in range(ns)]), device="cuda")
    h.set_log_k([theta])

    def J_of(th, precision=0):
        h.set_log_k([th])
        s = h.zeros_state()
        c = torch.zeros(ns * h.state_len, dtype=torch.float64, device="cuda")
        inf, st_ = h.step(ns, 0.0, s, checkpoints=c, rtol=1e-13, precision=precision)
        assert st_ == 0, inf
        e = torch.cat([c[h.state_len:], s])
        return h.misfit(ns, e, sens, p_obs)[0], c

    J0, chk0 = J_of(theta, precision=1)
    J, g, sa = h.adjoint(ns, 0.0, chk0, sens, p_obs, precision=1, rtol=1e-13)
    assert sa == 0
    assert abs(J[0] - J0) <= 1e-12 * abs(J0)
    g = g.cpu().numpy()
    dirs = W.unit_directions(W.C4_NDIRS, theta.size, W.C4_DIRECTION_SEED)
    # central differences: truncation O(eps^2), rounding (the forward solves end at a
    # relative residual of 1e-13, so J carries about 1e-13 J) O(1e-13 J / eps).  At
    # eps = 1e-5 that rounding, ~1e-8 absolute whatever the direction, is already 1e-3 of
    # the smallest directional derivatives here; eps = 1e-4 leaves it at ~1e-9.
    eps = 1e-4
    errs = []
    for d in dirs:
        jp, _ = J_of(theta + eps * d)
        jm, _ = J_of(theta - eps * d)
        fd = (jp - jm) / (2 * eps)
        ad = float(g @ d)
        errs.append((fd, ad))
    h.close()
    gn = float(np.linalg.norm(g))
    rel = [abs(fd - ad) / max(abs(ad), 1e-3 * gn) for fd, ad in errs]
    print(f"48^3 dG(2) adjoint: J {J0:.6e}, |grad| {gn:.3e}; directional derivatives (fd, adjoint) {errs}; "
          f"max rel diff {max(rel):.2e}")
    # directional derivatives of 2e-7 to 4e-5, each compared with the larger of itself and
    # 1e-3 |grad|
    assert max(rel) <= 1e-3, rel
