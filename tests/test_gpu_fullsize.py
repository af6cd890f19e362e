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
