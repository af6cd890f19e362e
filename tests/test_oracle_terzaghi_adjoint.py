"""Physics and adjoint pins of the oracle.

* Terzaghi consolidation (closed-form series): the series itself is checked
  against its PDE (c_v p_zz = p_t, drained top, no-flow bottom) and its
  undrained/drained limits; the oracle's 2D dG(0) solution on the unit-load
  workload converges to it at first order under joint (h, tau) refinement
  and is x-invariant.
* Discrete adjoint: the oracle gradient of the pressure misfit matches
  central finite differences of the oracle forward map.
"""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint, fe, slab, terzaghi

PHYS = dict(lam=1.0, mu=1.0, b=0.8, M=10.0, K=1.0, eta=1.0, sigma=1.0)


def test_series_satisfies_pde_and_limits():
    p0, cv = terzaghi.coefficients(**PHYS)
    assert abs(p0 - 0.8 / (3.0 * (0.1 + 0.64 / 3.0))) < 1e-15
    z = np.linspace(0.05, 0.95, 7)
    t, dz, dt = 0.05, 1e-4, 1e-6
    p = lambda zz, tt: terzaghi.pressure(zz, tt, **PHYS)
    pzz = (p(z + dz, t) - 2 * p(z, t) + p(z - dz, t)) / dz ** 2
    pt = (p(z, t + dt) - p(z, t - dt)) / (2 * dt)
    np.testing.assert_allclose(cv * pzz, pt, rtol=2e-4, atol=1e-6)
    assert abs(p(np.array([0.0]), 0.3)[0]) < 1e-14                        # drained top
    pb = (p(np.array([1.0]), 0.2) - p(np.array([1.0 - 1e-5]), 0.2)) / 1e-5
    assert abs(pb[0]) < 1e-4                                              # no-flow bottom
    np.testing.assert_allclose(p(np.array([0.5]), 1e-7), [p0], rtol=1e-3)  # undrained start
    s_inf = terzaghi.top_settlement(50.0, **PHYS)
    assert abs(s_inf - (-1.0 / 3.0)) < 1e-12                             # drained limit
    s0 = terzaghi.top_settlement(0.0, **PHYS)
    assert abs(s0 - (0.8 * p0 - 1.0) / 3.0) < 1e-3


def _terzaghi_errors(n, tau, nslabs):
    wl = W.c1_terzaghi().scaled((n, n), tau=tau, nslabs=nslabs)
    prob = slab.problem_from_workload(wl)
    Xs = prob.march(nslabs)
    depths = np.array([0.125, 0.375, 0.625, 0.875])
    pts = np.array([[0.3, 1.0 - z] for z in depths])
    P = fe.pressure_point_matrix(prob.mesh, pts)
    errs = []
    xinv = 0.0
    for k, X in enumerate(Xs):
        t = (k + 1) * tau
        end = prob.level(X, prob.r)
        if abs(t - 0.2) < 1e-12 or abs(t - 0.4) < 1e-12:
            ex = terzaghi.pressure(depths, t, **PHYS)
            errs.append(np.abs(P @ end - ex).max())
        # x-invariance: p at the same height in every column of cells
        pp = end[prob.mesh.off_p:].reshape(prob.mesh.sp[1], prob.mesh.sp[0])
        xinv = max(xinv, np.abs(pp - pp[:, :1]).max())
    return max(errs), xinv


def test_terzaghi_first_order_convergence():
    e1, x1 = _terzaghi_errors(8, 0.1, 4)
    e2, x2 = _terzaghi_errors(16, 0.05, 8)
    e3, x3 = _terzaghi_errors(32, 0.025, 16)
    assert max(x1, x2, x3) < 1e-12
    assert e1 < 0.15
    assert 1.6 < e1 / e2 < 2.5 and 1.6 < e2 / e3 < 2.5, (e1, e2, e3)


@pytest.mark.parametrize("d,n,r", [(2, (3, 3), 1), (3, (2, 2, 2), 0)])
def test_adjoint_gradient_matches_finite_differences(d, n, r):
    wl = W.Workload("t", d, n, r, 0.1, 3, lam=2.0, mu=1.0, b=0.9, M=5.0, eta=1.0,
                    k_sigma=1.0, k_ell=0.3, k_seed=11)
    theta = wl.log_k()
    mk = lambda th: slab.problem_from_workload(wl, theta=th)
    prob = mk(theta)
    sens = W.sensors(6, d, 12)
    P = fe.pressure_point_matrix(prob.mesh, sens)
    p_obs = 0.1 * np.random.default_rng(3).normal(size=(3, len(sens)))
    J, g, _ = adjoint.gradient(prob, 3, P, p_obs)
    for k, dirn in enumerate(W.unit_directions(3, theta.size, 21)):
        eps = 1e-5
        Jp = adjoint.misfit(mk(theta + eps * dirn), mk(theta + eps * dirn).march(3), P, p_obs)
        Jm = adjoint.misfit(mk(theta - eps * dirn), mk(theta - eps * dirn).march(3), P, p_obs)
        fd = (Jp - Jm) / (2 * eps)
        assert abs(fd - g @ dirn) <= 1e-7 * max(abs(fd), np.abs(g).max()), (k, fd, g @ dirn)


def test_adjoint_taylor_remainder_second_order():
    wl = W.Workload("t", 2, (3, 3), 1, 0.1, 2, k_sigma=1.0, k_ell=0.3, k_seed=5)
    theta = wl.log_k()
    mk = lambda th: slab.problem_from_workload(wl, theta=th)
    prob = mk(theta)
    P = fe.pressure_point_matrix(prob.mesh, W.sensors(5, 2, 8))
    p_obs = np.zeros((2, 5))
    J, g, _ = adjoint.gradient(prob, 2, P, p_obs)
    dirn = W.unit_directions(1, theta.size, 9)[0]
    rem = []
    for eps in (1e-1, 5e-2, 2.5e-2):
        pr = mk(theta + eps * dirn)
        rem.append(abs(adjoint.misfit(pr, pr.march(2), P, p_obs) - J - eps * (g @ dirn)))
    assert 3.0 < rem[0] / rem[1] < 5.0 and 3.0 < rem[1] / rem[2] < 5.0, rem
