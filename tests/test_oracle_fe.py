"""Pins of the oracle's spatial discretisation and slab system.

* closed-form 1D element matrices (Q2 mass/stiffness, Gauss-nodal Q1 mass,
  open/closed derivative coupling);
* the 2D elasticity element matrix rebuilt from those closed forms as
  Kronecker products (an independent construction);
* rigid-body null space of the unconstrained elasticity operator;
* exactness: fields in (Q2, RT1, DG-Q1) x P_r(t) with matching sources,
  tractions and drained-pressure data are reproduced to round-off
  (sections "Poroelasticity", "Discretisation in Time/Space");
* dG(0) equals backward Euler;
* cellwise mass balance with fluxes evaluated independently on faces;
* the LU solve's own residual.
"""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import fe, slab, temporal
from tests.polyfields import Manufactured, SepPoly

S3 = np.sqrt(3.0)


def test_1d_closed_forms():
    mat = fe.Material(1.0, 1.0, 0.8, 10.0, 1.0)
    h = 0.37
    em = fe.element_matrices(1, (h,), mat)
    K1 = np.array([[7, -8, 1], [-8, 16, -8], [1, -8, 7]]) / (3 * h)
    M1 = h / 30 * np.array([[4, 2, -1], [2, 16, 2], [-1, 2, 4]])
    np.testing.assert_allclose(em["A"], 3.0 * K1, rtol=1e-13)          # (lam + 2 mu) K
    np.testing.assert_allclose(em["Mq1"], M1, rtol=1e-13)
    np.testing.assert_allclose(em["Mp"], h / 2 * np.eye(2), atol=1e-15)
    G = np.array([[-(0.5 + 1 / S3), 2 / S3, 0.5 - 1 / S3],
                  [1 / S3 - 0.5, -2 / S3, 0.5 + 1 / S3]])              # int psi_a phi_b'
    np.testing.assert_allclose(em["E"], G.T, atol=1e-14)
    np.testing.assert_allclose(em["B"], -G.T, atol=1e-14)


def test_2d_elasticity_element_is_kronecker_sum():
    lam, mu = 1.7, 0.6
    h = (0.25, 0.4)
    em = fe.element_matrices(2, h, fe.Material(lam, mu, 0.8, 10.0, 1.0))
    K = lambda hh: np.array([[7, -8, 1], [-8, 16, -8], [1, -8, 7]]) / (3 * hh)
    M = lambda hh: hh / 30 * np.array([[4, 2, -1], [2, 16, 2], [-1, 2, 4]])
    C = np.array([[-0.5, -2 / 3, 1 / 6], [2 / 3, 0, -2 / 3], [-1 / 6, 2 / 3, 0.5]])  # int phi_a' phi_b
    # local index = a_x + 3 a_y  ->  kron(Y, X)
    Axx = (lam + 2 * mu) * np.kron(M(h[1]), K(h[0])) + mu * np.kron(K(h[1]), M(h[0]))
    Ayy = mu * np.kron(M(h[1]), K(h[0])) + (lam + 2 * mu) * np.kron(K(h[1]), M(h[0]))
    Axy = lam * np.kron(C.T, C) + mu * np.kron(C, C.T)                 # rows v_x, cols u_y
    A = np.block([[Axx, Axy], [Axy.T, Ayy]])
    np.testing.assert_allclose(em["A"], A, atol=1e-13)


@pytest.mark.parametrize("d,n", [(2, (3, 2)), (3, (2, 2, 1))])
def test_rigid_body_null_space(d, n):
    mesh = fe.Mesh(n, (1.0, 1.3, 0.8))
    mat = fe.Material(1.0, 1.0, 0.8, 10.0, 1.0)
    Ks, Mt = fe.assemble_spatial(mesh, mat, np.zeros(mesh.ncells))
    su = slice(0, mesh.off_q[0])
    A = Ks[su, su].toarray()
    X = fe.dof_coordinates(mesh)[su]
    comp = np.repeat(np.arange(d), mesh.nu1)
    modes = []
    for c in range(d):
        modes.append((comp == c).astype(float))
    pairs = [(0, 1)] if d == 2 else [(0, 1), (0, 2), (1, 2)]
    for i, j in pairs:                      # rotation in the (i, j) plane
        v = np.zeros(A.shape[0])
        v[comp == i] = -X[comp == i, j]
        v[comp == j] = X[comp == j, i]
        modes.append(v)
    for v in modes:
        assert np.linalg.norm(A @ v) < 1e-12 * np.linalg.norm(A) * np.linalg.norm(v)
    ev = np.linalg.eigvalsh(A)
    nzero = int(np.sum(ev < 1e-10 * ev.max()))
    assert nzero == {2: 3, 3: 6}[d]
    np.testing.assert_allclose(A, A.T, atol=1e-14)


def _manufactured(d, r, lam=1.3, mu=0.7, b=0.8, M=7.0, eta=1.5):
    T = SepPoly.term
    tu = [1.0, 0.5, -0.25][: r + 1]
    tq = [2.0, -1.0, 0.5][: r + 1]
    tp = [0.5, 1.0, 0.3][: r + 1]
    if d == 2:
        u = [T(2, 1.0, [[0, 1, -1], [0, 1]], tu),                    # x(1-x) y
             T(2, 1.0, [[1, 1], [0, 1, 1]], tu)]                     # (1+x)(y+y^2)
        q = [T(2, 1.0, [[0, 1, -1], [1, 1]], tq),                    # x(1-x)(1+y)
             T(2, 1.0, [[1, 1], [0, 2, -1]], tq)]                    # (1+x) y(2-y)
        p = T(2, 1.0, [[1, 2], [2, -1]], tp)                         # (1+2x)(2-y)
    else:
        u = [T(3, 1.0, [[0, 1, -1], [1, 1], [0, 1]], tu),            # x(1-x)(1+y) z
             T(3, 1.0, [[1, 1], [0, 1, -1], [0, 1]], tu),            # (1+x) y(1-y) z
             T(3, 1.0, [[1, 1], [1, 0.5], [0, 1, 1]], tu)]           # (1+x)(1+y/2)(z+z^2)
        q = [T(3, 1.0, [[0, 1, -1], [1, 1], [1, 1]], tq),
             T(3, 1.0, [[1, 1], [0, 1, -1], [2, -1]], tq),
             T(3, 1.0, [[1, 1], [1, 1], [0, 2, -1]], tq)]
        p = T(3, 1.0, [[1, 1], [1, 2], [2, -1]], tp)
    return Manufactured(d, u, q, p, lam, mu, b, M, eta)


@pytest.mark.parametrize("d,n,r", [(2, (3, 4), 0), (2, (3, 4), 1), (2, (2, 3), 2), (3, (2, 2, 2), 1)])
def test_polynomial_exactness(d, n, r):
    ms = _manufactured(d, r)
    mesh = fe.Mesh(n, (1.0, 1.0, 1.0))
    mat = fe.Material(ms.lam, ms.mu, ms.b, ms.M, ms.eta)
    rng = np.random.default_rng(7)
    theta = rng.normal(0.0, 1.0, mesh.ncells)

    def load(t):
        return fe.load_vector(mesh, mat, theta, t, fu=ms.fu, fq=ms.fq, fp=ms.fp,
                              traction=ms.traction, p_drained=ms.p_drained)

    tau = 0.1
    prob = slab.SlabProblem(mesh, mat, r, tau, theta, load)
    x0 = fe.interpolate(mesh, ms.u_fn, ms.q_fn, ms.p_fn, 0.0)
    assert np.abs(x0[prob.mask]).max() == 0.0          # homogeneous essential data
    Xs = prob.march(2, x0)
    for k, X in enumerate(Xs):
        for i in range(r + 1):
            ex = fe.interpolate(mesh, ms.u_fn, ms.q_fn, ms.p_fn, (k + prob.s[i]) * tau)
            err = np.abs(prob.level(X, i) - ex).max()
            assert err < 1e-11 * max(1.0, np.abs(ex).max()), (k, i, err)


def test_dg0_is_backward_euler():
    mesh = fe.Mesh((3, 3), (1.0, 1.0))
    mat = fe.Material(1.0, 1.0, 0.8, 10.0, 1.0)
    theta = np.random.default_rng(3).normal(0, 1, mesh.ncells)
    sig = slab.sigma_function(1, 1.0, 0.2)
    load = slab.traction_load(mesh, mat, theta, sig)
    tau = 0.05
    prob = slab.SlabProblem(mesh, mat, 0, tau, theta, load)
    Xs = prob.march(4)
    Ks, Mt = fe.assemble_spatial(mesh, mat, theta)
    free = (~fe.constrained_mask(mesh)).astype(float)
    Df = sp.diags(free)
    A = (Df @ (Mt + tau * Ks) @ Df + sp.diags(1 - free)).tocsc()
    x = np.zeros(mesh.N)
    for k in range(4):
        rhs = free * (tau * load((k + 1) * tau) + Mt @ x)
        x = spla.spsolve(A, rhs)
        np.testing.assert_allclose(Xs[k], x, rtol=1e-11, atol=1e-13)


def _face_flux(mesh, vec, blk_off, sizes, c, kind):
    """Integral of component c of a field over each cell's two c-faces.

    kind 'u' (Q2 nodal, Simpson weights along the face) or 'q' (RT1 normal
    component, 2-point Gauss nodal weights along the face).  Returns
    (ncells, 2): [lower face, upper face] integrals of the component.
    """
    d = mesh.d
    h = np.array(mesh.h)
    cells = mesh.cell_index_grid()
    out = np.zeros((mesh.ncells, 2))
    if kind == "u":
        wts1 = [np.array([1, 4, 1]) / 6.0] * d
        offs = [range(3)] * d
    else:
        wts1 = [np.array([0.5, 0.5])] * d
        offs = [range(2)] * d
    for side in (0, 1):
        other = [e for e in range(d) if e != c]
        for loc in itertools.product(*[offs[e] for e in other]):
            w = 1.0
            m = np.zeros((mesh.ncells, d), int)
            for k, e in enumerate(other):
                w *= wts1[e][loc[k]] * h[e]
                m[:, e] = 2 * cells[:, e] + loc[k]
            m[:, c] = 2 * cells[:, c] + 2 * side
            idx = blk_off + fe.Mesh._flat(m, sizes)
            out[:, side] += w * vec[idx]
    return out


@pytest.mark.parametrize("d,n,r", [(2, (4, 3), 1), (3, (2, 3, 2), 0)])
def test_cellwise_mass_balance(d, n, r):
    """Per cell and level: sum_j T_ij int(b div u_j + p_j/M) + tau oint q_i.n
    = g_i int(b div u^- + p^-/M)  (no mass source); boundary integrals via
    face quadrature of the nodal values, independent of the assembled B and E."""
    mesh = fe.Mesh(n, (1.0, 1.0, 1.0))
    mat = fe.Material(1.0, 1.0, 0.8, 10.0, 1.0)
    theta = np.random.default_rng(5).normal(0, 1.5, mesh.ncells)
    load = slab.traction_load(mesh, mat, theta, slab.sigma_function(1, 1.0, 0.2))
    prob = slab.SlabProblem(mesh, mat, r, 0.05, theta, load)
    Xs = prob.march(3)
    h = np.array(mesh.h)
    cells = mesh.cell_index_grid()

    def zeta(v):
        divu = np.zeros(mesh.ncells)
        for c in range(d):
            f = _face_flux(mesh, v, mesh.off_u[c], mesh.su, c, "u")
            divu += f[:, 1] - f[:, 0]
        pint = np.zeros(mesh.ncells)
        for a in itertools.product(range(2), repeat=d):
            m = 2 * cells + np.array(a)[None, :]
            pint += np.prod(h / 2) * v[mesh.off_p + fe.Mesh._flat(m, mesh.sp)]
        return mat.b * divu + pint / mat.M

    def qflux(v):
        out = np.zeros(mesh.ncells)
        for c in range(d):
            f = _face_flux(mesh, v, mesh.off_q[c], mesh.sq[c], c, "q")
            out += f[:, 1] - f[:, 0]
        return out

    xprev = np.zeros(mesh.N)
    for X in Xs:
        z = [zeta(prob.level(X, j)) for j in range(r + 1)]
        zm = zeta(xprev)
        for i in range(r + 1):
            bal = sum(prob.T[i, j] * z[j] for j in range(r + 1)) + prob.tau * qflux(prob.level(X, i)) \
                - prob.g[i] * zm
            scale = max(np.abs(z[i]).max(), 1e-30)
            assert np.abs(bal).max() < 1e-11 * scale
        xprev = prob.level(X, r)


def test_lu_residual_and_constraints():
    mesh = fe.Mesh((4, 4), (1.0, 1.0))
    mat = fe.Material(1.0, 1.0, 0.8, 10.0, 1.0)
    theta = np.random.default_rng(1).normal(0, 1, mesh.ncells)
    load = slab.traction_load(mesh, mat, theta, slab.sigma_function(1, 1.0, 0.2))
    prob = slab.SlabProblem(mesh, mat, 1, 0.05, theta, load)
    b = prob.rhs(0.0, np.zeros(mesh.N)) + 0.0
    b += np.random.default_rng(2).normal(0, 1, b.size) * np.tile(prob.free, 2)
    x = prob.solve(b)
    A = prob.slab_matrix()
    assert np.linalg.norm(A @ x - b) <= 1e-13 * np.linalg.norm(b)
    # identity rows for essential DoFs in every level
    m = np.tile(prob.mask, 2)
    np.testing.assert_array_equal(x[m], b[m])
    # constrained counts: 2D, n x n: u_x: bottom row + two lateral columns, u_y: bottom row
    nx, ny = mesh.n
    cu_x = (2 * nx + 1) + 2 * (2 * ny)
    cu_y = 2 * nx + 1
    cq_x = 2 * (2 * ny)
    cq_y = 2 * nx
    assert prob.mask.sum() == cu_x + cu_y + cq_x + cq_y
