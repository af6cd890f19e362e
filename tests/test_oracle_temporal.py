"""Pins of the oracle's dG(r) temporal matrices (section "Discretisation in Time").

dG(r) on right Radau points with Radau quadrature is the Radau IIA
collocation method; T = W^-1 D must be the inverse of its Butcher matrix.
The tableaux below are the textbook closed forms (Hairer & Wanner, Solving
ODEs II, section IV.5), independent of the oracle's construction.
"""
import numpy as np
import pytest

from oracle import temporal

S6 = np.sqrt(6.0)
RADAU_IIA = {
    0: (np.array([1.0]), np.array([[1.0]]), np.array([1.0])),
    1: (np.array([1.0 / 3.0, 1.0]),
        np.array([[5.0 / 12.0, -1.0 / 12.0], [3.0 / 4.0, 1.0 / 4.0]]),
        np.array([3.0 / 4.0, 1.0 / 4.0])),
    2: (np.array([(4 - S6) / 10, (4 + S6) / 10, 1.0]),
        np.array([[(88 - 7 * S6) / 360, (296 - 169 * S6) / 1800, (-2 + 3 * S6) / 225],
                  [(296 + 169 * S6) / 1800, (88 + 7 * S6) / 360, (-2 - 3 * S6) / 225],
                  [(16 - S6) / 36, (16 + S6) / 36, 1.0 / 9.0]]),
        np.array([(16 - S6) / 36, (16 + S6) / 36, 1.0 / 9.0])),
}


@pytest.mark.parametrize("r", [0, 1, 2])
def test_T_is_inverse_of_radau_iia(r):
    c, A, b = RADAU_IIA[r]
    s, w, D, T, g = temporal.dg_matrices(r)
    np.testing.assert_allclose(s, c, atol=1e-14)
    np.testing.assert_allclose(w, b, atol=1e-14)
    np.testing.assert_allclose(T @ A, np.eye(r + 1), atol=1e-12)
    np.testing.assert_allclose(g, np.linalg.solve(A, np.ones(r + 1)), atol=1e-12)


@pytest.mark.parametrize("r", [0, 1, 2, 3])
def test_collocation_identity_and_quadrature(r):
    s, w, D, T, g = temporal.dg_matrices(r)
    # Radau quadrature with r+1 points is exact to degree 2r, not 2r+1
    for m in range(2 * r + 1):
        assert abs(np.sum(w * s ** m) - 1.0 / (m + 1)) < 1e-14
    if r > 0:
        assert abs(np.sum(w * s ** (2 * r + 1)) - 1.0 / (2 * r + 2)) > 1e-6
    assert s[-1] == 1.0
    # int_0^{s_i} phi_j  is the inverse of T (collocation form of dG)
    np.testing.assert_allclose(temporal.collocation_matrix(r) @ T, np.eye(r + 1), atol=1e-12)
    # D 1 = phi(0): constants are preserved, so g = T 1
    np.testing.assert_allclose(T @ np.ones(r + 1), g, atol=1e-12)


def test_eigenvalues_known():
    # r=1: 2 +- i sqrt(2); r=2: the RADAU5 constants
    ev = np.sort_complex(np.linalg.eigvals(temporal.dg_matrices(1)[3]))
    np.testing.assert_allclose(ev, [2 - 1j * np.sqrt(2), 2 + 1j * np.sqrt(2)], atol=1e-13)
    ev = np.linalg.eigvals(temporal.dg_matrices(2)[3])
    real = ev[np.abs(ev.imag) < 1e-9].real
    cplx = ev[ev.imag > 1e-9][0]
    np.testing.assert_allclose(real, [3.637834252744496], atol=1e-12)
    np.testing.assert_allclose([cplx.real, cplx.imag], [2.681082873627752, 3.050430199247411], atol=1e-12)


@pytest.mark.parametrize("r", [0, 1, 2, 3])
def test_real_block_form(r):
    T = temporal.dg_matrices(r)[3]
    Q, Lam = temporal.real_block_form(T)
    np.testing.assert_allclose(np.linalg.solve(Q, T @ Q), Lam, atol=1e-11)
    # blocks: 1x1 or 2x2 [[a, b], [-b, a]] only
    k = 0
    while k < r + 1:
        if k + 1 < r + 1 and abs(Lam[k, k + 1]) > 1e-12:
            assert abs(Lam[k, k] - Lam[k + 1, k + 1]) < 1e-12
            assert abs(Lam[k, k + 1] + Lam[k + 1, k]) < 1e-12
            k += 2
        else:
            k += 1
    # all real parts positive (needed for the level blocks to be definite)
    assert np.all(np.diag(Lam) > 0)
