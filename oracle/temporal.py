"""dG(r) time discretisation on one slab (section "Discretisation in Time").

Test infrastructure only: part of the FP64 CPU oracle.

The slab solution is a polynomial of degree r in time with values in the
spatial FE space, discontinuous across slab ends; the discrete problem is
marched slab by slab.  The polynomials are represented in the Lagrange basis
on the r+1 right Gauss-Radau points of [0, 1] (the right end point is a node,
so the end-of-slab value is the last coefficient), and the same points serve
as quadrature.

With s = (t - t_{n-1}) / tau the dG equations tested with the i-th basis
function read, for a first-order system M_t dX/dt + K_s X = F,

    sum_j D_ij M_t X_j + tau * w_i K_s X_i = tau * w_i F(s_i) + phi_i(0) M_t X^-

where D_ij = int_0^1 phi_j' phi_i ds + phi_i(0) phi_j(0) (derivative term plus
upwind jump) and int phi_i phi_j = w_i delta_ij (Radau quadrature is exact to
degree 2r).  Dividing row i by w_i gives T = W^-1 D and g = W^-1 phi(0).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg
from numpy.polynomial import polynomial as nppoly


def radau_right(r: int):
    """Right Gauss-Radau nodes (ascending, last == 1) and weights on [0, 1].

    The nodes on [-1, 1] are the roots of P_{r+1} - P_r; the weights follow
    from exactness on the monomials 1, s, ..., s^r.
    """
    coef = np.zeros(r + 2)
    coef[r + 1] = 1.0
    coef[r] = -1.0
    x = np.sort(np.real(npleg.legroots(coef)))
    # Newton polish on P_{r+1} - P_r
    for _ in range(3):
        f = npleg.legval(x, coef)
        df = npleg.legval(x, npleg.legder(coef))
        step = np.where(np.abs(x - 1.0) < 1e-14, 0.0, f / np.where(df == 0, 1, df))
        x = x - step
    x[-1] = 1.0
    s = 0.5 * (x + 1.0)
    V = np.vander(s, r + 1, increasing=True).T      # V[m, k] = s_k^m
    w = np.linalg.solve(V, 1.0 / np.arange(1, r + 2))
    return s, w


def lagrange_basis(nodes):
    """Power-series coefficients of the Lagrange polynomials on `nodes`."""
    out = []
    for j, sj in enumerate(nodes):
        others = np.delete(nodes, j)
        c = nppoly.polyfromroots(others)
        out.append(c / nppoly.polyval(sj, c))
    return out


def dg_matrices(r: int):
    """Return (s, w, D, T, g) of the W^-1-scaled dG(r) slab system."""
    s, w = radau_right(r)
    phi = lagrange_basis(s)
    D = np.zeros((r + 1, r + 1))
    for i in range(r + 1):
        for j in range(r + 1):
            prod = nppoly.polymul(nppoly.polyder(phi[j]), phi[i])
            integ = nppoly.polyint(prod)
            D[i, j] = nppoly.polyval(1.0, integ) - nppoly.polyval(0.0, integ)
            D[i, j] += nppoly.polyval(0.0, phi[i]) * nppoly.polyval(0.0, phi[j])
    phi0 = np.array([nppoly.polyval(0.0, p) for p in phi])
    T = D / w[:, None]
    g = phi0 / w
    return s, w, D, T, g


def collocation_matrix(r: int):
    """A_ij = int_0^{s_i} phi_j(s) ds (the Radau IIA Butcher matrix)."""
    s, _ = radau_right(r)
    phi = lagrange_basis(s)
    A = np.zeros((r + 1, r + 1))
    for i in range(r + 1):
        for j in range(r + 1):
            integ = nppoly.polyint(phi[j])
            A[i, j] = nppoly.polyval(s[i], integ) - nppoly.polyval(0.0, integ)
    return A


def real_block_form(T):
    """Q, Lambda_R with Q^-1 T Q = Lambda_R in real block form.

    Real eigenvalue -> 1x1 block; complex pair alpha +- i beta with
    eigenvector a + i b (of alpha + i beta) -> columns [a, b] of Q and block
    [[alpha, beta], [-beta, alpha]].  This is the decomposition that makes
    the slab system split into decoupled dG(0)-type blocks up to the
    beta couplings (section "Monolithic Approach").
    """
    lam, V = np.linalg.eig(T)
    n = T.shape[0]
    cols, blocks = [], []
    used = np.zeros(n, bool)
    order = np.argsort(-lam.real)
    for k in order:
        if used[k]:
            continue
        if abs(lam[k].imag) < 1e-12:
            cols.append(np.real(V[:, k]))
            blocks.append(("real", lam[k].real))
            used[k] = True
        else:
            # take the member with positive imaginary part
            kk = k if lam[k].imag > 0 else int(np.argmin(np.abs(lam - np.conj(lam[k]))))
            partner = int(np.argmin(np.abs(lam - np.conj(lam[kk]))))
            v = V[:, kk]
            cols.append(np.real(v))
            cols.append(np.imag(v))
            blocks.append(("pair", lam[kk].real, lam[kk].imag))
            used[kk] = used[partner] = True
    Q = np.array(cols).T
    Lam = np.zeros((n, n))
    c = 0
    for blk in blocks:
        if blk[0] == "real":
            Lam[c, c] = blk[1]
            c += 1
        else:
            a, b = blk[1], blk[2]
            Lam[c:c + 2, c:c + 2] = [[a, b], [-b, a]]
            c += 2
    return Q, Lam
