"""Monolithic space-time slab system and slab-by-slab marching.

Test infrastructure only: part of the FP64 CPU oracle.

Section "Monolithic Approach": on each slab I_n the r+1 temporal
coefficients of (u, q, p) are solved together.  In the W^-1-scaled form
(see `oracle.temporal`) the slab matrix is

    A_slab = kron(T_r, M_t) + tau * kron(I_{r+1}, K_s)

with essential rows replaced by identity rows in every level, and the
right-hand side of slab n is  tau F(t_{n-1} + tau s_i) + g_i M_t X^-_{n-1}.
The end value X^-_n is the last Radau coefficient (s_r = 1).  The oracle
solves every slab exactly with a sparse LU factorisation (SuperLU) plus
FP64 iterative refinement with the same factors.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fe, temporal


@dataclass
class SlabProblem:
    mesh: fe.Mesh
    mat: fe.Material
    r: int
    tau: float
    theta: np.ndarray
    # load(t) -> F(t) of one spatial level; default: top traction sigma(t)
    load: Optional[Callable] = None
    # fill-reducing ordering of the sparse LU: "nd" or "colamd" (see factor)
    ordering: str = "nd"

    def __post_init__(self):
        self.s, self.w, self.D, self.T, self.g = temporal.dg_matrices(self.r)
        self.Ks, self.Mt = fe.assemble_spatial(self.mesh, self.mat, self.theta)
        self.mask = fe.constrained_mask(self.mesh)
        self.free = ~self.mask
        self.L = self.r + 1
        self.N = self.mesh.N
        self._A = None
        self._lu = None
        self._perm = None

    # -- the slab operator ------------------------------------------------------
    def slab_matrix(self):
        if self._A is None:
            full = sp.kron(sp.csr_matrix(self.T), self.Mt) + self.tau * sp.kron(
                sp.identity(self.L), self.Ks)
            fmask = np.tile(self.free, self.L).astype(float)
            cmask = 1.0 - fmask
            Df = sp.diags(fmask)
            self._A = (Df @ full @ Df + sp.diags(cmask)).tocsr()
            self._A.eliminate_zeros()
        return self._A

    def apply(self, x, transpose=False):
        A = self.slab_matrix()
        return (A.T @ x) if transpose else (A @ x)

    def slab_ordering(self):
        """Fill-reducing symmetric permutation of the slab unknowns: geometric
        nested dissection of the spatial coupling graph (K_s and M_t), every
        spatial DoF keeping its r+1 levels together."""
        G = (abs(self.Ks) + abs(self.Mt)).tocsr()
        G = (G + G.T).tocsr()
        ps = nested_dissection(G, fe.dof_coordinates(self.mesh))
        return (np.arange(self.L)[None, :] * self.N + ps[:, None]).reshape(-1)

    def factor(self):
        """Sparse LU of the slab matrix (SuperLU).  ordering "nd": nested
        dissection (slab_ordering) as a symmetric permutation, diagonal pivots
        preferred; "colamd": SuperLU's column ordering with partial pivoting.
        Both factor the same matrix: their spread is the oracle's own floor."""
        if self._lu is None:
            A = self.slab_matrix()
            if self.ordering == "nd":
                perm = self.slab_ordering()
                Ap = A[perm][:, perm].tocsc()
                lu = spla.splu(Ap, permc_spec="NATURAL", diag_pivot_thresh=0.0,
                               options=dict(Equil=True, IterRefine="DOUBLE", SymmetricMode=True))
            elif self.ordering == "colamd":
                perm = None
                lu = spla.splu(A.tocsc(), permc_spec="COLAMD",
                               options=dict(Equil=True, IterRefine="DOUBLE"))
            else:
                raise ValueError(f"unknown ordering {self.ordering!r}")
            self._lu, self._perm = lu, perm
        return self._lu

    def _lu_solve(self, b, trans):
        lu = self.factor()
        if self._perm is None:
            return lu.solve(b, trans=trans)
        # A = P^T A_p P with A_p = A[perm][:, perm]; the same holds for A^T
        y = lu.solve(b[self._perm], trans=trans)
        x = np.empty_like(y)
        x[self._perm] = y
        return x

    def solve(self, rhs, transpose=False, refine=2):
        A = self.slab_matrix()
        trans = "T" if transpose else "N"
        x = self._lu_solve(rhs, trans)
        for _ in range(refine):
            res = rhs - (A.T @ x if transpose else A @ x)
            x = x + self._lu_solve(res, trans)
        res = rhs - (A.T @ x if transpose else A @ x)
        nb = np.linalg.norm(rhs)
        if nb > 0 and not np.linalg.norm(res) <= 1e-10 * nb:
            raise RuntimeError(f"oracle LU residual {np.linalg.norm(res) / nb:.2e} above 1e-10")
        return x

    def condition_estimate(self):
        """1-norm condition estimate ||A||_1 ||A^-1||_1 (Hager-Higham block
        estimator on the LU factors)."""
        A = self.slab_matrix()
        n = A.shape[0]
        inv = spla.LinearOperator((n, n), matvec=lambda v: self._lu_solve(np.asarray(v, float).ravel(), "N"),
                                  rmatvec=lambda v: self._lu_solve(np.asarray(v, float).ravel(), "T"),
                                  dtype=float)
        return spla.onenormest(A) * spla.onenormest(inv)

    # -- right-hand side ----------------------------------------------------------
    def rhs(self, t_start, x_prev_end):
        """Slab RHS given the previous end state X^- (one spatial level)."""
        jump = self.Mt @ x_prev_end
        parts = []
        for i in range(self.L):
            Fi = self.load(t_start + self.tau * self.s[i]) if self.load else np.zeros(self.N)
            parts.append(self.tau * Fi + self.g[i] * jump)
        b = np.concatenate(parts)
        b[np.tile(self.mask, self.L)] = 0.0
        return b

    def march(self, nslabs, x0_end=None, t0=0.0):
        """Solve nslabs slabs; returns list of slab vectors ((r+1)*N each)."""
        x_end = np.zeros(self.N) if x0_end is None else np.asarray(x0_end, float)
        out = []
        for n in range(nslabs):
            b = self.rhs(t0 + n * self.tau, x_end)
            X = self.solve(b)
            out.append(X)
            x_end = X[self.r * self.N:(self.r + 1) * self.N].copy()
        return out

    def level(self, X, i):
        return X[i * self.N:(i + 1) * self.N]


def nested_dissection(G, X, leaf=64):
    """Geometric nested dissection of a graph with vertex coordinates.

    G: symmetric sparse adjacency (csr); X: (n, d) coordinates.  A vertex set
    larger than `leaf` is split at the median of its widest coordinate; the
    vertices of the lower half with a neighbour in the upper half form the
    separator.  The order is: lower half (recursively), upper half
    (recursively), separator; so no vertex of one half is coupled to the
    other half before the separator is eliminated.  Returns a permutation.
    """
    G = sp.csr_matrix(G)
    n = G.shape[0]

    def split(idx):
        if len(idx) <= leaf:
            return [idx]
        pts = X[idx]
        axis = int(np.argmax(pts.max(0) - pts.min(0)))
        cut = np.median(pts[:, axis])
        low = pts[:, axis] < cut
        if low.all() or not low.any():
            return [idx]
        upper = np.zeros(n)
        upper[idx[~low]] = 1.0
        lo = idx[low]
        touches = (G[lo] @ upper) > 0
        return split(lo[~touches]) + split(idx[~low]) + [lo[touches]]

    perm = np.concatenate(split(np.arange(n)))
    assert np.array_equal(np.sort(perm), np.arange(n))
    return perm


def traction_load(mesh: fe.Mesh, mat: fe.Material, theta, sigma_of_t):
    """Top-face compressive traction t_N = -sigma(t) e_top, zero sources.

    The load is linear in sigma, so the unit pattern is assembled once.
    """
    d = mesh.d
    unit = fe.load_vector(mesh, mat, theta, 0.0,
                          traction=lambda X, t, e, s: _unit_top(X, e, s, d))

    def load(t):
        return sigma_of_t(t) * unit

    return load


def _unit_top(X, e, side, d):
    out = np.zeros(X.shape[:-1] + (d,))
    if e == d - 1 and side == 1:
        out[..., d - 1] = -1.0
    return out


def sigma_function(load_kind, s0, t_ramp):
    """Load history: 0 = step (s0 for t > 0), 1 = ramp s0*min(t/t_ramp, 1)."""
    if load_kind == 0:
        return lambda t: s0 if t > 0 else 0.0
    return lambda t: s0 * min(max(t, 0.0) / t_ramp, 1.0)


def problem_from_workload(wl, theta=None, n=None):
    """Build the oracle problem of a `workloads.Workload` (optionally re-meshed)."""
    nn = tuple(n) if n is not None else tuple(wl.n)
    mesh = fe.Mesh(nn, wl.length)
    mat = fe.Material(wl.lam, wl.mu, wl.b, wl.M, wl.eta)
    if theta is None:
        theta = wl.scaled(nn).log_k()
    sig = sigma_function(wl.load_kind, wl.load_s0, wl.load_t_ramp)
    load = traction_load(mesh, mat, theta, sig)
    return SlabProblem(mesh, mat, wl.r, wl.tau, np.asarray(theta, float), load)


def field_errors(prob: SlabProblem, X, Xref):
    """Relative l2 error per field over all levels of one slab vector."""
    out = {}
    for name, s in prob.mesh.field_slices().items():
        a = np.concatenate([prob.level(X, i)[s] for i in range(prob.L)])
        b = np.concatenate([prob.level(Xref, i)[s] for i in range(prob.L)])
        nb = np.linalg.norm(b)
        out[name] = np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)
    return out
