"""Pressure-misfit functional and its log-permeability gradient.

Test infrastructure only: part of the FP64 CPU oracle.

J(theta) = 1/2 sum_n sum_s (p_h(x_s, t_n) - p_obs[n, s])^2 with p_h the
end-of-slab pressure (last Radau coefficient) and theta = log K per cell.
Every slab solves A(theta) X_n = tau F_n + G X_{n-1} with the jump operator
G X = P_free (g kron M_t) X_{n-1, r}.  Reverse sweep (discrete adjoint):

    A^T L_n = dJ/dX_n + G^T L_{n+1},      L_{N+1} = 0,

and dJ/dtheta_c = - sum_n L_n^T (dA/dtheta_c) X_n.  Only the flux mass
matrix depends on theta: dA/dtheta_c = -tau eta exp(-theta_c) P_free
(I kron Mq1_c) P_free, with Mq1_c the K == 1 flux mass matrix of cell c.
"""
from __future__ import annotations

import numpy as np

from . import fe
from .slab import SlabProblem


def misfit(prob: SlabProblem, Xs, P, p_obs):
    J = 0.0
    for n, X in enumerate(Xs):
        res = P @ prob.level(X, prob.r) - p_obs[n]
        J += 0.5 * float(res @ res)
    return J


def gradient(prob: SlabProblem, nslabs, P, p_obs, x0_end=None):
    """Return (J, dJ/dtheta, forward slab vectors)."""
    Xs = prob.march(nslabs, x0_end)
    J = misfit(prob, Xs, P, p_obs)
    N, L, r = prob.N, prob.L, prob.r
    free = prob.free.astype(float)
    Mq1, iq = fe.mq_cell_matrix(prob.mesh, prob.mat)
    G = fe.global_map(prob.mesh)[:, iq]                 # (ncells, nq_loc)
    grad = np.zeros(prob.mesh.ncells)
    lam_next = None
    for n in range(nslabs - 1, -1, -1):
        X = Xs[n]
        rhs = np.zeros(L * N)
        res = P @ prob.level(X, r) - p_obs[n]
        rhs[r * N:(r + 1) * N] += P.T @ res
        if lam_next is not None:
            comb = np.zeros(N)
            for i in range(L):
                comb += prob.g[i] * (free * prob.level(lam_next, i))
            rhs[r * N:(r + 1) * N] += prob.Mt.T @ comb
        lam = prob.solve(rhs, transpose=True)
        for i in range(L):
            Li = (free * prob.level(lam, i))[G]         # (ncells, nq_loc)
            Xi = (free * prob.level(X, i))[G]
            grad += prob.tau * np.exp(-prob.theta) * np.einsum("ca,ab,cb->c", Li, Mq1, Xi)
        lam_next = lam
    return J, grad, Xs
