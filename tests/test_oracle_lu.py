"""The oracle's direct solver: the nested-dissection LU and SuperLU's COLAMD
LU factor the same slab matrix (section "Monolithic Approach"), so their
solutions agree to rounding; that spread is the oracle's own floor.  The
condition estimate agrees with the exact 1-norm condition number of a small
slab matrix."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import fe, slab


def _problems(wl, n):
    a = slab.problem_from_workload(wl, n=n)
    b = slab.problem_from_workload(wl, theta=a.theta, n=n)
    b.ordering = "colamd"
    return a, b


@pytest.mark.parametrize("case", ["2d", "3d"])
def test_nd_and_colamd_agree(case):
    if case == "2d":
        wl, n = W.c2_hetero2d(), (21, 17)
    else:
        wl, n = W.c4_adjoint3d(), (4, 5, 3)
    nd, cm = _problems(wl, n)
    rng = np.random.default_rng(3)
    b = nd.rhs(0.1, rng.standard_normal(nd.N))
    for transpose in (False, True):
        x1 = nd.solve(b, transpose=transpose)
        x2 = cm.solve(b, transpose=transpose)
        errs = slab.field_errors(nd, x1, x2)
        assert max(errs.values()) <= 1e-12, errs
        A = nd.slab_matrix()
        r = b - (A.T @ x1 if transpose else A @ x1)
        assert np.linalg.norm(r) <= 1e-13 * np.linalg.norm(b)


def test_nested_dissection_separates_the_halves():
    """On a 2D grid graph the top-level separator disconnects the two halves:
    no edge joins a vertex of the first half to one of the second."""
    m = 17
    idx = np.arange(m * m).reshape(m, m)
    e = np.concatenate([np.stack([idx[:, :-1].ravel(), idx[:, 1:].ravel()], 1),
                        np.stack([idx[:-1, :].ravel(), idx[1:, :].ravel()], 1)])
    G = sp.coo_matrix((np.ones(len(e)), (e[:, 0], e[:, 1])), shape=(m * m, m * m))
    G = (G + G.T).tocsr()
    X = np.zeros((m * m, 2))
    X[:, 0] = np.arange(m * m) % m
    X[:, 1] = np.arange(m * m) // m
    perm = slab.nested_dissection(G, X, leaf=8)
    assert np.array_equal(np.sort(perm), np.arange(m * m))
    # the last block is the separator: the column x = 7 (17 vertices, the lower side of the median cut)
    sep = perm[-m:]
    assert set(X[sep, 0]) == {7.0}
    rest = np.setdiff1d(np.arange(m * m), sep)
    left = rest[X[rest, 0] < 7]
    right = rest[X[rest, 0] > 7]
    assert G[left][:, right].nnz == 0


def test_condition_estimate_matches_dense():
    wl = W.c2_hetero2d()
    prob = slab.problem_from_workload(wl, n=(4, 3))
    A = prob.slab_matrix().toarray()
    exact = np.linalg.cond(A, 1)
    est = prob.condition_estimate()
    assert exact / 3.0 <= est <= exact * (1 + 1e-9), (est, exact)
