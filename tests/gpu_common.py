"""Helpers shared by the GPU parity tests: build the HIP handle and the
oracle problem for the same workload, seeded inputs."""
import numpy as np
import pytest

import workloads as W


def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def make_pair(wls, thetas=None, pair_mode=0):
    """(BiotSlab over all wls, list of oracle SlabProblems); pair_mode 0 is
    the library's default (BIOT_PAIR_AUTO)."""
    from oracle import slab
    from paper_1801_04984_amd import BiotSlab
    thetas = thetas if thetas is not None else [w.log_k() for w in wls]
    h = BiotSlab(wls, thetas, pair_mode=pair_mode)
    probs = [slab.problem_from_workload(w, theta=t) for w, t in zip(wls, thetas)]
    return h, probs


def field_rel(prob, a, b):
    """max over fields of relative l2 difference (slab vectors)."""
    out = {}
    for name, s in prob.mesh.field_slices().items():
        aa = np.concatenate([prob.level(a, i)[s] for i in range(prob.L)])
        bb = np.concatenate([prob.level(b, i)[s] for i in range(prob.L)])
        nb = np.linalg.norm(bb)
        out[name] = np.linalg.norm(aa - bb) / (nb if nb > 0 else 1.0)
    return out


def small_workload(d, n, r, seed=1, **kw):
    base = dict(lam=1.3, mu=0.7, b=0.8, M=7.0, eta=1.2, k_sigma=1.0, k_ell=0.2, k_seed=seed)
    if d == 3:
        base.update(lam=2.0, mu=1.0, b=0.9, M=5.0)
    base.update(kw)
    return W.Workload(f"t{d}_{n}_{r}", d, tuple(n), r, 0.05, 3, **base)
