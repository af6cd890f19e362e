"""Seeded synthetic inputs for the space-time Biot slab workloads.

This module is shared by the CPU oracle, the tests and the benchmark.  It
holds workload descriptions (mesh, dG order, slab length, material constants,
load history) and seeded random generators (log-permeability fields, sensor
positions, random directions and vectors).  It contains none of the
discretisation's arithmetic: no basis functions, no quadrature, no operator.

The paper (Koecher, "Space-Time-Parallel Poroelasticity Simulation", section
"Numerical Simulations") shows its test setting only as a figure, so every
workload here is synthetic: heterogeneous media are drawn as Gaussian
log-permeability fields with a squared-exponential covariance on cell centres.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

# load_kind values (shared numbering with the C descriptor)
LOAD_STEP = 0   # sigma(t) = s0 for t > 0
LOAD_RAMP = 1   # sigma(t) = s0 * min(t / t_ramp, 1)


@dataclass
class Workload:
    """One slab-marching problem on the box [0, L]^dim with n cells per axis."""
    name: str
    dim: int
    n: Tuple[int, ...]
    r: int
    tau: float
    nslabs: int
    lam: float = 1.0
    mu: float = 1.0
    b: float = 0.8
    M: float = 10.0
    eta: float = 1.0
    length: Tuple[float, ...] = (1.0, 1.0, 1.0)
    t0: float = 0.0
    load_kind: int = LOAD_RAMP
    load_s0: float = 1.0
    load_t_ramp: float = 0.2
    k_sigma: float = 0.0        # log-K standard deviation (0 -> K == 1)
    k_ell: float = 0.1          # squared-exponential correlation length
    k_seed: int = 0

    @property
    def ncells(self) -> int:
        return int(np.prod(self.n))

    def log_k(self) -> np.ndarray:
        """Cellwise theta = log K, float64, x-fastest, length prod(n)."""
        if self.k_sigma == 0.0:
            return np.zeros(self.ncells)
        return log_k_field(self.n, self.length[: self.dim], self.k_sigma,
                           self.k_ell, self.k_seed)

    def scaled(self, n: Tuple[int, ...], **kw) -> "Workload":
        """Same physics on another mesh (and optionally other fields)."""
        return dataclasses.replace(self, n=tuple(n), **kw)


def log_k_field(n: Tuple[int, ...], length: Tuple[float, ...], sigma: float,
                ell: float, seed: int) -> np.ndarray:
    """Gaussian field with covariance sigma^2 exp(-|x-y|^2 / (2 ell^2)).

    The kernel is separable, so theta = sigma (L_z kron L_y kron L_x) xi with
    L_dir the symmetric square root of the 1D correlation matrix on the cell
    centres (negative eigenvalues from round-off clipped to zero) and xi iid
    N(0, 1) drawn from PCG64(seed) in x-fastest order.
    """
    d = len(n)
    rng = np.random.Generator(np.random.PCG64(seed))
    xi = rng.standard_normal(int(np.prod(n)))
    roots = []
    for e in range(d):
        h = length[e] / n[e]
        xc = (np.arange(n[e]) + 0.5) * h
        C = np.exp(-((xc[:, None] - xc[None, :]) ** 2) / (2.0 * ell * ell))
        w, V = np.linalg.eigh(C)
        roots.append((V * np.sqrt(np.maximum(w, 0.0))) @ V.T)
    field_ = xi.reshape(tuple(reversed(n)))      # (nz,) ny, nx
    # apply L_x along the last axis, L_y along the next, ...
    for e in range(d):
        axis = d - 1 - e
        field_ = np.moveaxis(np.tensordot(roots[e], field_, axes=([1], [axis])), 0, axis)
    return sigma * field_.reshape(-1)


def sensors(nsens: int, dim: int, seed: int) -> np.ndarray:
    """Sensor positions ~ U(0,1)^dim, shape (nsens, dim)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(0.0, 1.0, size=(nsens, dim))


def unit_directions(count: int, size: int, seed: int) -> np.ndarray:
    """count directions ~ N(0, I) normalised to unit 2-norm, shape (count, size)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    D = rng.standard_normal((count, size))
    return D / np.linalg.norm(D, axis=1, keepdims=True)


def random_vector(size: int, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(size)


# ---------------------------------------------------------------------------
# The five workloads.  T = 1 for all of them.
# ---------------------------------------------------------------------------

def c1_terzaghi() -> Workload:
    """2D 8x8, dG(0), 10 slabs, K == 1, unit step load: Terzaghi consolidation."""
    return Workload("c1_terzaghi_2d_8", 2, (8, 8), 0, 0.1, 10, lam=1.0, mu=1.0,
                    b=0.8, M=10.0, eta=1.0, load_kind=LOAD_STEP, load_s0=1.0)


def c2_hetero2d() -> Workload:
    """2D 128x128, dG(1), 50 slabs, log-normal K (sigma 1, ell 0.1, seed 2), ramp load."""
    return Workload("c2_hetero_2d_128_dg1", 2, (128, 128), 1, 0.02, 50, lam=1.0,
                    mu=1.0, b=0.8, M=10.0, eta=1.0, load_kind=LOAD_RAMP,
                    k_sigma=1.0, k_ell=0.1, k_seed=2)


def c3_hetero3d() -> Workload:
    """3D 32^3, dG(1), 20 slabs, log-normal K (sigma 1.5, ell 0.15, seed 3)."""
    return Workload("c3_hetero_3d_32_dg1", 3, (32, 32, 32), 1, 0.05, 20, lam=2.0,
                    mu=1.0, b=0.9, M=5.0, eta=1.0, load_kind=LOAD_RAMP,
                    k_sigma=1.5, k_ell=0.15, k_seed=3)


def c4_adjoint3d() -> Workload:
    """3D 48^3, dG(2), 10 slabs, c3 materials, log-normal K seed 4."""
    return Workload("c4_adjoint_3d_48_dg2", 3, (48, 48, 48), 2, 0.1, 10, lam=2.0,
                    mu=1.0, b=0.9, M=5.0, eta=1.0, load_kind=LOAD_RAMP,
                    k_sigma=1.5, k_ell=0.15, k_seed=4)


C4_SENSOR_SEED = 40
C4_DIRECTION_SEED = 41
C4_OBS_K_SEED = 5
C4_NSENS = 64
C4_NDIRS = 20


def c5_batch(count: int = 64, nmin: int = 32, nmax: int = 128) -> List[Workload]:
    """count independent 2D instances, n_i ~ U{nmin..nmax}, sigma_i ~ U[0.5, 2].

    Instance i draws (n_i, sigma_i) from PCG64(1000 + i) and its log-K field
    from seed 1000 + i; materials are those of the 2D heterogeneous workload.
    """
    out = []
    for i in range(count):
        rng = np.random.Generator(np.random.PCG64(1000 + i))
        ni = int(rng.integers(nmin, nmax + 1))
        sig = float(rng.uniform(0.5, 2.0))
        out.append(Workload(f"c5_inst{i}", 2, (ni, ni), 1, 0.05, 20, lam=1.0, mu=1.0,
                            b=0.8, M=10.0, eta=1.0, load_kind=LOAD_RAMP,
                            k_sigma=sig, k_ell=0.1, k_seed=1000 + i))
    return out


ALL = {
    "c1": c1_terzaghi,
    "c2": c2_hetero2d,
    "c3": c3_hetero3d,
    "c4": c4_adjoint3d,
}
