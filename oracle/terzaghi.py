"""Terzaghi one-dimensional consolidation series (closed form).

Test infrastructure only: an analytic reference for the oracle.

A column of height H, drained at the top, impermeable and fixed at the
bottom, laterally confined, loaded at t = 0+ by a compressive top traction
sigma.  With the Biot storage S = 1/M + b^2/(lam + 2 mu) the undrained
initial pressure is p0 = b sigma / ((lam + 2 mu) S) and the consolidation
coefficient c_v = K / (eta S).  With z the depth below the drained top,

  p(z, t) = p0 sum_k 4/((2k+1) pi) sin(a_k z / H) exp(-a_k^2 c_v t / H^2),
  a_k = (2k+1) pi / 2,

and the top settlement follows from integrating the vertical strain
eps = (b p - sigma) / (lam + 2 mu) over the column.
"""
from __future__ import annotations

import numpy as np


def coefficients(lam, mu, b, M, K, eta, sigma):
    S = 1.0 / M + b * b / (lam + 2.0 * mu)
    p0 = b * sigma / ((lam + 2.0 * mu) * S)
    cv = K / (eta * S)
    return p0, cv


def pressure(z, t, lam, mu, b, M, K, eta, sigma, H=1.0, nterms=400):
    p0, cv = coefficients(lam, mu, b, M, K, eta, sigma)
    z = np.atleast_1d(np.asarray(z, float))
    k = np.arange(nterms)
    a = (2 * k + 1) * np.pi / 2.0
    terms = (4.0 / ((2 * k + 1) * np.pi))[None, :] * np.sin(np.outer(z / H, a)) \
        * np.exp(-a * a * cv * t / (H * H))[None, :]
    return p0 * terms.sum(axis=1)


def top_settlement(t, lam, mu, b, M, K, eta, sigma, H=1.0, nterms=400):
    """Vertical displacement of the loaded top (negative = downward)."""
    p0, cv = coefficients(lam, mu, b, M, K, eta, sigma)
    k = np.arange(nterms)
    a = (2 * k + 1) * np.pi / 2.0
    # int_0^H p dz = p0 H sum 4/((2k+1) pi) * (1/a_k) exp(..)  = p0 H sum 8/((2k+1)^2 pi^2) exp(..)
    pint = p0 * H * np.sum(8.0 / ((2 * k + 1) ** 2 * np.pi ** 2) * np.exp(-a * a * cv * t / (H * H)))
    return (b * pint - sigma * H) / (lam + 2.0 * mu)
