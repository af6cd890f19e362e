"""Exact separable-polynomial fields for manufactured-solution tests.

A field is a sum of terms coef * prod_e P_e(x_e) * P_t(t) with numpy
Polynomial factors, so derivatives are exact polynomial algebra (no finite
differences).  Used to build sources and boundary data whose discrete
solution must be exact when the fields lie in the discrete space.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import Polynomial as Pn


class SepPoly:
    def __init__(self, d, terms):
        self.d = d
        self.terms = list(terms)      # (coef, [P_0..P_{d-1}], P_t)

    @staticmethod
    def term(d, coef, factors, pt):
        fs = [Pn(f) if not isinstance(f, Pn) else f for f in factors]
        fs += [Pn([1.0])] * (d - len(fs))
        return SepPoly(d, [(coef, fs, Pn(pt) if not isinstance(pt, Pn) else pt)])

    def __call__(self, X, t):
        out = np.zeros(X.shape[:-1])
        for c, fs, pt in self.terms:
            v = c * pt(t)
            for e in range(self.d):
                v = v * fs[e](X[..., e])
            out = out + v
        return out

    def __add__(self, o):
        return SepPoly(self.d, self.terms + o.terms)

    def __rmul__(self, s):
        return SepPoly(self.d, [(s * c, fs, pt) for c, fs, pt in self.terms])

    def dx(self, e):
        return SepPoly(self.d, [(c, [f.deriv() if k == e else f for k, f in enumerate(fs)], pt)
                                for c, fs, pt in self.terms])

    def dt(self):
        return SepPoly(self.d, [(c, fs, pt.deriv()) for c, fs, pt in self.terms])

    @staticmethod
    def zero(d):
        return SepPoly(d, [])


class Manufactured:
    """u, q, p polynomial fields with all sources for the Biot system."""

    def __init__(self, d, u, q, p, lam, mu, b, M, eta):
        self.d, self.u, self.q, self.p = d, u, q, p
        self.lam, self.mu, self.b, self.M, self.eta = lam, mu, b, M, eta

    def _vec(self, comps, X, t):
        return np.stack([c(X, t) for c in comps], -1)

    def u_fn(self, X, t):
        return self._vec(self.u, X, t)

    def q_fn(self, X, t):
        return self._vec(self.q, X, t)

    def p_fn(self, X, t):
        return self.p(X, t)

    def stress_comp(self, i, j):
        """Total stress component sigma_ij = 2 mu eps_ij + lam div u delta_ij - b p delta_ij."""
        d = self.d
        s = self.mu * self.u[i].dx(j) + self.mu * self.u[j].dx(i)
        if i == j:
            div = SepPoly.zero(d)
            for k in range(d):
                div = div + self.u[k].dx(k)
            s = s + self.lam * div + (-self.b) * self.p
        return s

    def fu(self, X, t):
        d = self.d
        out = []
        for i in range(d):
            acc = SepPoly.zero(d)
            for j in range(d):
                acc = acc + self.stress_comp(i, j).dx(j)
            out.append((-1.0) * acc)
        return self._vec(out, X, t)

    def fq(self, X, t, K):
        return self.eta / K[..., None] * self.q_fn(X, t) + self._vec(
            [self.p.dx(e) for e in range(self.d)], X, t)

    def fp(self, X, t):
        d = self.d
        divu = SepPoly.zero(d)
        divq = SepPoly.zero(d)
        for k in range(d):
            divu = divu + self.u[k].dx(k)
            divq = divq + self.q[k].dx(k)
        f = self.b * divu.dt() + (1.0 / self.M) * self.p.dt() + divq
        return f(X, t)

    def traction(self, X, t, e, side):
        sgn = 1.0 if side == 1 else -1.0
        return np.stack([sgn * self.stress_comp(i, e)(X, t) for i in range(self.d)], -1)

    def p_drained(self, X, t):
        return self.p(X, t)
