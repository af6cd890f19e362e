"""Mixed finite elements in space (section "Discretisation in Space").

Test infrastructure only: part of the FP64 CPU oracle.  Slow, assembled,
written from the definitions: every element matrix is a 3-point-Gauss
quadrature of basis-function products, assembled into scipy.sparse.

Spaces on a uniform box mesh of n_0 x ... x n_{d-1} cells:
  * displacement u: continuous Q2, one nodal array (2n+1)^d per component;
  * flux q: Raviart-Thomas of order 1 (the face element written Nc^f(2) in
    the paper): component c is quadratic Lagrange on {0, 1/2, 1} along x_c and
    linear Lagrange on the two Gauss points along the other axes, so the
    normal component is shared across faces (H(div)); array (2n+1) along c,
    2n along the others;
  * pressure p: discontinuous Q1 (dQ(1)) with Lagrange nodes on the 2-point
    Gauss points of each cell; array (2n)^d.
Arrays are lexicographic, x fastest.  A spatial level vector is
[u_0 .. u_{d-1}, q_0 .. q_{d-1}, p].

Forms (derived from the strong form of section "Poroelasticity" with the
mean-stress substitution; the mass equation is multiplied by -1):
  a(u,v)  = (2 mu eps(u), eps(v)) + (lam div u, div v)
  E_ij    = (psi_j, div phi_i)            (u rows, p columns)
  Mq_ij   = (eta K^-1 w_j, w_i)
  B_ij    = -(psi_j, div w_i)              (q rows, p columns)
  Mp_ij   = (psi_j, psi_i)
  K_s = [[A, 0, -bE], [0, Mq, B], [0, B^T, 0]]
  M_t = [[0, 0, 0], [0, 0, 0], [-bE^T, 0, -(1/M) Mp]]
Boundary conditions: bottom (x_{d-1} = 0) u = 0 and q.n = 0; lateral faces
u.n = 0 (roller) and q.n = 0; top (x_{d-1} = 1) traction and drained
pressure (natural).  Essential rows become identity rows, their columns are
dropped (all essential data are homogeneous here).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

SQ3 = np.sqrt(3.0)
CLOSED = np.array([0.0, 0.5, 1.0])
OPEN = np.array([0.5 - 0.5 / SQ3, 0.5 + 0.5 / SQ3])
GAUSS3_S = 0.5 + 0.5 * np.array([-np.sqrt(0.6), 0.0, np.sqrt(0.6)])
GAUSS3_W = np.array([5.0, 8.0, 5.0]) / 18.0


def lagrange_1d(nodes, s):
    """Values and derivatives of the Lagrange basis on `nodes` at points s.

    Returns (V, dV) with shape (len(nodes), len(s)).
    """
    nodes = np.asarray(nodes, float)
    s = np.atleast_1d(np.asarray(s, float))
    k = len(nodes)
    V = np.ones((k, len(s)))
    dV = np.zeros((k, len(s)))
    for a in range(k):
        for b in range(k):
            if b == a:
                continue
            V[a] *= (s - nodes[b]) / (nodes[a] - nodes[b])
        for c in range(k):
            if c == a:
                continue
            term = np.ones(len(s)) / (nodes[a] - nodes[c])
            for b in range(k):
                if b in (a, c):
                    continue
                term = term * (s - nodes[b]) / (nodes[a] - nodes[b])
            dV[a] += term
    return V, dV


@dataclass
class Mesh:
    n: tuple
    length: tuple

    def __post_init__(self):
        self.n = tuple(int(v) for v in self.n)
        self.d = len(self.n)
        self.length = tuple(float(v) for v in self.length[: self.d])
        self.h = tuple(L / n for L, n in zip(self.length, self.n))
        d = self.d
        self.su = tuple(2 * n + 1 for n in self.n)
        self.sq = [tuple(2 * self.n[e] + 1 if e == c else 2 * self.n[e] for e in range(d))
                   for c in range(d)]
        self.sp = tuple(2 * n for n in self.n)
        self.nu1 = int(np.prod(self.su))
        self.nq = [int(np.prod(s)) for s in self.sq]
        self.np_ = int(np.prod(self.sp))
        offs = []
        o = 0
        for c in range(d):
            offs.append(o)
            o += self.nu1
        self.off_u = offs
        offs = []
        for c in range(d):
            offs.append(o)
            o += self.nq[c]
        self.off_q = offs
        self.off_p = o
        self.N = o + self.np_
        self.ncells = int(np.prod(self.n))

    # -- field slices of one spatial level ---------------------------------
    def field_slices(self):
        return {
            "u": slice(0, self.off_q[0]),
            "q": slice(self.off_q[0], self.off_p),
            "p": slice(self.off_p, self.N),
        }

    # -- cells ---------------------------------------------------------------
    def cell_index_grid(self):
        """(ncells, d) integer cell coordinates, x fastest."""
        grids = np.meshgrid(*[np.arange(n) for n in self.n], indexing="ij")
        # ravel in x-fastest order: the last axis in C order must be x
        idx = np.stack([g.transpose(tuple(reversed(range(self.d)))).reshape(-1)
                        for g in grids], axis=1)
        return idx

    @staticmethod
    def _flat(m, sizes):
        out = np.zeros(m.shape[:-1], dtype=np.int64)
        stride = 1
        for e, s in enumerate(sizes):
            out += m[..., e] * stride
            stride *= s
        return out


def local_dofs(d):
    """Local DoF table: list of (block, comp, local multi-index)."""
    out = []
    for c in range(d):
        for a in itertools.product(range(3), repeat=d):
            out.append(("u", c, tuple(reversed(a))))
    for c in range(d):
        shape = [3 if e == c else 2 for e in range(d)]
        for a in itertools.product(*[range(s) for s in reversed(shape)]):
            out.append(("q", c, tuple(reversed(a))))
    for a in itertools.product(range(2), repeat=d):
        out.append(("p", 0, tuple(reversed(a))))
    return out


def global_map(mesh: Mesh):
    """(ncells, nloc) global indices of the local DoFs of every cell."""
    cells = mesh.cell_index_grid()
    loc = local_dofs(mesh.d)
    G = np.zeros((mesh.ncells, len(loc)), dtype=np.int64)
    for l, (blk, c, a) in enumerate(loc):
        m = 2 * cells + np.array(a)[None, :]
        if blk == "u":
            G[:, l] = mesh.off_u[c] + Mesh._flat(m, mesh.su)
        elif blk == "q":
            G[:, l] = mesh.off_q[c] + Mesh._flat(m, mesh.sq[c])
        else:
            G[:, l] = mesh.off_p + Mesh._flat(m, mesh.sp)
    return G


def eval_local_basis(d, pts, h):
    """Evaluate all local basis functions at reference points pts (npts, d).

    Returns dict with
      val  (nloc, npts, d)  vector value (u, q) ; p uses comp 0
      grad (nloc, npts, d, d) physical gradient of vector fields (u only)
      div  (nloc, npts)     physical divergence (u, q)
      pval (nloc, npts)     scalar value for p DoFs
    """
    loc = local_dofs(d)
    npts = pts.shape[0]
    Vc, dVc, Vo, dVo = [], [], [], []
    for e in range(d):
        v, dv = lagrange_1d(CLOSED, pts[:, e])
        Vc.append(v); dVc.append(dv / h[e])
        v, dv = lagrange_1d(OPEN, pts[:, e])
        Vo.append(v); dVo.append(dv / h[e])
    nl = len(loc)
    val = np.zeros((nl, npts, d))
    grad = np.zeros((nl, npts, d, d))
    div = np.zeros((nl, npts))
    pval = np.zeros((nl, npts))
    for l, (blk, c, a) in enumerate(loc):
        if blk == "u":
            V = [Vc[e][a[e]] for e in range(d)]
            dV = [dVc[e][a[e]] for e in range(d)]
        elif blk == "q":
            V = [(Vc if e == c else Vo)[e][a[e]] for e in range(d)]
            dV = [(dVc if e == c else dVo)[e][a[e]] for e in range(d)]
        else:
            V = [Vo[e][a[e]] for e in range(d)]
            dV = None
        phi = np.prod(np.array(V), axis=0)
        if blk == "p":
            pval[l] = phi
            continue
        val[l, :, c] = phi
        for e in range(d):
            fac = np.ones(npts)
            for e2 in range(d):
                fac = fac * (dV[e2] if e2 == e else V[e2])
            grad[l, :, c, e] = fac
        div[l] = grad[l, :, c, c]
    return loc, val, grad, div, pval


def gauss_points(d, n1=3):
    s, w = GAUSS3_S, GAUSS3_W
    pts = np.array(list(itertools.product(s, repeat=d)))[:, ::-1]
    wts = np.prod(np.array(list(itertools.product(w, repeat=d))), axis=1)
    return pts, wts


@dataclass
class Material:
    lam: float
    mu: float
    b: float
    M: float
    eta: float


def element_matrices(d, h, mat: Material):
    """Reference-cell matrices (same for every cell of a uniform mesh).

    Returns dict: A (nu,nu), E (nu,np), Mq1 (nq,nq) with K == 1, B (nq,np), Mp.
    """
    pts, wts = gauss_points(d)
    W = wts * np.prod(h)
    loc, val, grad, div, pval = eval_local_basis(d, pts, h)
    iu = [l for l, t in enumerate(loc) if t[0] == "u"]
    iq = [l for l, t in enumerate(loc) if t[0] == "q"]
    ip = [l for l, t in enumerate(loc) if t[0] == "p"]
    eps = 0.5 * (grad + np.swapaxes(grad, 2, 3))
    A = (2 * mat.mu * np.einsum("iqab,jqab,q->ij", eps[iu], eps[iu], W)
         + mat.lam * np.einsum("iq,jq,q->ij", div[iu], div[iu], W))
    E = np.einsum("iq,jq,q->ij", div[iu], pval[ip], W)
    Mq1 = mat.eta * np.einsum("iqa,jqa,q->ij", val[iq], val[iq], W)
    B = -np.einsum("iq,jq,q->ij", div[iq], pval[ip], W)
    Mp = np.einsum("iq,jq,q->ij", pval[ip], pval[ip], W)
    return dict(A=A, E=E, Mq1=Mq1, B=B, Mp=Mp, iu=iu, iq=iq, ip=ip)


def constrained_mask(mesh: Mesh):
    """Boolean mask over one spatial level: True for essential DoFs."""
    d = mesh.d
    mask = np.zeros(mesh.N, bool)

    def multi(sizes):
        g = np.meshgrid(*[np.arange(s) for s in sizes], indexing="ij")
        return np.stack([x.transpose(tuple(reversed(range(d)))).reshape(-1) for x in g], 1)

    mu_ = multi(mesh.su)
    for c in range(d):
        m = np.zeros(mesh.nu1, bool)
        m |= mu_[:, d - 1] == 0                         # bottom: all components
        if c < d - 1:                                   # lateral: normal component
            m |= (mu_[:, c] == 0) | (mu_[:, c] == mesh.su[c] - 1)
        mask[mesh.off_u[c]: mesh.off_u[c] + mesh.nu1] = m
    for c in range(d):
        mq = multi(mesh.sq[c])
        if c < d - 1:
            m = (mq[:, c] == 0) | (mq[:, c] == mesh.sq[c][c] - 1)
        else:
            m = mq[:, c] == 0                           # bottom no-flow; top drained
        mask[mesh.off_q[c]: mesh.off_q[c] + mesh.nq[c]] = m
    return mask


def cell_matrices(mesh: Mesh, mat: Material):
    """Per-cell blocks over the local DoFs (order of local_dofs):
    K_s of a cell = Ks_static + (1/K_cell) Mq_loc, and M_t of a cell = Mt_loc
    (section "Monolithic Approach" block structure, mass equation negated)."""
    em = element_matrices(mesh.d, mesh.h, mat)
    iu, iq, ip = em["iu"], em["iq"], em["ip"]
    nl = len(iu) + len(iq) + len(ip)
    Ks_static = np.zeros((nl, nl))
    Ks_static[np.ix_(iu, iu)] = em["A"]
    Ks_static[np.ix_(iu, ip)] = -mat.b * em["E"]
    Ks_static[np.ix_(iq, ip)] = em["B"]
    Ks_static[np.ix_(ip, iq)] = em["B"].T
    Mq_loc = np.zeros((nl, nl))
    Mq_loc[np.ix_(iq, iq)] = em["Mq1"]
    Mt_loc = np.zeros((nl, nl))
    Mt_loc[np.ix_(ip, iu)] = -mat.b * em["E"].T
    Mt_loc[np.ix_(ip, ip)] = -(1.0 / mat.M) * em["Mp"]
    return Ks_static, Mq_loc, Mt_loc


def assemble_spatial(mesh: Mesh, mat: Material, theta):
    """Global K_s and M_t (unconstrained), CSR, for cellwise theta = log K."""
    G = global_map(mesh)
    nl = G.shape[1]
    Ks_static, Mq_loc, Mt_loc = cell_matrices(mesh, mat)
    kinv = np.exp(-np.asarray(theta, float))
    rows = np.repeat(G, nl, axis=1).reshape(-1)
    cols = np.tile(G, (1, nl)).reshape(-1)

    def asm(vals):
        return sp.coo_matrix((vals.reshape(-1), (rows, cols)), shape=(mesh.N, mesh.N)).tocsr()

    nc = mesh.ncells
    Ks = asm(np.broadcast_to(Ks_static, (nc, nl, nl)))
    Ks = Ks + asm(kinv[:, None, None] * Mq_loc[None])
    Mt = asm(np.broadcast_to(Mt_loc, (nc, nl, nl)))
    Ks.eliminate_zeros()
    Mt.eliminate_zeros()
    return Ks, Mt


def mq_cell_matrix(mesh: Mesh, mat: Material):
    """Reference M_q element matrix with K == 1 and the q local index list."""
    em = element_matrices(mesh.d, mesh.h, mat)
    return em["Mq1"], em["iq"]


# -- loads --------------------------------------------------------------------

def load_vector(mesh: Mesh, mat: Material, theta, t, fu=None, fq=None, fp=None,
                traction=None, p_drained=None):
    """F(t) of one spatial level.

    fu(x, t) -> (..., d) body force; fq(x, t, K) -> (..., d) Darcy source;
    fp(x, t) -> (...) mass source; traction(x, t, e, side) -> (..., d) on the
    boundary face x_e = side*L_e; p_drained(x, t) -> (...) on the top face.
    Entries: [int fu.v + int_dOmega t.v ; int fq.w - int_top pD w.n ; -int fp psi].
    """
    d = mesh.d
    F = np.zeros(mesh.N)
    G = global_map(mesh)
    cells = mesh.cell_index_grid()
    h = np.array(mesh.h)
    pts, wts = gauss_points(d)
    loc, val, grad, div, pval = eval_local_basis(d, pts, h)
    W = wts * np.prod(h)
    X = (cells[:, None, :] + pts[None, :, :]) * h[None, None, :]     # (nc, nq, d)
    iu = [l for l, tt in enumerate(loc) if tt[0] == "u"]
    iq = [l for l, tt in enumerate(loc) if tt[0] == "q"]
    ip = [l for l, tt in enumerate(loc) if tt[0] == "p"]
    K = np.exp(np.asarray(theta, float))
    if fu is not None:
        f = fu(X, t)
        contrib = np.einsum("cqa,lqa,q->cl", f, val[iu], W)
        np.add.at(F, G[:, iu], contrib)
    if fq is not None:
        f = fq(X, t, K[:, None])
        contrib = np.einsum("cqa,lqa,q->cl", f, val[iq], W)
        np.add.at(F, G[:, iq], contrib)
    if fp is not None:
        f = fp(X, t)
        contrib = -np.einsum("cq,lq,q->cl", f, pval[ip], W)
        np.add.at(F, G[:, ip], contrib)
    if traction is not None or p_drained is not None:
        s1, w1 = GAUSS3_S, GAUSS3_W
        for e in range(d):
            for side in (0, 1):
                other = [e2 for e2 in range(d) if e2 != e]
                fp_ = np.array(list(itertools.product(s1, repeat=d - 1)))[:, ::-1] if d > 1 else np.zeros((1, 0))
                fw = np.prod(np.array(list(itertools.product(w1, repeat=d - 1))), axis=1)
                fw = fw * np.prod(h[other])
                fpts = np.zeros((len(fw), d))
                fpts[:, other] = fp_
                fpts[:, e] = float(side)
                _, fval, _, _, _ = eval_local_basis(d, fpts, h)
                sel = cells[:, e] == (0 if side == 0 else mesh.n[e] - 1)
                Xf = (cells[sel][:, None, :] + fpts[None]) * h[None, None, :]
                if traction is not None:
                    tr = traction(Xf, t, e, side)
                    contrib = np.einsum("cqa,lqa,q->cl", tr, fval[iu], fw)
                    np.add.at(F, G[sel][:, iu], contrib)
                if p_drained is not None and e == d - 1 and side == 1:
                    pdv = p_drained(Xf, t)
                    nrm = np.zeros(d); nrm[e] = 1.0
                    wn = np.einsum("lqa,a->lq", fval[iq], nrm)
                    contrib = -np.einsum("cq,lq,q->cl", pdv, wn, fw)
                    np.add.at(F, G[sel][:, iq], contrib)
    return F


# -- interpolation and point evaluation ----------------------------------------

def dof_coordinates(mesh: Mesh):
    """Physical coordinates of every DoF of one level, shape (N, d)."""
    d = mesh.d
    h = np.array(mesh.h)
    X = np.zeros((mesh.N, d))

    def grid(sizes, kinds):
        axes = []
        for e in range(d):
            if kinds[e] == "c":
                axes.append(np.arange(sizes[e]) * h[e] / 2.0)
            else:
                o = np.arange(sizes[e])
                axes.append((o // 2 + OPEN[o % 2]) * h[e])
        g = np.meshgrid(*axes, indexing="ij")
        return np.stack([x.transpose(tuple(reversed(range(d)))).reshape(-1) for x in g], 1)

    for c in range(d):
        X[mesh.off_u[c]: mesh.off_u[c] + mesh.nu1] = grid(mesh.su, "c" * d)
    for c in range(d):
        kinds = ["c" if e == c else "o" for e in range(d)]
        X[mesh.off_q[c]: mesh.off_q[c] + mesh.nq[c]] = grid(mesh.sq[c], kinds)
    X[mesh.off_p:] = grid(mesh.sp, "o" * d)
    return X


def interpolate(mesh: Mesh, u, q, p, t):
    """Nodal interpolant of fields u(x,t)->(...,d), q(x,t)->(...,d), p(x,t)->(...)."""
    X = dof_coordinates(mesh)
    v = np.zeros(mesh.N)
    d = mesh.d
    for c in range(d):
        s = slice(mesh.off_u[c], mesh.off_u[c] + mesh.nu1)
        v[s] = u(X[s], t)[..., c]
    for c in range(d):
        s = slice(mesh.off_q[c], mesh.off_q[c] + mesh.nq[c])
        v[s] = q(X[s], t)[..., c]
    s = slice(mesh.off_p, mesh.N)
    v[s] = p(X[s], t)
    return v


def pressure_point_matrix(mesh: Mesh, pts):
    """Sparse (npts, N) matrix evaluating the DG-Q1 pressure at points.

    The containing cell is floor(x / h) per axis, clipped to the mesh: a point
    on an interior face belongs to the cell above it along that axis (the cell
    whose lower face it lies on), a point on the upper boundary to the last cell.
    """
    d = mesh.d
    h = np.array(mesh.h)
    pts = np.atleast_2d(pts)
    rows, cols, vals = [], [], []
    for k, x in enumerate(pts):
        cell = np.minimum(np.floor(x / h).astype(int), np.array(mesh.n) - 1)
        cell = np.maximum(cell, 0)
        s = x / h - cell
        for a in itertools.product(range(2), repeat=d):
            w = 1.0
            for e in range(d):
                V, _ = lagrange_1d(OPEN, [s[e]])
                w *= V[a[e], 0]
            m = 2 * cell + np.array(a)
            idx = mesh.off_p + int(Mesh._flat(m[None, :], mesh.sp)[0])
            rows.append(k); cols.append(idx); vals.append(w)
    return sp.coo_matrix((vals, (rows, cols)), shape=(len(pts), mesh.N)).tocsr()
