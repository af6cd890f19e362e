"""ctypes binding of libbiotst.so (the C ABI in include/biotst.h).

Argument marshalling only: every step of the slab apply / solve runs in the
HIP library.  Torch is used for device memory (the caller-owned workspace
and vectors) and for the current HIP stream.  If the library is missing
this module raises; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbiotst.so")

BIOT_OK = 0
STATUS_NAMES = {0: "OK", 1: "ERR_ARG", 2: "ERR_WORKSPACE", 3: "ERR_DEVICE", 4: "ERR_NOCONV",
                5: "ERR_BREAKDOWN", 6: "ERR_NONFINITE"}

# every symbol the header declares
EXPORTS = [
    "biot_workspace_bytes", "create_slab_problem", "destroy_slab_problem", "biot_set_log_k",
    "biot_sizes", "biot_totals", "apply_operator", "slab_rhs", "solve_slab",
    "solve_slab_transposed", "step", "adjoint_sweep", "biot_misfit", "biot_autotune",
    "biot_get_tuning", "biot_set_tuning", "biot_misfit_noalloc", "biot_elasticity_apply", "solve_slab_fixed_stress", "biot_last_error",
]


class Desc(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("n", ctypes.c_int32 * 3), ("length", ctypes.c_double * 3),
        ("r", ctypes.c_int32), ("tau", ctypes.c_double), ("lam", ctypes.c_double),
        ("mu", ctypes.c_double), ("b", ctypes.c_double), ("M", ctypes.c_double),
        ("eta", ctypes.c_double), ("L_fs", ctypes.c_double), ("load_kind", ctypes.c_int32),
        ("load_s0", ctypes.c_double), ("load_t_ramp", ctypes.c_double), ("pair_mode", ctypes.c_int32),
    ]


class SolveOpts(ctypes.Structure):
    _fields_ = [
        ("rtol", ctypes.c_double), ("maxit", ctypes.c_int32), ("restart", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("inner_rtol", ctypes.c_double),
        ("max_refine", ctypes.c_int32), ("cheb_degree", ctypes.c_int32), ("graph", ctypes.c_int32),
    ]


class SolveInfo(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int32), ("restarts", ctypes.c_int32), ("ir_sweeps", ctypes.c_int32),
        ("status", ctypes.c_int32), ("rel_residual", ctypes.c_double),
    ]

    def as_dict(self):
        return dict(iterations=self.iterations, restarts=self.restarts, ir_sweeps=self.ir_sweeps,
                    status=self.status, rel_residual=self.rel_residual)


class FsOpts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("max_outer", ctypes.c_int32), ("inner_rtol", ctypes.c_double),
                ("inner_maxit", ctypes.c_int32)]


class FsInfo(ctypes.Structure):
    _fields_ = [("outer", ctypes.c_int32), ("flow_iterations", ctypes.c_int32), ("mech_iterations", ctypes.c_int32),
                ("status", ctypes.c_int32), ("rel_residual", ctypes.c_double)]

    def as_dict(self):
        return dict(outer=self.outer, flow_iterations=self.flow_iterations, mech_iterations=self.mech_iterations,
                    status=self.status, rel_residual=self.rel_residual)


class Tuning(ctypes.Structure):
    _fields_ = [
        ("apply_variant", ctypes.c_int32 * 2), ("n_variants", ctypes.c_int32),
        ("apply_us", (ctypes.c_double * 4) * 2),
    ]

    def as_dict(self):
        return dict(apply_variant=list(self.apply_variant), n_variants=self.n_variants,
                    apply_us=[list(r) for r in self.apply_us])


class BiotError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH):
    """Load the shared library (raises OSError if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError(f"{path} is missing: build it with paper_1801_04984_amd/build.py")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.biot_last_error.restype = ctypes.c_char_p
    lib.biot_workspace_bytes.argtypes = [ctypes.POINTER(Desc), i32, ctypes.POINTER(ctypes.c_size_t)]
    lib.create_slab_problem.argtypes = [ctypes.POINTER(Desc), i32, ctypes.POINTER(ctypes.POINTER(dbl)),
                                        P, ctypes.c_size_t, P, ctypes.POINTER(P)]
    lib.destroy_slab_problem.argtypes = [P]
    lib.biot_set_log_k.argtypes = [P, ctypes.POINTER(ctypes.POINTER(dbl)), P]
    lib.biot_sizes.argtypes = [P, i32, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.biot_totals.argtypes = [P, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.apply_operator.argtypes = [P, P, P, i32, i32, P]
    lib.biot_elasticity_apply.argtypes = [P, P, P, i32, P]
    lib.solve_slab_fixed_stress.argtypes = [P, P, P, ctypes.POINTER(FsOpts), ctypes.POINTER(FsInfo), P]
    lib.slab_rhs.argtypes = [P, P, dbl, P, P]
    lib.solve_slab.argtypes = [P, P, P, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo), P]
    lib.solve_slab_transposed.argtypes = [P, P, P, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo), P]
    lib.step.argtypes = [P, i32, dbl, P, P, P, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo), P]
    lib.adjoint_sweep.argtypes = [P, i32, dbl, P, ctypes.POINTER(dbl), i32, P, ctypes.POINTER(SolveOpts),
                                  ctypes.POINTER(dbl), P, P]
    lib.biot_misfit.argtypes = [P, i32, P, ctypes.POINTER(dbl), i32, P, ctypes.POINTER(dbl), P]
    lib.biot_misfit_noalloc.argtypes = [P, i32, P, ctypes.POINTER(dbl), i32, P, ctypes.POINTER(dbl), P]
    lib.biot_autotune.argtypes = [P, i32, ctypes.POINTER(Tuning), P]
    lib.biot_get_tuning.argtypes = [P, ctypes.POINTER(Tuning)]
    lib.biot_set_tuning.argtypes = [P, ctypes.POINTER(Tuning)]
    for name in EXPORTS:
        if name != "biot_last_error":
            getattr(lib, name).restype = ctypes.c_int32
    _lib = lib
    return lib


def _check(status):
    if status != BIOT_OK:
        msg = _lib.biot_last_error().decode()
        raise BiotError(status, msg)


PAIR_AUTO, PAIR_DROP, PAIR_PRESB, PAIR_SHIFT = 0, 1, 2, 3


def make_desc(wl, pair_mode=PAIR_AUTO, L_fs=0.0) -> Desc:
    """Descriptor from a workloads.Workload."""
    d = Desc()
    d.dim = wl.dim
    for e in range(3):
        d.n[e] = int(wl.n[e]) if e < wl.dim else 1
        d.length[e] = float(wl.length[e]) if e < len(wl.length) else 1.0
    d.r = wl.r
    d.tau = wl.tau
    d.lam, d.mu, d.b, d.M, d.eta = wl.lam, wl.mu, wl.b, wl.M, wl.eta
    d.L_fs = float(L_fs)
    d.load_kind = wl.load_kind
    d.load_s0 = wl.load_s0
    d.load_t_ramp = wl.load_t_ramp
    d.pair_mode = int(pair_mode)
    return d


def make_opts(rtol=1e-12, maxit=2000, restart=30, precision=0, inner_rtol=1e-2, max_refine=30,
              cheb_degree=-1, graph=1) -> SolveOpts:
    o = SolveOpts()
    o.rtol, o.maxit, o.restart, o.precision = rtol, maxit, restart, precision
    o.inner_rtol, o.max_refine, o.cheb_degree, o.graph = inner_rtol, max_refine, cheb_degree, graph
    return o


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream(torch, device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class BiotSlab:
    """A handle over one or several (batched) slab problems on one GPU."""

    def __init__(self, workloads: Sequence, log_k: Sequence[np.ndarray], device="cuda:0", pair_mode=PAIR_AUTO,
                 L_fs=0.0):
        import torch
        self.torch = torch
        self.lib = load_library()
        self.device = torch.device(device)
        self.wls = list(workloads)
        self.count = len(self.wls)
        self.descs = (Desc * self.count)(*[make_desc(w, pair_mode, L_fs) for w in self.wls])
        self._logk = [np.ascontiguousarray(np.asarray(k, dtype=np.float64)) for k in log_k]
        arr = (ctypes.POINTER(ctypes.c_double) * self.count)(
            *[k.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for k in self._logk])
        nbytes = ctypes.c_size_t()
        _check(self.lib.biot_workspace_bytes(self.descs, self.count, ctypes.byref(nbytes)))
        self.ws_bytes = nbytes.value
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        _check(self.lib.create_slab_problem(self.descs, self.count, arr, _ptr(self.workspace),
                                            self.ws_bytes, _stream(torch, self.device), ctypes.byref(h)))
        self.h = h
        sl, st = ctypes.c_int64(), ctypes.c_int64()
        _check(self.lib.biot_totals(self.h, ctypes.byref(sl), ctypes.byref(st)))
        self.slab_len, self.state_len = sl.value, st.value
        self.level_dofs, self.slab_offsets, self.state_offsets = [], [], []
        for k in range(self.count):
            a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
            _check(self.lib.biot_sizes(self.h, k, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
            self.level_dofs.append(a.value)
            self.slab_offsets.append(b.value)
            self.state_offsets.append(c.value)

    def close(self):
        if getattr(self, "h", None):
            self.lib.destroy_slab_problem(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers ---------------------------------------------------------------
    def _stream(self):
        return _stream(self.torch, self.device)

    def zeros_slab(self, dtype=None):
        return self.torch.zeros(self.slab_len, dtype=dtype or self.torch.float64, device=self.device)

    def zeros_state(self):
        return self.torch.zeros(self.state_len, dtype=self.torch.float64, device=self.device)

    def set_log_k(self, log_k):
        self._logk = [np.ascontiguousarray(np.asarray(k, dtype=np.float64)) for k in log_k]
        arr = (ctypes.POINTER(ctypes.c_double) * self.count)(
            *[k.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for k in self._logk])
        _check(self.lib.biot_set_log_k(self.h, arr, self._stream()))

    # -- calls -------------------------------------------------------------------
    def apply(self, x, y=None, transpose=False):
        torch = self.torch
        dtype = 1 if x.dtype == torch.float32 else 0
        if y is None:
            y = torch.empty_like(x)
        assert x.numel() == self.slab_len and y.numel() == self.slab_len and y.dtype == x.dtype
        assert x.is_contiguous() and y.is_contiguous()
        _check(self.lib.apply_operator(self.h, _ptr(x), _ptr(y), int(transpose), dtype, self._stream()))
        return y

    def elasticity_apply(self, x, y=None):
        """y_u = tau A x_u on the u-blocks of every level, essential DoFs eliminated (their rows 0;
        q, p entries of y untouched)."""
        torch = self.torch
        dtype = 1 if x.dtype == torch.float32 else 0
        if y is None:
            y = torch.zeros_like(x)
        assert x.numel() == self.slab_len and y.numel() == self.slab_len and y.dtype == x.dtype
        assert x.is_contiguous() and y.is_contiguous()
        _check(self.lib.biot_elasticity_apply(self.h, _ptr(x), _ptr(y), dtype, self._stream()))
        return y

    def rhs(self, state, t_start, out=None):
        if out is None:
            out = self.zeros_slab()
        _check(self.lib.slab_rhs(self.h, _ptr(state), float(t_start), _ptr(out), self._stream()))
        return out

    def solve(self, rhs, x=None, transpose=False, **opt):
        if x is None:
            x = self.zeros_slab()
        opts = make_opts(**opt)
        infos = (SolveInfo * self.count)()
        fn = self.lib.solve_slab_transposed if transpose else self.lib.solve_slab
        st = fn(self.h, _ptr(rhs), _ptr(x), ctypes.byref(opts), infos, self._stream())
        return x, [i.as_dict() for i in infos], st

    def solve_fixed_stress(self, rhs, x=None, rtol=1e-12, max_outer=1000, inner_rtol=1e-4, inner_maxit=500):
        """Fixed-stress iterative coupling of the slab system (solve_slab_fixed_stress)."""
        if x is None:
            x = self.zeros_slab()
        o = FsOpts()
        o.rtol, o.max_outer, o.inner_rtol, o.inner_maxit = rtol, max_outer, inner_rtol, inner_maxit
        infos = (FsInfo * self.count)()
        st = self.lib.solve_slab_fixed_stress(self.h, _ptr(rhs), _ptr(x), ctypes.byref(o), infos, self._stream())
        return x, [i.as_dict() for i in infos], st

    def step(self, nslabs, t_start, state, slabs_out=None, checkpoints=None, **opt):
        opts = make_opts(**opt)
        infos = (SolveInfo * (self.count * nslabs))()
        st = self.lib.step(self.h, int(nslabs), float(t_start), _ptr(state),
                           _ptr(slabs_out) if slabs_out is not None else None,
                           _ptr(checkpoints) if checkpoints is not None else None,
                           ctypes.byref(opts), infos, self._stream())
        return [i.as_dict() for i in infos], st

    def adjoint(self, nslabs, t_start, checkpoints, sensors_xyz, p_obs, grad=None, **opt):
        torch = self.torch
        sens = np.ascontiguousarray(np.asarray(sensors_xyz, dtype=np.float64))
        nsens = sens.shape[0]
        if grad is None:
            grad = torch.zeros(sum(int(np.prod(w.n)) for w in self.wls), dtype=torch.float64, device=self.device)
        J = (ctypes.c_double * self.count)()
        opts = make_opts(**opt)
        st = self.lib.adjoint_sweep(self.h, int(nslabs), float(t_start), _ptr(checkpoints),
                                    sens.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), nsens,
                                    _ptr(p_obs), ctypes.byref(opts), J, _ptr(grad), self._stream())
        return list(J), grad, st

    def misfit(self, nslabs, end_states, sensors_xyz, p_obs):
        sens = np.ascontiguousarray(np.asarray(sensors_xyz, dtype=np.float64))
        J = (ctypes.c_double * self.count)()
        _check(self.lib.biot_misfit(self.h, int(nslabs), _ptr(end_states),
                                    sens.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), sens.shape[0],
                                    _ptr(p_obs), J, self._stream()))
        return list(J)

    def misfit_noalloc(self, nslabs, end_states, sensors_xyz, p_obs):
        """biot_misfit_noalloc: the misfit with a static device scratch (no allocation)."""
        sens = np.ascontiguousarray(np.asarray(sensors_xyz, dtype=np.float64))
        J = (ctypes.c_double * self.count)()
        _check(self.lib.biot_misfit_noalloc(self.h, int(nslabs), _ptr(end_states),
                                            sens.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), sens.shape[0],
                                            _ptr(p_obs), J, self._stream()))
        return list(J)

    # -- tile autotuner ----------------------------------------------------------
    def autotune(self, reps=20):
        t = Tuning()
        _check(self.lib.biot_autotune(self.h, int(reps), ctypes.byref(t), self._stream()))
        return t.as_dict()

    def get_tuning(self):
        t = Tuning()
        _check(self.lib.biot_get_tuning(self.h, ctypes.byref(t)))
        return t.as_dict()

    def set_tuning(self, apply_variant):
        t = Tuning()
        t.apply_variant[0], t.apply_variant[1] = int(apply_variant[0]), int(apply_variant[1])
        _check(self.lib.biot_set_tuning(self.h, ctypes.byref(t)))

    # -- layout helpers (host) ---------------------------------------------------
    def instance_slab(self, vec, k):
        n = self.level_dofs[k] * (self.wls[k].r + 1)
        return vec[self.slab_offsets[k]: self.slab_offsets[k] + n]

    def instance_state(self, vec, k):
        return vec[self.state_offsets[k]: self.state_offsets[k] + self.level_dofs[k]]
