"""Pressure-misfit functional with a hand-written discrete adjoint behind
torch.autograd.

J(theta) = 1/2 sum_n sum_s (p_h(x_s, t_n) - p_obs[n, s])^2 over the slab end
times t_n of a march from a zero initial state, theta = cellwise log K.
Forward: the library marches the slabs and checkpoints the state entering
every slab (one spatial vector per slab), then evaluates J.  Backward: the
library's adjoint sweep recomputes each slab from its checkpoint, solves the
transposed slab system backward in time (the dG jump coupling transposed) and
accumulates dJ/dtheta per cell.  Every arithmetic step runs in libbiotst.
"""
from __future__ import annotations

import numpy as np
import torch

from .native import BiotSlab


class PressureMisfit(torch.autograd.Function):
    """J = PressureMisfit.apply(log_k, slab, nslabs, sensors, p_obs, opts).

    log_k: float64 tensor (concatenated cells of all instances of `slab`);
    returns a float64 tensor with one J per instance.
    """

    @staticmethod
    def forward(ctx, log_k, slab: BiotSlab, nslabs, sensors, p_obs, opts=None):
        opts = dict(opts or {})
        sizes = [int(np.prod(w.n)) for w in slab.wls]
        host = log_k.detach().to("cpu", torch.float64).numpy()
        parts, o = [], 0
        for s in sizes:
            parts.append(host[o:o + s])
            o += s
        slab.set_log_k(parts)
        dev = slab.device
        state = slab.zeros_state()
        chk = torch.zeros(nslabs * slab.state_len, dtype=torch.float64, device=dev)
        infos, st = slab.step(nslabs, 0.0, state, checkpoints=chk, **opts)
        if st != 0:
            raise RuntimeError(f"forward march failed: {infos}")
        # end-of-slab states: checkpoint n+1 is the state after slab n; the last is `state`
        ends = torch.cat([chk[slab.state_len:], state])
        obs = torch.as_tensor(p_obs, dtype=torch.float64, device=dev).reshape(-1)
        J = slab.misfit(nslabs, ends, sensors, obs)
        ctx.slab, ctx.nslabs, ctx.sensors, ctx.opts = slab, nslabs, sensors, opts
        # the handle is shared: another forward (a line search, a finite-difference
        # probe) may set a different field before this backward runs
        ctx.log_k_parts = [p.copy() for p in parts]
        ctx.save_for_backward(chk, obs)
        return torch.tensor(J, dtype=torch.float64, device=log_k.device)

    @staticmethod
    def backward(ctx, gJ):
        chk, obs = ctx.saved_tensors
        slab = ctx.slab
        slab.set_log_k(ctx.log_k_parts)
        J, grad, st = slab.adjoint(ctx.nslabs, 0.0, chk, ctx.sensors, obs, **ctx.opts)
        if st != 0:
            raise RuntimeError("adjoint sweep failed")
        # chain rule per instance: dL/dtheta = sum_k gJ_k dJ_k/dtheta
        scale = torch.cat([gJ[k].expand(int(np.prod(w.n))) for k, w in enumerate(slab.wls)])
        return (grad * scale).to(gJ.device), None, None, None, None, None
