"""biot_misfit_noalloc (the misfit with a static device scratch, for callers
that cannot allocate) against biot_misfit through the C ABI: two calls in a
row on the same GPU, the second on a smaller input (fewer slabs and sensors,
another handle), each equal to biot_misfit's J on the same states."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import small_workload, torch_cuda

pytestmark = pytest.mark.gpu


def _march(h, ns, torch):
    state = h.zeros_state()
    chk = torch.zeros(ns * h.state_len, dtype=torch.float64, device="cuda")
    infos, st = h.step(ns, 0.0, state, checkpoints=chk)
    assert st == 0, infos
    return torch.cat([chk[h.state_len:], state])


def test_misfit_noalloc_matches_misfit_twice():
    torch = torch_cuda()
    from paper_1801_04984_amd import BiotSlab
    big = [small_workload(2, (13, 11), 1, seed=3, load_kind=W.LOAD_RAMP),
           small_workload(2, (9, 16), 1, seed=4, load_kind=W.LOAD_RAMP)]
    small = [small_workload(3, (4, 3, 5), 1, seed=5, load_kind=W.LOAD_RAMP)]
    rng = np.random.default_rng(7)
    for wls, ns, nsens in ((big, 4, 200), (small, 2, 9)):
        h = BiotSlab(wls, [w.log_k() for w in wls])
        ends = _march(h, ns, torch)
        sens = W.sensors(nsens, wls[0].dim, 31 + nsens)
        p_obs = torch.tensor(0.05 * rng.standard_normal(len(wls) * ns * nsens), device="cuda")
        J_ref = h.misfit(ns, ends, sens, p_obs)
        J = h.misfit_noalloc(ns, ends, sens, p_obs)
        assert all(np.isfinite(J_ref)) and min(J_ref) > 0
        np.testing.assert_allclose(J, J_ref, rtol=1e-14, atol=0.0)
        h.close()


def test_misfit_noalloc_rejects_beyond_scratch():
    torch = torch_cuda()
    from paper_1801_04984_amd import BiotSlab
    from paper_1801_04984_amd.native import BiotError
    wl = small_workload(2, (6, 5), 0, seed=8)
    h = BiotSlab([wl], [wl.log_k()])
    ends = torch.zeros(h.state_len, dtype=torch.float64, device="cuda")
    nsens = 40000   # 40000 * 136 bytes > 4 MiB
    sens = W.sensors(nsens, 2, 9)
    p_obs = torch.zeros(nsens, dtype=torch.float64, device="cuda")
    with pytest.raises(BiotError, match="scratch"):
        h.misfit_noalloc(1, ends, sens, p_obs)
    h.close()
