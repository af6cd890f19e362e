"""Parity of the HIP slab operator (apply_operator through the C ABI) with the
oracle's assembled slab matrix, element by element on seeded inputs."""
import numpy as np
import pytest

from tests.gpu_common import field_rel, make_pair, small_workload, torch_cuda

pytestmark = pytest.mark.gpu

SHAPES_2D = [(1, 1), (3, 2), (20, 17), (31, 16), (46, 9)]


def _check_apply(wls, dtype, transpose, seed=0):
    torch = torch_cuda()
    h, probs = make_pair(wls)
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(h.slab_len)
    xt = torch.tensor(x, dtype=dtype, device="cuda")
    yt = h.apply(xt, transpose=transpose)
    torch.cuda.synchronize()
    y = yt.double().cpu().numpy()
    for k, prob in enumerate(probs):
        xs = x[h.slab_offsets[k]: h.slab_offsets[k] + prob.L * prob.N]
        if dtype == torch.float32:
            xs = xs.astype(np.float32).astype(np.float64)
        ref = prob.apply(xs, transpose=transpose)
        got = y[h.slab_offsets[k]: h.slab_offsets[k] + prob.L * prob.N]
        if dtype == torch.float64:
            tol = 1e-12 * np.abs(ref).max()
            bad = np.abs(got - ref) > tol
            assert not bad.any(), (wls[k].name, int(bad.sum()), np.abs(got - ref).max(), tol)
        else:
            err = field_rel(prob, got, ref)
            assert max(err.values()) < 2e-5, (wls[k].name, err)
    h.close()


@pytest.mark.parametrize("n", SHAPES_2D)
@pytest.mark.parametrize("r", [0, 1, 2, 3])
@pytest.mark.parametrize("transpose", [False, True])
def test_apply2d_fp64(n, r, transpose):
    torch = torch_cuda()
    _check_apply([small_workload(2, n, r, seed=3 + r)], torch.float64, transpose)


@pytest.mark.parametrize("n", [(20, 17), (31, 16)])
@pytest.mark.parametrize("r", [1, 2])
@pytest.mark.parametrize("transpose", [False, True])
def test_apply2d_fp32(n, r, transpose):
    torch = torch_cuda()
    _check_apply([small_workload(2, n, r, seed=5)], torch.float32, transpose)


@pytest.mark.parametrize("transpose", [False, True])
def test_apply2d_batched_uneven(transpose):
    torch = torch_cuda()
    wls = [small_workload(2, n, 1, seed=10 + i, lam=1.0 + 0.3 * i, b=0.5 + 0.1 * i)
           for i, n in enumerate([(5, 5), (17, 33), (16, 16), (2, 7)])]
    _check_apply(wls, torch.float64, transpose)


@pytest.mark.parametrize("r", [0, 1, 2])
def test_slab_rhs_2d(r):
    torch = torch_cuda()
    wl = small_workload(2, (19, 16), r, seed=2)
    h, (prob,) = make_pair([wl])
    state = np.random.default_rng(4).standard_normal(prob.N)
    state[prob.mask] = 0.0
    for t0 in (0.0, 0.13, 0.5):
        got = h.rhs(torch.tensor(state, device="cuda"), t0).cpu().numpy()
        ref = prob.rhs(t0, state)
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    h.close()


SHAPES_3D = [(1, 1, 1), (2, 3, 2), (9, 8, 10), (15, 7, 9)]


@pytest.mark.parametrize("n", SHAPES_3D)
@pytest.mark.parametrize("r", [0, 1, 2])
@pytest.mark.parametrize("transpose", [False, True])
def test_apply3d_fp64(n, r, transpose):
    torch = torch_cuda()
    _check_apply([small_workload(3, n, r, seed=7 + r)], torch.float64, transpose)


@pytest.mark.parametrize("transpose", [False, True])
def test_apply3d_fp32_and_batched(transpose):
    torch = torch_cuda()
    wls = [small_workload(3, n, 1, seed=30 + i) for i, n in enumerate([(3, 3, 3), (9, 8, 10)])]
    _check_apply(wls, torch.float32, transpose)
    _check_apply(wls, torch.float64, transpose)


@pytest.mark.parametrize("r", [0, 2])
def test_slab_rhs_3d(r):
    torch = torch_cuda()
    wl = small_workload(3, (5, 4, 6), r, seed=2)
    h, (prob,) = make_pair([wl])
    state = np.random.default_rng(4).standard_normal(prob.N)
    state[prob.mask] = 0.0
    for t0 in (0.0, 0.31):
        got = h.rhs(torch.tensor(state, device="cuda"), t0).cpu().numpy()
        ref = prob.rhs(t0, state)
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    h.close()


@pytest.mark.parametrize("d,r", [(2, 1), (2, 2), (2, 3), (3, 1)])
def test_tile_variants_identical_and_autotune(d, r, tmp_path):
    """Every tile variant of the apply (2D: 16x16 and 8x8 tiles with a level
    loop, 8x8 tiles with the levels in parallel; 3D: z-chunks) gives bitwise
    the same y (FP64, FP32, transposed), the autotuner selects a valid variant
    per precision, and a cached selection is restored by the tuning module."""
    torch = torch_cuda()
    from paper_1801_04984_amd import BiotSlab, native, tuning
    if d == 2:
        wls = [small_workload(2, (37, 21), r, seed=5), small_workload(2, (9, 30), r, seed=6)]
    else:
        wls = [small_workload(3, (9, 8, 19), r, seed=7), small_workload(3, (4, 6, 5), r, seed=8)]
    h = BiotSlab(wls, [w.log_k() for w in wls])
    nv = h.get_tuning()["n_variants"]
    assert nv == 3
    rng = np.random.default_rng(3)
    x64 = torch.tensor(rng.standard_normal(h.slab_len), device="cuda")
    for dtype in (torch.float64, torch.float32):
        x = x64.to(dtype)
        for tr in (False, True):
            outs = []
            for v in range(nv):
                h.set_tuning([v, v])
                outs.append(h.apply(x, transpose=tr).clone())
            torch.cuda.synchronize()
            for v in range(1, nv):
                assert torch.equal(outs[0], outs[v]), (dtype, tr, v)
    res = h.autotune(reps=3)
    assert all(0 <= v < nv for v in res["apply_variant"])
    assert all(res["apply_us"][q][v] > 0 for q in range(2) for v in range(nv))
    with pytest.raises(native.BiotError):
        h.set_tuning([nv, 0])
    path = str(tmp_path / "tiles.json")
    first = tuning.tune(h, path=path, reps=2)
    assert first["source"] == "timed"
    h.set_tuning([0, 0])
    again = tuning.tune(h, path=path)
    assert again["source"] == "cache" and h.get_tuning()["apply_variant"] == first["apply_variant"]
    h.close()


@pytest.mark.parametrize("dims,r", [(3, 2), (2, 1)])
@pytest.mark.parametrize("fp32", [False, True])
def test_elasticity_apply(dims, r, fp32):
    """The elasticity operator of the preconditioner's fine multigrid level
    (biot_elasticity_apply: y_u = tau A x_u per time level with the essential
    DoFs eliminated, so essential rows 0; q and p entries of y untouched)
    against tau times the u-u block of the oracle's assembled K_s with the
    essential rows and columns removed.  3D covers several xy tiles, z-chunks
    with their halo layer and a batch of two uneven instances."""
    torch = torch_cuda()
    if dims == 3:
        wls = [small_workload(3, (15, 7, 9), r, seed=51), small_workload(3, (9, 8, 10), r, seed=52)]
    else:
        wls = [small_workload(2, (31, 16), r, seed=53), small_workload(2, (20, 17), r, seed=54)]
    h, probs = make_pair(wls)
    rng = np.random.default_rng(5)
    dt = torch.float32 if fp32 else torch.float64
    x = rng.standard_normal(h.slab_len)
    if fp32:
        x = x.astype(np.float32).astype(np.float64)
    sentinel = 7.25
    yt = torch.full((h.slab_len,), sentinel, dtype=dt, device="cuda")
    h.elasticity_apply(torch.tensor(x, dtype=dt, device="cuda"), yt)
    torch.cuda.synchronize()
    y = yt.double().cpu().numpy()
    for k, prob in enumerate(probs):
        su = prob.mesh.field_slices()["u"]
        Kuu = prob.Ks[su, su]
        mu = prob.mask[su]
        xs = x[h.slab_offsets[k]: h.slab_offsets[k] + prob.L * prob.N]
        ys = y[h.slab_offsets[k]: h.slab_offsets[k] + prob.L * prob.N]
        for lev in range(prob.L):
            xl, yl = prob.level(xs, lev), prob.level(ys, lev)
            xu = np.where(mu, 0.0, xl[su])
            ref = prob.tau * (Kuu @ xu)
            ref[mu] = 0.0
            got = yl[su]
            tol = (1e-5 if fp32 else 1e-12) * np.abs(ref).max()
            bad = np.abs(got - ref) > tol
            assert not bad.any(), (wls[k].name, lev, int(bad.sum()), np.abs(got - ref).max(), tol)
            assert np.all(yl[su.stop:] == sentinel), (wls[k].name, lev)
    h.close()
