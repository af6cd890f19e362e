"""Parity of the HIP slab solver (solve_slab / step / adjoint_sweep through
the C ABI) with the oracle's direct sparse LU solves, per field."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import field_rel, make_pair, small_workload, torch_cuda

pytestmark = pytest.mark.gpu
TOL = 1e-10
RT = 1e-13


def _rhs(prob, seed=1, t=0.1):
    state = np.random.default_rng(seed).standard_normal(prob.N)
    state[prob.mask] = 0.0
    return prob.rhs(t, state)


@pytest.mark.parametrize("n", [(12, 10), (33, 20)])
@pytest.mark.parametrize("r", [0, 1, 2])
def test_solve_fp64(n, r):
    torch = torch_cuda()
    wl = small_workload(2, n, r, seed=3 + r)
    h, (prob,) = make_pair([wl])
    b = _rhs(prob)
    ref = prob.solve(b)
    x, info, st = h.solve(torch.tensor(b, device="cuda"), rtol=RT)
    assert st == 0 and info[0]["status"] == 0, info
    err = field_rel(prob, x.cpu().numpy(), ref)
    assert max(err.values()) < TOL, err
    assert info[0]["iterations"] < 120
    h.close()


@pytest.mark.parametrize("r", [0, 1])
def test_solve_mixed_refined(r):
    torch = torch_cuda()
    wl = small_workload(2, (24, 17), r, seed=9)
    h, (prob,) = make_pair([wl])
    b = _rhs(prob, seed=2)
    ref = prob.solve(b)
    x, info, st = h.solve(torch.tensor(b, device="cuda"), precision=1)
    assert st == 0 and info[0]["ir_sweeps"] >= 1, info
    err = field_rel(prob, x.cpu().numpy(), ref)
    assert max(err.values()) < TOL, err
    h.close()


@pytest.mark.parametrize("d,n,r", [(2, (20, 13), 1), (2, (33, 20), 2), (3, (5, 4, 6), 1)])
@pytest.mark.parametrize("transpose", [False, True])
def test_solve_fp32_preconditioned_flexible(d, n, r, transpose):
    """FP64 flexible GMRES with the preconditioner applied in FP32 reaches the
    oracle's solution to the FP64 tolerance, forward and transposed."""
    torch = torch_cuda()
    wl = small_workload(d, n, r, seed=60 + d + r)
    h, (prob,) = make_pair([wl])
    b = _rhs(prob, seed=8)
    ref = prob.solve(b, transpose=transpose)
    x, info, st = h.solve(torch.tensor(b, device="cuda"), rtol=RT, precision=2, transpose=transpose)
    assert st == 0 and info[0]["ir_sweeps"] == 0, info
    err = field_rel(prob, x.cpu().numpy(), ref)
    assert max(err.values()) < TOL, err
    h.close()


@pytest.mark.parametrize("r", [1, 2])
def test_solve_batched_deep_hierarchy(r):
    """Equal-size and uneven instances whose elasticity multigrid has three
    levels (two smoothed): the coarse levels store instances with a stride of
    r+1 time levels, which the set-up must cover for every instance."""
    torch = torch_cuda()
    sizes = [(24, 24), (24, 24), (26, 22)]
    wls = [small_workload(2, n, r, seed=40 + i) for i, n in enumerate(sizes)]
    h, probs = make_pair(wls)
    bs = [_rhs(p, seed=11 + i) for i, p in enumerate(probs)]
    x, info, st = h.solve(torch.tensor(np.concatenate(bs), device="cuda"), rtol=RT)
    assert st == 0, info
    xv = x.cpu().numpy()
    for k, (p, bk) in enumerate(zip(probs, bs)):
        got = xv[h.slab_offsets[k]: h.slab_offsets[k] + p.L * p.N]
        err = field_rel(p, got, p.solve(bk))
        assert max(err.values()) < TOL, (k, err)
    h.close()


def test_solve_batched_uneven_matches_single():
    torch = torch_cuda()
    wls = [small_workload(2, n, 1, seed=20 + i, b=0.6 + 0.1 * i) for i, n in enumerate([(9, 9), (21, 14), (16, 16)])]
    h, probs = make_pair(wls)
    bs = [_rhs(p, seed=5 + i) for i, p in enumerate(probs)]
    b = np.concatenate(bs)
    x, info, st = h.solve(torch.tensor(b, device="cuda"), rtol=RT)
    assert st == 0, info
    xv = x.cpu().numpy()
    for k, (p, bk) in enumerate(zip(probs, bs)):
        got = xv[h.slab_offsets[k]: h.slab_offsets[k] + p.L * p.N]
        err = field_rel(p, got, p.solve(bk))
        assert max(err.values()) < TOL, (k, err)
    h.close()


def test_solve_transposed():
    torch = torch_cuda()
    wl = small_workload(2, (14, 11), 1, seed=31)
    h, (prob,) = make_pair([wl])
    b = np.random.default_rng(8).standard_normal(prob.L * prob.N)
    ref = prob.solve(b, transpose=True)
    x, info, st = h.solve(torch.tensor(b, device="cuda"), transpose=True)
    assert st == 0, info
    err = field_rel(prob, x.cpu().numpy(), ref)
    assert max(err.values()) < TOL, err
    h.close()


@pytest.mark.parametrize("r", [0, 1])
def test_step_matches_oracle_march_and_resumes(r):
    torch = torch_cuda()
    wl = small_workload(2, (13, 9), r, seed=41, load_kind=W.LOAD_RAMP)
    h, (prob,) = make_pair([wl])
    ns = 4
    ref = prob.march(ns)
    state = h.zeros_state()
    slabs = torch.zeros(ns * h.slab_len, dtype=torch.float64, device="cuda")
    chk = torch.zeros(ns * h.state_len, dtype=torch.float64, device="cuda")
    infos, st = h.step(ns, 0.0, state, slabs_out=slabs, checkpoints=chk)
    assert st == 0, infos
    sv = slabs.cpu().numpy().reshape(ns, -1)
    for n in range(ns):
        err = field_rel(prob, sv[n], ref[n])
        assert max(err.values()) < TOL, (n, err)
    cv = chk.cpu().numpy().reshape(ns, -1)
    assert np.all(cv[0] == 0.0)
    for n in range(1, ns):
        np.testing.assert_array_equal(cv[n], sv[n - 1][r * prob.N:(r + 1) * prob.N])
    # resume: 2 + 2 slabs from the saved state equals 4 straight (bitwise), with
    # checkpoints (every slab starts from its entering state) and without (the
    # march predictor carries over from the first call to the second)
    s2 = h.zeros_state()
    c2 = torch.zeros(2 * h.state_len, dtype=torch.float64, device="cuda")
    h.step(2, 0.0, s2, checkpoints=c2)
    h.step(2, 2 * wl.tau, s2, checkpoints=c2)
    np.testing.assert_array_equal(s2.cpu().numpy(), state.cpu().numpy())
    s4 = h.zeros_state()
    h.step(4, 0.0, s4)
    s3 = h.zeros_state()
    h.step(2, 0.0, s3)
    h.step(2, 2 * wl.tau, s3)
    np.testing.assert_array_equal(s3.cpu().numpy(), s4.cpu().numpy())
    err = field_rel(prob, np.tile(s4.cpu().numpy(), prob.L), np.tile(ref[-1][r * prob.N:(r + 1) * prob.N], prob.L))
    assert max(err.values()) < TOL, err
    h.close()


def test_terzaghi_workload_on_gpu():
    torch = torch_cuda()
    wl = W.c1_terzaghi()
    h, (prob,) = make_pair([wl])
    ref = prob.march(wl.nslabs)
    state = h.zeros_state()
    slabs = torch.zeros(wl.nslabs * h.slab_len, dtype=torch.float64, device="cuda")
    infos, st = h.step(wl.nslabs, 0.0, state, slabs_out=slabs)
    assert st == 0
    sv = slabs.cpu().numpy().reshape(wl.nslabs, -1)
    for n in range(wl.nslabs):
        err = field_rel(prob, sv[n], ref[n])
        assert max(err.values()) < TOL, (n, err)
    # x-invariance of the GPU pressure (1D consolidation)
    p = sv[-1][prob.mesh.off_p:prob.N].reshape(prob.mesh.sp[1], prob.mesh.sp[0])
    assert np.abs(p - p[:, :1]).max() < 1e-9 * np.abs(p).max()
    h.close()


def test_error_paths():
    torch = torch_cuda()
    wl = small_workload(2, (10, 10), 1, seed=2)
    h, (prob,) = make_pair([wl])
    b = _rhs(prob)
    x, info, st = h.solve(torch.tensor(b, device="cuda"), maxit=1)
    assert st == 4 and info[0]["status"] == 4 and info[0]["iterations"] == 1
    assert np.isfinite(info[0]["rel_residual"]) and info[0]["rel_residual"] > 1e-13
    bad = b.copy()
    bad[5] = np.nan
    x, info, st = h.solve(torch.tensor(bad, device="cuda"))
    assert st == 6
    x, info, st = h.solve(torch.tensor(b, device="cuda"), restart=0)
    assert st == 1
    h.close()


@pytest.mark.parametrize("d,n", [(2, (12, 10)), (2, (21, 13)), (3, (4, 4, 3))])
def test_solve_dg3(d, n):
    """dG(3): four Radau levels whose real block eigenbasis holds two
    complex-pair blocks; forward and transposed FP64 solves, and the mixed
    refined solve, against the oracle's LU."""
    torch = torch_cuda()
    wl = small_workload(d, n, 3, seed=13 + d)
    h, (prob,) = make_pair([wl])
    b = _rhs(prob, seed=6)
    for transpose in (False, True):
        ref = prob.solve(b, transpose=transpose)
        x, info, st = h.solve(torch.tensor(b, device="cuda"), rtol=RT, transpose=transpose)
        assert st == 0 and info[0]["iterations"] < 200, info
        err = field_rel(prob, x.cpu().numpy(), ref)
        assert max(err.values()) < TOL, (transpose, err)
    x, info, st = h.solve(torch.tensor(b, device="cuda"), precision=1)
    assert st == 0, info
    err = field_rel(prob, x.cpu().numpy(), prob.solve(b))
    assert max(err.values()) < TOL, err
    h.close()


@pytest.mark.parametrize("r,precision", [(0, 0), (1, 0), (2, 0), (3, 0), (1, 1), (2, 1), (2, 2)])
def test_adjoint_gradient_matches_oracle(r, precision):
    """adjoint_sweep against the oracle's discrete adjoint, for dG(0..3) and
    with the forward and adjoint slab solves in both mixed modes."""
    torch = torch_cuda()
    from oracle import adjoint, fe
    wl = small_workload(2, (8, 7), r, seed=51, load_kind=W.LOAD_RAMP)
    theta = wl.log_k()
    h, (prob,) = make_pair([wl], [theta])
    ns = 3
    sens = W.sensors(7, 2, 61)
    P = fe.pressure_point_matrix(prob.mesh, sens)
    p_obs = 0.05 * np.random.default_rng(3).standard_normal((ns, len(sens)))
    Jref, gref, _ = adjoint.gradient(prob, ns, P, p_obs)
    state = h.zeros_state()
    chk = torch.zeros(ns * h.state_len, dtype=torch.float64, device="cuda")
    infos, st = h.step(ns, 0.0, state, checkpoints=chk, precision=precision)
    assert st == 0
    p_obs_d = torch.tensor(p_obs.reshape(-1), device="cuda")
    J, g, st = h.adjoint(ns, 0.0, chk, sens, p_obs_d, precision=precision)
    assert st == 0
    assert abs(J[0] - Jref) <= 1e-9 * abs(Jref)
    gv = g.cpu().numpy()
    assert np.linalg.norm(gv - gref) <= 1e-8 * np.linalg.norm(gref), (np.abs(gv - gref).max(), np.abs(gref).max())
    # the adjoint's recomputed slabs are the marched ones: its J equals the
    # misfit of the marched end states up to the order of the sum over slabs
    ends = torch.cat([chk[h.state_len:], state])
    Jf = h.misfit(ns, ends, sens, p_obs_d)
    assert abs(J[0] - Jf[0]) <= 8 * np.finfo(float).eps * abs(Jf[0]), (J[0], Jf[0])
    h.close()


@pytest.mark.parametrize("n,r", [((4, 4, 4), 1), ((9, 7, 8), 1), ((5, 5, 5), 2)])
def test_solve3d_fp64_and_mixed(n, r):
    torch = torch_cuda()
    wl = small_workload(3, n, r, seed=70 + r)
    h, (prob,) = make_pair([wl])
    b = _rhs(prob, seed=3)
    ref = prob.solve(b)
    x, info, st = h.solve(torch.tensor(b, device="cuda"), rtol=RT)
    assert st == 0 and info[0]["iterations"] < 150, info
    err = field_rel(prob, x.cpu().numpy(), ref)
    assert max(err.values()) < TOL, err
    x, info, st = h.solve(torch.tensor(b, device="cuda"), precision=1)
    assert st == 0, info
    err = field_rel(prob, x.cpu().numpy(), ref)
    assert max(err.values()) < TOL, err
    h.close()


# lines of 20 and 130 cells: one wavefront per line (1 and 4 equations per
# lane); 520 cells: one thread per line (Thomas sweep).  The strips keep
# square cells (length 0.01 per cell).
@pytest.mark.parametrize("d,n,length", [(2, (20, 13), (1.0, 1.0)), (2, (130, 3), (1.3, 0.03)),
                                        (2, (520, 2), (5.2, 0.02)), (3, (5, 4, 6), (1.0, 1.0, 1.0))])
def test_flux_block_variants(d, n, length):
    """The flux-mass block of the preconditioner solved exactly line by line
    (default) or by Chebyshev-Jacobi: both preconditioned solves reach the
    oracle's solution; the exact block needs no more iterations."""
    torch = torch_cuda()
    wl = small_workload(d, n, 1, seed=90 + d, length=tuple(length) + (1.0,) * (3 - d))
    h, (prob,) = make_pair([wl])
    b = _rhs(prob, seed=4)
    ref = prob.solve(b)
    its = {}
    for deg in (0, 8):
        x, info, st = h.solve(torch.tensor(b, device="cuda"), rtol=RT, cheb_degree=deg)
        assert st == 0, (deg, info)
        err = field_rel(prob, x.cpu().numpy(), ref)
        assert max(err.values()) < TOL, (deg, err)
        its[deg] = info[0]["iterations"]
    assert its[0] <= its[8] + 2, its
    h.close()


@pytest.mark.parametrize("r", [1, 2])
def test_step3d_and_adjoint(r):
    torch = torch_cuda()
    from oracle import adjoint, fe
    wl = small_workload(3, (4, 3, 4), r, seed=81, load_kind=W.LOAD_RAMP)
    theta = wl.log_k()
    h, (prob,) = make_pair([wl], [theta])
    ns = 2
    ref = prob.march(ns)
    state = h.zeros_state()
    slabs = torch.zeros(ns * h.slab_len, dtype=torch.float64, device="cuda")
    chk = torch.zeros(ns * h.state_len, dtype=torch.float64, device="cuda")
    infos, st = h.step(ns, 0.0, state, slabs_out=slabs, checkpoints=chk)
    assert st == 0
    sv = slabs.cpu().numpy().reshape(ns, -1)
    for k in range(ns):
        err = field_rel(prob, sv[k], ref[k])
        assert max(err.values()) < TOL, err
    sens = W.sensors(5, 3, 91)
    P = fe.pressure_point_matrix(prob.mesh, sens)
    p_obs = 0.05 * np.random.default_rng(5).standard_normal((ns, len(sens)))
    Jref, gref, _ = adjoint.gradient(prob, ns, P, p_obs)
    J, g, st = h.adjoint(ns, 0.0, chk, sens, torch.tensor(p_obs.reshape(-1), device="cuda"))
    assert st == 0
    assert abs(J[0] - Jref) <= 1e-9 * abs(Jref)
    gv = g.cpu().numpy()
    assert np.linalg.norm(gv - gref) <= 1e-8 * np.linalg.norm(gref)
    h.close()


@pytest.mark.parametrize("transpose", [False, True])
@pytest.mark.parametrize("precision", [0, 1, 2])
def test_graph_replay_matches_eager(precision, transpose):
    """The captured graphs (the preconditioner, and every Arnoldi step:
    preconditioner, operator, Gram-Schmidt, normalisation), replayed many
    times with eager work and host synchronisations in between, give
    bit-identical solves; so do graphs captured again after the operator's
    tile variant changes."""
    torch = torch_cuda()
    wls = [small_workload(2, n, 1, seed=90 + i) for i, n in enumerate([(17, 12), (9, 9)])]
    h, probs = make_pair(wls)
    b = torch.tensor(np.concatenate([_rhs(p, seed=i) for i, p in enumerate(probs)]), device="cuda")
    xe, ie, se = h.solve(b, precision=precision, graph=0, transpose=transpose)
    for rep in range(3):
        xg, ig, sg = h.solve(b, precision=precision, graph=1, transpose=transpose)
        torch.cuda.synchronize()
        assert se == 0 and sg == 0
        assert torch.equal(xg, xe), rep
        assert [i["iterations"] for i in ig] == [i["iterations"] for i in ie]
        _ = (b * 2.0).sum().item()      # eager work and a host synchronisation between replays
    tun = h.get_tuning()
    v = tun["apply_variant"]
    h.set_tuning([(v[0] + 1) % tun["n_variants"], (v[1] + 1) % tun["n_variants"]])
    xg, ig, sg = h.solve(b, precision=precision, graph=1, transpose=transpose)
    assert sg == 0 and torch.equal(xg, xe)
    h.close()


def test_full_length_restart_cycle():
    """A 64-step restart cycle run to its end (tolerance out of reach): the last
    Krylov index takes the separate norm pass, and the solution still matches
    the oracle's."""
    torch = torch_cuda()
    wl = small_workload(2, (12, 10), 1, seed=77)
    h, (prob,) = make_pair([wl])
    b = _rhs(prob, seed=3)
    ref = prob.solve(b)
    x, info, st = h.solve(torch.tensor(b, device="cuda"), rtol=1e-30, restart=64, maxit=64)
    assert info[0]["iterations"] == 64, info
    err = field_rel(prob, x.cpu().numpy(), ref)
    assert max(err.values()) < TOL, err
    h.close()


def test_flux_line_solve_full_wavefront():
    """Lines of 511 cells, the longest the wavefront line solve takes: 512
    cell-end equations, eight per lane, every slot of the reduction in use
    (the cross lines of 2 cells run in the same launch)."""
    test_flux_block_variants(2, (511, 2), (5.11, 0.02))


@pytest.mark.parametrize("n,length", [((511, 1, 1), (5.11, 0.01, 0.01)), ((520, 1, 1), (5.2, 0.01, 0.01))])
def test_flux_line_solve_3d_long_lines(n, length):
    """3D flux lines along x of 511 cells (the wavefront line solve, every slot
    in use) and 520 cells (one thread per line), in the same launch as the
    cross lines of one cell."""
    test_flux_block_variants(3, n, length)


def test_mixed_before_refinement_per_field_error():
    """The mixed path before refinement: one FP32 inner GMRES solve (FP32
    operator and preconditioner, FP64 dot accumulation) run to its FP32
    floor, per-field relative error against the oracle's LU.  The floor of a
    single-precision solve is bounded by cond(A) eps32; on this mesh the
    measured floor is above 1e-6 for u (it is stated, with the condition
    estimate, rather than the bound loosened); refinement then reaches 1e-10."""
    torch = torch_cuda()
    wl = small_workload(2, (24, 17), 1, seed=9)
    h, (prob,) = make_pair([wl])
    b = _rhs(prob, seed=2)
    ref = prob.solve(b)
    cond = prob.condition_estimate()
    x1, info1, st1 = h.solve(torch.tensor(b, device="cuda"), precision=1, max_refine=1, inner_rtol=1e-7)
    err1 = field_rel(prob, x1.cpu().numpy(), ref)
    eps32 = float(np.finfo(np.float32).eps)
    print(f"cond_1 estimate {cond:.3e}; one FP32 sweep per-field error {err1}; "
          f"iterations {info1[0]['iterations']}")
    # measured on this mesh (cond_1 ~ 2.3e6): u 1.1e-5, q 3.3e-7, p 2.4e-6 -- the
    # single-precision floor; 1e-6 is not reachable for u in FP32 arithmetic
    assert max(err1.values()) <= min(5e-5, cond * eps32), (err1, cond)
    assert err1["q"] <= 1e-6 and err1["p"] <= 1e-5, err1
    # refinement (default inner tolerance) reaches the FP64 tolerance
    x, info, st = h.solve(torch.tensor(b, device="cuda"), precision=1)
    assert st == 0, info
    err = field_rel(prob, x.cpu().numpy(), ref)
    assert max(err.values()) < TOL, err
    h.close()


@pytest.mark.parametrize("d,n,r", [(2, (20, 13), 1), (2, (33, 20), 2), (2, (16, 12), 3), (3, (5, 4, 6), 2),
                                   (3, (4, 5, 3), 3), (3, (5, 3, 4), 1)])
def test_pair_modes_reach_the_oracle(d, n, r):
    """The treatments of the complex-pair level blocks (couplings kept by the
    square-block factorisation, dropped, dropped with the shifted level
    solve) are preconditioners of one system: all reach the oracle's solution,
    forward and transposed, FP64 and FP32-preconditioned.  The default
    (automatic) mode takes the square-block factorisation in 3D at r >= 2 and
    drops the couplings otherwise: its iteration counts are those of that mode."""
    from paper_1801_04984_amd import native
    torch = torch_cuda()
    wl = small_workload(d, n, r, seed=110 + d + r)
    its = {}
    modes = (native.PAIR_DROP, native.PAIR_PRESB, native.PAIR_SHIFT, native.PAIR_AUTO)
    for mode in modes:
        h, (prob,) = make_pair([wl], pair_mode=mode)
        b = _rhs(prob, seed=12)
        for transpose in (False, True):
            ref = prob.solve(b, transpose=transpose)
            for precision in (0, 2):
                x, info, st = h.solve(torch.tensor(b, device="cuda"), rtol=RT, transpose=transpose,
                                      precision=precision)
                assert st == 0, (mode, transpose, precision, info)
                err = field_rel(prob, x.cpu().numpy(), ref)
                assert max(err.values()) < TOL, (mode, transpose, precision, err)
                its[(mode, transpose, precision)] = info[0]["iterations"]
        h.close()
    print(f"d={d} n={n} r={r} iterations (mode, transposed, precision): {its}")
    auto_is = native.PAIR_PRESB if (d == 3 and r >= 2) else native.PAIR_DROP
    for transpose in (False, True):
        for precision in (0, 2):
            assert its[(native.PAIR_AUTO, transpose, precision)] == its[(auto_is, transpose, precision)], its
    # the kept couplings save iterations wherever the level solves are good enough to show it
    if r >= 2:
        for transpose in (False, True):
            assert its[(native.PAIR_PRESB, transpose, 0)] < its[(native.PAIR_DROP, transpose, 0)], its


@pytest.mark.parametrize("d,n,r", [(2, (12, 10), 0), (2, (16, 11), 1), (2, (12, 9), 2), (3, (4, 3, 4), 1)])
def test_fixed_stress_coupling_reaches_the_oracle(d, n, r):
    """The standalone fixed-stress iterative coupling (flow with the fixed-stress
    term, then mechanics, in turn) converges to the slab solution: the oracle's
    LU solution per field <= 1e-10, and the monolithic GMRES solution."""
    torch = torch_cuda()
    wl = small_workload(d, n, r, seed=130 + d + r)
    h, (prob,) = make_pair([wl])
    b = _rhs(prob, seed=14)
    ref = prob.solve(b)
    x, info, st = h.solve_fixed_stress(torch.tensor(b, device="cuda"), rtol=1e-13)
    assert st == 0 and info[0]["rel_residual"] <= 1e-13, info
    err = field_rel(prob, x.cpu().numpy(), ref)
    assert max(err.values()) < TOL, (err, info)
    xm, infm, stm = h.solve(torch.tensor(b, device="cuda"), rtol=RT)
    assert stm == 0
    err = field_rel(prob, x.cpu().numpy(), xm.cpu().numpy())
    assert max(err.values()) < TOL, err
    print(f"d={d} n={n} r={r}: fixed-stress {info[0]}, monolithic GMRES {infm[0]['iterations']} iterations")
    h.close()


def test_fixed_stress_parameter_scan():
    """Outer iterations of the fixed-stress coupling against L: every L >= b^2 / (2 K_dr)
    converges to the oracle's solution; the counts are printed for the record."""
    torch = torch_cuda()
    from paper_1801_04984_amd import BiotSlab
    from oracle import slab
    wl = small_workload(2, (16, 12), 1, seed=141)
    theta = wl.log_k()
    prob = slab.problem_from_workload(wl, theta=theta)
    b = _rhs(prob, seed=15)
    ref = prob.solve(b)
    L0 = wl.b ** 2 / (wl.lam + wl.mu)
    counts = {}
    for f in (0.5, 0.75, 1.0, 1.5, 2.0):
        h = BiotSlab([wl], [theta], L_fs=f * L0)
        x, info, st = h.solve_fixed_stress(torch.tensor(b, device="cuda"), rtol=1e-12)
        assert st == 0, (f, info)
        err = field_rel(prob, x.cpu().numpy(), ref)
        assert max(err.values()) < 1e-9, (f, err)
        counts[f] = info[0]["outer"]
        h.close()
    print(f"fixed-stress outer iterations against L / (b^2 / K_dr): {counts}")
