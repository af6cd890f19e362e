"""Host-side logic of the library checked without a GPU: small C++ programs
built with hipcc against the library's own headers and run on the CPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1801_04984_amd", "csrc")


def _run(src, tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "check")
    r = subprocess.run([hipcc, "-O1", "-std=c++17", "-I", CSRC, os.path.join(ROOT, "tests", "host", src), "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr


def test_xcd_tile_order_is_a_contiguous_permutation(tmp_path):
    _run("xcd_order_check.cpp", tmp_path)


def test_temporal_constants_match_oracle(tmp_path):
    """The library's dG(r) constants (temporal.cpp, host code) against the
    oracle's: Radau nodes and weights, T = W^-1 D, g = W^-1 phi(0), and the
    real block eigenform Q^-1 T Q (2x2 blocks [[alpha, beta], [-beta, alpha]]
    for complex pairs, alpha on the diagonal for real eigenvalues)."""
    import json

    import numpy as np

    from oracle import temporal
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "dump")
    r = subprocess.run([gxx, "-O1", "-std=c++17", "-I", CSRC, os.path.join(ROOT, "tests", "host", "temporal_dump.cpp"),
                        os.path.join(CSRC, "temporal.cpp"), "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([exe], capture_output=True, text=True, timeout=60).stdout.strip().splitlines()
    for line in out:
        c = json.loads(line)
        rr = c["r"]
        L = rr + 1
        s, w, D, T, g = temporal.dg_matrices(rr)
        np.testing.assert_allclose(c["s"][:L], s, rtol=0, atol=1e-14)
        np.testing.assert_allclose(c["w"][:L], w, rtol=0, atol=1e-14)
        Tl = np.array(c["T"]).reshape(4, 4)[:L, :L]
        np.testing.assert_allclose(Tl, T, rtol=1e-12, atol=1e-12 * np.abs(T).max())
        np.testing.assert_allclose(c["g"][:L], g, rtol=1e-12, atol=1e-12 * np.abs(g).max())
        Q = np.array(c["Q"]).reshape(4, 4)[:L, :L]
        Qi = np.array(c["Qi"]).reshape(4, 4)[:L, :L]
        np.testing.assert_allclose(Qi @ Q, np.eye(L), atol=1e-11)
        Lam = Qi @ Tl @ Q
        alpha = np.array(c["alpha"][:L], dtype=float)
        beta = np.array(c["beta"][:L], dtype=float)
        expect = np.diag(alpha)
        for i in range(L):
            if beta[i] > 0:   # columns i, i+1 form a complex pair alpha_i +- i beta_i
                expect[i, i + 1], expect[i + 1, i] = beta[i], -beta[i]
        np.testing.assert_allclose(Lam, expect, atol=1e-10 * np.abs(Tl).max())
        # the eigenvalues of T are the alpha +- i beta the block form reports
        ev = np.sort_complex(np.linalg.eigvals(T))
        got = np.sort_complex(np.linalg.eigvals(expect))
        np.testing.assert_allclose(got, ev, atol=1e-10 * np.abs(ev).max())
        npairs = int((beta > 0).sum())
        assert npairs == (rr + 1) // 2   # Radau IIA: one real eigenvalue for odd stage counts
        for key in ("order_q", "order_pass"):
            o = c[key]
            perm = o["perm"][:L]
            assert sorted(perm) == list(range(L)), (rr, key, perm)
            assert len(o["first"]) == npairs
            # in the permuted basis each pair keeps its 2x2 block at (first, second)
            Lp = Qi[perm, :] @ Tl @ Q[:, perm]
            ex = np.diag(alpha[perm])
            for i, (f, s2) in enumerate(zip(o["first"], o["second"])):
                assert o["beta"][i] > 0 and beta[perm[f]] == o["beta"][i] and beta[perm[s2]] == -o["beta"][i]
                ex[f, s2], ex[s2, f] = o["beta"][i], -o["beta"][i]
            np.testing.assert_allclose(Lp, ex, atol=1e-10 * np.abs(Tl).max())
            if key == "order_q":
                assert perm == list(range(L)) and o["second"] == [f + 1 for f in o["first"]]
            else:   # pair firsts, real levels, pair seconds
                assert o["first"] == list(range(npairs))
                assert o["second"] == list(range(L - npairs, L))


def test_element_matrices_match_oracle(tmp_path):
    """The library's element matrices (element.cpp, host code; tau = 1):
    elasticity a(u, v) and the coupling (psi_g, d_c phi) on a 2D and a 3D box
    cell with unequal edges, against the oracle's quadrature of its own basis
    (both ordered component-major, nodes x fastest)."""
    import json

    import numpy as np

    from oracle import fe
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "edump")
    r = subprocess.run([hipcc, "-O1", "-std=c++17", "-x", "hip", "-I", CSRC,
                        os.path.join(ROOT, "tests", "host", "element_dump.cpp"), os.path.join(CSRC, "element.cpp"),
                        "--offload-arch=gfx950", "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([exe], capture_output=True, text=True, timeout=60).stdout.strip().splitlines()
    assert len(out) == 2
    h = [0.3, 0.7, 1.1]
    for line in out:
        c = json.loads(line)
        d = c["d"]
        em = fe.element_matrices(d, np.array(h[:d]), fe.Material(1.3, 0.7, 0.8, 10.0, 1.0))
        nu, npd = len(em["iu"]), len(em["ip"])
        A = np.array(c["A"]).reshape(nu, nu)
        E = np.array(c["E"]).reshape(nu, npd)
        np.testing.assert_allclose(A, em["A"], rtol=0, atol=1e-12 * np.abs(em["A"]).max())
        np.testing.assert_allclose(E, em["E"], rtol=0, atol=1e-12 * np.abs(em["E"]).max())


def test_binding_structs_match_header_layout(tmp_path):
    """Every struct of include/biotst.h, compiled with the host C compiler,
    has the size and field offsets of its ctypes mirror in the binding (the
    binding renames the descriptor's `lambda`, a Python keyword, to `lam`)."""
    import ctypes
    import json

    from paper_1801_04984_amd import native
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    exe = str(tmp_path / "layout")
    r = subprocess.run([cc, "-std=c99", "-Wall", "-I", os.path.join(ROOT, "include"),
                        os.path.join(ROOT, "tests", "host", "abi_layout.c"), "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    rows = [json.loads(l) for l in subprocess.run([exe], capture_output=True, text=True,
                                                  timeout=60).stdout.splitlines()]
    mirrors = {"biot_problem_desc": native.Desc, "biot_solve_opts": native.SolveOpts,
               "biot_solve_info": native.SolveInfo, "biot_tuning": native.Tuning,
               "biot_fs_opts": native.FsOpts, "biot_fs_info": native.FsInfo}
    assert sorted(r["name"] for r in rows) == sorted(mirrors)
    for row in rows:
        S = mirrors[row["name"]]
        assert ctypes.sizeof(S) == row["size"], row["name"]
        py = {("lambda" if n == "lam" else n): getattr(S, n).offset for n, _ in S._fields_}
        assert py == row["fields"], row["name"]
