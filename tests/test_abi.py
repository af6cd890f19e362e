"""C ABI checks that need no GPU: the library loads, exports every symbol
include/biotst.h declares, and rejects bad descriptors on the host with the
documented status codes and no device work."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "biotst.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:biot_status|const char\*)\s+(\w+)\s*\(", src, flags=re.M)))


def lib():
    from paper_1801_04984_amd import native
    try:
        return native.load_library()
    except OSError as e:
        pytest.skip(str(e))


def test_every_declared_symbol_is_exported():
    L = lib()
    from paper_1801_04984_amd import native
    names = header_functions()
    assert len(names) >= 12
    assert sorted(native.EXPORTS) == names
    for n in names:
        assert hasattr(L, n), n


def _ws(desc_list):
    from paper_1801_04984_amd import native
    arr = (native.Desc * len(desc_list))(*desc_list)
    nb = ctypes.c_size_t()
    st = lib().biot_workspace_bytes(arr, len(desc_list), ctypes.byref(nb))
    return st, nb.value, lib().biot_last_error().decode()


@pytest.mark.parametrize("field,value,msg", [
    ("dim", 4, "dim"), ("r", 4, "r must"), ("tau", 0.0, "tau"), ("mu", -1.0, "mu"),
    ("b", 1.0, "Biot coefficient"), ("b", 0.0, "Biot coefficient"), ("M", 0.0, "modulus"),
    ("eta", -2.0, "viscosity"), ("load_kind", 7, "load_kind"), ("load_t_ramp", 0.0, "ramp"),
    ("lam", -5.0, "lambda"), ("tau", float("nan"), "tau"),
])
def test_descriptor_validation(field, value, msg):
    from paper_1801_04984_amd import native
    d = native.make_desc(W.c2_hetero2d())
    setattr(d, field, value)
    st, _, err = _ws([d])
    assert st == 1 and msg in err


def test_batch_rules_and_sizes():
    from paper_1801_04984_amd import native
    a = native.make_desc(W.c2_hetero2d())
    b = native.make_desc(W.c3_hetero3d())
    st, _, err = _ws([a, b])
    assert st == 1 and "dim" in err
    c = native.make_desc(W.c2_hetero2d())
    c.r = 2
    st, _, err = _ws([a, c])
    assert st == 1 and "share r" in err
    e = native.make_desc(W.c2_hetero2d())
    e.tau = 0.5 * a.tau
    st, _, err = _ws([a, e])
    assert st == 1 and "share tau" in err
    st, n1, _ = _ws([a])
    st2, n2, _ = _ws([a, a])
    assert st == 0 and st2 == 0 and n2 > n1 > 0
    d = native.make_desc(W.c2_hetero2d())
    d.n[0] = 0
    assert _ws([d])[0] == 1


def test_create_rejects_small_workspace_and_nonfinite_logk():
    from paper_1801_04984_amd import native
    L = lib()
    wl = W.Workload("t", 2, (4, 4), 1, 0.1, 1)
    d = (native.Desc * 1)(native.make_desc(wl))
    th = np.zeros(16)
    th[3] = np.inf
    arr = (ctypes.POINTER(ctypes.c_double) * 1)(th.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    h = ctypes.c_void_p()
    buf = ctypes.create_string_buffer(64)
    st = L.create_slab_problem(d, 1, arr, ctypes.cast(buf, ctypes.c_void_p), 64, None, ctypes.byref(h))
    assert st == 1 and "not finite" in L.biot_last_error().decode()
    th[3] = 0.0
    st = L.create_slab_problem(d, 1, arr, ctypes.cast(buf, ctypes.c_void_p), 64, None, ctypes.byref(h))
    assert st == 2 and "workspace too small" in L.biot_last_error().decode()
    st = L.create_slab_problem(d, 1, arr, None, 1 << 30, None, ctypes.byref(h))
    assert st == 2
    assert not h.value
    assert L.apply_operator(None, None, None, 0, 0, None) == 1
    assert L.destroy_slab_problem(None) == 1


def test_instance_size_limit():
    """One instance's slab must stay below 2^31 unknowns (32-bit kernel indexing)."""
    from paper_1801_04984_amd import native
    d = native.make_desc(W.c4_adjoint3d())
    for e in range(3):
        d.n[e] = 1024
    st, _, err = _ws([d])
    assert st == 1 and "2^31" in err
    d = native.make_desc(W.c4_adjoint3d())
    st, nb, _ = _ws([d])
    assert st == 0 and nb > 0


def test_tuning_calls_reject_null():
    from paper_1801_04984_amd import native
    L = lib()
    t = native.Tuning()
    assert L.biot_get_tuning(None, ctypes.byref(t)) == 1
    assert L.biot_set_tuning(None, ctypes.byref(t)) == 1
    assert L.biot_autotune(None, 5, ctypes.byref(t), None) == 1


def _header_signatures():
    src = open(os.path.join(ROOT, "include", "biotst.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    out = {}
    for m in re.finditer(r"^\s*(biot_status|const char\*)\s+(\w+)\s*\(([^)]*)\)\s*;", src, flags=re.M):
        params = [" ".join(p.split()) for p in m.group(3).split(",")]
        out[m.group(2)] = (m.group(1), [] if params == ["void"] else params)
    return out


def test_binding_argtypes_match_header_signatures():
    """Every function of the binding declares the header's arity, and each
    argument's ctypes kind matches the C type: scalars by width, struct
    pointers to the struct's mirror, other pointers as pointers."""
    from paper_1801_04984_amd import native
    L = lib()
    structs = {"biot_problem_desc": native.Desc, "biot_solve_opts": native.SolveOpts,
               "biot_solve_info": native.SolveInfo, "biot_tuning": native.Tuning}
    scalars = {"int32_t": ctypes.c_int32, "double": ctypes.c_double, "size_t": ctypes.c_size_t}
    sigs = _header_signatures()
    assert sorted(sigs) == sorted(native.EXPORTS)
    for name, (ret, params) in sigs.items():
        fn = getattr(L, name)
        assert fn.restype is (ctypes.c_char_p if ret == "const char*" else ctypes.c_int32), name
        if not params:
            continue
        assert fn.argtypes is not None and len(fn.argtypes) == len(params), name
        for p, t in zip(params, fn.argtypes):
            ctype = p.rsplit(" ", 1)[0].replace("const ", "").strip()
            where = f"{name}: {p}"
            if ctype == "biot_problem" or "*" in ctype:
                assert t is ctypes.c_void_p or issubclass(t, ctypes._Pointer), where
                base = ctype.rstrip("* ").strip()
                if base in structs:
                    assert t._type_ is structs[base], where
                elif base in ("int64_t", "size_t") and issubclass(t, ctypes._Pointer):
                    assert t._type_ is {"int64_t": ctypes.c_int64, "size_t": ctypes.c_size_t}[base], where
                elif base == "double" and ctype.count("*") == 1 and issubclass(t, ctypes._Pointer):
                    assert t._type_ is ctypes.c_double, where
            else:
                assert t is scalars[ctype], where


def test_product_path_fails_loudly_without_the_library(monkeypatch):
    """With the shared library absent the binding raises before any device
    work; there is no fallback path."""
    from paper_1801_04984_amd import native
    monkeypatch.setattr(native, "_lib", None)
    monkeypatch.setattr(native.load_library, "__defaults__", (os.path.join(ROOT, "no_such_dir", "libbiotst.so"),))
    wl = W.Workload("t", 2, (4, 4), 1, 0.1, 1)
    with pytest.raises(OSError, match="missing"):
        native.BiotSlab([wl], [np.zeros(16)])


def test_product_package_never_imports_the_oracle():
    """The package and the benchmark's GPU legs do not reach the oracle: only
    tests, the smoke check and the benchmark's CPU baseline may."""
    pkg = os.path.join(ROOT, "paper_1801_04984_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle\b", src, flags=re.M), f
    bench = open(os.path.join(ROOT, "bench.py")).read()
    uses = [m.start() for m in re.finditer(r"from oracle import|import oracle", bench)]
    assert uses, "the CPU baseline leg times the oracle"
    for u in uses:
        fn = bench.rfind("\ndef ", 0, u)
        assert bench[fn:].startswith("\ndef cpu_baseline("), bench[fn:fn + 40]


def test_oracle_and_generators_never_reach_the_hip_package():
    """The oracle and the shared input generators import nothing of the HIP
    package and load no part of its library."""
    for sub in ("oracle", "workloads"):
        for dirpath, _, files in os.walk(os.path.join(ROOT, sub)):
            for f in files:
                if f.endswith(".py"):
                    src = open(os.path.join(dirpath, f)).read()
                    for word in ("paper_1801_04984_amd", "libbiotst", "csrc", "ctypes"):
                        assert word not in src, (f, word)
