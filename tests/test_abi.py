"""The C-ABI library loads and exports every symbol include/gmcp.h declares;
host-only entry points (workspace sizing, error strings) behave.  No GPU
compute here."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header="gmcp.h"):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gmcp_[a-z_0-9]+)\s*\(", src)))


def test_mlp_header_symbols_exported_and_param_count():
    from oracle import mlp as omlp
    from paper_2605_24339_amd import _native
    lib = _native.lib()
    names = _declared("gmcp_mlp.h")
    assert set(names) == set(_native.MLP_EXPORTS)
    assert not [n for n in names if not hasattr(lib, n)]
    lib.gmcp_mlp_param_count.restype = C.c_int64
    assert lib.gmcp_mlp_param_count() == omlp.N_PARAMS


def test_fem_header_symbols_exported():
    from paper_2605_24339_amd import _native
    lib = _native.lib()
    names = _declared("gmcp_fem.h")
    assert set(names) == set(_native.FEM_EXPORTS)
    assert not [n for n in names if not hasattr(lib, n)]


def test_header_declares_the_path_entry_points():
    names = _declared()
    for n in ("gmcp_build_samples", "gmcp_broadphase", "gmcp_assemble", "gmcp_ccd_step", "gmcp_hvp"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2605_24339_amd import _native
    lib = _native.lib()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(_native.EXPORTS) == set(_declared())


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_library_rule_exactness(n):
    """The library's own Gauss construction (independent of the oracle's):
    positive weights summing to 1/2 and exact monomials to degree 2n-1."""
    import math

    import numpy as np
    from paper_2605_24339_amd import _native as N
    out = (C.c_double * (3 * n * n))()
    assert N.lib().gmcp_rule(n, out) == 0
    r = np.array(out[:]).reshape(n * n, 3)
    xi, eta, w = r.T
    assert np.all(w > 0) and abs(w.sum() - 0.5) < 1e-14
    for a in range(2 * n):
        for b in range(2 * n - a):
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            assert abs(np.sum(w * xi ** a * eta ** b) - exact) < 1e-14, (n, a, b)
    assert N.lib().gmcp_rule(5, out) == N.GMCP_E_ARG


def test_workspace_size_and_strerror_host_only():
    from paper_2605_24339_amd import _native as N
    L = N.lib()
    i32 = lambda *v: (C.c_int32 * len(v))(*v)
    f64 = lambda *v: (C.c_double * len(v))(*v)
    keep = [i32(0, 289), i32(0, 512), i32(0, 642), i32(0, 1280), i32(2), f64(1e5), f64(1e-3), f64(0.0)]
    cast = lambda a, t: C.cast(a, C.POINTER(t))
    lay = N.Layout(1, *(cast(k, C.c_int32) for k in keep[:5]), *(cast(k, C.c_double) for k in keep[5:]),
                   None, 0)
    caps = N.Caps(10000, 20000, 10000, 2048, 2048, 512)
    n = L.gmcp_workspace_size(C.byref(lay), C.byref(caps))
    assert n > 0
    lay64 = N.Layout(1, *(cast(k, C.c_int32) for k in keep[:5]), *(cast(k, C.c_double) for k in keep[5:]),
                     None, N.GMCP_F64)
    assert L.gmcp_workspace_size(C.byref(lay64), C.byref(caps)) > n
    bad = i32(5)  # rule order out of range
    lay_bad = N.Layout(1, *(cast(k, C.c_int32) for k in keep[:4]), cast(bad, C.c_int32),
                       *(cast(k, C.c_double) for k in keep[5:]), None, 0)
    assert L.gmcp_workspace_size(C.byref(lay_bad), C.byref(caps)) == 0
    # edge / point samples need the clipped mortar samples
    lay_feat = N.Layout(1, *(cast(k, C.c_int32) for k in keep[:5]), *(cast(k, C.c_double) for k in keep[5:]),
                        None, N.GMCP_FEATURES)
    assert L.gmcp_workspace_size(C.byref(lay_feat), C.byref(caps)) == 0
    lay_feat.flags = N.GMCP_FEATURES | N.GMCP_MORTAR
    assert L.gmcp_workspace_size(C.byref(lay_feat), C.byref(caps)) > 0
    assert N.strerror(N.GMCP_E_PENETRATION).startswith("penetration")
    ctx = C.c_void_p()
    assert L.gmcp_create(C.byref(ctx), C.byref(lay_bad), C.byref(caps), None, None, None, 0, None) == N.GMCP_E_ARG


def test_dualmesh_header_symbols_exported():
    from paper_2605_24339_amd import _native
    lib = _native.lib()
    names = _declared("gmcp_dualmesh.h")
    assert set(names) == set(_native.DUALMESH_EXPORTS)
    assert not [n for n in names if not hasattr(lib, n)]


def test_dualmesh_argument_errors_host_only():
    """Argument checks return before any launch (no device needed)."""
    import ctypes as C
    from paper_2605_24339_amd import _native as N
    from paper_2605_24339_amd.dualmesh import _lib
    L = _lib()
    assert L.gmcp_dualmesh_embed(None, -1, None, None, 0, None, None, None, None, None) == N.GMCP_E_ARG
    assert L.gmcp_dualmesh_embed(None, 0, None, None, 0, None, None, None, None, None) == N.GMCP_OK
    assert L.gmcp_dualmesh_embed(C.c_void_p(8), 5, C.c_void_p(8), None, 0, None, None, None, None, None) == N.GMCP_E_ARG
    assert L.gmcp_dualmesh_update(None, None, None, None, None, -3, None, 0, None) == N.GMCP_E_ARG
    assert L.gmcp_dualmesh_update(None, None, None, None, None, 0, None, 0, None) == N.GMCP_OK
