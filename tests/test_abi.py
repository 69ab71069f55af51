"""The C-ABI library loads and exports every entry point declared in
include/hsp.h; host-side argument validation works without a GPU."""
import ctypes
import os
import re

import pytest

from paper_1412_0464_amd import hsp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "hsp.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hsp_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = hsp.load()
    names = _declared()
    assert "hsp_setup" in names and "hsp_solve" in names and "hsp_apply_precond" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(hsp.EXPORTS)


def test_default_options():
    o = hsp.make_options()
    assert (o.fine_stencil, o.two_grid, o.w_dd, o.nu, o.sweep, o.precision) == (5, 0, 4, 3, 0, 0)
    assert abs(o.omega_jac - 0.8) < 1e-15


def _ws(n=(127, 127), h=1 / 128, pml=(10, 10), J=4, **kw):
    return hsp.workspace_size(n, h, pml, J, **kw)


def test_workspace_size_valid_configs():
    assert _ws() > 0
    assert _ws(two_grid=True, n=(255, 255), pml=(16, 16), J=8) > 0
    assert _ws(precision="mixed") < _ws(precision="fp64")


@pytest.mark.parametrize("kw,msg", [
    (dict(J=0), "J"),
    (dict(J=60), "thinner than 3"),                     # cores thinner than 3 layers
    (dict(J=1), "slab thicker"),                        # 147 layers in one slab
    (dict(w_dd=0), "w_dd"),
    (dict(two_grid=True, n=(126, 127)), "even"),        # odd interior cell count
    (dict(fine_stencil=7), "fine_stencil"),
    (dict(h=-1.0), "h must"),
    (dict(nu=-1), "nu"),
    (dict(restart=0), "restart"),
    (dict(krylov_fp32=True), "krylov_fp32"),            # complex64 basis without mixed precision
])
def test_workspace_size_rejects_invalid(kw, msg):
    with pytest.raises(hsp.HspError) as e:
        _ws(**kw)
    assert e.value.status == hsp.HSP_EINVAL
    assert msg in str(e.value)


def test_null_arguments_rejected_without_device():
    lib = hsp.load()
    assert lib.hsp_workspace_size(None, 4, None, None) == hsp.HSP_EINVAL
    assert lib.hsp_apply_precond(None, None, None, None) == hsp.HSP_EINVAL
    assert lib.hsp_solve(None, None, None, 1e-6, 10, 0, None, None, None) == hsp.HSP_EINVAL
    out = ctypes.c_void_p()
    g = hsp.make_grid((31, 31), 0.1, (4, 4))
    o = hsp.make_options()
    assert lib.hsp_setup(None, 1.0, ctypes.byref(g), 2, ctypes.byref(o), None, 0, None,
                         ctypes.byref(out)) == hsp.HSP_EINVAL
    assert b"null" in lib.hsp_last_error()


def _ws3(n=(17, 8, 9), h=0.05, pml=(3, 3, 3), J=3, **kw):
    kw.setdefault("fine_stencil", 7)
    kw.setdefault("precision", "mixed")
    return hsp.workspace_size(n, h, pml, J, **kw)


def test_workspace_size_3d():
    assert _ws3() > 0
    assert _ws3(two_grid=True, n=(25, 9, 11), pml=(4, 4, 4)) > 0
    assert _ws3(fine_stencil=27) > _ws3()


def test_nested_dissection_plans_and_sizes():
    """The host plan of the nested dissection (its parent/child maps are
    checked while it is built) for planes from 1 x 1 to 63 x 63 nodes; a
    thin slab of a wide plane fits only the nested dissection; at the 3-D
    benchmark size (127^3 + 8 PML, J = 16 coarse slabs) its workspace is
    smaller than the block-tridiagonal one (fewer factor bytes)."""
    for m in [(1, 1, 1), (5, 1, 7), (9, 2, 3), (12, 13, 11), (30, 31, 17), (16, 61, 61)]:
        assert _ws3(n=m, pml=(1, 1, 1), J=1, w_dd=1, slab_factor="nd") > 0
    assert _ws3(n=(40, 8, 300), J=1, slab_factor="nd") > 0
    big = dict(n=(127, 127, 127), h=0.02, pml=(8, 8, 8), J=16, two_grid=True, w_dd=3)
    assert _ws3(slab_factor="nd", **big) < 0.7 * _ws3(slab_factor="block", **big)
    assert _ws3(slab_factor="auto", **big) == _ws3(slab_factor="nd", **big)


@pytest.mark.parametrize("kw,msg", [
    (dict(precision="fp64"), "HSP_MIXED"),                 # 3-D factors are complex64
    (dict(fine_stencil=5), "7 or 27"),
    (dict(two_grid=True, n=(17, 8, 9)), "even"),
    (dict(J=9), "thinner than 3"),
    (dict(n=(40, 8, 300), J=1, slab_factor="block"), "exceed"),  # slab planes beyond the panel kernel
    (dict(n=(40, 300, 300), J=1, slab_factor="nd"), "exceed"),   # fronts beyond the panel kernel
    (dict(krylov_fp32=True), "krylov_fp32"),
    (dict(slab_factor=3), "slab_factor"),
])
def test_workspace_size_3d_rejects_invalid(kw, msg):
    with pytest.raises(hsp.HspError) as e:
        _ws3(**kw)
    assert e.value.status == hsp.HSP_EINVAL
    assert msg in str(e.value)


def test_autotune_workspace_sizes_without_device():
    """The autotuner's workspace sizes are host logic: the largest setup and
    batch workspaces over its candidate chunk lengths (restart 1 keeps the
    batch workspace to the tuning itself); 3-D problems are refused."""
    lib = hsp.load()
    g = hsp.make_grid((255, 255), 0.04, (16, 16))
    o = hsp.make_options(two_grid=True, precision="mixed")
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.hsp_autotune_workspace_size(ctypes.byref(g), 8, ctypes.byref(o), 64, 1, ctypes.byref(a),
                                           ctypes.byref(b)) == hsp.HSP_OK
    ws = ctypes.c_size_t()
    for chunk in (16, 64):
        oc = hsp.make_options(two_grid=True, precision="mixed", chunk=chunk)
        assert lib.hsp_workspace_size(ctypes.byref(g), 8, ctypes.byref(oc), ctypes.byref(ws)) == hsp.HSP_OK
        assert ws.value <= a.value
    assert b.value > 0
    g3 = hsp.make_grid((17, 8, 9), 0.05, (3, 3, 3))
    o3 = hsp.make_options(fine_stencil=7, precision="mixed")
    assert lib.hsp_autotune_workspace_size(ctypes.byref(g3), 3, ctypes.byref(o3), 4, 1, ctypes.byref(a),
                                           ctypes.byref(b)) == hsp.HSP_EINVAL
