"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/gs.h declares, and host-only helpers behave."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names += re.findall(r"GS_API\s+[\w\s\*]+?\b(gs_\w+)\s*\(", txt)
    return sorted(set(names))


@pytest.fixture(scope="module")
def native():
    from paper_2405_20693_amd import _native
    if not os.path.exists(_native.LIB_PATH):
        from paper_2405_20693_amd import build
        build.build()
    return _native


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("gs_project_fwd", "gs_project_bwd", "gs_voxelize_fwd", "gs_voxelize_bwd",
              "gs_plan_create", "gs_plan_destroy", "gs_view_cone", "gs_loss_image", "gs_loss_tv"):
        assert n in names


def test_library_exports_every_declared_symbol(native):
    lib = native.lib()
    raw = ctypes.CDLL(native.LIB_PATH)
    for n in _declared():
        assert hasattr(raw, n), n
        assert n in native.EXPORTS, n
    assert set(native.EXPORTS) == set(_declared())
    assert lib.gs_last_error() == b""


def test_view_cone_matches_scanner_rotation(native):
    """Host helper: App. A rotation, computed in double and rounded to float,
    equals the oracle's (independently written) rounding of the same matrix."""
    v = native.GsView()
    for th in (0.0, 0.37, 2.1, 5.9):
        native.call("gs_view_cone", th, 13.64, 20.46, 64, 32, 0.05, ctypes.byref(v))
        ov = oracle.cone_view(th, 13.64, 20.46, 64, 32, 0.05)
        np.testing.assert_array_equal(np.array(v.rot[:], np.float64).reshape(3, 3), ov["W"])
        assert v.beam == native.GS_CONE and v.width == 64 and v.height == 32
        assert v.src_obj == np.float32(13.64) and v.src_det == np.float32(20.46)


def test_view_cone_rejects_bad_geometry(native):
    v = native.GsView()
    with pytest.raises(native.GsError, match="GS_EINVAL"):
        native.call("gs_view_cone", 0.0, 20.0, 10.0, 64, 64, 0.05, ctypes.byref(v))
    with pytest.raises(native.GsError, match="GS_EINVAL"):
        native.call("gs_view_cone", 0.0, 10.0, 20.0, 0, 64, 0.05, ctypes.byref(v))
    with pytest.raises(native.GsError, match="GS_EINVAL"):
        native.call("gs_view_cone", math.nan, 10.0, 20.0, 8, 8, 0.05, ctypes.byref(v))
    assert b"theta" in native.lib().gs_last_error()


def test_argument_errors_are_caught_before_any_launch(native):
    """Null pointers and bad sizes return GS_EINVAL from host checks only."""
    lib = native.lib()
    g = native.GsGaussians()
    g.n = 5  # non-zero count with NULL arrays
    v = native.GsView()
    native.call("gs_view_cone", 0.0, 10.0, 20.0, 8, 8, 0.05, ctypes.byref(v))
    st = lib.gs_project_fwd(ctypes.byref(g), ctypes.byref(v), 1, 3.0, None, None, None)
    assert st == 1 and b"NULL" in lib.gs_last_error()
    grid = native.GsGrid()
    grid.nx = 0
    g.n = 0
    st = lib.gs_voxelize_fwd(ctypes.byref(g), ctypes.byref(grid), 3.0, ctypes.c_void_p(8), None, None)
    assert st == 1
    st = lib.gs_loss_tv(None, 4, 4, 4, 1.0, None, None, 0, None, None)
    assert st == 1
    st = lib.gs_plan_create(ctypes.c_void_p(1), None, None, ctypes.byref(ctypes.c_void_p()))
    assert st == 1  # alloc without free
    # the image loss: sizes, and images of 2^29 pixels or more (the loss
    # kernel addresses one image with 32-bit byte offsets)
    d = ctypes.c_void_p(8)
    st = lib.gs_loss_image(d, d, 1, 0, 16, ctypes.c_float(0.25), d, None, None, None)
    assert st == 1  # GS_EINVAL
    st = lib.gs_loss_image(d, d, 1, 1 << 15, 1 << 14, ctypes.c_float(0.25), d, None, None, None)
    assert st == 5 and b"2^29" in lib.gs_last_error()
    st = lib.gs_loss_image_noalloc(d, d, 1, 1 << 15, 1 << 14, ctypes.c_float(0.25), d, None, None)
    assert st == 5
    # the kernels' size limits, refused before any plan or device memory
    g.mean = g.scale = g.quat = g.density = d
    g.n = 1 << 28  # entries carry the Gaussian index in 28 bits
    st = lib.gs_project_fwd(ctypes.byref(g), ctypes.byref(v), 1, 3.0, d, None, None)
    assert st == 5 and b"2^28" in lib.gs_last_error()
    g.n = 10
    wide = native.GsView()
    native.call("gs_view_cone", 0.0, 10.0, 20.0, 4096, 1040, 0.05, ctypes.byref(wide))
    st = lib.gs_project_fwd(ctypes.byref(g), ctypes.byref(wide), 1, 3.0, d, None, None)
    assert st == 5 and b"16384 tiles" in lib.gs_last_error()
    big = native.GsGrid()
    big.nx, big.ny, big.nz = 1040, 1040, 8
    for k in range(3):
        big.spacing[k] = 0.01
    st = lib.gs_voxelize_fwd(ctypes.byref(g), ctypes.byref(big), 3.0, d, None, None)
    assert st == 5 and b"16384 tiles" in lib.gs_last_error()


def test_product_path_does_not_use_the_oracle():
    """The HIP package imports nothing from oracle/ (and vice versa)."""
    pkg = os.path.join(ROOT, "paper_2405_20693_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith((".py", ".c")):
            txt = open(os.path.join(ROOT, "oracle", f)).read()
            assert "paper_2405_20693_amd" not in txt.replace("``paper_2405_20693_amd``", ""), f


def test_bindings_keep_temporary_plans_alive():
    """A temporary Plan must be bound to a name for the whole call: reading
    .handle off an unnamed `plan or Plan()` lets the Plan be collected (and
    its workspace freed) before the library uses it."""
    import ast
    pkg = os.path.join(ROOT, "paper_2405_20693_amd")
    for name in sorted(os.listdir(pkg)):
        if not name.endswith(".py"):
            continue
        tree = ast.parse(open(os.path.join(pkg, name)).read())
        for node in ast.walk(tree):
            if isinstance(node, ast.Attribute) and node.attr == "handle":
                inner = node.value
                assert not isinstance(inner, (ast.BoolOp, ast.Call)), f"{name}:{node.lineno}"


def test_reserve_bytes_counts_the_workspace(native):
    """gs_plan_reserve_bytes (host only): a tile-list entry costs 8 B of list
    and 24 B of backward slots; forward-only plans leave out the slots and
    chain partials; a record costs 32 B plus a 4-B slot offset."""
    def nbytes(**kw):
        r = native.GsReserve()
        for k, v in kw.items():
            setattr(r, k, v)
        out = ctypes.c_int64()
        native.call("gs_plan_reserve_bytes", ctypes.byref(r), ctypes.byref(out))
        return out.value
    base = dict(max_gaussians=100_000, max_views=8, width=512, height=512)
    e0 = nbytes(max_proj_entries=1 << 20, **base)
    e1 = nbytes(max_proj_entries=2 << 20, **base)
    assert e1 - e0 == (8 + 24) << 20
    f0 = nbytes(max_proj_entries=1 << 20, forward_only=1, **base)
    assert e0 - f0 >= (24 << 20) + 72 * 100_000
    r0 = nbytes(max_proj_entries=1 << 20, forward_only=1, max_records=400_000, **base)
    r1 = nbytes(max_proj_entries=1 << 20, forward_only=1, max_records=800_000, **base)
    assert r1 - r0 == 36 * 400_000
    with pytest.raises(native.GsError, match="GS_EINVAL"):
        nbytes(max_gaussians=1000, max_views=-1, width=8, height=8)
