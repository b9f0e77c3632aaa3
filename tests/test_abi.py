"""Host-side checks of the C ABI (no GPU work): the library loads, exports every
function include/tau1.h declares, and rejects bad descriptors before touching
the device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2312_14742_amd import tau1, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tau1.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(tau1_[a-z0-9_]+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(tau1.LIB_PATH):
        from paper_2312_14742_amd import build
        build.build()
    return tau1._lib()


def test_header_declares_expected_api():
    names = declared_functions()
    assert set(names) == set(tau1.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_strerror_covers_statuses(lib):
    for s in range(0, -7, -1):
        msg = lib.tau1_strerror(s).decode()
        assert msg and msg != "unknown status"
    assert lib.tau1_strerror(-99).decode() == "unknown status"


def _desc_for(samples, **kw):
    return tau1._desc([tau1.Sample(*s) for s in samples], kw.get("lattice", 19),
                      kw.get("precision", "f32"), kw.get("g", (1e-6, 0, 0)),
                      kw.get("graph_chunk", 0), kw.get("kernel", -1), kw.get("tile", -1),
                      kw.get("f16_scales", (0, 0)), None)


def test_workspace_size_host_only(lib):
    solid = inputs.channel(32, 32, 32)
    n32 = tau1.workspace_size([(solid,)], precision="f32")
    n64 = tau1.workspace_size([(solid,)], precision="f64")
    n16 = tau1.workspace_size([(solid,)], precision="f16")
    # state: two copies of four arrays per node
    N = 32 ** 3
    assert n32 >= 2 * 4 * 4 * N and n64 >= 2 * 4 * 8 * N and n16 >= 2 * 4 * 2 * N
    assert n64 > n32 > n16
    nb = tau1.workspace_size([(solid,), (solid,)], precision="f32")
    assert nb > n32


@pytest.mark.parametrize("bad", [
    dict(lattice=17), dict(precision=7), dict(graph_chunk=3), dict(graph_chunk=-2),
    dict(kernel=5), dict(g=(float("nan"), 0, 0)), dict(f16_scales=(-1, 0)),
])
def test_invalid_descriptor_rejected(lib, bad):
    solid = np.zeros((4, 4, 4), np.uint8)
    d, keep = _desc_for([(solid,)], **bad)
    n = ctypes.c_size_t(0)
    assert lib.tau1_workspace_size(ctypes.byref(d), ctypes.byref(n)) == tau1.TAU1_E_INVALID
    ctx = ctypes.c_void_p(None)
    assert lib.tau1_create(ctypes.byref(d), ctypes.byref(ctx)) == tau1.TAU1_E_INVALID
    assert not ctx.value


@pytest.mark.parametrize("shape,ok", [(-1, False), (0, True), (3, True), (4, False)])
def test_batch_graph_range(lib, shape, ok):
    """batch_graph takes 0-3 (3: one launch for the one-chunk rows)."""
    solid = np.zeros((4, 4, 64), np.uint8)
    d, keep = _desc_for([(solid,), (np.zeros((4, 4, 96), np.uint8),)])
    d.batch_graph = shape
    n = ctypes.c_size_t(0)
    st = lib.tau1_workspace_size(ctypes.byref(d), ctypes.byref(n))
    assert st == (tau1.TAU1_OK if ok else tau1.TAU1_E_INVALID)


def test_invalid_dims_rejected(lib):
    d, keep = _desc_for([(np.zeros((4, 4, 4), np.uint8),)])
    keep[0].nx = 0
    n = ctypes.c_size_t(0)
    assert lib.tau1_workspace_size(ctypes.byref(d), ctypes.byref(n)) == tau1.TAU1_E_INVALID


@pytest.mark.parametrize("dims", [
    (1, 1, (1 << 20) + 1),                 # nx above 2^20
    (1, (1 << 20) + 1, 1),                 # ny above 2^20
    ((1 << 20) + 1, 1, 1),                 # nz above 2^20
    (1, (1 << 11) + 1, 1 << 20),           # nx * ny above 2^31
    ((1 << 5) + 1, 1 << 15, 1 << 16),      # nx * ny * nz above 2^36
])
def test_dimension_limits_rejected(lib, dims):
    """Rejected by validation before the solid array is read (a 4^3 array
    stands in for the oversized one)."""
    d, keep = _desc_for([(np.zeros((4, 4, 4), np.uint8),)])
    keep[0].nz, keep[0].ny, keep[0].nx = dims
    n = ctypes.c_size_t(0)
    assert lib.tau1_workspace_size(ctypes.byref(d), ctypes.byref(n)) == tau1.TAU1_E_INVALID


def test_longest_row_accepted(lib):
    """A single row of 2^20 nodes is the largest extent accepted (served by
    the per-node gather kernel: no z-march lane layout has rows that long)."""
    solid = np.zeros((1, 1, 1 << 20), np.uint8)
    solid[0, 0, ::7] = 1
    n = tau1.workspace_size([(solid,)], precision="f32")
    assert n >= 2 * 4 * 4 * (1 << 20)


def test_nonfinite_initial_state_rejected(lib):
    solid = np.zeros((3, 3, 3), np.uint8)
    u = np.zeros((3, 3, 3, 3))
    u[1, 1, 1, 1] = np.nan
    d, keep = _desc_for([(solid, None, u)])
    d.workspace = 256
    d.workspace_bytes = 1 << 40
    ctx = ctypes.c_void_p(None)
    assert lib.tau1_create(ctypes.byref(d), ctypes.byref(ctx)) == tau1.TAU1_E_INVALID
    assert not ctx.value


def test_missing_or_small_workspace_rejected(lib):
    solid = np.zeros((3, 3, 3), np.uint8)
    d, keep = _desc_for([(solid,)])
    ctx = ctypes.c_void_p(None)
    d.workspace = None
    assert lib.tau1_create(ctypes.byref(d), ctypes.byref(ctx)) == tau1.TAU1_E_WORKSPACE
    d.workspace = 256 * 3 + 1                 # misaligned
    d.workspace_bytes = 1 << 30
    assert lib.tau1_create(ctypes.byref(d), ctypes.byref(ctx)) == tau1.TAU1_E_WORKSPACE
    d.workspace = 256
    d.workspace_bytes = 16                    # too small
    assert lib.tau1_create(ctypes.byref(d), ctypes.byref(ctx)) == tau1.TAU1_E_WORKSPACE
    assert not ctx.value


def test_null_context_calls(lib):
    assert lib.tau1_step(None, 1) == tau1.TAU1_E_INVALID
    assert lib.tau1_sync(None) == tau1.TAU1_E_INVALID
    lib.tau1_destroy(None)                    # NULL-safe


@pytest.mark.parametrize("kernel", [2, 3, 4])
def test_unknown_kernel_rejected(lib, kernel):
    """Kernels 0 (per-node gather) and 1 (z-march) exist on the 3-D lattices;
    2 is the D2Q9 kernel's own number and is not requested."""
    solid = np.zeros((1, 4, 8), np.uint8)
    d, keep = tau1._desc([tau1.Sample(solid)], 19, "f32", (0, 0, 0), 0, kernel, -1, (0, 0),
                         None, -1)
    n = ctypes.c_size_t(0)
    assert lib.tau1_workspace_size(ctypes.byref(d), ctypes.byref(n)) == tau1.TAU1_E_INVALID


def _create_status(lib, solid, drho=None, u=None, precision="f16", scales=(0, 0),
                   g=(1e-6, 0, 0)):
    d, keep = tau1._desc([tau1.Sample(solid, drho, u)], 19, precision, g, 0, -1, -1,
                         scales, None, -1)
    d.workspace = None                    # the field checks come before the workspace's
    ctx = ctypes.c_void_p(None)
    st = lib.tau1_create(ctypes.byref(d), ctypes.byref(ctx))
    assert not ctx.value
    return st


@pytest.mark.parametrize("scale,limit", [(0, 0.5 * 65504 * 2.0 ** -16),
                                         (20, 0.5 * 65504 * 2.0 ** -20),
                                         (12, 0.5 * 65504 * 2.0 ** -12)])
def test_f16_range_checked_at_create(lib, scale, limit):
    """FP16 storage keeps value * 2^s in half (largest finite 65504): an
    initial rho - 1 or u + g/2 at or above half of 65504 * 2^-s is refused
    before any GPU work, one just below passes the check (and only then
    meets the missing workspace); solid nodes and the other precisions are
    not checked."""
    solid = np.zeros((2, 2, 4), np.uint8)
    solid[0, 0, 0] = 1
    for field in ("drho", "ux", "uz"):
        for value, ok in ((0.999 * limit, True), (1.001 * limit, False), (-limit, False)):
            drho = np.zeros(solid.shape)
            u = np.zeros((3,) + solid.shape)
            if field == "drho":
                drho[1, 1, 2] = value
            else:
                u[0 if field == "ux" else 2, 1, 1, 2] = value - (1e-6 / 2 if field == "ux" else 0)
            st = _create_status(lib, solid, drho, u, scales=(scale, scale))
            assert st == (tau1.TAU1_E_WORKSPACE if ok else tau1.TAU1_E_INVALID), (field, value)
            if not (field == "drho" and value <= -1.0):      # rho <= 0 is invalid anyway
                assert _create_status(lib, solid, drho, u, precision="bf16") == \
                    tau1.TAU1_E_WORKSPACE
    # a solid node's value is not state
    drho = np.zeros(solid.shape)
    drho[0, 0, 0] = 10 * limit
    assert _create_status(lib, solid, drho, scales=(scale, scale)) == tau1.TAU1_E_WORKSPACE
    # the force shift alone can exceed the range
    assert _create_status(lib, solid, scales=(scale, scale),
                          g=(2.2 * limit, 0, 0)) == tau1.TAU1_E_INVALID
