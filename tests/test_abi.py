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


def test_fluid_list_kernel_workspace():
    """Kernel 3 adds, to the dense layout, one uint32 index per fluid node per
    sample and one 24-byte descriptor per sample (256-byte aligned pieces)."""
    def align(v):
        return (v + 255) // 256 * 256
    a = inputs.random_state(40, 6, 5, seed=77, solid_frac=0.8)[0]
    b = inputs.random_state(64, 3, 2, seed=78, solid_frac=0.3)[0]
    dense = tau1.workspace_size([(a,), (b,)], kernel=0)
    listed = tau1.workspace_size([(a,), (b,)], kernel=3)
    extra = align(24 * 2) + align(4 * int((a == 0).sum())) + align(4 * int((b == 0).sum()))
    assert listed == dense + extra
    # an all-solid sample still gets one (unused) slot
    s = np.ones((2, 2, 2), np.uint8)
    assert tau1.workspace_size([(s,)], kernel=3) == \
        tau1.workspace_size([(s,)], kernel=0) + align(24) + align(4)


@pytest.mark.parametrize("kw,status", [
    (dict(kernel=3, layout=1), tau1.TAU1_E_UNSUPPORTED),   # dense layout only
    (dict(kernel=3, lattice=9), tau1.TAU1_E_UNSUPPORTED),  # 3-D lattices only
    (dict(kernel=2), tau1.TAU1_E_INVALID),                 # 2 is the D2Q9 kernel's own
    (dict(kernel=4), tau1.TAU1_E_INVALID),
])
def test_fluid_list_kernel_requests(lib, kw, status):
    solid = np.zeros((1, 4, 8), np.uint8)
    d, keep = tau1._desc([tau1.Sample(solid)], kw.get("lattice", 19), "f32", (0, 0, 0), 0,
                         kw["kernel"], -1, (0, 0), None, kw.get("layout", -1))
    n = ctypes.c_size_t(0)
    assert lib.tau1_workspace_size(ctypes.byref(d), ctypes.byref(n)) == status


def test_fluid_list_kernel_rejects_more_than_2_32_nodes(lib):
    """Node indices of the lists are 32-bit (checked before the mask is read;
    a small array stands in for the large one)."""
    d, keep = tau1._desc([tau1.Sample(np.zeros((2, 2, 2), np.uint8))], 19, "f32", (0, 0, 0), 0,
                         3, -1, (0, 0), None, -1)
    keep[0].nz, keep[0].ny, keep[0].nx = 3, 1 << 11, 1 << 20
    n = ctypes.c_size_t(0)
    assert lib.tau1_workspace_size(ctypes.byref(d), ctypes.byref(n)) == tau1.TAU1_E_UNSUPPORTED
