"""Host-side checks of the D2Q9 validation lattice's descriptor (no GPU)."""
import ctypes

import numpy as np
import pytest

from paper_2312_14742_amd import tau1


@pytest.fixture(scope="module")
def lib():
    return tau1._lib()


def status(lib, solid, **kw):
    d, keep = tau1._desc([tau1.Sample(solid)], kw.pop("lattice", 9), kw.pop("precision", "f64"),
                         kw.pop("g", (0.0, 0.0, 0.0)), 0, kw.pop("kernel", -1), -1, (0, 0), None,
                         -1, kw.pop("x_boundary", 0), kw.pop("rho_in", 1.0),
                         kw.pop("rho_out", 1.0), kw.pop("wall_u", (0.0, 0.0, 0.0)))
    assert not kw
    n = ctypes.c_size_t(0)
    return lib.tau1_workspace_size(ctypes.byref(d), ctypes.byref(n)), n.value


def test_d2q9_workspace(lib):
    t = np.zeros((1, 12, 40), np.uint8)
    st, n = status(lib, t, x_boundary=1, rho_in=1.01, rho_out=0.99)
    assert st == tau1.TAU1_OK
    # two buffers of four FP64 arrays plus the node types
    assert n >= 2 * 4 * 8 * t.size + t.size


@pytest.mark.parametrize("kw,want", [
    (dict(solid=np.zeros((2, 4, 8), np.uint8)), "INVALID"),             # nz must be 1
    (dict(g=(0.0, 0.0, 1e-5)), "INVALID"),                               # no z axis
    (dict(x_boundary=2), "INVALID"),
    (dict(x_boundary=1, rho_in=0.0), "INVALID"),
    (dict(x_boundary=1, rho_out=float("nan")), "INVALID"),
    (dict(solid=np.zeros((1, 4, 2), np.uint8), x_boundary=1), "INVALID"),  # nx >= 3
    (dict(wall_u=(float("inf"), 0.0, 0.0)), "INVALID"),
    (dict(precision="f16"), "UNSUPPORTED"),
    (dict(kernel=1), "UNSUPPORTED"),
    (dict(lattice=19, x_boundary=1), "UNSUPPORTED"),                     # 3-D: periodic only
    (dict(lattice=19, wall_u=(0.1, 0.0, 0.0)), "UNSUPPORTED"),
])
def test_d2q9_descriptor_checks(lib, kw, want):
    solid = kw.pop("solid", np.zeros((1, 4, 8), np.uint8))
    st, _ = status(lib, solid, **kw)
    assert st == getattr(tau1, f"TAU1_E_{want}")
