"""Host side of the packed state layout (no GPU): the workspace it plans
holds exactly the lane chunks that contain a fluid node, counted here with
numpy, and the requests it cannot serve are refused."""
import ctypes

import numpy as np
import pytest

from paper_2312_14742_amd import inputs, tau1

# one-row-per-wave lane layouts: nx -> (chunk length K, groups of 64 chunks per row)
G1 = {64: (1, 1), 128: (2, 1), 192: (3, 1), 256: (4, 1), 320: (5, 1), 384: (3, 2), 512: (4, 2),
      96: (2, 1), 160: (4, 1), 224: (4, 1), 288: (6, 1)}


@pytest.fixture(scope="module")
def lib():
    return tau1._lib()


def align(v, a=256):
    return (v + a - 1) // a * a


def fluid_chunks(solid, k):
    nz, ny, nx = solid.shape
    return int(np.any(solid.reshape(nz, ny, nx // k, k) == 0, axis=-1).sum())


def zmarch_items(solids):
    """Longest z-march work list: rows padded to blocks of four, 16-plane segments."""
    return sum((s.shape[1] + 3) // 4 * 4 * ((s.shape[0] + 15) // 16) for s in solids)


def packed_extra(solids, packed, tile=-1):
    """Workspace the packed layout adds besides its smaller state buffers: per
    packed sample the chunk table (16 B per row and group); where the chunk
    tile is asked for or at most half of the sample's chunks are stored, the
    chunk list (4 B per stored chunk) and nine neighbour-row records (8 B
    each per stored chunk); and a work list long enough for the chunk tile
    (one 16-B item per 64 stored chunks of each such sample)."""
    extra = 0
    waves = 0
    for s in packed:
        nz, ny, nx = s.shape
        k, groups = G1[nx]
        nch = fluid_chunks(s, k)
        extra += align(16 * ny * nz * groups)
        if tile == 16 or 2 * nch <= ny * nz * (nx // k):
            extra += align(4 * max(nch, 1)) + align(72 * max(nch, 1))
            waves += (nch + 63) // 64
    items = zmarch_items(solids)
    return extra + align(16 * max(items, waves, 1)) - align(16 * max(items, 1))


@pytest.mark.parametrize("prec,es", [("f32", 4), ("f16", 2), ("bf16", 2)])
@pytest.mark.parametrize("nx", sorted(G1))
def test_packed_workspace_holds_fluid_chunks(lib, nx, prec, es):
    ny, nz = 3, 5
    solid = inputs.random_state(nx, ny, nz, seed=9000 + nx, solid_frac=0.7)[0]
    k, groups = G1[nx]
    dense = tau1.workspace_size([(solid,)], precision=prec, kernel=1, layout=0)
    packed = tau1.workspace_size([(solid,)], precision=prec, kernel=1, layout=1)
    n = nx * ny * nz
    ds = align(n * es) // es
    ps = align(max(fluid_chunks(solid, k) * k, 1) * es) // es
    # two buffers of four arrays each, plus the chunk table and list
    expect = dense - 2 * (align(4 * ds * es) - align(4 * ps * es)) + packed_extra([solid], [solid])
    assert packed == expect


def test_packed_is_default_for_zmarch_precisions(lib):
    solid = inputs.random_state(256, 3, 5, seed=9100, solid_frac=0.7)[0]
    for prec in ("f32", "f16", "bf16"):
        auto = tau1.workspace_size([(solid,)], precision=prec)
        dense = tau1.workspace_size([(solid,)], precision=prec, layout=0)
        packed = tau1.workspace_size([(solid,)], precision=prec, layout=1)
        assert packed < dense
        assert auto == packed
    # FP64 runs the per-node gather on the dense layout
    assert tau1.workspace_size([(solid,)], precision="f64") == \
        tau1.workspace_size([(solid,)], precision="f64", layout=0)
    # the chunk tile belongs to the packed layout; asked for, it also brings
    # the chunk list and records of a sample that keeps most of its chunks
    packed = tau1.workspace_size([(solid,)], layout=1)
    assert tau1.workspace_size([(solid,)], tile=16) == \
        packed + packed_extra([solid], [solid], tile=16) - packed_extra([solid], [solid])
    # a dense-layout tile keeps the automatic layout dense
    assert tau1.workspace_size([(solid,)], tile=6) == tau1.workspace_size([(solid,)], layout=0)
    assert tau1.workspace_size([(solid,)], tile=14) == tau1.workspace_size([(solid,)], layout=1)


def test_all_solid_and_all_fluid_samples(lib):
    ny, nz = 2, 3
    solid = np.ones((nz, ny, 512), np.uint8)
    fluid = np.zeros((nz, ny, 512), np.uint8)
    d_solid = tau1.workspace_size([(solid,)], layout=0)
    p_solid = tau1.workspace_size([(solid,)], layout=1)
    d_fluid = tau1.workspace_size([(fluid,)], layout=0)
    p_fluid = tau1.workspace_size([(fluid,)], layout=1)
    assert p_fluid == d_fluid + packed_extra([fluid], [fluid])
    assert p_solid == (d_solid - 2 * (align(4 * 512 * ny * nz * 4) - align(4 * 64 * 4)) +
                       packed_extra([solid], [solid]))


@pytest.mark.parametrize("kw", [
    dict(precision="f64"),                 # the FP64 path is the per-node gather
    dict(kernel=0),                        # the gather kernel reads the dense layout
    dict(nx=32),                           # two rows per wave: no packed kernel
    dict(nx=100),                          # no z-march lane layout at all
])
def test_packed_refused(lib, kw):
    nx = kw.pop("nx", 64)
    solid = np.zeros((4, 4, nx), np.uint8)
    d, keep = tau1._desc([tau1.Sample(solid)], 19, kw.get("precision", "f32"), (0, 0, 0), 0,
                         kw.get("kernel", -1), -1, (0, 0), None, 1)
    n = ctypes.c_size_t(0)
    assert lib.tau1_workspace_size(ctypes.byref(d), ctypes.byref(n)) == tau1.TAU1_E_UNSUPPORTED
    ctx = ctypes.c_void_p(None)
    d.workspace = 256
    d.workspace_bytes = 1 << 40
    assert lib.tau1_create(ctypes.byref(d), ctypes.byref(ctx)) == tau1.TAU1_E_UNSUPPORTED
    assert not ctx.value


@pytest.mark.parametrize("layout", [-2, 2])
def test_bad_layout_rejected(lib, layout):
    solid = np.zeros((4, 4, 64), np.uint8)
    d, keep = tau1._desc([tau1.Sample(solid)], 19, "f32", (0, 0, 0), 0, -1, -1, (0, 0), None,
                         layout)
    n = ctypes.c_size_t(0)
    assert lib.tau1_workspace_size(ctypes.byref(d), ctypes.byref(n)) == tau1.TAU1_E_INVALID


def test_oversized_layout_stays_dense(lib):
    """A lane layout is packed only if every sample of it fits 32-bit offsets
    over its four packed arrays; the other layouts of the context still pack."""
    big = np.zeros((520, 512, 512), np.uint8)       # 4 * 136M * 4 B > 2 GiB
    small = inputs.random_state(512, 3, 5, seed=9200, solid_frac=0.7)[0]
    other = inputs.random_state(256, 6, 5, seed=9201, solid_frac=0.7)[0]
    with pytest.raises(tau1.Tau1Error):
        tau1.workspace_size([(big,), (small,)], layout=1)
    dense = tau1.workspace_size([(big,), (small,), (other,)], layout=0)
    packed = tau1.workspace_size([(big,), (small,), (other,)], layout=1)
    k, groups = G1[256]
    ds = align(other.size * 4) // 4
    ps = align(fluid_chunks(other, k) * k * 4) // 4
    assert packed == (dense - 2 * (align(4 * ds * 4) - align(4 * ps * 4)) +
                      packed_extra([big, small, other], [other]))
