"""The packed state layout (lane chunks without a fluid node are not stored)
against the dense layout and the oracle.

All tile shapes form every sum in the same order, and an all-solid chunk of
the packed layout loads as the zeros the dense layout stores, so a packed
context and a dense one give the same bits, step after step, in readback and
in the FP64 reductions."""
import numpy as np
import pytest

from paper_2312_14742_amd import inputs, tau1

from gpu_helpers import reduced_errors, run_oracle

pytestmark = pytest.mark.gpu

# every one-row-per-wave lane layout (nx = C * 64 * K, and the layouts with
# idle lanes: 96 = 48 x 2, 160 = 40 x 4, 224 = 56 x 4, 288 = 48 x 6)
G1_DIMS = [(64, 5, 7), (128, 3, 4), (192, 2, 3), (256, 3, 2), (320, 2, 2), (384, 2, 3),
           (512, 2, 3), (96, 5, 5), (160, 3, 3), (224, 3, 2), (288, 3, 2)]


def state(nx, ny, nz, seed, solid_frac=0.6):
    """Random fields on a mostly solid mask, so that many chunks are all solid."""
    return inputs.random_state(nx, ny, nz, seed=seed, solid_frac=solid_frac)


def run(samples, q, prec, g, nsteps, **kw):
    sim = tau1.Sim([tau1.Sample(*s) for s in samples], lattice=q, precision=prec, g=g,
                   kernel=1, **kw)
    sim.step(nsteps)
    return sim, [sim.moments(i) for i in range(len(samples))]


def assert_same(a, b, label):
    assert a[0].tobytes() == b[0].tobytes(), label
    assert a[1].tobytes() == b[1].tobytes(), label


@pytest.mark.parametrize("lz", [0, 3])
@pytest.mark.parametrize("dims", G1_DIMS)
@pytest.mark.parametrize("q", [15, 19, 27])
def test_packed_equals_dense_bitwise(q, dims, lz):
    nx, ny, nz = dims
    solid, drho, u = state(nx, ny, nz, seed=8100 + nx + 5 * ny + 11 * nz + q)
    g = (1e-5, -2e-5, 3e-6)
    print(f"[case] packed vs dense q={q} dims={dims} lz={lz}", flush=True)
    dense, od = run([(solid, drho, u)], q, "f32", g, 6, tile=4 + lz, layout=0)
    packed, op = run([(solid, drho, u)], q, "f32", g, 6, tile=12 + lz, layout=1)
    assert dense.info()["layout"] == 0 and packed.info()["layout"] == 1
    assert_same(op[0], od[0], (q, dims, lz))
    for axis in range(3):
        assert packed.permeability(0, axis) == dense.permeability(0, axis)
    dense.close()
    packed.close()


def test_packed_against_oracle_f32():
    solid, drho, u = state(512, 3, 5, seed=8200)
    g = (1e-5, 0.0, 2e-6)
    print("[case] packed 512x3x5 vs oracle", flush=True)
    sim, out = run([(solid, drho, u)], 19, "f32", g, 6)
    assert sim.info()["layout"] == 1  # automatic for FP32
    ref = run_oracle(19, solid, drho, u, g, 6)
    err = reduced_errors(out[0], ref, solid)
    print(f"[err] {err}", flush=True)
    eps = 2.0 ** -24
    assert err["drho_abs"] <= (2.0 * eps + 16.0 * eps) * np.abs(u).max()
    assert err["u_rel_l2"] <= 8.0 * eps
    sim.close()


@pytest.mark.parametrize("prec", ["f16", "bf16"])
@pytest.mark.parametrize("dims", [(256, 3, 5), (512, 2, 3)])
def test_packed_16bit_bitwise(prec, dims):
    nx, ny, nz = dims
    solid, drho, u = state(nx, ny, nz, seed=8300 + nx, solid_frac=0.5)
    g = (1e-5, -2e-5, 3e-6)
    print(f"[case] packed {prec} dims={dims}", flush=True)
    dense, od = run([(solid, drho, u)], 19, prec, g, 5, tile=5, f16_scales=(18, 18))
    packed, op = run([(solid, drho, u)], 19, prec, g, 5, tile=13, layout=1,
                     f16_scales=(18, 18))
    assert dense.info()["layout"] == 0 and packed.info()["layout"] == 1
    assert_same(op[0], od[0], (prec, dims))
    dense.close()
    packed.close()


@pytest.mark.parametrize("geometry", ["random", "all_fluid", "all_solid", "solid_planes"])
@pytest.mark.parametrize("dims", [(64, 1, 1), (64, 3, 2), (64, 5, 3), (128, 6, 2), (64, 9, 4)])
def test_packed_degenerate(dims, geometry):
    """ny or nz of 1-3, ny not a multiple of the four rows of a workgroup, and
    masks with no stored chunk, every chunk stored, or whole solid planes."""
    nx, ny, nz = dims
    solid, drho, u = state(nx, ny, nz, seed=8400 + nx * ny * nz, solid_frac=0.7)
    if geometry == "all_fluid":
        solid, drho, u = inputs.random_state(nx, ny, nz, seed=8401, solid_frac=0.0)
    elif geometry == "all_solid":
        solid = np.ones_like(solid)
        drho = np.zeros_like(drho)
        u = np.zeros_like(u)
    elif geometry == "solid_planes":
        solid[::2] = 1
        drho[solid == 1] = 0.0
        u[:, solid == 1] = 0.0
    g = (1e-5, 3e-6, -2e-6)
    print(f"[case] packed degenerate dims={dims} {geometry}", flush=True)
    dense, od = run([(solid, drho, u)], 19, "f32", g, 5, tile=6, layout=0)
    packed, op = run([(solid, drho, u)], 19, "f32", g, 5, tile=14, layout=1)
    assert_same(op[0], od[0], (dims, geometry))
    dense.close()
    packed.close()


def test_mixed_batch_packed_and_dense_samples():
    """One-row layouts (64, 128) are packed, two-row layouts (96, 32) stay
    dense in the same context; each sample equals its dense solo run."""
    samples = []
    for i, (n, r) in enumerate([(64, 4.0), (96, 6.0), (128, 5.0), (32, 3.0)]):
        geo = inputs.spheres(n, n // 4 + 3, n // 4 + 5, r, 0.6, seed=950 + i)
        samples.append((geo.solid,))
    g = (1e-4, 2e-5, 0)
    print("[case] mixed batch", flush=True)
    sim, outs = run(samples, 19, "f32", g, 7, graph_chunk=2)
    assert sim.info()["layout"] == 1
    for i, s in enumerate(samples):
        solo, o = run([s], 19, "f32", g, 7, layout=0, tile=2)
        assert_same(outs[i], o[0], i)
        solo.close()
    sim.close()


def test_packed_rejects_dense_tiles():
    solid, drho, u = state(64, 4, 4, seed=8500)
    with pytest.raises(tau1.Tau1Error):
        tau1.Sim([tau1.Sample(solid, drho, u)], lattice=19, precision="f32", kernel=1,
                 tile=6, layout=1)
    with pytest.raises(tau1.Tau1Error):
        tau1.Sim([tau1.Sample(solid, drho, u)], lattice=19, precision="f32", kernel=1,
                 tile=14, layout=0)


@pytest.mark.parametrize("tile,layout", [(6, 0), (14, 1)])
def test_padding_rows_ignore_workspace_contents(tile, layout):
    """Shared-row tiles pad the rows of a z-segment to blocks of four waves;
    a padding row (y >= ny) reads nothing of the lattice's tables, so junk
    left in reused device memory does not change the work or the result."""
    import torch
    solid, drho, u = state(64, 5, 3, seed=8600)
    g = (1e-5, 3e-6, -2e-6)
    n = tau1.workspace_size([(solid, drho, u)], kernel=1, tile=tile, layout=layout)
    junk = torch.full((n + 256,), 0xC0, dtype=torch.uint8, device="cuda:0")
    torch.cuda.synchronize()
    del junk
    print(f"[case] padding rows over junk memory tile={tile}", flush=True)
    sim, out = run([(solid, drho, u)], 19, "f32", g, 5, tile=tile, layout=layout)
    ref = run_oracle(19, solid, drho, u, g, 5)
    err = reduced_errors(out[0], ref, solid)
    eps = 2.0 ** -24
    assert err["u_rel_l2"] <= 8.0 * eps
    sim.close()


def test_dense_one_row_layout_in_packed_context():
    """A one-row layout too large to pack (here nx = 512 with 4 * 136M * 4 B
    of state per buffer) runs the dense shared-row schedule next to a packed
    layout of the same context; both match their solo runs bit for bit."""
    big = np.zeros((520, 512, 512), np.uint8)
    small, ds_, us_ = state(512, 3, 5, seed=8700)
    other, do_, uo_ = state(256, 6, 5, seed=8701)
    g = (1e-5, 2e-6, 0.0)
    print("[case] dense one-row layout in a packed context", flush=True)
    sim = tau1.Sim([tau1.Sample(big), tau1.Sample(small, ds_, us_), tau1.Sample(other, do_, uo_)],
                   lattice=19, precision="f32", g=g, kernel=1, tile=13, layout=1)
    assert sim.info()["layout"] == 1
    sim.step(4)
    got_small, got_other = sim.moments(1), sim.moments(2)
    sim.close()
    solo_s, o_s = run([(small, ds_, us_)], 19, "f32", g, 4, tile=5, layout=0)
    solo_o, o_o = run([(other, do_, uo_)], 19, "f32", g, 4, tile=13, layout=1)
    assert_same(got_small, o_s[0], "dense 512 row layout")
    assert_same(got_other, o_o[0], "packed 256 row layout")
    solo_s.close()
    solo_o.close()
