"""Parity of the z-march step kernel (kernel=1) with the FP64 oracle, its
invariances, and its edge cases (lane layouts, ragged row groups, short
z-segments, periodic wrap onto itself)."""
import numpy as np
import pytest

import oracle
from paper_2312_14742_amd import inputs, tau1

from gpu_helpers import reduced_errors, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

UNIT_ROUNDOFF = {"f32": 2.0 ** -24, "f16": 2.0 ** -11, "bf16": 2.0 ** -8}


def bounds(prec, u_scale):
    eps = UNIT_ROUNDOFF[prec]
    return {"drho_abs": (2.0 * eps + 16.0 * 2.0 ** -24) * u_scale, "u_rel_l2": 8.0 * eps}


# nx values cover every lane layout: G rows per wave, C chunks x L lanes x K
# nodes (L = 64 / G, or fewer: the other lanes of the wave stay idle)
LAYOUT_DIMS = [
    (64, 5, 7),     # G=1 C=1 K=1
    (128, 3, 4),    # G=1 C=1 K=2
    (192, 2, 3),    # G=1 C=1 K=3
    (256, 3, 2),    # G=1 C=1 K=4
    (320, 2, 2),    # G=1 C=1 K=5
    (384, 2, 3),    # G=1 C=2 K=3
    (512, 2, 3),    # G=1 C=2 K=4
    (32, 9, 4),     # G=2 C=1 K=1
    (96, 5, 5),     # G=1 C=1 K=2, 48 lanes
    (160, 3, 3),    # G=1 C=1 K=4, 40 lanes
    (224, 3, 2),    # G=1 C=1 K=4, 56 lanes
    (288, 3, 2),    # G=1 C=1 K=6, 48 lanes
    (16, 6, 5),     # G=4 C=1 K=1
    (48, 7, 3),     # G=4 C=1 K=3
    (80, 5, 3),     # G=4 C=1 K=5
]


@pytest.mark.parametrize("tile", [2, 6, 10])
@pytest.mark.parametrize("dims", LAYOUT_DIMS)
@pytest.mark.parametrize("q", [15, 19, 27])
def test_layouts_f32(q, dims, tile):
    """Tile 2 loads each source row itself; tile 6 shares rows through LDS
    (one-row layouts) or prefetches them (multi-row layouts); tile 10
    prefetches them."""
    nx, ny, nz = dims
    solid, drho, u = inputs.random_state(nx, ny, nz, seed=5000 + nx + 3 * ny + 7 * nz)
    g = (1e-5, -2e-5, 3e-6)
    print(f"[case] zmarch f32 q={q} dims={dims} tile={tile}", flush=True)
    sim, out = run_gpu([(solid, drho, u)], q, "f32", g, 6, kernel=1, tile=tile)
    assert sim.info()["kernel"] == 1
    ref = run_oracle(q, solid, drho, u, g, 6)
    err = reduced_errors(out[0], ref, solid)
    print(f"[err] {err}", flush=True)
    for key, b in bounds("f32", np.abs(u).max()).items():
        assert err[key] <= b, (key, err[key], b)
    sim.close()


@pytest.mark.parametrize("prec", ["f16", "bf16"])
@pytest.mark.parametrize("dims", [(64, 5, 7), (96, 5, 5), (48, 7, 3)])
def test_layouts_16bit(prec, dims):
    nx, ny, nz = dims
    solid, drho, u = inputs.random_state(nx, ny, nz, seed=6000 + nx + ny)
    g = (1e-5, -2e-5, 3e-6)
    print(f"[case] zmarch {prec} dims={dims}", flush=True)
    sim, out = run_gpu([(solid, drho, u)], 19, prec, g, 6, kernel=1)   # default F16 scales
    ref = run_oracle(19, solid, drho, u, g, 6)
    err = reduced_errors(out[0], ref, solid)
    print(f"[err] {err}", flush=True)
    for key, b in bounds(prec, np.abs(u).max()).items():
        assert err[key] <= b, (key, err[key], b)
    sim.close()


@pytest.mark.parametrize("tile", [2, 6])
@pytest.mark.parametrize("dims", [(64, 1, 1), (32, 1, 3), (16, 2, 1), (64, 3, 2), (32, 5, 1),
                                  (64, 5, 3), (128, 6, 2), (64, 9, 4)])
def test_degenerate_periodic(dims, tile):
    """ny or nz of 1-3 (the stencil wraps onto the node's own row/plane) and
    ny not a multiple of the four rows a workgroup shares."""
    nx, ny, nz = dims
    solid, drho, u = inputs.random_state(nx, ny, nz, seed=77 + nx * ny * nz)
    g = (1e-5, 3e-6, -2e-6)
    print(f"[case] zmarch degenerate dims={dims} tile={tile}", flush=True)
    sim, out = run_gpu([(solid, drho, u)], 19, "f32", g, 5, kernel=1, tile=tile)
    ref = run_oracle(19, solid, drho, u, g, 5)
    err = reduced_errors(out[0], ref, solid)
    for key, b in bounds("f32", np.abs(u).max()).items():
        assert err[key] <= b, (key, err[key], b)
    sim.close()


def test_tile_shapes_bitwise_identical():
    """Every z-segment length gives the same bits (fixed per-node order)."""
    geo = inputs.spheres(64, 20, 70, 5.0, 0.7, seed=12)
    g = (1e-5, 0, 0)
    outs = []
    for tile in range(4):
        print(f"[case] tile {tile}", flush=True)
        sim, out = run_gpu([(geo.solid,)], 19, "f32", g, 9, kernel=1, tile=tile)
        outs.append(out[0])
        sim.close()
    for o in outs[1:]:
        assert o[0].tobytes() == outs[0][0].tobytes()
        assert o[1].tobytes() == outs[0][1].tobytes()


def test_batched_uneven_equals_solo_bitwise():
    samples = []
    for i, (n, r) in enumerate([(32, 3.0), (96, 6.0), (64, 4.0), (160, 7.0)]):
        geo = inputs.spheres(n, n // 2 + 3, n // 4 + 5, r, 0.6, seed=900 + i)
        samples.append((geo.solid,))
    g = (1e-5, 0, 0)
    print("[case] zmarch batched vs solo", flush=True)
    sim, outs = run_gpu(samples, 19, "f32", g, 7, kernel=1, graph_chunk=2)
    for i, s in enumerate(samples):
        solo, o = run_gpu([s], 19, "f32", g, 7, kernel=1)
        assert outs[i][0].tobytes() == o[0][0].tobytes()
        assert outs[i][1].tobytes() == o[0][1].tobytes()
        solo.close()
    sim.close()


def test_channel_config1_f32_closed_form():
    """32^3 channel with the z-march kernel against the transient closed form."""
    from test_oracle_pins import channel_closed_form
    solid = inputs.channel(32, 32, 32)
    print("[case] zmarch channel", flush=True)
    sim, out = run_gpu([(solid,)], 19, "f32", (1e-6, 0, 0), 200, kernel=1)
    ref = channel_closed_form(30, 1e-6, 200)
    ux = out[0][1][0][1:-1]
    assert np.abs(ux - ref[:, None, None]).max() <= 2e-5 * ref.max()
    sim.close()


def test_porous_against_oracle_f32():
    geo = inputs.spheres(64, 48, 40, 5.0, 0.7, seed=33)
    g = (1e-5, 0, 0)
    print("[case] zmarch porous 64x48x40", flush=True)
    sim, out = run_gpu([(geo.solid,)], 19, "f32", g, 100, kernel=1)
    ref = run_oracle(19, geo.solid, None, None, g, 100)
    err = reduced_errors(out[0], ref, geo.solid)
    print(f"[err] {err}", flush=True)
    assert err["u_rel_l2"] <= 1e-5
    k, m = sim.permeability(0, 0)
    mref, kref = oracle.reduce(ref, 0, g[0])
    assert abs(k - kref) <= 1e-5 * abs(kref)
    sim.close()


def test_prefetch_tiles_bitwise_identical():
    """Shared-row (4-7) and rolling-prefetch (8-11) tiles form every sum in
    the same order as the just-in-time tiles (0-3)."""
    geo = inputs.spheres(64, 20, 70, 5.0, 0.7, seed=12)
    g = (1e-5, 0, 0)
    outs = []
    for tile in (0, 4, 5, 6, 7, 8, 9, 10, 11):
        print(f"[case] tile {tile}", flush=True)
        sim, out = run_gpu([(geo.solid,)], 19, "f32", g, 9, kernel=1, tile=tile)
        outs.append(out[0])
        sim.close()
    for o in outs[1:]:
        assert o[0].tobytes() == outs[0][0].tobytes()
        assert o[1].tobytes() == outs[0][1].tobytes()


def test_graph_replays_match_single_launches():
    """A two-layout batch (two independent graph chains) replayed several
    times, with readback between replays, against single launches."""
    samples = [inputs.spheres(64, 20, 12, 4.0, 0.7, seed=5).solid,
               inputs.spheres(96, 10, 14, 5.0, 0.6, seed=6).solid]
    g = (1e-4, 2e-5, 0)
    print("[case] graph replays, two layouts", flush=True)
    a = tau1.Sim([tau1.Sample(s) for s in samples], lattice=19, precision="f32", g=g,
                 graph_chunk=2, kernel=1)
    b = tau1.Sim([tau1.Sample(s) for s in samples], lattice=19, precision="f32", g=g,
                 graph_chunk=1000, kernel=1)
    for r in range(5):
        a.step(2)
        b.step(2)
        for i in range(2):
            da, ua = a.moments(i)
            db, ub = b.moments(i)
            assert da.tobytes() == db.tobytes(), (r, i)
            assert ua.tobytes() == ub.tobytes(), (r, i)
    a.close()
    b.close()


def test_autotune_keeps_state_and_uses_cache(tmp_path):
    geo = inputs.spheres(64, 32, 40, 4.0, 0.7, seed=8)
    cache = str(tmp_path / "tau1_tune.txt")
    g = (1e-5, 0, 0)
    print("[case] autotune", flush=True)
    sim = tau1.Sim([tau1.Sample(geo.solid)], lattice=19, precision="f32", g=g, tune_cache=cache)
    sim.step(3)
    before = sim.moments(0)
    tuned = sim.autotune(2)["tile"]
    after = sim.moments(0)
    assert before[0].tobytes() == after[0].tobytes()
    assert before[1].tobytes() == after[1].tobytes()
    sim.step(2)
    ref = run_oracle(19, geo.solid, None, None, g, 5)
    err = reduced_errors(sim.moments(0), ref, geo.solid)
    assert err["u_rel_l2"] <= 8.0 * 2.0 ** -24
    sim.close()
    with open(cache) as f:
        assert any(line.startswith("tau1 gfx950 q19 p1 ") for line in f)
    again = tau1.Sim([tau1.Sample(geo.solid)], lattice=19, precision="f32", g=g,
                     tune_cache=cache)
    assert again.info()["tile"] == tuned
    again.close()


def test_batch_autotune_per_layout_bitwise():
    """The autotuner times each lane layout of a batch alone and gives each its
    own tile; every tile forms the sums in one order, so the tuned batch
    equals the batch at one fixed tile, bit for bit."""
    shapes = [(64, 8, 9), (256, 5, 6), (96, 7, 5), (320, 4, 4), (64, 3, 20)]
    samples = [inputs.random_state(nx, ny, nz, seed=8600 + i, solid_frac=0.4)
               for i, (nx, ny, nz) in enumerate(shapes)]
    g = (1e-5, -3e-6, 2e-6)
    print("[case] batch autotune per layout", flush=True)
    fixed = tau1.Sim([tau1.Sample(*s) for s in samples], lattice=19, precision="f32", g=g,
                     tile=13)
    fixed.step(7)
    tuned = tau1.Sim([tau1.Sample(*s) for s in samples], lattice=19, precision="f32", g=g)
    tuned.step(3)
    tuned.autotune(2)
    tuned.step(4)
    for i in range(len(samples)):
        a, b = fixed.moments(i), tuned.moments(i)
        assert a[0].tobytes() == b[0].tobytes(), i
        assert a[1].tobytes() == b[1].tobytes(), i
    fixed.close()
    tuned.close()


def expected_items(solid, lz, block):
    """Work items (row item x z-segment) holding a fluid node; shared-row
    tiles keep or drop blocks of four row items."""
    nz, ny, nx = solid.shape
    rowf = (solid == 0).any(axis=2)
    step = 4 if block else 1
    rows = (ny + 3) // 4 * 4 if block else ny
    n = 0
    for z0 in range(0, nz, lz):
        for r0 in range(0, rows, step):
            if rowf[z0:z0 + lz, r0:min(r0 + step, ny)].any():
                n += step
    return n


def test_all_solid_regions_are_skipped():
    """Row groups and z-segments without a fluid node are not visited; every
    tile still gives the oracle's result and the same bits."""
    nx, ny, nz = 64, 12, 48
    solid, drho, u = inputs.random_state(nx, ny, nz, seed=8800)
    solid[:32] = 1          # planes 0-31 solid
    solid[:, 4:8] = 1       # rows 4-7 solid in every plane
    drho[solid == 1] = 0.0
    u[:, solid == 1] = 0.0
    g = (1e-5, -2e-5, 3e-6)
    ref = run_oracle(19, solid, drho, u, g, 6)
    outs = []
    for tile in (0, 2, 4, 6, 8, 12, 14):
        print(f"[case] solid regions, tile {tile}", flush=True)
        sim, out = run_gpu([(solid, drho, u)], 19, "f32", g, 6, kernel=1, tile=tile,
                           layout=1 if tile >= 12 else 0)
        lz = (16, 32, 64, 128)[tile % 4]
        block = tile // 4 in (1, 3)
        assert sim.info()["work_items"] == expected_items(solid, lz, block), tile
        assert expected_items(solid, lz, block) < expected_items(np.zeros_like(solid), lz, block)
        err = reduced_errors(out[0], ref, solid)
        for key, b in bounds("f32", np.abs(u).max()).items():
            assert err[key] <= b, (tile, key, err[key], b)
        outs.append(out[0])
        sim.close()
    for o in outs[1:]:
        assert o[0].tobytes() == outs[0][0].tobytes()
        assert o[1].tobytes() == outs[0][1].tobytes()
