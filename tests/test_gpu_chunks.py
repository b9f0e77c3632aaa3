"""The chunk tile (one lane per stored chunk of the packed layout) against the
packed z-march and the oracle.

The chunk kernel forms every destination sum in the order in which the
z-march forms it, so the two give the same bits, step after step, on every
lane layout and storage mode; a batch mixing packed and dense lane layouts
runs the dense ones on the z-march within the same step."""
import numpy as np
import pytest

from paper_2312_14742_amd import inputs, tau1

from gpu_helpers import UNIT_ROUNDOFF, reduced_errors, run_oracle

pytestmark = pytest.mark.gpu

CHUNK_TILE = 16

# one-row lane layouts: chunks of K = 1, 2, 3, 4, 5 nodes with one chunk
# group per row, K = 3 and 4 with two groups (nx = 384, 512), and the
# layouts with idle lanes (96, 160, 224, 288: K = 2, 4, 4, 6)
DIMS = [(64, 5, 7), (128, 3, 4), (192, 2, 3), (256, 3, 2), (320, 2, 2), (384, 2, 3),
        (512, 2, 3), (96, 5, 5), (160, 3, 3), (224, 3, 2), (288, 3, 2)]


def run(samples, q, prec, g, nsteps, **kw):
    sim = tau1.Sim([tau1.Sample(*s) for s in samples], lattice=q, precision=prec, g=g,
                   kernel=1, layout=1, **kw)
    sim.step(nsteps)
    return sim, [sim.moments(i) for i in range(len(samples))]


def assert_same(a, b, label):
    assert a[0].tobytes() == b[0].tobytes(), label
    assert a[1].tobytes() == b[1].tobytes(), label


@pytest.mark.parametrize("solid_frac", [0.6, 0.92])
@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("q", [15, 19, 27])
def test_chunks_equal_zmarch_bitwise(q, dims, solid_frac):
    nx, ny, nz = dims
    solid, drho, u = inputs.random_state(nx, ny, nz, seed=9100 + nx + 7 * ny + q,
                                         solid_frac=solid_frac)
    g = (1e-5, -2e-5, 3e-6)
    print(f"[case] chunks vs z-march q={q} dims={dims} solid={solid_frac}", flush=True)
    zm, oz = run([(solid, drho, u)], q, "f32", g, 6, tile=12)
    ck, oc = run([(solid, drho, u)], q, "f32", g, 6, tile=CHUNK_TILE)
    assert ck.info()["tile"] == CHUNK_TILE and ck.info()["layout"] == 1
    assert_same(oc[0], oz[0], (q, dims, solid_frac))
    for axis in range(3):
        assert ck.permeability(0, axis) == zm.permeability(0, axis)
    zm.close()
    ck.close()


@pytest.mark.parametrize("prec", ["f16", "bf16"])
@pytest.mark.parametrize("dims", [(256, 3, 5), (512, 2, 3), (288, 3, 2)])
def test_chunks_16bit_bitwise(prec, dims):
    nx, ny, nz = dims
    solid, drho, u = inputs.random_state(nx, ny, nz, seed=9200 + nx, solid_frac=0.8)
    g = (1e-5, -2e-5, 3e-6)
    print(f"[case] chunks {prec} dims={dims}", flush=True)
    zm, oz = run([(solid, drho, u)], 19, prec, g, 5, tile=13)
    ck, oc = run([(solid, drho, u)], 19, prec, g, 5, tile=CHUNK_TILE)
    assert_same(oc[0], oz[0], (prec, dims))
    zm.close()
    ck.close()


@pytest.mark.parametrize("target", [0.05, 0.2])
def test_chunks_low_porosity_against_oracle(target):
    """A sphere packing of low porosity (r = 4, 64 x 48 x 40): FP32 chunk
    kernel against the FP64 oracle, within the FP32 bounds of the step tests."""
    geo = inputs.spheres(64, 48, 40, 4.0, target, seed=9300)
    solid = geo.solid
    rng = np.random.Generator(np.random.PCG64(9301))
    fl = solid == 0
    drho = np.where(fl, rng.uniform(-1e-3, 1e-3, solid.shape), 0.0)
    u = np.where(fl, rng.uniform(-0.02, 0.02, (3,) + solid.shape), 0.0)
    g = (1e-5, 0.0, -2e-6)
    print(f"[case] chunks phi={geo.porosity:.3f} vs oracle", flush=True)
    sim, out = run([(solid, drho, u)], 19, "f32", g, 8, tile=CHUNK_TILE)
    ref = run_oracle(19, solid, drho, u, g, 8)
    err = reduced_errors(out[0], ref, solid)
    print(f"[err] {err}", flush=True)
    eps = UNIT_ROUNDOFF["f32"]
    assert err["drho_abs"] <= (2.0 * eps + 16.0 * eps) * np.abs(u).max()
    assert err["u_rel_l2"] <= 8.0 * eps
    sim.close()


def test_chunks_batch_mixed_layouts():
    """A batch of packed layouts (nx = 64, 256, 96) and a dense two-rows-per-wave
    layout (nx = 32): the chunk tile runs the packed groups on the chunk kernel
    and the dense group on the z-march; every sample equals its own z-march run."""
    g = (1e-5, 2e-6, -1e-6)
    shapes = [(64, 4, 6), (256, 3, 4), (96, 5, 3), (32, 6, 4), (64, 3, 5)]
    samples = [inputs.random_state(nx, ny, nz, seed=9400 + i, solid_frac=0.85)
               for i, (nx, ny, nz) in enumerate(shapes)]
    print("[case] chunks batch of mixed layouts", flush=True)
    sim = tau1.Sim([tau1.Sample(*s) for s in samples], lattice=19, precision="f32", g=g,
                   kernel=1, tile=CHUNK_TILE, graph_chunk=4)
    sim.step(10)   # two 4-step graphs and two single launches
    assert sim.info()["tile"] == CHUNK_TILE
    for i, s in enumerate(samples):
        # the nx = 32 layout is never packed: its own run is a dense z-march
        dense = shapes[i][0] == 32
        zm = tau1.Sim([tau1.Sample(*s)], lattice=19, precision="f32", g=g, kernel=1,
                      tile=2 if dense else 14, layout=0 if dense else 1)
        zm.step(10)
        assert_same(sim.moments(i), zm.moments(0), ("batch", i))
        zm.close()
    sim.close()


def test_chunks_all_solid_and_all_fluid_samples():
    """Degenerate samples in one chunk-tile batch: an all-solid sample (no
    stored chunk, no work item), an all-fluid one (every chunk stored, every
    lane's x-neighbours in the neighbouring lanes), and a sample whose only
    fluid is one chunk per row at the periodic x wrap (chunks 0 and nch - 1)."""
    g = (1e-5, -1e-5, 2e-6)
    rng = np.random.Generator(np.random.PCG64(9600))
    solid_all = np.ones((4, 5, 256), np.uint8)
    fluid_all = np.zeros((3, 4, 256), np.uint8)
    wrap = np.ones((5, 6, 256), np.uint8)
    wrap[:, :, :3] = 0          # chunk 0 (nodes 0-3) partly fluid
    wrap[:, :, -2:] = 0         # chunk 63 (nodes 252-255) partly fluid
    samples = []
    for solid in (solid_all, fluid_all, wrap):
        fl = solid == 0
        drho = np.where(fl, rng.uniform(-1e-3, 1e-3, solid.shape), 0.0)
        u = np.where(fl, rng.uniform(-0.02, 0.02, (3,) + solid.shape), 0.0)
        samples.append((solid, drho, u))
    print("[case] chunks degenerate samples", flush=True)
    ck = tau1.Sim([tau1.Sample(*s) for s in samples], lattice=19, precision="f32", g=g,
                  kernel=1, tile=CHUNK_TILE)
    ck.step(6)
    for i, s in enumerate(samples):
        zm, oz = run([s], 19, "f32", g, 6, tile=12)
        assert_same(ck.moments(i), oz[0], ("degenerate", i))
        zm.close()
    ck.close()


def test_autotune_mixed_chunk_records():
    """A batch where only some lane layouts hold the chunk tile's records (a
    mostly solid sample gets them, samples that keep most of their chunks do
    not): the autotuner offers the chunk tile only to the former, and the tuned
    batch equals the batch at one fixed z-march tile, bit for bit."""
    g = (1e-5, -2e-6, 1e-6)
    specs = [((256, 6, 8), 0.95), ((128, 5, 6), 0.3), ((256, 4, 5), 0.3), ((96, 5, 4), 0.97)]
    samples = [inputs.random_state(nx, ny, nz, seed=9700 + i, solid_frac=sf)
               for i, ((nx, ny, nz), sf) in enumerate(specs)]
    print("[case] autotune with and without chunk records", flush=True)
    fixed = tau1.Sim([tau1.Sample(*s) for s in samples], lattice=19, precision="f32", g=g,
                     kernel=1, tile=12)
    fixed.step(6)
    tuned = tau1.Sim([tau1.Sample(*s) for s in samples], lattice=19, precision="f32", g=g,
                     kernel=1)
    tuned.step(2)
    tuned.autotune(2)
    tuned.step(4)
    for i in range(len(samples)):
        assert_same(tuned.moments(i), fixed.moments(i), ("mixed records", i))
    fixed.close()
    tuned.close()


def test_chunks_graph_replays():
    """100 steps as 10-step graph replays equal 100 single launches."""
    solid, drho, u = inputs.random_state(128, 6, 8, seed=9500, solid_frac=0.9)
    g = (2e-5, 0.0, 0.0)
    print("[case] chunks graph replays", flush=True)
    a, oa = run([(solid, drho, u)], 19, "f32", g, 100, tile=CHUNK_TILE, graph_chunk=10)
    # graph_chunk above the step count: single launches only
    b, ob = run([(solid, drho, u)], 19, "f32", g, 100, tile=CHUNK_TILE, graph_chunk=200)
    assert_same(oa[0], ob[0], "graph")
    a.close()
    b.close()
