"""One launch for a batch's one-chunk rows (batch_graph 3) against the
per-layout launches.

Every sample whose row is 64-320 nodes long runs in one launch of
k_zmarch_rows, which switches to the sample's lane layout per work item and
forms each sum as that layout's own kernel does: the batch gives the same
bits as the chains of per-layout launches.  Rows of 512 nodes (two lane
chunks) and 32 (two rows per wave) launch on their own beside it."""
import numpy as np
import pytest

from paper_2312_14742_amd import inputs, tau1

from gpu_helpers import UNIT_ROUNDOFF, reduced_errors, run_oracle

pytestmark = pytest.mark.gpu

ONE_CHUNK = [64, 96, 128, 160, 192, 224, 256, 288, 320]


def batch(seed, nz=40, solid_frac=0.5, extra=(512, 32)):
    shapes = [(nx, 5 + i % 3, nz - 3 * (i % 4)) for i, nx in enumerate(ONE_CHUNK + list(extra))]
    return shapes, [inputs.random_state(nx, ny, nz_, seed=seed + i, solid_frac=solid_frac)
                    for i, (nx, ny, nz_) in enumerate(shapes)]


def make(samples, q, prec, g, shape, **kw):
    return tau1.Sim([tau1.Sample(*s) for s in samples], lattice=q, precision=prec, g=g,
                    kernel=1, batch_graph=shape, **kw)


def assert_same(a, b, label):
    assert a[0].tobytes() == b[0].tobytes(), label
    assert a[1].tobytes() == b[1].tobytes(), label


@pytest.mark.parametrize("layout,tile", [(0, 5), (1, 13)])
@pytest.mark.parametrize("q", [15, 19, 27])
def test_rows_launch_equals_chains(q, layout, tile):
    shapes, samples = batch(9800 + q + layout)
    g = (1e-5, -2e-6, 3e-6)
    print(f"[case] rows launch q={q} layout={layout} tile={tile}", flush=True)
    one = make(samples, q, "f32", g, 3, layout=layout, tile=tile)
    ch = make(samples, q, "f32", g, 2, layout=layout, tile=tile)
    # the nine one-chunk layouts in one launch; 512 and 32 alone
    assert one.info()["launches_per_step"] == 3
    assert ch.info()["launches_per_step"] == len(shapes)
    assert one.info()["work_items"] == ch.info()["work_items"]
    one.step(6)
    ch.step(6)
    for i in range(len(samples)):
        assert_same(one.moments(i), ch.moments(i), (q, layout, shapes[i]))
        assert one.permeability(i, 0) == ch.permeability(i, 0)
    one.close()
    ch.close()


def test_rows_launch_against_oracle():
    """Two samples of a one-launch batch against the FP64 oracle (FP32
    bounds of the step tests)."""
    shapes, samples = batch(9900, nz=12, extra=())
    g = (1e-5, 0.0, -2e-6)
    print("[case] rows launch vs oracle", flush=True)
    sim = make(samples, 19, "f32", g, 3, layout=1, tile=12)
    assert sim.info()["launches_per_step"] == 1
    sim.step(8)
    eps = UNIT_ROUNDOFF["f32"]
    for i in (1, 7):   # rows of 96 and 288 nodes: lanes 48..63 idle
        solid, drho, u = samples[i]
        ref = run_oracle(19, solid, drho, u, g, 8)
        err = reduced_errors(sim.moments(i), ref, solid)
        print(f"[err] {shapes[i]} {err}", flush=True)
        assert err["drho_abs"] <= (2.0 * eps + 16.0 * eps) * np.abs(u).max()
        assert err["u_rel_l2"] <= 8.0 * eps
    sim.close()


@pytest.mark.parametrize("prec", ["f16", "bf16"])
def test_rows_launch_16bit(prec):
    shapes, samples = batch(9950, extra=(512,))
    g = (1e-5, -2e-6, 3e-6)
    print(f"[case] rows launch {prec}", flush=True)
    one = make(samples, 19, prec, g, 3, tile=14)
    ch = make(samples, 19, prec, g, 2, tile=14)
    assert one.info()["launches_per_step"] == 2
    one.step(5)
    ch.step(5)
    for i in range(len(samples)):
        assert_same(one.moments(i), ch.moments(i), (prec, shapes[i]))
    one.close()
    ch.close()


def test_rows_launch_graph_replays():
    """Steps in 4-step graphs (and two single launches) equal single launches."""
    _, samples = batch(9970, nz=20, extra=())
    g = (2e-5, 0.0, 0.0)
    print("[case] rows launch graph replays", flush=True)
    a = make(samples, 19, "f32", g, 3, graph_chunk=4)
    b = make(samples, 19, "f32", g, 3, graph_chunk=200)
    a.step(10)
    b.step(10)
    for i in range(len(samples)):
        assert_same(a.moments(i), b.moments(i), ("graph", i))
    a.close()
    b.close()


def test_rows_launch_autotune_bitwise():
    """The autotuner times each layout alone, then lays the layouts whose
    tiles share the leading schedule into one launch; a layout that picks the
    chunk tile launches alone.  The tuned batch equals the batch at one fixed
    tile in per-layout chains, bit for bit."""
    shapes = [(64, 8, 9), (256, 5, 6), (96, 7, 5), (320, 4, 4), (160, 6, 7), (128, 9, 6)]
    fracs = [0.4, 0.4, 0.4, 0.4, 0.96, 0.4]
    samples = [inputs.random_state(nx, ny, nz, seed=9990 + i, solid_frac=sf)
               for i, ((nx, ny, nz), sf) in enumerate(zip(shapes, fracs))]
    g = (1e-5, -3e-6, 2e-6)
    print("[case] rows launch autotune", flush=True)
    fixed = make(samples, 19, "f32", g, 2, tile=13)
    fixed.step(7)
    tuned = make(samples, 19, "f32", g, 3)
    tuned.step(3)
    tuned.autotune(2)
    print(f"[info] tuned {tuned.info()}", flush=True)
    assert 1 <= tuned.info()["launches_per_step"] <= len(shapes)
    tuned.step(4)
    for i in range(len(samples)):
        assert_same(tuned.moments(i), fixed.moments(i), ("autotune", i))
    fixed.close()
    tuned.close()


def test_rows_launch_single_layout():
    """A batch of one lane layout (and a single sample) keeps its own
    per-layout kernel under batch_graph 3: one launch, the same bits."""
    g = (1e-5, 0.0, 2e-6)
    samples = [inputs.random_state(128, 6, 9, seed=9995 + i, solid_frac=0.5) for i in range(2)]
    print("[case] rows launch, one layout", flush=True)
    for group in (samples, samples[:1]):
        a = make(group, 19, "f32", g, 3)
        b = make(group, 19, "f32", g, 0)
        assert a.info()["launches_per_step"] == 1
        a.step(4)
        b.step(4)
        for i in range(len(group)):
            assert_same(a.moments(i), b.moments(i), ("one layout", len(group), i))
        a.close()
        b.close()
