"""Parity at the benchmark sizes, in the benchmark's launch configuration.

The oracle cannot run these lattices for many steps, so each case takes the
GPU state after a few steps, advances the GPU by one more step and compares
sampled nodes with the oracle's single-node update (``step_nodes``) of that
same state.  Every z-march lane layout and tile these workloads use is the one
the autotuner picks, as in bench.py.
"""
import numpy as np
import pytest

from paper_2312_14742_amd import inputs, tau1

from gpu_helpers import check_step, sample_nodes

pytestmark = pytest.mark.gpu

def random_fields(solid, seed, drho_amp=1e-3, u_amp=0.05):
    rng = np.random.Generator(np.random.PCG64(seed))
    drho = rng.uniform(-drho_amp, drho_amp, solid.shape)
    u = rng.uniform(-u_amp, u_amp, (3,) + solid.shape)
    drho[solid == 1] = 0.0
    u[:, solid == 1] = 0.0
    return drho, u


@pytest.mark.parametrize("q", [19, 15, 27])
def test_512_cube_porosity07_f32(q):
    """Headline and lattice-sweep workload: 512^3, r = 12, porosity 0.7."""
    geo = inputs.spheres(512, 512, 512, 12.0, 0.7, seed=3000)
    drho, u = random_fields(geo.solid, seed=41 + q)
    g = (1e-6, 0.0, 0.0)
    print(f"[case] 512^3 porosity 0.7 D3Q{q} f32", flush=True)
    with tau1.Sim([tau1.Sample(geo.solid, drho, u)], lattice=q, precision="f32", g=g,
                  graph_chunk=100) as sim:
        sim.autotune(5)
        assert sim.info()["kernel"] == 1
        sim.step(3)
        idx = sample_nodes(geo.solid, 40000, seed=q)
        check_step(sim, 0, geo.solid, q, "f32", g, idx, f"D3Q{q} tile {sim.info()['tile']}")


@pytest.mark.parametrize("prec", ["f16", "bf16"])
def test_512_cube_porosity06_16bit(prec):
    """Reduced-storage workload: 512^3, r = 12, porosity 0.6."""
    geo = inputs.spheres(512, 512, 512, 12.0, 0.6, seed=4000)
    drho, u = random_fields(geo.solid, seed=7, drho_amp=1e-4, u_amp=0.01)
    g = (1e-6, 0.0, 0.0)
    print(f"[case] 512^3 porosity 0.6 D3Q19 {prec}", flush=True)
    with tau1.Sim([tau1.Sample(geo.solid, drho, u)], lattice=19, precision=prec, g=g,
                  graph_chunk=100) as sim:                      # default F16 scales
        sim.autotune(5)
        sim.step(2)
        idx = sample_nodes(geo.solid, 40000, seed=5)
        check_step(sim, 0, geo.solid, 19, prec, g, idx, f"{prec} tile {sim.info()['tile']}")


@pytest.mark.parametrize("transform", ["mirror_x", "permute_axes"])
def test_512_cube_symmetry(transform):
    """A property that holds at any size, checked at the full size where the
    oracle cannot follow many steps: running the x-mirrored, or the
    axis-permuted ((x, y, z) -> (y, z, x)), copy of the headline workload
    gives the mirrored or permuted result.  The two runs round their sums in
    different orders, so they agree to FP32 rounding: rel-L2(u) within
    steps x 2 x 2^-24 and drho within that times max|u|."""
    geo = inputs.spheres(512, 512, 512, 12.0, 0.7, seed=3000)
    drho, u = random_fields(geo.solid, seed=43)
    g = (1e-6, 2e-7, -3e-7)
    steps = 20
    if transform == "mirror_x":
        tf = lambda a: np.ascontiguousarray(a[:, :, ::-1])        # noqa: E731
        ut = np.stack([-tf(u[0]), tf(u[1]), tf(u[2])])
        gt = (-g[0], g[1], g[2])
        back = lambda uu: np.stack([-tf(uu[0]), tf(uu[1]), tf(uu[2])])  # noqa: E731
    else:
        tf = lambda a: np.ascontiguousarray(a.transpose(2, 0, 1))  # noqa: E731
        ut = np.stack([tf(u[1]), tf(u[2]), tf(u[0])])
        gt = (g[1], g[2], g[0])
        back = lambda uu: np.stack([tf(uu[1]), tf(uu[2]), tf(uu[0])])  # noqa: E731
    print(f"[case] 512^3 porosity 0.7 f32 {transform}", flush=True)
    res = []
    for solid, d0, u0, gg in ((geo.solid, drho, u, g), (tf(geo.solid), tf(drho), ut, gt)):
        with tau1.Sim([tau1.Sample(solid, d0, u0)], lattice=19, precision="f32", g=gg,
                      graph_chunk=10) as sim:
            sim.autotune(3)
            assert sim.info()["kernel"] == 1
            sim.step(steps)
            res.append(sim.moments(0))
    (d_a, u_a), (d_b, u_b) = res
    fl = tf(geo.solid) == 0
    want_u = back(u_a)
    eu = float(np.sqrt(np.sum((u_b - want_u)[:, fl] ** 2) / np.sum(want_u[:, fl] ** 2)))
    ed = float(np.abs(d_b - tf(d_a)).max())
    bound = steps * 2.0 * 2.0 ** -24
    print(f"[err] {transform}: rel-L2(u) {eu:.3e}, max|ddrho| {ed:.3e}", flush=True)
    assert eu <= bound
    assert ed <= bound * np.abs(u_a).max()


def test_arrays_beyond_32bit_offsets():
    """512 x 512 x 2048 (537M nodes): each FP32 state array is larger than the
    z-march kernels' 32-bit buffer offsets reach, so the context runs the
    per-node gather kernel on the dense layout (64-bit indexing)."""
    geo = inputs.spheres(512, 512, 2048, 12.0, 0.7, seed=3100)
    g = (1e-5, -2e-6, 3e-6)
    print("[case] 512x512x2048 porosity 0.7 D3Q19 f32", flush=True)
    with tau1.Sim([tau1.Sample(geo.solid)], lattice=19, precision="f32", g=g,
                  graph_chunk=100) as sim:
        sim.autotune(2)
        inf = sim.info()
        assert inf["kernel"] == 0 and inf["layout"] == 0
        sim.step(3)
        idx = sample_nodes(geo.solid, 20000, seed=11)
        check_step(sim, 0, geo.solid, 19, "f32", g, idx, "512x512x2048 gather")
        k, mass = sim.permeability(0, 0)
    assert abs(mass - geo.n_fluid) <= 1e-9 * geo.n_fluid
    assert np.isfinite(k) and k > 0


def test_batch_of_64_samples():
    """Batched workload: 64 uneven samples in one context, sampled per sample."""
    batch = inputs.batch_recipe(64, 5000, workers=8)
    g = (1e-3, 2e-4, -3e-4)
    print("[case] batch of 64 samples", flush=True)
    with tau1.Sim([tau1.Sample(b.geometry.solid) for b in batch], lattice=19, precision="f32",
                  g=g, graph_chunk=100) as sim:
        sim.autotune(3)
        sim.step(4)
        sides = [b.side for b in batch]
        picks = sorted({0, int(np.argmin(sides)), int(np.argmax(sides)), 33})
        for i in picks:
            solid = batch[i].geometry.solid
            idx = sample_nodes(solid, 8000, seed=100 + i)
            # one more step for the whole batch per checked sample
            check_step(sim, i, solid, 19, "f32", g, idx, f"sample {i} side {sides[i]}")


def test_batch_of_64_samples_one_launch():
    """The same batch with one launch per step for every sample (batch_graph
    3, k_zmarch_rows): sampled nodes against the oracle's update."""
    batch = inputs.batch_recipe(64, 5000, workers=8)
    g = (1e-3, 2e-4, -3e-4)
    print("[case] batch of 64 samples, one launch", flush=True)
    with tau1.Sim([tau1.Sample(b.geometry.solid) for b in batch], lattice=19, precision="f32",
                  g=g, graph_chunk=100, batch_graph=3) as sim:
        sim.autotune(3)
        assert sim.info()["launches_per_step"] == 1
        sim.step(4)
        sides = [b.side for b in batch]
        picks = sorted({int(np.argmin(sides)), int(np.argmax(sides)), 7, 40})
        for i in picks:
            solid = batch[i].geometry.solid
            idx = sample_nodes(solid, 8000, seed=200 + i)
            check_step(sim, i, solid, 19, "f32", g, idx, f"one launch: sample {i} side {sides[i]}")
