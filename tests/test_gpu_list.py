"""The gather over lists of fluid nodes (kernel 3): the same arithmetic, in
the same order, as the per-node gather over every node (kernel 0), so the two
must give the same bits; against the FP64 oracle; batched samples (the
list-block to sample mapping) and graph replays; and a low-porosity lattice,
the case the kernel is for."""
import numpy as np
import pytest

from paper_2312_14742_amd import inputs, tau1

from gpu_helpers import assert_f64_parity, check_step, run_gpu, run_oracle, sample_nodes

pytestmark = pytest.mark.gpu

G = (1e-5, -2e-5, 3e-6)


def moments_bits(sim, n):
    out = []
    for i in range(n):
        d, u = sim.moments(i)
        out.append((d.tobytes(), u.tobytes()))
    return out


@pytest.mark.parametrize("q", [15, 19, 27])
@pytest.mark.parametrize("prec", ["f64", "f32", "f16", "bf16"])
@pytest.mark.parametrize("dims", [(1, 1, 1), (5, 3, 7), (33, 9, 4), (70, 37, 5)])
def test_list_kernel_equals_gather_bitwise(q, prec, dims):
    nx, ny, nz = dims
    st = inputs.random_state(nx, ny, nz, seed=6000 + nx + 7 * ny + 31 * nz, solid_frac=0.5)
    print(f"[case] list vs gather q={q} {prec} dims={dims}", flush=True)
    a, outa = run_gpu([st], q, prec, G, 10, kernel=0, f16_scales=(18, 18), graph_chunk=4)
    b, outb = run_gpu([st], q, prec, G, 10, kernel=3, f16_scales=(18, 18), graph_chunk=4)
    assert b.info()["kernel"] == 3
    assert outa[0][0].tobytes() == outb[0][0].tobytes()
    assert outa[0][1].tobytes() == outb[0][1].tobytes()
    a.close()
    b.close()


@pytest.mark.parametrize("q", [15, 19, 27])
@pytest.mark.parametrize("case", ["random", "all_fluid", "all_solid", "one_fluid"])
def test_list_kernel_f64_vs_oracle(q, case):
    solid, drho, u = inputs.random_state(12, 10, 9, seed=6100 + q, solid_frac=0.4)
    if case == "all_fluid":
        solid[:] = 0
    elif case in ("all_solid", "one_fluid"):
        solid[:] = 1
        if case == "one_fluid":
            solid[4, 5, 6] = 0
    drho[solid == 1] = 0.0
    u[:, solid == 1] = 0.0
    print(f"[case] list f64 q={q} {case}", flush=True)
    sim, out = run_gpu([(solid, drho, u)], q, "f64", G, 12, kernel=3)
    sim.close()
    ref = run_oracle(q, solid, drho, u, G, 12)
    assert_f64_parity(out[0], ref, solid)


def test_list_kernel_batch_equals_gather_batch():
    """Uneven samples, one of them all solid (no list blocks at all): each
    sample's list blocks must land on that sample."""
    samples = [inputs.random_state(20, 8, 6, seed=6200, solid_frac=0.6),
               (np.ones((3, 4, 5), np.uint8),),
               inputs.random_state(64, 3, 17, seed=6201, solid_frac=0.9),
               inputs.random_state(7, 30, 2, seed=6202, solid_frac=0.2)]
    print("[case] list batch", flush=True)
    a, outa = run_gpu(samples, 19, "f32", G, 9, kernel=0)
    b, outb = run_gpu(samples, 19, "f32", G, 9, kernel=3)
    for (da, ua), (db, ub) in zip(outa, outb):
        assert da.tobytes() == db.tobytes() and ua.tobytes() == ub.tobytes()
    for i in range(len(samples)):
        assert a.permeability(i, 0, with_k=False)[1] == b.permeability(i, 0, with_k=False)[1]
    a.close()
    b.close()


def test_list_kernel_graph_replay_equals_single_launches():
    st = inputs.random_state(24, 12, 10, seed=6300, solid_frac=0.7)
    print("[case] list graph replay", flush=True)
    a, outa = run_gpu([st], 19, "f32", G, 13, kernel=3, graph_chunk=4)
    b, outb = run_gpu([st], 19, "f32", G, 13, kernel=3, graph_chunk=1000)
    assert outa[0][0].tobytes() == outb[0][0].tobytes()
    assert outa[0][1].tobytes() == outb[0][1].tobytes()
    a.close()
    b.close()


def test_list_kernel_low_porosity_256():
    """256^3 sphere packing at porosity 0.05 (r = 8, seed 2000), FP32: after
    a few steps one more step at sampled nodes against the oracle's update of
    the same state, and the permeability against the packed z-march run (same
    inputs, different summation order: FP32 rounding only)."""
    geo = inputs.spheres(256, 256, 256, 8.0, 0.05, seed=2000)
    g = (1e-6, 0.0, 0.0)
    print(f"[case] 256^3 porosity {geo.porosity:.4f} list kernel", flush=True)
    with tau1.Sim([tau1.Sample(geo.solid)], lattice=19, precision="f32", g=g, kernel=3,
                  layout=0, graph_chunk=100) as sim:
        sim.autotune(2)
        assert sim.info()["kernel"] == 3
        sim.step(99)
        idx = sample_nodes(geo.solid, 20000, seed=3)
        check_step(sim, 0, geo.solid, 19, "f32", g, idx, "list kernel porosity 0.05")
        k3, m3 = sim.permeability(0, 0)
    with tau1.Sim([tau1.Sample(geo.solid)], lattice=19, precision="f32", g=g,
                  graph_chunk=100) as ref:
        ref.step(100)
        k1, m1 = ref.permeability(0, 0)
    print(f"[err] list k {k3:.9e} z-march k {k1:.9e}", flush=True)
    assert abs(k3 - k1) <= 100 * 2.0 * 2.0 ** -24 * abs(k1)
    assert abs(m3 - geo.n_fluid) <= 1e-9 * geo.n_fluid
