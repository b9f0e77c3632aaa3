"""Porosity sweep: D3Q19 FP32 on 256^3 periodic sphere packings (r = 8,
target porosity 0.5 ... 0.9, seeds 2000 + i), body force 1e-6 along x,
1000 steps, permeability reported.

The oracle cannot run 1000 steps of 256^3, so each porosity checks:
- the 1000th step at sampled nodes against the oracle's single-node update of
  the GPU state after 999 steps (same bounds as the other full-size cases);
- the FP32 permeability against the library's FP64 mode (itself within 1e-12
  of the oracle on the small cases) on the same input, within
  1000 steps x 2 x 2^-24 relative, FP32 rounding growing at most linearly;
- mass conservation: sum of rho over the fluid nodes stays N_f to 1e-9;
and across the sweep the permeability must grow with the porosity.

At porosity 0.7 the whole 1000-step run is also compared with the oracle's
1000 steps (about 1.2e10 node updates of the FP64 oracle): FP64 mode to the
FP64 parity bar, FP32 rel-L2(u) and permeability within 1000 x 2 x 2^-24."""
import time

import numpy as np
import pytest

import oracle
from paper_2312_14742_amd import inputs, tau1

from gpu_helpers import TOL_F64, check_step, rel_l2, sample_nodes

pytestmark = pytest.mark.gpu

PHIS = [0.5, 0.6, 0.7, 0.8, 0.9]
STEPS = 1000
G = (1e-6, 0.0, 0.0)
_K = {}


@pytest.mark.parametrize("i,phi", list(enumerate(PHIS)))
def test_porosity_sweep_256(i, phi):
    geo = inputs.spheres(256, 256, 256, 8.0, phi, seed=2000 + i)
    nf = geo.n_fluid
    print(f"[case] 256^3 r=8 target porosity {phi} (achieved {geo.porosity:.4f})", flush=True)
    with tau1.Sim([tau1.Sample(geo.solid)], lattice=19, precision="f32", g=G,
                  graph_chunk=100) as sim:
        sim.autotune(3)
        sim.step(STEPS - 1)
        idx = sample_nodes(geo.solid, 20000, seed=i)
        check_step(sim, 0, geo.solid, 19, "f32", G, idx, f"porosity {phi}")
        k32, m32 = sim.permeability(0, 0)
        layout = sim.info()["layout"]
    with tau1.Sim([tau1.Sample(geo.solid)], lattice=19, precision="f64", g=G,
                  graph_chunk=100) as ref:
        ref.step(STEPS)
        k64, m64 = ref.permeability(0, 0)
    print(f"[err] porosity {phi}: layout {layout}, k32 {k32:.9e} k64 {k64:.9e} "
          f"rel {abs(k32 - k64) / k64:.2e}, mass32-Nf {m32 - nf:.3e}", flush=True)
    assert layout == 1
    assert abs(k32 - k64) <= STEPS * 2.0 * 2.0 ** -24 * abs(k64)
    assert abs(m32 - nf) <= 1e-9 * nf
    assert abs(m64 - nf) <= 1e-12 * nf
    _K[phi] = k64


def test_permeability_grows_with_porosity():
    if len(_K) != len(PHIS):
        pytest.skip("needs every porosity of the sweep")
    ks = [_K[p] for p in PHIS]
    assert all(a < b for a, b in zip(ks, ks[1:])), ks


@pytest.mark.timeout(600)    # the oracle's 1000 steps take about 90 s on 16 host threads
def test_porosity_07_full_run_against_oracle():
    i, phi = 2, 0.7
    geo = inputs.spheres(256, 256, 256, 8.0, phi, seed=2000 + i)
    fl = geo.solid == 0
    print(f"[case] 256^3 r=8 porosity {phi}: oracle {STEPS} steps", flush=True)
    t = time.perf_counter()
    ref = oracle.run(19, oracle.State(geo.solid), G, STEPS)
    m_ref, k_ref = oracle.reduce(ref, 0, G[0])
    print(f"[oracle] {time.perf_counter() - t:.1f} s", flush=True)
    for prec in ("f64", "f32"):
        with tau1.Sim([tau1.Sample(geo.solid)], lattice=19, precision=prec, g=G,
                      graph_chunk=100) as sim:
            sim.step(STEPS)
            drho, u = sim.moments(0)
            k, m = sim.permeability(0, 0)
        e_u = rel_l2(u, ref.u, fl)
        e_k = abs(k - k_ref) / abs(k_ref)
        print(f"[err] full run {prec}: rel-L2(u) {e_u:.3e}, k rel {e_k:.3e}", flush=True)
        if prec == "f64":
            assert np.abs(drho - ref.drho).max() <= TOL_F64
            assert np.abs(u - ref.u).max() <= TOL_F64 * np.abs(ref.u).max()
            assert e_k <= 1e-12
            assert abs(m - m_ref) <= 1e-12 * geo.n_fluid
        else:
            assert e_u <= STEPS * 2.0 * 2.0 ** -24
            assert e_k <= STEPS * 2.0 * 2.0 ** -24


LOW_PHIS = [0.05, 0.1, 0.2, 0.3]


@pytest.mark.parametrize("i,phi", list(enumerate(LOW_PHIS)))
def test_low_porosity_sampled_nodes(i, phi):
    """Media of low porosity (the bench's sweep below 0.5: 256^3, r = 8, seeds
    2000 + i of that sweep's order), packed and dense layouts, each with the
    tile the autotuner picks: after 200 steps from rest, one more step is
    compared at sampled fluid nodes with the oracle's single-node update of
    the same state (the FP32 bounds of the full-size cases), and the two
    layouts give the same bits."""
    seed = 2000 + i
    geo = inputs.spheres(256, 256, 256, 8.0, phi, seed=seed)
    print(f"[case] 256^3 r=8 low porosity {phi} (achieved {geo.porosity:.4f})", flush=True)
    idx = sample_nodes(geo.solid, 20000, seed=100 + i)
    states = []
    for layout in (1, 0):
        with tau1.Sim([tau1.Sample(geo.solid)], lattice=19, precision="f32", g=(1e-5, 0.0, 0.0),
                      graph_chunk=100, layout=layout) as sim:
            sim.autotune(3)
            assert sim.info()["layout"] == layout
            sim.step(200)
            check_step(sim, 0, geo.solid, 19, "f32", (1e-5, 0.0, 0.0), idx,
                       f"porosity {phi} layout {layout} tile {sim.info()['tile']}")
            d, u = sim.moments(0)
            states.append((d.tobytes(), u.tobytes(), sim.info()["tile"]))
    # the same tile schedule family on both layouts forms the same sums
    assert states[0][0] == states[1][0] and states[0][1] == states[1][1]
