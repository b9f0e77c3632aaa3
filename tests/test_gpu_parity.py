"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Every case runs the same seeded inputs through libtau1.so on the GPU and
through the oracle on the CPU and compares element by element.
"""
import numpy as np
import pytest

import oracle
from paper_2312_14742_amd import inputs, tau1

from gpu_helpers import (TOL_F64, assert_f64_parity, reduced_errors, run_gpu,
                         run_oracle)

pytestmark = pytest.mark.gpu

LATTICES = (15, 19, 27)

# Normwise bounds of the reduced-precision modes against the FP64 oracle.
# eps is the unit roundoff of the storage format (2^-24, 2^-11, 2^-8): every
# step rounds each stored value once.  Velocity: relative L2 over fluid nodes
# <= 8 eps.  Density: |drho - drho_ref| <= (2 eps + 16 eps32) U, U the largest
# initial velocity component: the new density is a weighted sum of neighbour
# velocities, so velocity rounding in storage (eps) and in the FP32 arithmetic
# (eps32 = 2^-24, some tens of operations per node) dominates it.
UNIT_ROUNDOFF = {"f32": 2.0 ** -24, "f16": 2.0 ** -11, "bf16": 2.0 ** -8}


def reduced_bounds(prec, u_scale):
    eps = UNIT_ROUNDOFF[prec]
    return {"drho_abs": (2.0 * eps + 16.0 * 2.0 ** -24) * u_scale,
            "u_rel_l2": 8.0 * eps}


def _config1():
    return inputs.channel(32, 32, 32)


@pytest.mark.parametrize("kernel", [0])
def test_config1_channel_f64(kernel):
    """32^3 channel, D3Q19, FP64, 200 steps: GPU vs oracle at 1e-12."""
    solid = _config1()
    g = (1e-6, 0.0, 0.0)
    print(f"[case] config1 f64 kernel={kernel}", flush=True)
    sim, out = run_gpu([(solid,)], 19, "f64", g, 200, kernel=kernel)
    ref = run_oracle(19, solid, None, None, g, 200)
    assert_f64_parity(out[0], ref, solid)
    k, mass = sim.permeability(0, 0)
    mref, kref = oracle.reduce(ref, 0, g[0])
    assert abs(k - kref) <= TOL_F64 * abs(kref)
    assert abs(mass - mref) <= 1e-12 * mref
    sim.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("q", LATTICES)
def test_config1_channel_steady_state(q, prec):
    """The 32^3 channel after 20000 steps against the mathematics, not the
    oracle: the discrete steady profile of halfway bounce-back at tau = 1
    (the Poiseuille parabola of the 30 fluid layers plus the uniform slip
    g/4) and its Darcy permeability (N^3 + N) / (12 (N + 2)) = 70.390625 for
    N = 30.  FP64 to 1e-11 relative (the oracle's own pin); FP32 within
    20000 x 2 x 2^-24 (linear growth of FP32 rounding)."""
    solid = _config1()
    g = 1e-6
    steps = 20000
    print(f"[case] config1 steady q={q} {prec}", flush=True)
    sim, out = run_gpu([(solid,)], q, prec, (g, 0.0, 0.0), steps, graph_chunk=100)
    k, mass = sim.permeability(0, 0)
    sim.close()
    z = np.arange(1, 31, dtype=np.float64)
    ref = g / (2.0 / 6.0) * (z - 0.5) * (30.5 - z) + g / 4.0
    u = out[0][1]
    tol = 1e-11 if prec == "f64" else steps * 2.0 * 2.0 ** -24
    assert np.abs(u[0][1:-1] - ref[:, None, None]).max() <= tol * ref.max()
    assert np.abs(u[1:]).max() <= tol * ref.max()
    assert abs(k - 70.390625) <= tol * 70.390625
    assert abs(mass - 30.0 * 32 * 32) <= (1e-12 if prec == "f64" else 1e-9) * mass


SMALL = [(1, 1, 1), (2, 2, 2), (3, 3, 3), (5, 5, 5), (7, 7, 7), (5, 3, 7),
         (1, 4, 6), (33, 9, 4), (70, 37, 5)]


@pytest.mark.parametrize("q", LATTICES)
@pytest.mark.parametrize("dims", SMALL)
def test_small_random_f64(q, dims):
    nx, ny, nz = dims
    solid, drho, u = inputs.random_state(nx, ny, nz, seed=1000 + nx + 7 * ny + 31 * nz)
    g = (1e-5, -2e-5, 3e-6)
    print(f"[case] small f64 q={q} dims={dims}", flush=True)
    sim, out = run_gpu([(solid, drho, u)], q, "f64", g, 10, kernel=0)
    ref = run_oracle(q, solid, drho, u, g, 10)
    assert_f64_parity(out[0], ref, solid)
    sim.close()


@pytest.mark.parametrize("q", LATTICES)
@pytest.mark.parametrize("prec", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("dims", [(5, 3, 7), (33, 9, 4), (70, 37, 5)])
def test_small_random_reduced(q, prec, dims):
    nx, ny, nz = dims
    solid, drho, u = inputs.random_state(nx, ny, nz, seed=2000 + nx + 7 * ny + 31 * nz)
    g = (1e-5, -2e-5, 3e-6)
    print(f"[case] small {prec} q={q} dims={dims}", flush=True)
    sim, out = run_gpu([(solid, drho, u)], q, prec, g, 10, kernel=0)   # default F16 scales
    ref = run_oracle(q, solid, drho, u, g, 10)
    err = reduced_errors(out[0], ref, solid)
    print(f"[err] {prec} q={q} {dims} {err}", flush=True)
    bounds = reduced_bounds(prec, np.abs(u).max())
    for key, bound in bounds.items():
        assert err[key] <= bound, (key, err[key], bound)
    sim.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("dims", [(1 << 20, 1, 1), (1, 1 << 20, 1), (1, 1, 1 << 20)])
def test_longest_extent(prec, dims):
    """The largest extent one axis may have (2^20 nodes), along each axis."""
    nx, ny, nz = dims
    solid, drho, u = inputs.random_state(nx, ny, nz, seed=4100 + (nx > 1) + 2 * (ny > 1))
    g = (1e-5, -2e-5, 3e-6)
    print(f"[case] longest extent {prec} dims={dims}", flush=True)
    sim, out = run_gpu([(solid, drho, u)], 19, prec, g, 4)
    sim.close()
    ref = run_oracle(19, solid, drho, u, g, 4)
    if prec == "f64":
        assert_f64_parity(out[0], ref, solid)
    else:
        err = reduced_errors(out[0], ref, solid)
        print(f"[err] {prec} {dims} {err}", flush=True)
        for key, bound in reduced_bounds(prec, np.abs(u).max()).items():
            assert err[key] <= bound, (key, err[key], bound)


def test_graph_replay_equals_single_launches():
    solid, drho, u = inputs.random_state(20, 12, 9, seed=77)
    g = (1e-5, 0, 0)
    print("[case] graph replay", flush=True)
    a, outa = run_gpu([(solid, drho, u)], 19, "f32", g, 13, kernel=0, graph_chunk=4)
    b, outb = run_gpu([(solid, drho, u)], 19, "f32", g, 13, kernel=0, graph_chunk=1000)
    assert outa[0][0].tobytes() == outb[0][0].tobytes()
    assert outa[0][1].tobytes() == outb[0][1].tobytes()
    a.close()
    b.close()


def test_batched_equals_solo_bitwise():
    samples = []
    for i, dims in enumerate([(9, 7, 5), (16, 16, 16), (3, 4, 5), (40, 8, 6)]):
        samples.append(inputs.random_state(*dims, seed=300 + i))
    g = (1e-5, 2e-6, 0)
    print("[case] batched vs solo", flush=True)
    sim, outs = run_gpu(samples, 19, "f32", g, 12, kernel=0)
    for i, s in enumerate(samples):
        solo, o = run_gpu([s], 19, "f32", g, 12, kernel=0)
        assert outs[i][0].tobytes() == o[0][0].tobytes()
        assert outs[i][1].tobytes() == o[0][1].tobytes()
        solo.close()
    sim.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_reductions_vs_oracle(prec):
    geo = inputs.spheres(24, 20, 16, 3.5, 0.65, seed=21)
    g = (1e-5, 0, 0)
    print(f"[case] reductions {prec}", flush=True)
    sim, out = run_gpu([(geo.solid,)], 19, prec, g, 50, kernel=0)
    ref = run_oracle(19, geo.solid, None, None, g, 50)
    mref, kref = oracle.reduce(ref, 0, g[0])
    k, m = sim.permeability(0, 0)
    tol = TOL_F64 if prec == "f64" else 1e-5
    assert abs(k - kref) <= tol * abs(kref), (k, kref)
    assert abs(m - mref) <= 1e-12 * mref if prec == "f64" else abs(m - mref) <= 1e-6 * mref
    sim.close()


@pytest.mark.parametrize("kernel,prec", [(0, "f64"), (0, "f32"), (1, "f32"), (1, "bf16")])
def test_runs_are_deterministic(kernel, prec):
    """Two contexts over the same inputs give the same bits: state, mass and
    permeability (no atomics in the step; the reductions use a fixed order of
    lane shuffles and wave sums)."""
    geo = inputs.spheres(64, 48, 40, 5.0, 0.6, seed=31)
    g = (1e-5, 2e-6, 0.0)
    print(f"[case] determinism kernel={kernel} {prec}", flush=True)
    res = []
    for _ in range(2):
        with tau1.Sim([tau1.Sample(geo.solid)], lattice=19, precision=prec, g=g,
                      kernel=kernel, graph_chunk=10) as sim:
            sim.step(37)
            d, u = sim.moments(0)
            k, m = sim.permeability(0, 0)
            res.append((d.tobytes(), u.tobytes(), np.float64(k).tobytes(),
                        np.float64(m).tobytes()))
    assert res[0] == res[1]


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_moments_physical_density(prec):
    """tau1_moments reads back the physical density rho = 1 + (rho - 1),
    formed in FP64 (1 at solid nodes), beside the same velocity as
    tau1_moments_drho; in FP64 mode rho matches the oracle's 1 + drho."""
    solid, drho, u = inputs.random_state(33, 9, 4, seed=91)
    g = (1e-5, -2e-5, 3e-6)
    print(f"[case] physical density {prec}", flush=True)
    with tau1.Sim([tau1.Sample(solid, drho, u)], lattice=19, precision=prec, g=g) as sim:
        sim.step(3)
        d, u1 = sim.moments(0)
        r, u2 = sim.rho_u(0)
    assert np.array_equal(r, 1.0 + d)
    assert np.array_equal(u1, u2)
    assert (r[solid != 0] == 1.0).all()
    if prec == "f64":
        ref = run_oracle(19, solid, drho, u, g, 3)
        assert np.abs(r - (1.0 + ref.drho)).max() <= TOL_F64
