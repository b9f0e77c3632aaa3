"""The D2Q9 validation path on the GPU against the 2-D oracle: walls, moving
lid, Zou-He pressure columns; FP64 within 1e-12, FP32 within the storage
bounds; pressure-driven Poiseuille against Eq. (12) and the lid-driven
cavity's invariants."""
import numpy as np
import pytest

import oracle
from paper_2312_14742_amd import tau1

pytestmark = pytest.mark.gpu

EPS32 = 2.0 ** -24


def gpu_run(st, steps, prec="f64", graph_chunk=0, **bc):
    ny, nx = st.types.shape
    u3 = np.zeros((3, 1, ny, nx))
    u3[:2, 0] = st.u
    g = bc.pop("g", (0.0, 0.0))
    sim = tau1.Sim([tau1.Sample(st.types[None], st.drho[None], u3)], lattice=9, precision=prec,
                   g=(g[0], g[1], 0.0), graph_chunk=graph_chunk, **bc)
    assert sim.info()["kernel"] == 2
    sim.step(steps)
    d, u = sim.moments(0)
    return sim, d[0], u[:2, 0]


def oracle_run(st, steps, **bc):
    kw = dict(bc)
    if "wall_u" in kw:
        kw["uw"] = kw.pop("wall_u")[:2]
    if "x_boundary" in kw:
        kw["xbc"] = kw.pop("x_boundary")
    return oracle.run_2d(st, steps, **kw)


def random_state(nx, ny, seed, wall_frac=0.2, lid=False, pressure=False):
    rng = np.random.default_rng(seed)
    t = (rng.random((ny, nx)) < wall_frac).astype(np.uint8)
    if lid:
        t[0, :] = 1
        t[-1, :] = 2
    if pressure:
        t[0, :] = 1
        t[-1, :] = 1
    fl = t == 0
    return oracle.State2D(t, rng.uniform(-1e-3, 1e-3, (ny, nx)) * fl,
                          rng.uniform(-0.05, 0.05, (2, ny, nx)) * fl)


CASES = {
    "periodic_walls_lid": (dict(nx=37, ny=23, lid=True),
                           dict(g=(1e-4, -2e-5), wall_u=(0.1, 0.02, 0.0))),
    "pressure_obstacles": (dict(nx=64, ny=18, pressure=True, wall_frac=0.1),
                           dict(x_boundary=1, rho_in=1.01, rho_out=0.99)),
    "pressure_forced": (dict(nx=3, ny=5, pressure=True, wall_frac=0.0),
                        dict(x_boundary=1, rho_in=1.002, rho_out=0.998, g=(1e-5, 0.0))),
    "one_row": (dict(nx=16, ny=1, wall_frac=0.1), dict(g=(1e-5, 0.0))),
    "one_column": (dict(nx=1, ny=16, wall_frac=0.1), dict(g=(0.0, 1e-5))),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_d2q9_f64_matches_oracle(name):
    shape, bc = CASES[name]
    st = random_state(seed=len(name), **shape)
    print(f"[case] d2q9 f64 {name}", flush=True)
    sim, d, u = gpu_run(st, 30, **dict(bc))
    ref = oracle_run(st, 30, **dict(bc))
    fl = st.types == 0
    umax = max(np.abs(ref.u).max(), 1e-300)
    assert np.abs(d - ref.drho)[fl].max() <= 1e-12
    assert np.abs(u - ref.u).max() <= 1e-12 * umax
    assert np.all(d[~fl] == 0) and np.all(u[:, ~fl] == 0)
    sim.close()


@pytest.mark.parametrize("name", sorted(CASES))
def test_d2q9_f32_within_storage_bounds(name):
    shape, bc = CASES[name]
    st = random_state(seed=100 + len(name), **shape)
    print(f"[case] d2q9 f32 {name}", flush=True)
    sim, d, u = gpu_run(st, 5, prec="f32", **dict(bc))
    ref = oracle_run(st, 5, **dict(bc))
    fl = st.types == 0
    umax = np.abs(ref.u).max()
    assert np.abs(d - ref.drho)[fl].max() <= (2 * EPS32 + 16 * EPS32) * max(umax, 1e-2)
    num = np.sqrt(np.sum((u - ref.u)[:, fl] ** 2))
    assert num <= 8 * EPS32 * np.sqrt(np.sum(ref.u[:, fl] ** 2))
    sim.close()


def test_d2q9_graph_equals_single_launches():
    st = random_state(40, 20, seed=7, lid=True)
    bc = dict(wall_u=(0.05, 0.0, 0.0), g=(1e-5, 0.0))
    a, da, ua = gpu_run(st, 300, graph_chunk=100, **dict(bc))
    b, db, ub = gpu_run(st, 300, graph_chunk=1000, **dict(bc))
    assert da.tobytes() == db.tobytes() and ua.tobytes() == ub.tobytes()
    a.close()
    b.close()


def test_pressure_driven_poiseuille_on_gpu():
    """Zou-He inlet/outlet, walls at y = 0 and ny - 1, 40000 steps in FP64:
    the oracle's state to 1e-12 and Eq. (12) plus the g/4 halfway-wall slip to
    1e-5 at the middle column."""
    nx, ny = 100, 12
    t = np.zeros((ny, nx), np.uint8)
    t[0] = 1
    t[-1] = 1
    st = oracle.State2D(t)
    bc = dict(x_boundary=1, rho_in=1.001, rho_out=0.999)
    print("[case] d2q9 Poiseuille 100x12", flush=True)
    sim, d, u = gpu_run(st, 40000, graph_chunk=100, **dict(bc))
    ref = oracle_run(st, 40000, **dict(bc))
    assert np.abs(u - ref.u).max() <= 1e-12 * np.abs(ref.u).max()
    xc, H = nx // 2, ny - 2
    y = np.arange(1, ny - 1) - 0.5
    rho = 1.0 + d[1:-1, xc].mean()
    g = -((0.999 - 1.001) / 3.0 / (nx - 1)) / rho
    want = g / (2.0 / 6.0) * y * (H - y) + g / 4.0
    assert np.abs(u[0, 1:-1, xc] - want).max() <= 1e-5 * want.max()
    sim.close()


def test_lid_driven_cavity_on_gpu():
    """Closed cavity, lid moving at U = 0.1: the oracle's state to 1e-12 after
    3000 FP64 steps, FP64 mass conserved, and the FP32 flow for -U the mirror
    image of the flow for +U."""
    n = 24
    t = np.zeros((n, n), np.uint8)
    t[0, :] = 1
    t[:, 0] = 1
    t[:, -1] = 1
    t[-1, :] = 2
    st = oracle.State2D(t)
    print("[case] d2q9 cavity 24x24", flush=True)
    sim, d, u = gpu_run(st, 3000, graph_chunk=100, wall_u=(0.1, 0.0, 0.0))
    ref = oracle_run(st, 3000, wall_u=(0.1, 0.0, 0.0))
    assert np.abs(u - ref.u).max() <= 1e-12 * np.abs(ref.u).max()
    _, mass = sim.permeability(0, 0, with_k=False)
    assert abs(mass - (t == 0).sum()) <= 1e-12 * (t == 0).sum()
    sim.close()
    a, da, ua = gpu_run(st, 2000, prec="f32", graph_chunk=100, wall_u=(0.1, 0.0, 0.0))
    b, db, ub = gpu_run(st, 2000, prec="f32", graph_chunk=100, wall_u=(-0.1, 0.0, 0.0))
    scale = np.abs(ua).max()
    assert np.abs(db - da[:, ::-1]).max() <= 1e-6 * scale
    assert np.abs(ub[0] + ua[0][:, ::-1]).max() <= 1e-5 * scale
    assert np.abs(ub[1] - ua[1][:, ::-1]).max() <= 1e-5 * scale
    a.close()
    b.close()


def test_d2q9_batch_equals_solo_bitwise():
    """Several 2-D samples of different sizes in one context (one launch per
    step for all) give each sample's solo bits, with pressure columns."""
    states = [random_state(40, 12, seed=21, pressure=True, wall_frac=0.05),
              random_state(17, 9, seed=22, pressure=True, wall_frac=0.1),
              random_state(64, 30, seed=23, pressure=True, wall_frac=0.0)]
    bc = dict(x_boundary=1, rho_in=1.004, rho_out=0.998)
    samples = []
    for st in states:
        ny, nx = st.types.shape
        u3 = np.zeros((3, 1, ny, nx))
        u3[:2, 0] = st.u
        samples.append(tau1.Sample(st.types[None], st.drho[None], u3))
    sim = tau1.Sim(samples, lattice=9, precision="f32", graph_chunk=50, **bc)
    sim.step(120)
    for i, st in enumerate(states):
        d, u = sim.moments(i)
        solo, ds, us = gpu_run(st, 120, prec="f32", graph_chunk=50, **dict(bc))
        assert d[0].tobytes() == ds.tobytes() and u[:2, 0].tobytes() == us.tobytes(), i
        solo.close()
    sim.close()
