"""Pins of the two-dimensional (D2Q9) oracle of the validation workloads:
walls, moving walls (lid-driven cavity) and Zou-He pressure columns
(pressure-driven Poiseuille flow).  CPU only."""
import numpy as np
import pytest

import oracle
from test_oracle_pins import channel_closed_form, channel_steady


def random_state(nx, ny, seed, wall_frac=0.2, lid=False):
    rng = np.random.default_rng(seed)
    t = (rng.random((ny, nx)) < wall_frac).astype(np.uint8)
    if lid:
        t[0, :] = 1
        t[-1, :] = 2
    fl = t == 0
    return oracle.State2D(t, rng.uniform(-1e-3, 1e-3, (ny, nx)) * fl,
                          rng.uniform(-0.05, 0.05, (2, ny, nx)) * fl)


def test_d2q9_lattice_identities():
    """Textbook D2Q9: exact rational moments up to fourth order (c_s^2 = 1/3)."""
    from fractions import Fraction as F
    c, w, opp = oracle.lattice_2d()
    wf = [F(4, 9)] + [F(1, 9)] * 4 + [F(1, 36)] * 4
    assert all(abs(float(a) - b) == 0.0 for a, b in zip(wf, w))
    assert sum(wf) == 1
    for a in range(2):
        assert sum(wk * int(ck[a]) for wk, ck in zip(wf, c)) == 0
        for b in range(2):
            m2 = sum(wk * int(ck[a]) * int(ck[b]) for wk, ck in zip(wf, c))
            assert m2 == (F(1, 3) if a == b else 0)
    # fourth order: sum w c_a c_b c_c c_d = (d_ab d_cd + d_ac d_bd + d_ad d_bc) / 9
    for a in range(2):
        for b in range(2):
            for cc in range(2):
                for d in range(2):
                    m4 = sum(wk * int(ck[a]) * int(ck[b]) * int(ck[cc]) * int(ck[d])
                             for wk, ck in zip(wf, c))
                    want = F((a == b) * (cc == d) + (a == cc) * (b == d) + (a == d) * (b == cc), 9)
                    assert m4 == want
    for k in range(9):
        assert (c[opp[k]] == -c[k]).all()


@pytest.mark.parametrize("dims", [(12, 9), (1, 1), (5, 1), (1, 6), (7, 13)])
def test_tau1_equals_bgk_bitwise_walls_and_lid(dims):
    """Tau1 and full-population LBGK at omega = 1 with static and moving walls
    give the same bits; omega = 1.2 differs (the check can fail)."""
    nx, ny = dims
    st = random_state(nx, ny, seed=nx * 31 + ny, lid=ny > 2)
    kw = dict(g=(1e-4, -2e-5), uw=(0.1, 0.02))
    a = oracle.run_2d(st, 20, **kw)
    b = oracle.bgk_run_2d(st, 20, 1.0, **kw)
    assert a.drho.tobytes() == b.drho.tobytes()
    assert a.u.tobytes() == b.u.tobytes()
    if (st.types == 0).sum() > 1:
        c = oracle.bgk_run_2d(st, 20, 1.2, **kw)
        assert np.abs(c.u - a.u).max() > 1e-9


def test_tau1_equals_bgk_with_pressure_columns():
    """With Zou-He columns the population form rebuilds the unknown
    populations and sums them; the Tau1 form sets rho_b and u_y = 0 exactly.
    They agree to rounding."""
    st = random_state(30, 10, seed=5, wall_frac=0.1)
    st.types[0, :] = 1
    st.types[-1, :] = 1
    st.drho[st.types != 0] = 0
    st.u[:, st.types != 0] = 0
    kw = dict(xbc=1, rho_in=1.01, rho_out=0.99, g=(2e-5, 0.0))
    a = oracle.run_2d(st, 60, **kw)
    b = oracle.bgk_run_2d(st, 60, 1.0, **kw)
    assert np.abs(a.drho - b.drho).max() <= 1e-15
    assert np.abs(a.u - b.u).max() <= 1e-15 * max(np.abs(a.u).max(), 1e-3)
    fl = st.types == 0
    assert np.all(a.drho[:, 0][fl[:, 0]] == 0.01) or np.allclose(a.drho[:, 0][fl[:, 0]], 0.01,
                                                                  rtol=0, atol=1e-17)
    assert np.all(a.u[1][:, 0][fl[:, 0]] == 0.0)


def test_force_driven_channel_matches_closed_form():
    """Walls at y = 0 and y = 31, g along x: the laminar channel reduces to
    the same one-dimensional update as on the 3-D lattices (the weights
    pointing across the channel add up to 1/6 on both), so the transient
    closed form of the 3-D pin applies, and after many steps the parabola
    with the g/4 slip of halfway bounce-back."""
    t = np.zeros((32, 8), np.uint8)
    t[0] = 1
    t[-1] = 1
    st = oracle.State2D(t)
    g = 1e-6
    a = oracle.run_2d(st, 200, g=(g, 0.0))
    ref = channel_closed_form(30, g, 200)
    assert np.abs(a.u[0][1:-1] - ref[:, None]).max() <= 1e-12 * ref.max()
    b = oracle.run_2d(st, 20000, g=(g, 0.0))
    ss = channel_steady(30, g)
    assert np.abs(b.u[0][1:-1] - ss[:, None]).max() <= 1e-6 * ss.max()


def poiseuille_profile(nx, ny, rho_in, rho_out, steps):
    t = np.zeros((ny, nx), np.uint8)
    t[0] = 1
    t[-1] = 1
    a = oracle.run_2d(oracle.State2D(t), steps, xbc=1, rho_in=rho_in, rho_out=rho_out)
    xc = nx // 2
    H = ny - 2
    y = np.arange(1, ny - 1) - 0.5
    rho = 1.0 + a.drho[1:-1, xc].mean()
    dpdx = (rho_out - rho_in) / 3.0 / (nx - 1)     # p = c_s^2 rho
    g = -dpdx / rho                                  # equivalent body acceleration
    eq12 = g / (2.0 * (1.0 / 6.0)) * y * (H - y)
    return a, a.u[0, 1:-1, xc], eq12, g


def test_pressure_driven_poiseuille_eq12():
    """Constant-pressure inlet and outlet, walls at y = 0 and ny - 1: the
    steady profile is Eq. (12) (with the physical sign: flow from high to low
    pressure) plus the uniform g/4 slip of halfway bounce-back at tau = 1,
    g = -(dp/dx)/rho; the small density drop keeps compressibility effects
    below 1e-5."""
    a, u, eq12, g = poiseuille_profile(100, 12, 1.001, 0.999, 40000)
    rel = np.abs(u - (eq12 + g / 4.0)) / (eq12 + g / 4.0)
    assert rel.max() <= 1e-5
    # steady: one more step changes the velocity by less than 1e-8 of its size
    b = oracle.run_2d(a, 1, xbc=1, rho_in=1.001, rho_out=0.999)
    assert np.abs(b.u - a.u).max() <= 1e-8 * np.abs(a.u).max()
    # without the slip the mean error is the slip's share, about 0.7 % here
    mape = np.mean(np.abs(u - eq12) / eq12)
    assert 0.005 < mape < 0.009


def cavity(n, lid_u, steps):
    t = np.zeros((n, n), np.uint8)
    t[0, :] = 1          # bottom
    t[:, 0] = 1          # left
    t[:, -1] = 1         # right
    t[-1, :] = 2         # moving lid on top
    return oracle.run_2d(oracle.State2D(t), steps, uw=(lid_u, 0.0)), t


def test_lid_driven_cavity_mass_mirror_and_circulation():
    """Closed cavity with a tangentially moving lid: mass is conserved (the
    lid's momentum terms cancel pairwise), the flow for -U is the mirror image
    of the flow for +U, and the primary vortex turns with the lid."""
    n = 24
    a, t = cavity(n, 0.1, 3000)
    b, _ = cavity(n, -0.1, 3000)
    fl = t == 0
    m, _ = oracle.reduce_2d(a)
    assert abs(m - fl.sum()) <= 1e-12 * fl.sum()
    assert np.abs(b.drho - a.drho[:, ::-1]).max() <= 1e-14
    assert np.abs(b.u[0] + a.u[0][:, ::-1]).max() <= 1e-14
    assert np.abs(b.u[1] - a.u[1][:, ::-1]).max() <= 1e-14
    mid = n // 2
    assert a.u[0][n - 2, mid] > 0.01        # dragged along below the lid
    assert a.u[0][n // 3, mid] < 0.0        # return flow lower down


def two_node_2d_error(axis: int) -> float:
    """Deviation of one D2Q9 step on a periodic two-node lattice (two nodes
    along `axis`, one across) from the moment closed form of the 3-D pin:
    drho'(0) = (2/3) drho_0 + (1/3) drho_1 + rho_1 v_a^2 and the mirror
    value at node 1, j'(0) = rho_1 (v_a, v_b / 3), j'(1) = rho_1 (0, 2 v_b / 3),
    with v = 0 at node 0 and g = 0.  It rests on the D2Q9 equilibrium's
    momentum flux rho/3 I + rho v v, its third moment rho v_b / 3 and the
    c_a != 0 weights adding up to 1/3."""
    shape = (1, 2) if axis == 0 else (2, 1)     # (ny, nx)
    d0, d1 = 3.0e-3, -2.0e-3
    v1 = np.array([0.029, -0.021])
    i0 = (0, 0)
    i1 = (0, 1) if axis == 0 else (1, 0)
    drho = np.zeros(shape)
    u = np.zeros((2,) + shape)
    drho[i0], drho[i1] = d0, d1
    u[(0,) + i1], u[(1,) + i1] = v1
    out = oracle.run_2d(oracle.State2D(np.zeros(shape, np.uint8), drho, u), 1)
    rho1 = 1.0 + d1
    va2 = v1[axis] ** 2
    across = np.arange(2) != axis
    err = max(abs(out.drho[i0] - ((2.0 / 3.0) * d0 + d1 / 3.0 + rho1 * va2)),
              abs(out.drho[i1] - ((2.0 / 3.0) * d1 + d0 / 3.0 - rho1 * va2)))
    for idx, want in ((i0, rho1 * np.where(across, v1 / 3.0, v1)),
                      (i1, rho1 * np.where(across, 2.0 * v1 / 3.0, 0.0))):
        j = np.array([out.u[(b,) + idx] for b in range(2)]) * (1.0 + out.drho[idx])
        err = max(err, np.abs(j - want).max())
    return float(err)


@pytest.mark.parametrize("axis", (0, 1))
def test_two_node_second_and_third_moments_d2q9(axis):
    assert two_node_2d_error(axis) <= 1e-16


def couette_error(ny: int, lid_u: float, steps: int) -> float:
    """Plane Couette flow: a resting wall at y = 0, a lid at y = ny - 1 moving
    along x with lid_u, periodic x.  With halfway bounce-back the walls sit
    half a node beyond the outer fluid rows, a distance ny - 2 apart, and the
    steady profile is the straight line u_x(y) = lid_u (y - 1/2) / (ny - 2)
    through the no-slip wall and the lid speed, with rho = 1 and u_y = 0.  The
    moving-wall rule must hand the fluid exactly the lid's momentum; a wrong
    amplitude of its 6 w_k rho (c_k . u_w) term scales the whole line.
    Returns the largest deviation relative to lid_u."""
    t = np.zeros((ny, 3), np.uint8)
    t[0] = 1
    t[-1] = 2
    a = oracle.run_2d(oracle.State2D(t), steps, uw=(lid_u, 0.0))
    y = np.arange(1, ny - 1)
    want = lid_u * (y - 0.5) / (ny - 2)
    err = max(np.abs(a.u[0][1:-1] - want[:, None]).max(), np.abs(a.u[1]).max(),
              np.abs(a.drho).max())
    return float(err / abs(lid_u))


def test_couette_profile_of_the_moving_wall():
    # the slowest mode of 8 fluid rows decays by e in ~40 steps: 3000 steps
    # reach the steady line to FP64 rounding
    assert couette_error(10, 0.05, 3000) <= 1e-13
    assert couette_error(10, -0.02, 3000) <= 1e-13


def test_rest_state_with_all_boundaries_stays_zero():
    t = np.zeros((10, 16), np.uint8)
    t[0] = 1
    t[-1] = 2
    a = oracle.run_2d(oracle.State2D(t), 50, xbc=1, rho_in=1.0, rho_out=1.0)
    assert not a.drho.any() and not a.u.any()
