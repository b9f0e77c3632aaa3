"""Pins of the FP64 oracle against facts fixed outside the oracle itself.

Each test names what it pins.  None re-types the oracle's own formula: they
use exact lattice algebra, closed-form solutions of the update on special
flows, conservation laws, a brute-force standard LBGK with populations, and
the linear (Fourier) theory of the update.
"""
from fractions import Fraction
import itertools

import numpy as np
import pytest

import oracle
from paper_2312_14742_amd import inputs

LATTICES = (15, 19, 27)


# --------------------------------------------------------------------------
# P1: lattice tables.  Exact rational moment identities of a DdQq set with
# c_s^2 = 1/3 (isotropy up to fourth order), the opposite-direction map.
# A wrong weight, a missing or duplicated direction, a wrong opposite fails.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("q", LATTICES)
def test_lattice_identities_exact(q):
    c, w, opp = oracle.lattice(q)
    assert c.shape == (q, 3)
    # the double is the correctly rounded value of a small rational
    W = [Fraction(x).limit_denominator(1000) for x in w]
    for x, f in zip(w, W):
        assert float(f) == x
    dirs = {tuple(v) for v in c}
    assert len(dirs) == q, "duplicate direction"
    assert all(max(abs(a) for a in v) <= 1 for v in c)
    assert tuple(c[0]) == (0, 0, 0)
    n_face = sum(1 for v in c if sum(abs(a) for a in v) == 1)
    assert n_face == 6
    # zeroth .. fourth moments
    assert sum(W) == 1
    for a in range(3):
        assert sum(Wk * int(ck[a]) for Wk, ck in zip(W, c)) == 0
    for a, b in itertools.product(range(3), repeat=2):
        m2 = sum(Wk * int(ck[a]) * int(ck[b]) for Wk, ck in zip(W, c))
        assert m2 == (Fraction(1, 3) if a == b else 0)
    for a, b, g in itertools.product(range(3), repeat=3):
        assert sum(Wk * int(ck[a]) * int(ck[b]) * int(ck[g])
                   for Wk, ck in zip(W, c)) == 0
    for a, b, g, d in itertools.product(range(3), repeat=4):
        m4 = sum(Wk * int(ck[a]) * int(ck[b]) * int(ck[g]) * int(ck[d])
                 for Wk, ck in zip(W, c))
        iso = Fraction((a == b) * (g == d) + (a == g) * (b == d)
                       + (a == d) * (b == g), 9)
        assert m4 == iso
    # opposite map: involution, c_opp = -c, equal weights
    for k in range(q):
        assert opp[opp[k]] == k
        assert tuple(c[opp[k]]) == tuple(-c[k])
        assert w[opp[k]] == w[k]


# --------------------------------------------------------------------------
# P2: Tau1 equals a brute-force standard LBGK at omega = 1 bit for bit
# (Eq. (8) is Eq. (4) with tau = 1).  Pins the gather direction, bounce-back
# reconstruction, periodic wrap and where the forcing shift enters.
# --------------------------------------------------------------------------
SIZES = [(1, 1, 1), (2, 2, 2), (3, 3, 3), (5, 5, 5), (7, 7, 7), (5, 3, 7),
         (1, 4, 6), (8, 2, 3)]


@pytest.mark.parametrize("q", LATTICES)
@pytest.mark.parametrize("dims", SIZES)
def test_tau1_equals_bgk_bitwise(q, dims):
    nx, ny, nz = dims
    solid, drho, u = inputs.random_state(nx, ny, nz, seed=100 + nx * 7 + nz)
    st = oracle.State(solid, drho, u)
    g = [1.0e-5, -2.0e-5, 3.0e-6]
    a = oracle.run(q, st, g, 10)
    b = oracle.bgk_run(q, st, g, 10, omega=1.0)
    assert a.drho.tobytes() == b.drho.tobytes()
    assert a.u.tobytes() == b.u.tobytes()


def test_bgk_comparison_can_fail():
    """Control: at omega != 1 the standard LBGK is a different method."""
    solid, drho, u = inputs.random_state(5, 5, 5, seed=3)
    st = oracle.State(solid, drho, u)
    a = oracle.run(19, st, [1e-5, 0, 0], 5)
    b = oracle.bgk_run(19, st, [1e-5, 0, 0], 5, omega=1.2)
    assert np.abs(a.u - b.u).max() > 1e-8


def test_config1_channel_bitwise_bgk():
    """The 32^3 FP64 channel, 200 steps: Tau1 and LBGK agree exactly."""
    st = oracle.State(inputs.channel(32, 32, 32))
    g = [1e-6, 0.0, 0.0]
    a = oracle.run(19, st, g, 200)
    b = oracle.bgk_run(19, st, g, 200)
    assert a.drho.tobytes() == b.drho.tobytes()
    assert a.u.tobytes() == b.u.tobytes()


# --------------------------------------------------------------------------
# P3: body-forced plane channel.  With walls at z = 0 and z = N+1 the update
# is exactly the 1-D recurrence u <- S(u + g/2) + g/2, S = I + (1/6) D2 with
# bounce-back ghosts u(0) = -u(1), u(N+1) = -u(N); rho stays 1 and the
# transverse velocity stays 0 for every lattice (isotropy of the weights).
# Its eigen-solution (sine modes sin(m pi (z - 1/2) / N), eigenvalues
# 1 - (2/3) sin^2(m pi / (2N))) and its steady state, the parabola with a
# g/4 slip, are written out here independently of the oracle.
# --------------------------------------------------------------------------
def channel_closed_form(N: int, g: float, n: int) -> np.ndarray:
    z = np.arange(1, N + 1, dtype=np.float64)
    u = np.zeros(N)
    for m in range(1, N + 1):
        e = np.sin(m * np.pi * (z - 0.5) / N)
        norm = np.dot(e, e)
        proj = np.sum(e) / norm                       # projection of ones
        mu = 1.0 - (2.0 / 3.0) * np.sin(m * np.pi / (2 * N)) ** 2
        beta = (mu + 1.0) * 0.5 * g * proj
        u += beta * (1.0 - mu ** n) / (1.0 - mu) * e
    return u


def channel_steady(N: int, g: float) -> np.ndarray:
    nu = 1.0 / 6.0
    z = np.arange(1, N + 1, dtype=np.float64)
    return g / (2 * nu) * (z - 0.5) * (N + 0.5 - z) + g / 4.0


def test_channel_closed_form_reference_values():
    """Numbers of the closed form itself (32^3 channel, g = 1e-6)."""
    u1 = channel_closed_form(30, 1e-6, 1)
    assert u1[0] == pytest.approx(1e-6 * 5.0 / 6.0, rel=1e-12)
    assert u1[10] == pytest.approx(1e-6, rel=1e-12)
    u200 = channel_closed_form(30, 1e-6, 200)
    assert u200[14] == pytest.approx(1.925555e-4, rel=1e-6)
    ss = channel_steady(30, 1e-6)
    assert ss[14] == pytest.approx(6.745e-4, rel=1e-3)


@pytest.mark.parametrize("q", LATTICES)
def test_channel_transient_200_steps(q):
    nx, ny, nz = 6, 5, 32
    st = oracle.State(inputs.channel(nx, ny, nz))
    g = 1e-6
    out = oracle.run(q, st, [g, 0.0, 0.0], 200)
    ref = channel_closed_form(nz - 2, g, 200)
    fl = out.u[0][1:-1]                               # (N, ny, nx)
    assert np.abs(fl - ref[:, None, None]).max() <= 1e-12 * np.abs(ref).max()
    assert np.abs(out.drho).max() <= 1e-15
    assert np.abs(out.u[1]).max() <= 1e-18
    assert np.abs(out.u[2]).max() <= 1e-18
    # walls report zero
    assert not out.u[:, 0].any() and not out.u[:, -1].any()


def test_channel_config1_center_value():
    """BASELINE config 1 geometry (32^3, D3Q19): centre after 200 steps."""
    st = oracle.State(inputs.channel(32, 32, 32))
    out = oracle.run(19, st, [1e-6, 0, 0], 200)
    ref = channel_closed_form(30, 1e-6, 200)
    assert np.abs(out.u[0][1:-1, 7, 9] - ref).max() <= 1e-12 * ref.max()


@pytest.mark.parametrize("q", LATTICES)
def test_channel_steady_parabola_with_slip(q):
    """20000 steps on a 1x1x32 column reach the discrete steady state."""
    g = 1e-6
    st = oracle.State(inputs.channel(1, 1, 32))
    out = oracle.run(q, st, [g, 0.0, 0.0], 20000)
    ref = channel_steady(30, g)
    got = out.u[0][1:-1, 0, 0]
    assert np.abs(got - ref).max() <= 1e-11 * ref.max()
    # Darcy permeability of the discrete steady channel: (N^3 + N)/(12 (N+2))
    mass, k = oracle.reduce(out, 0, g)
    assert k == pytest.approx((30 ** 3 + 30) / (12 * 32), rel=1e-11)
    assert k == pytest.approx(70.390625, rel=1e-11)
    assert mass == pytest.approx(30.0, abs=1e-13)


def test_single_layer_channel_steady():
    """N = 1: the steady velocity of a one-node-wide channel is exactly g."""
    g = 1e-6
    st = oracle.State(inputs.channel(1, 1, 3))
    out = oracle.run(19, st, [g, 0.0, 0.0], 200)
    assert out.u[0][1, 0, 0] == pytest.approx(g, rel=1e-12)


# --------------------------------------------------------------------------
# P4: periodic shear wave.  u_x = U sin(2 pi m z / nz) with rho = 1 decays
# exactly as U mu^n, mu = 1 - (2/3) sin^2(pi m / nz), any amplitude.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("q", LATTICES)
@pytest.mark.parametrize("mode", [1, 3])
def test_shear_wave_decay(q, mode):
    nx, ny, nz = 4, 3, 24
    U = 1e-3
    solid, drho, u = inputs.shear_wave(nx, ny, nz, U, mode)
    st = oracle.State(solid, drho, u)
    n = 37
    out = oracle.run(q, st, [0, 0, 0], n)
    mu = 1.0 - (2.0 / 3.0) * np.sin(np.pi * mode / nz) ** 2
    z = np.arange(nz)
    ref = U * mu ** n * np.sin(2 * np.pi * mode * z / nz)
    assert np.abs(out.u[0] - ref[:, None, None]).max() <= 1e-15
    assert np.abs(out.drho).max() <= 1e-15
    assert np.abs(out.u[1:]).max() <= 1e-18


# --------------------------------------------------------------------------
# P5: uniform flow under a body force accelerates as u_n = U + n g.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("q", LATTICES)
def test_uniform_flow_acceleration(q):
    nx, ny, nz = 3, 4, 5
    U = np.array([2e-3, -1e-3, 5e-4])
    g = np.array([1e-5, 2e-5, -3e-6])
    u = np.broadcast_to(U[:, None, None, None], (3, nz, ny, nx)).copy()
    st = oracle.State(np.zeros((nz, ny, nx), np.uint8), None, u)
    n = 50
    out = oracle.run(q, st, g, n)
    ref = U + n * g
    for a in range(3):
        assert np.abs(out.u[a] - ref[a]).max() <= 1e-16
    assert np.abs(out.drho).max() <= 1e-15


# --------------------------------------------------------------------------
# P6: the rest state is a fixed point, bit for bit, in any geometry.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("q", LATTICES)
def test_rest_state_exact(q):
    geo = inputs.spheres(20, 18, 16, 3.0, 0.6, seed=9)
    st = oracle.State(geo.solid)
    out = oracle.run(q, st, [0, 0, 0], 30)
    assert not out.drho.any() and not out.u.any()


# --------------------------------------------------------------------------
# P7: mass.  Every population is delivered once (streamed or bounced back)
# and the equilibrium's zeroth moment is rho, so total mass is conserved.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("q", LATTICES)
def test_mass_conservation_porous(q):
    geo = inputs.spheres(24, 20, 16, 3.5, 0.65, seed=21)
    rng = np.random.default_rng(5)
    drho = rng.uniform(-1e-3, 1e-3, geo.solid.shape)
    u = rng.uniform(-0.02, 0.02, (3,) + geo.solid.shape)
    st = oracle.State(geo.solid, drho, u)
    st = oracle.run(q, st, [0, 0, 0], 0)          # zero the solids
    m0, _ = oracle.reduce(st, 0, 1.0)
    out = oracle.run(q, st, [1e-5, 0, 0], 2000)
    m1, _ = oracle.reduce(out, 0, 1.0)
    assert abs(m1 - m0) / m0 <= 1e-13


# --------------------------------------------------------------------------
# P8: linear theory.  A small-amplitude Fourier mode (drho, v) of wavevector
# kappa is advanced by M(kappa) = sum_k w_k exp(-i kappa.c_k)
# [[1, 3 c_k^T], [c_k, 3 c_k c_k^T]] per step, up to O(amplitude^2).  This
# checks every direction and weight, sound as well as shear.
# --------------------------------------------------------------------------
def _linear_matrix(c, w, kappa):
    M = np.zeros((4, 4), dtype=complex)
    for ck, wk in zip(c.astype(float), w):
        ph = wk * np.exp(-1j * np.dot(kappa, ck))
        B = np.zeros((4, 4))
        B[0, 0] = 1.0
        B[0, 1:] = 3.0 * ck
        B[1:, 0] = ck
        B[1:, 1:] = 3.0 * np.outer(ck, ck)
        M += ph * B
    return M


@pytest.mark.parametrize("q", LATTICES)
def test_linear_fourier_mode(q):
    c, w, _ = oracle.lattice(q)
    nx, ny, nz = 8, 6, 5
    m = np.array([1, 2, 1])
    kappa = 2 * np.pi * m / np.array([nx, ny, nz])
    rng = np.random.default_rng(11)
    amp = 1e-9 * (rng.normal(size=4) + 1j * rng.normal(size=4))
    Z, Y, X = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx),
                          indexing="ij")
    phase = np.exp(1j * (kappa[0] * X + kappa[1] * Y + kappa[2] * Z))
    field = np.real(amp[:, None, None, None] * phase[None])
    st = oracle.State(np.zeros((nz, ny, nx), np.uint8), field[0], field[1:])
    n = 6
    out = oracle.run(q, st, [0, 0, 0], n)
    Mn = np.linalg.matrix_power(_linear_matrix(c, w, kappa), n)
    pred = np.real((Mn @ amp)[:, None, None, None] * phase[None])
    got = np.concatenate([out.drho[None], out.u])
    scale = np.abs(pred).max()
    assert np.abs(got - pred).max() <= 1e-6 * scale


# --------------------------------------------------------------------------
# P9: second and third moments of the equilibrium (Eq. (3), Section 2).  On
# a periodic lattice of two nodes along axis a (one node across the other
# axes), node 0 receives its c_a = 0 directions from itself and its
# c_a = +-1 directions from node 1, and node 1 the other way round.  The
# equilibrium of Eq. (3) has the momentum-flux tensor sum_k c c f_k^eq =
# rho/3 I + rho v v and the third moment sum_k c_a^2 c_b f_k^eq = rho v_b / 3
# (b != a, from fourth-order isotropy), and the c_a != 0 weights add up to
# 1/3.  With v = 0 at node 0 and g = 0, one step therefore gives exactly
#   drho'(0) = (2/3) drho_0 + (1/3) drho_1 + rho_1 v_a^2,
#   drho'(1) = (2/3) drho_1 + (1/3) drho_0 - rho_1 v_a^2,
#   j'(0) = rho_1 (v_a along a, v_b / 3 across),
#   j'(1) = rho_1 (0 along a, 2 v_b / 3 across).
# A rescaled or dropped O(u^2) term moves rho_1 v_a^2; a wrong linear term
# or weight moves j'.  These flows cancel nothing quadratic, unlike the
# channel, shear-wave, uniform-flow and linear-mode pins.
# --------------------------------------------------------------------------
def two_node_moments_error(q: int, axis: int) -> float:
    """Largest deviation of one oracle step from the closed form above."""
    shape = [1, 1, 1]                       # (nz, ny, nx)
    shape[2 - axis] = 2
    d0, d1 = 3.0e-3, -2.0e-3
    v1 = np.array([0.031, -0.017, 0.023])
    drho = np.zeros(shape)
    u = np.zeros((3,) + tuple(shape))
    idx0 = (0, 0, 0)
    idx1 = tuple(1 if i == 2 - axis else 0 for i in range(3))
    drho[idx0], drho[idx1] = d0, d1
    for b in range(3):
        u[(b,) + idx1] = v1[b]
    st = oracle.State(np.zeros(shape, np.uint8), drho, u)
    out = oracle.run(q, st, [0.0, 0.0, 0.0], 1)
    rho1 = 1.0 + d1
    va2 = v1[axis] ** 2
    want_d0 = (2.0 / 3.0) * d0 + d1 / 3.0 + rho1 * va2
    want_d1 = (2.0 / 3.0) * d1 + d0 / 3.0 - rho1 * va2
    across = np.arange(3) != axis
    want_j0 = rho1 * np.where(across, v1 / 3.0, v1)
    want_j1 = rho1 * np.where(across, 2.0 * v1 / 3.0, 0.0)
    err = max(abs(out.drho[idx0] - want_d0), abs(out.drho[idx1] - want_d1))
    for idx, want in ((idx0, want_j0), (idx1, want_j1)):
        j = np.array([out.u[(b,) + idx] for b in range(3)]) * (1.0 + out.drho[idx])
        err = max(err, np.abs(j - want).max())
    return float(err)


@pytest.mark.parametrize("q", LATTICES)
@pytest.mark.parametrize("axis", (0, 1, 2))
def test_two_node_second_and_third_moments(q, axis):
    # terms are O(1e-3); FP64 rounding of one step is O(1e-18)
    assert two_node_moments_error(q, axis) <= 1e-16


# --------------------------------------------------------------------------
# Consistency of the two oracle forms (rho vs drho storage).
# --------------------------------------------------------------------------
@pytest.mark.parametrize("q", LATTICES)
def test_rhoform_agrees_with_drho_form(q):
    solid, drho, u = inputs.random_state(6, 5, 7, seed=44)
    st = oracle.State(solid, drho, u)
    a = oracle.run(q, st, [1e-5, 0, 0], 20)
    b = oracle.run_rhoform(q, st, [1e-5, 0, 0], 20)
    assert np.abs(a.drho - b.drho).max() <= 1e-10
    assert np.abs(a.u - b.u).max() <= 1e-10


def test_step_nodes_matches_run():
    solid, drho, u = inputs.random_state(7, 6, 5, seed=8)
    st = oracle.State(solid, drho, u)
    g = [2e-5, 0, -1e-5]
    full = oracle.run(19, st, g, 1)
    idx = np.arange(7 * 6 * 5)
    one = oracle.step_nodes(19, st, g, idx)
    assert np.array_equal(one[:, 0], full.drho.ravel())
    for a in range(3):
        assert np.array_equal(one[:, 1 + a], full.u[a].ravel())
