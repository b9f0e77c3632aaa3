"""Planted mistakes in the 2-D oracle must be caught by its pins.

As for the 3-D oracle: each case copies ``oracle/tau1_oracle_2d.c``, plants
one plausible mistake by a text substitution (in the Tau1 form, in the
population form, or consistently in both, where only the physical pins can
see it), compiles the copy and runs a fast subset of the 2-D pins against
it.  The real oracle is never modified."""
import os
import subprocess

import numpy as np
import pytest

import oracle

SRC = os.path.join(os.path.dirname(oracle.__file__), "tau1_oracle_2d.c")

# name: list of (old, new, count) substitutions; count -1 = every occurrence
MUTANTS = {
    "moving_wall_sign_tau1": [("f += 6.0 * W9[k]", "f -= 6.0 * W9[k]", 1)],
    "moving_wall_sign_both": [("f += 6.0 * W9[k]", "f -= 6.0 * W9[k]", 1),
                              ("fi[k] += 6.0 * W9[k]", "fi[k] -= 6.0 * W9[k]", 1)],
    "moving_wall_neighbour_density": [("f += 6.0 * W9[k] * (1.0 + dr[i])",
                                       "f += 6.0 * W9[k] * (1.0 + dr[s])", 1)],
    "bounce_back_same_direction": [("double f = feqm(opp9(k), dr[i]", "double f = feqm(k, dr[i]", 1)],
    "inlet_single_weight_tau1": [("s = (f[0] + f[3] + f[4]) + 2.0 * ((f[2] + f[6]) + f[8]);",
                                  "s = (f[0] + f[3] + f[4]) + 1.0 * ((f[2] + f[6]) + f[8]);", 1)],
    "outlet_sign_tau1": [("out[1] = (s - db) / (1.0 + db)", "out[1] = (db - s) / (1.0 + db)", 1)],
    "inlet_wrong_diagonal_both": [("((f[2] + f[6]) + f[8])", "((f[2] + f[5]) + f[8])", 1),
                                  ("((fi[2] + fi[6]) + fi[8])", "((fi[2] + fi[5]) + fi[8])", 1)],
    "outlet_density_both": [("const double db = inlet ? G->din : G->dout;",
                             "const double db = inlet ? G->din : G->din;", 1),
                            ("const double db = inlet ? rho_in - 1.0 : rho_out - 1.0;",
                             "const double db = inlet ? rho_in - 1.0 : rho_in - 1.0;", 1)],
    "diagonal_weight": [("1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};",
                         "1.0 / 36.0, 1.0 / 36.0, 1.0 / 30.0, 1.0 / 36.0};", 1)],
    "opposite_map": [("(k % 2 ? k + 1 : k - 1)", "(k % 2 ? k : k - 1)", 1)],
    "zou_he_rebuild_bgk": [("fi[1] = fi[2] + (2.0 / 3.0) * ru;", "fi[1] = fi[2] + (1.0 / 3.0) * ru;", 1)],
    "pull_from_wrong_side": [("long sx = x - C9[k][0];", "long sx = x + C9[k][0];", 1)],
    # amplitude of the moving wall's momentum, in both forms (only the
    # Couette profile sees it)
    "moving_wall_amplitude_both": [("f += 6.0 * W9[k]", "f += 3.0 * W9[k]", 1),
                                   ("fi[k] += 6.0 * W9[k]", "fi[k] += 3.0 * W9[k]", 1)],
    # the O(u^2) part of Eq. (3), shared by both forms
    "quadratic_doubled": [("(4.5 * cu) * cu) - 1.5 * vv;", "(9.0 * cu) * cu) - 3.0 * vv;", 1)],
    "quadratic_dropped": [("(3.0 * cu + (4.5 * cu) * cu) - 1.5 * vv;", "(3.0 * cu);", 1)],
}


def _quick_pins():
    failed = []

    def check(name, fn):
        try:
            ok = fn()
        except Exception:                       # noqa: BLE001 - any crash counts
            ok = False
        if not ok:
            failed.append(name)

    def lattice_ok():
        c, w, opp = oracle.lattice_2d()
        m2 = (w[:, None, None] * c[:, :, None] * c[:, None, :]).sum(0)
        return (abs(w.sum() - 1) <= 1e-15 and np.abs(m2 - np.eye(2) / 3).max() <= 1e-15
                and all(tuple(c[opp[k]]) == tuple(-c[k]) for k in range(9)))

    def bitwise_ok():
        rng = np.random.default_rng(3)
        t = (rng.random((9, 12)) < 0.2).astype(np.uint8)
        t[0] = 1
        t[-1] = 2
        fl = t == 0
        st = oracle.State2D(t, rng.uniform(-1e-3, 1e-3, t.shape) * fl,
                            rng.uniform(-0.05, 0.05, (2,) + t.shape) * fl)
        kw = dict(g=(1e-4, -2e-5), uw=(0.1, 0.02))
        a = oracle.run_2d(st, 10, **kw)
        b = oracle.bgk_run_2d(st, 10, 1.0, **kw)
        return a.u.tobytes() == b.u.tobytes() and a.drho.tobytes() == b.drho.tobytes()

    def pressure_ok():
        t = np.zeros((8, 20), np.uint8)
        t[0] = 1
        t[-1] = 1
        kw = dict(xbc=1, rho_in=1.01, rho_out=0.99)
        a = oracle.run_2d(oracle.State2D(t), 30, **kw)
        b = oracle.bgk_run_2d(oracle.State2D(t), 30, 1.0, **kw)
        return np.abs(a.u - b.u).max() <= 1e-15 and np.abs(a.drho - b.drho).max() <= 1e-15

    def channel_ok():
        from test_oracle_pins import channel_closed_form
        t = np.zeros((32, 4), np.uint8)
        t[0] = 1
        t[-1] = 1
        a = oracle.run_2d(oracle.State2D(t), 200, g=(1e-6, 0.0))
        ref = channel_closed_form(30, 1e-6, 200)
        return np.abs(a.u[0][1:-1] - ref[:, None]).max() <= 1e-12 * ref.max()

    def poiseuille_ok():
        nx, ny = 40, 12
        t = np.zeros((ny, nx), np.uint8)
        t[0] = 1
        t[-1] = 1
        a = oracle.run_2d(oracle.State2D(t), 20000, xbc=1, rho_in=1.001, rho_out=0.999)
        y = np.arange(1, ny - 1) - 0.5
        rho = 1.0 + a.drho[1:-1, nx // 2].mean()
        g = -((0.999 - 1.001) / 3.0 / (nx - 1)) / rho
        want = g * 3.0 * y * (ny - 2 - y) + g / 4.0
        return np.abs(a.u[0, 1:-1, nx // 2] - want).max() <= 1e-4 * want.max()

    def cavity_ok():
        n = 16
        t = np.zeros((n, n), np.uint8)
        t[0, :] = 1
        t[:, 0] = 1
        t[:, -1] = 1
        t[-1, :] = 2
        a = oracle.run_2d(oracle.State2D(t), 1500, uw=(0.1, 0.0))
        m, _ = oracle.reduce_2d(a)
        return (abs(m - (t == 0).sum()) <= 1e-12 * (t == 0).sum()
                and a.u[0][n - 2, n // 2] > 0.01 and a.u[0][n // 3, n // 2] < 0.0)

    def two_node_ok():
        from test_oracle_2d import two_node_2d_error
        return max(two_node_2d_error(0), two_node_2d_error(1)) <= 1e-16

    def couette_ok():
        from test_oracle_2d import couette_error
        return couette_error(6, 0.05, 600) <= 1e-12

    check("lattice", lattice_ok)
    check("bgk_bitwise", bitwise_ok)
    check("two_node_moments", two_node_ok)
    check("couette", couette_ok)
    check("pressure_vs_bgk", pressure_ok)
    check("channel_closed_form", channel_ok)
    check("poiseuille_eq12", poiseuille_ok)
    check("cavity", cavity_ok)
    return failed


def test_pins_pass_on_real_2d_oracle():
    assert _quick_pins() == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    src = open(SRC).read()
    for old, new, count in MUTANTS[name]:
        assert src.count(old) >= 1, f"mutation site for {name} not found: {old}"
        src = src.replace(old, new, count)
    path_c = tmp_path / "mutant2d.c"
    path_c.write_text(src)
    so = tmp_path / "libmutant2d.so"
    subprocess.run(["gcc", *oracle.CFLAGS, str(path_c), "-o", str(so), "-lm"],
                   check=True, capture_output=True)
    with oracle.use_library_2d(str(so)):
        failed = _quick_pins()
    print(f"[mutant] {name}: caught by {failed}")
    assert failed, f"mutant {name} passed every pin"
