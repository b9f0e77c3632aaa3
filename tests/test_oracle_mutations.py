"""Planted mistakes in the oracle must be caught by its pins.

Each case copies ``oracle/tau1_oracle.c``, plants one plausible mistake by a
text substitution (a dropped term, a flipped sign, a wrong index or
direction, a transposed operand, a wrong weight), compiles the copy and runs
a fast subset of the pins against it.  The mutant passes this test only if at
least one pin rejects it.  The real oracle is never modified.
"""
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_2312_14742_amd import inputs

SRC = os.path.join(os.path.dirname(oracle.__file__), "tau1_oracle.c")

MUTANTS = {
    "bounce_back_same_direction": ("            dir = L->opp[k];\n",
                                   "            dir = k;\n"),
    "bounce_back_neighbour_state": ("            src = i;\n",
                                    "            src = s;\n"),
    "pull_from_wrong_side": ("long sx = wrap(x - L->c[k][0], nx);\n        long sy",
                             "long sx = wrap(x + L->c[k][0], nx);\n        long sy"),
    "no_force_shift_in_source": ("dr[src], ux[src] + G->gh[0],",
                                 "dr[src], ux[src],"),
    "no_force_shift_in_output": ("out[1] = jx * r + G->gh[0];",
                                 "out[1] = jx * r;"),
    "quadratic_sign": ("- 1.5 * vv;", "+ 1.5 * vv;"),
    "quadratic_operand": ("(4.5 * cu) * cu", "(4.5 * cu) * vv"),
    "linear_coefficient": ("(3.0 * cu +", "(1.0 * cu +"),
    "momentum_along_source_direction": (
        "jx += (double)L->c[k][0] * f;\n        jy += (double)L->c[k][1] * f;\n"
        "        jz += (double)L->c[k][2] * f;\n    }\n    r = 1.0 / (1.0 + d);\n    out",
        "jx += (double)L->c[dir][0] * f;\n        jy += (double)L->c[dir][1] * f;\n"
        "        jz += (double)L->c[dir][2] * f;\n    }\n    r = 1.0 / (1.0 + d);\n    out"),
    "reciprocal_sign": ("    r = 1.0 / (1.0 + d);\n    out", "    r = 1.0 / (1.0 - d);\n    out"),
    "edge_weight": ("we = 1.0 / 36.0;", "we = 1.0 / 30.0;"),
    "drho_term_dropped": ("return wk * (ds + rho * p);", "return wk * (rho * p);"),
    "opposite_map": ("L->opp[i] = (i % 2 == 1) ? i + 1 : i - 1;",
                     "L->opp[i] = (i % 2 == 1) ? i : i - 1;"),
    "velocity_component_swap": ("uy[src] + G->gh[1], uz[src] + G->gh[2]);",
                                "uz[src] + G->gh[1], uy[src] + G->gh[2]);"),
    # the O(u^2) part of Eq. (3): twice the coefficients, or none at all
    "quadratic_doubled": ("(4.5 * cu) * cu) - 1.5 * vv;", "(9.0 * cu) * cu) - 3.0 * vv;"),
    "quadratic_dropped": ("(3.0 * cu + (4.5 * cu) * cu) - 1.5 * vv;", "(3.0 * cu);"),
    "quadratic_velocity_term_only": ("- 1.5 * vv;", "- 0.5 * vv;"),
}


def _quick_pins():
    """Returns the names of the pins that fail on the currently routed oracle."""
    failed = []

    def check(name, fn):
        try:
            ok = fn()
        except Exception:                       # noqa: BLE001 - any crash counts
            ok = False
        if not ok:
            failed.append(name)

    def lattice_ok():
        for q in (15, 19, 27):
            c, w, opp = oracle.lattice(q)
            if abs(w.sum() - 1) > 1e-15:
                return False
            if np.abs((w[:, None, None] * c[:, :, None] * c[:, None, :]).sum(0)
                      - np.eye(3) / 3).max() > 1e-15:
                return False
            if any(tuple(c[opp[k]]) != tuple(-c[k]) for k in range(q)):
                return False
        return True

    def bgk_ok():
        for q in (15, 19, 27):
            solid, drho, u = inputs.random_state(5, 3, 7, seed=17)
            st = oracle.State(solid, drho, u)
            g = [1e-5, -2e-5, 3e-6]
            a = oracle.run(q, st, g, 6)
            b = oracle.bgk_run(q, st, g, 6)
            if a.u.tobytes() != b.u.tobytes() or a.drho.tobytes() != b.drho.tobytes():
                return False
        return True

    def channel_ok():
        from test_oracle_pins import channel_closed_form
        st = oracle.State(inputs.channel(3, 2, 32))
        out = oracle.run(19, st, [1e-6, 0, 0], 200)
        ref = channel_closed_form(30, 1e-6, 200)
        return np.abs(out.u[0][1:-1] - ref[:, None, None]).max() <= 1e-12 * ref.max()

    def uniform_ok():
        U = np.array([2e-3, -1e-3, 5e-4])
        g = np.array([1e-5, 2e-5, -3e-6])
        u = np.broadcast_to(U[:, None, None, None], (3, 4, 3, 3)).copy()
        st = oracle.State(np.zeros((4, 3, 3), np.uint8), None, u)
        out = oracle.run(27, st, g, 20)
        return (np.abs(out.u - (U + 20 * g)[:, None, None, None]).max() <= 1e-16
                and np.abs(out.drho).max() <= 1e-15)

    def linear_ok():
        from test_oracle_pins import _linear_matrix
        q = 19
        c, w, _ = oracle.lattice(q)
        nx, ny, nz = 8, 6, 5
        kappa = 2 * np.pi * np.array([1, 2, 1]) / np.array([nx, ny, nz])
        amp = 1e-9 * np.array([1 + 0.5j, -0.3 + 1j, 0.7 - 0.2j, 0.1 + 0.9j])
        Z, Y, X = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx),
                              indexing="ij")
        phase = np.exp(1j * (kappa[0] * X + kappa[1] * Y + kappa[2] * Z))
        field = np.real(amp[:, None, None, None] * phase[None])
        st = oracle.State(np.zeros((nz, ny, nx), np.uint8), field[0], field[1:])
        out = oracle.run(q, st, [0, 0, 0], 4)
        Mn = np.linalg.matrix_power(_linear_matrix(c, w, kappa), 4)
        pred = np.real((Mn @ amp)[:, None, None, None] * phase[None])
        got = np.concatenate([out.drho[None], out.u])
        return np.abs(got - pred).max() <= 1e-6 * np.abs(pred).max()

    def two_node_ok():
        from test_oracle_pins import two_node_moments_error
        return all(two_node_moments_error(q, a) <= 1e-16 for q in (15, 19, 27) for a in range(3))

    check("lattice", lattice_ok)
    check("bgk_bitwise", bgk_ok)
    check("two_node_moments", two_node_ok)
    check("channel_closed_form", channel_ok)
    check("uniform_flow", uniform_ok)
    check("linear_modes", linear_ok)
    return failed


def test_pins_pass_on_real_oracle():
    assert _quick_pins() == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    mutated = src.replace(old, new)
    path_c = tmp_path / "mutant.c"
    path_c.write_text(mutated)
    so = tmp_path / "libmutant.so"
    subprocess.run(["gcc", *oracle.CFLAGS, str(path_c), "-o", str(so), "-lm"],
                   check=True, capture_output=True)
    with oracle.use_library(str(so)):
        failed = _quick_pins()
    print(f"[mutant] {name}: caught by {failed}")
    assert failed, f"mutant {name} passed every pin"
