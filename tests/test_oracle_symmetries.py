"""Symmetry pins of the 3-D oracle (CPU only).  The lattices D3Q15/19/27 are
invariant under mirroring an axis and under permuting the axes, and so is the
update (equilibria, halfway bounce-back, periodic wrap, body force): running a
mirrored or axis-permuted copy of a porous state must give the mirrored or
permuted result, up to the order in which the sums are rounded.  A wrong
weight, sign or component on any single direction breaks one of them."""
import numpy as np
import pytest

import oracle
from paper_2312_14742_amd import inputs

LATTICES = (15, 19, 27)
STEPS = 10
G = (2e-5, -1e-5, 3e-6)


def porous_state(seed):
    solid, drho, u = inputs.random_state(9, 7, 6, seed=seed, solid_frac=0.3, u_amp=0.03)
    return solid, drho, u


def run(q, solid, drho, u, g):
    return oracle.run(q, oracle.State(solid, drho, u), g, STEPS)


def close(a, b, scale):
    return np.abs(a - b).max() <= 1e-13 * scale


@pytest.mark.parametrize("q", LATTICES)
@pytest.mark.parametrize("axis", [0, 1, 2])      # mirror x, y or z
def test_mirror_symmetry(q, axis):
    solid, drho, u = porous_state(7100 + q + axis)
    ref = run(q, solid, drho, u, G)
    ax = 2 - axis                                   # array axis of the mirrored coordinate
    flip = lambda a: np.flip(a, axis=ax)            # noqa: E731
    um = np.stack([flip(u[c]) * (-1.0 if c == axis else 1.0) for c in range(3)])
    gm = tuple(-G[c] if c == axis else G[c] for c in range(3))
    out = run(q, flip(solid).copy(), flip(drho).copy(), um, gm)
    umax = np.abs(ref.u).max()
    assert close(out.drho, flip(ref.drho), 1.0)
    for c in range(3):
        want = flip(ref.u[c]) * (-1.0 if c == axis else 1.0)
        assert close(out.u[c], want, umax), (q, axis, c)


@pytest.mark.parametrize("q", LATTICES)
def test_axis_permutation_symmetry(q):
    """New axes (x', y', z') = (y, z, x): arrays indexed [z, y, x] become
    [x, z, y], and velocity components and force follow."""
    solid, drho, u = porous_state(7200 + q)
    ref = run(q, solid, drho, u, G)
    perm = lambda a: np.ascontiguousarray(a.transpose(2, 0, 1))   # noqa: E731
    up = np.stack([perm(u[1]), perm(u[2]), perm(u[0])])
    gp = (G[1], G[2], G[0])
    out = run(q, perm(solid), perm(drho), up, gp)
    umax = np.abs(ref.u).max()
    assert close(out.drho, perm(ref.drho), 1.0)
    for c, src in enumerate((1, 2, 0)):
        assert close(out.u[c], perm(ref.u[src]), umax), (q, c)
