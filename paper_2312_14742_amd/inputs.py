"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module only builds geometries and initial fields.  It holds none of the
lattice Boltzmann arithmetic, so the oracle and the GPU path can both be fed
from it without sharing any of the method.

Geometries follow the paper's porous-medium experiment (randomly placed,
overlapping spherical obstacles in a periodic box, swept over porosity).  The
paper leaves the sphere radius, the random generator and the stopping rule
unstated; the rule used here is:

* centres are drawn one at a time from ``numpy.random.Generator(PCG64(seed))``
  as ``rng.uniform(0, (nx, ny, nz))`` (continuous positions);
* node (x, y, z) is solid when its periodic minimum-image squared distance to
  a centre is <= r**2;
* spheres are added until the porosity (fluid fraction) first drops to or
  below the target.

All arrays use shape (nz, ny, nx): x is the fastest axis, flat index
x + nx*(y + ny*z).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class Geometry:
    solid: np.ndarray          # uint8 (nz, ny, nx), 1 = solid
    porosity: float            # achieved fluid fraction
    spheres: int               # spheres placed
    radius: float
    seed: int
    target: float

    @property
    def dims(self):
        nz, ny, nx = self.solid.shape
        return nx, ny, nz

    @property
    def n_fluid(self) -> int:
        return int(self.solid.size - np.count_nonzero(self.solid))


def channel(nx: int, ny: int, nz: int) -> np.ndarray:
    """Plane channel: solid layers at z = 0 and z = nz - 1, fluid between."""
    s = np.zeros((nz, ny, nx), dtype=np.uint8)
    s[0] = 1
    s[nz - 1] = 1
    return s


def _axis_candidates(c: np.ndarray, r: float, L: int):
    """Per-axis candidate node indices and signed offsets for centres c (M,)."""
    D = int(math.floor(2.0 * r)) + 2
    if D >= L:
        a = np.broadcast_to(np.arange(L), (c.size, L))
        d = (a - c[:, None] + 0.5 * L) % L - 0.5 * L
        return a.astype(np.int64), d
    base = np.floor(c - r).astype(np.int64)
    cand = base[:, None] + np.arange(D)[None, :]
    d = cand - c[:, None]
    return cand % L, d


def spheres(nx: int, ny: int, nz: int, radius: float, target: float,
            seed: int, rng: np.random.Generator | None = None) -> Geometry:
    """Overlapping spheres of one radius added until porosity <= target.

    ``rng`` may be passed to continue an existing stream (the batch recipe
    draws its per-sample parameters from the same generator first).
    """
    if rng is None:
        rng = np.random.Generator(np.random.PCG64(seed))
    N = nx * ny * nz
    solid = np.zeros(N, dtype=bool)
    fluid = N
    placed = 0
    r2 = float(radius) * float(radius)
    if target >= 1.0 or fluid / N <= target:
        return Geometry(solid.reshape(nz, ny, nx).astype(np.uint8),
                        fluid / N, 0, radius, seed, target)
    D = int(math.floor(2.0 * radius)) + 2
    M = max(16, min(4096, (2 << 20) // (D ** 3)))
    hi = np.array([nx, ny, nz], dtype=np.float64)
    while True:
        centres = rng.uniform(0.0, hi, size=(M, 3))
        ix, dx = _axis_candidates(centres[:, 0], radius, nx)
        iy, dy = _axis_candidates(centres[:, 1], radius, ny)
        iz, dz = _axis_candidates(centres[:, 2], radius, nz)
        d2 = (dz[:, :, None, None] ** 2 + dy[:, None, :, None] ** 2
              + dx[:, None, None, :] ** 2)
        inside = d2 <= r2
        sid, a, b, c = np.nonzero(inside)          # sphere-major order
        flat = (iz[sid, a] * ny + iy[sid, b]) * nx + ix[sid, c]
        new = ~solid[flat]
        flat = flat[new]
        sid = sid[new]
        # first sphere (in draw order) that covers each newly covered node
        uniq, first = np.unique(flat, return_index=True)
        first_sid = sid[first]
        counts = np.bincount(first_sid, minlength=M)
        after = fluid - np.cumsum(counts)
        hit = np.nonzero(after <= target * N)[0]
        if hit.size:
            m = int(hit[0])
            sel = first_sid <= m
            solid[uniq[sel]] = True
            fluid = int(after[m])
            placed += m + 1
            break
        solid[uniq] = True
        fluid = int(after[-1])
        placed += M
    return Geometry(solid.reshape(nz, ny, nx).astype(np.uint8), fluid / N,
                    placed, radius, seed, target)


@dataclass
class BatchSample:
    geometry: Geometry
    side: int
    target: float
    radius: float


def _batch_one(args):
    seed, sides = args
    rng = np.random.Generator(np.random.PCG64(seed))
    side = 64 + 32 * int(rng.integers(0, 9))
    if sides is not None:
        side = int(sides(side))
    target = float(rng.uniform(0.4, 0.95))
    radius = float(rng.uniform(4.0, 16.0))
    geo = spheres(side, side, side, radius, target, seed, rng=rng)
    return BatchSample(geo, side, target, radius)


def batch_recipe(n_samples: int = 64, seed0: int = 5000,
                 sides=None, workers: int = 1) -> list[BatchSample]:
    """Uneven porous samples for the batched path.

    Per sample i, from PCG64(seed0 + i) in this order: side = 64 + 32 *
    integers(0, 9); target porosity ~ U[0.4, 0.95]; radius ~ U[4, 16]; then
    the sphere centres.  ``sides`` (optional) caps the sides for small tests.
    ``workers`` > 1 draws the samples in a process pool (same results: each
    sample depends only on its own seed); call it before any GPU use.
    """
    jobs = [(seed0 + i, sides) for i in range(n_samples)]
    if workers <= 1 or sides is not None:
        return [_batch_one(j) for j in jobs]
    import multiprocessing as mp
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(_batch_one, jobs, chunksize=1)


def random_state(nx: int, ny: int, nz: int, seed: int, solid_frac: float = 0.3,
                 drho_amp: float = 1e-3, u_amp: float = 0.05):
    """Random mask, drho and u for small parity cases (|u| <= u_amp per axis)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    solid = (rng.random((nz, ny, nx)) < solid_frac).astype(np.uint8)
    drho = rng.uniform(-drho_amp, drho_amp, (nz, ny, nx))
    u = rng.uniform(-u_amp, u_amp, (3, nz, ny, nx))
    drho[solid == 1] = 0.0
    u[:, solid == 1] = 0.0
    return solid, drho, u


def shear_wave(nx: int, ny: int, nz: int, amplitude: float, mode: int = 1):
    """u_x = U sin(2 pi m z / nz), rho = 1, no solids."""
    z = np.arange(nz, dtype=np.float64)
    prof = amplitude * np.sin(2.0 * np.pi * mode * z / nz)
    u = np.zeros((3, nz, ny, nx))
    u[0] = prof[:, None, None]
    return np.zeros((nz, ny, nx), dtype=np.uint8), np.zeros((nz, ny, nx)), u
