"""Shared helpers of the GPU tests: run the HIP path and the oracle on the same
seeded inputs and compare them."""
from __future__ import annotations

import numpy as np

import oracle
from paper_2312_14742_amd import tau1

# Tolerance of the HIP path against the FP64 oracle in FP64 mode (normwise:
# absolute on rho, relative to max|u| on u).  The reduced-precision modes use
# bounds derived from the storage rounding unit, written in their tests.
TOL_F64 = 1e-12


def run_gpu(samples, lattice, precision, g, nsteps, **kw):
    sim = tau1.Sim([tau1.Sample(*s) for s in samples], lattice=lattice,
                   precision=precision, g=g, **kw)
    sim.step(nsteps)
    out = [sim.moments(i) for i in range(len(samples))]
    return sim, out


def run_oracle(q, solid, drho, u, g, nsteps):
    st = oracle.State(solid, drho, u)
    return oracle.run(q, st, g, nsteps)


def assert_f64_parity(gpu, ref, solid, tol=TOL_F64):
    """max|drho - drho_ref| <= tol and max|u - u_ref| <= tol * max|u_ref|."""
    drho, u = gpu
    fl = solid == 0
    assert np.all(drho[~fl] == 0) and np.all(u[:, ~fl] == 0)
    ed = np.abs(drho - ref.drho).max() if fl.any() else 0.0
    umax = np.abs(ref.u).max()
    eu = np.abs(u - ref.u).max()
    assert ed <= tol, f"drho err {ed}"
    assert eu <= tol * max(umax, 1e-300), f"u err {eu} vs max|u| {umax}"


def rel_l2(a, b, mask):
    num = np.sqrt(np.sum((a - b)[..., mask] ** 2))
    den = np.sqrt(np.sum(b[..., mask] ** 2))
    return num / den if den > 0 else num


def reduced_errors(gpu, ref, solid):
    drho, u = gpu
    fl = solid == 0
    return {
        "drho_abs": float(np.abs(drho - ref.drho)[fl].max()) if fl.any() else 0.0,
        "u_rel_l2": float(rel_l2(u, ref.u, fl)),
        "u_max_rel": float(np.abs(u - ref.u).max() / max(np.abs(ref.u).max(), 1e-300)),
    }


# Unit roundoff of the storage formats of the reduced-precision modes.
UNIT_ROUNDOFF = {"f32": 2.0 ** -24, "f16": 2.0 ** -11, "bf16": 2.0 ** -8}


def sample_nodes(solid, n_random, seed):
    """Random fluid nodes plus whole rows and planes at the periodic edges."""
    nz, ny, nx = solid.shape
    rng = np.random.Generator(np.random.PCG64(seed))
    fluid = np.flatnonzero(solid.ravel() == 0)
    idx = [rng.choice(fluid, size=min(n_random, fluid.size), replace=False)]
    for (y, z) in [(0, 0), (ny - 1, nz - 1), (ny // 2, 0), (0, nz // 2), (ny - 1, 1)]:
        idx.append(np.arange(nx) + nx * (y + ny * z))
    for x in (0, nx - 1):
        yy, zz = np.meshgrid(np.arange(0, ny, 7), np.arange(0, nz, 7), indexing="ij")
        idx.append((x + nx * (yy + ny * zz)).ravel())
    idx = np.unique(np.concatenate(idx))
    return idx[solid.ravel()[idx] == 0]


def check_step(sim, sample, solid, q, prec, g, idx, label):
    d0, u0 = sim.moments(sample)
    sim.step(1)
    d1, u1 = sim.moments(sample)
    ref = oracle.step_nodes(q, oracle.State(solid, d0, u0), g, idx)
    got_d = d1.ravel()[idx]
    got_u = np.stack([u1[a].ravel()[idx] for a in range(3)], axis=1)
    eps = UNIT_ROUNDOFF[prec]
    umax = np.abs(ref[:, 1:]).max()
    ed = np.abs(got_d - ref[:, 0]).max()
    eu = np.sqrt(np.sum((got_u - ref[:, 1:]) ** 2) / np.sum(ref[:, 1:] ** 2))
    print(f"[err] {label}: {idx.size} nodes, max|ddrho| {ed:.3e}, rel-L2(u) {eu:.3e}, "
          f"max|u| {umax:.3e}", flush=True)
    assert ed <= (2.0 * eps + 16.0 * 2.0 ** -24) * umax, (label, ed)
    assert eu <= 8.0 * eps, (label, eu)
