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
