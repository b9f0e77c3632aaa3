"""Long-run accuracy of every storage precision against the FP64 oracle, on
the 128^3 crop of the precision workload's mask (512^3 sphere packing, r = 12,
target porosity 0.6, seed 4000), run periodic for 2000 steps from rest with
g = 1e-6 along x.

- FP64 mode: the FP64 parity bar of the short cases (1e-12 absolute on
  rho - 1, 1e-12 of max|u| on u, permeability 1e-12 relative).  Rounding of
  order 2^-53 per step that grows at most linearly stays near 2000 x 2^-53 =
  2.2e-13.
- FP32 mode: rel-L2(u) and the relative permeability error within
  2000 x 2 x 2^-24 (the same linear growth of FP32 rounding as the porosity
  sweep), mass to 1e-9 relative.
- FP16 (default scale 2^16) and BF16 storage: every step rounds each stored
  value once, to a relative error of at most the unit roundoff eps (2^-11,
  2^-8).  Those errors enter the flow as independent perturbations that the
  update carries along without amplifying them, so after n steps their sum
  is bounded by sqrt(n) eps relative: rel-L2(u) and the relative
  permeability error must stay within sqrt(2000) eps (2.2e-2 FP16, 0.17
  BF16).  Mass changes only through the rounding of the stored rho - 1, at
  most eps |rho - 1| per node and step: the relative mass drift must stay
  within n eps mean|rho - 1| (mean over fluid nodes of the oracle's final
  state, the largest along a run that starts from rest).
"""
import time

import numpy as np
import pytest

import oracle
from paper_2312_14742_amd import inputs, tau1

from gpu_helpers import TOL_F64, rel_l2

pytestmark = pytest.mark.gpu

STEPS = 2000
G = (1e-6, 0.0, 0.0)


@pytest.fixture(scope="module")
def crop_and_oracle():
    geo = inputs.spheres(512, 512, 512, 12.0, 0.6, seed=4000)
    crop = np.ascontiguousarray(geo.solid[:128, :128, :128])
    print(f"[case] 128^3 crop of the porosity-0.6 packing, oracle {STEPS} steps", flush=True)
    t = time.perf_counter()
    st = oracle.run(19, oracle.State(crop), G, STEPS)
    mass, k = oracle.reduce(st, 0, G[0])
    print(f"[oracle] {time.perf_counter() - t:.1f} s", flush=True)
    return crop, st, mass, k


@pytest.mark.parametrize("prec", ["f64", "f32", "f16", "bf16"])
def test_crop_2000_steps_against_oracle(crop_and_oracle, prec):
    crop, ref, m_ref, k_ref = crop_and_oracle
    fl = crop == 0
    nf = float(fl.sum())
    print(f"[case] crop {prec}", flush=True)
    with tau1.Sim([tau1.Sample(crop)], lattice=19, precision=prec, g=G,
                  graph_chunk=100) as sim:
        sim.step(STEPS)
        drho, u = sim.moments(0, allow_nonfinite=True)
        k, m = sim.permeability(0, 0)
    e_u = rel_l2(u, ref.u, fl)
    e_k = abs(k - k_ref) / abs(k_ref)
    print(f"[err] {prec}: rel-L2(u) {e_u:.3e}, k rel {e_k:.3e}, mass drift {(m - nf) / nf:.3e} "
          f"(oracle {(m_ref - nf) / nf:.3e})", flush=True)
    assert np.isfinite(drho).all() and np.isfinite(u).all()
    if prec == "f64":
        assert np.abs(drho - ref.drho).max() <= TOL_F64
        assert np.abs(u - ref.u).max() <= TOL_F64 * np.abs(ref.u).max()
        assert e_k <= 1e-12
        assert abs(m - m_ref) <= 1e-12 * nf
    elif prec == "f32":
        bound = STEPS * 2.0 * 2.0 ** -24
        assert e_u <= bound
        assert e_k <= bound
        assert abs(m - nf) <= 1e-9 * nf
    else:
        eps = 2.0 ** -11 if prec == "f16" else 2.0 ** -8
        b_uk = np.sqrt(STEPS) * eps
        b_m = STEPS * eps * np.abs(ref.drho[fl]).mean()
        print(f"[bound] {prec}: rel-L2(u), k <= {b_uk:.3e}; |mass drift| <= {b_m:.3e}", flush=True)
        assert e_u <= b_uk and e_k <= b_uk
        assert abs(m - nf) / nf <= b_m
