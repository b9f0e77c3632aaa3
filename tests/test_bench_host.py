"""Host side of bench.py (no GPU): the one-GPU guard, the chunk statistics of
the porous-media bandwidth model on hand-counted lattices, and the counter
profile that the roofline's traffic figure is read from."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused(capsys):
    assert bench.main(["--gpus", "2"]) == 2
    assert "exactly one GPU" in capsys.readouterr().err


def test_chunk_stats_hand_counted():
    # one plane, 4 rows of 8 nodes, chunks of 4: row 0 all solid, row 1 one
    # solid node, rows 2-3 all fluid.  Periodic D3Q19 neighbours (nz = 1 means
    # the z links see the same plane).
    solid = np.zeros((1, 4, 8), np.uint8)
    solid[0, 0, :] = 1
    solid[0, 1, 5] = 1
    st = bench.chunk_stats(solid, 4)
    assert st["chunk_nodes"] == 4
    # 8 chunks, the two of row 0 hold no fluid
    assert st["stored_chunk_frac"] == 6 / 8
    # 23 fluid nodes in 6 stored chunks of 4
    assert st["phi_chunk"] == 23 / 24
    # mixed: both chunks of row 1 (next to row 0 / holding the solid node) and
    # both chunks of row 3 (its y + 1 neighbour, periodic, is row 0); row 2
    # chunk 1 sees the solid node of row 1 along (+-1, -1, 0) and (0, -1, 0)
    assert st["r_mixed"] == 5 / 6


def test_chunk_stats_all_fluid_and_all_solid():
    fl = bench.chunk_stats(np.zeros((2, 3, 8), np.uint8), 4)
    assert fl["stored_chunk_frac"] == 1.0 and fl["phi_chunk"] == 1.0 and fl["r_mixed"] == 0.0
    so = bench.chunk_stats(np.ones((2, 3, 8), np.uint8), 4)
    assert so["stored_chunk_frac"] == 0.0 and so["phi_chunk"] == 0.0 and so["r_mixed"] == 0.0


def test_counter_profile_matches_kernel_sources():
    """The HBM traffic in the bench line comes from this profile only while it
    was taken on the current kernel sources; a kernel change must come with
    new counters."""
    cnt = bench.read_counters()
    assert cnt is not None
    assert cnt["source_sha256"] == bench.kernel_source_hash()
    # the tile the autotuner picks for this workload
    assert float(cnt["hbm_bytes_per_launch_tile15"]) > 0


def test_bandwidth_model_recovers_its_penalty():
    """Rates generated from Eq. (13) with a known delta_p give that delta_p
    back, and B_est then equals the generated rates."""
    b_max, delta = 6000.0, 1.7
    rows = []
    for phi_c, r in ((0.58, 0.97), (0.7, 0.85), (0.88, 0.45), (0.97, 0.12)):
        b = phi_c * b_max / (1.0 + delta * r / 2.0)
        rows.append({"phi_chunk": phi_c, "r_mixed": r, "packed": {"alg_gbs": b}})
    got = bench.bandwidth_model(rows, b_max)
    assert abs(got - delta) <= 1e-12
    for row in rows:
        assert abs(row["b_est_gbs"] - row["packed"]["alg_gbs"]) <= 1e-9 * row["b_est_gbs"]
        assert row["b_chunk_only_gbs"] == row["phi_chunk"] * b_max
