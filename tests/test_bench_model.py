"""CPU checks of bench.py's byte model and measurement bookkeeping (no GPU):
the algorithmic bytes per voxel of the mechanics iteration forms follow from
their passes' reads and writes, and the counter-measured traffic table is
keyed by a hash of the kernel sources."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_form_bytes_consistent():
    n = 1024
    sp = 16.0 * (n // 2 + 1) / n  # one component's half spectrum per voxel
    three = bench.algo_bytes_sr(n, passes=3)
    two = bench.algo_bytes_sr(n, passes=2)
    # the fused row stage = stiffness + transform pass + inverse pass, minus
    # the re-read of p (16 B) that fusing removes
    assert abs(two["mech_row_fwd"] - (three["mech_row_fwd"] + three["mech_row_inv"] - 16.0)) < 1e-9
    assert two["mech_col"] == three["mech_col"] == 8 * sp
    assert abs(sum(three.values()) - 185.2) < 0.1 and abs(sum(two.values()) - 169.2) < 0.1
    # the four-pass form (ALGO_BYTES) moves more per iteration than either
    assert sum(bench.ALGO_BYTES.values()) > sum(three.values()) > sum(two.values())
    assert bench.kinds_of(2) == ["mech_row_fwd", "mech_col"]
    assert set(bench.kinds_of(3)) == set(three) and set(bench.kinds_of(2)) == set(two)


def test_traffic_table_is_keyed_by_source_hash():
    h = bench.csrc_hash()
    assert len(h) == 64 and all(c in "0123456789abcdef" for c in h)
    for key, kinds in bench.MEASURED_TRAFFIC.items():
        assert len(key) == 64
        assert all(k in ("mech_kp", "mech_row_fwd", "mech_col", "mech_row_inv") and v > 0 for k, v in kinds.items())
