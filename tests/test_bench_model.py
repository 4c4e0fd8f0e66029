"""The benchmark's byte and flop models against the values the survey's
formulas give for the workloads' sizes (host only)."""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402

# (K, Np, Nfp, E_int, Algorithm 1, fields) of the 256x256 N=4, 512x512 N=6 and
# 708x708 N=3 four-field meshes
SIZES = {
    "contrast_256x256_N4": (131072, 15, 5, 196096, True, 1),
    "loguniformD_512x512_N6": (524288, 28, 7, 785408, True, 1),
    "convdiff_708x708_N3_4f": (1002528, 10, 4, 1502376, False, 4),
}


@pytest.mark.parametrize("name,s,edge_mb,stage_mb", [
    ("contrast_256x256_N4", 8, 36.4, 130),
    ("contrast_256x256_N4", 4, 24.6, 99),
    ("loguniformD_512x512_N6", 8, 212.7, 873),
    ("loguniformD_512x512_N6", 4, 132.0, 653),
    ("convdiff_708x708_N3_4f", 4, 346.7, 1774),
])
def test_algorithmic_bytes_match_the_survey_table(name, s, edge_mb, stage_mb):
    K, Np, Nfp, E, alg1, nf = SIZES[name]
    edge, elem = bench.algorithmic_bytes(K, Np, Nfp, E, s, alg1, nf)
    assert abs(edge / 1e6 - edge_mb) < 0.06
    # the survey rounds its per-stage totals to whole MB (99 for 97.7)
    assert abs((edge + elem) / 1e6 - stage_mb) / stage_mb < 0.02


def test_rk4_stage_bytes_per_dof():
    # FP64: 24, 40, 40, 24 bytes per degree of freedom; FP32 stage vectors:
    # 4 + 16 + 4, 4 + 24 + 4 (twice), 4 + 16 + 4
    assert bench.rk4_dof_bytes(8, True) == pytest.approx((24 + 40 + 40 + 24) / 4)
    assert bench.rk4_dof_bytes(4, False) == pytest.approx((24 + 32 + 32 + 24) / 4)


def test_stored_bytes_exceed_table_free_model_by_the_tables():
    # the stored model differs from the survey's only in the tables and the
    # stage averaging: with no convection, no Algorithm 1 and no boundary
    # faces, the edge kernels differ by 4 bytes per edge (56 vs 60)
    K, Np, Nfp, E = 1000, 10, 4, 1500
    a_edge, _ = bench.algorithmic_bytes(K, Np, Nfp, E, 8, False, 2)
    s_edge, _ = bench.stored_bytes(K, Np, Nfp, E, 0, 8, False, 2, False)
    assert a_edge - s_edge == 4 * E


def test_flop_model():
    # per field and interior edge at N = 3: 4 (100 + 30) + 2 (8)(20) c
    e1, el = bench.algorithmic_flops(1, 10, 4, 3, 1, False, 1)
    assert e1 == 4 * (100 + 30) + 2 * 8 * 20
    e2, _ = bench.algorithmic_flops(1, 10, 4, 3, 1, True, 1)
    assert e2 - e1 == 2 * 8 * 20
    assert el == 2 * (4 * 100 + 3 * 10 * 4)
