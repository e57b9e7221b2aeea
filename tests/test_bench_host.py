"""Host-side helpers of bench.py: the first-pass ranking used for the
before-rescore recall and the comparison against the float64 fixture."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def test_first_pass_topk_orders_by_score_then_id():
    S = np.array([[0.5, 0.9, 0.9, 0.1, 0.7]], np.float32)
    ids, sc = bench.first_pass_topk(S, 4)
    assert ids.tolist() == [[1, 2, 4, 0]]
    assert sc.tolist() == [[np.float32(0.9), np.float32(0.9), np.float32(0.7), np.float32(0.5)]]


def test_fp64_compare_recall_and_rankwise_error():
    fx = {"ids": np.array([[3, 1, 2], [0, 1, 2]]), "scores": np.array([[0.9, 0.8, 0.7],
                                                                       [0.6, 0.5, 0.4]])}
    ids = np.array([[3, 1, 4], [0, 1, 2]])
    sc = np.array([[0.9, 0.8, 0.65], [0.6, 0.5, 0.4]], np.float32)
    r = bench.fp64_compare(ids, sc, fx, 3)
    assert abs(r["at100_mean"] - (2 / 3 + 1) / 2) < 1e-12 and abs(r["at100_min"] - 2 / 3) < 1e-12
    assert abs(r["max_abs_score_err"] - 0.05) < 1e-6


def test_fixture_matches_its_script_shape():
    f = np.load(bench.FP64_FIXTURE)
    assert f["ids"].shape == (256, 100) and f["scores"].shape == (256, 100)
    # ranked by score descending; the 101st score is below the 100th
    assert (np.diff(f["scores"], axis=1) <= 0).all()
    assert (f["next"] <= f["scores"][:, -1]).all()
