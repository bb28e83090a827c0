"""Host helpers of bench.py on the CPU: the equal-NRMSE summary (target 10%
below the speckle average's NRMSE, iterations and time to reach it, best
iterate from iteration 1) and the counter record lookup, which returns the
stored bytes only while the kernel sources hash to the value stored with
them."""

import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _forms():
    # nrmse[0] is the speckle average (every form's initial image): 0.30,
    # so the target is 0.27
    return {
        "plain": {"nrmse": [0.30, 0.29, 0.26, 0.28], "ms_per_iter": 1.0},
        "learned": {"nrmse": [0.30, 0.25, 0.20, 0.22], "ms_per_iter": 2.0},
        "forward_only": {"nrmse": [0.30, 0.31, 0.29, 0.295], "ms_per_iter": 0.5},
    }


def test_equal_nrmse_target_and_iterations():
    eq = bench.equal_nrmse_summary(_forms(), 3)
    assert eq["target_nrmse"] == pytest.approx(0.27)
    assert eq["plain"]["iterations"] == 2 and eq["plain"]["ms_to_target"] == pytest.approx(2.0)
    assert eq["learned"]["iterations"] == 1 and eq["learned"]["ms_to_target"] == pytest.approx(2.0)
    assert eq["forward_only"]["iterations"] is None and eq["forward_only"]["ms_to_target"] is None
    # best iterate counted from iteration 1 (iteration 0 is the common start)
    assert eq["forward_only"]["best_iteration"] == 2 and eq["forward_only"]["nrmse_best"] == pytest.approx(0.29)
    assert eq["learned"]["best_iteration"] == 2
    assert eq["plain"]["iters_per_s"] == pytest.approx(1000.0)
    # equal times to the target: not faster
    assert eq["learned_faster_than_plain"] is False


def test_equal_nrmse_learned_faster_when_plain_never_reaches():
    f = _forms()
    f["plain"]["nrmse"] = [0.30, 0.29, 0.28, 0.285]
    eq = bench.equal_nrmse_summary(f, 3)
    assert eq["plain"]["iterations"] is None
    assert eq["learned_faster_than_plain"] is True


def test_equal_nrmse_iteration_zero_never_counts():
    f = _forms()
    f["learned"]["nrmse"] = [0.30, 0.295, 0.29, 0.285]
    f["plain"]["nrmse"][0] = 0.30
    eq = bench.equal_nrmse_summary(f, 3)
    assert eq["learned"]["iterations"] is None
    assert eq["learned_faster_than_plain"] is False


def test_counter_record_needs_matching_source_hash(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    good = bench.kernel_source_hash("fwd")
    rec = {"fresh": {"source_sha256": good, "stages": {"row_grad": {"read_bytes": 1.0}}},
           "stale": {"source_sha256": "0" * 64, "stages": {}}}
    (prof / "counter_traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.counter_traffic("fresh", "fwd")["stages"]["row_grad"]["read_bytes"] == 1.0
    assert bench.counter_traffic("stale", "fwd") is None
    assert bench.counter_traffic("missing", "fwd") is None
    # the CNN group hashes other sources: a forward-path hash does not match it
    assert bench.counter_traffic("fresh", "cnn") is None


def test_counter_record_missing_file(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.counter_traffic("anything", "fwd") is None
