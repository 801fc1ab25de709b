"""JSON-lines records of a pair's energy trace (host code, no GPU)."""
import json

import numpy as np

from paper_1703_01545_amd import metrics


def test_trace_records_steps_and_values(tmp_path):
    tr = np.array([[1.0, 1.5, 0.5], [2.0, 2.25, 0.25]])
    recs = list(metrics.trace_records(tr, 40, 20, **{"pass": "timed"}))
    assert [r["step"] for r in recs] == [60, 80]
    assert recs[1] == {"step": 80, "E_A": 2.0, "E_B": 2.25, "dE": 0.25, "pass": "timed"}
    path = tmp_path / "m.jsonl"
    assert metrics.write_jsonl(str(path), recs + [{"step": 80, "alive_A": 3}]) == 3
    lines = [json.loads(x) for x in path.read_text().splitlines()]
    assert lines[0]["dE"] == 0.5 and lines[2]["alive_A"] == 3


def test_empty_trace_has_no_records():
    assert list(metrics.trace_records(np.empty((0, 3)), 0, 20)) == []
