"""JSON-lines records (paper_1606_02162_amd/records.py): host-only."""
import math

import numpy as np

from paper_1606_02162_amd import records


def test_iteration_records_skip_rows_not_run(tmp_path):
    hist = np.array([[10.0, 2.0, 7.0, 0.0], [5.0, 1.0, 3.0, 2.0], [np.nan] * 4])
    temps = np.array([4.0, 3.0, 2.0])
    recs = records.iteration_records(hist, temps, workload="w")
    assert [r["h"] for r in recs] == [0, 1]
    assert recs[1] == {"kind": "iteration", "h": 1, "cap": 3.0, "energy": 5.0, "max_disp": 1.0,
                       "moved": 3, "coincident": 2, "workload": "w"}
    # h0 shifts the iteration numbers and the caps read
    recs = records.iteration_records(hist[1:2], temps, h0=1)
    assert recs[0]["h"] == 1 and recs[0]["cap"] == 3.0


def test_job_record_arithmetic():
    r = records.job_record(0.5, pairs=1000, nnz=200, n_active=50, iterations=10, job=3)
    assert r["interactions"] == (1000 + 200) * 10
    assert math.isclose(r["interactions_per_s"], 12000 / 0.5)
    assert math.isclose(r["bytes_per_s"], (4 * 1000 + 4 * 200 + 32 * 50) * 10 / 0.5)
    assert math.isclose(r["roofline_frac"], r["bytes_per_s"] / 8e12)
    assert r["latency_ms"] == 500.0 and r["job"] == 3 and r["kind"] == "job"


def test_write_and_read_back(tmp_path):
    path = str(tmp_path / "r.jsonl")
    a = [{"kind": "job", "x": 1}]
    b = [{"kind": "served_job", "x": 2}, {"kind": "served_job", "x": 3}]
    assert records.write_jsonl(path, a) == 1
    assert records.write_jsonl(path, b, append=True) == 2
    assert records.read_jsonl(path) == a + b
    records.write_jsonl(path, b)              # not appending: replaced
    assert records.read_jsonl(path) == b
