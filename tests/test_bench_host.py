"""Host logic of bench.py, on the CPU: the one-GPU rule, the algorithmic bytes
a step moves per cell, and the rule that the committed HBM counter figures
count only for the kernel sources they were taken on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

WORKLOAD_CELLS = {"c2_channel": 200 * 4000,
                  "c2_channel_1000x16000": 1000 * 16000,
                  "c3_dense": 1536 * 1536}


def traffic_record(workload):
    path = os.path.join(ROOT, "profiles", f"traffic_k_step_{workload}.json")
    with open(path) as fh:
        return json.load(fh)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"),
                        "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_bytes_per_cell_follow_the_storage_layout():
    """Two D2Q9 lattices, each population read once and written once per
    step, plus the [df_s/dt] carrier (FP32 under the 16-bit forms) read and
    written once."""
    pop = {"fp64": 8, "fp32": 4, "fp16s": 2, "bf16s": 2}
    carrier = {"fp64": 8, "fp32": 4, "fp16s": 4, "bf16s": 4}
    for prec in pop:
        assert bench.BYTES_PER_CELL[prec] == 2 * 2 * 9 * pop[prec] \
            + 2 * carrier[prec]


def test_code_only_ignores_comments_and_spacing():
    a = "int x = 1; // note\n/* a block\n   comment */ int y;\n"
    b = "int x = 1;\n\n    int y;"
    assert bench.code_only(a, False) == bench.code_only(b, False)
    assert bench.code_only("x = 1  # note\n", True) == \
        bench.code_only("x = 1\n", True)
    assert bench.code_only("int x = 1;", False) != \
        bench.code_only("int x = 2;", False)


@pytest.mark.parametrize("workload", sorted(WORKLOAD_CELLS))
def test_committed_traffic_is_near_the_algorithmic_bytes(workload):
    """The counter summary's bytes per launch lie between 1 % below and 12 %
    above the algorithmic bytes of its workload, for every storage form it
    holds (the cavity's scattered tile order re-reads up to a fifth of the
    16-bit forms' neighbour rows; the channels stay within 2 %)."""
    rec = traffic_record(workload)
    assert rec["workload"] == workload
    for prec, ent in rec["per_precision"].items():
        alg = bench.BYTES_PER_CELL[prec] * WORKLOAD_CELLS[workload]
        assert ent["algorithmic_bytes"] == alg
        # each part rounded to whole bytes on its own
        assert abs(ent["bytes_per_launch"]
                   - (ent["read_bytes"] + ent["write_bytes"])) <= 1
        hi = 1.12 if workload == "c3_dense" else 1.02
        assert 0.99 * alg < ent["bytes_per_launch"] < hi * alg, (prec, ent)


def test_traffic_counts_only_for_its_kernel_sources(monkeypatch):
    for w in WORKLOAD_CELLS:
        rec = traffic_record(w)
        if rec["kernel_hash"] == bench.kernel_hash():
            assert bench.measured_traffic(w, "fp64") == \
                rec["per_precision"]["fp64"]["bytes_per_launch"]
    monkeypatch.setattr(bench, "kernel_hash", lambda: "0" * 16)
    for w in WORKLOAD_CELLS:
        assert bench.measured_traffic(w, "fp64") is None
    assert bench.measured_traffic("no_such_workload", "fp64") is None
