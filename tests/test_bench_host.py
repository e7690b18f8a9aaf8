"""Host logic of bench.py (CPU): the one-GPU contract, the algorithmic byte
count of the roofline, and the rule that committed counter summaries are
used only for the kernel source they were taken on."""

import json
import os
import subprocess
import sys

import numpy as np

import oracle
from paper_2207_03936_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert out.returncode == 2
    assert "one GPU" in out.stdout + out.stderr


def test_algorithmic_bytes_counts_inputs_and_outputs():
    b = synth.make_batch("mu7.6", 3)
    eto, tho, th = oracle.reconstruct(b)
    E, H, M = b.n_events, b.n_hits, b.n_modules
    T = int(eto[-1])
    inputs = (b.x.nbytes + b.y.nbytes + b.z.nbytes + np.asarray(b.module_offsets, np.int32).nbytes +
              np.asarray(b.event_offsets, np.int32).nbytes)
    outputs = 4 * len(th) + 4 * (T + 1) + 4 * (E + 1)
    assert len(b.module_offsets) == E * M + 1 and len(b.event_offsets) == E + 1
    assert bench.algorithmic_bytes(b, eto, tho) == inputs + outputs
    assert len(th) == int(tho[T]) <= H


def test_counter_summaries_follow_the_kernel_source(monkeypatch):
    path = os.path.join(ROOT, "profiles", "k_persistent_mu7.6_x1000_traffic.json")
    with open(path) as f:
        d = json.load(f)
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: d["kernel_source_hash"])
    assert bench.measured_traffic(d["n_hits"]) == d["hbm_bytes_per_launch"]
    assert bench.measured_traffic(d["n_hits"] + 1) is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.measured_traffic(d["n_hits"]) is None
    assert bench.measured_sq(d["n_hits"]) is None
