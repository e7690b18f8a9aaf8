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


def test_counter_summaries_follow_the_kernel_source_and_tuning(monkeypatch, tmp_path):
    """A summary is used only for the kernel source, batch size and launch
    configuration it was taken on."""
    tuning = dict(threads_per_event=512, blocks_per_cu=2, lds_window_hits=672, lds_owner_hits=16384)
    d = {"kernel_source_hash": "ab" * 8, "n_hits": 1234, "tuning": dict(tuning),
         "fabric_bytes_per_launch": 777, "SQ_INSTS_VALU": 5, "SQ_INSTS_SALU": 6, "SQ_INSTS_LDS": 7}
    (tmp_path / "profiles").mkdir()
    for name in ("k_persistent_mu7.6_x1000_traffic.json", "k_persistent_mu7.6_x1000_sq.json"):
        (tmp_path / "profiles" / name).write_text(json.dumps(d))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "ab" * 8)
    assert bench.measured_traffic(1234, tuning) == 777
    assert bench.measured_sq(1234, tuning)["SQ_INSTS_VALU"] == 5
    assert bench.measured_traffic(1235, tuning) is None
    for k, v in (("threads_per_event", 1024), ("blocks_per_cu", 1), ("lds_window_hits", 768)):
        other = dict(tuning, **{k: v})
        assert bench.measured_traffic(1234, other) is None, k
        assert bench.measured_sq(1234, other) is None, k
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.measured_traffic(1234, tuning) is None
    assert bench.measured_sq(1234, tuning) is None


def test_committed_summaries_name_their_tuning():
    """Every committed counter summary records the launch configuration it
    was taken on, so bench.py can tell whether it describes the timed one."""
    for name in ("k_persistent_mu7.6_x1000_traffic.json", "k_persistent_mu7.6_x1000_sq.json"):
        path = os.path.join(ROOT, "profiles", name)
        with open(path) as f:
            d = json.load(f)
        assert set(bench.TUNING_KEYS) <= set(d["tuning"]), name
        assert "kernel" in d and "commands" in d, name


def test_guarded_leg_reports_listed_errors_only():
    """A leg after the headline reports a listed error in its place; any
    other error still ends the run."""
    import pytest
    assert bench.guarded("ok", lambda: {"v": 1}, (RuntimeError,)) == {"v": 1}

    def fail():
        raise RuntimeError("no memory")
    assert bench.guarded("bad", fail, (RuntimeError,)) == {"error": "RuntimeError: no memory"}

    def other():
        raise KeyError("x")
    with pytest.raises(KeyError):
        bench.guarded("other", other, (RuntimeError,))


def test_committed_summaries_describe_the_committed_kernels():
    """The committed counter summaries were taken on the kernel source as it
    is (comments aside), so the benchmark line carries their traffic and
    instruction counts; a kernel change needs them taken again."""
    h = bench.kernel_source_hash()
    for name in ("k_persistent_mu7.6_x1000_traffic.json", "k_persistent_mu7.6_x1000_sq.json"):
        with open(os.path.join(ROOT, "profiles", name)) as f:
            assert json.load(f)["kernel_source_hash"] == h, name
