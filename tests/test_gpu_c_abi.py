"""The GPU entry points from plain C: tests/c_abi_gpu_driver.c, compiled with
gcc against include/sbt.h and linked to libsbt.so and the HIP runtime, runs
the plain form, the batched form (graph capture and replay on its own
stream) and the form that allocates nothing on a batch this test writes, and
each result must be the oracle's."""

import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_2207_03936_amd import sbt, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_2207_03936_amd")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
FORMS = ("plain", "batched capture", "batched replay", "no allocation")


def build_driver(tmp_path):
    if not os.path.exists(os.path.join(LIBDIR, "libsbt.so")):
        pytest.skip("libsbt.so is not built")
    exe = tmp_path / "c_abi_gpu_driver"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROCM, "include"), os.path.join(ROOT, "tests", "c_abi_gpu_driver.c"),
                    "-L", LIBDIR, "-lsbt", "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
                    "-Wl,-rpath," + LIBDIR, "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-o", str(exe)], check=True)
    return exe


def write_batch(path, b):
    p = sbt.DEFAULT_PARAMS
    with open(path, "wb") as f:
        np.array([b.n_modules, b.n_events, b.n_hits], np.int32).tofile(f)
        np.asarray(b.module_z, np.float32).tofile(f)
        np.array([p["reverse"], p["max_doublet_candidates"], p["phi_window_seeding"], p["phi_window_forwarding"]],
                 np.int32).tofile(f)
        np.array([p["max_scatter_seeding"], p["max_scatter_forwarding"], p["max_tracklet_chi2"]],
                 np.float32).tofile(f)
        np.array([p["max_consecutive_misses"], p["max_event_hits"]], np.int32).tofile(f)
        np.asarray(b.event_offsets, np.int32).tofile(f)
        np.asarray(b.module_offsets, np.int32).tofile(f)
        for a in (b.x, b.y, b.z):
            np.asarray(a, np.float32).tofile(f)


def read_results(path, n_events):
    a = np.fromfile(path, np.int32)
    out, i = [], 0
    for _ in FORMS:
        eto = a[i:i + n_events + 1]
        i += n_events + 1
        T = int(eto[-1])
        tho = a[i:i + T + 1]
        i += T + 1
        th = a[i:i + int(tho[-1])]
        i += int(tho[-1])
        st = a[i:i + n_events]
        i += n_events
        out.append((eto, tho, th, st))
    assert i == a.size
    return out


def test_driver_compiles(tmp_path):
    """The driver builds against the public header and the HIP runtime's C API."""
    assert build_driver(tmp_path).exists()


@pytest.mark.gpu
@pytest.mark.parametrize("config,n,first", [("mu7.6", 30, 3), ("mu1-25", 20, 40), ("mu30", 3, 0)])
def test_c_program_matches_oracle(tmp_path, config, n, first):
    exe = build_driver(tmp_path)
    b = synth.make_batch(config, n, first=first)
    write_batch(tmp_path / "batch.bin", b)
    print(f"C driver on {config} x{n}", flush=True)
    run = subprocess.run([str(exe), str(tmp_path / "batch.bin"), str(tmp_path / "tracks.bin")],
                         capture_output=True, text=True, timeout=120)
    assert run.returncode == 0, run.stdout + run.stderr
    want = oracle.reconstruct(b)
    for form, (eto, tho, th, st) in zip(FORMS, read_results(tmp_path / "tracks.bin", b.n_events)):
        assert not st.any(), form
        assert np.array_equal(eto, want[0]), form
        assert np.array_equal(tho, want[1]), form
        assert np.array_equal(th, want[2]), form
