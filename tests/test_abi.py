"""The C ABI library loads, exports every symbol include/sbt.h declares, and
its host-side argument checks behave as documented (no GPU needed)."""

import ctypes
import os
import re

import numpy as np
import pytest

from paper_2207_03936_amd import sbt, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "sbt.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sbt_[a-z0-9_]+)\s*\(", txt)))


def test_exports_every_declared_symbol():
    names = _declared()
    assert len(names) >= 20
    L = ctypes.CDLL(sbt.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(sbt.PROTOTYPES)


def test_error_strings():
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert sbt.lib().sbt_error_string(code)


def test_params_validation():
    L = sbt.lib()
    p = sbt.make_params(synth.PLANE_Z)
    assert L.sbt_params_validate(ctypes.byref(p)) == 0
    bad = [dict(max_doublet_candidates=0), dict(phi_window_seeding=32768), dict(phi_window_forwarding=-1),
           dict(max_consecutive_misses=-1), dict(reverse=2), dict(max_event_hits=-1)]
    for b in bad:
        assert L.sbt_params_validate(ctypes.byref(sbt.make_params(synth.PLANE_Z, **b))) == sbt.SBT_ERR_INVALID_ARG
    assert L.sbt_params_validate(ctypes.byref(sbt.make_params(synth.PLANE_Z[:2]))) == sbt.SBT_ERR_INVALID_ARG
    z = synth.PLANE_Z.copy()
    z[5] = z[4]
    assert L.sbt_params_validate(ctypes.byref(sbt.make_params(z))) == sbt.SBT_ERR_INVALID_ARG
    assert L.sbt_params_validate(ctypes.byref(sbt.make_params(synth.PLANE_Z[::-1]))) == 0
    assert L.sbt_params_validate(None) == sbt.SBT_ERR_INVALID_ARG


def _check_offsets(M, eo, mo, H):
    eo = np.ascontiguousarray(eo, np.int32)
    mo = np.ascontiguousarray(mo, np.int32)
    ip = ctypes.POINTER(ctypes.c_int32)
    return sbt.lib().sbt_validate_offsets_host(M, eo.size - 1, H, eo.ctypes.data_as(ip), mo.ctypes.data_as(ip))


def test_offsets_validation():
    b = synth.make_batch("tiny", 3)
    M, H = b.n_modules, b.n_hits
    assert _check_offsets(M, b.event_offsets, b.module_offsets, H) == 0
    mo = b.module_offsets.copy()
    mo[5], mo[6] = mo[6], mo[5] + 0
    mo[5] = mo[6] + 1
    assert _check_offsets(M, b.event_offsets, mo, H) == sbt.SBT_ERR_INVALID_ARG
    eo = b.event_offsets.copy()
    eo[-1] += 1
    assert _check_offsets(M, eo, b.module_offsets, H) == sbt.SBT_ERR_INVALID_ARG
    # one event above the 16-bit id range
    n = 65536
    eo = np.array([0, n], np.int32)
    mo = np.concatenate([[0], np.full(M, n // M), [0]])[:M + 1].cumsum().astype(np.int32)
    mo[-1] = n
    assert _check_offsets(M, eo, mo, n) == sbt.SBT_ERR_EVENT_TOO_LARGE


def test_workspace_size_monotone():
    a = sbt.sbt_workspace_size(10, 1000)
    b = sbt.sbt_workspace_size(10, 100000)
    c = sbt.sbt_workspace_size(1000, 100000)
    assert 0 < a < b < c
    with pytest.raises(sbt.SbtError):
        sbt.sbt_workspace_size(-1, 10)


def test_product_path_fails_loudly_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(RuntimeError):
        sbt.DeviceBatch(synth.make_batch("tiny", 1))


def test_tune_cache_roundtrip(tmp_path, monkeypatch):
    monkeypatch.setenv("SBT_TUNE_CACHE", str(tmp_path / "t.json"))
    assert sbt._tune_cache_get("gfx950|E1|N1|X1") is None
    sbt._tune_cache_put("gfx950|E1|N1|X1", dict(threads_per_event=512, blocks_per_cu=2, lds_window_hits=672,
                                                 lds_owner_hits=16384))
    got = sbt._tune_cache_get("gfx950|E1|N1|X1")
    assert got["threads_per_event"] == 512 and got["lds_window_hits"] == 672
    assert [sbt._bucket(v) for v in (1, 2, 3, 4, 5, 6, 8, 1000)] == [1, 2, 3, 4, 6, 6, 8, 1024]
