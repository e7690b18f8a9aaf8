"""Search by triplet CPU oracle (test infrastructure only).

Plain single-threaded C (``sbt_oracle.c``) behind ctypes; the steps around
the method in the paper's sequence (global event cut, consolidation) are plain
float64 numpy in ``sequence.py``.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package; the HIP library never
does.

``build()`` compiles ``liboracle.so`` with gcc at -O2, -ffp-contract=off and
no fast-math, so binary32 arithmetic is evaluated exactly as written.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sbt_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_ABI_H = os.path.join(_HERE, "sbt_oracle_abi.h")
_lib = None

# default tolerances (also used by the HIP path's callers); see the design notes
DEFAULTS = dict(
    reverse=1,
    max_doublet_candidates=4,
    phi_window_seeding=416,
    phi_window_forwarding=416,
    max_scatter_seeding=0.04,
    max_scatter_forwarding=0.04,
    max_tracklet_chi2=0.002,
    max_consecutive_misses=1,
    max_event_hits=0,
)


def build() -> str:
    """Compile the oracle shared library (always recompiles)."""
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(_SRC),
                                                                    os.path.getmtime(_ABI_H)):
            build()
        L = ctypes.CDLL(_LIB)
        f32p = ctypes.POINTER(ctypes.c_float)
        i32p = ctypes.POINTER(ctypes.c_int32)
        L.sbt_oracle_phi16.restype = ctypes.c_uint16
        L.sbt_oracle_phi16.argtypes = [ctypes.c_float, ctypes.c_float]
        L.sbt_oracle_phi16_array.restype = None
        L.sbt_oracle_phi16_array.argtypes = [ctypes.c_int64, f32p, f32p, ctypes.POINTER(ctypes.c_uint16)]
        L.sbt_oracle_in_window.restype = ctypes.c_int
        L.sbt_oracle_in_window.argtypes = [ctypes.c_uint16, ctypes.c_uint16, ctypes.c_int32]
        L.sbt_oracle_sort_event.restype = None
        L.sbt_oracle_sort_event.argtypes = [ctypes.c_int, i32p, f32p, f32p, i32p]
        L.sbt_oracle_pendulum.restype = ctypes.c_int
        L.sbt_oracle_pendulum.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_uint16),
                                          ctypes.POINTER(ctypes.c_uint8), ctypes.c_uint16,
                                          ctypes.c_int32, i32p]
        L.sbt_oracle_tracklet_chi2.restype = ctypes.c_float
        L.sbt_oracle_tracklet_chi2.argtypes = [f32p, f32p, f32p]
        L.sbt_reconstruct_cpu.restype = ctypes.c_int
        L.sbt_reconstruct_cpu.argtypes = [ctypes.POINTER(OrcAbiParams), ctypes.POINTER(OrcAbiHits),
                                          ctypes.POINTER(OrcAbiTracks)]
        L.sbt_oracle_reconstruct.restype = ctypes.c_int
        L.sbt_oracle_reconstruct.argtypes = (
            [ctypes.c_int32, f32p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
             ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_int32, ctypes.c_int32,
             ctypes.c_int32, i32p, i32p, f32p, f32p, f32p, i32p, i32p, i32p])
        _lib = L
    return _lib


class OrcAbiParams(ctypes.Structure):
    """orc_abi_params of sbt_oracle_abi.h."""
    _fields_ = [("n_modules", ctypes.c_int32), ("module_z", ctypes.c_float * 64), ("reverse", ctypes.c_int32),
                ("max_doublet_candidates", ctypes.c_int32), ("phi_window_seeding", ctypes.c_int32),
                ("phi_window_forwarding", ctypes.c_int32), ("max_scatter_seeding", ctypes.c_float),
                ("max_scatter_forwarding", ctypes.c_float), ("max_tracklet_chi2", ctypes.c_float),
                ("max_consecutive_misses", ctypes.c_int32), ("max_event_hits", ctypes.c_int32)]


class OrcAbiHits(ctypes.Structure):
    """orc_abi_hits of sbt_oracle_abi.h (host pointers)."""
    _fields_ = [("n_events", ctypes.c_int32), ("n_hits", ctypes.c_int32),
                ("event_offsets", ctypes.c_void_p), ("module_offsets", ctypes.c_void_p),
                ("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("z", ctypes.c_void_p)]


class OrcAbiTracks(ctypes.Structure):
    """orc_abi_tracks of sbt_oracle_abi.h (host pointers)."""
    _fields_ = [("event_track_offsets", ctypes.c_void_p), ("track_hit_offsets", ctypes.c_void_p),
                ("track_hits", ctypes.c_void_p), ("event_status", ctypes.c_void_p)]


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def phi16(x, y) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    out = np.empty(x.shape, dtype=np.uint16)
    lib().sbt_oracle_phi16_array(x.size, _p(x, ctypes.c_float), _p(y, ctypes.c_float),
                                 _p(out, ctypes.c_uint16))
    return out


def in_window(q, centre, w) -> bool:
    return bool(lib().sbt_oracle_in_window(int(q), int(centre), int(w)))


def sort_event(module_offsets_local, x, y) -> np.ndarray:
    """Hit ids of one event, module by module, each ordered by (phi16, id)."""
    mo = np.ascontiguousarray(module_offsets_local, dtype=np.int32)
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    out = np.empty(int(mo[-1]), dtype=np.int32)
    lib().sbt_oracle_sort_event(mo.size - 1, _p(mo, ctypes.c_int32), _p(x, ctypes.c_float),
                                _p(y, ctypes.c_float), _p(out, ctypes.c_int32))
    return out


def pendulum(q_sorted, flagged, target, k) -> np.ndarray:
    q = np.ascontiguousarray(q_sorted, dtype=np.uint16)
    f = np.ascontiguousarray(flagged, dtype=np.uint8)
    out = np.empty(max(q.size, 1), dtype=np.int32)
    n = lib().sbt_oracle_pendulum(q.size, _p(q, ctypes.c_uint16), _p(f, ctypes.c_uint8),
                                  int(target), int(k), _p(out, ctypes.c_int32))
    return out[:n].copy()


def tracklet_chi2(x3, y3, z3) -> float:
    a = [np.ascontiguousarray(v, dtype=np.float32) for v in (x3, y3, z3)]
    return float(lib().sbt_oracle_tracklet_chi2(*[_p(v, ctypes.c_float) for v in a]))


def reconstruct(batch, **overrides):
    """Reconstruct a packed batch (any object with x, y, z, event_offsets,
    module_offsets, module_z).  Returns (event_track_offsets,
    track_hit_offsets, track_hits) as int32 numpy arrays, trimmed."""
    p = dict(DEFAULTS)
    p.update(overrides)
    M = int(batch.module_z.shape[0])
    E = int(batch.event_offsets.shape[0] - 1)
    H = int(batch.event_offsets[-1]) if E > 0 else 0
    mz = np.ascontiguousarray(batch.module_z, dtype=np.float32)
    eo = np.ascontiguousarray(batch.event_offsets, dtype=np.int32)
    mo = np.ascontiguousarray(batch.module_offsets, dtype=np.int32)
    x = np.ascontiguousarray(batch.x, dtype=np.float32)
    y = np.ascontiguousarray(batch.y, dtype=np.float32)
    z = np.ascontiguousarray(batch.z, dtype=np.float32)
    eto = np.zeros(E + 1, dtype=np.int32)
    tho = np.zeros(H // 3 + 1, dtype=np.int32)
    th = np.zeros(max(H, 1), dtype=np.int32)
    rc = lib().sbt_oracle_reconstruct(
        M, _p(mz, ctypes.c_float), int(p["reverse"]), int(p["max_doublet_candidates"]),
        int(p["phi_window_seeding"]), int(p["phi_window_forwarding"]),
        float(p["max_scatter_seeding"]), float(p["max_scatter_forwarding"]),
        float(p["max_tracklet_chi2"]), int(p["max_consecutive_misses"]), int(p["max_event_hits"]),
        E, _p(eo, ctypes.c_int32), _p(mo, ctypes.c_int32),
        _p(x, ctypes.c_float), _p(y, ctypes.c_float), _p(z, ctypes.c_float),
        _p(eto, ctypes.c_int32), _p(tho, ctypes.c_int32), _p(th, ctypes.c_int32))
    if rc != 0:
        raise RuntimeError(f"oracle reconstruct failed: {rc}")
    T = int(eto[-1])
    return eto, tho[:T + 1].copy(), th[:int(tho[T])].copy()


def reconstruct_abi(batch, **overrides):
    """The same reconstruction through the structure entry point
    (sbt_reconstruct_cpu), which also checks every event's offsets and size
    and reports them per event.  Returns (event_track_offsets,
    track_hit_offsets, track_hits, event_status) as int32 numpy arrays,
    trimmed."""
    p = dict(DEFAULTS)
    p.update(overrides)
    mz = np.ascontiguousarray(batch.module_z, dtype=np.float32)
    eo = np.ascontiguousarray(batch.event_offsets, dtype=np.int32)
    mo = np.ascontiguousarray(batch.module_offsets, dtype=np.int32)
    x = np.ascontiguousarray(batch.x, dtype=np.float32)
    y = np.ascontiguousarray(batch.y, dtype=np.float32)
    z = np.ascontiguousarray(batch.z, dtype=np.float32)
    E, H = int(eo.size - 1), int(x.size)
    prm = OrcAbiParams()
    prm.n_modules = int(mz.size)
    for k, v in enumerate(mz):
        prm.module_z[k] = float(v)
    for key in ("reverse", "max_doublet_candidates", "phi_window_seeding", "phi_window_forwarding",
                "max_scatter_seeding", "max_scatter_forwarding", "max_tracklet_chi2", "max_consecutive_misses",
                "max_event_hits"):
        setattr(prm, key, p[key])
    hits = OrcAbiHits(E, H, eo.ctypes.data, mo.ctypes.data, x.ctypes.data, y.ctypes.data, z.ctypes.data)
    eto = np.zeros(E + 1, dtype=np.int32)
    tho = np.zeros(H // 3 + 1, dtype=np.int32)
    th = np.zeros(max(H, 1), dtype=np.int32)
    st = np.zeros(max(E, 1), dtype=np.int32)
    out = OrcAbiTracks(eto.ctypes.data, tho.ctypes.data, th.ctypes.data, st.ctypes.data)
    rc = lib().sbt_reconstruct_cpu(ctypes.byref(prm), ctypes.byref(hits), ctypes.byref(out))
    if rc != 0:
        raise RuntimeError(f"oracle reconstruct failed: {rc}")
    T = int(eto[-1])
    return eto, tho[:T + 1].copy(), th[:int(tho[T])].copy(), st[:E].copy()
