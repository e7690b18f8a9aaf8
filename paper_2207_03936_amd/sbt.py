"""Python binding of ``libsbt.so`` (include/sbt.h): argument marshalling only.

Every step of the reconstruction runs in the library's HIP kernels; this
module fills the C structs, allocates device buffers with torch and passes
torch's current stream.  It never computes tracks itself: if the library is
not built, or no GPU is present, the calls raise.

The functions carry the C names (``sbt_reconstruct``,
``sbt_reconstruct_batched``, ``sbt_context_create`` ...).  ``DeviceBatch``
and ``DeviceTracks`` hold the device buffers of one call.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsbt.so")

MAX_MODULES = 64
SBT_OK = 0
SBT_ERR_INVALID_ARG = -1
SBT_ERR_EVENT_TOO_LARGE = -2
SBT_ERR_HIP = -3
SBT_ERR_WORKSPACE = -4
SBT_ERR_NOMEM = -5
SBT_ERR_NOT_READY = -6
SBT_EV_TOO_LARGE = 1
SBT_EV_BAD_OFFSETS = 2
SBT_EV_INTERNAL = 4
SBT_EV_CUT = 8

DEFAULT_PARAMS = dict(
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


class SbtParams(ctypes.Structure):
    _fields_ = [("n_modules", ctypes.c_int32),
                ("module_z", ctypes.c_float * MAX_MODULES),
                ("reverse", ctypes.c_int32),
                ("max_doublet_candidates", ctypes.c_int32),
                ("phi_window_seeding", ctypes.c_int32),
                ("phi_window_forwarding", ctypes.c_int32),
                ("max_scatter_seeding", ctypes.c_float),
                ("max_scatter_forwarding", ctypes.c_float),
                ("max_tracklet_chi2", ctypes.c_float),
                ("max_consecutive_misses", ctypes.c_int32),
                ("max_event_hits", ctypes.c_int32)]


class SbtHits(ctypes.Structure):
    _fields_ = [("n_events", ctypes.c_int32), ("n_hits", ctypes.c_int32),
                ("event_offsets", ctypes.c_void_p), ("module_offsets", ctypes.c_void_p),
                ("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("z", ctypes.c_void_p)]


class SbtHitsF16(ctypes.Structure):
    _fields_ = [("n_events", ctypes.c_int32), ("n_hits", ctypes.c_int32),
                ("event_offsets", ctypes.c_void_p), ("module_offsets", ctypes.c_void_p),
                ("xyzw", ctypes.c_void_p)]


class SbtTracks(ctypes.Structure):
    _fields_ = [("event_track_offsets", ctypes.c_void_p), ("track_hit_offsets", ctypes.c_void_p),
                ("track_hits", ctypes.c_void_p), ("event_status", ctypes.c_void_p)]


class SbtTrackStates(ctypes.Structure):
    _fields_ = [("hit_x", ctypes.c_void_p), ("hit_y", ctypes.c_void_p), ("hit_z", ctypes.c_void_p),
                ("state", ctypes.c_void_p)]


class SbtTuning(ctypes.Structure):
    _fields_ = [("threads_per_event", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("lds_window_hits", ctypes.c_int32), ("lds_owner_hits", ctypes.c_int32),
                ("events_per_block", ctypes.c_int32), ("deferred_window_hits", ctypes.c_int32)]

    def as_dict(self):
        return dict(threads_per_event=self.threads_per_event, blocks_per_cu=self.blocks_per_cu,
                    lds_window_hits=self.lds_window_hits, lds_owner_hits=self.lds_owner_hits,
                    events_per_block=max(1, self.events_per_block), deferred_window_hits=self.deferred_window_hits)


class SbtGraphStats(ctypes.Structure):
    _fields_ = [("cached", ctypes.c_int32), ("capacity", ctypes.c_int32), ("captures", ctypes.c_int64),
                ("replays", ctypes.c_int64), ("evictions", ctypes.c_int64), ("direct", ctypes.c_int64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class SbtServerConfig(ctypes.Structure):
    _fields_ = [("device_budget_bytes", ctypes.c_size_t), ("n_slots", ctypes.c_int32),
                ("slot_events", ctypes.c_int32), ("slot_hits", ctypes.c_int32),
                ("max_wait_us", ctypes.c_int32), ("coords_f16", ctypes.c_int32)]


class SbtServerResult(ctypes.Structure):
    _fields_ = [("request_id", ctypes.c_int64), ("status", ctypes.c_int32), ("n_tracks", ctypes.c_int32),
                ("track_hit_offsets", ctypes.POINTER(ctypes.c_int32)),
                ("track_hits", ctypes.POINTER(ctypes.c_int32)),
                ("t_submit_us", ctypes.c_double), ("t_done_us", ctypes.c_double)]


# exported symbols and their prototypes (restype, argtypes)
_P = ctypes.POINTER
_VP = ctypes.c_void_p
PROTOTYPES = {
    "sbt_error_string": (ctypes.c_char_p, [ctypes.c_int]),
    "sbt_params_validate": (ctypes.c_int, [_P(SbtParams)]),
    "sbt_validate_offsets_host": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                 _P(ctypes.c_int32), _P(ctypes.c_int32)]),
    "sbt_workspace_size": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, _P(ctypes.c_size_t)]),
    "sbt_reconstruct": (ctypes.c_int, [_P(SbtParams), _P(SbtHits), _P(SbtTracks), _VP, ctypes.c_size_t, _VP]),
    "sbt_context_create": (ctypes.c_int, [_P(SbtParams), _P(SbtTuning), ctypes.c_int32, ctypes.c_int32, _P(_VP)]),
    "sbt_context_destroy": (None, [_VP]),
    "sbt_context_set_tuning": (ctypes.c_int, [_VP, _P(SbtTuning)]),
    "sbt_context_get_tuning": (ctypes.c_int, [_VP, _P(SbtTuning)]),
    "sbt_reconstruct_batched": (ctypes.c_int, [_VP, _P(SbtHits), _P(SbtTracks), _VP]),
    "sbt_reconstruct_batched_f16": (ctypes.c_int, [_VP, _P(SbtHitsF16), _P(SbtTracks), _VP]),
    "sbt_reconstruct_batched_static": (ctypes.c_int, [_P(SbtParams), _P(SbtHits), _P(SbtTracks), _VP]),
    "sbt_autotune": (ctypes.c_int, [_VP, _P(SbtHits), _P(SbtTracks), _VP, ctypes.c_int32, _P(SbtTuning),
                                    _P(ctypes.c_float)]),
    "sbt_context_set_profiling": (ctypes.c_int, [_VP, ctypes.c_int32]),
    "sbt_context_stage_ms": (ctypes.c_int, [_VP, _P(ctypes.c_float), ctypes.c_int32]),
    "sbt_context_graph_stats": (ctypes.c_int, [_VP, _P(SbtGraphStats)]),
    "sbt_debug_reconstruct_fill_candidates": (ctypes.c_int, [_P(SbtParams), _P(SbtHits), _P(SbtTracks), _VP,
                                                             ctypes.c_size_t, _VP]),
    "sbt_debug_phi_sort": (ctypes.c_int, [_P(SbtParams), _P(SbtHits), _VP, _VP, _VP, ctypes.c_size_t, _VP]),
    "sbt_debug_phi_sort_rank": (ctypes.c_int, [_P(SbtParams), _P(SbtHits), _VP, _VP, _VP, ctypes.c_size_t, _VP]),
    "sbt_debug_half_records": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int32, _VP]),
    "sbt_server_create": (ctypes.c_int, [_P(SbtParams), _P(SbtTuning), _P(SbtServerConfig), _P(_VP)]),
    "sbt_server_destroy": (None, [_VP]),
    "sbt_server_submit": (ctypes.c_int, [_VP, ctypes.c_int64, ctypes.c_int32, _P(ctypes.c_int32),
                                         _P(ctypes.c_float), _P(ctypes.c_float), _P(ctypes.c_float)]),
    "sbt_server_poll": (ctypes.c_int, [_VP, _P(SbtServerResult), ctypes.c_int32, ctypes.c_int32]),
    "sbt_server_pending": (ctypes.c_int, [_VP, _P(ctypes.c_int32), _P(ctypes.c_int32)]),
    "sbt_server_result_blocks": (ctypes.c_int, [_VP, _P(ctypes.c_int32), _P(ctypes.c_int32)]),
    "sbt_server_replay": (ctypes.c_int, [_VP, ctypes.c_int32, _P(ctypes.c_double), _P(ctypes.c_int32),
                                         ctypes.c_int32, _P(ctypes.c_int32), _P(ctypes.c_int32),
                                         _P(ctypes.c_float), _P(ctypes.c_float), _P(ctypes.c_float),
                                         _P(ctypes.c_double), _P(ctypes.c_int32), _P(ctypes.c_double)]),
    "sbt_now_us": (ctypes.c_double, []),
    "sbt_gec_threshold": (ctypes.c_int, [ctypes.c_int32, _P(ctypes.c_int32), ctypes.c_double, _P(ctypes.c_int32)]),
    "sbt_consolidate": (ctypes.c_int, [_P(SbtHits), _P(SbtTracks), _P(SbtTrackStates), _VP]),
}

_lib = None


def lib():
    """Load libsbt.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2207_03936_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in PROTOTYPES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class SbtError(RuntimeError):
    def __init__(self, code, what=""):
        msg = lib().sbt_error_string(code).decode()
        super().__init__(f"{what}: {msg} ({code})" if what else f"{msg} ({code})")
        self.code = code


def _check(code, what=""):
    if code != SBT_OK:
        raise SbtError(code, what)
    return code


def make_params(module_z, **overrides) -> SbtParams:
    p = dict(DEFAULT_PARAMS)
    p.update(overrides)
    module_z = np.asarray(module_z, dtype=np.float32)
    sp = SbtParams()
    sp.n_modules = int(module_z.size)
    for k, v in enumerate(module_z):
        sp.module_z[k] = float(v)
    for key in DEFAULT_PARAMS:
        setattr(sp, key, p[key])
    return sp


def make_tuning(threads_per_event=512, blocks_per_cu=2, lds_window_hits=672, lds_owner_hits=16384,
                events_per_block=1, deferred_window_hits=0) -> SbtTuning:
    t = SbtTuning()
    t.threads_per_event = threads_per_event
    t.blocks_per_cu = blocks_per_cu
    t.lds_window_hits = lds_window_hits
    t.lds_owner_hits = lds_owner_hits
    t.events_per_block = events_per_block
    t.deferred_window_hits = deferred_window_hits
    return t


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU available: the Search by triplet library runs only on the device")
    return torch


def _stream_handle(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class DeviceBatch:
    """Device copy of a packed batch (any object with x, y, z, event_offsets,
    module_offsets): the sbt_hits of a call."""

    def __init__(self, batch, device="cuda"):
        torch = _torch()
        self.n_events = int(batch.event_offsets.shape[0] - 1)
        self.n_hits = int(batch.event_offsets[-1]) if self.n_events > 0 else 0
        self.n_modules = int(batch.module_z.shape[0])
        self.module_z = np.asarray(batch.module_z, dtype=np.float32)

        def dev(a, dt):
            t = torch.from_numpy(np.ascontiguousarray(a, dtype=dt))
            if t.numel() == 0:
                t = torch.zeros(1, dtype=t.dtype)
            return t.to(device)
        self.x = dev(batch.x, np.float32)
        self.y = dev(batch.y, np.float32)
        self.z = dev(batch.z, np.float32)
        self.eo = dev(batch.event_offsets, np.int32)
        self.mo = dev(batch.module_offsets, np.int32)
        self.hits = SbtHits(self.n_events, self.n_hits, self.eo.data_ptr(), self.mo.data_ptr(),
                            self.x.data_ptr(), self.y.data_ptr(), self.z.data_ptr())


def to_f16_aos(x, y, z) -> np.ndarray:
    """Hit coordinates as binary16 (IEEE round to nearest even) in array-of-
    structures form: [n, 4] uint16 bit patterns x, y, z, 0."""
    n = int(np.asarray(x).shape[0])
    out = np.zeros((n, 4), np.float16)
    out[:, 0] = np.asarray(x, np.float32)
    out[:, 1] = np.asarray(y, np.float32)
    out[:, 2] = np.asarray(z, np.float32)
    return out.view(np.uint16)


def half_records(x, y, z) -> np.ndarray:
    """The server's host conversion for binary16 transfer (sbt_debug_half_records):
    [n, 4] uint16 records x, y, z, 0, each rounded to the nearest binary16."""
    x = np.ascontiguousarray(x, np.float32)
    y = np.ascontiguousarray(y, np.float32)
    z = np.ascontiguousarray(z, np.float32)
    n = int(x.shape[0])
    assert y.shape == (n,) and z.shape == (n,)
    out = np.full((n, 4), 0xFFFF, np.uint16)
    _check(lib().sbt_debug_half_records(x.ctypes.data, y.ctypes.data, z.ctypes.data, n, out.ctypes.data),
           "sbt_debug_half_records")
    return out


class DeviceBatchF16:
    """Device copy of a batch with binary16 array-of-structures coordinates
    (the sbt_hits_f16 of a call); xyzw: a [n, 4] uint16 array from
    to_f16_aos, or None to convert the batch's binary32 coordinates."""

    def __init__(self, batch, xyzw=None, device="cuda"):
        torch = _torch()
        self.n_events = int(batch.event_offsets.shape[0] - 1)
        self.n_hits = int(batch.event_offsets[-1]) if self.n_events > 0 else 0
        self.n_modules = int(batch.module_z.shape[0])
        self.module_z = np.asarray(batch.module_z, dtype=np.float32)
        if xyzw is None:
            xyzw = to_f16_aos(batch.x, batch.y, batch.z)
        assert xyzw.shape == (self.n_hits, 4) and xyzw.dtype == np.uint16

        def dev(a, dt):
            t = torch.from_numpy(np.ascontiguousarray(a, dtype=dt))
            if t.numel() == 0:
                t = torch.zeros(1, dtype=t.dtype)
            return t.to(device)
        # int16 on the device (torch has no uint16 tensors); the bits are what count
        self.xyzw = dev(xyzw.reshape(-1).view(np.int16), np.int16)
        self.eo = dev(batch.event_offsets, np.int32)
        self.mo = dev(batch.module_offsets, np.int32)
        self.hits = SbtHitsF16(self.n_events, self.n_hits, self.eo.data_ptr(), self.mo.data_ptr(),
                               self.xyzw.data_ptr())


class DeviceTracks:
    """Output buffers sized for a batch: the sbt_tracks of a call.  With
    pinned=True they are pinned host memory that the kernels write directly
    (read them after synchronising the stream of the call)."""

    def __init__(self, n_events, n_hits, device="cuda", pinned=False):
        torch = _torch()
        self.n_events, self.n_hits = int(n_events), int(n_hits)
        kw = dict(dtype=torch.int32, pin_memory=True) if pinned else dict(dtype=torch.int32, device=device)
        self.eto = torch.zeros(self.n_events + 1, **kw)
        self.tho = torch.zeros(self.n_hits // 3 + 1, **kw)
        self.th = torch.zeros(max(self.n_hits, 1), **kw)
        self.status = torch.zeros(max(self.n_events, 1), **kw)
        self.tracks = SbtTracks(self.eto.data_ptr(), self.tho.data_ptr(), self.th.data_ptr(),
                                self.status.data_ptr())

    def fill_(self, value=-7):
        for t in (self.eto, self.tho, self.th, self.status):
            t.fill_(value)
        return self

    def to_host(self):
        """(event_track_offsets, track_hit_offsets, track_hits, event_status),
        trimmed, as int32 numpy arrays (synchronises)."""
        eto = self.eto.cpu().numpy()
        T = int(eto[-1])
        tho = self.tho[:T + 1].cpu().numpy()
        th = self.th[:int(tho[-1])].cpu().numpy()
        return eto, tho, th, self.status[:self.n_events].cpu().numpy()


# ------------------------------------------------------------------ plain form

def sbt_workspace_size(n_events, n_hits) -> int:
    n = ctypes.c_size_t(0)
    _check(lib().sbt_workspace_size(int(n_events), int(n_hits), ctypes.byref(n)), "sbt_workspace_size")
    return int(n.value)


class Workspace:
    def __init__(self, n_events, n_hits, device="cuda"):
        torch = _torch()
        self.bytes = sbt_workspace_size(n_events, n_hits)
        self.buf = torch.empty(self.bytes + 256, dtype=torch.uint8, device=device)
        base = self.buf.data_ptr()
        self.ptr = (base + 255) & ~255


def sbt_reconstruct(params: SbtParams, batch: DeviceBatch, out: Optional[DeviceTracks] = None,
                    workspace: Optional[Workspace] = None, stream=None) -> DeviceTracks:
    """Plain per-event kernels (asynchronous on torch's current stream)."""
    out = out or DeviceTracks(batch.n_events, batch.n_hits)
    ws = workspace or Workspace(batch.n_events, batch.n_hits)
    _check(lib().sbt_reconstruct(ctypes.byref(params), ctypes.byref(batch.hits), ctypes.byref(out.tracks),
                                 ctypes.c_void_p(ws.ptr), ws.bytes, _stream_handle(stream)), "sbt_reconstruct")
    out._keep = ws
    return out


def sbt_debug_reconstruct_fill_candidates(params: SbtParams, batch: DeviceBatch, out: Optional[DeviceTracks] = None,
                                          workspace: Optional[Workspace] = None, stream=None) -> DeviceTracks:
    """The plain per-event kernels with the separate candidate pass before
    seeding (asynchronous on torch's current stream)."""
    out = out or DeviceTracks(batch.n_events, batch.n_hits)
    ws = workspace or Workspace(batch.n_events, batch.n_hits)
    _check(lib().sbt_debug_reconstruct_fill_candidates(ctypes.byref(params), ctypes.byref(batch.hits),
                                                       ctypes.byref(out.tracks), ctypes.c_void_p(ws.ptr), ws.bytes,
                                                       _stream_handle(stream)),
           "sbt_debug_reconstruct_fill_candidates")
    out._keep = ws
    return out


def sbt_debug_phi_sort(params: SbtParams, batch: DeviceBatch, stream=None, method: str = "bucket",
                       workspace: Optional[Workspace] = None, out=None, to_host: bool = True):
    """(phi16, ids) of every hit position after the per-module phi sort;
    method "rank" runs the paper's insertion-rank sort instead.  With
    to_host=False the device tensors are returned without synchronising."""
    torch = _torch()
    ws = workspace or Workspace(batch.n_events, batch.n_hits)
    if out is None:
        out = (torch.zeros(max(batch.n_hits, 1), dtype=torch.int16, device="cuda"),
               torch.zeros(max(batch.n_hits, 1), dtype=torch.int16, device="cuda"))
    phi, ids = out
    name = {"bucket": "sbt_debug_phi_sort", "rank": "sbt_debug_phi_sort_rank"}[method]
    _check(getattr(lib(), name)(ctypes.byref(params), ctypes.byref(batch.hits),
                                ctypes.c_void_p(phi.data_ptr()), ctypes.c_void_p(ids.data_ptr()),
                                ctypes.c_void_p(ws.ptr), ws.bytes, _stream_handle(stream)), name)
    if not to_host:
        return phi, ids
    n = batch.n_hits
    return (phi[:n].cpu().numpy().view(np.uint16), ids[:n].cpu().numpy().view(np.uint16))


STATIC_SCRATCH_BYTES = 64 << 20


def sbt_reconstruct_batched_static(params: SbtParams, batch: DeviceBatch, out: Optional[DeviceTracks] = None,
                                   stream=None) -> DeviceTracks:
    """The batched form with the library's static scratch as its workspace
    (no allocation inside the call; asynchronous on torch's current stream)."""
    out = out or DeviceTracks(batch.n_events, batch.n_hits)
    _check(lib().sbt_reconstruct_batched_static(ctypes.byref(params), ctypes.byref(batch.hits),
                                                ctypes.byref(out.tracks), _stream_handle(stream)),
           "sbt_reconstruct_batched_static")
    return out


# ------------------------------------------------------------------ sequence steps

def sbt_gec_threshold(event_offsets, fraction: float) -> int:
    """Hit-count threshold of the global event cut (host computation)."""
    eo = np.ascontiguousarray(event_offsets, dtype=np.int32)
    out = ctypes.c_int32(0)
    _check(lib().sbt_gec_threshold(int(eo.size - 1), eo.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                   float(fraction), ctypes.byref(out)), "sbt_gec_threshold")
    return int(out.value)


class TrackStates:
    """Output buffers of sbt_consolidate sized for a batch of n_hits hits."""

    def __init__(self, n_hits, device="cuda", pinned=False):
        torch = _torch()
        kw = dict(dtype=torch.float32, pin_memory=True) if pinned else dict(dtype=torch.float32, device=device)
        n = max(int(n_hits), 1)
        self.hit_x = torch.zeros(n, **kw)
        self.hit_y = torch.zeros(n, **kw)
        self.hit_z = torch.zeros(n, **kw)
        self.state = torch.zeros(6 * max(int(n_hits) // 3, 1), **kw)
        self.states = SbtTrackStates(self.hit_x.data_ptr(), self.hit_y.data_ptr(), self.hit_z.data_ptr(),
                                     self.state.data_ptr())

    def to_host(self, n_tracks, n_track_hits):
        """(hit_x, hit_y, hit_z, state[n_tracks, 6]) trimmed, as numpy (synchronises)."""
        a = int(n_track_hits)
        return (self.hit_x[:a].cpu().numpy(), self.hit_y[:a].cpu().numpy(), self.hit_z[:a].cpu().numpy(),
                self.state[:6 * int(n_tracks)].cpu().numpy().reshape(-1, 6))


def sbt_consolidate(batch: DeviceBatch, tracks: DeviceTracks, out: Optional[TrackStates] = None,
                    stream=None) -> TrackStates:
    """Packed track coordinates and straight-line states (asynchronous)."""
    out = out or TrackStates(batch.n_hits)
    _check(lib().sbt_consolidate(ctypes.byref(batch.hits), ctypes.byref(tracks.tracks), ctypes.byref(out.states),
                                 _stream_handle(stream)), "sbt_consolidate")
    return out


# ------------------------------------------------------------------ batched form

class Context:
    """sbt_context: workspace, launch configuration and graph cache."""

    def __init__(self, params: SbtParams, max_events: int, max_hits: int, tuning: Optional[SbtTuning] = None):
        _torch()
        self.params = params
        h = ctypes.c_void_p(0)
        _check(lib().sbt_context_create(ctypes.byref(params), ctypes.byref(tuning) if tuning else None,
                                        int(max_events), int(max_hits), ctypes.byref(h)), "sbt_context_create")
        self.handle = h

    def close(self):
        if self.handle:
            lib().sbt_context_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_tuning(self, tuning: SbtTuning):
        _check(lib().sbt_context_set_tuning(self.handle, ctypes.byref(tuning)), "sbt_context_set_tuning")

    def get_tuning(self) -> SbtTuning:
        t = SbtTuning()
        _check(lib().sbt_context_get_tuning(self.handle, ctypes.byref(t)), "sbt_context_get_tuning")
        return t

    def set_profiling(self, on: bool):
        _check(lib().sbt_context_set_profiling(self.handle, 1 if on else 0), "sbt_context_set_profiling")

    def stage_ms(self):
        arr = (ctypes.c_float * 3)()
        _check(lib().sbt_context_stage_ms(self.handle, arr, 3), "sbt_context_stage_ms")
        return [float(v) for v in arr]

    def graph_stats(self) -> dict:
        """The graph cache's counters (sbt_context_graph_stats)."""
        st = SbtGraphStats()
        _check(lib().sbt_context_graph_stats(self.handle, ctypes.byref(st)), "sbt_context_graph_stats")
        return st.as_dict()

    def reconstruct(self, batch: DeviceBatch, out: Optional[DeviceTracks] = None, stream=None) -> DeviceTracks:
        out = out or DeviceTracks(batch.n_events, batch.n_hits)
        _check(lib().sbt_reconstruct_batched(self.handle, ctypes.byref(batch.hits), ctypes.byref(out.tracks),
                                             _stream_handle(stream)), "sbt_reconstruct_batched")
        return out

    def reconstruct_f16(self, batch: DeviceBatchF16, out: Optional[DeviceTracks] = None,
                        stream=None) -> DeviceTracks:
        out = out or DeviceTracks(batch.n_events, batch.n_hits)
        _check(lib().sbt_reconstruct_batched_f16(self.handle, ctypes.byref(batch.hits), ctypes.byref(out.tracks),
                                                 _stream_handle(stream)), "sbt_reconstruct_batched_f16")
        return out

    def autotune(self, sample: DeviceBatch, reps: int = 3, stream=None, cache: bool = True):
        """Time the launch configurations on `sample` and install the fastest.
        With cache, a result stored for the same GPU architecture and batch
        shape (events, mean and largest event size, in coarse buckets) is
        installed without timing; new results are stored.  Returns
        (SbtTuning, ms per launch or None when taken from the cache)."""
        key = _tune_key(sample) if cache else None
        if key is not None:
            hit = _tune_cache_get(key)
            if hit is not None:
                t = make_tuning(**hit)
                self.set_tuning(t)
                return t, None
        out = DeviceTracks(sample.n_events, sample.n_hits)
        best = SbtTuning()
        ms = ctypes.c_float(0)
        _check(lib().sbt_autotune(self.handle, ctypes.byref(sample.hits), ctypes.byref(out.tracks),
                                  _stream_handle(stream), int(reps), ctypes.byref(best), ctypes.byref(ms)),
               "sbt_autotune")
        if key is not None:
            _tune_cache_put(key, best.as_dict())
        return best, float(ms.value)


# ------------------------------------------------------------------ autotune cache
# JSON file: {"<arch>|E<bucket>|N<bucket>|X<bucket>": tuning dict}.  The
# location is $SBT_TUNE_CACHE, else ~/.cache/sbt/tuning.json.

def _tune_cache_path() -> str:
    return os.environ.get("SBT_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "sbt", "tuning.json"))


def _bucket(v: float) -> int:
    """Coarse bucket: nearest power of sqrt(2), rounded to an integer."""
    import math
    v = max(1.0, float(v))
    return int(round(2.0 ** (round(2.0 * math.log2(v)) / 2.0)))


def _tune_key(sample: "DeviceBatch"):
    torch = _torch()
    arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]
    eo = sample.eo.cpu().numpy()[:sample.n_events + 1]
    mo = sample.mo.cpu().numpy()[:sample.n_events * sample.n_modules + 1]
    sizes = np.diff(eo)
    mean = float(sizes.mean()) if sizes.size else 0.0
    big = int(np.diff(mo).max()) if mo.size > 1 else 0
    return f"{arch}|E{_bucket(sample.n_events)}|N{_bucket(mean)}|X{_bucket(big)}"


def _tune_cache_get(key):
    import json
    try:
        with open(_tune_cache_path()) as f:
            return json.load(f).get(key)
    except (OSError, ValueError):
        return None


def _tune_cache_put(key, value):
    import json
    path = _tune_cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        try:
            with open(path) as f:
                data = json.load(f)
        except (OSError, ValueError):
            data = {}
        data[key] = value
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def sbt_context_create(params, max_events, max_hits, tuning=None) -> Context:
    return Context(params, max_events, max_hits, tuning)


def sbt_reconstruct_batched(ctx: Context, batch: DeviceBatch, out=None, stream=None) -> DeviceTracks:
    return ctx.reconstruct(batch, out, stream)


def sbt_autotune(ctx: Context, sample: DeviceBatch, reps=3, stream=None):
    return ctx.autotune(sample, reps, stream)


# ------------------------------------------------------------------ serving

class Server:
    """sbt_server: continuous batching over resident device slots."""

    def __init__(self, params: SbtParams, device_budget_bytes: int, n_slots: int = 4, slot_events: int = 256,
                 slot_hits: int = 1 << 21, max_wait_us: int = 200, tuning: Optional[SbtTuning] = None,
                 coords_f16: bool = False):
        """coords_f16: hits travel to the device as binary16 (rounded on the
        host); results are those of the rounded hits."""
        _torch()
        self.n_modules = params.n_modules
        cfg = SbtServerConfig(int(device_budget_bytes), int(n_slots), int(slot_events), int(slot_hits),
                              int(max_wait_us), 1 if coords_f16 is True else int(coords_f16))
        h = ctypes.c_void_p(0)
        _check(lib().sbt_server_create(ctypes.byref(params), ctypes.byref(tuning) if tuning else None,
                                       ctypes.byref(cfg), ctypes.byref(h)), "sbt_server_create")
        self.handle = h
        self._res = (SbtServerResult * 1024)()

    def close(self):
        if self.handle:
            lib().sbt_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, request_id, module_offsets, x, y, z) -> int:
        mo = np.ascontiguousarray(module_offsets, dtype=np.int32)
        x = np.ascontiguousarray(x, dtype=np.float32)
        y = np.ascontiguousarray(y, dtype=np.float32)
        z = np.ascontiguousarray(z, dtype=np.float32)
        f = ctypes.POINTER(ctypes.c_float)
        return lib().sbt_server_submit(self.handle, int(request_id), int(x.size),
                                       mo.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                       x.ctypes.data_as(f), y.ctypes.data_as(f), z.ctypes.data_as(f))

    def poll(self, wait_us: int = 0, max_results: Optional[int] = None):
        """List of (request_id, status, track_hit_offsets, track_hits,
        t_submit_us, t_done_us) for the events completed so far (at most
        max_results of them)."""
        cap = len(self._res) if max_results is None else max(0, min(int(max_results), len(self._res)))
        n = lib().sbt_server_poll(self.handle, self._res, cap, int(wait_us))
        if n < 0:
            raise SbtError(n, "sbt_server_poll")
        out = []
        for i in range(n):
            r = self._res[i]
            nt = r.n_tracks
            tho = np.ctypeslib.as_array(r.track_hit_offsets, shape=(nt + 1,)).copy()
            th = (np.ctypeslib.as_array(r.track_hits, shape=(int(tho[-1]),)).copy()
                  if tho[-1] > 0 else np.zeros(0, np.int32))
            out.append((int(r.request_id), int(r.status), tho, th, float(r.t_submit_us), float(r.t_done_us)))
        return out

    def replay(self, pool, arrival_us, picks):
        """Arrival i is event picks[i] of the host batch `pool`, submitted at
        arrival_us[i] (us from the start); returns (latency_us, n_tracks,
        wall_us)."""
        arr = np.ascontiguousarray(arrival_us, dtype=np.float64)
        pk = np.ascontiguousarray(picks, dtype=np.int32)
        assert arr.size == pk.size
        n = int(arr.size)
        E = int(pool.event_offsets.shape[0] - 1)
        eo = np.ascontiguousarray(pool.event_offsets, dtype=np.int32)
        mo = np.ascontiguousarray(pool.module_offsets, dtype=np.int32)
        x = np.ascontiguousarray(pool.x, dtype=np.float32)
        y = np.ascontiguousarray(pool.y, dtype=np.float32)
        z = np.ascontiguousarray(pool.z, dtype=np.float32)
        lat = np.zeros(n, np.float64)
        nt = np.zeros(n, np.int32)
        wall = ctypes.c_double(0)
        P = ctypes.POINTER
        _check(lib().sbt_server_replay(self.handle, n, arr.ctypes.data_as(P(ctypes.c_double)),
                                       pk.ctypes.data_as(P(ctypes.c_int32)), E,
                                       eo.ctypes.data_as(P(ctypes.c_int32)), mo.ctypes.data_as(P(ctypes.c_int32)),
                                       x.ctypes.data_as(P(ctypes.c_float)), y.ctypes.data_as(P(ctypes.c_float)),
                                       z.ctypes.data_as(P(ctypes.c_float)), lat.ctypes.data_as(P(ctypes.c_double)),
                                       nt.ctypes.data_as(P(ctypes.c_int32)), ctypes.byref(wall)), "sbt_server_replay")
        return lat, nt, float(wall.value)

    def pending(self):
        q, f = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(lib().sbt_server_pending(self.handle, ctypes.byref(q), ctypes.byref(f)), "sbt_server_pending")
        return int(q.value), int(f.value)

    def result_blocks(self):
        """(result blocks held, most the server will hold)."""
        n, cap = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(lib().sbt_server_result_blocks(self.handle, ctypes.byref(n), ctypes.byref(cap)),
               "sbt_server_result_blocks")
        return int(n.value), int(cap.value)


def sbt_now_us() -> float:
    return float(lib().sbt_now_us())
