"""Benchmark: events/s of Search by triplet on one MI355X.

Workload: the fixed batch of 1,000 upgrade-like events (Poisson(7.6)
vertices, Poisson(40) tracks each, 26 planes), synthetic and seeded.  A step
is one pass of the whole hot path (phi sort, seeding and following, tracklet
filter, compaction) over the batch, with inputs and outputs resident in HBM.
`value` is the batched path: the persistent kernel and its tail captured as
one HIP graph and replayed on a stream of its own, in the launch
configuration the library chooses for the batch's size.  Beside it: the same
sequence launched directly (`direct_ms`), per-run HIP-event times (median and
min), the plain per-event kernels on one stream and on 2 and 3 streams over
slices of the batch, and the autotuner's pick.  Further legs, each reported
apart from `value`: the insertion-rank sort beside the bucket sort; the
paper's separate candidate pass before seeding beside the fused search; binary16
input; end to end from pinned host memory (one stream, then three); the
paper's sequence around the method (event cut, transfer, reconstruction,
consolidation); the uneven mu ~ U{1..25} x 10,000 and the dense mu = 30 x
2,000 batches (autotuned, each against the oracle on a sample); a short
serving leg with p50/p99 event latency under continuous batching at 50 % and
at 80 % of its burst rate (and the same with hits sent to the device as
binary16, at 80 % of its own);
and the CPU oracle on a bounded sample of the same events, on one core and
on the host's CPU share.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import re
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
WORKLOADS = {
    "mu7.6": "{E} events, Poisson(7.6) vertices x Poisson(40) tracks, 26 planes, 99% hit efficiency, 1% noise (seed 2)",
    "mu1-25": "{E} events, U{{1..25}} vertices x Poisson(40) tracks, 26 planes, 99% hit efficiency, 1% noise (seed 3)",
    "mu30": "{E} events, Poisson(30) vertices x Poisson(40) tracks, 26 planes, 97% hit efficiency, 5% noise, "
            "20% of tracks kinked by N(0, 2 mrad) (seed 4)",
}
KERNEL = "k_persistent"


def log(msg):
    """Progress line on stderr (the JSON result alone goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def guarded(name, fn, errors):
    """One leg run after the headline: an error of the kinds listed is
    reported in that leg's place in the line instead of ending the run."""
    try:
        return fn()
    except errors as e:
        log(f"{name} failed: {type(e).__name__}: {e}")
        return {"error": f"{type(e).__name__}: {e}"}


def algorithmic_bytes(batch, eto, tho) -> int:
    """Bytes the method must move for a batch: hits in (3 x 4 B), module and
    event offsets in (4 B each), track hit ids and track offsets out (4 B
    each)."""
    H = batch.n_hits
    E = batch.n_events
    M = batch.n_modules
    T = int(eto[-1])
    assigned = int(tho[T])
    return 12 * H + 4 * (E * M + 1) + 4 * (E + 1) + 4 * assigned + 4 * (T + 1) + 4 * (E + 1)


def _code_only(text: str) -> str:
    """Source text without comments and with whitespace collapsed, so that a
    change of comments alone leaves the hash as it was."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def _layouts(text: str) -> str:
    """The constants and struct layouts of a header, comments left out:
    what device code compiles against (function declarations generate no
    code)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    parts = re.findall(r"^[ \t]*#define[^\n]*", text, flags=re.M)
    parts += re.findall(r"typedef\s+struct\b.*?\}\s*\w+\s*;", text, flags=re.S)
    return " ".join(" ".join(parts).split())


def kernel_source_hash() -> str:
    """Hash of the code the batched kernels are compiled from: the
    persistent kernel's translation unit, the device header, the kernel
    table, the public header's constants and argument layouts, and the
    event-ordering kernel that runs before it (k_prepare, in sbt.hip),
    comments left out.
    Host-side code elsewhere in sbt.hip does not enter, so that an unrelated
    change does not void the committed counter summaries."""
    csrc = os.path.join(ROOT, "paper_2207_03936_amd", "csrc")
    h = hashlib.sha256()
    for f in (os.path.join(csrc, "sbt_device.h"), os.path.join(csrc, "sbt_persistent.hip"),
              os.path.join(csrc, "sbt_kernels.h")):
        with open(f) as fh:
            h.update(_code_only(fh.read()).encode())
    with open(os.path.join(ROOT, "include", "sbt.h")) as fh:
        h.update(_layouts(fh.read()).encode())
    with open(os.path.join(csrc, "sbt.hip")) as fh:
        text = fh.read()
    start = text.index("constexpr int kOrderThreads")
    h.update(_code_only(text[start:text.index("\n}\n", start)]).encode())
    return h.hexdigest()[:16]


def _summary(name, per_launch_hits: int, tuning: dict):
    """A committed counter summary of the dominant kernel, if it was taken on
    the current kernel source, the same batch and the same launch
    configuration (lanes per event, workgroups per CU, LDS slot capacity);
    else None."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_hash") != kernel_source_hash() or d.get("n_hits") != per_launch_hits:
        return None
    if _tuning_key(d.get("tuning", {})) != _tuning_key(tuning):
        return None
    return d


TUNING_KEYS = ("threads_per_event", "blocks_per_cu", "lds_window_hits", "events_per_block", "deferred_window_hits")
_TUNING_DEFAULTS = {"events_per_block": 1, "deferred_window_hits": 0}


def _tuning_key(t: dict):
    """The launch configuration a summary is valid for (events per workgroup
    reads as 1 and the second pass as none where a configuration does not
    name them)."""
    return tuple(int(t.get(k, _TUNING_DEFAULTS[k])) if k in _TUNING_DEFAULTS else t.get(k) for k in TUNING_KEYS)


def measured_traffic(per_launch_hits: int, tuning: dict):
    """Bytes per launch of the dominant kernel between L2 and the memory
    fabric (FETCH_SIZE + WRITE_SIZE, each scaled by what it reads for a copy
    of known size) from the committed summary, or None."""
    d = _summary("k_persistent_mu7.6_x1000_traffic.json", per_launch_hits, tuning)
    return None if d is None else d.get("fabric_bytes_per_launch")


def measured_sq(per_launch_hits: int, tuning: dict):
    """Instruction counts of the dominant kernel from the committed SQ counter
    summary, or None."""
    return _summary("k_persistent_mu7.6_x1000_sq.json", per_launch_hits, tuning)


def host_cpu():
    """CPU model and logical CPU count of this host (lscpu)."""
    model, cpus = None, os.cpu_count()
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() == "Model name":
                model = v.strip()
            elif k.strip() == "CPU(s)":
                cpus = int(v.strip())
    except (OSError, ValueError, subprocess.SubprocessError):
        pass
    return dict(cpu_model=model, host_cpus=cpus)


def copy_bandwidth(torch, mib=1024, reps=10):
    """Device-to-device copy bandwidth measured on this GPU (bytes read plus
    bytes written per second, GB/s)."""
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    b.synchronize()
    sec = a.elapsed_time(b) * 1e-3 / reps
    del src, dst
    return 2 * 4 * n / sec / 1e9


def end_to_end(torch, sbt, params, tuning, batch, steps, pipelined, f16=False, streams=None, d2h=False, lanes=None):
    """Whole-batch rate with the hits in pinned host memory at the start and
    the tracks in pinned host memory at the end: H2D copies of the inputs,
    then the reconstruction, whose kernels write the tracks straight into
    pinned host buffers (no D2H copy queues in the copy engine behind them).
    Sequential: everything on one stream.  Pipelined: one context per stream
    (three by default), so the input copy of one batch overlaps the
    reconstruction of the others; with two, the streams' copies and kernels
    sometimes fell into one order and the rate halved.  The streams should be
    the same for every pipelined leg: HIP maps streams onto a few hardware
    queues (four by default), and streams that share one run their work in a
    single order."""
    def pinned(a, dt):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).pin_memory()
    heo, hmo = pinned(batch.event_offsets, np.int32), pinned(batch.module_offsets, np.int32)
    E, H = batch.n_events, batch.n_hits
    lanes = lanes or (len(streams) if pipelined and streams else (2 if pipelined else 1))
    ctxs = [sbt.Context(params, E, H, tuning) for _ in range(lanes)]
    if f16:
        xyzw = sbt.to_f16_aos(batch.x, batch.y, batch.z)
        hcoords = [pinned(xyzw.reshape(-1).view(np.int16), np.int16)]
        devs = [sbt.DeviceBatchF16(batch, xyzw) for _ in range(lanes)]
        coords = lambda dev: [dev.xyzw]
        run = lambda c, dev, out, st: c.reconstruct_f16(dev, out, st)
        coord_bytes = 8 * H
    else:
        hcoords = [pinned(batch.x, np.float32), pinned(batch.y, np.float32), pinned(batch.z, np.float32)]
        devs = [sbt.DeviceBatch(batch) for _ in range(lanes)]
        coords = lambda dev: [dev.x, dev.y, dev.z]
        run = lambda c, dev, out, st: c.reconstruct(dev, out, st)
        coord_bytes = 12 * H
    outs = [sbt.DeviceTracks(E, H, pinned=not d2h) for _ in range(lanes)]
    if d2h:
        hout = [sbt.DeviceTracks(E, H, pinned=True) for _ in range(lanes)]
    if not pipelined:
        streams = [torch.cuda.current_stream()]
    elif streams is None:
        streams = [torch.cuda.Stream() for _ in range(lanes)]

    def step(k):
        i = k % lanes
        dev, out, st = devs[i], outs[i], streams[i]
        with torch.cuda.stream(st):
            for d, h in list(zip(coords(dev), hcoords)) + [(dev.eo, heo), (dev.mo, hmo)]:
                d.copy_(h, non_blocking=True)
            run(ctxs[i], dev, out, st)
            if d2h:
                for a in ("eto", "tho", "th", "status"):
                    getattr(hout[i], a).copy_(getattr(out, a), non_blocking=True)
    for k in range(2 * lanes):
        step(k)
    torch.cuda.synchronize()
    T = int(outs[0].eto[-1])
    A = int(outs[0].tho[T])
    if d2h:
        T, A = int(hout[0].eto[-1]), int(hout[0].tho[T])
    t0 = time.perf_counter()
    for k in range(steps):
        step(k)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    for c in ctxs:
        c.close()
    in_bytes = coord_bytes + 4 * (E + 1) + 4 * batch.module_offsets.shape[0]
    out_bytes = 4 * (E + 1) + 4 * (T + 1) + 4 * A + 4 * E
    return dict(events_per_s=round(E / sec, 1), ms_per_step=round(sec * 1e3, 4),
                pcie_bytes_per_step=int(in_bytes + out_bytes),
                note=(f"{lanes} contexts on {lanes} streams: the input copy of one batch overlaps the reconstruction "
                      "of the others" if pipelined else "H2D copy and reconstruction on one stream") +
                     "; hits in pinned host memory before, tracks written by the kernels into pinned host memory")


def plain_streams_leg(torch, sbt, params, batch, steps, warmup, streams):
    """The paper's way to fill the device with the plain per-event kernels
    (Section 4: t streams, each running the sequence over its own n events):
    the batch split into n_streams contiguous slices, each reconstructed by
    the plain form on a stream of its own, all in flight together."""
    n_streams = len(streams)
    E = batch.n_events
    cuts = np.linspace(0, E, n_streams + 1).astype(int)
    parts = [batch.select(range(cuts[i], cuts[i + 1])) for i in range(n_streams)]
    devs = [sbt.DeviceBatch(b) for b in parts]
    outs = [sbt.DeviceTracks(b.n_events, b.n_hits) for b in parts]
    wss = [sbt.Workspace(b.n_events, b.n_hits) for b in parts]

    def step():
        for i in range(n_streams):
            with torch.cuda.stream(streams[i]):
                sbt.sbt_reconstruct(params, devs[i], outs[i], wss[i], streams[i])
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    return dict(streams=n_streams, events_per_stream=int(cuts[1] - cuts[0]), events_per_s=round(E / sec, 1),
                ms_per_step=round(sec * 1e3, 4))


def sequence_leg(torch, sbt, params, tuning, batch, steps, streams, fraction=0.1):
    """The paper's sequence around the method (Section 4), decoding aside:
    global event cut, H2D copy of the hits from pinned host memory,
    reconstruction, consolidation.  The cut threshold is calibrated once on
    the batch (the sizes are known before transfer) and applied inside the
    reconstruction; cut events still cross PCIe.  Tracks and consolidated
    states stay on the device for the algorithms that follow.  One context per
    stream, so one batch's input copy overlaps the others' kernels.  The rate
    counts every input event, cut or not."""
    import ctypes
    E, H = batch.n_events, batch.n_hits
    cut = sbt.sbt_gec_threshold(batch.event_offsets, fraction)
    p = sbt.SbtParams.from_buffer_copy(params)
    p.max_event_hits = cut
    def pinned(a, dt):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).pin_memory()
    host = [pinned(batch.x, np.float32), pinned(batch.y, np.float32), pinned(batch.z, np.float32),
            pinned(batch.event_offsets, np.int32), pinned(batch.module_offsets, np.int32)]
    lanes = len(streams)
    ctxs = [sbt.Context(p, E, H, tuning) for _ in range(lanes)]
    devs = [sbt.DeviceBatch(batch) for _ in range(lanes)]
    outs = [sbt.DeviceTracks(E, H) for _ in range(lanes)]
    states = [sbt.TrackStates(H) for _ in range(lanes)]

    def step(k):
        i = k % lanes
        dev, st = devs[i], streams[i]
        with torch.cuda.stream(st):
            for d, h in zip([dev.x, dev.y, dev.z, dev.eo, dev.mo], host):
                d.copy_(h, non_blocking=True)
            ctxs[i].reconstruct(dev, outs[i], st)
            sbt.sbt_consolidate(dev, outs[i], states[i], st)
    for k in range(2 * lanes):
        step(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        step(k)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    status = outs[0].status[:E].cpu().numpy()
    n_cut = int((status & sbt.SBT_EV_CUT != 0).sum())
    # device-resident reconstruction and consolidation alone, with the cut
    for _ in range(3):
        ctxs[0].reconstruct(devs[0], outs[0])
        sbt.sbt_consolidate(devs[0], outs[0], states[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctxs[0].reconstruct(devs[0], outs[0])
    torch.cuda.synchronize()
    sec_k = (time.perf_counter() - t0) / steps
    t0 = time.perf_counter()
    for _ in range(steps):
        sbt.sbt_consolidate(devs[0], outs[0], states[0])
    torch.cuda.synchronize()
    sec_c = (time.perf_counter() - t0) / steps
    for c in ctxs:
        c.close()
    return dict(events_per_s=round(E / sec, 1), ms_per_step=round(sec * 1e3, 4),
                reconstruction_ms_device=round(sec_k * 1e3, 4), consolidation_ms_device=round(sec_c * 1e3, 4),
                cut_hits=int(cut),
                events_cut=n_cut, n_tracks=int(outs[0].eto[-1].item()),
                note="global event cut (densest 10 %), H2D copy, reconstruction and consolidation; "
                     f"results stay on the device; {lanes} contexts on {lanes} streams; no decoding step")


def _oracle_slice(args):
    lo, hi, target_s = args
    import oracle
    from paper_2207_03936_amd import synth
    b = _PAR_BATCH.select(range(lo, hi))
    n = 0
    t0 = time.perf_counter()
    while True:
        oracle.reconstruct(b)
        n += hi - lo
        dt = time.perf_counter() - t0
        if dt >= target_s:
            return n, dt


def cpu_parallel_baseline(batch, workload, procs, target_s=6.0):
    """The oracle as it stands, as `procs` independent single-threaded
    processes on disjoint contiguous slices of the batch, each repeating its
    slice for about target_s; aggregate = events done / slowest wall time.
    Runs before the GPU is initialised (fork)."""
    import multiprocessing as mp
    global _PAR_BATCH
    _PAR_BATCH = batch
    E = batch.n_events
    procs = max(1, min(procs, E))
    bounds = [(E * i // procs, E * (i + 1) // procs, target_s) for i in range(procs)]
    with mp.get_context("fork").Pool(procs) as pool:
        res = pool.map(_oracle_slice, bounds)
    n = sum(r[0] for r in res)
    wall = max(r[1] for r in res)
    return dict(value=round(n / wall, 2), unit="events/s", cores=procs, kind="oracle",
                sample=f"{workload} batch split into {procs} contiguous slices, one single-threaded process each, "
                       f"each slice repeated for about {target_s:.0f} s")


_PAR_BATCH = None


def serving_leg(params, seconds, fraction=0.5, coords_f16=False, bytes_per_event=None):
    """Continuous-batching server fed by Poisson arrivals of events from the
    mu ~ U{1..25} serving mixture: saturated throughput first, then latency
    percentiles at `fraction` of it.  coords_f16: hits sent as binary16.
    bytes_per_event: the pool's algorithmic bytes per event, to state the
    sustained rate as a fraction of the HBM bandwidth."""
    from paper_2207_03936_amd import serve_bench, synth
    pool = synth.make_batch("serve", 2000)
    srv = serve_bench.make_server(params, coords_f16=coords_f16)
    sat = serve_bench.saturation(srv, pool, 40_000)
    rate = fraction * sat["sustained_events_per_s"]
    res = serve_bench.run_rate(srv, pool, rate, seconds)
    srv.close()
    res["saturation_events_per_s"] = sat["sustained_events_per_s"]
    res["workload"] = "Poisson arrivals of mu ~ U{1..25} events (pool of 2,000, seed 5)"
    if bytes_per_event:
        gbps = res["sustained_events_per_s"] * bytes_per_event / 1e9
        res["hbm"] = {"algorithmic_bytes_per_event": round(bytes_per_event, 1), "achieved_GBps": round(gbps, 3),
                      "peak_GBps": HBM_PEAK_GBPS, "frac": round(gbps / HBM_PEAK_GBPS, 6)}
    return res


def cpu_baseline(batch, gpu_out, workload="mu7.6", target_s=10.0):
    """The oracle as it stands, single-threaded, on a bounded sample of the
    same events (repeated passes up to about target_s); also confirms the GPU
    track sets on that sample."""
    import oracle
    E = batch.n_events
    n = min(E, 200)
    t = time.perf_counter()
    sub = batch.select(range(n))
    want = oracle.reconstruct(sub)
    dt = time.perf_counter() - t
    per_event = dt / n
    n = min(E, max(n, int(target_s / max(per_event, 1e-6))))
    sub = batch.select(range(n))
    passes, done = 0, 0.0
    t = time.perf_counter()
    while True:
        want = oracle.reconstruct(sub)
        passes += 1
        done = time.perf_counter() - t
        if done >= 0.9 * target_s:
            break
    ok = sample_matches(gpu_out, want, n)
    return dict(value=round(passes * n / done, 2), unit="events/s", cores=1, kind="oracle",
                sample=f"first {n} events of the {workload} batch, {passes} pass(es), single thread",
                hits_per_s=round(passes * int(sub.n_hits) / done, 1), gpu_matches_oracle_on_sample=bool(ok))


def sample_matches(gpu_out, want, n):
    """Whether the first n events of a GPU output equal the oracle's tracks
    for those events (CSR arrays byte for byte)."""
    eto, tho, th = gpu_out[:3]
    T = int(eto[n])
    return bool(np.array_equal(eto[:n + 1], want[0]) and np.array_equal(tho[:T + 1], want[1])
                and np.array_equal(th[:int(tho[T])], want[2]))


def event_times(torch, fn, stream, runs=20, warmup=3):
    """Milliseconds of each of `runs` back-to-back calls, from HIP events
    recorded on `stream` around each call: (median, min)."""
    for _ in range(warmup):
        fn()
    pairs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(runs)]
    for a, b in pairs:
        a.record(stream)
        fn()
        b.record(stream)
    stream.synchronize()
    ms = sorted(a.elapsed_time(b) for a, b in pairs)
    return float(np.median(ms)), float(ms[0])


def kernel_ms(ctx, dev, out, stream, n):
    """Mean milliseconds of the persistent kernel, the scan and the CSR write
    over n direct launches, from the context's HIP events on `stream`."""
    ctx.set_profiling(True)
    stage = np.zeros(3)
    for _ in range(n):
        ctx.reconstruct(dev, out, stream)
        stage += np.array(ctx.stage_ms())
    ctx.set_profiling(False)
    return stage / n


def workload_leg(torch, sbt, batch, workload, steps, warmup, stream, oracle_events):
    """One more batch on the batched path in the autotuner's configuration:
    events/s and hits/s of graph replays (wall clock over `steps`, and the
    median and min of 20 HIP-event-timed runs), the persistent kernel's
    algorithmic HBM rate, the plain per-event kernels, and the GPU's tracks
    against the oracle on the batch's first events."""
    import oracle
    E, H = batch.n_events, batch.n_hits
    params = sbt.make_params(batch.module_z)
    dev = sbt.DeviceBatch(batch)
    out = sbt.DeviceTracks(E, H)
    ctx = sbt.Context(params, E, H)
    rule = ctx.get_tuning().as_dict()
    best, tune_ms = ctx.autotune(dev, reps=2, stream=stream, cache=False)
    tuning = ctx.get_tuning().as_dict()
    run = lambda: ctx.reconstruct(dev, out, stream)
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    med, mn = event_times(torch, run, stream)
    got = out.to_host()
    k = kernel_ms(ctx, dev, out, stream, 5)
    alg = algorithmic_bytes(batch, got[0], got[1])
    ws = sbt.Workspace(E, H)
    plain_steps = max(3, steps // 4)
    sbt.sbt_reconstruct(params, dev, out, ws, stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(plain_steps):
        sbt.sbt_reconstruct(params, dev, out, ws, stream)
    torch.cuda.synchronize()
    sec_plain = (time.perf_counter() - t0) / plain_steps
    plain_same = all(np.array_equal(a, b) for a, b in zip(out.to_host()[:3], got[:3]))
    n = min(E, oracle_events)
    t0 = time.perf_counter()
    want = oracle.reconstruct(batch.select(range(n)))
    cpu_s = time.perf_counter() - t0
    stats = ctx.graph_stats()
    ctx.close()
    del ws
    achieved = alg / (k[0] * 1e-3) / 1e9
    return {"workload": WORKLOADS[workload].format(E=E), "n_events": E, "n_hits": H,
            "events_per_s": round(E / sec, 1), "hits_per_s": round(H / sec, 1), "ms_per_step": round(sec * 1e3, 4),
            "event_timed_ms": {"median": round(med, 4), "min": round(mn, 4), "runs": 20},
            "launch": "graph" if stats["replays"] >= steps else "direct",
            "tuning": tuning, "rule_tuning": rule, "autotune_ms": round(tune_ms, 4),
            "k_persistent_ms": round(float(k[0]), 4),
            "roofline": {"bound": "hbm", "achieved": round(achieved, 3), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBPS, 6), "algorithmic_bytes_per_launch": int(alg)},
            "plain": {"events_per_s": round(E / sec_plain, 1), "ms_per_step": round(sec_plain * 1e3, 4),
                      "equals_batched": bool(plain_same)},
            "n_tracks": int(got[0][-1]),
            "oracle_sample": {"events": n, "gpu_matches": sample_matches(got, want, n),
                              "cpu_events_per_s_1core": round(n / cpu_s, 2)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="mu7.6", choices=["mu7.6", "mu1-25", "mu30"],
                    help="mu7.6: 1,000 events (the headline); mu1-25: 10,000 uneven events; mu30: 2,000 dense events")
    ap.add_argument("--events", type=int, default=0, help="events (0: the workload's size)")
    ap.add_argument("--serve-seconds", type=float, default=5.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-e2e", action="store_true", help="skip the end-to-end legs")
    ap.add_argument("--no-workloads", action="store_true", help="skip the mu1-25 and mu30 legs")
    ap.add_argument("--kernel-only", action="store_true",
                    help="the headline batch alone (graph replays, direct launches, stage timing): for profiles")
    ap.add_argument("--plain-only", action="store_true",
                    help="the plain per-event kernels alone on the headline batch: for profiles")
    ap.add_argument("--tpe", type=int, default=0, help="threads per event (0: the library's choice)")
    ap.add_argument("--bpc", type=int, default=0, help="blocks per CU (with --tpe)")
    ap.add_argument("--cap", type=int, default=672, help="LDS slot capacity in hits (with --tpe/--bpc)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run one elementwise multiply over this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): events are independent, so "
              "several GPUs would each run this same per-GPU path on their own events.", file=sys.stderr)
        sys.exit(2)
    if args.kernel_only or args.plain_only:
        args.no_cpu = args.no_serve = args.no_e2e = args.no_workloads = True

    from paper_2207_03936_amd import synth
    batch = synth.make_batch(args.workload, args.events or None)
    log(f"{args.workload}: {batch.n_events} events, {batch.n_hits} hits")
    cpu_par = None
    cpu_share = 16       # processes a one-GPU host share runs at once
    if not args.no_cpu:
        # before the GPU is touched: the processes are forked
        cpu_par = cpu_parallel_baseline(batch, args.workload, min(cpu_share, os.cpu_count() or 1))
        cpu_par.update(host_cpu())
        log(f"oracle on {cpu_par['cores']} processes: {cpu_par['value']} events/s")
    extra = {}
    if not args.no_workloads:
        extra = {"mu1-25": synth.make_batch("mu1-25"), "mu30": synth.make_batch("mu30")}
        log("mu1-25 and mu30 batches generated")

    import torch
    from paper_2207_03936_amd import sbt
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    E, H = batch.n_events, batch.n_hits
    params = sbt.make_params(batch.module_z)
    dev = sbt.DeviceBatch(batch)
    out = sbt.DeviceTracks(E, H)
    ws = sbt.Workspace(E, H)
    # the headline context: the configuration the library chooses for the
    # batch's size (or one given on the command line)
    ctx = sbt.Context(params, E, H, sbt.make_tuning(args.tpe, args.bpc, args.cap) if args.tpe else None)
    tuning = ctx.get_tuning().as_dict()
    # three streams for every multi-stream leg: with the null stream they take the four hardware
    # queues HIP opens by default, so no two busy streams share a queue
    extra_streams = [torch.cuda.Stream() for _ in range(3)]
    gstream = extra_streams[0]        # non-null: the calls capture and replay a graph
    null = torch.cuda.current_stream()

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    if args.plain_only:
        sec_plain = timed(lambda: sbt.sbt_reconstruct(params, dev, out, ws), args.steps, args.warmup)
        got_plain = out.to_host()
        ctx.close()
        print(json.dumps({"metric": "events/s of the plain per-event kernels", "value": round(E / sec_plain, 1),
                          "unit": "events/s", "steps": args.steps, "warmup": args.warmup,
                          "ms_per_step": round(sec_plain * 1e3, 4), "form": "plain",
                          "config": {"workload": WORKLOADS[args.workload].format(E=E), "n_events": E, "n_hits": H},
                          "n_tracks": int(got_plain[0][-1])}), flush=True)
        return

    # batched: the persistent kernel and its tail replayed as a captured graph
    graph_call = lambda: ctx.reconstruct(dev, out, gstream)
    g0 = ctx.graph_stats()
    sec_batched = timed(graph_call, args.steps, args.warmup)
    g1 = ctx.graph_stats()
    launch = "graph" if g1["replays"] - g0["replays"] >= args.steps and g1["direct"] == g0["direct"] else "direct"
    got = out.to_host()
    med_ms, min_ms = event_times(torch, graph_call, gstream)
    # the same sequence launched directly, on the null stream
    sec_direct = timed(lambda: ctx.reconstruct(dev, out, null), args.steps, args.warmup)
    direct_same = all(np.array_equal(a, b) for a, b in zip(out.to_host()[:3], got[:3]))
    log(f"headline: {sec_batched * 1e3:.4f} ms per batch ({launch}), direct {sec_direct * 1e3:.4f} ms")

    # dominant kernel duration: HIP events around the persistent kernel on the
    # stream it is launched on (profiling mode launches without the graph)
    stage = kernel_ms(ctx, dev, out, gstream, max(5, min(args.steps, 20)))
    k_ms = float(stage[0])
    alg = algorithmic_bytes(batch, got[0], got[1])
    achieved = alg / (k_ms * 1e-3) / 1e9
    traffic = measured_traffic(H, tuning)
    sq = measured_sq(H, tuning)
    copy_gbps = copy_bandwidth(torch)

    result = {
        "metric": "events/s on 1 MI355X at mu=7.6 (batched vs plain) + p99 event latency",
        "value": round(E / sec_batched, 1),
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sec_batched * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload].format(E=E),
                   "n_events": E, "n_hits": H, "tuning": tuning, "launch": launch},
        "hits_per_s": round(H / sec_batched, 1),
        "launch": launch,
        "graph_stats": g1,
        "event_timed_ms": {"median": round(med_ms, 4), "min": round(min_ms, 4), "runs": 20},
        "direct_ms": round(sec_direct * 1e3, 4),
        "direct_equals_graph": bool(direct_same),
        "stage_ms": {"k_persistent": round(k_ms, 4), "k_scan": round(float(stage[1]), 4),
                     "k_write": round(float(stage[2]), 4)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 3), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 6),
                     "traffic": traffic, "algorithmic_bytes_per_launch": int(alg), "kernel": KERNEL,
                     "measured_copy_GBps": round(copy_gbps, 1),
                     "frac_of_measured_copy": round(achieved / copy_gbps, 6)},
        "n_tracks": int(got[0][-1]),
    }
    if sq is not None:
        # VALU issue: a wave64 instruction takes a SIMD for 4 cycles (16 lanes);
        # 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3 T lane-operations/s
        lane_ops = 64.0 * sq["SQ_INSTS_VALU"]
        peak = 256 * 4 * 16 * 2.4e9
        result["valu"] = {"bound": "alu", "achieved": round(lane_ops / (k_ms * 1e-3) / 1e12, 4),
                          "peak": round(peak / 1e12, 2), "unit": "T lane-ops/s",
                          "frac": round(lane_ops / (k_ms * 1e-3) / peak, 4),
                          "valu_instructions_per_launch": int(sq["SQ_INSTS_VALU"]),
                          "salu_instructions_per_launch": int(sq["SQ_INSTS_SALU"]),
                          "lds_instructions_per_launch": int(sq["SQ_INSTS_LDS"])}
    if args.kernel_only:
        if args.calibrate_copy:
            calibrate(torch, args.calibrate_copy, result)
        ctx.close()
        print(json.dumps(result), flush=True)
        return

    # plain per-event kernels
    sec_plain = timed(lambda: sbt.sbt_reconstruct(params, dev, out, ws), args.steps, args.warmup)
    log(f"plain: {sec_plain * 1e3:.4f} ms per batch")
    got_plain = out.to_host()
    same_paths = all(np.array_equal(a, b) for a, b in zip(got[:3], got_plain[:3]))
    plain_multi = [plain_streams_leg(torch, sbt, params, batch, args.steps, args.warmup, extra_streams[:t])
                   for t in (2, 3)]
    # the paper's insertion-rank sort beside the bucket sort (each call: sort kernel + copy-out kernel)
    sort_ms = {}
    sort_out = (torch.zeros(H, dtype=torch.int16, device="cuda"), torch.zeros(H, dtype=torch.int16, device="cuda"))
    for method in ("bucket", "rank"):
        sec = timed(lambda: sbt.sbt_debug_phi_sort(params, dev, method=method, workspace=ws, out=sort_out,
                                                   to_host=False), max(5, args.steps // 2), 2)
        sort_ms[method] = round(sec * 1e3, 4)
    # the paper's separate candidate pass before seeding, on the plain form
    sec_fill = timed(lambda: sbt.sbt_debug_reconstruct_fill_candidates(params, dev, out, ws), args.steps,
                     args.warmup)
    fill_same = all(np.array_equal(a, b) for a, b in zip(out.to_host()[:3], got[:3]))
    log(f"plain with the candidate pass: {sec_fill * 1e3:.4f} ms per batch")
    # the autotuner on the headline batch, in a context of its own
    tctx = sbt.Context(params, E, H)
    best, tuned_ms = tctx.autotune(dev, reps=3, stream=gstream, cache=False)
    tout = sbt.DeviceTracks(E, H)
    sec_tuned = timed(lambda: tctx.reconstruct(dev, tout, gstream), args.steps, args.warmup)
    tuned_same = all(np.array_equal(a, b) for a, b in zip(tout.to_host()[:3], got[:3]))
    autotune = {"tuning": tctx.get_tuning().as_dict(), "autotune_ms": round(tuned_ms, 4),
                "events_per_s": round(E / sec_tuned, 1), "ms_per_step": round(sec_tuned * 1e3, 4),
                "equals_headline": bool(tuned_same)}
    tctx.close()
    del tout
    log(f"autotune picked {autotune['tuning']}: {autotune['ms_per_step']} ms")
    # the legs from here on report a library or runtime error in their place
    errors = (sbt.SbtError, RuntimeError)
    if not args.no_e2e:
        e2e = guarded("end_to_end", lambda: end_to_end(torch, sbt, params, ctx.get_tuning(), batch,
                                                       max(5, min(args.steps, 20)), False), errors)
        pipe_streams = extra_streams
        e2e_p = guarded("end_to_end_pipelined", lambda: end_to_end(
            torch, sbt, params, ctx.get_tuning(), batch, max(10, min(args.steps, 40)), True,
            streams=pipe_streams), errors)
    # half-precision array-of-structures input (the paper's hit-storage optimisation)
    dev16 = sbt.DeviceBatchF16(batch)
    out16 = sbt.DeviceTracks(E, H)
    sec_f16 = timed(lambda: ctx.reconstruct_f16(dev16, out16, gstream), args.steps, args.warmup)
    got16 = out16.to_host()
    if not args.no_e2e:
        e2e_f16 = guarded("end_to_end_f16", lambda: end_to_end(
            torch, sbt, params, ctx.get_tuning(), batch, max(10, min(args.steps, 40)), True, True,
            streams=pipe_streams), errors)
        seq_leg = guarded("sequence", lambda: sequence_leg(torch, sbt, params, ctx.get_tuning(), batch,
                                                           max(10, min(args.steps, 40)), pipe_streams), errors)
    del dev16, out16
    log("binary16, end-to-end and sequence legs done")

    result.update({
        "plain": {"events_per_s": round(E / sec_plain, 1), "ms_per_step": round(sec_plain * 1e3, 4),
                  "hits_per_s": round(H / sec_plain, 1)},
        "plain_streams": plain_multi,
        "sort_ablation": {"bucket_sort_call_ms": sort_ms["bucket"], "insertion_rank_sort_call_ms": sort_ms["rank"],
                          "note": "whole batch; each call is the sort kernel, a copy of the sorted angles and ids, "
                                  "and for the rank sort a host read of the event offsets"},
        "fill_candidates_ablation": {"plain_ms": round(sec_plain * 1e3, 4),
                                     "plain_with_candidate_pass_ms": round(sec_fill * 1e3, 4),
                                     "fused_over_separate": round(sec_fill / sec_plain, 3),
                                     "equals_batched": bool(fill_same),
                                     "note": "plain per-event kernels; the candidate pass writes every hit's "
                                             "pendulum start before the seeding kernel, which reads it instead "
                                             "of searching"},
        "batched_over_plain": round(sec_plain / sec_batched, 3),
        "plain_equals_batched": bool(same_paths),
        "autotune": autotune,
    })
    if not args.no_e2e:
        result["end_to_end"] = e2e
        result["end_to_end_pipelined"] = e2e_p
    result["f16_aos"] = {"events_per_s": round(E / sec_f16, 1), "ms_per_step": round(sec_f16 * 1e3, 4),
                         "input_bytes_per_hit": 8, "n_tracks": int(got16[0][-1]),
                         "note": "binary16 x, y, z, unused per hit, widened exactly on load; tracks equal the "
                                 "binary32 path on the rounded coordinates (GPU parity tests)"}
    if not args.no_e2e:
        result["f16_aos"]["end_to_end_pipelined"] = e2e_f16
        result["sequence"] = seq_leg
    del ws
    ctx.close()
    for name, b in extra.items():
        result[name] = guarded(name, lambda: workload_leg(torch, sbt, b, name, max(5, args.steps // 5), 2, gstream,
                                                          50 if name == "mu1-25" else 20), errors)
        log(f"{name}: {result[name].get('events_per_s')} events/s")
    extra.clear()
    if not args.no_serve:
        # algorithmic bytes per event of the serving pool, from one batched call over it
        pool = synth.make_batch("serve", 2000)
        pctx = sbt.Context(sbt.make_params(pool.module_z), pool.n_events, pool.n_hits)
        pgot = pctx.reconstruct(sbt.DeviceBatch(pool)).to_host()
        pctx.close()
        per_event = algorithmic_bytes(pool, pgot[0], pgot[1]) / pool.n_events
        result["serving"] = guarded("serving", lambda: serving_leg(params, args.serve_seconds,
                                                                   bytes_per_event=per_event), errors)
        result["p99_event_latency_ms"] = result["serving"].get("p99_ms")
        log(f"serving: p99 {result['serving'].get('p99_ms')} ms")
        # the same server closer to its burst saturation
        result["serving_80pct"] = guarded("serving_80pct", lambda: serving_leg(
            params, args.serve_seconds, fraction=0.8, bytes_per_event=per_event), errors)
        log(f"serving at 80 %: p99 {result['serving_80pct'].get('p99_ms')} ms")
        # the same with hits sent to the device as binary16 (results are those
        # of the rounded hits): 80 % of its own burst saturation
        result["serving_f16"] = guarded("serving_f16", lambda: serving_leg(
            params, args.serve_seconds, fraction=0.8, coords_f16=True, bytes_per_event=per_event), errors)
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(batch, got, args.workload)
        result["cpu_baseline"].update(host_cpu())
        result["cpu_baseline_all_cores"] = cpu_par
    if args.calibrate_copy:
        calibrate(torch, args.calibrate_copy, result)
    print(json.dumps(result), flush=True)


def calibrate(torch, mib, result):
    """One elementwise multiply over `mib` MiB, for scaling the fabric
    counters: it reads and writes 4n bytes."""
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 2.0, out=dst)
    torch.cuda.synchronize()
    result["calibration_copy_bytes"] = 4 * n


if __name__ == "__main__":
    main()
