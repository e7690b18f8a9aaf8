"""GPU parity: the HIP library against the oracle, byte for byte.

Every case prints its name before touching the GPU.  Track sets are integer
outputs, so the bar is exact equality of the three CSR arrays.
"""

import os
import sys

import numpy as np
import pytest

import oracle
from _util import event_batch, jet_event, rounded_to_f16, tiny_random_event
from paper_2207_03936_amd import sbt, synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    sbt.lib()
    yield
    torch.cuda.synchronize()


def _same(got, want, what):
    eto, tho, th = want
    g_eto, g_tho, g_th = got[:3]
    assert np.array_equal(g_eto, eto), f"{what}: event track offsets differ"
    assert np.array_equal(g_tho, tho), f"{what}: track hit offsets differ"
    assert np.array_equal(g_th, th), f"{what}: track hits differ"


def _first_diff(got, want):
    eto, tho, th = want
    for e in range(len(eto) - 1):
        a = [tuple(th[tho[t]:tho[t + 1]]) for t in range(eto[e], eto[e + 1])]
        b = [tuple(got[2][got[1][t]:got[1][t + 1]]) for t in range(got[0][e], got[0][e + 1])]
        if a != b:
            return e, a, b
    return None


def run_plain(batch, **kw):
    p = sbt.make_params(batch.module_z, **kw)
    return sbt.sbt_reconstruct(p, sbt.DeviceBatch(batch)).to_host()


def run_batched(batch, tuning=None, **kw):
    p = sbt.make_params(batch.module_z, **kw)
    ctx = sbt.Context(p, max(batch.n_events, 1), max(batch.n_hits, 1), tuning)
    out = ctx.reconstruct(sbt.DeviceBatch(batch)).to_host()
    ctx.close()
    return out


def graph_replays(ctx, dev, out, stream, reps=3, f16=False):
    """The batched call on a non-null stream (captured once, then replayed
    from the context's graph cache), `reps` times; before each call the
    outputs are overwritten on the same stream, and after it the stream is
    synchronised and the outputs read back.  Returns every call's outputs
    and the cache counters after each call."""
    import torch
    got, stats = [], []
    for _ in range(reps):
        with torch.cuda.stream(stream):
            out.fill_(-1)
            if f16:
                ctx.reconstruct_f16(dev, out, stream)
            else:
                ctx.reconstruct(dev, out, stream)
        stream.synchronize()
        got.append(out.to_host())
        stats.append(ctx.graph_stats())
    return got, stats


def check_replays(got, stats, want, what, captures0=0, replays0=0):
    """Every call equals the oracle; the first was captured, the others
    came from the cache."""
    for i, g in enumerate(got):
        _same(g, want, f"{what} graph call {i}")
    assert stats[0]["captures"] == captures0 + 1, stats
    for i, st in enumerate(stats):
        assert st["captures"] == captures0 + 1 and st["replays"] == replays0 + i, stats
        assert st["direct"] == stats[0]["direct"], stats


# ------------------------------------------------------------------ phi sort

@pytest.mark.parametrize("method", ["bucket", "rank"])
@pytest.mark.parametrize("config,n", [("tiny", 8), ("mu7.6", 8), ("mu30", 3)])
def test_phi_sort_matches_oracle(config, n, method):
    say(f"phi sort {config} x{n} ({method})")
    b = synth.make_batch(config, n)
    phi, ids = sbt.sbt_debug_phi_sort(sbt.make_params(b.module_z), sbt.DeviceBatch(b), method=method)
    M = b.n_modules
    for e in range(b.n_events):
        lo, hi = int(b.event_offsets[e]), int(b.event_offsets[e + 1])
        mo = b.module_offsets[e * M:(e + 1) * M + 1] - lo
        want_ids = oracle.sort_event(mo, b.x[lo:hi], b.y[lo:hi])
        want_q = oracle.phi16(b.x[lo:hi], b.y[lo:hi])
        assert np.array_equal(ids[lo:hi], want_ids)
        assert np.array_equal(phi[lo:hi], want_q[want_ids])


# ------------------------------------------------------------------ plain and batched vs oracle

CASES = [("tiny", 20), ("mu7.6", 40), ("mu1-25", 30), ("mu30", 6)]


@pytest.mark.parametrize("config,n", CASES)
def test_plain_matches_oracle(config, n):
    say(f"plain {config} x{n}")
    b = synth.make_batch(config, n)
    want = oracle.reconstruct(b)
    got = run_plain(b)
    assert not got[3].any()
    assert _first_diff(got, want) is None, _first_diff(got, want)
    _same(got, want, f"plain {config}")


@pytest.mark.parametrize("config,n", CASES)
def test_batched_matches_oracle(config, n):
    """Direct launch on the null stream, then the captured graph on a stream
    of its own: three calls, the last two replayed from the cache."""
    import torch
    say(f"batched {config} x{n}")
    b = synth.make_batch(config, n)
    want = oracle.reconstruct(b)
    got = run_batched(b)
    assert not got[3].any()
    assert _first_diff(got, want) is None, _first_diff(got, want)
    _same(got, want, f"batched {config}")
    say(f"batched {config} x{n}: graph replays")
    p = sbt.make_params(b.module_z)
    ctx = sbt.Context(p, b.n_events, b.n_hits)
    dev = sbt.DeviceBatch(b)
    out = sbt.DeviceTracks(b.n_events, b.n_hits)
    got, stats = graph_replays(ctx, dev, out, torch.cuda.Stream())
    assert not any(g[3].any() for g in got)
    check_replays(got, stats, want, f"batched {config}")
    ctx.close()


def test_graph_cache_eviction():
    """More argument sets than the cache holds: the least recently used
    graphs are evicted, an evicted set is captured again, a cached one is
    replayed, and every call gives the oracle's tracks."""
    import torch
    say("graph cache eviction")
    b = synth.make_batch("mu7.6", 12, first=40)
    want = oracle.reconstruct(b)
    p = sbt.make_params(b.module_z)
    ctx = sbt.Context(p, b.n_events, b.n_hits)
    dev = sbt.DeviceBatch(b)
    st = torch.cuda.Stream()
    cap = ctx.graph_stats()["capacity"]
    outs = [sbt.DeviceTracks(b.n_events, b.n_hits) for _ in range(cap + 2)]

    def call(k):
        with torch.cuda.stream(st):
            outs[k].fill_(-1)
            ctx.reconstruct(dev, outs[k], st)
        st.synchronize()
        _same(outs[k].to_host(), want, f"argument set {k}")
    for k in range(cap + 2):          # distinct output buffers: distinct argument sets
        call(k)
    s = ctx.graph_stats()
    assert (s["cached"], s["captures"], s["replays"], s["evictions"]) == (cap, cap + 2, 0, 2), s
    call(cap + 1)                     # most recent: replayed
    s = ctx.graph_stats()
    assert (s["captures"], s["replays"], s["evictions"]) == (cap + 2, 1, 2), s
    call(0)                           # evicted first: captured again, evicting the next oldest
    s = ctx.graph_stats()
    assert (s["cached"], s["captures"], s["replays"], s["evictions"]) == (cap, cap + 3, 1, 3), s
    call(0)
    s = ctx.graph_stats()
    assert (s["captures"], s["replays"]) == (cap + 3, 2), s
    # a new configuration drops the cache; the same set is then captured anew
    ctx.set_tuning(sbt.make_tuning(256, 3, 448))
    assert ctx.graph_stats()["cached"] == 0
    call(0)
    s = ctx.graph_stats()
    assert (s["cached"], s["captures"]) == (1, cap + 4), s
    ctx.close()


@pytest.mark.parametrize("tpe", [64, 128, 256, 512, 1024])
@pytest.mark.parametrize("bpc", [1, 3, 8])
def test_batched_independent_of_launch_configuration(tpe, bpc):
    say(f"batched tuning tpe={tpe} bpc={bpc}")
    b = synth.make_batch("mu7.6", 24, first=100)
    want = oracle.reconstruct(b)
    got = run_batched(b, sbt.make_tuning(tpe, bpc))
    _same(got, want, f"tpe={tpe} bpc={bpc}")


@pytest.mark.parametrize("config,n,first", [("mu7.6", 40, 340), ("mu7.6", 30, 620), ("mu1-25", 40, 0), ("mu30", 4, 1),
                                            ("tiny", 30, 0)])
def test_six_waves_instance_matches_oracle(config, n, first):
    """512 lanes at three workgroups per CU run the instance held to six
    waves per SIMD; with 448-hit slots, events whose busiest module is larger
    (two of the mu=7.6 slices hold one) run from memory beside the others.
    Direct launch, then the captured graph."""
    import torch
    say(f"six-waves instance {config} x{n} from {first}")
    b = synth.make_batch(config, n, first=first)
    want = oracle.reconstruct(b)
    _same(run_batched(b, sbt.make_tuning(512, 3, 448)), want, f"dense {config}")
    p = sbt.make_params(b.module_z)
    ctx = sbt.Context(p, b.n_events, b.n_hits, sbt.make_tuning(512, 3, 448))
    got, stats = graph_replays(ctx, sbt.DeviceBatch(b), sbt.DeviceTracks(b.n_events, b.n_hits), torch.cuda.Stream(),
                               reps=2)
    check_replays(got, stats, want, f"dense {config} graph")
    ctx.close()


@pytest.mark.parametrize("config,n,first,deferred", [("mu1-25", 40, 0, 768), ("mu1-25", 30, 100, 1536),
                                                     ("mu30", 4, 1, 768), ("mu30", 3, 5, 1536),
                                                     ("mu7.6", 30, 340, 672), ("tiny", 20, 0, 768)])
def test_two_pass_launch_matches_oracle(config, n, first, deferred):
    """A two-pass tuning: the six-waves instance with 448-hit slots sets aside
    the events its slots cannot hold (none, some or all of a batch), and a
    second pass runs them with larger slots.  Direct launch, then the
    captured graph."""
    import torch
    say(f"two passes {config} x{n} from {first}, second pass {deferred}-hit slots")
    b = synth.make_batch(config, n, first=first)
    want = oracle.reconstruct(b)
    t = sbt.make_tuning(512, 3, 448, deferred_window_hits=deferred)
    got = run_batched(b, t)
    assert not got[3].any()
    _same(got, want, f"two passes {config}")
    p = sbt.make_params(b.module_z)
    ctx = sbt.Context(p, b.n_events, b.n_hits, t)
    assert ctx.get_tuning().as_dict()["deferred_window_hits"] == deferred
    got, stats = graph_replays(ctx, sbt.DeviceBatch(b), sbt.DeviceTracks(b.n_events, b.n_hits), torch.cuda.Stream(),
                               reps=2)
    check_replays(got, stats, want, f"two passes {config} graph")
    ctx.close()


def test_two_pass_tunings_are_checked():
    """A second pass needs the six-waves first pass (512 lanes, three or more
    per CU, 448-hit slots) and larger slots than the first."""
    b = synth.make_batch("tiny", 4)
    p = sbt.make_params(b.module_z)
    for bad in (sbt.make_tuning(256, 3, 448, deferred_window_hits=768),
                sbt.make_tuning(512, 2, 448, deferred_window_hits=768),
                sbt.make_tuning(512, 3, 672, deferred_window_hits=768),
                sbt.make_tuning(512, 3, 448, deferred_window_hits=448),
                sbt.make_tuning(512, 3, 448, deferred_window_hits=-1)):
        with pytest.raises(sbt.SbtError):
            sbt.Context(p, b.n_events, b.n_hits, bad).close()


# 64-lane events several to a workgroup, one wave each: (events per
# workgroup, slot capacity, LDS flag capacity, workgroups per CU).  Each
# workgroup's LDS (the events' regions together) stays within 159 KiB.
EPB_CASES = [(2, 256, 4096, 2), (4, 256, 4096, 1), (3, 448, 4096, 1), (8, 0, 4096, 1), (2, 672, 16384, 1),
             (10, 0, 0, 2)]


@pytest.mark.parametrize("epb,cap,own,bpc", EPB_CASES)
def test_events_per_block_matches_oracle(epb, cap, own, bpc):
    """Several 64-lane events per workgroup give the oracle's tracks on every
    recipe: events whose modules or flags do not fit the LDS regions run from
    memory beside ones that do, and batches with fewer events than waves
    leave waves without work."""
    say(f"events per block {epb}, cap={cap} own={own} bpc={bpc}")
    for config, n, first in (("mu7.6", 24, 100), ("tiny", 40, 0), ("mu1-25", 30, 5), ("mu30", 4, 2), ("tiny", 3, 9)):
        b = synth.make_batch(config, n, first=first)
        want = oracle.reconstruct(b)
        t = sbt.make_tuning(64, bpc, cap, own, events_per_block=epb)
        got = run_batched(b, t)
        assert not got[3].any()
        _same(got, want, f"epb={epb} cap={cap} {config} x{n}")


def test_events_per_block_graph_replays_and_tuning_checks():
    """The grouped configuration through the captured graph (three calls,
    two replays) gives the oracle's tracks; more than one event per
    workgroup is refused for events wider than one wave, and so is a
    workgroup whose LDS would exceed 159 KiB."""
    import torch
    b = synth.make_batch("mu1-25", 40, first=11)
    want = oracle.reconstruct(b)
    p = sbt.make_params(b.module_z)
    ctx = sbt.Context(p, b.n_events, b.n_hits, sbt.make_tuning(64, 1, 256, 4096, events_per_block=4))
    assert ctx.get_tuning().as_dict()["events_per_block"] == 4
    dev = sbt.DeviceBatch(b)
    out = sbt.DeviceTracks(b.n_events, b.n_hits)
    got, stats = graph_replays(ctx, dev, out, torch.cuda.Stream())
    check_replays(got, stats, want, "events per block 4")
    for bad in (sbt.make_tuning(128, 1, 256, 4096, events_per_block=2),
                sbt.make_tuning(64, 1, 672, 16384, events_per_block=3),
                sbt.make_tuning(64, 1, 256, 4096, events_per_block=17)):
        with pytest.raises(sbt.SbtError):
            ctx.set_tuning(bad)
    ctx.close()


# LDS capacities: 0 or 1 forces every module window / the owner flags to be
# read from memory, intermediate values mix both within one event
LDS_CASES = [(0, 0), (1, 1), (64, 1000), (200, 3000), (256, 16384), (448, 16384), (672, 16384),
             (768, 16384), (1024, 65536), (1536, 0)]


@pytest.mark.parametrize("cap,own", LDS_CASES)
@pytest.mark.parametrize("config,n", [("mu7.6", 16), ("mu30", 4)])
def test_lds_overflow_fallbacks(cap, own, config, n):
    say(f"lds cap={cap} own={own} {config} x{n}")
    b = synth.make_batch(config, n, first=7)
    want = oracle.reconstruct(b)
    for tpe in (64, 256, 1024):
        _same(run_batched(b, sbt.make_tuning(tpe, 2, cap, own)), want, f"cap={cap} own={own} tpe={tpe}")


def test_random_batches_and_launch_configurations():
    """Seeded random draws of recipe, batch slice, launch configuration (any
    width, workgroups per CU, slot and flag capacities, several 64-lane
    events per workgroup) and call path (direct or captured graph): every
    result is the oracle's.  Configurations the library refuses (LDS above
    159 KiB) are skipped."""
    import torch
    rng = np.random.default_rng(2207)
    stream = torch.cuda.Stream()
    ran = 0
    for i in range(40):
        config = str(rng.choice(["tiny", "mu7.6", "mu1-25", "mu30", "pairs7.6", "bw7.6"]))
        n = int(rng.integers(1, 6 if config == "mu30" else 30))
        first = int(rng.integers(0, 200))
        tpe = int(rng.choice([64, 128, 256, 512, 1024]))
        epb = int(rng.choice([1, 2, 4])) if tpe == 64 else 1
        t = sbt.make_tuning(tpe, int(rng.integers(1, 9)), int(rng.choice([0, 200, 256, 448, 672, 768, 1024, 1536])),
                            int(rng.choice([0, 1000, 4096, 16384])), events_per_block=epb)
        if rng.integers(0, 4) == 0:
            # two passes: the six-waves first pass, a second on larger slots
            t = sbt.make_tuning(512, int(rng.integers(3, 5)), 448, int(rng.choice([4096, 16384])),
                                deferred_window_hits=int(rng.choice([672, 768, 1024, 1536])))
        graph = bool(rng.integers(0, 2))
        b = synth.make_batch(config, n, first=first)
        p = sbt.make_params(b.module_z)
        try:
            ctx = sbt.Context(p, b.n_events, b.n_hits, t)
        except sbt.SbtError:
            continue
        say(f"random {i}: {config} x{n} from {first}, {t.as_dict()}, graph={graph}")
        out = sbt.DeviceTracks(b.n_events, b.n_hits)
        if graph:
            with torch.cuda.stream(stream):
                ctx.reconstruct(sbt.DeviceBatch(b), out, stream)
            stream.synchronize()
        else:
            ctx.reconstruct(sbt.DeviceBatch(b), out)
        got = out.to_host()
        ctx.close()
        assert not got[3].any()
        _same(got, oracle.reconstruct(b), f"random {i}")
        ran += 1
    assert ran >= 25


def test_random_tiny_events_and_parameters():
    """Crowded tiny events with random tolerances, traversal direction and
    miss allowance: the same events the oracle's brute-force pins use."""
    rng = np.random.default_rng(77)
    for i in range(30):
        evs = [tiny_random_event(rng, M=7, jitter_z=bool(i % 2)) for _ in range(8)]
        b = synth.concat([dict(x=x, y=y, z=z, module_counts=np.diff(mo).astype(np.int64),
                               truth=np.full(len(x), -1, np.int32)) for (x, y, z, mo, mz) in evs], evs[0][4])
        kw = dict(reverse=int(rng.integers(0, 2)),
                  max_doublet_candidates=int(rng.choice([1, 2, 3, 4, 8, 16, 64])),
                  phi_window_seeding=int(rng.choice([20, 416, 32767])),
                  phi_window_forwarding=int(rng.choice([20, 416, 32767])),
                  max_scatter_seeding=float(rng.choice([0.05, 1.0, 20.0])),
                  max_scatter_forwarding=float(rng.choice([0.05, 1.0, 20.0])),
                  max_tracklet_chi2=float(rng.choice([0.001, 0.05, 5.0])),
                  max_consecutive_misses=int(rng.choice([0, 1, 2])))
        say(f"random tiny batch {i} {kw}")
        want = oracle.reconstruct(b, **kw)
        _same(run_plain(b, **kw), want, f"plain random {i}")
        _same(run_batched(b, **kw), want, f"batched random {i}")


# ------------------------------------------------------------------ edge cases

def test_empty_batch():
    say("empty batch")
    b = synth.make_batch("tiny", 0)
    for got in (run_plain(b), run_batched(b)):
        assert list(got[0]) == [0] and list(got[1]) == [0] and got[2].size == 0


def test_empty_and_degenerate_events():
    say("empty and degenerate events")
    mz = synth.PLANE_Z.astype(np.float32)
    empty = dict(x=np.zeros(0, np.float32), y=np.zeros(0, np.float32), z=np.zeros(0, np.float32),
                 module_counts=np.zeros(26, np.int64), truth=np.zeros(0, np.int32))
    two = dict(x=np.array([10, 10.5], np.float32), y=np.array([1, 1.05], np.float32),
               z=np.array([mz[3], mz[4]], np.float32),
               module_counts=np.eye(26, dtype=np.int64)[3] + np.eye(26, dtype=np.int64)[4],
               truth=np.zeros(2, np.int32))
    tiny = synth.make_batch("tiny", 3)
    evs = [empty, synth._slice(tiny, 0), two, empty, synth._slice(tiny, 1), synth._slice(tiny, 2), empty]
    b = synth.concat(evs, mz)
    want = oracle.reconstruct(b)
    _same(run_plain(b), want, "plain degenerate")
    _same(run_batched(b), want, "batched degenerate")


def test_largest_event_and_oversized_event():
    """An event of exactly 65,535 hits is reconstructed; one of 65,536 is
    flagged SBT_EV_TOO_LARGE with no tracks, and its neighbours are intact."""
    say("largest and oversized events")
    parts = []
    k = 0
    while sum(p["x"].size for p in parts) < 65535:
        parts.append(synth._slice(synth.make_batch("mu30", 1, first=k), 0))
        k += 1
    big = synth.concat(parts, synth.PLANE_Z)

    def cut(n):
        # first n hits of the merged event (hits stay grouped by module)
        M = big.n_modules
        mo = np.zeros(M + 1, np.int64)
        counts = np.zeros(M, np.int64)
        # regroup all hits by module, then keep n of them
        mod = np.repeat(np.tile(np.arange(M), len(parts)), np.diff(big.module_offsets))
        order = np.argsort(mod, kind="stable")[:n]
        order = order[np.argsort(mod[order], kind="stable")]
        counts = np.bincount(mod[order], minlength=M)
        return dict(x=big.x[order], y=big.y[order], z=big.z[order], module_counts=counts.astype(np.int64),
                    truth=np.zeros(n, np.int32))
    small = synth._slice(synth.make_batch("tiny", 1), 0)
    b = synth.concat([small, cut(65535), small, cut(65536), small], synth.PLANE_Z)
    ok = synth.concat([small, cut(65535), small, small], synth.PLANE_Z)
    want_ok = oracle.reconstruct(ok)
    for name, got in (("plain", run_plain(b)), ("batched", run_batched(b))):
        say(f"{name}: statuses {list(got[3])}")
        assert list(got[3]) == [0, 0, 0, sbt.SBT_EV_TOO_LARGE, 0]
        eto, tho, th = got[:3]
        assert eto[4] == eto[3], "oversized event produced tracks"
        # drop the oversized event and compare the rest with the oracle
        keep = [0, 1, 2, 4]
        mine = [[tuple(th[tho[t]:tho[t + 1]]) for t in range(eto[e], eto[e + 1])] for e in keep]
        ref = [[tuple(want_ok[2][want_ok[1][t]:want_ok[1][t + 1]]) for t in range(want_ok[0][e], want_ok[0][e + 1])]
               for e in range(4)]
        assert mine == ref, name


def test_bad_offsets_are_reported():
    say("bad offsets")
    b = synth.make_batch("tiny", 3)
    mo = b.module_offsets.copy()
    M = b.n_modules
    mo[M + 5] = mo[M + 7] + 3      # event 1: module offsets decrease
    bad = synth.Batch(b.x, b.y, b.z, b.event_offsets, mo, b.module_z, b.truth)
    want = oracle.reconstruct(synth.concat([synth._slice(b, 0), synth._slice(b, 2)], b.module_z))
    for name, got in (("plain", run_plain(bad)), ("batched", run_batched(bad))):
        assert list(got[3]) == [0, sbt.SBT_EV_BAD_OFFSETS, 0], name
        assert got[0][2] == got[0][1]
        assert list(np.delete(np.diff(got[0]), 1)) == list(np.diff(want[0]))


def test_capacity_errors_are_reported():
    """A context smaller than the batch and a short workspace are refused
    before any launch."""
    say("capacity errors")
    b = synth.make_batch("tiny", 4)
    p = sbt.make_params(b.module_z)
    dev = sbt.DeviceBatch(b)
    ctx = sbt.Context(p, b.n_events - 1, b.n_hits)
    with pytest.raises(sbt.SbtError) as ei:
        ctx.reconstruct(dev)
    assert ei.value.code == sbt.SBT_ERR_WORKSPACE
    ctx.close()
    ctx = sbt.Context(p, b.n_events, b.n_hits - 1)
    with pytest.raises(sbt.SbtError) as ei:
        ctx.reconstruct(dev)
    assert ei.value.code == sbt.SBT_ERR_WORKSPACE
    ctx.close()
    ws = sbt.Workspace(b.n_events, b.n_hits // 4)
    with pytest.raises(sbt.SbtError) as ei:
        sbt.sbt_reconstruct(p, dev, workspace=ws)
    assert ei.value.code == sbt.SBT_ERR_WORKSPACE


# ------------------------------------------------------------------ full sizes

def _invariants(b, got):
    eto, tho, th = got[:3]
    assert np.all(np.diff(eto) >= 0) and np.all(np.diff(tho) >= 3)
    M = b.n_modules
    for e in range(b.n_events):
        lo, hi = int(b.event_offsets[e]), int(b.event_offsets[e + 1])
        ids = th[tho[eto[e]]:tho[eto[e + 1]]]
        assert ids.size == np.unique(ids).size
        assert ids.size == 0 or (ids.min() >= 0 and ids.max() < hi - lo)


def test_full_mu7_6_batch_all_events():
    """The 1,000-event mu = 7.6 batch in the launch configuration the
    benchmark times (chosen per call, graph replays on a stream of its own):
    every event against the oracle, plain, direct batched launch, and three
    graph calls (capture, then two replays from the cache)."""
    import torch
    say("full mu7.6 x1000")
    b = synth.make_batch("mu7.6")
    want = oracle.reconstruct(b)
    p = sbt.make_params(b.module_z)
    dev = sbt.DeviceBatch(b)
    _same(sbt.sbt_reconstruct(p, dev).to_host(), want, "plain mu7.6 x1000")
    ctx = sbt.Context(p, b.n_events, b.n_hits)
    out = sbt.DeviceTracks(b.n_events, b.n_hits)
    say("  batched, direct launch")
    out.fill_(-1)
    ctx.reconstruct(dev, out)
    _same(out.to_host(), want, "batched mu7.6 x1000 direct")
    assert ctx.graph_stats()["direct"] == 1
    say("  batched, graph replays")
    got, stats = graph_replays(ctx, dev, out, torch.cuda.Stream())
    check_replays(got, stats, want, "batched mu7.6 x1000")
    ctx.close()


# ------------------------------------------------------------------ half-precision input

def run_batched_f16(batch, tuning=None):
    p = sbt.make_params(batch.module_z)
    ctx = sbt.Context(p, max(batch.n_events, 1), max(batch.n_hits, 1), tuning)
    out = ctx.reconstruct_f16(sbt.DeviceBatchF16(batch)).to_host()
    ctx.close()
    return out


@pytest.mark.parametrize("config,n", [("tiny", 20), ("mu7.6", 40), ("mu1-25", 30), ("mu30", 6)])
def test_f16_matches_oracle_on_rounded_inputs(config, n):
    """Binary16 array-of-structures input: the oracle on the same values
    widened to binary32 (numpy's IEEE rounding) defines the tracks."""
    say(f"f16 {config} x{n}")
    b = synth.make_batch(config, n)
    want = oracle.reconstruct(rounded_to_f16(b))
    got = run_batched_f16(b)
    assert not got[3].any()
    _same(got, want, f"f16 {config}")


@pytest.mark.parametrize("tpe,cap", [(64, 0), (256, 448), (1024, 1536)])
def test_f16_independent_of_launch_configuration(tpe, cap):
    say(f"f16 tuning tpe={tpe} cap={cap}")
    b = synth.make_batch("mu30", 4, first=11)
    want = oracle.reconstruct(rounded_to_f16(b))
    _same(run_batched_f16(b, sbt.make_tuning(tpe, 2, cap)), want, f"f16 tpe={tpe} cap={cap}")


def test_f16_full_mu7_6_batch():
    """Binary16 input on the full mu = 7.6 batch: a direct launch, then three
    graph calls on a stream of their own."""
    import torch
    say("f16 full mu7.6 x1000")
    b = synth.make_batch("mu7.6")
    want = oracle.reconstruct(rounded_to_f16(b))
    p = sbt.make_params(b.module_z)
    ctx = sbt.Context(p, b.n_events, b.n_hits)
    dev = sbt.DeviceBatchF16(b)
    out = sbt.DeviceTracks(b.n_events, b.n_hits)
    out.fill_(-1)
    ctx.reconstruct_f16(dev, out)
    _same(out.to_host(), want, "f16 mu7.6 x1000 direct")
    got, stats = graph_replays(ctx, dev, out, torch.cuda.Stream(), f16=True)
    check_replays(got, stats, want, "f16 mu7.6 x1000")
    ctx.close()


def test_f16_rejects_misaligned_coordinates():
    b = synth.make_batch("tiny", 2)
    p = sbt.make_params(b.module_z)
    ctx = sbt.Context(p, b.n_events, b.n_hits)
    dev = sbt.DeviceBatchF16(b)
    dev.hits.xyzw = dev.xyzw.data_ptr() + 2
    with pytest.raises(sbt.SbtError) as ei:
        ctx.reconstruct_f16(dev)
    assert ei.value.code == sbt.SBT_ERR_INVALID_ARG
    ctx.close()


_FULL = {}


def _full_batch(config, n):
    """A full-size batch and the oracle's tracks for all of it (computed once
    per module; about half a minute of CPU on the GPU host for each batch)."""
    if (config, n) not in _FULL:
        b = synth.make_batch(config, n)
        _FULL[(config, n)] = (b, oracle.reconstruct(b))
    return _FULL[(config, n)]


# full batches in the launch configurations the autotuner and the per-call
# rule pick for them (the two-pass one for the 10,000-event mixture): every
# event against the oracle.  Tuples: lanes per event, workgroups per CU, slot
# capacity[, LDS flag capacity, events per workgroup, second-pass slots].
@pytest.mark.parametrize("config,n,tuning", [("mu1-25", 10000, (512, 2, 672)),
                                             ("mu1-25", 10000, (512, 2, 768)),
                                             ("mu1-25", 10000, (512, 3, 448, 16384, 1, 768)),
                                             ("mu30", 2000, (1024, 1, 1536)),
                                             ("mu30", 2000, (512, 2, 672))])
def test_full_size_all_events(config, n, tuning):
    say(f"full {config} x{n}, tuning {tuning}: oracle on every event")
    b, want = _full_batch(config, n)
    say(f"  oracle done, {int(want[0][-1])} tracks")
    got = run_batched(b, sbt.make_tuning(*tuning))
    assert not got[3].any()
    _same(got, want, f"{config} x{n} {tuning}")
    _invariants(b, got)
    if tuning == (512, 2, 672):
        say("  plain form")
        _same(run_plain(b), want, f"plain {config} x{n}")


def test_full_size_half_precision():
    """The binary16 entry point on the full mu in U{1..25} batch: every event
    against the oracle on the rounded coordinates."""
    say("full mu1-25 x10000, binary16 input")
    b = rounded_to_f16(synth.make_batch("mu1-25", 10000))
    want = oracle.reconstruct(b)
    got = run_batched_f16(b, sbt.make_tuning(512, 2, 672))
    assert not got[3].any()
    _same(got, want, "f16 mu1-25 x10000")


def _expected_choice(n_events, n_hits, cus):
    """(lanes per event, workgroups per CU, slot capacity, second-pass slots)"""
    small = n_hits <= 2500 * n_events
    large = n_hits >= 4000 * n_events
    huge = n_hits >= 9000 * n_events
    if small:
        return (256, 5, 256, 0) if n_events > 2 * cus else (512, 2, 448, 0)
    if n_events <= cus or (n_events <= 2 * cus and large) or huge:
        return (1024, 1, 1536, 0)
    if large and n_events >= 15 * cus:
        return (512, 3, 448, 768)
    if not large and n_events >= 6 * cus:
        return (512, 3, 448, 0)
    return (512, 2, 768 if large else 672, 0)


@pytest.mark.parametrize("config,n", [("mu7.6", 40), ("mu7.6", 300), ("mu1-25", 300), ("mu1-25", 1000),
                                      ("mu7.6", 3600), ("mu30", 600), ("tiny", 100), ("tiny", 700),
                                      ("mu1-25", 4000)])
def test_configuration_chosen_per_call(config, n):
    """A context created without a launch configuration chooses one per call
    from the batch's size.  Each choice, a smaller batch through the same
    context and an installed configuration all give the oracle's tracks."""
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    say(f"per-call configuration {config} x{n} ({cus} CUs)")
    b = synth.make_batch(config, n)
    p = sbt.make_params(b.module_z)
    ctx = sbt.Context(p, b.n_events, b.n_hits)
    t = ctx.get_tuning()
    assert (t.threads_per_event, t.blocks_per_cu, t.lds_window_hits, t.deferred_window_hits) == \
        _expected_choice(n, b.n_hits, cus)
    assert t.lds_owner_hits == 16384
    want = oracle.reconstruct(b)
    _same(ctx.reconstruct(sbt.DeviceBatch(b)).to_host(), want, f"{config} x{n} per call")
    small = synth.make_batch(config, 20, first=5)
    _same(ctx.reconstruct(sbt.DeviceBatch(small)).to_host(), oracle.reconstruct(small), "smaller batch")
    ctx.set_tuning(sbt.make_tuning(256, 4, 448))
    t = ctx.get_tuning()
    assert (t.threads_per_event, t.blocks_per_cu, t.lds_window_hits) == (256, 4, 448)
    _same(ctx.reconstruct(sbt.DeviceBatch(b)).to_host(), want, f"{config} x{n} installed")
    ctx.close()


def test_repeat_runs_identical():
    say("20 repeated batched runs")
    b = synth.make_batch("mu30", 40)
    p = sbt.make_params(b.module_z)
    dev = sbt.DeviceBatch(b)
    ctx = sbt.Context(p, b.n_events, b.n_hits, sbt.make_tuning(256, 8))
    first = ctx.reconstruct(dev).to_host()
    for i in range(19):
        _same(ctx.reconstruct(dev).to_host(), first[:3], f"repeat {i}")
    ctx.close()


@pytest.mark.parametrize("form", ["plain", "batched"])
def test_backward_tracks_match_oracle(form):
    say(f"backward tracks, {form}")
    b = synth.make_batch("bw7.6", 40)
    got = run_plain(b) if form == "plain" else run_batched(b)
    _same(got, oracle.reconstruct(b), f"backward {form}")


@pytest.mark.parametrize("form", ["plain", "batched", "f16"])
def test_module_pairs_match_oracle(form):
    """Module pairs: hits of a module at two z values, neither the nominal one."""
    import torch
    say(f"module pairs, {form}")
    b = synth.make_batch("pairs7.6", 40)
    if form == "plain":
        _same(run_plain(b), oracle.reconstruct(b), "pairs plain")
    elif form == "batched":
        _same(run_batched(b), oracle.reconstruct(b), "pairs batched")
    else:
        _same(run_batched_f16(b), oracle.reconstruct(rounded_to_f16(b)), "pairs f16")


@pytest.mark.parametrize("form", ["plain", "batched", "f16"])
def test_outputs_in_pinned_host_memory(form):
    """Tracks written by the kernels straight into pinned host buffers equal
    the oracle's (the kernels only write the outputs, never read them)."""
    import torch
    say(f"pinned host outputs, {form}")
    b = synth.make_batch("mu1-25", 24)
    p = sbt.make_params(b.module_z)
    out = sbt.DeviceTracks(b.n_events, b.n_hits, pinned=True).fill_(-7)
    if form == "plain":
        sbt.sbt_reconstruct(p, sbt.DeviceBatch(b), out)
        want = oracle.reconstruct(b)
    else:
        ctx = sbt.Context(p, b.n_events, b.n_hits)
        if form == "batched":
            ctx.reconstruct(sbt.DeviceBatch(b), out)
            want = oracle.reconstruct(b)
        else:
            ctx.reconstruct_f16(sbt.DeviceBatchF16(b), out)
            want = oracle.reconstruct(rounded_to_f16(b))
        torch.cuda.synchronize()
        ctx.close()
    torch.cuda.synchronize()
    got = out.to_host()
    _same(got, want, f"pinned {form}")
    assert not got[3].any()


def _line_events(rng, M, n_events, n_tracks, noise, pitch=20.0):
    """Straight tracks from near the axis over M planes plus uniform noise."""
    mz = (-300.0 + pitch * np.arange(M)).astype(np.float32)
    events = []
    for _ in range(n_events):
        per = [[] for _ in range(M)]
        for _ in range(n_tracks):
            phi = rng.uniform(-np.pi, np.pi)
            slope = rng.uniform(0.01, 0.03)
            x0, y0 = rng.normal(0, 0.01, 2)
            for k in range(M):
                if rng.random() < 0.97:
                    r = slope * (mz[k] + 600.0)
                    per[k].append((x0 + r * np.cos(phi) + rng.normal(0, 0.012),
                                   y0 + r * np.sin(phi) + rng.normal(0, 0.012)))
        for _ in range(noise):
            k = int(rng.integers(0, M))
            r, phi = rng.uniform(5, 40), rng.uniform(-np.pi, np.pi)
            per[k].append((r * np.cos(phi), r * np.sin(phi)))
        for k in range(M):
            rng.shuffle(per[k])
        xs = np.array([h[0] for p in per for h in p], np.float32)
        ys = np.array([h[1] for p in per for h in p], np.float32)
        zs = np.repeat(mz, [len(p) for p in per]).astype(np.float32)
        events.append(dict(x=xs, y=ys, z=zs, module_counts=np.array([len(p) for p in per], np.int64),
                           truth=np.full(xs.size, -1, np.int32)))
    return synth.concat(events, mz)


@pytest.mark.parametrize("M", [3, 64])
def test_fewest_and_most_modules(M):
    """The module count at both ends of its range (3 and 64 modules)."""
    say(f"{M} modules")
    b = _line_events(np.random.default_rng(M), M, 12, 40, 30)
    want = oracle.reconstruct(b)
    assert int(want[0][-1]) > 0
    _same(run_plain(b), want, f"plain M={M}")
    for tuning in (None, sbt.make_tuning(64, 4, 256), sbt.make_tuning(1024, 1, 1536)):
        _same(run_batched(b, tuning), want, f"batched M={M} {tuning and tuning.as_dict()}")
    _same(run_plain(b, reverse=0), oracle.reconstruct(b, reverse=0), f"plain forward M={M}")


def test_autotune_installs_a_candidate_and_keeps_results():
    """sbt_autotune on a 40-event sample installs one of its candidate
    configurations; the next calls (a graph capture and a replay on a stream
    of their own) give the oracle's tracks on the full sample and on another
    batch through the same context."""
    import torch
    say("autotune on 40 events")
    b = synth.make_batch("mu7.6", 40, first=200)
    other = synth.make_batch("mu1-25", 25, first=60)
    p = sbt.make_params(b.module_z)
    ctx = sbt.Context(p, b.n_events + other.n_events, b.n_hits + other.n_hits)
    dev = sbt.DeviceBatch(b)
    stream = torch.cuda.Stream()
    best, ms = ctx.autotune(dev, reps=2, stream=stream, cache=False)
    t = ctx.get_tuning()
    say(f"  picked {t.as_dict()} at {ms:.3f} ms")
    assert t.as_dict() == best.as_dict()
    assert t.threads_per_event in (64, 128, 256, 512, 1024)
    assert t.lds_window_hits in (256, 448, 672, 768, 1024, 1536)
    assert 1 <= t.blocks_per_cu <= 16
    if t.threads_per_event == 64:
        assert t.events_per_block in (2, 4, 8) and t.lds_window_hits in (256, 448) and t.lds_owner_hits == 4096
    else:
        assert t.events_per_block == 1 and t.lds_owner_hits == 16384
    assert ms > 0
    out = sbt.DeviceTracks(b.n_events, b.n_hits)
    got, stats = graph_replays(ctx, dev, out, stream, reps=2)
    check_replays(got, stats, oracle.reconstruct(b), "autotuned")
    dev2 = sbt.DeviceBatch(other)
    out2 = sbt.DeviceTracks(other.n_events, other.n_hits)
    got2, _ = graph_replays(ctx, dev2, out2, stream, reps=1)
    _same(got2[0], oracle.reconstruct(other), "autotuned, another batch")
    ctx.close()


@pytest.mark.parametrize("config,n", [("tiny", 20), ("mu7.6", 40), ("mu1-25", 30), ("mu30", 6), ("pairs7.6", 20),
                                      ("bw7.6", 20)])
def test_fill_candidates_pass_matches_oracle(config, n):
    """The plain form with the separate candidate pass (the paper's Fill
    candidates kernel, as an ablation) gives the oracle's tracks."""
    say(f"fill candidates {config} x{n}")
    b = synth.make_batch(config, n)
    p = sbt.make_params(b.module_z)
    got = sbt.sbt_debug_reconstruct_fill_candidates(p, sbt.DeviceBatch(b)).to_host()
    assert not got[3].any()
    _same(got, oracle.reconstruct(b), f"fill candidates {config}")


def test_fill_candidates_pass_random_parameters():
    """The candidate pass on crowded tiny events with random parameters and
    both traversal directions (the pendulum start must not depend on them
    beyond the traversal order)."""
    rng = np.random.default_rng(99)
    for i in range(8):
        evs = [tiny_random_event(rng, M=6, jitter_z=bool(i % 2)) for _ in range(8)]
        b = synth.concat([dict(x=x, y=y, z=z, module_counts=np.diff(mo).astype(np.int64),
                               truth=np.full(len(x), -1, np.int32)) for (x, y, z, mo, mz) in evs], evs[0][4])
        kw = dict(reverse=int(rng.integers(0, 2)), max_doublet_candidates=int(rng.choice([1, 2, 3, 4, 8, 16, 64])),
                  phi_window_seeding=int(rng.choice([20, 416, 32767])),
                  max_consecutive_misses=int(rng.choice([0, 1, 2])))
        say(f"fill candidates random batch {i} {kw}")
        p = sbt.make_params(b.module_z, **kw)
        got = sbt.sbt_debug_reconstruct_fill_candidates(p, sbt.DeviceBatch(b)).to_host()
        _same(got, oracle.reconstruct(b, **kw), f"fill candidates random {i}")


def test_fill_candidates_full_mu7_6_batch():
    say("fill candidates full mu7.6 x1000")
    b = synth.make_batch("mu7.6")
    p = sbt.make_params(b.module_z)
    _same(sbt.sbt_debug_reconstruct_fill_candidates(p, sbt.DeviceBatch(b)).to_host(), oracle.reconstruct(b),
          "fill candidates mu7.6 x1000")


_JETS = {}


def _jets():
    """Seven dense-jet events (120 to 1,200 tracks in one narrow cone; the
    busiest module holds 86 to 853 hits), with cones on the phi16 wrap at
    angle 0 and on the +-pi branch of the angle, exactly duplicated hits and
    noise in the cone, and the oracle's tracks for them (computed once)."""
    if not _JETS:
        rng = np.random.default_rng(11)
        specs = ((300, 0.0, 0.004), (300, np.pi, 0.004), (120, 1.0, 0.004), (700, -np.pi / 2, 0.004),
                 (700, 0.0, 0.004), (1200, np.pi, 0.004), (1200, 0.0, 0.001))
        b = synth.concat([jet_event(rng, n, phi0, sig) for n, phi0, sig in specs], synth.PLANE_Z)
        _JETS["b"] = b
        _JETS["want"] = oracle.reconstruct(b)
        _JETS["b16"] = rounded_to_f16(b)
        _JETS["want16"] = oracle.reconstruct(_JETS["b16"])
    return _JETS


# dense jets in every form: hundreds of hits per phi window make long window
# scans, crowded pendulum lists and many competing claims, and the busiest
# modules cross every LDS slot capacity (memory form included)
@pytest.mark.parametrize("form", ["plain", "per-call", "512x2x672", "512x2x0", "64x4x0", "256x3x448",
                                  "1024x1x1536", "two-pass", "f16"])
def test_dense_jets_match_oracle(form):
    J = _jets()
    say(f"dense jets, {form}")
    if form == "plain":
        got, want = run_plain(J["b"]), J["want"]
    elif form == "per-call":
        got, want = run_batched(J["b"]), J["want"]
    elif form == "two-pass":
        got, want = run_batched(J["b"], sbt.make_tuning(512, 3, 448, deferred_window_hits=1536)), J["want"]
    elif form == "f16":
        got, want = run_batched_f16(J["b16"], sbt.make_tuning(512, 2, 672)), J["want16"]
    else:
        tpe, bpc, cap = (int(v) for v in form.split("x"))
        got, want = run_batched(J["b"], sbt.make_tuning(tpe, bpc, cap)), J["want"]
    assert not got[3].any()
    _same(got, want, f"dense jets {form}")
    _invariants(J["b"], got)


_PARAM_BATCH = {}


def _param_batch():
    """Eight mu = 7.6 events, one mu = 30 event and two module-pair events."""
    if "b" not in _PARAM_BATCH:
        evs = ([synth._slice(synth.make_batch("mu7.6", 8, first=500), e) for e in range(8)]
               + [synth._slice(synth.make_batch("mu30", 1, first=7), 0)]
               + [synth._slice(synth.make_batch("pairs7.6", 2), e) for e in range(2)])
        _PARAM_BATCH["b"] = synth.concat(evs, synth.PLANE_Z)
    return _PARAM_BATCH["b"]


# method parameters away from the defaults on full-size events: doublet
# candidates K = 8 and 16 (the K partners of a middle hit on K adjacent
# lanes), 3 and 64 (all K on one lane), 1 and 2; windows of the whole circle
# and of one phi16 unit; forward traversal; looser thresholds
PARAM_SETS = {
    "K8": dict(max_doublet_candidates=8),
    "K16": dict(max_doublet_candidates=16),
    "K3": dict(max_doublet_candidates=3),
    "K1-nomiss": dict(max_doublet_candidates=1, max_consecutive_misses=0),
    "K2-forward": dict(max_doublet_candidates=2, reverse=0),
    "K64-fullcircle": dict(max_doublet_candidates=64, phi_window_seeding=32767, phi_window_forwarding=32767),
    "W0": dict(phi_window_seeding=0, phi_window_forwarding=0),
    "loose": dict(max_scatter_seeding=1.0, max_scatter_forwarding=1.0, max_tracklet_chi2=1.0,
                  max_consecutive_misses=2),
}


@pytest.mark.parametrize("name", list(PARAM_SETS))
def test_parameters_at_scale(name):
    kw = PARAM_SETS[name]
    b = _param_batch()
    say(f"parameters {name} on {b.n_events} full-size events")
    want = oracle.reconstruct(b, **kw)
    _same(run_plain(b, **kw), want, f"plain {name}")
    for t in (None, sbt.make_tuning(512, 2, 672), sbt.make_tuning(256, 3, 448), sbt.make_tuning(1024, 1, 1536),
              sbt.make_tuning(512, 2, 0), sbt.make_tuning(64, 8, 256, 4096, 2),
              sbt.make_tuning(512, 3, 448), sbt.make_tuning(512, 3, 448, deferred_window_hits=768)):
        got = run_batched(b, t, **kw)
        assert not got[3].any()
        _same(got, want, f"batched {name} {None if t is None else t.as_dict()}")


def test_thirty_thousand_small_events():
    """30,000 single-vertex events (12.9 M hits) in one call: the event
    ordering, the scan over events and the CSR write loop over many batches
    of events; the per-call configuration (small-event branch), the plain
    form, 64-lane events four to a workgroup, and the captured graph."""
    import torch
    say("30,000 tiny events")
    b = synth.make_batch("tiny", 30000)
    want = oracle.reconstruct(b)
    say(f"  oracle done, {int(want[0][-1])} tracks")
    _same(run_batched(b), want, "30k per-call")
    _same(run_plain(b), want, "30k plain")
    _same(run_batched(b, sbt.make_tuning(64, 2, 256, 4096, 4)), want, "30k 64-lane x4")
    p = sbt.make_params(b.module_z)
    ctx = sbt.Context(p, b.n_events, b.n_hits)
    got, stats = graph_replays(ctx, sbt.DeviceBatch(b), sbt.DeviceTracks(b.n_events, b.n_hits), torch.cuda.Stream(),
                               reps=2)
    check_replays(got, stats, want, "30k graph")
    ctx.close()
