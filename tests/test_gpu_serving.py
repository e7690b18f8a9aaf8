"""Serving loop (continuous batching) on the GPU.

Each served event's tracks must equal the oracle's for that event alone,
byte for byte, while other events are admitted and run around it; the
admission rules (size limits, queue limit, memory budget) are exercised too.
"""

import sys
import time

import numpy as np
import pytest

import oracle
from _util import rounded_to_f16
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


def _event(b, e):
    M = b.n_modules
    lo, hi = int(b.event_offsets[e]), int(b.event_offsets[e + 1])
    return (b.module_offsets[e * M:(e + 1) * M + 1] - lo, b.x[lo:hi], b.y[lo:hi], b.z[lo:hi])


def _oracle_tracks(b):
    eto, tho, th = oracle.reconstruct(b)
    out = []
    for e in range(b.n_events):
        t0, t1 = int(eto[e]), int(eto[e + 1])
        offs = tho[t0:t1 + 1] - tho[t0]
        out.append((offs, th[tho[t0]:tho[t1]]))
    return out


def _drain(srv, want_n, timeout_s=60.0):
    got = {}
    t_end = time.time() + timeout_s
    while len(got) < want_n:
        for (rid, st, tho, th, ts, td) in srv.poll(1000):
            got[rid] = (st, tho, th, ts, td)
        assert time.time() < t_end, f"serving stalled with {len(got)}/{want_n} results"
    return got


@pytest.mark.parametrize("coords_f16", [False, True])
def test_served_results_equal_alone(coords_f16):
    """Bursts of events arrive while earlier ones are on the GPU; small slots
    force many launches on several streams at once.  With binary16 transfer
    the results are the oracle's on the rounded coordinates."""
    say(f"serving mix vs alone, binary16 transfer {coords_f16}")
    b = synth.make_batch("mu1-25", 120)
    want = _oracle_tracks(rounded_to_f16(b) if coords_f16 else b)
    params = sbt.make_params(b.module_z)
    srv = sbt.Server(params, device_budget_bytes=2 << 30, n_slots=3, slot_events=16, slot_hits=1 << 17,
                     max_wait_us=50, coords_f16=coords_f16)
    got = {}
    rng = np.random.default_rng(9)
    e = 0
    while e < b.n_events:
        burst = int(rng.integers(1, 20))
        for _ in range(burst):
            if e >= b.n_events:
                break
            assert srv.submit(e, *_event(b, e)) == 0
            e += 1
        for (rid, st, tho, th, ts, td) in srv.poll(0):
            got[rid] = (st, tho, th, ts, td)
    got.update(_drain(srv, b.n_events - len(got)))
    srv.close()
    assert sorted(got) == list(range(b.n_events))
    for i in range(b.n_events):
        st, tho, th, ts, td = got[i]
        assert st == 0
        assert np.array_equal(tho, want[i][0]) and np.array_equal(th, want[i][1]), f"event {i}"
        assert td >= ts


@pytest.mark.parametrize("grouped", [False, True])
def test_served_equals_plain_path_on_same_events(grouped):
    """Served results equal the plain form's, with the server's per-launch
    configuration or with an installed one that runs several 64-lane events
    per workgroup."""
    say(f"serving vs plain path, grouped events {grouped}")
    b = synth.make_batch("mu7.6", 40, first=500)
    params = sbt.make_params(b.module_z)
    plain = sbt.sbt_reconstruct(params, sbt.DeviceBatch(b)).to_host()
    tuning = sbt.make_tuning(64, 2, 448, 4096, events_per_block=3) if grouped else None
    srv = sbt.Server(params, device_budget_bytes=1 << 30, n_slots=2, slot_events=7, slot_hits=1 << 16,
                     max_wait_us=0, tuning=tuning)
    for e in range(b.n_events):
        assert srv.submit(100 + e, *_event(b, e)) == 0
    got = _drain(srv, b.n_events)
    srv.close()
    eto, tho, th = plain[:3]
    for e in range(b.n_events):
        t0, t1 = int(eto[e]), int(eto[e + 1])
        assert np.array_equal(got[100 + e][1], tho[t0:t1 + 1] - tho[t0])
        assert np.array_equal(got[100 + e][2], th[tho[t0]:tho[t1]])


def test_admission_rules():
    say("serving admission rules")
    params = sbt.make_params(synth.PLANE_Z)
    M = 26
    # budget too small for the requested slots
    with pytest.raises(sbt.SbtError) as ei:
        sbt.Server(params, device_budget_bytes=1 << 20, n_slots=2, slot_events=8, slot_hits=1 << 16)
    assert ei.value.code == sbt.SBT_ERR_WORKSPACE
    # the transfer format is 0 or 1
    with pytest.raises(sbt.SbtError) as ei:
        sbt.Server(params, device_budget_bytes=1 << 30, n_slots=1, slot_events=2, slot_hits=1 << 16, coords_f16=2)
    assert ei.value.code == sbt.SBT_ERR_INVALID_ARG
    srv = sbt.Server(params, device_budget_bytes=1 << 30, n_slots=1, slot_events=2, slot_hits=1 << 16,
                     max_wait_us=1000)
    # oversized and malformed events are refused at submission
    big = np.zeros(M + 1, np.int32)
    big[1:] = 65536
    z = np.zeros(65536, np.float32)
    assert srv.submit(1, big, z, z, z) == sbt.SBT_ERR_EVENT_TOO_LARGE
    bad = np.arange(M + 1, dtype=np.int32)
    bad[5] = 10
    z = np.zeros(M, np.float32)
    assert srv.submit(2, bad, z, z, z) == sbt.SBT_ERR_INVALID_ARG
    # the host queue holds n_slots * slot_events * 4 events, then refuses
    b = synth.make_batch("tiny", 1)
    ev = _event(b, 0)
    codes = [srv.submit(10 + i, *ev) for i in range(12)]
    assert codes[:8] == [0] * 8 and all(c == sbt.SBT_ERR_NOT_READY for c in codes[8:])
    got = _drain(srv, 8)
    assert sorted(got) == list(range(10, 18))
    assert srv.pending() == (0, 0)
    srv.close()


def test_empty_event_is_served():
    say("serving empty event")
    params = sbt.make_params(synth.PLANE_Z)
    srv = sbt.Server(params, device_budget_bytes=1 << 30, n_slots=1, slot_events=4, slot_hits=1 << 16)
    z = np.zeros(0, np.float32)
    assert srv.submit(7, np.zeros(27, np.int32), z, z, z) == 0
    got = _drain(srv, 1)
    st, tho, th, ts, td = got[7]
    assert st == 0 and list(tho) == [0] and th.size == 0
    srv.close()


def test_replay_driver_counts_match_oracle():
    """The C++ load replay (used for the serving measurements) returns every
    arrival, each with the track count of its event reconstructed alone."""
    say("serving replay driver")
    pool = synth.make_batch("serve", 40)
    want = oracle.reconstruct(pool)
    counts = np.diff(want[0])
    params = sbt.make_params(pool.module_z)
    srv = sbt.Server(params, device_budget_bytes=2 << 30, n_slots=3, slot_events=32, slot_hits=1 << 18,
                     max_wait_us=100)
    rng = np.random.default_rng(4)
    n = 400
    arrivals = np.cumsum(rng.exponential(50.0, n))
    picks = rng.integers(0, pool.n_events, n)
    lat, nt, wall = srv.replay(pool, arrivals, picks)
    srv.close()
    assert np.array_equal(nt, counts[picks])
    assert np.all(lat > 0) and wall > 0


def test_replay_refused_while_events_are_pending():
    """The replay driver matches results to arrivals by request id, so it is
    refused while events submitted earlier are queued, on the device or not
    yet collected; once they are drained it runs."""
    say("serving replay refused while busy")
    pool = synth.make_batch("serve", 6)
    params = sbt.make_params(pool.module_z)
    srv = sbt.Server(params, device_budget_bytes=1 << 30, n_slots=2, slot_events=8, slot_hits=1 << 17,
                     max_wait_us=100)
    assert srv.submit(123456789, *_event(pool, 0)) == 0
    with pytest.raises(sbt.SbtError) as ei:
        srv.replay(pool, np.zeros(3), np.array([0, 1, 2]))
    assert ei.value.code == sbt.SBT_ERR_NOT_READY
    got = _drain(srv, 1)
    assert list(got) == [123456789]
    assert srv.pending() == (0, 0)
    with pytest.raises(sbt.SbtError) as ei:
        srv.replay(pool, np.zeros(2), np.array([0, 6]))      # pick outside the pool
    assert ei.value.code == sbt.SBT_ERR_INVALID_ARG
    lat, nt, wall = srv.replay(pool, np.zeros(3), np.array([0, 1, 2]))
    assert np.array_equal(nt, np.diff(oracle.reconstruct(pool)[0])[[0, 1, 2]])
    srv.close()


def test_slow_consumer_holds_a_bounded_number_of_result_blocks():
    """A caller that takes one result per poll leaves completed results
    unreturned.  The server then holds at most 3 * n_slots + 2 pinned result
    blocks: further launches wait, their events stay queued, until polls have
    returned enough results.  Every event still comes back, equal to the
    oracle's."""
    say("serving with a slow consumer")
    b = synth.make_batch("tiny", 300)
    want = _oracle_tracks(b)
    params = sbt.make_params(b.module_z)
    srv = sbt.Server(params, device_budget_bytes=1 << 30, n_slots=2, slot_events=8, slot_hits=1 << 16,
                     max_wait_us=0)
    got, seen = {}, []
    e = 0
    t_end = time.time() + 120.0
    while len(got) < b.n_events:
        while e < b.n_events and srv.submit(e, *_event(b, e)) == 0:
            e += 1
        for (rid, st, tho, th, ts, td) in srv.poll(0, max_results=1):
            got[rid] = (st, tho, th)
        seen.append(srv.result_blocks())
        assert time.time() < t_end, f"serving stalled with {len(got)}/{b.n_events} results"
    srv.close()
    limit = seen[0][1]
    assert limit == 3 * 2 + 2
    assert max(n for n, _ in seen) == limit   # the limit was reached and held
    for i in range(b.n_events):
        st, tho, th = got[i]
        assert st == 0
        assert np.array_equal(tho, want[i][0]) and np.array_equal(th, want[i][1]), f"event {i}"
