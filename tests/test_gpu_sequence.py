"""GPU parity of the steps around the method in the paper's sequence
(Section 4): the global event cut inside the reconstruction, and
consolidation against the float64 oracle.

The consolidation oracle is fed the oracle's own tracks, and each test first
asserts that the GPU's tracks equal them byte for byte, so no input of the
comparison comes from the HIP path.

Tolerances of the binary32 fit (n hits, unit roundoff u = 2^-24, v one of
x, y, z; first-order error propagation, each bound taken twice or four
times as slack):
  - a mean: recursive summation of n terms errs by at most (n - 1) u sum|v|,
    so with the division a mean errs by at most n u max|v|; allowed 2 n u
    max|v| (call it dm_v).
  - a slope: a ratio of sums of products of centred values, each centred
    value carrying the mean's error: a few n u (|t| + sqrt(n) max|v - mean|
    / sqrt(Szz)); allowed 4 n u (...) (call it dt).
  - chi2 / (2n - 4): every residual r = v - (vm + t dz), dz = z - zm, is
    computed from the rounded mean and slope, so it errs by at most
    e = dm_v + |t| (dm_z + u |dz|) + |dz| dt + u (|t dz| + |vm + t dz| + |r|);
    a square then errs by 2 |r| e + e^2, and the sum of n squares by the sum
    of those plus n u chi2; the division adds u chi2 / (2n - 4).  Allowed
    twice that.
Packed coordinates are copies: exact.
"""

import sys

import numpy as np
import pytest

import oracle
import oracle.sequence as seq
from _util import rounded_to_f16
from paper_2207_03936_amd import sbt, synth

pytestmark = pytest.mark.gpu
U = 2.0 ** -24


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


@pytest.mark.parametrize("form", ["plain", "batched", "f16"])
def test_event_cut_matches_oracle(form):
    b = synth.make_batch("mu7.6", 60)
    c = sbt.sbt_gec_threshold(b.event_offsets, 0.1)
    say(f"event cut {form}, threshold {c}")
    p = sbt.make_params(b.module_z, max_event_hits=c)
    if form == "plain":
        got = sbt.sbt_reconstruct(p, sbt.DeviceBatch(b)).to_host()
        want = oracle.reconstruct(b, max_event_hits=c)
    else:
        ctx = sbt.Context(p, b.n_events, b.n_hits)
        if form == "batched":
            got = ctx.reconstruct(sbt.DeviceBatch(b)).to_host()
            want = oracle.reconstruct(b, max_event_hits=c)
        else:
            got = ctx.reconstruct_f16(sbt.DeviceBatchF16(b)).to_host()
            want = oracle.reconstruct(rounded_to_f16(b), max_event_hits=c)
        ctx.close()
    for g, w in zip(got[:3], want):
        assert np.array_equal(g, w)
    sizes = np.diff(b.event_offsets)
    assert np.array_equal(got[3], np.where(sizes > c, sbt.SBT_EV_CUT, 0))
    assert (sizes > c).sum() == 6


def _check_states(b, got_tracks, got_states, **params):
    """The GPU's tracks equal the oracle's; the GPU's consolidation of them
    equals the float64 consolidation of the oracle's tracks, within the
    derived bounds."""
    eto, tho, th = oracle.reconstruct(b, **params)
    for g, w, what in zip(got_tracks[:3], (eto, tho, th), ("event track offsets", "track hit offsets", "hits")):
        assert np.array_equal(g, w), f"GPU tracks differ from the oracle's: {what}"
    px, py, pz, st = seq.consolidate(b, eto, tho, th)
    gx, gy, gz, gs = got_states
    assert np.array_equal(gx, px) and np.array_equal(gy, py) and np.array_equal(gz, pz)
    assert gs.shape == st.shape
    for t in range(st.shape[0]):
        lo, hi = int(tho[t]), int(tho[t + 1])
        n = hi - lo
        x, y, z = (v[lo:hi].astype(np.float64) for v in (px, py, pz))
        dm = [2 * n * U * np.abs(v).max() for v in (x, y, z)]
        rz = np.sqrt(((z - z.mean()) ** 2).sum())
        dt = [4 * n * U * (abs(st[t, 3 + j]) + np.sqrt(n) * np.abs(v - v.mean()).max() / rz)
              for j, v in enumerate((x, y))]
        zm = st[t, 2]
        dz = z - zm
        c2_err, c2 = 0.0, 0.0
        for j, v in enumerate((x, y)):
            vm, tv = st[t, j], st[t, 3 + j]
            r = v - (vm + tv * dz)
            e = (dm[j] + abs(tv) * (dm[2] + U * np.abs(dz)) + np.abs(dz) * dt[j]
                 + U * (np.abs(tv * dz) + np.abs(vm + tv * dz) + np.abs(r)))
            c2_err += float((2 * np.abs(r) * e + e * e).sum())
            c2 += float((r * r).sum())
        tol_c2 = 2 * (c2_err + n * U * c2 + U * c2) / (2 * n - 4)
        tol = np.array(dm + dt + [tol_c2])
        err = np.abs(gs[t].astype(np.float64) - st[t])
        assert np.all(err <= tol), (t, gs[t], st[t], err, tol)


@pytest.mark.parametrize("config,n", [("tiny", 30), ("mu7.6", 40), ("pairs7.6", 40), ("mu30", 4)])
def test_consolidate_matches_oracle(config, n):
    import torch
    say(f"consolidate {config} x{n}")
    b = synth.make_batch(config, n)
    p = sbt.make_params(b.module_z)
    dev = sbt.DeviceBatch(b)
    ctx = sbt.Context(p, b.n_events, b.n_hits)
    out = ctx.reconstruct(dev)
    states = sbt.sbt_consolidate(dev, out)
    torch.cuda.synchronize()
    tracks = out.to_host()[:3]
    _check_states(b, tracks, states.to_host(tracks[0][-1], tracks[1][-1]))
    ctx.close()


def test_consolidate_into_pinned_host_memory():
    import torch
    say("consolidate into pinned host memory")
    b = synth.make_batch("mu1-25", 20)
    dev = sbt.DeviceBatch(b)
    out = sbt.sbt_reconstruct(sbt.make_params(b.module_z), dev)
    states = sbt.sbt_consolidate(dev, out, sbt.TrackStates(b.n_hits, pinned=True))
    torch.cuda.synchronize()
    tracks = out.to_host()[:3]
    _check_states(b, tracks, states.to_host(tracks[0][-1], tracks[1][-1]))


def test_consolidate_empty_batch_and_trackless_events():
    import torch
    say("consolidate empty batch and events without tracks")
    b0 = synth.make_batch("tiny", 0)
    d0 = sbt.DeviceBatch(b0)
    sbt.sbt_consolidate(d0, sbt.sbt_reconstruct(sbt.make_params(b0.module_z), d0))
    b = synth.make_batch("mu7.6", 10)
    c = sbt.sbt_gec_threshold(b.event_offsets, 0.5)
    p = sbt.make_params(b.module_z, max_event_hits=c)
    dev = sbt.DeviceBatch(b)
    out = sbt.sbt_reconstruct(p, dev)
    states = sbt.sbt_consolidate(dev, out)
    torch.cuda.synchronize()
    eto, tho, th, st = out.to_host()
    _check_states(b, (eto, tho, th), states.to_host(eto[-1], tho[-1]), max_event_hits=c)


def test_consolidate_tracks_longer_than_the_register_path():
    """48 modules: tracks of up to 48 hits take the path that reads the hits
    again for every pass of the fit."""
    import torch
    say("consolidate 48-module tracks")
    rng = np.random.default_rng(12)
    mz = (-500.0 + 25.0 * np.arange(48)).astype(np.float32)
    events = []
    for _ in range(6):
        per = [[] for _ in range(mz.size)]
        for _ in range(5):
            phi = rng.uniform(-np.pi, np.pi)
            slope = rng.uniform(0.01, 0.03)
            x0, y0 = rng.normal(0, 0.01, 2)
            for k in range(mz.size):
                r = slope * (mz[k] + 800.0)
                per[k].append((x0 + r * np.cos(phi) + rng.normal(0, 0.01), y0 + r * np.sin(phi) + rng.normal(0, 0.01)))
        xs = np.array([h[0] for p in per for h in p], np.float32)
        ys = np.array([h[1] for p in per for h in p], np.float32)
        zs = np.repeat(mz, [len(p) for p in per]).astype(np.float32)
        events.append(dict(x=xs, y=ys, z=zs, module_counts=np.array([len(p) for p in per], np.int64),
                           truth=np.full(xs.size, -1, np.int32)))
    b = synth.concat(events, mz)
    dev = sbt.DeviceBatch(b)
    out = sbt.sbt_reconstruct(sbt.make_params(b.module_z), dev)
    states = sbt.sbt_consolidate(dev, out)
    torch.cuda.synchronize()
    eto, tho, th, st = out.to_host()
    assert np.diff(tho).max() > 32
    _check_states(b, (eto, tho, th), states.to_host(eto[-1], tho[-1]))
