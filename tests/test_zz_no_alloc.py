"""The batched entry point that allocates nothing (sbt_reconstruct_batched_static):
called through the C ABI, its outputs equal those of sbt_reconstruct_batched
on the same inputs and the oracle's, on two calls in a row (the second with a
smaller batch, so the static scratch still holds the first call's contents),
a batch beyond the scratch capacity is refused before any launch, and the
call can be captured into a caller's graph.  The file name sorts last so
that it also runs after every other GPU test."""

import ctypes
import sys

import numpy as np
import pytest

import oracle
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


def _static_call(params, dev, out, stream):
    return sbt.lib().sbt_reconstruct_batched_static(ctypes.byref(params), ctypes.byref(dev.hits),
                                                    ctypes.byref(out.tracks), ctypes.c_void_p(stream))


def _same(a, b, what):
    for x, y, name in zip(a[:4], b[:4], ("event track offsets", "track hit offsets", "track hits", "status")):
        assert np.array_equal(x, y), f"{what}: {name} differ"


@pytest.mark.parametrize("on_stream", [False, True])
def test_static_scratch_equals_context_path(on_stream):
    import torch
    big = synth.make_batch("mu7.6", 150, first=0)          # about 500,000 hits
    small = synth.make_batch("mu1-25", 12, first=300)
    assert sbt.sbt_workspace_size(big.n_events, big.n_hits) <= sbt.STATIC_SCRATCH_BYTES
    stream = torch.cuda.Stream() if on_stream else torch.cuda.current_stream()
    handle = stream.cuda_stream
    for name, b in (("mu7.6 x150", big), ("mu1-25 x12", small)):
        say(f"static scratch {name} ({b.n_hits} hits), {'own stream' if on_stream else 'null stream'}")
        p = sbt.make_params(b.module_z)
        dev = sbt.DeviceBatch(b)
        out = sbt.DeviceTracks(b.n_events, b.n_hits)
        with torch.cuda.stream(stream):
            out.fill_(-1)
            assert _static_call(p, dev, out, handle) == sbt.SBT_OK
        stream.synchronize()
        got = out.to_host()
        ctx = sbt.Context(p, b.n_events, b.n_hits)
        ref = ctx.reconstruct(dev).to_host()
        ctx.close()
        _same(got, ref, f"static vs context, {name}")
        want = oracle.reconstruct(b)
        for x, y in zip(got[:3], want):
            assert np.array_equal(x, y), f"static vs oracle, {name}"
        assert not got[3].any()


def test_static_scratch_refuses_oversized_batch():
    say("static scratch: oversized batch refused")
    b = synth.make_batch("mu7.6", 250)       # about 830,000 hits: beyond the scratch
    assert sbt.sbt_workspace_size(b.n_events, b.n_hits) > sbt.STATIC_SCRATCH_BYTES
    p = sbt.make_params(b.module_z)
    dev = sbt.DeviceBatch(b)
    out = sbt.DeviceTracks(b.n_events, b.n_hits).fill_(-7)
    assert _static_call(p, dev, out, 0) == sbt.SBT_ERR_WORKSPACE
    import torch
    torch.cuda.synchronize()
    assert int(out.eto[0]) == -7, "a refused call wrote outputs"


def test_static_scratch_under_caller_graph_capture():
    """Captured into a caller's HIP graph (torch.cuda.graph) and replayed
    three times, with the outputs overwritten eagerly between replays: every
    replay equals the oracle."""
    import torch
    torch.cuda.set_device(0)
    b = synth.make_batch("mu7.6", 60, first=500)
    want = oracle.reconstruct(b)
    p = sbt.make_params(b.module_z)
    dev = sbt.DeviceBatch(b)
    out = sbt.DeviceTracks(b.n_events, b.n_hits)
    s = torch.cuda.Stream()
    say("static scratch: eager call before capture")
    with torch.cuda.stream(s):
        assert _static_call(p, dev, out, s.cuda_stream) == sbt.SBT_OK
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    say("static scratch: capture")
    with torch.cuda.graph(g, stream=s):
        rc = _static_call(p, dev, out, torch.cuda.current_stream().cuda_stream)
    assert rc == sbt.SBT_OK
    for rep in range(3):
        say(f"static scratch: replay {rep}")
        out.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = out.to_host()
        for x, y in zip(got[:3], want):
            assert np.array_equal(x, y), f"replay {rep} differs from the oracle"
        assert not got[3].any()
