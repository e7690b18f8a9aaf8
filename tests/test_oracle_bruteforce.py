"""The oracle's search mechanics against exhaustive enumeration on tiny events.

With loose thresholds many triplets, follow-up hits and claims compete, so a
wrong index, a wrong window edge, a wrong pendulum order, a wrong tie-break or
a wrong claim rule changes the track set.
"""

import numpy as np
import pytest

import oracle
from bruteforce import reconstruct_event
from _util import event_batch, tiny_random_event, tracks_per_event


def _params(rng):
    return dict(
        reverse=int(rng.integers(0, 2)),
        max_doublet_candidates=int(rng.choice([1, 2, 3, 4, 8, 64])),
        phi_window_seeding=int(rng.choice([20, 60, 416, 32767])),
        phi_window_forwarding=int(rng.choice([20, 60, 416, 32767])),
        max_scatter_seeding=float(rng.choice([0.01, 0.05, 1.0, 20.0])),
        max_scatter_forwarding=float(rng.choice([0.01, 0.05, 1.0, 20.0])),
        max_tracklet_chi2=float(rng.choice([0.001, 0.05, 5.0])),
        max_consecutive_misses=int(rng.choice([0, 1, 2])),
    )


def _run_both(ev, p):
    x, y, z, mo, mz = ev
    got = tracks_per_event(*oracle.reconstruct(event_batch(x, y, z, mo, mz), **p))[0]
    want = reconstruct_event(
        x, y, z, mo, mz, reverse=p["reverse"], K=p["max_doublet_candidates"],
        Ws=p["phi_window_seeding"], Wf=p["phi_window_forwarding"],
        Ss=p["max_scatter_seeding"], Sf=p["max_scatter_forwarding"],
        X=p["max_tracklet_chi2"], misses=p["max_consecutive_misses"])
    return got, [tuple(t) for t in want]


@pytest.mark.parametrize("seed", range(8))
def test_exhaustive_full_windows(seed):
    """K >= n and W = 32767: seeding and following reduce to the exhaustive
    argmin over all triplets / all next-module hits under threshold."""
    rng = np.random.default_rng(1000 + seed)
    n_nonempty = 0
    for _ in range(40):
        ev = tiny_random_event(rng)
        p = _params(rng)
        p.update(max_doublet_candidates=64, phi_window_seeding=32767, phi_window_forwarding=32767)
        got, want = _run_both(ev, p)
        assert got == want
        n_nonempty += bool(got)
    assert n_nonempty > 10


@pytest.mark.parametrize("seed", range(8))
def test_exhaustive_random_parameters(seed):
    """Pendulum with K < n, narrow windows, z off the nominal module z, both
    traversal directions and 0..2 allowed misses."""
    rng = np.random.default_rng(2000 + seed)
    n_nonempty = 0
    for _ in range(40):
        ev = tiny_random_event(rng, jitter_z=bool(rng.integers(0, 2)))
        p = _params(rng)
        got, want = _run_both(ev, p)
        assert got == want
        n_nonempty += bool(got)
    assert n_nonempty > 5


def test_exact_ties_broken_by_lower_ids():
    """Two identical hits in the third module give equal scatters: the seed
    and the follow-up take the lower id."""
    mz = np.array([0.0, 40.0, 80.0, 120.0], np.float32)
    # module 3 (first in reverse traversal) .. module 0
    pts = {3: [(12.0, 0.0)], 2: [(11.0, 0.0)], 1: [(10.0, 0.0), (10.0, 0.0)], 0: [(9.0, 0.0), (9.0, 0.0)]}
    xs, ys, zs, counts = [], [], [], []
    for k in range(4):
        counts.append(len(pts[k]))
        for (a, b) in pts[k]:
            xs.append(a); ys.append(b); zs.append(mz[k])
    mo = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    ev = (np.array(xs, np.float32), np.array(ys, np.float32), np.array(zs, np.float32), mo, mz)
    got, want = _run_both(ev, dict(oracle.DEFAULTS))
    assert got == want
    # ids: module0 -> 0,1 ; module1 -> 2,3 ; module2 -> 4 ; module3 -> 5
    assert got == [(5, 4, 2, 0)]
