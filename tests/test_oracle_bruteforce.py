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


def _event_from_modules(pts, mz):
    xs, ys, zs, counts = [], [], [], []
    for k in range(len(mz)):
        counts.append(len(pts.get(k, [])))
        for (a, b) in pts.get(k, []):
            xs.append(a); ys.append(b); zs.append(mz[k])
    mo = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    return (np.array(xs, np.float32), np.array(ys, np.float32), np.array(zs, np.float32), mo,
            np.asarray(mz, np.float32))


def test_seed_tie_breaks_on_first_hit_then_third():
    """Mirror-image doublets give two exactly-zero scatters, (a, d) and
    (b, c) with a < b and c < d: the seed is the lexicographic minimum of
    (scatter, id of first hit, id of third hit), i.e. (a, d)."""
    mz = [0.0, 40.0, 80.0]
    # reverse traversal: first module is index 2, middle 1, third 0
    # module 0 (third): c=(10,+0.5) id 0, d=(10,-0.5) id 1
    # module 1 (middle): (10, 0) id 2
    # module 2 (first): a=(10,+0.5) id 3, b=(10,-0.5) id 4
    ev = _event_from_modules({0: [(10.0, 0.5), (10.0, -0.5)], 1: [(10.0, 0.0)],
                              2: [(10.0, 0.5), (10.0, -0.5)]}, mz)
    p = dict(oracle.DEFAULTS)
    got, want = _run_both(ev, p)
    assert got == want == [(3, 2, 1)]


def _straight_event(mz, x0, y0, tx, ty, zv=0.0):
    pts = {k: [(x0 + tx * (z - zv), y0 + ty * (z - zv))] for k, z in enumerate(mz)}
    return _event_from_modules(pts, mz)


def test_thresholds_are_strict():
    """A scatter or chi2 exactly equal to its threshold is rejected; the next
    binary32 value above it accepts (strict '<' reading)."""
    mz = [0.0, 40.0, 80.0]
    x, y, z, mo, mzf = _event_from_modules({0: [(10.05, 0.1)], 1: [(10.0, 0.0)], 2: [(10.0, 0.0)]}, mz)
    # reverse traversal: h0 = module 2 (id 2), h1 = module 1 (id 1), h2 = module 0 (id 0)
    F = np.float32
    d01 = F(z[1] - z[2]); tx = F(F(x[1] - x[2]) / d01); ty = F(F(y[1] - y[2]) / d01)
    dz = F(z[0] - z[1]); dx = F(F(x[1] + F(tx * dz)) - x[0]); dy = F(F(y[1] + F(ty * dz)) - y[0])
    sc = F(F(dx * dx) + F(dy * dy))
    chi2 = F(oracle.tracklet_chi2(x[[2, 1, 0]], y[[2, 1, 0]], z[[2, 1, 0]]))
    assert sc > 0 and chi2 > 0
    up = lambda v: float(np.nextafter(F(v), F(np.inf)))
    base = dict(oracle.DEFAULTS, max_tracklet_chi2=1.0)
    ev = (x, y, z, mo, mzf)
    assert _run_both(ev, dict(base, max_scatter_seeding=float(sc)))[0] == []
    assert _run_both(ev, dict(base, max_scatter_seeding=up(sc)))[0] == [(2, 1, 0)]
    base = dict(oracle.DEFAULTS, max_scatter_seeding=1.0)
    assert _run_both(ev, dict(base, max_tracklet_chi2=float(chi2)))[0] == []
    assert _run_both(ev, dict(base, max_tracklet_chi2=up(chi2)))[0] == [(2, 1, 0)]


def test_following_never_meets_a_flagged_hit():
    """The following search into a module never finds a flagged hit there:
    hits are flagged only when their module is resolved, which comes after
    its search (the step order of Section 3).  The HIP path relies on this
    to skip the flag test in its following search."""
    import bruteforce
    rng = np.random.default_rng(77)
    bruteforce.FLAGGED_FOLLOW_CANDIDATES[0] = 0
    n_tracks = 0
    for _ in range(60):
        ev = tiny_random_event(rng)
        p = _params(rng)
        got, want = _run_both(ev, p)
        assert got == want
        n_tracks += len(want)
    assert n_tracks > 50
    assert bruteforce.FLAGGED_FOLLOW_CANDIDATES[0] == 0
