"""Pins of the steps around the method in the paper's sequence (Section 4):
the global event cut and consolidation (oracle), and the library's host-side
event-cut threshold against the oracle."""

import numpy as np
import pytest

import oracle
import oracle.sequence as seq
from _util import tracks_per_event
from paper_2207_03936_amd import synth


# ------------------------------------------------------------ global event cut

def test_gec_threshold_examples():
    assert seq.gec_threshold(np.arange(1, 11), 0.1) == 9        # rejects only the 10-hit event
    assert seq.gec_threshold(np.arange(1, 11), 0.25) == 8       # floor(2.5) = 2 rejected
    assert seq.gec_threshold([5, 5, 5, 5], 0.5) == 5            # ties are kept: nobody rejected
    assert seq.gec_threshold([7, 3, 9], 0.0) == 9               # nothing rejected
    assert seq.gec_threshold([0, 0, 3], 1.0) == 1               # at least one hit
    assert seq.gec_threshold([], 0.1) == 1


def test_gec_threshold_brute_force():
    """Against the definition over every integer threshold."""
    rng = np.random.default_rng(3)
    for _ in range(300):
        sizes = rng.integers(0, 30, int(rng.integers(0, 25)))
        f = float(rng.choice([0.0, 0.1, 0.25, 0.5, 0.9, 1.0, rng.random()]))
        k = int(np.floor(f * sizes.size))
        want = next(c for c in range(1, 32) if int((sizes > c).sum()) <= k)
        assert seq.gec_threshold(sizes, f) == want
        keep = seq.gec_keep(sizes, f)
        assert (~keep).sum() <= k and np.all(sizes[~keep] > sizes[keep].max(initial=0))


def test_library_gec_threshold_matches_oracle():
    from paper_2207_03936_amd import sbt
    rng = np.random.default_rng(4)
    for _ in range(200):
        sizes = rng.integers(0, 12000, int(rng.integers(0, 2000)))
        f = float(rng.choice([0.0, 0.1, 0.5, 1.0, rng.random()]))
        eo = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
        assert sbt.sbt_gec_threshold(eo, f) == seq.gec_threshold(sizes, f)
    b = synth.make_batch("mu7.6", 200)
    sizes = np.diff(b.event_offsets)
    c = sbt.sbt_gec_threshold(b.event_offsets, 0.1)
    assert c == seq.gec_threshold(sizes, 0.1) and (sizes > c).sum() == 20


def test_library_gec_threshold_rejects_bad_arguments():
    from paper_2207_03936_amd import sbt
    with pytest.raises(sbt.SbtError):
        sbt.sbt_gec_threshold(np.array([0, 5, 3], np.int32), 0.1)   # decreasing offsets
    with pytest.raises(sbt.SbtError):
        sbt.sbt_gec_threshold(np.array([0, 5], np.int32), 1.5)


def test_cut_events_get_no_tracks_and_others_are_unchanged():
    b = synth.make_batch("mu7.6", 30)
    sizes = np.diff(b.event_offsets)
    c = seq.gec_threshold(sizes, 0.1)
    full = tracks_per_event(*oracle.reconstruct(b))
    cut = tracks_per_event(*oracle.reconstruct(b, max_event_hits=c))
    for e in range(b.n_events):
        assert cut[e] == ([] if sizes[e] > c else full[e])
    assert sum(1 for e in range(b.n_events) if sizes[e] > c) == 3


# ------------------------------------------------------------ consolidation

def test_fit_recovers_an_exact_line():
    z = np.array([-275.0, -115.0, 5.0, 125.0, 525.0])
    x = 1.5 + 0.031 * z
    y = -0.25 - 0.0125 * z
    xm, ym, zm, tx, ty, c = seq.fit_line(x, y, z)
    assert zm == pytest.approx(z.mean(), abs=1e-12)
    assert xm == pytest.approx(1.5 + 0.031 * zm, abs=1e-12)
    assert ym == pytest.approx(-0.25 - 0.0125 * zm, abs=1e-12)
    assert tx == pytest.approx(0.031, abs=1e-14) and ty == pytest.approx(-0.0125, abs=1e-14)
    assert c == pytest.approx(0.0, abs=1e-20)


def test_fit_three_points_by_hand():
    # z = -1, 0, 1; x = 0, 1, 0 -> mean 1/3, slope 0, residuals -1/3, 2/3, -1/3
    xm, ym, zm, tx, ty, c = seq.fit_line([0.0, 1.0, 0.0], [0.0, 0.0, 0.0], [-1.0, 0.0, 1.0])
    assert (xm, zm, tx, ty) == pytest.approx((1 / 3, 0.0, 0.0, 0.0))
    assert c == pytest.approx((1 / 9 + 4 / 9 + 1 / 9) / 2)       # 2n - 4 = 2


def test_fit_matches_numpy_polyfit():
    rng = np.random.default_rng(9)
    for _ in range(200):
        n = int(rng.integers(3, 27))
        z = np.sort(rng.uniform(-300, 750, n))
        x = rng.normal(0, 10) + rng.normal(0, 0.1) * z + rng.normal(0, 0.02, n)
        y = rng.normal(0, 10) + rng.normal(0, 0.1) * z + rng.normal(0, 0.02, n)
        xm, ym, zm, tx, ty, c = seq.fit_line(x, y, z)
        px, py = np.polyfit(z, x, 1), np.polyfit(z, y, 1)
        assert tx == pytest.approx(px[0], rel=1e-9, abs=1e-12)
        assert ty == pytest.approx(py[0], rel=1e-9, abs=1e-12)
        assert xm == pytest.approx(np.polyval(px, zm), abs=1e-9)
        assert ym == pytest.approx(np.polyval(py, zm), abs=1e-9)
        r = np.concatenate([x - np.polyval(px, z), y - np.polyval(py, z)])
        assert c == pytest.approx(float((r * r).sum()) / (2 * n - 4), rel=1e-7, abs=1e-15)


def test_consolidate_packs_the_track_hits():
    b = synth.make_batch("pairs7.6", 4)
    eto, tho, th = oracle.reconstruct(b)
    px, py, pz, st = seq.consolidate(b, eto, tho, th)
    assert px.dtype == np.float32 and st.shape == (int(eto[-1]), 6)
    for e in range(b.n_events):
        base = int(b.event_offsets[e])
        for t in range(int(eto[e]), int(eto[e + 1])):
            ids = base + th[tho[t]:tho[t + 1]]
            assert np.array_equal(px[tho[t]:tho[t + 1]], b.x[ids])
            assert np.array_equal(pz[tho[t]:tho[t + 1]], b.z[ids])
    # straight tracks with 12 um smearing: chi2 per degree of freedom of order sigma^2
    assert np.median(st[:, 5]) < 4 * 0.012 ** 2
