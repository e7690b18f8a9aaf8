"""Pins of the oracle's building blocks against what mathematics fixes.

Each test compares the oracle with an independent formulation: a float64
library routine, a closed form or a direct enumeration of the definition
(paper, Section 3).
"""

import math
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _exact_q(x, y):
    """Nearest phi16 of the true angle, in float64 (mod 2^16)."""
    a = np.arctan2(np.asarray(y, np.float64), np.asarray(x, np.float64))
    return np.round(a * 32768.0 / np.pi).astype(np.int64) & 0xFFFF


def _circ(a, b):
    d = (np.asarray(a, np.int64) - np.asarray(b, np.int64)) % 65536
    return np.minimum(d, 65536 - d)


# ---------------------------------------------------------------- phi16 (Sort by phi)

def test_phi16_within_one_unit_of_float64_atan2():
    rng = np.random.default_rng(11)
    n = 1_000_000
    r = np.sqrt(rng.uniform(5.1 ** 2, 42.0 ** 2, n))
    ang = rng.uniform(-np.pi, np.pi, n)
    x = (r * np.cos(ang)).astype(np.float32)
    y = (r * np.sin(ang)).astype(np.float32)
    q = oracle.phi16(x, y)
    d = _circ(q, _exact_q(x, y))
    assert d.max() <= 1
    # the approximation error is 0.12 units, so almost every value is the nearest one
    assert (d == 0).mean() > 0.7


def test_phi16_wide_dynamic_range():
    rng = np.random.default_rng(12)
    n = 200_000
    x = (rng.standard_normal(n) * 10.0 ** rng.uniform(-20, 20, n)).astype(np.float32)
    y = (rng.standard_normal(n) * 10.0 ** rng.uniform(-20, 20, n)).astype(np.float32)
    ok = (x != 0) | (y != 0)
    q = oracle.phi16(x[ok], y[ok])
    assert _circ(q, _exact_q(x[ok], y[ok])).max() <= 1


def test_phi16_golden_points():
    """Points on the axes and diagonals map to exact multiples of 2^16/8
    (closed forms of the 16-bit angle; -pi and +pi are the same point)."""
    rows = []
    with open(os.path.join(GOLDEN, "phi16_closed_forms.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                xs, ys, qs = line.split()
                rows.append((float(xs), float(ys), int(qs)))
    assert len(rows) >= 10
    for x, y, q in rows:
        assert int(oracle.phi16([x], [y])[0]) == q, (x, y, q)


def test_phi16_monotone_sweep():
    """Along a dense counter-clockwise sweep the 16-bit angle never steps back."""
    ang = np.linspace(-np.pi, np.pi, 400_001)
    for r in (5.1, 17.0, 42.0):
        x = (r * np.cos(ang)).astype(np.float32)
        y = (r * np.sin(ang)).astype(np.float32)
        q = oracle.phi16(x, y).astype(np.int64)
        step = (np.diff(q) + 32768) % 65536 - 32768
        assert step.min() >= 0
        assert step.max() <= 2


def test_phi16_reflections():
    """phi16 is odd under y -> -y (mod 2^16) up to one unit of rounding."""
    rng = np.random.default_rng(13)
    x = rng.uniform(-40, 40, 100_000).astype(np.float32)
    y = rng.uniform(-40, 40, 100_000).astype(np.float32)
    q = oracle.phi16(x, y).astype(np.int64)
    qm = oracle.phi16(x, -y).astype(np.int64)
    assert _circ(q, (-qm) & 0xFFFF).max() <= 1


# ---------------------------------------------------------------- window membership

@pytest.mark.parametrize("w", [0, 1, 7, 416, 16384, 32767])
def test_window_membership_exhaustive(w):
    """Inclusive window on the circle: circular distance <= w, checked for all
    2^16 values against a few centres (including the wrap-around ones)."""
    qs = np.arange(65536)
    for centre in (0, 1, 416, 32768, 65535, 40000):
        expect = _circ(qs, centre) <= w
        # sample the oracle on every value near the edges and a stride elsewhere
        near = np.nonzero(np.abs(_circ(qs, centre) - w) <= 2)[0]
        probe = np.unique(np.concatenate([near, qs[::97], [centre, (centre + 32768) % 65536]]))
        got = np.array([oracle.in_window(int(q), centre, w) for q in probe])
        assert np.array_equal(got, expect[probe]), (w, centre)


# ---------------------------------------------------------------- sort

def test_sort_matches_lexsort():
    from paper_2207_03936_amd import synth
    b = synth.make_batch("mu30", 2)
    M = b.n_modules
    for e in range(b.n_events):
        lo, hi = int(b.event_offsets[e]), int(b.event_offsets[e + 1])
        mo = b.module_offsets[e * M:(e + 1) * M + 1] - lo
        x, y = b.x[lo:hi], b.y[lo:hi]
        got = oracle.sort_event(mo, x, y)
        q = oracle.phi16(x, y)
        for k in range(M):
            ids = np.arange(mo[k], mo[k + 1])
            want = ids[np.lexsort((ids, q[ids]))]
            assert np.array_equal(got[mo[k]:mo[k + 1]], want)


def test_sort_ties_by_lower_id():
    # duplicated coordinates give equal phi16: the lower id must come first
    x = np.array([3.0, 3.0, -1.0, 3.0, 5.0, -1.0], np.float32)
    y = np.array([4.0, 4.0, 2.0, 4.0, 0.5, 2.0], np.float32)
    got = oracle.sort_event(np.array([0, 6]), x, y)
    q = oracle.phi16(x, y)
    want = np.lexsort((np.arange(6), q))
    assert np.array_equal(got, want)


# ---------------------------------------------------------------- pendulum

def _pendulum_by_definition(q_sorted, flagged, target, k):
    """The pendulum as an ordered enumeration: offsets from the start position
    in order of (|offset|, offset > 0) -- 0, -1, +1, -2, +2, ... -- restricted
    to n consecutive offsets, mapped onto positions modulo n."""
    n = len(q_sorted)
    if n == 0:
        return []
    s0 = int(np.searchsorted(np.asarray(q_sorted), target, side="left"))
    if s0 == n:
        s0 = 0
    offsets = sorted(range(-(n // 2), n - n // 2), key=lambda o: (abs(o), o > 0))
    out = []
    for o in offsets:
        pos = (s0 + o) % n
        if not flagged[pos]:
            out.append(pos)
        if len(out) == k:
            break
    return out


def test_pendulum_random():
    rng = np.random.default_rng(21)
    for _ in range(3000):
        n = int(rng.integers(0, 20))
        q = np.sort(rng.integers(0, 65536, n)).astype(np.uint16)
        flagged = (rng.random(n) < rng.uniform(0, 0.9)).astype(np.uint8)
        target = int(rng.integers(0, 65536))
        if n and rng.random() < 0.3:
            target = int(q[rng.integers(0, n)])     # exact phi matches
        k = int(rng.integers(1, 8))
        assert list(oracle.pendulum(q, flagged, target, k)) == _pendulum_by_definition(q, flagged, target, k)


def test_pendulum_figure_case():
    """Four unflagged hits nearest in index to the target are taken and the
    flagged hits interleaved with them are skipped (the paper's pendulum
    figure: flagged c_a, c_d, c_e)."""
    q = np.array([100, 200, 300, 400, 500, 600, 700, 800], np.uint16)
    flagged = np.array([0, 0, 1, 0, 1, 1, 0, 0], np.uint8)
    # target 450 -> start at position 4 (first >= 450): visits 4F,3,5F,2F,6,1,7 ...
    got = list(oracle.pendulum(q, flagged, 450, 4))
    assert got == [3, 6, 1, 7]
    # target beyond the last value starts at 0 and wraps downwards to 7
    assert list(oracle.pendulum(q, flagged, 900, 3)) == [0, 7, 1]


# ---------------------------------------------------------------- tracklet chi2

def test_chi2_matches_float64_lstsq():
    rng = np.random.default_rng(31)
    for _ in range(2000):
        z = np.sort(rng.choice(np.arange(-275, 726, 40), 3, replace=False)).astype(np.float32)
        if rng.random() < 0.5:
            z = z[::-1].copy()
        x = rng.uniform(-40, 40, 3).astype(np.float32)
        y = rng.uniform(-40, 40, 3).astype(np.float32)
        got = oracle.tracklet_chi2(x, y, z)
        A = np.stack([np.ones(3), z.astype(np.float64)], axis=1)
        ssr = 0.0
        for v in (x, y):
            c, *_ = np.linalg.lstsq(A, v.astype(np.float64), rcond=None)
            ssr += float(((A @ c - v) ** 2).sum())
        assert got == pytest.approx(ssr, rel=2e-4, abs=1e-4)


def test_chi2_collinear_is_zero_and_scatter_identity():
    # exactly collinear binary32 points on a line with power-of-two slopes
    z = np.array([725.0, 685.0, 645.0], np.float32)
    x = np.array([10.0, 9.5, 9.0], np.float32)
    y = np.array([-4.0, -3.75, -3.5], np.float32)
    assert oracle.tracklet_chi2(x, y, z) == 0.0
    # chi2 * |v|^2 == scatter * (z1 - z0)^2 for the scatter of the third hit
    # against the line of the first two (float64 closed form)
    rng = np.random.default_rng(32)
    for _ in range(500):
        z = np.array([725.0, 685.0, 605.0], np.float32)
        x = rng.uniform(5, 40, 3).astype(np.float32)
        y = rng.uniform(5, 40, 3).astype(np.float32)
        zf, xf, yf = (v.astype(np.float64) for v in (z, x, y))
        tx = (xf[1] - xf[0]) / (zf[1] - zf[0])
        ty = (yf[1] - yf[0]) / (zf[1] - zf[0])
        dx = xf[1] + tx * (zf[2] - zf[1]) - xf[2]
        dy = yf[1] + ty * (zf[2] - zf[1]) - yf[2]
        v = np.array([zf[2] - zf[1], zf[0] - zf[2], zf[1] - zf[0]])
        want = (dx * dx + dy * dy) * (zf[1] - zf[0]) ** 2 / (v @ v)
        assert oracle.tracklet_chi2(x, y, z) == pytest.approx(want, rel=1e-3, abs=1e-6)


def test_phi16_coefficients_follow_their_derivation():
    """The oracle's polynomial literals are the binary32 rounding of the
    float64 fit in oracle/derive_phi16.py, and that fit's binary32 error is
    within 0.15 phi16 units."""
    import re
    import sys
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.dirname(__file__)), "oracle"))
    import derive_phi16
    c = derive_phi16.fit()
    src = open(os.path.join(os.path.dirname(os.path.dirname(__file__)), "oracle", "sbt_oracle.c")).read()
    lits = [float.fromhex(m) for m in re.findall(r"ORC_C\d = (-?0x[0-9a-f.p+-]+)f;", src)]
    assert len(lits) == 5
    assert [float(v) for v in c] == lits
    assert derive_phi16.max_error(c) * 32768 / np.pi < 0.15
