"""The steps around Search by triplet in the paper's reconstruction sequence
(Section 4): the global event cut before it and the consolidation after it.
Test infrastructure only, like the rest of this package.

Global event cut.  The sequence rejects the most densely populated tenth of
the events.  Reading: density is the event's hit count; the cut is a hit-count
threshold of at least one hit, the smallest one that leaves at most
floor(fraction * E) events above it; events with more hits than the threshold
are rejected (events tied at the threshold are kept, so at most that many are
rejected).

Consolidation.  The sequence packs the resulting track data for the
algorithms that follow.  Reading: per accepted track, the coordinates of its
hits laid out in track order (x, y, z arrays aligned with the track-hit
list), and a straight-line state from an unweighted least-squares fit of x
and y against z over the track's hits: the mean point (x, y, z), the slopes
tx, ty and chi2 per degree of freedom (2n - 4 for n hits).  The fit is written
here in float64 from its definition.
"""

from __future__ import annotations

import numpy as np


def gec_threshold(sizes, fraction: float) -> int:
    """The smallest hit count c >= 1 such that at most floor(fraction * E) of
    the event sizes exceed c (plain search over the candidate values 1 and the
    sizes)."""
    sizes = np.asarray(sizes, dtype=np.int64)
    k = int(np.floor(float(fraction) * sizes.size))
    for c in sorted(set(int(v) for v in sizes if v >= 1) | {1}):
        if int((sizes > c).sum()) <= k:
            return c
    raise AssertionError("the largest size always qualifies")


def gec_keep(sizes, fraction: float) -> np.ndarray:
    """Boolean mask of the events the cut keeps."""
    sizes = np.asarray(sizes, dtype=np.int64)
    return sizes <= gec_threshold(sizes, fraction)


def fit_line(x, y, z):
    """Unweighted least-squares straight line through the points, from its
    definition in float64: returns (xm, ym, zm, tx, ty, chi2 / (2n - 4))."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    n = x.size
    xm, ym, zm = x.mean(), y.mean(), z.mean()
    dz = z - zm
    szz = float((dz * dz).sum())
    tx = float((dz * (x - xm)).sum()) / szz
    ty = float((dz * (y - ym)).sum()) / szz
    rx = x - (xm + tx * dz)
    ry = y - (ym + ty * dz)
    chi2 = float((rx * rx).sum() + (ry * ry).sum())
    return xm, ym, zm, tx, ty, chi2 / (2 * n - 4)


def consolidate(batch, eto, tho, th):
    """(px, py, pz, states): the coordinates of every track hit in track order
    (float32, copies of the inputs) and one float64 state row per track."""
    eto = np.asarray(eto)
    tho = np.asarray(tho)
    th = np.asarray(th)
    E = eto.size - 1
    A = int(tho[-1]) if tho.size else 0
    px = np.empty(A, np.float32)
    py = np.empty(A, np.float32)
    pz = np.empty(A, np.float32)
    states = np.empty((int(eto[-1]), 6), np.float64)
    for e in range(E):
        base = int(batch.event_offsets[e])
        for t in range(int(eto[e]), int(eto[e + 1])):
            lo, hi = int(tho[t]), int(tho[t + 1])
            ids = base + th[lo:hi].astype(np.int64)
            px[lo:hi] = batch.x[ids]
            py[lo:hi] = batch.y[ids]
            pz[lo:hi] = batch.z[ids]
            states[t] = fit_line(px[lo:hi], py[lo:hi], pz[lo:hi])
    return px, py, pz, states
