"""Seeded synthetic vertex-detector events.

This module only draws inputs: straight particle trajectories from primary
vertices, their intersections with a stack of detector planes, per-plane hit
inefficiency, Gaussian position smearing and uniform noise hits.  It holds none
of the reconstruction method's arithmetic, so both the CPU oracle and the HIP
path can consume what it produces.

The detector is the one the paper's method is stated for (Section 1 and
Section 3): planes perpendicular to the beam (z) axis, particles travelling in
straight lines because the detector sits outside the magnet, hits carrying
(x, y, z) and the index of the plane ("module") they were measured on.

Geometry used for every workload: 26 planes at z = -275 + 40 k mm
(k = 0..25) with an active annulus 5.1 mm <= r <= 42 mm.

Event recipes (``CONFIGS``):

* ``tiny``   - one primary vertex, exactly 40 tracks, 99 % hit efficiency,
  1 % noise (about 500 hits).
* ``mu7.6``  - Poisson(7.6) primary vertices, Poisson(40) tracks each
  (about 3,000 hits per event).
* ``mu1-25`` - per-event pileup mu ~ U{1..25} vertices, Poisson(40) tracks
  each (200 to 10,000 hits per event).
* ``mu30``   - Poisson(30) vertices, 97 % hit efficiency, 5 % noise, 20 % of
  tracks get a N(0, 2 mrad) kink in both slopes at one crossed plane
  (about 12,000 hits per event).
* ``bw7.6``  - the ``mu7.6`` mixture with a quarter of the tracks flying
  backwards (towards -z, through the planes upstream of their vertex).
* ``pairs7.6`` - the ``mu7.6`` mixture on module pairs: each traversal plane is
  two half-planes, x < 0 at z - 6 mm and x >= 0 at z + 6 mm, so the hits of
  one module carry two z values, neither equal to the module's nominal z (the
  method treats a pair as one module, Section 3).

Hits of an event are grouped by plane index ascending and shuffled within a
plane; a hit's event-local ID is its position in the event.  The random stream
of event ``i`` of a recipe with seed ``s`` is ``default_rng([s, i])``, so any
event can be regenerated on its own.
"""

from __future__ import annotations

import dataclasses
import os
from typing import Optional

import numpy as np

N_PLANES = 26
PLANE_Z = (-275.0 + 40.0 * np.arange(N_PLANES)).astype(np.float64)
R_MIN = 5.1
R_MAX = 42.0
SMEAR_MM = 0.012


@dataclasses.dataclass(frozen=True)
class Recipe:
    name: str
    seed: int
    n_events: int
    pv: str                 # "fixed1", "poisson", "uniform"
    pv_mean: float = 0.0
    pv_max: int = 0         # for "uniform": mu ~ U{1..pv_max}
    tracks_fixed: int = 0   # > 0: exactly this many tracks per vertex
    tracks_mean: float = 40.0
    efficiency: float = 0.99
    noise_fraction: float = 0.01
    kink_fraction: float = 0.0
    kink_sigma: float = 0.002
    half_dz: float = 0.0    # > 0: module pairs, half-planes at z -/+ half_dz by the sign of x
    backward_fraction: float = 0.0   # tracks flying towards -z


CONFIGS = {
    "tiny": Recipe("tiny", 1, 1, "fixed1", tracks_fixed=40),
    "mu7.6": Recipe("mu7.6", 2, 1000, "poisson", pv_mean=7.6),
    "mu1-25": Recipe("mu1-25", 3, 10000, "uniform", pv_max=25),
    "mu30": Recipe("mu30", 4, 2000, "poisson", pv_mean=30.0,
                   efficiency=0.97, noise_fraction=0.05, kink_fraction=0.2),
    "serve": Recipe("serve", 5, 0, "uniform", pv_max=25),
    "pairs7.6": Recipe("pairs7.6", 6, 1000, "poisson", pv_mean=7.6, half_dz=6.0),
    "bw7.6": Recipe("bw7.6", 7, 1000, "poisson", pv_mean=7.6, backward_fraction=0.25),
}


@dataclasses.dataclass
class Batch:
    """Flat structure-of-arrays hits of several events.

    ``module_offsets`` holds ``n_events * n_modules + 1`` absolute offsets:
    module ``k`` of event ``e`` is the hit range
    ``[module_offsets[e*M + k], module_offsets[e*M + k + 1])``.
    """

    x: np.ndarray            # float32 [H]
    y: np.ndarray            # float32 [H]
    z: np.ndarray            # float32 [H]
    event_offsets: np.ndarray   # int32 [E+1]
    module_offsets: np.ndarray  # int32 [E*M+1]
    module_z: np.ndarray     # float32 [M]
    truth: np.ndarray        # int32 [H]: particle index within its event, -1 noise

    @property
    def n_events(self) -> int:
        return int(self.event_offsets.shape[0] - 1)

    @property
    def n_hits(self) -> int:
        return int(self.event_offsets[-1])

    @property
    def n_modules(self) -> int:
        return int(self.module_z.shape[0])

    def event(self, e: int) -> "Batch":
        """A one-event batch holding a copy of event ``e``."""
        return self.select([e])

    def select(self, events) -> "Batch":
        """A new batch made of the listed events, in the listed order."""
        return concat([_slice(self, int(e)) for e in events], self.module_z)


def _slice(b: Batch, e: int) -> dict:
    M = b.n_modules
    lo, hi = int(b.event_offsets[e]), int(b.event_offsets[e + 1])
    mo = b.module_offsets[e * M:(e + 1) * M + 1].astype(np.int64) - lo
    return dict(x=b.x[lo:hi], y=b.y[lo:hi], z=b.z[lo:hi],
                module_counts=np.diff(mo).astype(np.int64), truth=b.truth[lo:hi])


def concat(events, module_z) -> Batch:
    """Pack per-event dicts (x, y, z, module_counts, truth) into a Batch."""
    module_z = np.asarray(module_z, dtype=np.float32)
    M = module_z.shape[0]
    E = len(events)
    sizes = np.array([ev["x"].shape[0] for ev in events], dtype=np.int64)
    eo = np.zeros(E + 1, dtype=np.int64)
    np.cumsum(sizes, out=eo[1:])
    if eo[-1] > np.iinfo(np.int32).max:
        raise ValueError("batch exceeds 2^31-1 hits")
    counts = (np.concatenate([ev["module_counts"] for ev in events])
              if E else np.zeros(0, dtype=np.int64))
    mo = np.zeros(E * M + 1, dtype=np.int64)
    np.cumsum(counts, out=mo[1:])
    def cat(key, dt):
        if E == 0:
            return np.zeros(0, dtype=dt)
        return np.ascontiguousarray(np.concatenate([ev[key] for ev in events]).astype(dt))
    return Batch(x=cat("x", np.float32), y=cat("y", np.float32), z=cat("z", np.float32),
                 event_offsets=eo.astype(np.int32), module_offsets=mo.astype(np.int32),
                 module_z=module_z.copy(), truth=cat("truth", np.int32))


def _n_vertices(r: Recipe, rng: np.random.Generator) -> int:
    if r.pv == "fixed1":
        return 1
    if r.pv == "poisson":
        return int(rng.poisson(r.pv_mean))
    if r.pv == "uniform":
        return int(rng.integers(1, r.pv_max + 1))
    raise ValueError(r.pv)


def make_event(recipe: Recipe, index: int) -> dict:
    """Draw event ``index`` of ``recipe`` (see the module docstring)."""
    rng = np.random.default_rng([recipe.seed, index])
    n_pv = _n_vertices(recipe, rng)
    if recipe.tracks_fixed > 0:
        per_pv = np.full(n_pv, recipe.tracks_fixed, dtype=np.int64)
    else:
        per_pv = rng.poisson(recipe.tracks_mean, size=n_pv).astype(np.int64)
    pvx = rng.normal(0.0, 0.01, n_pv)
    pvy = rng.normal(0.0, 0.01, n_pv)
    pvz = rng.normal(0.0, 50.0, n_pv)
    T = int(per_pv.sum())
    src = np.repeat(np.arange(n_pv), per_pv)
    xv, yv, zv = pvx[src], pvy[src], pvz[src]
    eta = rng.uniform(2.0, 5.0, T)
    phi = rng.uniform(0.0, 2.0 * np.pi, T)
    theta = 2.0 * np.arctan(np.exp(-eta))
    tx = np.tan(theta) * np.cos(phi)
    ty = np.tan(theta) * np.sin(phi)

    zp = PLANE_Z[None, :]
    if recipe.half_dz > 0.0:
        # the half-plane a track crosses follows the sign of x at the nominal plane
        xn = xv[:, None] + tx[:, None] * (zp - zv[:, None])
        zp = zp + np.where(xn >= 0.0, recipe.half_dz, -recipe.half_dz)
    if recipe.backward_fraction > 0.0:
        # a backward track crosses the planes below its vertex; its transverse
        # offset grows with the distance flown
        assert recipe.kink_fraction == 0.0 and recipe.half_dz == 0.0
        back = rng.random(T) < recipe.backward_fraction
        flown = np.where(back[:, None], zv[:, None] - zp, zp - zv[:, None])
        crossed = flown > 0.0
        px = xv[:, None] + tx[:, None] * flown
        py = yv[:, None] + ty[:, None] * flown
    else:
        crossed = zp > zv[:, None]                           # [T, P]
        px = xv[:, None] + tx[:, None] * (zp - zv[:, None])
        py = yv[:, None] + ty[:, None] * (zp - zv[:, None])

    if recipe.kink_fraction > 0.0 and T > 0:
        kinked = rng.random(T) < recipe.kink_fraction
        n_crossed = crossed.sum(axis=1)
        pick = rng.random(T)
        dtx = rng.normal(0.0, recipe.kink_sigma, T)
        dty = rng.normal(0.0, recipe.kink_sigma, T)
        for t in np.nonzero(kinked & (n_crossed > 0))[0]:
            planes = np.nonzero(crossed[t])[0]
            kp = planes[min(int(pick[t] * planes.size), planes.size - 1)]
            after = np.arange(N_PLANES) > kp
            zt = np.broadcast_to(zp, (T, N_PLANES))[t]
            dz = zt[after] - zt[kp]
            px[t, after] = px[t, kp] + (tx[t] + dtx[t]) * dz
            py[t, after] = py[t, kp] + (ty[t] + dty[t]) * dz

    r = np.hypot(px, py)
    accepted = crossed & (r >= R_MIN) & (r <= R_MAX)
    fired = rng.random((T, N_PLANES)) < recipe.efficiency
    keep = accepted & fired
    sx = px + rng.normal(0.0, SMEAR_MM, (T, N_PLANES))
    sy = py + rng.normal(0.0, SMEAR_MM, (T, N_PLANES))

    tid, plane = np.nonzero(keep)
    hx, hy = sx[tid, plane], sy[tid, plane]
    hz = np.broadcast_to(zp, (T, N_PLANES))[tid, plane]
    n_noise = int(round(recipe.noise_fraction * tid.size))
    nplane = rng.integers(0, N_PLANES, n_noise)
    nr = np.sqrt(rng.uniform(R_MIN * R_MIN, R_MAX * R_MAX, n_noise))
    nphi = rng.uniform(0.0, 2.0 * np.pi, n_noise)
    nx = nr * np.cos(nphi)
    nz = PLANE_Z[nplane]
    if recipe.half_dz > 0.0:
        nz = nz + np.where(nx >= 0.0, recipe.half_dz, -recipe.half_dz)
    all_plane = np.concatenate([plane, nplane])
    all_x = np.concatenate([hx, nx])
    all_y = np.concatenate([hy, nr * np.sin(nphi)])
    all_z = np.concatenate([hz, nz])
    all_truth = np.concatenate([tid, np.full(n_noise, -1)])
    # group by plane ascending, random order within a plane
    order = np.lexsort((rng.random(all_plane.size), all_plane))
    all_plane = all_plane[order]
    counts = np.bincount(all_plane, minlength=N_PLANES).astype(np.int64)
    return dict(x=all_x[order].astype(np.float32),
                y=all_y[order].astype(np.float32),
                z=all_z[order].astype(np.float32),
                module_counts=counts,
                truth=all_truth[order].astype(np.int32))


def _make_range(args):
    name, lo, hi = args
    return [make_event(CONFIGS[name], i) for i in range(lo, hi)]


def make_batch(config: str, n_events: Optional[int] = None, first: int = 0,
               workers: Optional[int] = None) -> Batch:
    """Events ``first .. first+n_events-1`` of a named recipe, packed.

    Large batches are drawn in ``workers`` processes (default: up to 16);
    every event has its own random stream, so the result does not depend on
    the number of workers."""
    recipe = CONFIGS[config]
    n = recipe.n_events if n_events is None else int(n_events)
    if workers is None:
        workers = min(16, os.cpu_count() or 1) if n >= 1000 else 1
    if workers <= 1:
        return concat([make_event(recipe, first + i) for i in range(n)], PLANE_Z)
    import multiprocessing as mp
    step = (n + workers * 4 - 1) // (workers * 4)
    chunks = [(config, first + a, first + min(a + step, n)) for a in range(0, n, step)]
    with mp.get_context("fork").Pool(workers) as pool:
        parts = pool.map(_make_range, chunks)
    return concat([ev for part in parts for ev in part], PLANE_Z)
