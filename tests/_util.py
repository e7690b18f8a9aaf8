"""Helpers shared by the test modules (no reconstruction arithmetic here)."""

import numpy as np

from paper_2207_03936_amd import synth


def tracks_per_event(eto, tho, th):
    """CSR output -> list (per event) of lists of hit-id tuples."""
    out = []
    for e in range(len(eto) - 1):
        ev = []
        for t in range(int(eto[e]), int(eto[e + 1])):
            ev.append(tuple(int(h) for h in th[tho[t]:tho[t + 1]]))
        out.append(ev)
    return out


def tiny_random_event(rng, M=None, max_per_module=8, jitter_z=False, duplicates=True):
    """A small event crowded into a narrow phi sector so that windows, pendulum
    candidates and competing claims all occur.  Returns (x, y, z, mo, module_z)
    with hits grouped by module."""
    M = int(rng.integers(4, 9)) if M is None else M
    module_z = (-100.0 + 40.0 * np.arange(M)).astype(np.float32)
    n_tracks = int(rng.integers(1, 5))
    per_mod = [[] for _ in range(M)]
    base_phi = rng.uniform(-np.pi, np.pi)
    for _ in range(n_tracks):
        phi = base_phi + rng.normal(0, 0.01)
        slope = rng.uniform(0.02, 0.06)
        z0 = rng.uniform(-300, -150)
        for k in range(M):
            if rng.random() < 0.85:
                r = slope * (module_z[k] - z0)
                per_mod[k].append((r * np.cos(phi) + rng.normal(0, 0.03),
                                   r * np.sin(phi) + rng.normal(0, 0.03)))
    for k in range(M):
        for _ in range(int(rng.integers(0, 4))):
            r = rng.uniform(5, 20)
            phi = base_phi + rng.normal(0, 0.02)
            per_mod[k].append((r * np.cos(phi), r * np.sin(phi)))
        if duplicates and per_mod[k] and rng.random() < 0.3:
            per_mod[k].append(per_mod[k][int(rng.integers(0, len(per_mod[k])))])
        rng.shuffle(per_mod[k])
        per_mod[k] = per_mod[k][:max_per_module]
    xs, ys, zs, counts = [], [], [], []
    for k in range(M):
        counts.append(len(per_mod[k]))
        for (hx, hy) in per_mod[k]:
            xs.append(hx)
            ys.append(hy)
            zs.append(module_z[k] + (rng.uniform(-0.5, 0.5) if jitter_z else 0.0))
    mo = np.zeros(M + 1, np.int32)
    mo[1:] = np.cumsum(counts)
    return (np.array(xs, np.float32), np.array(ys, np.float32), np.array(zs, np.float32),
            mo, module_z)


def event_batch(x, y, z, mo, module_z):
    """One-event Batch from raw arrays."""
    return synth.concat([dict(x=np.asarray(x, np.float32), y=np.asarray(y, np.float32),
                              z=np.asarray(z, np.float32), module_counts=np.diff(mo).astype(np.int64),
                              truth=np.full(len(x), -1, np.int32))], module_z)


def rounded_to_f16(batch):
    """The batch with its coordinates rounded to binary16 (numpy, IEEE round
    to nearest even) and widened back to binary32: the values the
    half-precision input form carries."""
    import dataclasses
    r = lambda a: np.asarray(a, np.float32).astype(np.float16).astype(np.float32)
    return dataclasses.replace(batch, x=r(batch.x), y=r(batch.y), z=r(batch.z))
