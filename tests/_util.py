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


def jet_event(rng, n_tracks, phi0, sigma_phi=0.004, efficiency=0.95, dup_fraction=0.02):
    """An event of the 26-plane geometry whose tracks all leave one vertex in
    a narrow cone: phi ~ N(phi0, sigma_phi), eta ~ U(2, 5), so that hundreds
    of hits of a module share one phi window (long window scans, crowded
    pendulum lists, many competing claims).  A fraction of the hits is
    duplicated exactly (ties on every score), and noise is spread over the
    same cone.  Returns the per-event dict that synth.concat packs."""
    zp = synth.PLANE_Z
    zv = rng.normal(0.0, 20.0)
    eta = rng.uniform(2.0, 5.0, n_tracks)
    phi = rng.normal(phi0, sigma_phi, n_tracks)
    theta = 2.0 * np.arctan(np.exp(-eta))
    tx, ty = np.tan(theta) * np.cos(phi), np.tan(theta) * np.sin(phi)
    dz = zp[None, :] - zv
    px = tx[:, None] * dz + rng.normal(0.0, synth.SMEAR_MM, (n_tracks, zp.size))
    py = ty[:, None] * dz + rng.normal(0.0, synth.SMEAR_MM, (n_tracks, zp.size))
    r = np.hypot(px, py)
    keep = (dz > 0) & (r >= synth.R_MIN) & (r <= synth.R_MAX) & (rng.random(px.shape) < efficiency)
    tid, plane = np.nonzero(keep)
    hx, hy = px[tid, plane], py[tid, plane]
    n_noise = max(1, tid.size // 50)
    nplane = rng.integers(0, zp.size, n_noise)
    nr = rng.uniform(synth.R_MIN, synth.R_MAX, n_noise)
    nphi = rng.normal(phi0, 3 * sigma_phi, n_noise)
    truth = np.concatenate([tid, np.full(n_noise, -1)])
    plane = np.concatenate([plane, nplane])
    hx = np.concatenate([hx, nr * np.cos(nphi)])
    hy = np.concatenate([hy, nr * np.sin(nphi)])
    dup = rng.random(plane.size) < dup_fraction
    truth = np.concatenate([truth, np.full(int(dup.sum()), -1)])   # a copy belongs to no particle
    plane = np.concatenate([plane, plane[dup]])
    hx = np.concatenate([hx, hx[dup]])
    hy = np.concatenate([hy, hy[dup]])
    order = np.lexsort((rng.random(plane.size), plane))
    plane = plane[order]
    return dict(x=hx[order].astype(np.float32), y=hy[order].astype(np.float32),
                z=zp[plane].astype(np.float32),
                module_counts=np.bincount(plane, minlength=zp.size).astype(np.int64),
                truth=truth[order].astype(np.int32))
