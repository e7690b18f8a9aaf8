"""Track-reconstruction quality indicators (paper, Section 1, eqs. (1)-(5)).

A reconstructed track is associated with a generated particle when at least
70 % of its hits come from that particle; otherwise it is a fake (ghost).
Tracks associated with a particle that another track is already associated
with are clones.  A particle is reconstructible here when it left hits on at
least three consecutive modules.

* efficiency     = reconstructed and reconstructible / reconstructible   (1)
* fake fraction  = fake tracks / reconstructed tracks                     (2)
* clone fraction = clone tracks / reconstructed tracks                    (3)
* hit purity     = matched track hits from the particle / track hits      (4)
* hit efficiency = matched track hits from the particle / particle hits   (5)

(4) and (5) are pooled over associated tracks.
"""

from __future__ import annotations

from collections import Counter

import numpy as np


def _reconstructible(truth: np.ndarray, module_of_hit: np.ndarray, min_consecutive: int = 3) -> set:
    out = set()
    parts = np.unique(truth[truth >= 0])
    for p in parts:
        mods = np.unique(module_of_hit[truth == p])
        run = best = 1
        for a, b in zip(mods[:-1], mods[1:]):
            run = run + 1 if b == a + 1 else 1
            best = max(best, run)
        if mods.size and best >= min_consecutive:
            out.add(int(p))
    return out


def evaluate(batch, event_track_offsets, track_hit_offsets, track_hits, match_fraction: float = 0.7) -> dict:
    """The five indicators, summed over all events of ``batch``."""
    M = batch.n_modules
    n_reco = n_fake = n_clone = 0
    n_recible = n_found = 0
    hits_in_particle = hits_total = 0
    particle_hits_total = 0
    for e in range(batch.n_events):
        lo, hi = int(batch.event_offsets[e]), int(batch.event_offsets[e + 1])
        truth = batch.truth[lo:hi]
        mo = batch.module_offsets[e * M:(e + 1) * M + 1] - lo
        module_of_hit = np.repeat(np.arange(M), np.diff(mo))
        recible = _reconstructible(truth, module_of_hit)
        n_recible += len(recible)
        counts = Counter(truth[truth >= 0].tolist())
        matched = set()
        for t in range(int(event_track_offsets[e]), int(event_track_offsets[e + 1])):
            ids = track_hits[track_hit_offsets[t]:track_hit_offsets[t + 1]]
            n_reco += 1
            labels = truth[ids]
            c = Counter(labels.tolist())
            part, k = c.most_common(1)[0]
            if part < 0 or k < match_fraction * len(ids):
                n_fake += 1
                continue
            if part in matched:
                n_clone += 1
            matched.add(part)
            hits_in_particle += k
            hits_total += len(ids)
            particle_hits_total += counts[part]
        n_found += len(matched & recible)
    safe = lambda a, b: (a / b) if b else float("nan")
    return dict(
        efficiency=safe(n_found, n_recible),
        fake_fraction=safe(n_fake, n_reco),
        clone_fraction=safe(n_clone, n_reco),
        hit_purity=safe(hits_in_particle, hits_total),
        hit_efficiency=safe(hits_in_particle, particle_hits_total),
        n_tracks=n_reco,
        n_reconstructible=n_recible,
    )
