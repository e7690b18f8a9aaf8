"""Exhaustive-search formulation of Search by triplet for tiny events.

An independent, deliberately naive restatement of the method (paper,
Section 3) used to pin the C oracle's search mechanics:

* windows are tested by circular distance on the 16-bit circle (no binary
  search, no wrap-around walk);
* doublet partners come from an explicit ordered enumeration of the pendulum
  offsets 0, -1, +1, -2, +2, ...;
* every triplet and every follow-up hit is enumerated and the minimum is taken
  with Python tuple ordering;
* conflicting claims are resolved by listing, per hit, every claimant's
  (score, key) tuple (no 64-bit packing of float bits).

Arithmetic is binary32 through numpy float32 scalars, in the paper's order.
phi16 and the tracklet chi2 come from the oracle's exported functions, which
are pinned separately against float64 references.
"""

from __future__ import annotations

import numpy as np

import oracle

F = np.float32
FREE = None
# times the following search met a flagged hit in the module it searches
# (never, by the step order: a module's hits are flagged only when that
# module is resolved, after its search)
FLAGGED_FOLLOW_CANDIDATES = [0]


def _circ(a, b):
    d = (int(a) - int(b)) % 65536
    return min(d, 65536 - d)


def reconstruct_event(x, y, z, mo, module_z, *, reverse=1, K=4, Ws=416, Wf=416,
                      Ss=0.04, Sf=0.04, X=0.002, misses=1):
    x = np.asarray(x, np.float32)
    y = np.asarray(y, np.float32)
    z = np.asarray(z, np.float32)
    module_z = np.asarray(module_z, np.float32)
    M = len(mo) - 1
    N = int(mo[-1])
    Ss, Sf, X = F(Ss), F(Sf), F(X)
    q = oracle.phi16(x, y) if N else np.zeros(0, np.uint16)
    kmod = (lambda t: M - 1 - t) if reverse else (lambda t: t)
    members = [list(range(int(mo[k]), int(mo[k + 1]))) for k in range(M)]
    owner = [FREE] * N
    forming = []   # dicts: hits, last, key, final

    def phi_of(px, py):
        return int(oracle.phi16(np.array([px], np.float32), np.array([py], np.float32))[0])

    def seeding(t):
        A, B, C = kmod(t - 2), kmod(t - 1), kmod(t)
        Zc = module_z[C]
        sortedA = sorted(members[A], key=lambda h: (int(q[h]), h))
        n = len(sortedA)
        new = []
        for h1 in members[B]:
            if owner[h1] is not FREE or n == 0:
                continue
            s0 = next((i for i, h in enumerate(sortedA) if int(q[h]) >= int(q[h1])), 0)
            offsets = sorted(range(-(n // 2), n - n // 2), key=lambda o: (abs(o), o > 0))
            cands = [sortedA[(s0 + o) % n] for o in offsets if owner[sortedA[(s0 + o) % n]] is FREE][:K]
            x1, y1, z1 = x[h1], y[h1], z[h1]
            options = []
            for h0 in cands:
                d01 = F(z1 - z[h0])
                tx = F(F(x1 - x[h0]) / d01)
                ty = F(F(y1 - y[h0]) / d01)
                dzc = F(Zc - z1)
                qe = phi_of(F(x1 + F(tx * dzc)), F(y1 + F(ty * dzc)))
                for h2 in members[C]:
                    if owner[h2] is not FREE or _circ(q[h2], qe) > Ws:
                        continue
                    dz = F(z[h2] - z1)
                    dx = F(F(x1 + F(tx * dz)) - x[h2])
                    dy = F(F(y1 + F(ty * dz)) - y[h2])
                    sc = F(F(dx * dx) + F(dy * dy))
                    if sc < Ss:
                        options.append((sc, h0, h2))
            if options:
                sc, h0, h2 = min(options)
                new.append(dict(hits=[h0, h1, h2], last=t, key=h1, final=False))
        forming.extend(new)

    def following(t):
        C = kmod(t)
        Zc = module_z[C]
        bids = {}
        for i, f in enumerate(forming):
            if f["final"] or t - f["last"] > misses + 1:
                continue
            if any(owner[h] is not FREE and owner[h] != f["key"] for h in f["hits"]):
                continue
            ha, hb = f["hits"][-2], f["hits"][-1]
            dab = F(z[hb] - z[ha])
            tx = F(F(x[hb] - x[ha]) / dab)
            ty = F(F(y[hb] - y[ha]) / dab)
            dzc = F(Zc - z[hb])
            qe = phi_of(F(x[hb] + F(tx * dzc)), F(y[hb] + F(ty * dzc)))
            options = []
            for h in members[C]:
                if owner[h] is not FREE:
                    FLAGGED_FOLLOW_CANDIDATES[0] += 1
                    continue
                if _circ(q[h], qe) > Wf:
                    continue
                dz = F(z[h] - z[hb])
                dx = F(F(x[hb] + F(tx * dz)) - x[h])
                dy = F(F(y[hb] + F(ty * dz)) - y[h])
                sc = F(F(dx * dx) + F(dy * dy))
                if sc < Sf:
                    options.append((sc, h))
            if options:
                bids[i] = min(options)
        claimants = {}
        claim_sets = {}
        for i, (sc, h) in bids.items():
            f = forming[i]
            cs = {h} | (set(f["hits"]) if len(f["hits"]) == 3 else set())
            claim_sets[i] = cs
            for hh in cs:
                claimants.setdefault(hh, []).append((sc, f["key"]))
        winners = [i for i in bids
                   if all(min(claimants[hh]) == (bids[i][0], forming[i]["key"]) for hh in claim_sets[i])]
        for i in winners:
            f = forming[i]
            for hh in claim_sets[i]:
                owner[hh] = f["key"]
            f["hits"].append(bids[i][1])
            f["last"] = t
        for f in forming:
            if not f["final"] and t - f["last"] >= misses + 1:
                f["final"] = True

    if N > 0:
        seeding(2)
        for t in range(3, M):
            following(t)
            seeding(t)
    accepted = [f for f in forming if len(f["hits"]) >= 4]
    cands = []
    for f in forming:
        if len(f["hits"]) != 3:
            continue
        hs = f["hits"]
        c2 = F(oracle.tracklet_chi2(x[hs], y[hs], z[hs]))
        if c2 < X and all(owner[h] is FREE for h in hs):
            cands.append((c2, f))
    claimants = {}
    for c2, f in cands:
        for h in f["hits"]:
            claimants.setdefault(h, []).append((c2, f["key"]))
    for c2, f in cands:
        if all(min(claimants[h]) == (c2, f["key"]) for h in f["hits"]):
            accepted.append(f)
    accepted.sort(key=lambda f: f["key"])
    return [list(map(int, f["hits"])) for f in accepted]
