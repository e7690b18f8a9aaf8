"""The oracle's structure entry point (sbt_reconstruct_cpu, declared in
oracle/sbt_oracle_abi.h): its structures have the layouts of the GPU
library's header, a C caller can hand it the library's own structures, it
gives the positional entry's tracks, and it reports events that cannot be
reconstructed with the status bits the library's header defines."""

import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_2207_03936_amd import sbt, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_DIR = os.path.join(ROOT, "oracle")

LAYOUTS = r"""
#include <stddef.h>
#include <stdio.h>
#include "sbt.h"
#include "sbt_oracle_abi.h"

#define SAME(A, B, f) printf("%s %d %d\n", #f, (int)offsetof(A, f), (int)offsetof(B, f))
int main(void)
{
    printf("size_params %d %d\n", (int)sizeof(sbt_params), (int)sizeof(orc_abi_params));
    printf("size_hits %d %d\n", (int)sizeof(sbt_hits), (int)sizeof(orc_abi_hits));
    printf("size_tracks %d %d\n", (int)sizeof(sbt_tracks), (int)sizeof(orc_abi_tracks));
    SAME(sbt_params, orc_abi_params, n_modules);
    SAME(sbt_params, orc_abi_params, module_z);
    SAME(sbt_params, orc_abi_params, reverse);
    SAME(sbt_params, orc_abi_params, max_doublet_candidates);
    SAME(sbt_params, orc_abi_params, phi_window_seeding);
    SAME(sbt_params, orc_abi_params, phi_window_forwarding);
    SAME(sbt_params, orc_abi_params, max_scatter_seeding);
    SAME(sbt_params, orc_abi_params, max_scatter_forwarding);
    SAME(sbt_params, orc_abi_params, max_tracklet_chi2);
    SAME(sbt_params, orc_abi_params, max_consecutive_misses);
    SAME(sbt_params, orc_abi_params, max_event_hits);
    SAME(sbt_hits, orc_abi_hits, n_events);
    SAME(sbt_hits, orc_abi_hits, n_hits);
    SAME(sbt_hits, orc_abi_hits, event_offsets);
    SAME(sbt_hits, orc_abi_hits, module_offsets);
    SAME(sbt_hits, orc_abi_hits, x);
    SAME(sbt_hits, orc_abi_hits, y);
    SAME(sbt_hits, orc_abi_hits, z);
    SAME(sbt_tracks, orc_abi_tracks, event_track_offsets);
    SAME(sbt_tracks, orc_abi_tracks, track_hit_offsets);
    SAME(sbt_tracks, orc_abi_tracks, track_hits);
    SAME(sbt_tracks, orc_abi_tracks, event_status);
    printf("modules %d %d\n", SBT_MAX_MODULES, (int)(sizeof(((orc_abi_params *)0)->module_z) / sizeof(float)));
    printf("too_large %d %d\n", (int)SBT_EV_TOO_LARGE, ORC_EV_TOO_LARGE);
    printf("bad_offsets %d %d\n", (int)SBT_EV_BAD_OFFSETS, ORC_EV_BAD_OFFSETS);
    printf("cut %d %d\n", (int)SBT_EV_CUT, ORC_EV_CUT);
    return 0;
}
"""

# a C caller holding the library's structures (host pointers) calls the oracle
CALLER = r"""
#include <stdio.h>
#include <string.h>
#include "sbt.h"

int sbt_reconstruct_cpu(const sbt_params *, const sbt_hits *, sbt_tracks *);

int main(void)
{
    /* two events, 3 modules: a straight line through three modules, then an empty event */
    float x[3] = {10.0f, 10.5f, 11.0f}, y[3] = {1.0f, 1.05f, 1.1f}, z[3] = {0.0f, 40.0f, 80.0f};
    int32_t eo[3] = {0, 3, 3}, mo[7] = {0, 1, 2, 3, 3, 3, 3};
    sbt_params p;
    memset(&p, 0, sizeof p);
    p.n_modules = 3;
    p.module_z[0] = 0.0f; p.module_z[1] = 40.0f; p.module_z[2] = 80.0f;
    p.reverse = 0;
    p.max_doublet_candidates = 4;
    p.phi_window_seeding = 416;
    p.phi_window_forwarding = 416;
    p.max_scatter_seeding = 0.04f;
    p.max_scatter_forwarding = 0.04f;
    p.max_tracklet_chi2 = 0.002f;
    p.max_consecutive_misses = 1;
    sbt_hits h = {2, 3, eo, mo, x, y, z};
    int32_t eto[3], tho[2], th[3], st[2];
    sbt_tracks t = {eto, tho, th, st};
    int rc = sbt_reconstruct_cpu(&p, &h, &t);
    printf("%d %d %d %d %d %d %d %d\n", rc, eto[1], eto[2], tho[1], th[0], th[1], th[2], st[0] | st[1]);
    return rc;
}
"""


def _compile(tmp_path, name, text, link_oracle):
    src = tmp_path / f"{name}.c"
    src.write_text(text)
    exe = tmp_path / name
    cmd = ["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), "-I", ORACLE_DIR, str(src)]
    if link_oracle:
        oracle.lib()
        cmd += ["-L", ORACLE_DIR, "-loracle", "-Wl,-rpath," + ORACLE_DIR]
    subprocess.run(cmd + ["-o", str(exe)], check=True)
    return exe


def test_structures_have_the_library_layouts(tmp_path):
    out = subprocess.run([str(_compile(tmp_path, "layouts", LAYOUTS, False))], capture_output=True, text=True,
                         check=True).stdout
    rows = [line.split() for line in out.strip().splitlines()]
    assert len(rows) == 29
    for name, a, b in rows:
        assert a == b, name


def test_binding_structures_match_the_oracle_structures():
    """The Python binding's structures and the oracle's ctypes structures
    agree field by field (each side declared on its own)."""
    for lib_t, orc_t in ((sbt.SbtParams, oracle.OrcAbiParams), (sbt.SbtHits, oracle.OrcAbiHits),
                         (sbt.SbtTracks, oracle.OrcAbiTracks)):
        assert ctypes.sizeof(lib_t) == ctypes.sizeof(orc_t)
        assert [f for f, _ in lib_t._fields_] == [f for f, _ in orc_t._fields_]
        for f, _ in lib_t._fields_:
            assert getattr(lib_t, f).offset == getattr(orc_t, f).offset, f


def test_c_caller_passes_the_library_structures(tmp_path):
    exe = _compile(tmp_path, "caller", CALLER, True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stdout + out.stderr
    # one tracklet of the three hits in traversal order, no track in the empty event, no status
    assert out.stdout.split() == ["0", "1", "1", "3", "0", "1", "2", "0"]


@pytest.mark.parametrize("config,n", [("mu7.6", 12), ("mu1-25", 6), ("tiny", 30), ("pairs7.6", 8)])
def test_structure_entry_equals_positional_entry(config, n):
    b = synth.make_batch(config, n)
    want = oracle.reconstruct(b)
    got = oracle.reconstruct_abi(b)
    for a, c in zip(want, got[:3]):
        assert np.array_equal(a, c)
    assert not got[3].any()


def edge_batch():
    """Five events: ordinary, one with decreasing module offsets, ordinary,
    one of 65,536 hits, ordinary (tiny recipe)."""
    tiny = synth.make_batch("tiny", 3, first=4)
    evs = [synth._slice(tiny, i) for i in range(3)]
    big = dict(x=np.full(65536, 20.0, np.float32), y=np.full(65536, 3.0, np.float32),
               z=np.full(65536, synth.PLANE_Z[5], np.float32),
               module_counts=np.eye(26, dtype=np.int64)[5] * 65536, truth=np.zeros(65536, np.int32))
    b = synth.concat([evs[0], evs[1], evs[2], big, evs[0]], synth.PLANE_Z)
    mo = b.module_offsets.copy()
    M = b.n_modules
    mo[M + 5] = mo[M + 7] + 1          # event 1: module offsets decrease
    return synth.Batch(b.x, b.y, b.z, b.event_offsets, mo, b.module_z, b.truth), [evs[0], evs[2], evs[0]]


def test_structure_entry_reports_events_it_cannot_reconstruct():
    b, good = edge_batch()
    eto, tho, th, st = oracle.reconstruct_abi(b)
    assert list(st) == [0, oracle_status("bad"), 0, oracle_status("large"), 0]
    assert eto[2] == eto[1] and eto[4] == eto[3]
    want = oracle.reconstruct(synth.concat(good, synth.PLANE_Z))
    keep = [0, 2, 4]
    mine = [[tuple(th[tho[t]:tho[t + 1]]) for t in range(eto[e], eto[e + 1])] for e in keep]
    ref = [[tuple(want[2][want[1][t]:want[1][t + 1]]) for t in range(want[0][e], want[0][e + 1])] for e in range(3)]
    assert mine == ref
    # the global event cut: events above 600 hits get the cut bit and no tracks
    c = synth.make_batch("mu1-25", 8, first=3)
    sizes = np.diff(c.event_offsets)
    eto, tho, th, st = oracle.reconstruct_abi(c, max_event_hits=600)
    assert list(st) == [oracle_status("cut") if s > 600 else 0 for s in sizes]
    assert all(eto[e + 1] == eto[e] for e in range(c.n_events) if sizes[e] > 600)


def oracle_status(kind):
    return {"large": 1, "bad": 2, "cut": 8}[kind]


@pytest.mark.gpu
def test_gpu_statuses_equal_the_oracle_structure_entry():
    """The GPU's per-event statuses and tracks equal the oracle structure
    entry's on the edge batch and under the global event cut, for the plain
    and the batched form."""
    b, _ = edge_batch()
    c = synth.make_batch("mu1-25", 8, first=3)
    for batch, kw in ((b, {}), (c, dict(max_event_hits=600))):
        want = oracle.reconstruct_abi(batch, **kw)
        p = sbt.make_params(batch.module_z, **kw)
        plain = sbt.sbt_reconstruct(p, sbt.DeviceBatch(batch)).to_host()
        ctx = sbt.Context(p, batch.n_events, batch.n_hits)
        batched = ctx.reconstruct(sbt.DeviceBatch(batch)).to_host()
        ctx.close()
        for name, got in (("plain", plain), ("batched", batched)):
            assert list(got[3]) == list(want[3]), name
            for a, w in zip(got[:3], want[:3]):
                assert np.array_equal(a, w), name
