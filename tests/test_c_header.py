"""The C ABI from plain C: a program compiled with gcc against include/sbt.h
and linked to libsbt.so calls the host-side entry points (no GPU needed)."""

import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_2207_03936_amd")

PROGRAM = r"""
#include <stdio.h>
#include <string.h>
#include "sbt.h"

int main(void)
{
    sbt_params p;
    memset(&p, 0, sizeof p);
    p.n_modules = 26;
    for (int k = 0; k < 26; ++k) p.module_z[k] = -275.0f + 40.0f * (float)k;
    p.reverse = 1;
    p.max_doublet_candidates = 4;
    p.phi_window_seeding = 416;
    p.phi_window_forwarding = 416;
    p.max_scatter_seeding = 0.04f;
    p.max_scatter_forwarding = 0.04f;
    p.max_tracklet_chi2 = 0.002f;
    p.max_consecutive_misses = 1;
    p.max_event_hits = 0;
    if (sbt_params_validate(&p) != SBT_OK) return 1;
    p.max_event_hits = -1;
    if (sbt_params_validate(&p) != SBT_ERR_INVALID_ARG) return 2;
    const int32_t eo[6] = {0, 10, 30, 60, 100, 150};
    int32_t cut = 0;
    if (sbt_gec_threshold(5, eo, 0.2, &cut) != SBT_OK || cut != 40) return 3;
    size_t bytes = 0;
    if (sbt_workspace_size(5, 150, &bytes) != SBT_OK || bytes == 0) return 4;
    printf("%s|%d|%zu\n", sbt_error_string(SBT_ERR_WORKSPACE), cut, bytes);
    return 0;
}
"""


def test_c_program_links_and_runs(tmp_path):
    lib = os.path.join(LIBDIR, "libsbt.so")
    if not os.path.exists(lib):
        pytest.skip("libsbt.so is not built")
    src = tmp_path / "abi.c"
    src.write_text(PROGRAM)
    exe = tmp_path / "abi"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src),
                    "-L", LIBDIR, "-lsbt", "-Wl,-rpath," + LIBDIR, "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stdout + out.stderr
    msg, cut, nbytes = out.stdout.strip().split("|")
    assert msg == "workspace or context too small" and cut == "40" and int(nbytes) > 0


LAYOUT = r"""
#include <stddef.h>
#include <stdio.h>
#include "sbt.h"

#define FIELD(T, f) printf(#T "." #f " %zu\n", offsetof(T, f))
int main(void)
{
    printf("sbt_params %zu\nsbt_tuning %zu\nsbt_hits %zu\nsbt_hits_f16 %zu\nsbt_tracks %zu\n",
           sizeof(sbt_params), sizeof(sbt_tuning), sizeof(sbt_hits), sizeof(sbt_hits_f16), sizeof(sbt_tracks));
    printf("sbt_server_config %zu\nsbt_server_result %zu\n", sizeof(sbt_server_config), sizeof(sbt_server_result));
    FIELD(sbt_server_config, coords_f16);
    FIELD(sbt_server_result, t_done_us);
    FIELD(sbt_params, max_event_hits);
    return 0;
}
"""


def test_struct_layouts_match_the_binding(tmp_path):
    """The ctypes structures of the Python binding have the sizes and field
    offsets that a C compiler gives the header's structures."""
    import ctypes
    from paper_2207_03936_amd import sbt
    src = tmp_path / "layout.c"
    src.write_text(LAYOUT)
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src),
                    "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60, check=True).stdout
    got = dict(line.rsplit(" ", 1) for line in out.strip().splitlines())
    want = {
        "sbt_params": ctypes.sizeof(sbt.SbtParams), "sbt_tuning": ctypes.sizeof(sbt.SbtTuning),
        "sbt_hits": ctypes.sizeof(sbt.SbtHits), "sbt_hits_f16": ctypes.sizeof(sbt.SbtHitsF16),
        "sbt_tracks": ctypes.sizeof(sbt.SbtTracks), "sbt_server_config": ctypes.sizeof(sbt.SbtServerConfig),
        "sbt_server_result": ctypes.sizeof(sbt.SbtServerResult),
        "sbt_server_config.coords_f16": sbt.SbtServerConfig.coords_f16.offset,
        "sbt_server_result.t_done_us": sbt.SbtServerResult.t_done_us.offset,
        "sbt_params.max_event_hits": sbt.SbtParams.max_event_hits.offset,
    }
    assert {k: int(v) for k, v in got.items()} == want
