/* Drives the GPU entry points of libsbt.so from plain C (no C++, no Python):
 * reads a batch written by tests/test_gpu_c_abi.py, reconstructs it with the
 * plain form, the batched form (a capture and a replay of its graph on a
 * stream of the program's own) and the form that allocates nothing, and
 * writes each result for the test to compare with the oracle.
 *
 *   c_abi_gpu_driver <batch.bin> <tracks.bin>
 *
 * batch.bin (little endian): int32 n_modules, n_events, n_hits; float
 * module_z[n_modules]; int32 reverse, max_doublet_candidates,
 * phi_window_seeding, phi_window_forwarding; float max_scatter_seeding,
 * max_scatter_forwarding, max_tracklet_chi2; int32 max_consecutive_misses,
 * max_event_hits; int32 event_offsets[n_events+1], module_offsets[n_events *
 * n_modules + 1]; float x[n_hits], y[n_hits], z[n_hits].
 * tracks.bin: per form, event_track_offsets[n_events+1],
 * track_hit_offsets[T+1], track_hits[track_hit_offsets[T]] and
 * event_status[n_events] (int32, T = event_track_offsets[n_events]).     */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "sbt.h"

#define CHECK(expr, code)                                                      \
    do {                                                                       \
        if (!(expr)) {                                                         \
            fprintf(stderr, "failed: %s (line %d)\n", #expr, __LINE__);        \
            return code;                                                       \
        }                                                                      \
    } while (0)

static int read_all(FILE *f, void *p, size_t n) { return fread(p, 1, n, f) == n; }

static void *dev_copy(const void *h, size_t n)
{
    void *d = NULL;
    if (hipMalloc(&d, n ? n : 4) != hipSuccess) return NULL;
    if (n && hipMemcpy(d, h, n, hipMemcpyHostToDevice) != hipSuccess) return NULL;
    return d;
}

/* appends one form's result, read back from the device, to `out` */
static int dump(FILE *out, const sbt_tracks *t, int32_t E, int32_t H)
{
    int32_t *eto = (int32_t *)malloc(sizeof(int32_t) * (size_t)(E + 1));
    int32_t *tho = (int32_t *)malloc(sizeof(int32_t) * (size_t)(H / 3 + 1));
    int32_t *th = (int32_t *)malloc(sizeof(int32_t) * (size_t)(H > 0 ? H : 1));
    int32_t *st = (int32_t *)malloc(sizeof(int32_t) * (size_t)(E > 0 ? E : 1));
    CHECK(eto && tho && th && st, 10);
    CHECK(hipMemcpy(eto, t->event_track_offsets, sizeof(int32_t) * (size_t)(E + 1), hipMemcpyDeviceToHost) ==
              hipSuccess, 11);
    const int32_t T = eto[E];
    CHECK(T >= 0 && T <= H / 3, 12);
    CHECK(hipMemcpy(tho, t->track_hit_offsets, sizeof(int32_t) * (size_t)(T + 1), hipMemcpyDeviceToHost) ==
              hipSuccess, 13);
    const int32_t nh = tho[T];
    CHECK(nh >= 0 && nh <= H, 14);
    if (nh > 0)
        CHECK(hipMemcpy(th, t->track_hits, sizeof(int32_t) * (size_t)nh, hipMemcpyDeviceToHost) == hipSuccess, 15);
    if (E > 0)
        CHECK(hipMemcpy(st, t->event_status, sizeof(int32_t) * (size_t)E, hipMemcpyDeviceToHost) == hipSuccess, 16);
    fwrite(eto, sizeof(int32_t), (size_t)(E + 1), out);
    fwrite(tho, sizeof(int32_t), (size_t)(T + 1), out);
    fwrite(th, sizeof(int32_t), (size_t)nh, out);
    fwrite(st, sizeof(int32_t), (size_t)E, out);
    free(eto);
    free(tho);
    free(th);
    free(st);
    return 0;
}

/* overwrites the outputs so that each form's result is its own */
static int poison(const sbt_tracks *t, int32_t E, int32_t H)
{
    CHECK(hipMemset(t->event_track_offsets, 0xff, sizeof(int32_t) * (size_t)(E + 1)) == hipSuccess, 20);
    CHECK(hipMemset(t->track_hit_offsets, 0xff, sizeof(int32_t) * (size_t)(H / 3 + 1)) == hipSuccess, 21);
    CHECK(hipMemset(t->track_hits, 0xff, sizeof(int32_t) * (size_t)(H > 0 ? H : 1)) == hipSuccess, 22);
    CHECK(hipMemset(t->event_status, 0xff, sizeof(int32_t) * (size_t)(E > 0 ? E : 1)) == hipSuccess, 23);
    CHECK(hipDeviceSynchronize() == hipSuccess, 24);
    return 0;
}

int main(int argc, char **argv)
{
    CHECK(argc == 3, 1);
    FILE *f = fopen(argv[1], "rb");
    CHECK(f != NULL, 2);
    int32_t hdr[3];
    CHECK(read_all(f, hdr, sizeof hdr), 3);
    const int32_t M = hdr[0], E = hdr[1], H = hdr[2];
    CHECK(M >= 3 && M <= SBT_MAX_MODULES && E >= 0 && H >= 0, 4);
    sbt_params p;
    memset(&p, 0, sizeof p);
    p.n_modules = M;
    int32_t ints[4], tail[2];
    float floats[3];
    CHECK(read_all(f, p.module_z, sizeof(float) * (size_t)M) && read_all(f, ints, sizeof ints) &&
              read_all(f, floats, sizeof floats) && read_all(f, tail, sizeof tail), 5);
    p.reverse = ints[0];
    p.max_doublet_candidates = ints[1];
    p.phi_window_seeding = ints[2];
    p.phi_window_forwarding = ints[3];
    p.max_scatter_seeding = floats[0];
    p.max_scatter_forwarding = floats[1];
    p.max_tracklet_chi2 = floats[2];
    p.max_consecutive_misses = tail[0];
    p.max_event_hits = tail[1];
    CHECK(sbt_params_validate(&p) == SBT_OK, 6);
    const size_t n_mo = (size_t)E * (size_t)M + 1;
    int32_t *eo = (int32_t *)malloc(sizeof(int32_t) * (size_t)(E + 1));
    int32_t *mo = (int32_t *)malloc(sizeof(int32_t) * n_mo);
    float *xyz = (float *)malloc(sizeof(float) * 3 * (size_t)(H > 0 ? H : 1));
    CHECK(eo && mo && xyz, 7);
    CHECK(read_all(f, eo, sizeof(int32_t) * (size_t)(E + 1)) && read_all(f, mo, sizeof(int32_t) * n_mo) &&
              read_all(f, xyz, sizeof(float) * 3 * (size_t)H), 8);
    fclose(f);
    CHECK(sbt_validate_offsets_host(M, E, H, eo, mo) == SBT_OK, 9);

    sbt_hits hits;
    hits.n_events = E;
    hits.n_hits = H;
    hits.event_offsets = (const int32_t *)dev_copy(eo, sizeof(int32_t) * (size_t)(E + 1));
    hits.module_offsets = (const int32_t *)dev_copy(mo, sizeof(int32_t) * n_mo);
    hits.x = (const float *)dev_copy(xyz, sizeof(float) * (size_t)H);
    hits.y = (const float *)dev_copy(xyz + H, sizeof(float) * (size_t)H);
    hits.z = (const float *)dev_copy(xyz + 2 * (size_t)H, sizeof(float) * (size_t)H);
    CHECK(hits.event_offsets && hits.module_offsets && hits.x && hits.y && hits.z, 30);
    sbt_tracks tr;
    CHECK(hipMalloc((void **)&tr.event_track_offsets, sizeof(int32_t) * (size_t)(E + 1)) == hipSuccess, 31);
    CHECK(hipMalloc((void **)&tr.track_hit_offsets, sizeof(int32_t) * (size_t)(H / 3 + 1)) == hipSuccess, 32);
    CHECK(hipMalloc((void **)&tr.track_hits, sizeof(int32_t) * (size_t)(H > 0 ? H : 1)) == hipSuccess, 33);
    CHECK(hipMalloc((void **)&tr.event_status, sizeof(int32_t) * (size_t)(E > 0 ? E : 1)) == hipSuccess, 34);
    FILE *out = fopen(argv[2], "wb");
    CHECK(out != NULL, 35);

    /* plain form, caller-owned workspace, null stream */
    size_t ws_bytes = 0;
    CHECK(sbt_workspace_size(E, H, &ws_bytes) == SBT_OK, 40);
    void *ws = NULL;
    CHECK(hipMalloc(&ws, ws_bytes) == hipSuccess, 41);
    CHECK(poison(&tr, E, H) == 0, 42);
    CHECK(sbt_reconstruct(&p, &hits, &tr, ws, ws_bytes, NULL) == SBT_OK, 43);
    CHECK(hipDeviceSynchronize() == hipSuccess, 44);
    CHECK(dump(out, &tr, E, H) == 0, 45);
    CHECK(sbt_reconstruct(&p, &hits, &tr, ws, ws_bytes / 2, NULL) == SBT_ERR_WORKSPACE || ws_bytes < 2, 46);

    /* batched form on a stream of its own: the first call captures a graph,
     * the second replays it */
    sbt_context *ctx = NULL;
    CHECK(sbt_context_create(&p, NULL, E, H, &ctx) == SBT_OK, 50);
    hipStream_t s;
    CHECK(hipStreamCreate(&s) == hipSuccess, 51);
    for (int call = 0; call < 2; ++call) {
        CHECK(poison(&tr, E, H) == 0, 52);
        CHECK(sbt_reconstruct_batched(ctx, &hits, &tr, (void *)s) == SBT_OK, 53);
        CHECK(hipStreamSynchronize(s) == hipSuccess, 54);
        CHECK(dump(out, &tr, E, H) == 0, 55);
    }
    sbt_graph_stats gs;
    CHECK(sbt_context_graph_stats(ctx, &gs) == SBT_OK, 56);
    CHECK(gs.captures == 1 && gs.replays == 1 && gs.direct == 0, 57);
    sbt_context_destroy(ctx);

    /* the form that allocates nothing */
    CHECK(poison(&tr, E, H) == 0, 60);
    CHECK(sbt_reconstruct_batched_static(&p, &hits, &tr, (void *)s) == SBT_OK, 61);
    CHECK(hipStreamSynchronize(s) == hipSuccess, 62);
    CHECK(dump(out, &tr, E, H) == 0, 63);
    fclose(out);

    CHECK(hipStreamDestroy(s) == hipSuccess, 70);
    hipFree(ws);
    hipFree((void *)hits.event_offsets);
    hipFree((void *)hits.module_offsets);
    hipFree((void *)hits.x);
    hipFree((void *)hits.y);
    hipFree((void *)hits.z);
    hipFree(tr.event_track_offsets);
    hipFree(tr.track_hit_offsets);
    hipFree(tr.track_hits);
    hipFree(tr.event_status);
    free(eo);
    free(mo);
    free(xyz);
    printf("ok %d %d\n", E, H);
    return 0;
}
