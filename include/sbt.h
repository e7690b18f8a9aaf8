/*
 * sbt.h -- C ABI of the MI355X (gfx950) Search by triplet library.
 *
 * Search by triplet reconstructs straight tracks in a vertex detector made of
 * planes ("modules") perpendicular to the beam axis (paper, Section 1: the
 * problem is to partition the hits into disjoint sets compatible with straight
 * trajectories, allowing for noise; Section 3: the method).  One call
 * reconstructs a batch of independent events (Section 3, "levels of
 * parallelism": events are independent tasks).  Per event the library runs:
 *
 *   1. Sort by phi: a 16-bit angle per hit and the hits of every module
 *      ordered by (phi16, hit id).
 *   2. Track seeding and track following, alternating over consecutive
 *      modules: seeds are the best-scatter triplet per unflagged middle hit
 *      (pendulum search for doublet partners, phi window on the extrapolation
 *      into the third module); following extends forming tracks by the
 *      best-scatter hit of the next module and flags the hits it takes; a
 *      forming track ends after two consecutive misses or at the last module.
 *   3. Tracklet filter: three-hit tracks are kept only if a straight-line
 *      least-squares fit is under a threshold and none of their hits is
 *      flagged.
 *   4. Output compaction into CSR arrays.
 *
 * Precise readings of the points the paper leaves open (tie-breaks, flag
 * semantics, conflicting claims, thresholds) are given with each parameter
 * below; every stage is deterministic, so the track set of an event does not
 * depend on the batch, the launch configuration or the run.
 *
 * Conventions for every entry point
 *   - Pointers inside sbt_hits / sbt_tracks are DEVICE pointers, owned by the
 *     caller; the library neither frees them nor keeps them after the call
 *     (except that a context's graph cache remembers their values).
 *   - `stream` is a hipStream_t (NULL = the null stream).  GPU entry points are
 *     asynchronous: they only enqueue work; outputs are valid once the stream
 *     has reached that point.  They return an error code for invalid host-side
 *     arguments or a failed HIP call; per-event problems found on the device
 *     are reported in sbt_tracks.event_status.
 *   - Hit coordinates are binary32 millimetres.  Hits of an event are stored
 *     contiguously and grouped by module index; a hit's event-local id is its
 *     position inside its event.  Events hold at most 65,535 hits (hit ids
 *     are 16-bit internally).
 *   - Arithmetic is binary32, round to nearest even, no fused multiply-add
 *     contraction, correctly rounded division, denormals kept.
 */
#ifndef SBT_H
#define SBT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SBT_MAX_MODULES 64
#define SBT_MAX_EVENT_HITS 65535

/* return codes */
#define SBT_OK 0
#define SBT_ERR_INVALID_ARG (-1)     /* null pointer, parameter out of range          */
#define SBT_ERR_EVENT_TOO_LARGE (-2) /* host-checked event above 65,535 hits          */
#define SBT_ERR_HIP (-3)             /* a HIP runtime call failed                      */
#define SBT_ERR_WORKSPACE (-4)       /* workspace or context capacity too small        */
#define SBT_ERR_NOMEM (-5)           /* device or host allocation failed              */
#define SBT_ERR_NOT_READY (-6)       /* serving: nothing to return yet / queue full    */

/* event_status bits (0 = reconstructed) */
#define SBT_EV_TOO_LARGE 1u   /* more than 65,535 hits: no tracks written           */
#define SBT_EV_BAD_OFFSETS 2u /* offsets inconsistent or out of range: no tracks    */
#define SBT_EV_INTERNAL 4u    /* internal consistency check failed (never expected) */
#define SBT_EV_CUT 8u         /* rejected by the global event cut: no tracks written */

/* Physics and geometry parameters.  They change results; the oracle takes the
 * same values.  Defaults used by the tests and benchmark are in parentheses.
 *
 * n_modules       M, 3..64.  module_z[k] is the nominal z of module k; the phi
 *                 window of an extrapolation is centred on the extrapolated
 *                 position at this z (Section 3, seeding: "each doublet is
 *                 extrapolated to the third module").
 * reverse         1: traverse modules from index M-1 down to 0, i.e. starting
 *                 furthest from the interaction region when z grows with the
 *                 index; 0: from 0 up to M-1 (Section 3: the traversal
 *                 direction is configurable).  (1)
 * max_doublet_candidates
 *                 K, unflagged partners collected by the pendulum search
 *                 (Section 3: "until a threshold number of candidate hits that
 *                 are not flagged is found"; its figure uses four).  >= 1.  (4)
 * phi_window_seeding / phi_window_forwarding
 *                 inclusive half-width W of the phi window, in phi16 units
 *                 (2^16 per turn), 0..32767.  A hit is in the window of centre
 *                 c iff its signed 16-bit difference to c is within [-W, W];
 *                 the window wraps around the circle.  (416, 416)
 * max_scatter_seeding / max_scatter_forwarding
 *                 strict upper bound on the scatter dx^2 + dy^2 (mm^2)
 *                 between a linear extrapolation and a candidate hit, both at
 *                 the candidate's z (Section 3).  (0.04, 0.04)
 * max_tracklet_chi2
 *                 strict upper bound (mm^2) on the sum of squared residuals of
 *                 least-squares lines x(z), y(z) through a three-hit track
 *                 (Section 3, "Tracklet filter").  (0.002)
 * max_consecutive_misses
 *                 modules a forming track may skip in a row and still be
 *                 followed (Section 3: "allowed for tracks to miss a
 *                 module").  >= 0.  (1)
 * max_event_hits  global event cut (Section 4, the first step of the paper's
 *                 sequence, which drops the most densely populated events):
 *                 an event with more hits is not reconstructed, gets status
 *                 SBT_EV_CUT and no tracks.  0: no cut.  >= 0.  (0)
 *                 sbt_gec_threshold computes the value that rejects a given
 *                 fraction of a sample.
 */
typedef struct sbt_params {
    int32_t n_modules;
    float module_z[SBT_MAX_MODULES];
    int32_t reverse;
    int32_t max_doublet_candidates;
    int32_t phi_window_seeding;
    int32_t phi_window_forwarding;
    float max_scatter_seeding;
    float max_scatter_forwarding;
    float max_tracklet_chi2;
    int32_t max_consecutive_misses;
    int32_t max_event_hits;
} sbt_params;

/* Input batch (device pointers).
 * event_offsets   [n_events+1], event_offsets[0] = 0, non-decreasing,
 *                 event_offsets[n_events] = n_hits.
 * module_offsets  [n_events*M + 1] absolute hit offsets: module k of event e
 *                 is [module_offsets[e*M+k], module_offsets[e*M+k+1]);
 *                 module_offsets[e*M] = event_offsets[e].
 * x, y, z         [n_hits] structure of arrays.                          */
typedef struct sbt_hits {
    int32_t n_events;
    int32_t n_hits;
    const int32_t *event_offsets;
    const int32_t *module_offsets;
    const float *x;
    const float *y;
    const float *z;
} sbt_hits;

/* Input batch with half-precision coordinates in array-of-structures form,
 * the paper's storage optimisation for hit coordinates (Section 4,
 * optimisation table: fp-16 and AOS for VELO hit coordinates).
 * xyzw            [4*n_hits] binary16 bit patterns, hit i at 4i: x, y, z and
 *                 one unused value (8 bytes per hit instead of 12).
 * Offsets as in sbt_hits.  Coordinates are widened to binary32 exactly when
 * loaded and every computation is the binary32 one of sbt_hits, so the
 * result equals sbt_reconstruct_batched on the binary16 values widened.  */
typedef struct sbt_hits_f16 {
    int32_t n_events;
    int32_t n_hits;
    const int32_t *event_offsets;
    const int32_t *module_offsets;
    const uint16_t *xyzw;
} sbt_hits_f16;

/* Output, CSR over events and tracks: device memory, or pinned host memory
 * (hipHostMalloc) that the kernels write directly; they never read it back.
 * Capacities follow from the method: tracks are disjoint and have >= 3 hits.
 * event_track_offsets [n_events+1]: tracks of event e are
 *                 [event_track_offsets[e], event_track_offsets[e+1]).
 * track_hit_offsets   [n_hits/3 + 1]: hits of track t are
 *                 track_hits[track_hit_offsets[t] .. track_hit_offsets[t+1]).
 * track_hits      [n_hits]: event-local hit ids in traversal order.
 * event_status    [n_events] or NULL: SBT_EV_* bits, 0 when reconstructed.
 * Tracks of an event are ordered by the id of their seed's middle hit.    */
typedef struct sbt_tracks {
    int32_t *event_track_offsets;
    int32_t *track_hit_offsets;
    int32_t *track_hits;
    int32_t *event_status;
} sbt_tracks;

/* Launch configuration of the batched path.  It never changes results.
 * threads_per_event   64, 128, 256, 512 or 1024 lanes cooperating on one event.
 * blocks_per_cu       persistent workgroups per compute unit (1..16).
 * lds_window_hits     capacity, in hits, of each of the four LDS slots that
 *                     hold the phi-sorted hits of consecutive modules
 *                     (0..2048), rounded down to a compiled one (0, 256,
 *                     448, 672, 768, 1024, 1536); an event with a larger
 *                     module reads all its modules from memory.
 * lds_owner_hits      events with at most this many hits keep their hit
 *                     flags (one bit per hit) in LDS, larger ones in
 *                     memory (0..65536).
 * events_per_block    events one workgroup runs side by side (0 or 1: one;
 *                     up to 16, only with threads_per_event = 64).  Each
 *                     64-lane event is one wave with its own LDS region and
 *                     takes its next event from the queue on its own, so the
 *                     waves of a workgroup never wait for one another.
 * deferred_window_hits 0: events whose busiest module exceeds the slots run
 *                     from memory.  > 0 (only with 512 lanes, three or more
 *                     workgroups per CU and 448-hit slots, which run the
 *                     kernel instance held to six waves per SIMD): such events
 *                     are set aside and run in a second pass with slots of
 *                     this many hits (512 lanes x 2 per CU, or 1,024 x 1 above
 *                     768 hits).  Must exceed the first pass's slots.
 * The LDS of a workgroup (both capacities, times events_per_block for
 * 64-lane events) is at most 159 KiB.                                      */
typedef struct sbt_tuning {
    int32_t threads_per_event;
    int32_t blocks_per_cu;
    int32_t lds_window_hits;
    int32_t lds_owner_hits;
    int32_t events_per_block;
    int32_t deferred_window_hits;
} sbt_tuning;

/* Message for a return code (static storage). */
const char *sbt_error_string(int code);

/* Check a parameter block (host memory).  SBT_OK or SBT_ERR_INVALID_ARG. */
int sbt_params_validate(const sbt_params *params);

/* Host-side check of offsets held in HOST memory (optional; the device
 * checks the same conditions per event and reports them in event_status).
 * Returns SBT_OK, SBT_ERR_INVALID_ARG or SBT_ERR_EVENT_TOO_LARGE.         */
int sbt_validate_offsets_host(int32_t n_modules, int32_t n_events, int32_t n_hits,
                              const int32_t *event_offsets, const int32_t *module_offsets);

/* ---- plain per-event form --------------------------------------------------
 * Bytes of device workspace sbt_reconstruct needs for a batch of this size. */
int sbt_workspace_size(int32_t n_events, int32_t n_hits, size_t *bytes);

/* Reconstruct a batch with the plain per-event kernels: one workgroup of 512
 * lanes per event and one launch per stage (phi sort, seeding and following, tracklet
 * filter, per-event compaction, scan over events, CSR write), all enqueued on
 * `stream`.  `workspace` is caller-owned device memory of at least
 * sbt_workspace_size() bytes, 256-byte aligned; it must not be used by
 * another call until this one has completed on the stream.               */
int sbt_reconstruct(const sbt_params *params, const sbt_hits *hits, sbt_tracks *tracks,
                    void *workspace, size_t workspace_bytes, void *stream);

/* ---- batched form ------------------------------------------------------------
 * A context owns device workspace for up to max_events events / max_hits
 * hits, the launch configuration and a cache of captured HIP graphs (one per
 * distinct argument set).  Create and destroy on the host thread that uses it;
 * a context runs one batch at a time (calls on different streams serialise on
 * its workspace only if the caller orders them).                         */
typedef struct sbt_context sbt_context;

/* tuning: the launch configuration of every call, or NULL to choose it per
 * call from the batch's size on the current device (lds_owner_hits 16,384
 * throughout):
 *   - events of 2,500 hits or fewer on average: 256 lanes, five workgroups
 *     per compute unit and 256-hit LDS slots when there are more than two
 *     events per compute unit, else 512 lanes, two per compute unit,
 *     448-hit slots;
 *   - at most one event per compute unit, or at most two of 4,000 hits or
 *     more on average, or any number of 9,000 hits or more on average:
 *     1,024 lanes, one workgroup per compute unit, 1,536-hit slots;
 *   - fifteen or more events per compute unit of 4,000 hits or more on
 *     average: two passes, 512 lanes, three workgroups per compute unit,
 *     448-hit slots, then the events those slots cannot hold with 768-hit
 *     slots (deferred_window_hits);
 *   - other events of 4,000 hits or more on average: 512 lanes, two per
 *     compute unit, 768-hit slots;
 *   - six or more other events per compute unit: 512 lanes, three per
 *     compute unit, 448-hit slots;
 *   - otherwise 512 lanes, two per compute unit, 672-hit slots.
 * sbt_context_set_tuning and sbt_autotune install one configuration for
 * every later call; sbt_context_get_tuning reports the installed one, or
 * without one the choice for a batch of max_events events and max_hits
 * hits.  Results never depend on the configuration.                      */
int sbt_context_create(const sbt_params *params, const sbt_tuning *tuning,
                       int32_t max_events, int32_t max_hits, sbt_context **out);
void sbt_context_destroy(sbt_context *ctx);
int sbt_context_set_tuning(sbt_context *ctx, const sbt_tuning *tuning);
int sbt_context_get_tuning(const sbt_context *ctx, sbt_tuning *out);

/* Reconstruct a batch with the persistent work-stealing kernel: every stage
 * of an event runs inside one workgroup, which then takes the next event
 * from a device counter; the counter reset, the persistent kernel, the scan
 * over events and the CSR write are replayed as one captured HIP graph.
 * Same outputs as sbt_reconstruct, byte for byte.                        */
int sbt_reconstruct_batched(sbt_context *ctx, const sbt_hits *hits, sbt_tracks *tracks,
                            void *stream);

/* sbt_reconstruct_batched for half-precision array-of-structures hits
 * (sbt_hits_f16).  Same errors; xyzw must be 8-byte aligned.             */
int sbt_reconstruct_batched_f16(sbt_context *ctx, const sbt_hits_f16 *hits, sbt_tracks *tracks, void *stream);

/* ---- the batched form without allocation -------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * kernels as sbt_reconstruct_batched, in the launch configuration the
 * context chooses per call from the batch's size, with their workspace in a
 * static device array of SBT_STATIC_SCRATCH_BYTES that the library holds on
 * every GPU it runs on until the process ends (no context, no allocation, no
 * graph capture of its own; the caller may capture the call).  A batch fits
 * when sbt_workspace_size(n_events, n_hits) <= SBT_STATIC_SCRATCH_BYTES
 * (about 680,000 hits for 200 events); a larger one is refused with
 * SBT_ERR_WORKSPACE before anything is enqueued.  The first call on a device
 * looks the array's device address up (hipGetSymbolAddress).
 * Every call on one GPU shares that GPU's array: calls whose work overlaps
 * on the device (different streams, or different host threads, without
 * ordering between them) race on it and give undefined results; order them
 * on one stream or with events.  The kernels initialise all of the array
 * they read, so the previous call's contents never change a result.
 * Same outputs as sbt_reconstruct_batched, byte for byte.  Returns SBT_OK,
 * SBT_ERR_INVALID_ARG, SBT_ERR_WORKSPACE or SBT_ERR_HIP.                   */
#define SBT_STATIC_SCRATCH_BYTES (64u << 20)
int sbt_reconstruct_batched_static(const sbt_params *params, const sbt_hits *hits, sbt_tracks *tracks,
                                   void *stream);

/* Time the candidate launch configurations on `sample` (reps launches each,
 * after one warm-up) and install the fastest in the context.  `tracks` is
 * scratch output of the sample's size.  Writes the chosen tuning and its mean
 * milliseconds per launch.  Synchronises `stream`.                        */
int sbt_autotune(sbt_context *ctx, const sbt_hits *sample, sbt_tracks *tracks, void *stream,
                 int32_t reps, sbt_tuning *best, float *best_ms);

/* Stage timing of the last call on this context, in milliseconds, measured
 * with HIP events on the call's stream when profiling is on (graphs are then
 * bypassed).  stage_ms[0] = persistent kernel, [1] = scan, [2] = CSR write.
 * Synchronises on the events.                                             */
int sbt_context_set_profiling(sbt_context *ctx, int32_t on);
int sbt_context_stage_ms(sbt_context *ctx, float *stage_ms, int32_t n);

/* Graph cache of a context.  sbt_reconstruct_batched on a non-null stream
 * with profiling off captures the batched sequence once per argument set
 * (batch size, every device pointer of the hits and the tracks) and replays
 * the instantiated graph on later calls with the same set; at most
 * `capacity` graphs are kept, the least recently used one is evicted.  On
 * the null stream or with profiling on, the kernels are launched directly.
 *   cached     graphs in the cache now
 *   capacity   most graphs kept (8)
 *   captures   graphs captured and instantiated (each launched once at once)
 *   replays    calls served by a graph already in the cache
 *   evictions  graphs dropped to make room (sbt_context_set_tuning clears
 *              the cache without counting evictions)
 *   direct     calls launched without a graph
 * Host-side counters only; returns SBT_OK or SBT_ERR_INVALID_ARG.        */
typedef struct sbt_graph_stats {
    int32_t cached;
    int32_t capacity;
    int64_t captures;
    int64_t replays;
    int64_t evictions;
    int64_t direct;
} sbt_graph_stats;

int sbt_context_graph_stats(const sbt_context *ctx, sbt_graph_stats *out);

/* ---- inspection ----------------------------------------------------------------
 * Run only the phi sort of the plain form and copy its result: for every
 * hit position p of the batch (module by module, phi16 ascending, ties by
 * lower id) phi_sorted[p] is the 16-bit angle and ids_sorted[p] the
 * event-local id.  Device pointers of n_hits uint16 each.                */
int sbt_debug_phi_sort(const sbt_params *params, const sbt_hits *hits, uint16_t *phi_sorted,
                       uint16_t *ids_sorted, void *workspace, size_t workspace_bytes,
                       void *stream);

/* The same result from the paper's sort (Section 3, "Sort by phi": a parallel
 * insertion sort computes the permutation), for comparison with the library's
 * bucket sort: each hit's rank is the number of hits of its module with a
 * smaller (phi16, id) key, O(n^2) per module.  Same arguments and errors as
 * sbt_debug_phi_sort; synchronises `stream` once to size its LDS.          */
int sbt_debug_phi_sort_rank(const sbt_params *params, const sbt_hits *hits, uint16_t *phi_sorted,
                            uint16_t *ids_sorted, void *workspace, size_t workspace_bytes,
                            void *stream);

/* The plain form with the paper's separate candidate pass, for comparison
 * with the fused search (Section 4, optimisation table: a "Fill candidates"
 * kernel was split from the tracklet filter and later removed; the paper
 * does not say what it computes).  Reading taken here: the pass computes,
 * for every hit of every module but the first in traversal order, the part of
 * the doublet search that does not depend on the flags -- its pendulum start,
 * the first position of the preceding module whose phi16 is >= the hit's
 * (0 when there is none) -- and writes it into the workspace; the seeding
 * kernel then reads the start instead of searching for it.  Same arguments,
 * errors and outputs as sbt_reconstruct, byte for byte.                    */
int sbt_debug_reconstruct_fill_candidates(const sbt_params *params, const sbt_hits *hits, sbt_tracks *tracks,
                                          void *workspace, size_t workspace_bytes, void *stream);

/* The host conversion of the server's binary16 transfer: n hits from binary32
 * x, y, z (HOST memory) to the 8-byte records of sbt_hits_f16 (x, y, z, 0;
 * each rounded to the nearest binary16, ties to even) in `out` (HOST, 4n
 * uint16).  SBT_OK, or SBT_ERR_INVALID_ARG for null pointers or n < 0.     */
int sbt_debug_half_records(const float *x, const float *y, const float *z, int32_t n, uint16_t *out);

/* ---- the steps around Search by triplet in the paper's sequence (Section 4) ----------
 *
 * Global event cut: the threshold on the hit count that rejects at most
 * floor(fraction * n_events) of the events, the most densely populated ones.
 * It is the smallest count c, among 0 and the event sizes, that at most that
 * many events exceed; events tied at c are kept.  event_offsets is a HOST
 * array of n_events+1 entries.  fraction in [0, 1].  Put the result in
 * sbt_params.max_event_hits.  Returns SBT_OK or SBT_ERR_INVALID_ARG.      */
int sbt_gec_threshold(int32_t n_events, const int32_t *event_offsets, double fraction, int32_t *max_hits);

/* Consolidation: the track data packed for the algorithms that follow.  For
 * every track of `tracks` (device arrays, as sbt_reconstruct* wrote them):
 *   hit_x/hit_y/hit_z [sum of track lengths]: the coordinates of track_hits,
 *                 in the same order (copies of the input values);
 *   state [6 * n_tracks]: per track x, y, z (the mean of its hits), tx, ty
 *                 (dx/dz, dy/dz) and chi2 / (2n - 4), from an unweighted
 *                 least-squares fit of x and y against z over its n hits.
 * The fit is binary32: means first, then sums centred on the means, each
 * accumulated in track order.  Capacities: n_hits floats for each hit_*
 * array and 6 * (n_hits / 3) for state.  Device pointers, or pinned host
 * memory the kernels write.  Asynchronous on `stream`.  `hits` must be the
 * batch the tracks came from.  Returns SBT_OK, SBT_ERR_INVALID_ARG or SBT_ERR_HIP. */
typedef struct sbt_track_states {
    float *hit_x, *hit_y, *hit_z;
    float *state;
} sbt_track_states;

int sbt_consolidate(const sbt_hits *hits, const sbt_tracks *tracks, sbt_track_states *out, void *stream);

/* ---- serving ---------------------------------------------------------------------
 * Continuous batching of single events that arrive over time.  The server
 * keeps `n_slots` batches of device memory resident (inputs and workspace,
 * `slot_hits`/`slot_events` capacity each, all inside `device_budget_bytes`),
 * admits queued events into the open slot while it has room, and launches a
 * slot on its own stream as soon as its previous launch is complete and
 * either it is full or `max_wait_us` passed since its oldest event was
 * queued.  Several slots are in flight at once, so events that arrive while
 * others are on the GPU overlap with them.  The kernels write each event's
 * tracks into pinned host memory owned by the server (about
 * 5.4 * slot_hits bytes per block, n_slots + 1 blocks, more while the caller
 * holds results across polls).  Results of an event are identical to
 * reconstructing it alone.                                               */
typedef struct sbt_server sbt_server;

typedef struct sbt_server_config {
    size_t device_budget_bytes;  /* upper bound on the server's device memory    */
    int32_t n_slots;             /* resident batches (>= 1)                        */
    int32_t slot_events;         /* events per batch (>= 1)                        */
    int32_t slot_hits;           /* hits per batch (>= 65,535 so any event fits)   */
    int32_t max_wait_us;         /* launch a partial batch after this wait         */
    int32_t coords_f16;          /* 1: hits travel to the device as binary16 (each
                                    coordinate rounded to nearest even on the host,
                                    8 bytes per hit instead of 12); results are those
                                    of the rounded hits, as sbt_reconstruct_batched_f16
                                    gives them.  0: binary32.                       */
} sbt_server_config;

/* A completed event: its tracks in the same CSR form as one event of
 * sbt_tracks (offsets local to this event), valid until the next
 * sbt_server_poll call on this server.                                    */
typedef struct sbt_server_result {
    int64_t request_id;
    int32_t status;              /* event_status bits                             */
    int32_t n_tracks;
    const int32_t *track_hit_offsets;  /* host, [n_tracks+1]                    */
    const int32_t *track_hits;         /* host                                   */
    double t_submit_us;          /* host clock (microseconds, monotonic)           */
    double t_done_us;            /* when the result was visible on the host        */
} sbt_server_result;

/* tuning: the launch configuration of every slot, or NULL to choose it per
 * launch from the slot's size by the rule sbt_context_create describes
 * (slots of at most one event per compute unit, or two large ones, run
 * 1,024 lanes per event, each event then finishing sooner).  Results never
 * depend on it.                                                          */
int sbt_server_create(const sbt_params *params, const sbt_tuning *tuning,
                      const sbt_server_config *config, sbt_server **out);
void sbt_server_destroy(sbt_server *srv);

/* Queue one event from HOST memory (copied before return).  module_offsets
 * has n_modules+1 event-local entries.  Returns SBT_OK, SBT_ERR_INVALID_ARG,
 * SBT_ERR_EVENT_TOO_LARGE, or SBT_ERR_NOT_READY when the host queue holds
 * max queued events (n_slots * slot_events * 4).                          */
int sbt_server_submit(sbt_server *srv, int64_t request_id, int32_t n_hits,
                      const int32_t *module_offsets, const float *x, const float *y,
                      const float *z);

/* Drive the server: admit, launch and collect.  Writes up to max_results
 * completed events; returns their number (>= 0) or an error.  With
 * wait_us > 0 it blocks up to that long for at least one completion.
 * Each launch writes its results into a pinned host result block, which is
 * reused once no slot and no completed result refers to it.  The server
 * holds at most 3 * n_slots + 2 blocks: while completed results stay
 * unreturned (polls with a small max_results), further launches wait, and
 * their events stay queued, until polls have returned enough results.     */
int sbt_server_poll(sbt_server *srv, sbt_server_result *results, int32_t max_results,
                    int32_t wait_us);

/* Load replay, for measuring the server.  Arrival i (0..n_arrivals-1) is
 * event picks[i] of a packed HOST pool (pool_events events; event_offsets
 * [pool_events+1], module_offsets [pool_events*M+1] absolute, x/y/z); it is
 * submitted at start + arrival_us[i] (microseconds, non-decreasing) while the
 * server is polled continuously, its hits read in place (the pool must stay
 * unchanged during the call).  Writes each arrival's latency (result visible
 * on the host minus its arrival time) into latency_us[i], its track count
 * into n_tracks[i] (may be NULL), and the wall time into *wall_us.
 * The server must be idle (nothing queued, on the device or uncollected;
 * see sbt_server_pending): otherwise SBT_ERR_NOT_READY, since results are
 * matched to arrivals by request id.  SBT_ERR_INVALID_ARG for a pick outside
 * the pool or negative event size, SBT_ERR_EVENT_TOO_LARGE for an event of
 * more than 65,535 hits; both are checked before the first submission.   */
int sbt_server_replay(sbt_server *srv, int32_t n_arrivals, const double *arrival_us, const int32_t *picks,
                      int32_t pool_events, const int32_t *event_offsets, const int32_t *module_offsets,
                      const float *x, const float *y, const float *z,
                      double *latency_us, int32_t *n_tracks, double *wall_us);

/* Events queued on the host, and events on the device. */
int sbt_server_pending(const sbt_server *srv, int32_t *queued, int32_t *in_flight);

/* Result blocks the server holds (each the pinned host memory for one
 * slot's results) and the most it will hold (3 * n_slots + 2).  Either
 * pointer may be NULL.  SBT_OK, or SBT_ERR_INVALID_ARG for a NULL server. */
int sbt_server_result_blocks(const sbt_server *srv, int32_t *n_blocks, int32_t *limit);

/* Host monotonic clock in microseconds (the clock of t_submit_us). */
double sbt_now_us(void);

#ifdef __cplusplus
}
#endif

#endif /* SBT_H */
