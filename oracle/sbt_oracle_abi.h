/*
 * Search by triplet CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * The batch entry point with structures of the same layout as the GPU
 * library's public parameter, input and output structures, declared here
 * anew: the oracle includes nothing of the library.  A C caller can pass the
 * library's own structures, holding host pointers, to sbt_reconstruct_cpu;
 * a test compiles both headers and compares every size and field offset.
 *
 * Per-event status bits (written when event_status is not NULL); an event
 * with a status gets no tracks:
 *   ORC_EV_TOO_LARGE   1  more than 65,535 hits (hit ids are 16-bit)
 *   ORC_EV_BAD_OFFSETS 2  event range outside [0, n_hits] or decreasing, or
 *                         module offsets not running from the event's first
 *                         hit to its end without decreasing
 *   ORC_EV_CUT         8  more than max_event_hits hits (global event cut)
 * The first condition that holds, in the order bad range, too large, cut,
 * then bad module offsets, sets the status.
 */
#ifndef SBT_ORACLE_ABI_H
#define SBT_ORACLE_ABI_H

#include <stdint.h>

#define ORC_EV_TOO_LARGE 1
#define ORC_EV_BAD_OFFSETS 2
#define ORC_EV_CUT 8

typedef struct orc_abi_params {
    int32_t n_modules;
    float module_z[64];
    int32_t reverse;
    int32_t max_doublet_candidates;
    int32_t phi_window_seeding;
    int32_t phi_window_forwarding;
    float max_scatter_seeding;
    float max_scatter_forwarding;
    float max_tracklet_chi2;
    int32_t max_consecutive_misses;
    int32_t max_event_hits;
} orc_abi_params;

typedef struct orc_abi_hits {
    int32_t n_events;
    int32_t n_hits;
    const int32_t *event_offsets;    /* [n_events+1] */
    const int32_t *module_offsets;   /* [n_events*n_modules+1], absolute */
    const float *x;
    const float *y;
    const float *z;
} orc_abi_hits;

typedef struct orc_abi_tracks {
    int32_t *event_track_offsets;    /* [n_events+1] */
    int32_t *track_hit_offsets;      /* [n_hits/3+1] */
    int32_t *track_hits;             /* [n_hits] */
    int32_t *event_status;           /* [n_events] or NULL */
} orc_abi_tracks;

/* Reconstructs every event in order (host memory).  Returns 0, -1 for a
 * null pointer or a parameter out of range, -5 when memory runs out. */
int sbt_reconstruct_cpu(const orc_abi_params *params, const orc_abi_hits *hits, orc_abi_tracks *tracks);

#endif
