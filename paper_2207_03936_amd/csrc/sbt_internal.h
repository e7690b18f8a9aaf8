// Library-internal entry points shared between the kernel translation unit
// and the serving loop.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "sbt.h"

namespace sbt {

// Device workspace bytes for a batch of E events and H hits.
size_t workspace_bytes(int32_t E, int32_t H);

// The batched sequence (counter reset, persistent kernel, scan, CSR write)
// on `stream` with an explicit workspace, without graph capture.
int launch_batched_raw(const sbt_params &params, const sbt_tuning &tuning, const sbt_hits &hits,
                       const sbt_tracks &tracks, void *workspace, hipStream_t stream);

// Per-event track lists, each a CSR of its own, for a batch of E events with
// T accepted tracks in all.  Any memory the device can write (device or
// pinned host memory).
struct EventOut {
    int32_t *eto;     // [E+1] the batch's track offsets per event
    int32_t *status;  // [E]   event_status bits
    int32_t *hoff;    // [E]   first position of event e's hits in th
    int32_t *tho;     // [T+E] event e's offsets, from 0, at tho[eto[e]+e .. eto[e+1]+e]
    int32_t *th;      // [sum of track lengths] hit ids, event by event
};

// The batched sequence writing per-event lists (E >= 1), from binary32 or
// binary16 hits.
int launch_batched_events(const sbt_params &params, const sbt_tuning &tuning, const sbt_hits &hits,
                          const EventOut &out, void *workspace, hipStream_t stream);
int launch_batched_events_f16(const sbt_params &params, const sbt_tuning &tuning, const sbt_hits_f16 &hits,
                              const EventOut &out, void *workspace, hipStream_t stream);

// The library's default launch configuration, and the one it chooses for a
// batch of E events and H hits on a device of `cus` compute units.
sbt_tuning default_tuning_config();
sbt_tuning batch_tuning(int32_t E, int32_t H, int cus);
int tuning_valid(const sbt_tuning &t);

}  // namespace sbt
