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

// The library's default launch configuration.
sbt_tuning default_tuning_config();
int tuning_valid(const sbt_tuning &t);

}  // namespace sbt
