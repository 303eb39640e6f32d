// Deposits of track events (ct_track.hip), called by the host side at
// seeding.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ct_internal.hpp"

namespace ct {

// For every event b with seg_len[b] > 0: replace the start point held in
// deposits[dep_off[b]] by the midpoints of the event's walk, in deposit slots
// dep_off[b] .. dep_off[b + 1] - 1 (one thread per event, on stream s).
hipError_t launch_track(const DevParams &dp, int32_t n_events, uint64_t first_event_id,
                        const int32_t *dep_off, const double *seg_len, double *deposits,
                        hipStream_t s);

}  // namespace ct
