// batch.h -- host interface of a batch: one handle that holds `slots` independent 2D
// problems of one size and advances all of them with one captured step per launch.
//
// Slot k owns the k-th [n*n] block of every level array and its own DevState; a parked
// slot (done = 1) costs one flag read per kernel.  Every call below is asynchronous on
// the batch's stream and ordered with the replays, so a slot can be retired and
// re-admitted between two replays without waiting for the device.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <string>

#include "mg.h"
#include "mg_internal.h"

namespace mgb {

// The leading fields of DevState, read for every slot after a chunk of replays.
struct SlotFlags {
  int done, checks, status, stall;
};

// Device bytes of a batch of `slots` problems (the handle owns level-0 f and u).
size_t footprint(const mg_config *cfg, int slots);
// A batch for cfg (dim 2), its steps captured into one graph, every slot parked.
mg_status create(const mg_config *cfg, int slots, hipStream_t stream, mg_ctx **out);
void destroy(mg_ctx *c);
// Copies f (device, n*n FP64) into slot k, zeroes its iterate and starts its solve
// (state reset, ||f|| on the device).  f may be reused once the batch stream passes
// this point.
mg_status admit(mg_ctx *c, int slot, const double *f);
// `count` replays of the captured step over all slots.
mg_status step(mg_ctx *c, int count);
// Copies every slot's SlotFlags into host (pinned, `slots` entries).
mg_status read_flags(mg_ctx *c, SlotFlags *host);
// Copies slot k's iterate to u_dst (device) and its state to host_state (pinned).
mg_status retire(mg_ctx *c, int slot, double *u_dst, mgk::DevState *host_state);
// The result of a finished slot from its state.
void result(const mg_ctx *c, const mgk::DevState &hs, mg_result *res, mg_status *outcome);
// Sets the calling thread's mg_last_error message.
void set_error(const std::string &msg);

}  // namespace mgb
