// dpd_runtime.hpp -- host-side calls of the runtime (dpd_capi.hip) that the
// request server (dpd_server.cpp) uses beside the public ABI of dpd.h: they
// enqueue work without synchronising, so that one quantum of a batch can run
// on the GPU while the host retires the previous one and admits new requests.
#pragma once
#include <hip/hip_runtime.h>

#include "dpd.h"
#include "dpd_internal.hpp"

namespace dpd {

// Make later work of the box (its result reads, and the waits of the batches
// it belongs to) go to stream s.  The box must be idle on its old stream.
int box_set_stream(dpd_box b, hipStream_t s);

// Enqueue, on the box's stream and without synchronising, the copies of its
// final state and device statistics to host memory: pos_n3 and vel_n3 (n x 3
// floats, id order, as dpd_read of DPD_POS and DPD_VEL) and *dev_stats.  The
// host buffers must be pinned (hipHostMalloc) for the copies to run
// asynchronously, and stay untouched until the stream has passed them.
int box_enqueue_results(dpd_box b, float* pos_n3, float* vel_n3, DevStats* dev_stats);

// The public statistics of a device record (as dpd_get_stats fills them).
void stats_from_device(const DevStats& s, dpd_stats* out);

// Destroy a box without synchronising its stream: the caller has seen every
// piece of work that touches the box complete.
void box_release(dpd_box b);

// Replace the boxes of a batch (at most the count its tables were sized for
// at dpd_batch_create) and enqueue the new tables on the batch stream,
// ordered after the work already on it; nothing is synchronised.
int batch_set_boxes(dpd_batch bt, const dpd_box* boxes, int32_t nboxes);

}  // namespace dpd
