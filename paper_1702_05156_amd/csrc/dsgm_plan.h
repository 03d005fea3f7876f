// dsgm_plan.h -- the host image of a batch plan (internal, host only).
//
// dsgm_plan_batched builds this image and copies it to the caller's plan
// buffer; the host-side geometry checker of the test suite builds it too and
// walks every work item and counter stripe in it.
#pragma once

#include <stdint.h>

#include <vector>

#include "dsgm.h"
#include "dsgm_internal.h"

namespace dsgm {

struct PlanImage {
  int P = 4;  // pixels per lane, common to all instances
  int64_t n_items = 0, total = 0;
  // byte offsets in the plan buffer: item counter at 0, instance descriptors
  // (BatchInst) at inst_off, work items (BatchItem, LPT order) at items_off,
  // foreground-count stripes at stripes_off; bytes in all
  int64_t inst_off = 0, items_off = 0, stripes_off = 0, bytes = 0;
  bool bg = false, counts = false;
  std::vector<char> host;  // the buffer's contents, pointers as on the device
};

// Validate the instances and build the plan's image for a plan buffer at
// `plan_buffer` (device address, only stored into the descriptors).  No HIP
// call; returns a dsgm_status.
int plan_image(const dsgm_instance* instances, int32_t n, int in_dtype, int acc, void* plan_buffer,
               PlanImage* img);

}  // namespace dsgm
