// Host side of the work-unit queue of the persistent batch kernel: turns a
// list of independent transforms into pass descriptors and work units in
// queue order.  Shared by the batch API and the serving loop.
#pragma once

#include <cstdint>
#include <stdexcept>
#include <vector>

#include "batch.h"
#include "jt.h"
#include "plan.h"

namespace jt {

// A size/precision combination the kernels are not built for.
struct unsupported : std::runtime_error {
    using std::runtime_error::runtime_error;
};

// One transform: d axes (axis plans and the device images their section
// offsets are relative to), a direction and byte offsets of its input and
// output tensors from the run's base pointers.
struct QueueItem {
    int d = 0;
    const AxisPlan *ax[3] = {nullptr, nullptr, nullptr};
    const unsigned char *base[3] = {nullptr, nullptr, nullptr};
    int dir = JT_FORWARD;
    uint64_t in_off = 0, out_off = 0;
};

struct WorkQueue {
    std::vector<PassDesc> passes;
    std::vector<WorkUnit> units;
    std::vector<int32_t> pass_item, pass_axis;
    double cost = 0;
    size_t off_units = 0, off_passes = 0, off_counters = 0, bytes = 0;
};

// Passes along axes d-1 .. 0 for every item (first pass reads the input,
// later ones work in place on the output), cut into units whose rank split
// follows opt; queue order puts every first pass before every second pass
// before every third pass, costliest units first within each.  Throws
// std::invalid_argument (bad item) or unsupported.
void build_queue(const std::vector<QueueItem> &items, const jt_batch_options &opt, bool fp32, jt_dtype tin,
                 jt_dtype tout, WorkQueue &q);

// Fill the factor pointers of every pass from its item's image bases.
void resolve_factors(WorkQueue &q, const std::vector<QueueItem> &items, bool fp32);

// Device image of the queue: units, passes, zeroed counters (q.bytes long).
std::vector<unsigned char> queue_image(const WorkQueue &q);

}  // namespace jt
