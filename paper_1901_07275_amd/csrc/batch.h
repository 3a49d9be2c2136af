// Work description of the persistent batch kernel: many independent
// transforms of uneven size, dimension and (a, b) in one launch.
//
// Every axis pass of every item becomes one PassDesc; every pass is cut into
// work units of a few lines (a small multi-axis item instead becomes a single
// unit that runs all its passes in order inside one block).  The units sit in a device table in queue order;
// the blocks of one persistent grid take them one at a time from an atomic
// head counter.  A unit of a later axis pass of an item waits until every unit
// of that item's previous pass has been counted done (the passes of one item
// must run in order; different items never wait on each other).  Units of
// first passes come first in the queue, so a wait only ever targets units that
// running blocks already hold, and the grid cannot deadlock.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "dense_shape.h"

namespace jt {

// One axis pass of one item.  Tensor pointers are byte offsets from the
// run's input and output base pointers, so one table serves any pair of
// buffers with the same layout (and a captured graph serves one pair).
struct PassDesc {
    uint64_t in_off = 0, out_off = 0;
    int32_t in_from_out = 0;  // 1: read the output buffer (every pass after the item's first)
    int32_t in_f64 = 1, out_f64 = 1;
    int32_t lines = 0, stride = 1;
    int32_t n = 0, L = 0, nu0 = 0, rank = 0, max_per_bin = 0;
    int32_t forward = 1;
    int32_t publish = 0;      // a later pass of the item waits for this one (cross-block)
    int32_t split = 1, cap = 1;  // rank split and lines per chunk of this pass
    // factor sections of the item's bound plan (device pointers)
    const void *tw = nullptr;
    const int *bins = nullptr;
    const int *binptr = nullptr;
    const void *wv = nullptr;
    const void *u = nullptr;
    const void *v = nullptr;
};

// A contiguous range of lines of one pass, processed by one block.
struct WorkUnit {
    int32_t pass = 0;        // index into the PassDesc table
    int32_t line0 = 0;       // first line
    int32_t nlines = 0;      // lines (the block's capacity at split S, or fewer at the end)
    int32_t split = 1;       // S: split groups sharing each line (rank terms divided among them)
    int32_t wait_pass = -1;  // pass that must be complete first (-1: none)
    int32_t wait_count = 0;  // number of units of wait_pass
    int32_t npass = 0;       // > 0: a whole small item, passes pass .. pass + npass - 1, every line,
                             // in order inside the block (no cross-block waits)
};

// Status bits the kernel can raise in the error word.
enum : uint32_t { kBatchErrWaitTimeout = 1u, kBatchErrBadLength = 2u };

struct BatchLaunch {
    const WorkUnit *units = nullptr;
    const PassDesc *passes = nullptr;
    uint32_t *counters = nullptr;  // [0] queue head, [1] error word, [2 + p] units of pass p done
    int32_t nunits = 0;
    int32_t npasses = 0;
    const unsigned char *in_base = nullptr;
    unsigned char *out_base = nullptr;
    int32_t fp32 = 1;
    int32_t grid = 0;
};

// Threads per block of the persistent kernel, the most lanes a thread
// carries, and the dynamic LDS a block needs: a 16384-point line (fp32) or
// 512 threads' worth of shorter lines (17 complex values per thread with the
// padding) - 139264 bytes in both precisions.
constexpr int kBatchThreads = 512;
constexpr int batch_threads(bool) { return kBatchThreads; }
constexpr size_t batch_lds_bytes(bool fp32) { return fp32 ? (size_t)17408 * 8 : (size_t)17 * kBatchThreads * 16; }
// Dynamic LDS of a block: the line buffers plus one word for the dequeued unit.
constexpr size_t batch_lds_total(bool fp32) { return batch_lds_bytes(fp32) + 16; }
// Lanes per thread for length L (lines of more than 512 lanes double up).
inline int lanes_per_thread(int L) { return (L / 16 > kBatchThreads) ? (L / 16) / kBatchThreads : 1; }
// Line-group shape for length L: threads per group and lines per group.
inline int group_threads(int L)
{
    const int tpl = (L / 16) / lanes_per_thread(L);
    return tpl < 64 ? 64 : tpl;
}
inline int group_lines(int L) { return group_threads(L) / ((L / 16) / lanes_per_thread(L)); }
// Multi-axis items with at most this many elements per axis pass, summed over
// the passes, run whole inside one block (when their work is also below one
// block's share of the batch).
constexpr long long kFuseMaxElems = 1LL << 19;
// Persistent grid assumed when the options leave it open (one block per
// compute unit of an MI355X).
constexpr int kDefaultGrid = 256;
// Dense (matrix-core) units: lines per unit (as many as the block's LDS
// holds: 64, 32 or 16) and the longest dense line.
inline int dense_unit_lines(int n, int lines, bool fp32)
{
    return dense_rows(n, fp32 ? 4 : 8, batch_lds_bytes(fp32), lines);
}
constexpr int kDenseMaxLine = kDenseMax;

// Zero the counters and launch the persistent kernel on `stream`.
hipError_t launch_batch(const BatchLaunch &b, hipStream_t stream);

// Counters of runs that bring no counter memory of their own: a
// library-owned array of this many 32-bit words per device (256 KiB), kept
// until the process ends.  Every such run on one device shares it.
constexpr int kStaticCounterWords = 1 << 16;
// Device address of that array on the current device (looked up once per
// device, then cached).  Returns the lookup's error, if any.
hipError_t static_counters(uint32_t **ptr);
// Copy one 32-bit word on the device (a one-thread kernel on `stream`).
hipError_t copy_word(uint32_t *dst, const uint32_t *src, hipStream_t stream);

}  // namespace jt
