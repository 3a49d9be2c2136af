// C ABI of the batched form (include/jt.h): many plans at once, and the
// work-unit queue of the persistent batch kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "batch.h"
#include "handle.h"
#include "queue.h"
#include "threads.h"

using jt::fail;
using jt::ok;

struct jt_batch_s {
    std::vector<jt_plan_t> plans;
    std::vector<jt::QueueItem> items;
    jt::WorkQueue q;
    bool fp32 = true;
    jt_dtype tin = JT_F64, tout = JT_F64;
    jt_batch_options opt{};
    unsigned char *dev = nullptr;
    int grid = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;

    ~jt_batch_s()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};


extern "C" {

jt_status jt_plan_many(int count, const int *dims, const int *n, const double *a, const double *b, double tol,
                       const jt_plan_options *opt, jt_plan_t *plans)
{
    if (count < 0) return fail(JT_EINVAL, "negative count");
    if (count > 0 && (!dims || !n || !a || !b || !plans)) return fail(JT_EINVAL, "null argument");
    std::vector<size_t> start(count + 1, 0);
    for (int i = 0; i < count; ++i) {
        if (dims[i] < 1 || dims[i] > 3) return fail(JT_EINVAL, "item " + std::to_string(i) + ": d must be 1, 2 or 3");
        start[i + 1] = start[i] + dims[i];
    }
    std::vector<jt_plan_t> out(count, nullptr);
    std::mutex mu;
    jt_status first = JT_OK;
    std::string first_msg;
    int first_item = count;
    std::atomic<int> next(0);
    auto work = [&]() {
        jt::tl_serial = true;  // one plan per host thread
        for (;;) {
            const int i = next.fetch_add(1);
            if (i >= count) break;
            jt_plan_t p = nullptr;
            jt_status st = jt::guarded([&]() -> jt_status {
                p = jt::build_plan(dims[i], n + start[i], a + start[i], b + start[i], tol,
                                   jt::plan_options(opt ? opt + i : nullptr));
                return JT_OK;
            });
            if (st != JT_OK) {
                std::lock_guard<std::mutex> g(mu);
                if (i < first_item) {
                    first_item = i;
                    first = st;
                    first_msg = jt::g_err;
                }
            }
            out[i] = p;
        }
        jt::tl_serial = false;
    };
    unsigned hw = std::thread::hardware_concurrency();
    const int nt = std::max(1, std::min<int>(count, (int)std::min<unsigned>(hw ? hw : 1, 16)));
    std::vector<std::thread> th;
    for (int k = 1; k < nt; ++k) th.emplace_back(work);
    work();
    for (auto &t : th) t.join();
    if (first != JT_OK) {
        for (jt_plan_t p : out) delete p;
        return fail(first, "item " + std::to_string(first_item) + ": " + first_msg);
    }
    for (int i = 0; i < count; ++i) plans[i] = out[i];
    return ok();
}

jt_status jt_batch_create(int count, const jt_plan_t *plans, const int *dirs, const uint64_t *in_off,
                          const uint64_t *out_off, jt_dtype tin, jt_dtype tout, jt_prec prec,
                          const jt_batch_options *opt, jt_batch_t *batch)
{
    if (!batch) return fail(JT_EINVAL, "null output handle");
    *batch = nullptr;
    if (count < 1) return fail(JT_EINVAL, "a batch needs at least one item");
    if (!plans || !dirs || !in_off || !out_off) return fail(JT_EINVAL, "null argument");
    if ((tin != JT_F64 && tin != JT_F32) || (tout != JT_F64 && tout != JT_F32)) return fail(JT_EINVAL, "bad dtype");
    if (prec != JT_PREC_FP64 && prec != JT_PREC_FP32_BULK) return fail(JT_EINVAL, "bad precision");
    return jt::guarded([&]() -> jt_status {
        auto *B = new jt_batch_s();
        std::unique_ptr<jt_batch_s> hold(B);
        B->fp32 = (prec == JT_PREC_FP32_BULK);
        B->tin = tin;
        B->tout = tout;
        if (opt) B->opt = *opt;
        if (B->opt.max_split < 0 || B->opt.min_units < 0 || B->opt.grid < 0) return fail(JT_EINVAL, "negative option");
        for (int i = 0; i < count; ++i) {
            jt_plan_t p = plans[i];
            if (!p) return fail(JT_EINVAL, "item " + std::to_string(i) + ": null plan");
            if (dirs[i] != JT_FORWARD && dirs[i] != JT_INVERSE)
                return fail(JT_EINVAL, "item " + std::to_string(i) + ": bad direction");
            if (dirs[i] == JT_INVERSE && (p->ax[0].points || p->ax[0].kind == 2))
                return fail(JT_EUNSUPPORTED, "item " + std::to_string(i) + ": a plan at given points or of the "
                                             "second kind has only the forward transform");
            jt::QueueItem it;
            it.d = p->d;
            for (int k = 0; k < p->d; ++k) it.ax[k] = &p->ax[k];
            it.dir = dirs[i];
            it.in_off = in_off[i];
            it.out_off = out_off[i];
            B->plans.push_back(p);
            B->items.push_back(it);
        }
        jt::build_queue(B->items, B->opt, B->fp32, tin, tout, B->q);
        *batch = hold.release();
        return ok();
    });
}

jt_status jt_batch_destroy(jt_batch_t batch)
{
    delete batch;
    return ok();
}

jt_status jt_batch_info_get(jt_batch_t batch, jt_batch_info *info)
{
    if (!batch || !info) return fail(JT_EINVAL, "null argument");
    info->units = (int)batch->q.units.size();
    info->passes = (int)batch->q.passes.size();
    info->grid = batch->grid;
    info->threads = jt::batch_threads(batch->fp32);
    info->lds_bytes = jt::batch_lds_total(batch->fp32);
    info->cost = batch->q.cost;
    return ok();
}

jt_status jt_batch_tables(jt_batch_t batch, int32_t *units, int32_t *passes)
{
    if (!batch) return fail(JT_EINVAL, "null batch");
    const jt::WorkQueue &q = batch->q;
    if (units)
        for (size_t i = 0; i < q.units.size(); ++i) {
            const jt::WorkUnit &w = q.units[i];
            const int32_t row[7] = {w.pass, w.line0, w.nlines, w.split, w.wait_pass, w.wait_count, w.npass};
            std::memcpy(units + 7 * i, row, sizeof(row));
        }
    if (passes) {
        std::vector<int32_t> nunits(q.passes.size(), 0);
        for (const jt::WorkUnit &w : q.units) nunits[w.pass]++;
        for (size_t p = 0; p < q.passes.size(); ++p) {
            passes[4 * p] = q.pass_item[p];
            passes[4 * p + 1] = q.pass_axis[p];
            passes[4 * p + 2] = q.passes[p].lines;
            passes[4 * p + 3] = nunits[p];
        }
    }
    return ok();
}

jt_status jt_batch_device_bytes(jt_batch_t batch, size_t *bytes)
{
    if (!batch || !bytes) return fail(JT_EINVAL, "null argument");
    *bytes = batch->q.bytes;
    return ok();
}

jt_status jt_batch_bind(jt_batch_t batch, void *dev_buf, size_t bytes, void *stream)
{
    if (!batch || !dev_buf) return fail(JT_EINVAL, "null argument");
    if (bytes < batch->q.bytes) return fail(JT_ENOMEM, "device buffer smaller than jt_batch_device_bytes");
    if ((reinterpret_cast<uintptr_t>(dev_buf) & 255u) != 0) return fail(JT_EINVAL, "device buffer not 256-byte aligned");
    // the factor pointers of every pass live inside its plan's bound image
    for (size_t i = 0; i < batch->items.size(); ++i) {
        if (!batch->plans[i]->dev) return fail(JT_ESTATE, "item " + std::to_string(i) + ": plan is not bound");
        for (int k = 0; k < batch->items[i].d; ++k) batch->items[i].base[k] = batch->plans[i]->dev;
    }
    jt::resolve_factors(batch->q, batch->items, batch->fp32);
    std::vector<unsigned char> img = jt::queue_image(batch->q);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(dev_buf, img.data(), batch->q.bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(JT_EDEVICE, std::string("batch table copy: ") + hipGetErrorString(e));
    int dev = 0, cus = 0;
    e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess || cus <= 0) return fail(JT_EDEVICE, "cannot query the compute-unit count");
    // one block per compute unit: the dynamic LDS (139 KB) admits no second one
    const int want = batch->opt.grid > 0 ? batch->opt.grid : cus;
    batch->grid = std::max(1, std::min<int>(want, (int)batch->q.units.size()));
    batch->dev = static_cast<unsigned char *>(dev_buf);
    return ok();
}

static jt::BatchLaunch launch_args(jt_batch_t batch, const void *in_base, void *out_base)
{
    jt::BatchLaunch b;
    b.units = reinterpret_cast<const jt::WorkUnit *>(batch->dev + batch->q.off_units);
    b.passes = reinterpret_cast<const jt::PassDesc *>(batch->dev + batch->q.off_passes);
    b.counters = reinterpret_cast<uint32_t *>(batch->dev + batch->q.off_counters);
    b.nunits = (int32_t)batch->q.units.size();
    b.npasses = (int32_t)batch->q.passes.size();
    b.in_base = static_cast<const unsigned char *>(in_base);
    b.out_base = static_cast<unsigned char *>(out_base);
    b.fp32 = batch->fp32 ? 1 : 0;
    b.grid = batch->grid;
    return b;
}

jt_status jt_batch_run(jt_batch_t batch, const void *in_base, void *out_base, void *stream)
{
    if (!batch || !in_base || !out_base) return fail(JT_EINVAL, "null argument");
    if (!batch->dev) return fail(JT_ESTATE, "batch is not bound (jt_batch_bind)");
    if (in_base == out_base && batch->tin != batch->tout) return fail(JT_EINVAL, "in-place batch needs equal dtypes");
    hipError_t e = jt::launch_batch(launch_args(batch, in_base, out_base), reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail(JT_EDEVICE, std::string("batch launch failed: ") + hipGetErrorString(e));
    return ok();
}

jt_status jt_batch_run_static(jt_batch_t batch, const void *in_base, void *out_base, void *stream)
{
    if (!batch || !in_base || !out_base) return fail(JT_EINVAL, "null argument");
    const long long words = 2LL + (long long)batch->q.passes.size();
    if (words > jt::kStaticCounterWords)
        return fail(JT_EINVAL, "batch has " + std::to_string(batch->q.passes.size()) +
                                   " axis passes; the library's counter array holds at most " +
                                   std::to_string(jt::kStaticCounterWords - 2));
    if (!batch->dev) return fail(JT_ESTATE, "batch is not bound (jt_batch_bind)");
    if (in_base == out_base && batch->tin != batch->tout) return fail(JT_EINVAL, "in-place batch needs equal dtypes");
    if (batch->q.units.empty()) return ok();
    uint32_t *ctr = nullptr;
    hipError_t e = jt::static_counters(&ctr);
    if (e != hipSuccess)
        return fail(JT_EDEVICE, std::string("cannot find the device counter array: ") + hipGetErrorString(e));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    jt::BatchLaunch b = launch_args(batch, in_base, out_base);
    b.counters = ctr;
    e = jt::launch_batch(b, s);
    // the run's error word goes to the batch's own slot, where jt_batch_errors reads it
    if (e == hipSuccess)
        e = jt::copy_word(reinterpret_cast<uint32_t *>(batch->dev + batch->q.off_counters) + 1, ctr + 1, s);
    if (e != hipSuccess) return fail(JT_EDEVICE, std::string("batch launch failed: ") + hipGetErrorString(e));
    return ok();
}

jt_status jt_batch_capture(jt_batch_t batch, const void *in_base, void *out_base)
{
    if (!batch || !in_base || !out_base) return fail(JT_EINVAL, "null argument");
    if (!batch->dev) return fail(JT_ESTATE, "batch is not bound (jt_batch_bind)");
    if (in_base == out_base && batch->tin != batch->tout) return fail(JT_EINVAL, "in-place batch needs equal dtypes");
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return fail(JT_EDEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));
    hipGraph_t g = nullptr;
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t le = jt::launch_batch(launch_args(batch, in_base, out_base), cs);
        e = hipStreamEndCapture(cs, &g);
        if (le != hipSuccess) e = le;
    }
    hipGraphExec_t x = nullptr;
    if (e == hipSuccess) e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(JT_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    }
    if (batch->exec) (void)hipGraphExecDestroy(batch->exec);
    if (batch->graph) (void)hipGraphDestroy(batch->graph);
    batch->graph = g;
    batch->exec = x;
    return ok();
}

jt_status jt_batch_replay(jt_batch_t batch, void *stream)
{
    if (!batch) return fail(JT_EINVAL, "null batch");
    if (!batch->exec) return fail(JT_ESTATE, "no captured graph (jt_batch_capture)");
    hipError_t e = hipGraphLaunch(batch->exec, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail(JT_EDEVICE, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
    return ok();
}

jt_status jt_batch_errors(jt_batch_t batch, void *stream, uint32_t *flags)
{
    if (!batch || !flags) return fail(JT_EINVAL, "null argument");
    if (!batch->dev) return fail(JT_ESTATE, "batch is not bound (jt_batch_bind)");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    uint32_t v = 0;
    hipError_t e = hipMemcpyAsync(&v, batch->dev + batch->q.off_counters + sizeof(uint32_t), sizeof(v),
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(JT_EDEVICE, std::string("error word copy: ") + hipGetErrorString(e));
    *flags = v;
    return ok();
}

}  // extern "C"
