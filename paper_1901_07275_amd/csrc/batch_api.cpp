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
#include "threads.h"

using jt::fail;
using jt::ok;

struct jt_batch_s {
    struct Item {
        jt_plan_t plan;
        int dir;
        uint64_t in_off, out_off;
    };
    std::vector<Item> items;
    std::vector<jt::PassDesc> passes;
    std::vector<jt::WorkUnit> units;
    std::vector<int32_t> pass_item, pass_axis;
    bool fp32 = true;
    jt_dtype tin = JT_F64, tout = JT_F64;
    jt_batch_options opt{};
    double cost = 0;
    size_t off_units = 0, off_passes = 0, off_counters = 0, bytes = 0;
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

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int pow2_at_least(int v)
{
    int p = 1;
    while (p < v) p *= 2;
    return p;
}

// Split S for a pass: S groups share each line set, so a unit holds
// (groups / S) * LPB lines.  Lines beyond what the pass has would leave
// groups idle, so S grows until the unit's capacity fits the lines (a single
// line gets every group); it never exceeds the groups, the rank (rounded up to
// a power of two) or the option's cap.  min_units raises S further while the
// pass has fewer units than asked for.
int choose_split(int L, int lines, int rank, const jt_batch_options &o, bool fp32)
{
    const int NT = jt::batch_threads(fp32);
    const int gt = jt::group_threads(L), lpb = jt::group_lines(L);
    const int groups = NT / gt;
    const int cap = std::max(1, std::min({groups, o.max_split > 0 ? o.max_split : 16, pow2_at_least(std::max(rank, 1))}));
    int S = 1;
    while (S < cap && (groups / S) * lpb > lines) S *= 2;
    const int want = std::max(1, o.min_units);
    while (S < cap && (lines + (groups / S) * lpb - 1) / ((groups / S) * lpb) < want) S *= 2;
    return S;
}

}  // namespace

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
        const size_t isz = tin == JT_F64 ? 8 : 4, osz = tout == JT_F64 ? 8 : 4;
        struct Pending {
            int pass_in_item;
            jt::WorkUnit u;
            double cost;
        };
        std::vector<Pending> pend;
        for (int i = 0; i < count; ++i) {
            jt_plan_t p = plans[i];
            if (!p) return fail(JT_EINVAL, "item " + std::to_string(i) + ": null plan");
            if (dirs[i] != JT_FORWARD && dirs[i] != JT_INVERSE) return fail(JT_EINVAL, "item " + std::to_string(i) + ": bad direction");
            if (in_off[i] % isz || out_off[i] % osz) return fail(JT_EINVAL, "item " + std::to_string(i) + ": misaligned offset");
            long long total = 1;
            for (int k = 0; k < p->d; ++k) total *= p->ax[k].n;
            if (total >= (1LL << 31)) return fail(JT_EUNSUPPORTED, "item " + std::to_string(i) + ": 2^31 elements or more");
            B->items.push_back({p, dirs[i], in_off[i], out_off[i]});
            // axes d-1 .. 0; the first pass reads the input, later ones work in place on the output
            int prev = -1, prev_units = 0;
            for (int k = p->d - 1, q = 0; k >= 0; --k, ++q) {
                const jt::AxisPlan &ax = p->ax[k];
                if (!B->fp32 && ax.L > 8192) return fail(JT_EUNSUPPORTED, "item " + std::to_string(i) + ": fp64 path supports n <= 8192");
                long long stride = 1;
                for (int m = k + 1; m < p->d; ++m) stride *= p->ax[m].n;
                jt::PassDesc d;
                d.in_off = q == 0 ? in_off[i] : out_off[i];
                d.out_off = out_off[i];
                d.in_from_out = q == 0 ? 0 : 1;
                d.in_f64 = (q == 0 ? tin : tout) == JT_F64;
                d.out_f64 = tout == JT_F64;
                d.lines = (int32_t)(total / ax.n);
                d.stride = (int32_t)stride;
                d.n = ax.n;
                d.L = ax.L;
                d.nu0 = ax.nu0;
                d.rank = ax.rank;
                d.max_per_bin = ax.max_per_bin;
                d.forward = dirs[i] == JT_FORWARD;
                const int pid = (int)B->passes.size();
                B->passes.push_back(d);
                B->pass_item.push_back(i);
                B->pass_axis.push_back(k);
                const int S = choose_split(ax.L, d.lines, ax.rank, B->opt, B->fp32);
                const int cap = (jt::batch_threads(B->fp32) / jt::group_threads(ax.L) / S) * jt::group_lines(ax.L);
                const int nu = (d.lines + cap - 1) / cap;
                // work of one unit: its share of the rank FFTs plus the direct block, per line set
                const double per_term = (double)ax.L * std::log2((double)ax.L);
                const double c = ((ax.rank + S - 1) / S) * per_term * 5.0 + 2.0 * ax.nu0 * ax.n + 4.0 * ax.n;
                for (int u = 0; u < nu; ++u) {
                    jt::WorkUnit w;
                    w.pass = pid;
                    w.line0 = u * cap;
                    w.nlines = std::min(cap, d.lines - u * cap);
                    w.split = S;
                    w.wait_pass = prev;
                    w.wait_count = prev < 0 ? 0 : prev_units;
                    pend.push_back({q, w, c});
                    B->cost += c;
                }
                prev = pid;
                prev_units = nu;
            }
        }
        // queue order: every first pass, then every second pass, then third;
        // within a rank the costliest units first (longest-processing-time rule)
        std::stable_sort(pend.begin(), pend.end(), [](const Pending &x, const Pending &y) {
            if (x.pass_in_item != y.pass_in_item) return x.pass_in_item < y.pass_in_item;
            return x.cost > y.cost;
        });
        if (pend.size() >= (size_t)1 << 30) return fail(JT_EUNSUPPORTED, "too many work units");
        for (const Pending &p : pend) B->units.push_back(p.u);
        B->off_units = 0;
        B->off_passes = align256(B->units.size() * sizeof(jt::WorkUnit));
        B->off_counters = B->off_passes + align256(B->passes.size() * sizeof(jt::PassDesc));
        B->bytes = B->off_counters + align256((2 + B->passes.size()) * sizeof(uint32_t));
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
    info->units = (int)batch->units.size();
    info->passes = (int)batch->passes.size();
    info->grid = batch->grid;
    info->threads = jt::batch_threads(batch->fp32);
    info->lds_bytes = jt::batch_lds_bytes(batch->fp32);
    info->cost = batch->cost;
    return ok();
}

jt_status jt_batch_tables(jt_batch_t batch, int32_t *units, int32_t *passes)
{
    if (!batch) return fail(JT_EINVAL, "null batch");
    if (units)
        for (size_t i = 0; i < batch->units.size(); ++i) {
            const jt::WorkUnit &w = batch->units[i];
            const int32_t row[6] = {w.pass, w.line0, w.nlines, w.split, w.wait_pass, w.wait_count};
            std::memcpy(units + 6 * i, row, sizeof(row));
        }
    if (passes) {
        std::vector<int32_t> nunits(batch->passes.size(), 0);
        for (const jt::WorkUnit &w : batch->units) nunits[w.pass]++;
        for (size_t p = 0; p < batch->passes.size(); ++p) {
            passes[4 * p] = batch->pass_item[p];
            passes[4 * p + 1] = batch->pass_axis[p];
            passes[4 * p + 2] = batch->passes[p].lines;
            passes[4 * p + 3] = nunits[p];
        }
    }
    return ok();
}

jt_status jt_batch_device_bytes(jt_batch_t batch, size_t *bytes)
{
    if (!batch || !bytes) return fail(JT_EINVAL, "null argument");
    *bytes = batch->bytes;
    return ok();
}

jt_status jt_batch_bind(jt_batch_t batch, void *dev_buf, size_t bytes, void *stream)
{
    if (!batch || !dev_buf) return fail(JT_EINVAL, "null argument");
    if (bytes < batch->bytes) return fail(JT_ENOMEM, "device buffer smaller than jt_batch_device_bytes");
    if ((reinterpret_cast<uintptr_t>(dev_buf) & 255u) != 0) return fail(JT_EINVAL, "device buffer not 256-byte aligned");
    // resolve the factor pointers of every pass inside its plan's bound image
    for (size_t p = 0; p < batch->passes.size(); ++p) {
        const jt_plan_t plan = batch->items[batch->pass_item[p]].plan;
        if (!plan->dev) return fail(JT_ESTATE, "item " + std::to_string(batch->pass_item[p]) + ": plan is not bound");
        const jt::AxisPlan &ax = plan->ax[batch->pass_axis[p]];
        const bool f32 = batch->fp32;
        unsigned char *d = plan->dev;
        jt::PassDesc &pd = batch->passes[p];
        pd.tw = d + (f32 ? ax.off_tw32 : ax.off_tw64);
        pd.bins = reinterpret_cast<const int *>(d + ax.off_bins);
        pd.binptr = reinterpret_cast<const int *>(d + ax.off_binptr);
        pd.wv = d + (f32 ? ax.off_wv32 : ax.off_wv64);
        pd.wvt = d + (f32 ? ax.off_wvt32 : ax.off_wvt64);
        pd.u = d + (f32 ? ax.off_u32 : ax.off_u64);
        pd.v = d + (f32 ? ax.off_v32 : ax.off_v64);
    }
    std::vector<unsigned char> img(batch->bytes, 0);
    std::memcpy(img.data() + batch->off_units, batch->units.data(), batch->units.size() * sizeof(jt::WorkUnit));
    std::memcpy(img.data() + batch->off_passes, batch->passes.data(), batch->passes.size() * sizeof(jt::PassDesc));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(dev_buf, img.data(), batch->bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(JT_EDEVICE, std::string("batch table copy: ") + hipGetErrorString(e));
    int dev = 0, cus = 0;
    e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess || cus <= 0) return fail(JT_EDEVICE, "cannot query the compute-unit count");
    // one block per compute unit: the dynamic LDS (139 KB) admits no second one
    const int want = batch->opt.grid > 0 ? batch->opt.grid : cus;
    batch->grid = std::max(1, std::min<int>(want, (int)batch->units.size()));
    batch->dev = static_cast<unsigned char *>(dev_buf);
    return ok();
}

static jt::BatchLaunch launch_args(jt_batch_t batch, const void *in_base, void *out_base)
{
    jt::BatchLaunch b;
    b.units = reinterpret_cast<const jt::WorkUnit *>(batch->dev + batch->off_units);
    b.passes = reinterpret_cast<const jt::PassDesc *>(batch->dev + batch->off_passes);
    b.counters = reinterpret_cast<uint32_t *>(batch->dev + batch->off_counters);
    b.nunits = (int32_t)batch->units.size();
    b.npasses = (int32_t)batch->passes.size();
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
    hipError_t e = hipMemcpyAsync(&v, batch->dev + batch->off_counters + sizeof(uint32_t), sizeof(v),
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(JT_EDEVICE, std::string("error word copy: ") + hipGetErrorString(e));
    *flags = v;
    return ok();
}

}  // extern "C"
