// Serving loop (include/jt.h, jt_server_*): continuous batching of
// independent transform requests on one GPU.
//
// Requests arrive from any thread with host input and output buffers.  A
// scheduler thread admits them in arrival order while the caller's device
// arena has room for their input and output (HBM-footprint admission),
// copies their inputs in, and launches every admitted request whose axis
// plans are resident as one persistent batch launch (the batch kernel's work
// queue).  Requests that arrive while launches run are admitted as memory
// frees up and go into the next launch, which the GPU picks up as soon as the
// running one drains; input copies, launches and output copies run on
// separate streams, so transfers overlap compute.
//
// Axis plans are cached on the device keyed by (n, a, b, tol), built on host
// threads on a miss, and evicted least-recently-used when the arena needs the
// room and no admitted request uses them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "batch.h"
#include "handle.h"
#include "queue.h"
#include "threads.h"

using jt::fail;
using jt::ok;

namespace {

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// First-fit allocator over [0, size) of the caller's arena, 256-byte granules,
// coalescing on free.
class Arena {
public:
    explicit Arena(size_t size) : size_(size) { free_[0] = size; }
    bool alloc(size_t bytes, size_t &off)
    {
        bytes = align256(std::max<size_t>(bytes, 1));
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            off = it->first;
            const size_t rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[off + bytes] = rest;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = align256(std::max<size_t>(bytes, 1));
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    size_t size() const { return size_; }

private:
    size_t size_, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;
};

struct Key {
    int n;
    int dense;  // 1: the whole matrix (dense matrix-core pass), 0: direct block + FFT terms
    uint64_t a, b, tol;
    bool operator==(const Key &o) const
    {
        return n == o.n && dense == o.dense && a == o.a && b == o.b && tol == o.tol;
    }
};
struct KeyHash {
    size_t operator()(const Key &k) const
    {
        uint64_t h = 1469598103934665603ull;
        for (uint64_t v : {(uint64_t)k.n, (uint64_t)k.dense, k.a, k.b, k.tol}) h = (h ^ v) * 1099511628211ull;
        return (size_t)h;
    }
};

uint64_t bits(double v)
{
    uint64_t u;
    std::memcpy(&u, &v, 8);
    return u;
}

enum PlanState { kPlanning = 0, kHostReady = 1, kResident = 2, kPlanFailed = 3, kEvicted = 4 };

struct PlanEntry {
    Key key{};
    int state = kPlanning;
    jt::AxisPlan ax;                   // after upload only its sizes and section offsets are kept
    std::vector<unsigned char> blob;   // packed image until uploaded
    size_t dev_off = 0, bytes = 0;
    int refs = 0;                      // admitted requests using it
    uint64_t last_use = 0;
    double plan_seconds = 0;
    jt_status err = JT_OK;
    std::string msg;
    hipEvent_t uploaded = nullptr;     // copy of the image finished (host image may be freed)
};

enum ReqState { kQueued = 0, kAdmitted = 1, kRunning = 2, kDone = 3, kFailed = 4 };

struct Request {
    uint64_t id = 0;
    int d = 0;
    int n[3] = {0, 0, 0};
    double a[3] = {0, 0, 0}, b[3] = {0, 0, 0};
    int dir = JT_FORWARD;
    const void *hin = nullptr;
    void *hout = nullptr;
    size_t elems = 0, in_bytes = 0, out_bytes = 0, in_off = 0, out_off = 0;
    PlanEntry *pe[3] = {nullptr, nullptr, nullptr};
    int state = kQueued;
    bool cold = false;
    double t_submit = 0, t_admit = 0, t_launch = 0, t_done = 0, plan_seconds = 0;
    jt_status err = JT_OK;
};

struct Flight {
    std::vector<Request *> reqs;
    std::vector<unsigned char> image;  // host copy of the launch's tables (alive until the copy is done)
    size_t table_off = 0;
    hipEvent_t done = nullptr;         // outputs copied back
    // the launch's error word (bit 0: a wait for a previous pass timed out,
    // bit 1: unsupported length), copied back with the outputs into a slot of
    // the server's pinned ring (a copy into pageable memory would block the
    // scheduler until the flight's outputs are back)
    uint32_t *err_word = nullptr;
    double coeffs = 0;
};

}  // namespace

struct jt_server_s {
    unsigned char *arena_ptr = nullptr;
    Arena arena{0};
    jt_server_options opt{};
    bool fp32 = true;
    jt_dtype tin = JT_F32, tout = JT_F32;
    int device = 0, cus = 1;
    hipStream_t s_in = nullptr, s_out = nullptr, s_comp[2] = {nullptr, nullptr};
    // pinned host words for the flights' error words, used round robin: more
    // slots than flights in flight, and flights retire in launch order, so a
    // slot is free again when its turn comes
    uint32_t *err_ring = nullptr;
    int err_slots = 0;
    uint64_t launches_made = 0;
    int next_comp = 0;

    std::mutex mu;
    std::condition_variable cv_sched, cv_done, cv_plan;
    bool stop = false;
    std::thread scheduler;
    std::vector<std::thread> planners;

    uint64_t next_id = 1, clock = 0;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
    std::deque<Request *> queue;     // arrived, not admitted (arrival order)
    std::vector<Request *> admitted; // inputs copied in, waiting for plans or a launch
    std::deque<Flight> flights;
    std::unordered_map<Key, std::unique_ptr<PlanEntry>, KeyHash> cache;
    std::deque<PlanEntry *> plan_queue;
    jt_server_stats st{};

    jt_server_s(size_t bytes) : arena(bytes) {}

    // ---- plan cache --------------------------------------------------
    // Whether an axis of n points in a d-dimensional request keeps the whole
    // matrix: the crossover differs between one-line passes (1D requests) and
    // passes over many lines.
    bool dense_axis(int n, int d) const
    {
        const int th = (d == 1 && opt.dense_below_1d > 0) ? opt.dense_below_1d : opt.dense_below;
        return n < th && n <= 1024;
    }

    // Entry for (n, dense, a, b, tol), created and queued for planning on a miss.
    PlanEntry *find_or_plan(int n, bool dense, double a, double b, bool &miss)
    {
        Key k{n, dense ? 1 : 0, bits(a), bits(b), bits(opt.tol)};
        auto it = cache.find(k);
        if (it != cache.end()) {
            if (it->second->state == kEvicted) {
                replan(it->second.get());
                miss = true;
            }
            return it->second.get();
        }
        auto pe = std::make_unique<PlanEntry>();
        pe->key = k;
        pe->ax.n = n;
        pe->ax.a = a;
        pe->ax.b = b;
        PlanEntry *p = pe.get();
        cache.emplace(k, std::move(pe));
        plan_queue.push_back(p);
        cv_plan.notify_one();
        miss = true;
        return p;
    }

    void replan(PlanEntry *p)
    {
        p->state = kPlanning;
        plan_queue.push_back(p);
        cv_plan.notify_one();
    }

    void planner_main()
    {
        jt::tl_serial = true;  // host-only work: no HIP calls on these threads
        for (;;) {
            PlanEntry *p = nullptr;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_plan.wait(lk, [&] { return stop || !plan_queue.empty(); });
                if (stop) return;
                p = plan_queue.front();
                plan_queue.pop_front();
            }
            const double t0 = now_s();
            jt::AxisPlan ax;
            std::vector<unsigned char> blob;
            jt_status err = JT_OK;
            std::string msg;
            try {
                jt::PlanOptions po;
                po.dense_below = p->key.dense ? p->ax.n + 1 : 0;
                jt::build_axis(ax, p->ax.n, p->ax.a, p->ax.b, opt.tol, po);
                // only the sections of the server's precision go to the device
                const size_t bytes = jt::layout_axis(ax, 0, fp32 ? jt::kPackF32 : jt::kPackF64);
                blob.assign(bytes, 0);
                jt::pack_axis(ax, blob.data());
            } catch (const std::invalid_argument &e) {
                err = JT_EINVAL;
                msg = e.what();
            } catch (const std::exception &e) {
                err = JT_ENOTCONV;
                msg = e.what();
            }
            const double dt = now_s() - t0;
            {
                std::lock_guard<std::mutex> lk(mu);
                p->plan_seconds = dt;
                if (err != JT_OK) {
                    p->state = kPlanFailed;
                    p->err = err;
                    p->msg = msg;
                } else {
                    p->bytes = blob.size();
                    host_blob_bytes += blob.size();
                    p->blob = std::move(blob);
                    // keep only what the launches need: sizes and section offsets
                    ax.t.clear(); ax.x.clear(); ax.omega.clear(); ax.bins.clear(); ax.binptr.clear();
                    ax.WV.clear(); ax.U.clear(); ax.V.clear();
                    ax.t.shrink_to_fit(); ax.x.shrink_to_fit(); ax.omega.shrink_to_fit(); ax.bins.shrink_to_fit();
                    ax.binptr.shrink_to_fit(); ax.WV.shrink_to_fit(); ax.U.shrink_to_fit(); ax.V.shrink_to_fit();
                    p->ax = std::move(ax);
                    p->state = kHostReady;
                }
            }
            cv_sched.notify_one();
        }
    }

    // Free arena room by dropping a resident plan no admitted request uses,
    // least recently used first.  Its host image, if still held, stays (a
    // later request uploads it again); otherwise the entry goes.
    bool evict_one()
    {
        PlanEntry *victim = nullptr;
        for (auto &kv : cache) {
            PlanEntry *p = kv.second.get();
            if (p->state == kResident && p->refs == 0 && (!victim || p->last_use < victim->last_use)) victim = p;
        }
        if (!victim) return false;
        if (victim->uploaded) {
            (void)hipEventSynchronize(victim->uploaded);
            (void)hipEventDestroy(victim->uploaded);
            victim->uploaded = nullptr;
        }
        arena.release(victim->dev_off, victim->bytes);
        st.plans_evicted++;
        // entries are never deleted (queued requests point at them): without
        // a host image the plan is rebuilt when a request needs it again
        victim->state = victim->blob.empty() ? kEvicted : kHostReady;
        return true;
    }

    bool alloc_evicting(size_t bytes, size_t &off)
    {
        while (!arena.alloc(bytes, off))
            if (!evict_one()) return false;
        return true;
    }

    // ---- scheduler ---------------------------------------------------
    void fail_request(Request *r, jt_status e)
    {
        r->state = kFailed;
        r->err = e;
        r->t_done = now_s();
        st.failed++;
    }

    void release_request(Request *r)
    {
        arena.release(r->in_off, r->in_bytes);
        arena.release(r->out_off, r->out_bytes);
        for (int k = 0; k < r->d; ++k)
            if (r->pe[k]) {
                r->pe[k]->refs--;
                r->pe[k]->last_use = ++clock;
                r->pe[k] = nullptr;  // the entry may be evicted from now on
            }
    }

    bool retire_flights()
    {
        bool any = false;
        while (!flights.empty()) {
            Flight &f = flights.front();
            if (hipEventQuery(f.done) != hipSuccess) break;
            const double t = now_s();
            const bool bad = *f.err_word != 0;
            for (Request *r : f.reqs) {
                release_request(r);
                if (bad) {
                    fail_request(r, JT_EDEVICE);
                    continue;
                }
                r->state = kDone;
                r->t_done = t;
                st.completed++;
            }
            if (!bad) st.coeffs += f.coeffs;
            arena.release(f.table_off, f.image.size());
            (void)hipEventDestroy(f.done);
            flights.pop_front();
            any = true;
        }
        if (any) cv_done.notify_all();
        return any;
    }

    // Host images of resident plans are dropped once their copy is done and
    // the host cache holds more than this.
    static constexpr size_t kHostBlobCap = (size_t)4 << 30;
    size_t host_blob_bytes = 0;

    bool upload(PlanEntry *p)
    {
        size_t off = 0;
        if (!alloc_evicting(p->bytes, off)) return false;
        p->dev_off = off;
        hipError_t e = hipMemcpyAsync(arena_ptr + off, p->blob.data(), p->bytes, hipMemcpyHostToDevice, s_in);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->uploaded, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(p->uploaded, s_in);
        if (e != hipSuccess) {
            arena.release(off, p->bytes);
            p->state = kPlanFailed;
            p->err = JT_EDEVICE;
            p->msg = hipGetErrorString(e);
            return false;
        }
        p->state = kResident;
        p->last_use = ++clock;
        st.plans_cached++;
        return true;
    }

    // Start planning for every arrival's missing axis plans (host only).
    void plan_arrivals()
    {
        for (Request *r : queue)
            if (!r->pe[0]) {
                bool miss = false;
                for (int k = 0; k < r->d; ++k) {
                    r->pe[k] = find_or_plan(r->n[k], dense_axis(r->n[k], r->d), r->a[k], r->b[k], miss);
                    if (miss) st.plan_misses++;
                    else st.plan_hits++;
                    r->cold = r->cold || miss || r->pe[k]->state == kPlanning;
                    miss = false;
                }
            }
    }

    // Admit in arrival order.  The head request needs its axis plans resident
    // (uploaded now, pinned by the request) and room for its input and output;
    // if memory is short it waits for running launches to free some.  Only
    // admitted requests pin device memory, and every admitted request can be
    // launched, so admission never deadlocks; a request that cannot fit even
    // with nothing else resident fails with JT_ENOMEM.
    bool admit()
    {
        bool any = false;
        while (!queue.empty()) {
            Request *r = queue.front();
            bool waiting = false;
            jt_status bad = JT_OK;
            for (int k = 0; k < r->d; ++k) {
                if (r->pe[k]->state == kEvicted) replan(r->pe[k]);
                if (r->pe[k]->state == kPlanFailed) bad = r->pe[k]->err ? r->pe[k]->err : JT_ENOTCONV;
                if (r->pe[k]->state == kPlanning) waiting = true;
            }
            if (bad != JT_OK) {
                queue.pop_front();
                for (int k = 0; k < r->d; ++k) r->pe[k] = nullptr;
                fail_request(r, bad);
                cv_done.notify_all();
                continue;
            }
            if (waiting) break;
            for (int k = 0; k < r->d; ++k) r->pe[k]->refs++;  // pin while allocating
            bool ok_mem = true;
            for (int k = 0; k < r->d && ok_mem; ++k)
                if (r->pe[k]->state == kHostReady) ok_mem = upload(r->pe[k]);
            size_t in_off = 0, out_off = 0;
            if (ok_mem) ok_mem = alloc_evicting(r->in_bytes, in_off);
            if (ok_mem && !alloc_evicting(r->out_bytes, out_off)) {
                arena.release(in_off, r->in_bytes);
                ok_mem = false;
            }
            if (!ok_mem) {
                for (int k = 0; k < r->d; ++k) r->pe[k]->refs--;
                if (flights.empty() && admitted.empty()) {
                    // nothing will free memory: this request can never fit
                    queue.pop_front();
                    for (int k = 0; k < r->d; ++k) r->pe[k] = nullptr;
                    fail_request(r, JT_ENOMEM);
                    cv_done.notify_all();
                    continue;
                }
                break;
            }
            queue.pop_front();
            r->in_off = in_off;
            r->out_off = out_off;
            hipError_t e = hipMemcpyAsync(arena_ptr + in_off, r->hin, r->in_bytes, hipMemcpyHostToDevice, s_in);
            if (e != hipSuccess) {
                release_request(r);
                fail_request(r, JT_EDEVICE);
                cv_done.notify_all();
                continue;
            }
            r->state = kAdmitted;
            r->t_admit = now_s();
            admitted.push_back(r);
            any = true;
        }
        return any;
    }

    // Drop host images of resident plans whose copy finished, beyond the cap.
    void trim_host_images()
    {
        if (host_blob_bytes <= kHostBlobCap) return;
        for (auto &kv : cache) {
            PlanEntry *p = kv.second.get();
            if (host_blob_bytes <= kHostBlobCap) break;
            if (p->state == kResident && !p->blob.empty() && p->uploaded && hipEventQuery(p->uploaded) == hipSuccess) {
                host_blob_bytes -= p->blob.size();
                std::vector<unsigned char>().swap(p->blob);
            }
        }
    }

    bool launch()
    {
        if ((int)flights.size() >= opt.max_inflight) return false;
        std::vector<Request *> take;
        for (size_t i = 0; i < admitted.size() && (int)take.size() < opt.max_batch;) {
            Request *r = admitted[i];
            bool ready = true;  // admission made its plans resident
            for (int k = 0; k < r->d; ++k) ready = ready && r->pe[k]->state == kResident;
            if (ready) {
                take.push_back(r);
                admitted.erase(admitted.begin() + i);
            } else {
                ++i;
            }
        }
        if (take.empty()) return false;
        Flight f;
        f.reqs = take;
        f.err_word = &err_ring[launches_made++ % (uint64_t)err_slots];
        *f.err_word = 0;
        std::vector<jt::QueueItem> items;
        for (Request *r : take) {
            jt::QueueItem it;
            it.d = r->d;
            for (int k = 0; k < r->d; ++k) {
                it.ax[k] = &r->pe[k]->ax;
                it.base[k] = arena_ptr + r->pe[k]->dev_off;
            }
            it.dir = r->dir;
            it.in_off = r->in_off;
            it.out_off = r->out_off;
            items.push_back(it);
            f.coeffs += (double)r->elems;
        }
        jt::WorkQueue q;
        jt_status st_build = jt::guarded([&]() -> jt_status {
            jt::build_queue(items, opt.batch, fp32, tin, tout, q);
            return JT_OK;
        });
        size_t toff = 0;
        if (st_build != JT_OK || !alloc_evicting(q.bytes, toff)) {
            // cannot happen for validated requests unless the arena is exhausted by tables:
            // put them back and retry after completions
            for (Request *r : take) admitted.push_back(r);
            return false;
        }
        jt::resolve_factors(q, items, fp32);
        f.image = jt::queue_image(q);
        f.table_off = toff;
        hipStream_t sc = s_comp[next_comp];
        next_comp ^= 1;
        hipEvent_t ready = nullptr, computed = nullptr;
        hipError_t e = hipMemcpyAsync(arena_ptr + toff, f.image.data(), f.image.size(), hipMemcpyHostToDevice, s_in);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ready, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(ready, s_in);
        if (e == hipSuccess) e = hipStreamWaitEvent(sc, ready, 0);
        jt::BatchLaunch b;
        b.units = reinterpret_cast<const jt::WorkUnit *>(arena_ptr + toff + q.off_units);
        b.passes = reinterpret_cast<const jt::PassDesc *>(arena_ptr + toff + q.off_passes);
        b.counters = reinterpret_cast<uint32_t *>(arena_ptr + toff + q.off_counters);
        b.nunits = (int32_t)q.units.size();
        b.npasses = (int32_t)q.passes.size();
        b.in_base = arena_ptr;
        b.out_base = arena_ptr;
        b.fp32 = fp32 ? 1 : 0;
        b.grid = std::max(1, std::min<int>(opt.batch.grid > 0 ? opt.batch.grid : cus, (int)q.units.size()));
        if (e == hipSuccess) e = jt::launch_batch(b, sc);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&computed, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(computed, sc);
        if (e == hipSuccess) e = hipStreamWaitEvent(s_out, computed, 0);
        for (Request *r : take)
            if (e == hipSuccess)
                e = hipMemcpyAsync(r->hout, arena_ptr + r->out_off, r->out_bytes, hipMemcpyDeviceToHost, s_out);
        if (e == hipSuccess)
            e = hipMemcpyAsync(f.err_word, b.counters + 1, sizeof(uint32_t), hipMemcpyDeviceToHost, s_out);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&f.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(f.done, s_out);
        // the events above only order the streams; the flight's own event marks completion
        if (ready) (void)hipEventDestroy(ready);
        if (computed) (void)hipEventDestroy(computed);
        const double t = now_s();
        if (e != hipSuccess) {
            (void)hipDeviceSynchronize();
            for (Request *r : take) {
                release_request(r);
                fail_request(r, JT_EDEVICE);
            }
            arena.release(toff, f.image.size());
            if (f.done) (void)hipEventDestroy(f.done);
            cv_done.notify_all();
            return false;
        }
        for (Request *r : take) {
            r->state = kRunning;
            r->t_launch = t;
            double ps = 0;
            for (int k = 0; k < r->d; ++k) ps += r->pe[k]->plan_seconds;
            r->plan_seconds = r->cold ? ps : 0;
        }
        st.launches++;
        flights.push_back(std::move(f));
        return true;
    }

    void scheduler_main()
    {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        while (!stop) {
            bool progress = false;
            progress |= retire_flights();
            plan_arrivals();
            progress |= admit();
            progress |= launch();
            trim_host_images();
            if (progress) continue;
            if (flights.empty()) {
                cv_sched.wait_for(lk, std::chrono::milliseconds(2));
            } else {
                // completions are seen by polling the flights' events
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(20));
                lk.lock();
            }
        }
        // shut down: finish what runs, fail what waits
        lk.unlock();
        (void)hipDeviceSynchronize();
        lk.lock();
        retire_flights();
        for (Request *r : admitted) {
            release_request(r);
            fail_request(r, JT_ESTATE);
        }
        admitted.clear();
        for (Request *r : queue) {
            for (int k = 0; k < r->d; ++k) r->pe[k] = nullptr;
            fail_request(r, JT_ESTATE);
        }
        queue.clear();
        cv_done.notify_all();
    }
};

extern "C" {

double jt_clock(void) { return now_s(); }

jt_status jt_server_create(void *dev_arena, size_t bytes, const jt_server_options *opt, jt_server_t *out)
{
    if (!out) return fail(JT_EINVAL, "null output handle");
    *out = nullptr;
    if (!dev_arena || bytes < 4096) return fail(JT_EINVAL, "need a device arena of at least 4 KiB");
    if ((reinterpret_cast<uintptr_t>(dev_arena) & 255u) != 0) return fail(JT_EINVAL, "device arena not 256-byte aligned");
    jt_server_options o{};
    if (opt) o = *opt;
    if (o.tol == 0) o.tol = 1e-7;
    if (!(o.tol >= 1e-14 && o.tol <= 1e-2)) return fail(JT_EINVAL, "tol must lie in [1e-14, 1e-2]");
    if (o.prec != JT_PREC_FP64 && o.prec != JT_PREC_FP32_BULK) return fail(JT_EINVAL, "bad precision");
    if (o.max_batch <= 0) o.max_batch = 256;
    if (o.max_inflight <= 0) o.max_inflight = 2;
    if (o.dense_below <= 0) o.dense_below = 64;
    if (o.dense_below_1d <= 0) o.dense_below_1d = o.dense_below;
    if (o.plan_threads <= 0) {
        const unsigned hw = std::thread::hardware_concurrency();
        o.plan_threads = (int)std::max(1u, std::min(hw ? hw : 1u, 16u));
    }
    if (o.in_dtype != JT_F32 && o.in_dtype != JT_F64) return fail(JT_EINVAL, "bad input dtype");
    if (o.out_dtype != JT_F32 && o.out_dtype != JT_F64) return fail(JT_EINVAL, "bad output dtype");
    return jt::guarded([&]() -> jt_status {
        auto S = std::make_unique<jt_server_s>(bytes);
        S->arena_ptr = static_cast<unsigned char *>(dev_arena);
        S->opt = o;
        S->fp32 = o.prec == JT_PREC_FP32_BULK;
        S->tin = (jt_dtype)o.in_dtype;
        S->tout = (jt_dtype)o.out_dtype;
        S->st.arena_bytes = bytes;
        hipError_t e = hipGetDevice(&S->device);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&S->cus, hipDeviceAttributeMultiprocessorCount, S->device);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->s_in, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->s_out, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->s_comp[0], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->s_comp[1], hipStreamNonBlocking);
        S->err_slots = o.max_inflight + 2;
        if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&S->err_ring), sizeof(uint32_t) * S->err_slots);
        if (e != hipSuccess) {
            for (hipStream_t s : {S->s_in, S->s_out, S->s_comp[0], S->s_comp[1]})
                if (s) (void)hipStreamDestroy(s);
            if (S->err_ring) (void)hipHostFree(S->err_ring);
            return fail(JT_EDEVICE, std::string("server streams: ") + hipGetErrorString(e));
        }
        jt_server_s *raw = S.get();
        for (int i = 0; i < o.plan_threads; ++i) raw->planners.emplace_back([raw] { raw->planner_main(); });
        raw->scheduler = std::thread([raw] { raw->scheduler_main(); });
        *out = S.release();
        return ok();
    });
}

jt_status jt_server_submit(jt_server_t S, int d, const int *n, const double *a, const double *b, jt_direction dir,
                           const void *host_in, void *host_out, uint64_t *ticket)
{
    if (!S || !n || !a || !b || !host_in || !host_out || !ticket) return fail(JT_EINVAL, "null argument");
    if (d < 1 || d > 3) return fail(JT_EINVAL, "d must be 1, 2 or 3");
    if (dir != JT_FORWARD && dir != JT_INVERSE) return fail(JT_EINVAL, "bad direction");
    auto r = std::make_unique<Request>();
    r->d = d;
    size_t elems = 1;
    for (int k = 0; k < d; ++k) {
        if (n[k] < 1 || n[k] > 16384) return fail(JT_EINVAL, "n must be in [1, 16384]");
        if (!(a[k] > -1 && a[k] < 1 && b[k] > -1 && b[k] < 1)) return fail(JT_EINVAL, "a and b must lie in (-1, 1)");
        if (!S->fp32 && n[k] > 8192) return fail(JT_EUNSUPPORTED, "fp64 path supports n <= 8192");
        r->n[k] = n[k];
        r->a[k] = a[k];
        r->b[k] = b[k];
        elems *= (size_t)n[k];
    }
    if (elems >= ((size_t)1 << 31)) return fail(JT_EUNSUPPORTED, "2^31 elements or more");
    r->dir = dir;
    r->hin = host_in;
    r->hout = host_out;
    r->elems = elems;
    r->in_bytes = elems * (S->tin == JT_F64 ? 8 : 4);
    r->out_bytes = elems * (S->tout == JT_F64 ? 8 : 4);
    if (align256(r->in_bytes) + align256(r->out_bytes) > S->arena.size())
        return fail(JT_ENOMEM, "request does not fit in the server's device arena");
    r->t_submit = now_s();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop) return fail(JT_ESTATE, "server is shutting down");
        r->id = S->next_id++;
        *ticket = r->id;
        S->queue.push_back(r.get());
        S->reqs.emplace(r->id, std::move(r));
        S->st.submitted++;
    }
    S->cv_sched.notify_one();
    return ok();
}

static void fill_info(const Request &r, jt_request_info *info)
{
    info->state = r.state;
    info->cold = r.cold ? 1 : 0;
    info->t_submit = r.t_submit;
    info->t_admit = r.t_admit;
    info->t_launch = r.t_launch;
    info->t_done = r.t_done;
    info->plan_seconds = r.plan_seconds;
    info->status = r.err;
}

jt_status jt_server_poll(jt_server_t S, uint64_t ticket, jt_request_info *info)
{
    if (!S || !info) return fail(JT_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return fail(JT_EINVAL, "unknown ticket");
    fill_info(*it->second, info);
    return ok();
}

jt_status jt_server_wait(jt_server_t S, uint64_t ticket, jt_request_info *info)
{
    if (!S) return fail(JT_EINVAL, "null server");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return fail(JT_EINVAL, "unknown ticket");
    Request *r = it->second.get();
    S->cv_done.wait(lk, [&] { return r->state == kDone || r->state == kFailed; });
    if (info) fill_info(*r, info);
    const jt_status e = r->err;
    S->reqs.erase(it);
    if (e != JT_OK) return fail(e, "request failed");
    return ok();
}

jt_status jt_server_stats_get(jt_server_t S, jt_server_stats *out)
{
    if (!S || !out) return fail(JT_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->st;
    out->arena_used = S->arena.used();
    out->arena_peak = S->arena.peak();
    out->queued = (int)S->queue.size();
    out->admitted = (int)S->admitted.size();
    int running = 0;
    for (const Flight &f : S->flights) running += (int)f.reqs.size();
    out->running = running;
    return ok();
}

jt_status jt_server_destroy(jt_server_t S)
{
    if (!S) return ok();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_sched.notify_all();
    S->cv_plan.notify_all();
    if (S->scheduler.joinable()) S->scheduler.join();
    for (auto &t : S->planners) t.join();
    for (auto &kv : S->cache)
        if (kv.second->uploaded) (void)hipEventDestroy(kv.second->uploaded);
    for (hipStream_t s : {S->s_in, S->s_out, S->s_comp[0], S->s_comp[1]})
        if (s) (void)hipStreamDestroy(s);
    if (S->err_ring) (void)hipHostFree(S->err_ring);
    delete S;
    return ok();
}

}  // extern "C"
