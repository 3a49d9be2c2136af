#include "queue.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

namespace jt {

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
    const int NT = batch_threads(fp32);
    const int gt = group_threads(L), lpb = group_lines(L);
    const int groups = NT / gt;
    const int cap = std::max(1, std::min({groups, o.max_split > 0 ? o.max_split : 16, pow2_at_least(std::max(rank, 1))}));
    int S = 1;
    while (S < cap && (groups / S) * lpb > lines) S *= 2;
    const int want = std::max(1, o.min_units);
    while (S < cap && (lines + (groups / S) * lpb - 1) / ((groups / S) * lpb) < want) S *= 2;
    return S;
}

// Modelled cost of one cross-block dependency (a device-wide publish and the
// wait for it), on the scale of the unit costs below: a few microseconds,
// about a small FFT unit's work.
constexpr double kSyncCost = 2e5;

// Shape and modelled cost of one axis pass: its split, lines per unit, unit
// count and the work of one unit (its share of the rank FFTs plus the direct
// block, per line set; a dense unit is one small matrix product).
struct PassShape {
    int S = 1, cap = 1, nu = 0;
    double unit_cost = 0;
};

PassShape pass_shape(const AxisPlan &ax, int lines, const jt_batch_options &opt, bool fp32)
{
    PassShape p;
    const bool dense = ax.nu0 == ax.n;
    p.S = dense ? 1 : choose_split(ax.L, lines, ax.rank, opt, fp32);
    p.cap = dense ? dense_unit_lines(ax.n, lines, fp32)
                  : (batch_threads(fp32) / group_threads(ax.L) / p.S) * group_lines(ax.L);
    p.nu = (lines + p.cap - 1) / p.cap;
    const double per_term = (double)ax.L * std::log2((double)ax.L);
    p.unit_cost = dense ? 2.0 * ax.n * ax.n * p.cap / 8.0
                        : ((ax.rank + p.S - 1) / p.S) * per_term * 5.0 + 2.0 * ax.nu0 * ax.n + 4.0 * ax.n;
    return p;
}

}  // namespace

void build_queue(const std::vector<QueueItem> &items, const jt_batch_options &opt, bool fp32, jt_dtype tin,
                 jt_dtype tout, WorkQueue &q)
{
    q = WorkQueue();
    const size_t isz = tin == JT_F64 ? 8 : 4, osz = tout == JT_F64 ? 8 : 4;
    struct Pending {
        int pass_in_item;
        WorkUnit u;
        double cost;
    };
    std::vector<Pending> pend;
    // A small multi-axis item may run whole inside one block (no cross-block
    // waits or device-wide fences).  That stretches its critical path from
    // one unit per pass to every unit of every pass, so it is done only while
    // the fused item stays within what bounds the batch anyway: one block's
    // share of the total work, or the longest critical path of an item left
    // split (a 1D item is one unit; a split item takes one unit per pass and
    // a cross-block wait between passes).
    // Otherwise a few mid-size items would occupy a few blocks and leave the
    // other compute units idle.
    const int blocks = opt.grid > 0 ? opt.grid : kDefaultGrid;
    std::vector<double> item_cost(items.size(), 0.0), item_path(items.size(), 0.0);
    double total_cost = 0;
    for (size_t i = 0; i < items.size(); ++i) {
        const QueueItem &it = items[i];
        if (it.d < 1 || it.d > 3) continue;  // rejected below
        long long total = 1;
        bool ok = true;
        for (int k = 0; k < it.d; ++k) {
            if (!it.ax[k]) ok = false;
            else total *= it.ax[k]->n;
        }
        if (!ok || total >= (1LL << 31)) continue;
        for (int k = 0; k < it.d; ++k) {
            const PassShape ps = pass_shape(*it.ax[k], (int)(total / it.ax[k]->n), opt, fp32);
            item_cost[i] += ps.unit_cost * ps.nu;
            item_path[i] += ps.unit_cost + (k > 0 ? kSyncCost : 0.0);
        }
        total_cost += item_cost[i];
    }
    double fuse_cost_max = total_cost / blocks;
    for (double p : item_path) fuse_cost_max = std::max(fuse_cost_max, p);
    for (size_t i = 0; i < items.size(); ++i) {
        const QueueItem &it = items[i];
        const std::string who = "item " + std::to_string(i) + ": ";
        if (it.d < 1 || it.d > 3) throw std::invalid_argument(who + "d must be 1, 2 or 3");
        if (it.dir != JT_FORWARD && it.dir != JT_INVERSE) throw std::invalid_argument(who + "bad direction");
        if (it.in_off % isz || it.out_off % osz) throw std::invalid_argument(who + "misaligned offset");
        long long total = 1;
        for (int k = 0; k < it.d; ++k) {
            if (!it.ax[k]) throw std::invalid_argument(who + "missing axis plan");
            total *= it.ax[k]->n;
        }
        if (total >= (1LL << 31)) throw unsupported(who + "2^31 elements or more");
        // a small multi-axis item runs whole inside one block: no cross-block
        // waits, no device-wide fences
        long long item_elems_axes = 0;
        for (int k = 0; k < it.d; ++k) item_elems_axes += total;
        const bool fuse = it.d > 1 && item_elems_axes <= kFuseMaxElems && item_cost[i] <= fuse_cost_max;
        const int first_pid = (int)q.passes.size();
        double fused_cost = 0;
        int prev = -1, prev_units = 0;
        for (int k = it.d - 1, qq = 0; k >= 0; --k, ++qq) {
            const AxisPlan &ax = *it.ax[k];
            if (!fp32 && ax.L > 8192) throw unsupported(who + "fp64 path supports n <= 8192");
            long long stride = 1;
            for (int m = k + 1; m < it.d; ++m) stride *= it.ax[m]->n;
            PassDesc d;
            d.in_off = qq == 0 ? it.in_off : it.out_off;
            d.out_off = it.out_off;
            d.in_from_out = qq == 0 ? 0 : 1;
            d.in_f64 = (qq == 0 ? tin : tout) == JT_F64;
            d.out_f64 = tout == JT_F64;
            d.lines = (int32_t)(total / ax.n);
            d.stride = (int32_t)stride;
            d.n = ax.n;
            d.L = ax.L;
            d.nu0 = ax.nu0;
            d.rank = ax.rank;
            d.max_per_bin = ax.max_per_bin;
            d.forward = it.dir == JT_FORWARD;
            const int pid = (int)q.passes.size();
            const bool dense = ax.nu0 == ax.n;  // every degree in the direct block: matrix-core units
            if (dense && ax.n > kDenseMaxLine) throw unsupported(who + "dense axis longer than the matrix-core pass supports");
            const PassShape ps = pass_shape(ax, d.lines, opt, fp32);
            const int S = ps.S, cap = ps.cap, nu = ps.nu;
            const double c = ps.unit_cost;
            d.split = S;
            d.cap = cap;
            d.publish = (!fuse && k > 0) ? 1 : 0;
            q.passes.push_back(d);
            q.pass_item.push_back((int32_t)i);
            q.pass_axis.push_back(k);
            if (fuse) {
                fused_cost += c * nu;
                continue;
            }
            for (int u = 0; u < nu; ++u) {
                WorkUnit w;
                w.pass = pid;
                w.line0 = u * cap;
                w.nlines = std::min(cap, d.lines - u * cap);
                w.split = S;
                w.wait_pass = prev;
                w.wait_count = prev < 0 ? 0 : prev_units;
                pend.push_back({qq, w, c});
                q.cost += c;
            }
            prev = pid;
            prev_units = nu;
        }
        if (fuse) {
            WorkUnit w;
            w.pass = first_pid;
            w.line0 = 0;
            w.nlines = 0;
            w.split = 1;
            w.npass = it.d;
            pend.push_back({0, w, fused_cost});
            q.cost += fused_cost;
        }
    }
    std::stable_sort(pend.begin(), pend.end(), [](const Pending &x, const Pending &y) {
        if (x.pass_in_item != y.pass_in_item) return x.pass_in_item < y.pass_in_item;
        return x.cost > y.cost;
    });
    if (pend.size() >= (size_t)1 << 30) throw unsupported("too many work units");
    q.units.reserve(pend.size());
    for (const Pending &p : pend) q.units.push_back(p.u);
    q.off_units = 0;
    q.off_passes = align256(q.units.size() * sizeof(WorkUnit));
    q.off_counters = q.off_passes + align256(q.passes.size() * sizeof(PassDesc));
    q.bytes = q.off_counters + align256((2 + q.passes.size()) * sizeof(uint32_t));
}

void resolve_factors(WorkQueue &q, const std::vector<QueueItem> &items, bool fp32)
{
    for (size_t p = 0; p < q.passes.size(); ++p) {
        const QueueItem &it = items[q.pass_item[p]];
        const int k = q.pass_axis[p];
        const AxisPlan &ax = *it.ax[k];
        const unsigned char *d = it.base[k];
        PassDesc &pd = q.passes[p];
        pd.tw = d + (fp32 ? ax.off_tw32 : ax.off_tw64);
        pd.bins = reinterpret_cast<const int *>(d + ax.off_bins);
        pd.binptr = reinterpret_cast<const int *>(d + ax.off_binptr);
        pd.wv = d + (fp32 ? ax.off_wv32 : ax.off_wv64);
        pd.u = d + (fp32 ? ax.off_u32 : ax.off_u64);
        pd.v = d + (fp32 ? ax.off_v32 : ax.off_v64);
    }
}

std::vector<unsigned char> queue_image(const WorkQueue &q)
{
    std::vector<unsigned char> img(q.bytes, 0);
    std::memcpy(img.data() + q.off_units, q.units.data(), q.units.size() * sizeof(WorkUnit));
    std::memcpy(img.data() + q.off_passes, q.passes.data(), q.passes.size() * sizeof(PassDesc));
    return img;
}

}  // namespace jt
