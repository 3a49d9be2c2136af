// C ABI (include/jt.h) on top of the host plan and the HIP axis-pass kernels.
#include "jt.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <exception>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "handle.h"
#include "launch.h"
#include "plan.h"

namespace {

using jt::fail;
using jt::ok;
using jt::guarded;
using jt::g_err;

jt_status check_axis(jt_plan_t p, int axis)
{
    if (!p) return fail(JT_EINVAL, "null plan");
    if (axis < 0 || axis >= p->d) return fail(JT_EINVAL, "axis out of range");
    return JT_OK;
}

long long total_elems(const jt_plan_s *p)
{
    long long t = 1;
    for (int i = 0; i < p->d; ++i) t *= p->ax[i].n;
    return t;
}

jt_status run_axis(jt_plan_t p, int axis, bool forward, const void *in, jt_dtype tin, void *out,
                   jt_dtype tout, jt_prec prec, void *stream)
{
    if (!p) return fail(JT_EINVAL, "null plan");
    if (axis < 0 || axis >= p->d) return fail(JT_EINVAL, "axis out of range");
    if (!p->dev) return fail(JT_ESTATE, "plan is not bound to device memory (jt_plan_bind)");
    if (!in || !out) return fail(JT_EINVAL, "null tensor pointer");
    if ((tin != JT_F64 && tin != JT_F32) || (tout != JT_F64 && tout != JT_F32))
        return fail(JT_EINVAL, "bad dtype");
    if (prec != JT_PREC_FP64 && prec != JT_PREC_FP32_BULK) return fail(JT_EINVAL, "bad precision");
    if (in == out && tin != tout) return fail(JT_EINVAL, "in-place pass needs equal input and output dtypes");
    const jt::AxisPlan &ax = p->ax[axis];
    if ((ax.points || ax.kind == 2) && !forward)
        return fail(JT_EUNSUPPORTED, "a plan at given points or of the second kind has only the forward "
                                     "transform (its matrix is not orthogonal: the inverse is a solve, "
                                     "not the transpose)");
    long long stride = 1;
    for (int i = axis + 1; i < p->d; ++i) stride *= p->ax[i].n;
    jt::AxisLaunch a;
    a.in = in;
    a.out = out;
    a.in_f64 = (tin == JT_F64);
    a.out_f64 = (tout == JT_F64);
    a.lines = total_elems(p) / ax.n;
    a.stride = stride;
    a.n = ax.n;
    a.L = ax.L;
    a.nu0 = ax.nu0;
    a.rank = ax.rank;
    a.max_per_bin = ax.max_per_bin;
    a.forward = forward ? 1 : 0;
    a.fp32 = (prec == JT_PREC_FP32_BULK);
    const bool f32 = a.fp32;
    unsigned char *d = p->dev;
    a.tw = d + (f32 ? ax.off_tw32 : ax.off_tw64);
    a.bins = reinterpret_cast<const int *>(d + ax.off_bins);
    a.binptr = reinterpret_cast<const int *>(d + ax.off_binptr);
    a.wv = d + (f32 ? ax.off_wv32 : ax.off_wv64);
    a.u = d + (f32 ? ax.off_u32 : ax.off_u64);
    a.v = d + (f32 ? ax.off_v32 : ax.off_v64);
    if (!f32 && ax.L > 8192) return fail(JT_EUNSUPPORTED, "fp64 path supports n <= 8192");
    if (total_elems(p) >= (1LL << 31)) return fail(JT_EUNSUPPORTED, "tensors must hold fewer than 2^31 elements");
    hipError_t e = jt::launch_axis(a, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail(JT_EDEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
    return JT_OK;
}

jt_status run_all(jt_plan_t p, bool forward, const void *in, jt_dtype tin, void *out, jt_dtype tout,
                  jt_prec prec, void *stream)
{
    if (!p) return fail(JT_EINVAL, "null plan");
    if (in == out && tin != tout) return fail(JT_EINVAL, "in-place transform needs equal dtypes");
    // first pass reads the input, the others work in place on the output
    for (int i = p->d - 1, first = 1; i >= 0; --i, first = 0) {
        jt_status st = first ? run_axis(p, i, forward, in, tin, out, tout, prec, stream)
                             : run_axis(p, i, forward, out, tout, out, tout, prec, stream);
        if (st != JT_OK) return st;
    }
    return ok();
}

}  // namespace

namespace jt {

PlanOptions plan_options(const jt_plan_options *opt)
{
    PlanOptions po;
    if (opt) {
        if (opt->nu0 > 0) po.nu0 = opt->nu0;
        if (opt->dense_below >= 0) po.dense_below = opt->dense_below;
        if (opt->oversample > 0) po.oversample = opt->oversample;
        if (opt->iterations > 0) po.iterations = opt->iterations;
        po.seed = opt->seed;
        if (opt->kind != 0) po.kind = opt->kind;
        po.planner = opt->planner;
    }
    return po;
}

jt_plan_s *build_plan(int d, const int *n, const double *a, const double *b, double tol, const PlanOptions &po,
                      const double *t)
{
    if (d < 1 || d > 3) throw std::invalid_argument("d must be 1, 2 or 3");
    jt_plan_s *p = new jt_plan_s();
    try {
        p->d = d;
        size_t off = 0;
        size_t t0 = 0;
        for (int i = 0; i < d; ++i) {
            if (t) {
                build_axis_points(p->ax[i], n[i], t + t0, a[i], b[i], tol, po);
                t0 += (size_t)std::max(n[i], 0);
            } else {
                build_axis(p->ax[i], n[i], a[i], b[i], tol, po);
            }
            off = layout_axis(p->ax[i], off);
        }
        p->dev_bytes = off;
        p->blob.assign(off, 0);
        for (int i = 0; i < d; ++i) pack_axis(p->ax[i], p->blob.data());
    } catch (...) {
        delete p;
        throw;
    }
    return p;
}

}  // namespace jt

extern "C" {

int jt_version(void) { return 124; }

const char *jt_last_error(void) { return g_err.c_str(); }

jt_status jt_plan_ex(int d, const int *n, const double *a, const double *b, double tol,
                     const jt_plan_options *opt, jt_plan_t *out)
{
    return guarded([&]() -> jt_status {
        if (!out) return fail(JT_EINVAL, "null output handle");
        *out = nullptr;
        if (d < 1 || d > 3) return fail(JT_EINVAL, "d must be 1, 2 or 3");
        if (!n || !a || !b) return fail(JT_EINVAL, "null parameter array");
        *out = jt::build_plan(d, n, a, b, tol, jt::plan_options(opt));
        return ok();
    });
}

jt_status jt_plan_points(int d, const int *n, const double *t, const double *a, const double *b, double tol,
                         const jt_plan_options *opt, jt_plan_t *out)
{
    return guarded([&]() -> jt_status {
        if (!out) return fail(JT_EINVAL, "null output handle");
        *out = nullptr;
        if (d < 1 || d > 3) return fail(JT_EINVAL, "d must be 1, 2 or 3");
        if (!n || !a || !b || !t) return fail(JT_EINVAL, "null parameter array");
        *out = jt::build_plan(d, n, a, b, tol, jt::plan_options(opt), t);
        return ok();
    });
}

jt_status jt_plan(int d, const int *n, const double *a, const double *b, double tol, jt_plan_t *out)
{
    return jt_plan_ex(d, n, a, b, tol, nullptr, out);
}

jt_status jt_plan_destroy(jt_plan_t plan)
{
    delete plan;
    return ok();
}

jt_status jt_plan_dims(jt_plan_t plan, int *d)
{
    if (!plan || !d) return fail(JT_EINVAL, "null argument");
    *d = plan->d;
    return ok();
}

jt_status jt_plan_info(jt_plan_t plan, int axis, jt_axis_info *info)
{
    jt_status st = check_axis(plan, axis);
    if (st != JT_OK) return st;
    if (!info) return fail(JT_EINVAL, "null info");
    const jt::AxisPlan &ax = plan->ax[axis];
    info->n = ax.n;
    info->L = ax.L;
    info->nu0 = ax.nu0;
    info->rank = ax.rank;
    info->max_per_bin = ax.max_per_bin;
    info->rsvd_rounds = ax.rsvd_rounds;
    info->rel_err = ax.rel_err;
    info->fro = ax.fro;
    info->planner = ax.planner;
    return ok();
}

jt_status jt_plan_nodes(jt_plan_t plan, int axis, double *t, double *x, double *omega)
{
    jt_status st = check_axis(plan, axis);
    if (st != JT_OK) return st;
    const jt::AxisPlan &ax = plan->ax[axis];
    if (t) std::memcpy(t, ax.t.data(), sizeof(double) * ax.n);
    if (x) std::memcpy(x, ax.x.data(), sizeof(double) * ax.n);
    if (omega) std::memcpy(omega, ax.omega.data(), sizeof(double) * ax.n);
    return ok();
}

jt_status jt_plan_factors(jt_plan_t plan, int axis, int32_t *bins, double *wv, double *u, double *v)
{
    jt_status st = check_axis(plan, axis);
    if (st != JT_OK) return st;
    const jt::AxisPlan &ax = plan->ax[axis];
    const int n = ax.n, nc = ax.n - ax.nu0;
    if (bins) std::memcpy(bins, ax.bins.data(), sizeof(int32_t) * n);
    if (wv) std::memcpy(wv, ax.WV.data(), sizeof(double) * ax.WV.size());
    if (u)
        for (size_t i = 0; i < ax.U.size(); ++i) {
            u[2 * i] = ax.U[i].real();
            u[2 * i + 1] = ax.U[i].imag();
        }
    if (v)
        for (int l = 0; l < ax.rank; ++l)
            for (int c = 0; c < nc; ++c) {
                const jt::cd z = ax.V[(size_t)l * ax.L + ax.nu0 + c];
                v[2 * ((size_t)l * nc + c)] = z.real();
                v[2 * ((size_t)l * nc + c) + 1] = z.imag();
            }
    return ok();
}

jt_status jt_plan_entries(jt_plan_t plan, int axis, int count, const int *rows, const int *degrees,
                          double *out)
{
    jt_status st = check_axis(plan, axis);
    if (st != JT_OK) return st;
    if (count < 0 || (count > 0 && (!rows || !degrees || !out))) return fail(JT_EINVAL, "bad arrays");
    return guarded([&]() -> jt_status {
        const jt::AxisPlan &ax = plan->ax[axis];
        for (int i = 0; i < count; ++i)
            if (degrees[i] < ax.nu0 || degrees[i] >= ax.n)
                return fail(JT_EINVAL, "degree outside [nu0, n)");
        std::vector<jt::cd> tmp(count);
        jt::exact_entries(ax, count, rows, degrees, tmp.data());
        for (int i = 0; i < count; ++i) {
            out[2 * i] = tmp[i].real();
            out[2 * i + 1] = tmp[i].imag();
        }
        return ok();
    });
}

jt_status jt_plan_device_bytes(jt_plan_t plan, size_t *bytes)
{
    if (!plan || !bytes) return fail(JT_EINVAL, "null argument");
    *bytes = plan->dev_bytes;
    return ok();
}

jt_status jt_plan_bind(jt_plan_t plan, void *dev_buf, size_t bytes, void *stream)
{
    if (!plan || !dev_buf) return fail(JT_EINVAL, "null argument");
    if (bytes < plan->dev_bytes) return fail(JT_ENOMEM, "device buffer smaller than jt_plan_device_bytes");
    if ((reinterpret_cast<uintptr_t>(dev_buf) & 255u) != 0) return fail(JT_EINVAL, "device buffer not 256-byte aligned");
    hipError_t e = hipMemcpyAsync(dev_buf, plan->blob.data(), plan->dev_bytes, hipMemcpyHostToDevice,
                                  reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail(JT_EDEVICE, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
    // the host image must outlive the asynchronous copy: wait for it here
    e = hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail(JT_EDEVICE, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
    plan->dev = static_cast<unsigned char *>(dev_buf);
    return ok();
}

jt_status jt_plan_pack(jt_plan_t plan, void *host_dst, size_t bytes)
{
    if (!plan || !host_dst) return fail(JT_EINVAL, "null argument");
    if (bytes < plan->dev_bytes) return fail(JT_ENOMEM, "host buffer smaller than jt_plan_device_bytes");
    std::memcpy(host_dst, plan->blob.data(), plan->dev_bytes);
    return ok();
}

jt_status jt_workspace_bytes(jt_plan_t plan, jt_prec prec, size_t *bytes)
{
    (void)prec;
    if (!plan || !bytes) return fail(JT_EINVAL, "null argument");
    *bytes = 0;
    return ok();
}

jt_status jt_forward(jt_plan_t plan, const void *alpha_dev, jt_dtype in, void *g_dev, jt_dtype out,
                     jt_prec prec, void *stream)
{
    return run_all(plan, true, alpha_dev, in, g_dev, out, prec, stream);
}

jt_status jt_inverse(jt_plan_t plan, const void *g_dev, jt_dtype in, void *alpha_dev, jt_dtype out,
                     jt_prec prec, void *stream)
{
    return run_all(plan, false, g_dev, in, alpha_dev, out, prec, stream);
}

jt_status jt_apply_axis(jt_plan_t plan, int axis, jt_direction dir, const void *in_dev, jt_dtype in,
                        void *out_dev, jt_dtype out, jt_prec prec, void *stream)
{
    if (dir != JT_FORWARD && dir != JT_INVERSE) return fail(JT_EINVAL, "bad direction");
    jt_status st = run_axis(plan, axis, dir == JT_FORWARD, in_dev, in, out_dev, out, prec, stream);
    return st == JT_OK ? ok() : st;
}

}  // extern "C"
