// Private pieces of the C ABI shared by its translation units: the plan
// handle and the thread-local error reporting.
#pragma once

#include "jt.h"

#include <exception>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "plan.h"
#include "queue.h"

struct jt_plan_s {
    int d = 0;
    jt::AxisPlan ax[3];
    std::vector<unsigned char> blob;  // packed device image
    size_t dev_bytes = 0;
    unsigned char *dev = nullptr;     // caller-owned device buffer (after bind)
};

namespace jt {

inline thread_local std::string g_err;

inline jt_status fail(jt_status st, const std::string &msg)
{
    g_err = msg;
    return st;
}

inline jt_status ok()
{
    g_err.clear();
    return JT_OK;
}

template <class F>
jt_status guarded(F f)
{
    try {
        return f();
    } catch (const std::invalid_argument &e) {
        return fail(JT_EINVAL, e.what());
    } catch (const unsupported &e) {
        return fail(JT_EUNSUPPORTED, e.what());
    } catch (const std::bad_alloc &) {
        return fail(JT_ENOMEM, "host allocation failed");
    } catch (const std::runtime_error &e) {
        return fail(JT_ENOTCONV, e.what());
    } catch (const std::exception &e) {
        return fail(JT_EINVAL, e.what());
    } catch (...) {
        return fail(JT_EINVAL, "unknown error");
    }
}

// Build one plan (host).  Throws on failure.
// With t (the axes' points concatenated): the nonuniform forward transform.
jt_plan_s *build_plan(int d, const int *n, const double *a, const double *b, double tol, const PlanOptions &po,
                      const double *t = nullptr);
// Plan options from the ABI struct (NULL: defaults).
PlanOptions plan_options(const jt_plan_options *opt);

}  // namespace jt
