// C ABI entry points of libmw that enqueue device work.
#include <cstring>
#include <string>

#include "mw_internal.h"

using namespace mw;

extern "C" const mw::DevPlan *mw_internal_devplan(mw_plan plan);

static mw_status bound_plan(mw_plan plan, const DevPlan **out)
{
    if (!plan) return fail(MW_EINVAL, "plan is NULL");
    const DevPlan *d = mw_internal_devplan(plan);
    if (!d) return fail(MW_EWORKSPACE, "plan has no workspace: call mw_plan_upload first");
    *out = d;
    return MW_OK;
}

extern "C" {

mw_status mw_sigma(mw_plan plan, int32_t nroots, const void *c, void *sigma, mw_stream_t stream)
{
    const DevPlan *d;
    mw_status st = bound_plan(plan, &d);
    if (st != MW_OK) return st;
    if (nroots < 1 || nroots > d->max_roots) return fail(MW_EINVAL, "nroots must be in 1..max_roots");
    if (!c || !sigma) return fail(MW_EINVAL, "c and sigma must be device pointers");
    if (c == sigma) return fail(MW_EINVAL, "c and sigma must not overlap");
    return launch_sigma(*d, nroots, c, sigma, (hipStream_t)stream);
}

mw_status mw_diag(mw_plan plan, void *out, mw_stream_t stream)
{
    const DevPlan *d;
    mw_status st = bound_plan(plan, &d);
    if (st != MW_OK) return st;
    if (!out) return fail(MW_EINVAL, "out is NULL");
    size_t nb = (size_t)d->ndet * (d->kind == MW_SPINOR ? 16 : 8);
    if (hipMemcpyAsync(out, d->diag, nb, hipMemcpyDeviceToDevice, (hipStream_t)stream) != hipSuccess)
        return fail(MW_EHIP, "hipMemcpyAsync failed");
    return MW_OK;
}

mw_status mw_connect_dump(mw_plan plan, int64_t *count, int64_t *out, mw_stream_t stream)
{
    const DevPlan *d;
    mw_status st = bound_plan(plan, &d);
    if (st != MW_OK) return st;
    if (!count) return fail(MW_EINVAL, "count is NULL");
    return launch_connect(*d, count, out, (hipStream_t)stream);
}

}  // extern "C"

