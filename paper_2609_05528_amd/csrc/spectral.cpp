// Spectral drivers and estimators (filled in by the dense-kernel layer).
#include "rtt_internal.h"

using namespace rtt;

extern "C" int rsvd(const rtt_geometry*, const rtt_svd_opts*, const float*, rtt_svd** out, void*)
{
    if (out) *out = nullptr;
    return fail(RTT_ESTATE, "rsvd: not available in this build");
}
extern "C" int svd_free(rtt_svd*) { return RTT_OK; }
extern "C" int svd_get(const rtt_svd*, int32_t*, double*, const float**, const float**, double*)
{
    return fail(RTT_ESTATE, "svd_get: not available in this build");
}
extern "C" int tsvd_solve(const rtt_geometry*, const rtt_svd*, const float*, int32_t, int32_t, double, float*,
                          void*)
{
    return fail(RTT_ESTATE, "tsvd_solve: not available in this build");
}
extern "C" int ridge_solve(const rtt_geometry* g, const float*, int32_t, float, const rtt_cg_opts*, float*,
                           rtt_solve_info*, void*)
{
    if (!valid_handle(g)) return fail(RTT_EINVAL, "invalid geometry handle");
    return fail(RTT_ESTATE, "ridge_solve: not available in this build");
}
