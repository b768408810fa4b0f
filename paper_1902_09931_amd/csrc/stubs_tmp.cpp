// Temporary: entry points not implemented yet.
#include "plans.h"
using namespace mxs;
extern "C" {
mxs_status mxs_create_cyclic_solve(int, const double *, int, int, int, long long, int, const long long *, int, const void *, void *, mxs_plan *p) { if (p) *p = nullptr; return fail(MXS_ERR_UNSUPPORTED, "not implemented"); }
mxs_status mxs_ch_create(int, int, double, double, double, double, double, int, void *, void *, void *, mxs_plan *p) { if (p) *p = nullptr; return fail(MXS_ERR_UNSUPPORTED, "not implemented"); }
mxs_status mxs_ch_ensemble_create(int, const int *, const int *, const double *, const double *, const double *, double, double, int, void *const *, void *const *, void *const *, mxs_plan *p) { if (p) *p = nullptr; return fail(MXS_ERR_UNSUPPORTED, "not implemented"); }
mxs_status mxs_ch_step(mxs_plan, int, int, void *) { return fail(MXS_ERR_UNSUPPORTED, "not implemented"); }
mxs_status mxs_ch_state(mxs_plan, int, void **, void **) { return fail(MXS_ERR_UNSUPPORTED, "not implemented"); }
mxs_status mxs_ch_steps_taken(mxs_plan, long long *) { return fail(MXS_ERR_UNSUPPORTED, "not implemented"); }
mxs_status mxs_ch_mass(mxs_plan, double *, void *) { return fail(MXS_ERR_UNSUPPORTED, "not implemented"); }
}
