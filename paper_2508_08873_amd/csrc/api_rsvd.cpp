#include "lrpr_internal.h"
extern "C" {
lrpr_status lrpr_rsvd_build(lrpr_ctx ctx, int, const lrpr_slice_desc *, int, lrpr_prec, lrpr_coarse *, double *, int *) { return lrpr::fail(ctx, LRPR_ERR_ARG, "not built"); }
void lrpr_coarse_destroy(lrpr_coarse) {}
lrpr_status lrpr_coarse_get(lrpr_coarse, int, const double **, const double **, const double **, int *, int64_t *) { return LRPR_ERR_ARG; }
lrpr_status lrpr_coarse_apply(lrpr_ctx ctx, lrpr_coarse, int, int, const double *, double *) { return lrpr::fail(ctx, LRPR_ERR_ARG, "not built"); }
lrpr_status lrpr_parareal_solve(lrpr_ctx ctx, lrpr_coarse, const lrpr_fac *, int, lrpr_prec, int, const double *, const double *, const double *, double, int, double *, int *, double *, double *) { return lrpr::fail(ctx, LRPR_ERR_ARG, "not built"); }
}
