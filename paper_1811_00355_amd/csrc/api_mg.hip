// C ABI, part 2: multigrid setup, transfer, coarse operator and solver.
#include "dd_internal.h"

extern "C" {
size_t dd_coarse_vec_bytes(const dd_mg*, dd_dtype, int) { return 0; }
dd_status dd_pack_coarse(const dd_mg*, dd_dtype, int, const double*, void*, void*) { return DD_EINVAL; }
dd_status dd_unpack_coarse(const dd_mg*, dd_dtype, int, const void*, double*, void*) { return DD_EINVAL; }
dd_status dd_setup(dd_gauge*, const dd_mg_params*, dd_mg**) { return DD_EINVAL; }
dd_status dd_setup_from_vectors(dd_gauge*, const dd_mg_params*, const double*, dd_mg**) { return DD_EINVAL; }
dd_status dd_mg_destroy(dd_mg*) { return DD_EINVAL; }
dd_status dd_restrict(dd_mg*, dd_dtype, int, const void*, void*, void*) { return DD_EINVAL; }
dd_status dd_prolong(dd_mg*, dd_dtype, int, const void*, void*, void*) { return DD_EINVAL; }
dd_status dd_coarse_apply(dd_mg*, dd_dtype, int, const void*, void*, void*) { return DD_EINVAL; }
dd_status dd_coarse_solve(dd_mg*, dd_dtype, int, const void*, void*, int*, void*) { return DD_EINVAL; }
dd_status dd_precond_apply(dd_mg*, int, const void*, void*, void*) { return DD_EINVAL; }
dd_status dd_solve(dd_mg*, int, const double*, double*, double, dd_solve_info*, void*) { return DD_EINVAL; }
dd_status dd_export_coarse(const dd_mg*, double*) { return DD_EINVAL; }
dd_status dd_export_vectors(const dd_mg*, double*) { return DD_EINVAL; }
}
