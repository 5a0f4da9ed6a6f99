// 3D stencil kernels beyond the 7-point star, instantiated for double (the radius-2 star;
// the radius-1 box variant is disabled, see stencil.hip).
#include "stencil3d_wide.hpp"
#include "stencil_api.hpp"

namespace perks {

template <>
int run3d_wide<double>(double *grid, const double *coeffs, const perks_shape &s, int64_t steps, int radius, bool box,
                    hipStream_t st, const perks_tuning *tu) {
    if (radius == 2 && !box) return run_wide3<double, 2, false>(grid, coeffs, s, steps, st, tu);
    return PERKS_E_UNSUPPORTED;
}

template <>
int baseline3d_wide<double>(double *grid, const double *coeffs, const perks_shape &s, int64_t steps, int radius,
                         bool box, hipStream_t st) {
    if (radius == 2 && !box) return baseline_wide3<double, 2, false>(grid, coeffs, s, steps, st);
    return PERKS_E_UNSUPPORTED;
}

template <>
int plan3d_wide_query<double>(const perks_shape &s, int radius, bool box, const perks_tuning *tu,
                           perks_stencil_plan *plan) {
    if (radius == 2 && !box) return plan_wide3_query<double, 2, false>(s, tu, plan);
    return PERKS_E_UNSUPPORTED;
}

}  // namespace perks
