// Radius-1..4 2D stencil kernels of the wide family and launchers instantiated for float.
#include "stencil2d_wide.hpp"
#include "stencil_api.hpp"

namespace perks {

template <>
int run2d_wide<float>(float *grid, const double *coeffs, const perks_shape &s, int64_t steps, int radius, bool box,
                    hipStream_t st, const perks_tuning *tu) {
    if (box) {
        if (radius == 1) return run_wide<float, 1, true>(grid, coeffs, s, steps, st, tu);
        return radius == 2 ? run_wide<float, 2, true>(grid, coeffs, s, steps, st, tu) : PERKS_E_UNSUPPORTED;
    }
    switch (radius) {
        case 1: return run_wide<float, 1, false>(grid, coeffs, s, steps, st, tu);
        case 2: return run_wide<float, 2, false>(grid, coeffs, s, steps, st, tu);
        case 3: return run_wide<float, 3, false>(grid, coeffs, s, steps, st, tu);
        case 4: return run_wide<float, 4, false>(grid, coeffs, s, steps, st, tu);
        default: return PERKS_E_UNSUPPORTED;
    }
}

template <>
int baseline2d_wide<float>(float *grid, const double *coeffs, const perks_shape &s, int64_t steps, int radius,
                         bool box, hipStream_t st) {
    if (box) {
        if (radius == 1) return baseline_wide<float, 1, true>(grid, coeffs, s, steps, st);
        return radius == 2 ? baseline_wide<float, 2, true>(grid, coeffs, s, steps, st) : PERKS_E_UNSUPPORTED;
    }
    switch (radius) {
        case 1: return baseline_wide<float, 1, false>(grid, coeffs, s, steps, st);
        case 2: return baseline_wide<float, 2, false>(grid, coeffs, s, steps, st);
        case 3: return baseline_wide<float, 3, false>(grid, coeffs, s, steps, st);
        case 4: return baseline_wide<float, 4, false>(grid, coeffs, s, steps, st);
        default: return PERKS_E_UNSUPPORTED;
    }
}

template <>
int plan2d_wide_query<float>(const perks_shape &s, int radius, bool box, const perks_tuning *tu,
                           perks_stencil_plan *plan) {
    if (box) {
        if (radius == 1) return plan_wide_query<float, 1, true>(s, tu, plan);
        return radius == 2 ? plan_wide_query<float, 2, true>(s, tu, plan) : PERKS_E_UNSUPPORTED;
    }
    switch (radius) {
        case 1: return plan_wide_query<float, 1, false>(s, tu, plan);
        case 2: return plan_wide_query<float, 2, false>(s, tu, plan);
        case 3: return plan_wide_query<float, 3, false>(s, tu, plan);
        case 4: return plan_wide_query<float, 4, false>(s, tu, plan);
        default: return PERKS_E_UNSUPPORTED;
    }
}

}  // namespace perks
