// Host side of the stencil entry points: argument checks, launch planning
// (tile depth, grid size, cached vs streamed tiles) and kernel dispatch.
#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "stencil_api.hpp"

namespace perks {
namespace {

enum Kind { K_2D5 = 0, K_2D9 = 1, K_3D7 = 2 };

int classify(const double *c, const perks_shape &s, Kind *kind) {
    if (s.ndim == 2) {
        // [dy][dx]: corners are indices 0, 2, 6, 8
        bool corners = c[0] != 0.0 || c[2] != 0.0 || c[6] != 0.0 || c[8] != 0.0;
        *kind = corners ? K_2D9 : K_2D5;
        return PERKS_OK;
    }
    // 3D: only the centre and the six face neighbours may be non-zero
    for (int dz = 0; dz < 3; ++dz)
        for (int dy = 0; dy < 3; ++dy)
            for (int dx = 0; dx < 3; ++dx) {
                int off = (dz != 1) + (dy != 1) + (dx != 1);
                if (off > 1 && c[(dz * 3 + dy) * 3 + dx] != 0.0)
                    return set_error(PERKS_E_UNSUPPORTED,
                                     "3D weights outside the 7-point star are not supported");
            }
    *kind = K_3D7;
    return PERKS_OK;
}

int check_common(const void *grid, const double *coeffs, const perks_shape &s, int64_t steps, perks_dtype dt) {
    if (!grid || !coeffs) return set_error(PERKS_E_INVAL, "grid and coeffs must not be NULL");
    if (s.ndim != 2 && s.ndim != 3) return set_error(PERKS_E_INVAL, "ndim must be 2 or 3 (got %d)", s.ndim);
    if (dt != PERKS_F32 && dt != PERKS_F64) return set_error(PERKS_E_INVAL, "dtype must be PERKS_F32 or PERKS_F64");
    if (steps < 0) return set_error(PERKS_E_INVAL, "steps must be >= 0");
    if (s.nx < 3 || s.ny < 3 || (s.ndim == 3 && s.nz < 3))
        return set_error(PERKS_E_INVAL, "every extent must be >= 3 (ring of width 1 on both sides)");
    const int64_t lim = int64_t(1) << 30;
    if (s.nx > lim || s.ny > lim || (s.ndim == 3 && s.nz > lim))
        return set_error(PERKS_E_INVAL, "extent too large");
    const int64_t cells = s.nx * s.ny * (s.ndim == 3 ? s.nz : 1);
    if (cells > (int64_t(1) << 36)) return set_error(PERKS_E_INVAL, "grid too large");
    const int n = s.ndim == 3 ? 27 : 9;
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(coeffs[i])) return set_error(PERKS_E_INVAL, "coeffs must be finite");
    return PERKS_OK;
}

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace
}  // namespace perks

using namespace perks;

extern "C" {

int perks_stencil_run(void *grid, const double *coeffs, perks_shape shape, int64_t steps, perks_dtype dt,
                      void *stream, const perks_tuning *tune) {
    int rc = check_common(grid, coeffs, shape, steps, dt);
    if (rc) return rc;
    Kind kind;
    rc = classify(coeffs, shape, &kind);
    if (rc) return rc;
    if (steps == 0) return PERKS_OK;
    hipStream_t st = as_stream(stream);
    if (shape.ndim == 2) {
        const bool box = kind == K_2D9;
        return dt == PERKS_F64 ? run2d<double>((double *)grid, coeffs, shape, steps, box, st, tune)
                               : run2d<float>((float *)grid, coeffs, shape, steps, box, st, tune);
    }
    return dt == PERKS_F64 ? run3d<double>((double *)grid, coeffs, shape, steps, st, tune)
                           : run3d<float>((float *)grid, coeffs, shape, steps, st, tune);
}

int perks_stencil_run_baseline(void *grid, const double *coeffs, perks_shape shape, int64_t steps, perks_dtype dt,
                               void *stream) {
    int rc = check_common(grid, coeffs, shape, steps, dt);
    if (rc) return rc;
    Kind kind;
    rc = classify(coeffs, shape, &kind);
    if (rc) return rc;
    if (steps == 0) return PERKS_OK;
    hipStream_t st = as_stream(stream);
    if (shape.ndim == 2) {
        if (kind == K_2D9)
            return dt == PERKS_F64 ? baseline2d<double, true>((double *)grid, coeffs, shape, steps, st)
                                   : baseline2d<float, true>((float *)grid, coeffs, shape, steps, st);
        return dt == PERKS_F64 ? baseline2d<double, false>((double *)grid, coeffs, shape, steps, st)
                               : baseline2d<float, false>((float *)grid, coeffs, shape, steps, st);
    }
    return dt == PERKS_F64 ? baseline3d<double>((double *)grid, coeffs, shape, steps, st)
                           : baseline3d<float>((float *)grid, coeffs, shape, steps, st);
}

int perks_stencil_plan_query(const double *coeffs, perks_shape shape, perks_dtype dt, const perks_tuning *tune,
                             perks_stencil_plan *plan) {
    int dummy = 0;
    int rc = check_common(&dummy, coeffs, shape, 1, dt);
    if (rc) return rc;
    if (!plan) return set_error(PERKS_E_INVAL, "plan must not be NULL");
    Kind kind;
    rc = classify(coeffs, shape, &kind);
    if (rc) return rc;
    memset(plan, 0, sizeof(*plan));
    if (shape.ndim == 2)
        return dt == PERKS_F64 ? plan2d_query<double>(shape, kind == K_2D9, tune, plan)
                               : plan2d_query<float>(shape, kind == K_2D9, tune, plan);
    return dt == PERKS_F64 ? plan3d_query<double>(shape, tune, plan) : plan3d_query<float>(shape, tune, plan);
}

}  // extern "C"
