// 3D stencil kernels and launchers instantiated for double.
#include "stencil3d.hpp"
#include "stencil_api.hpp"

namespace perks {
template int run3d<double>(double *, const double *, const perks_shape &, int64_t, hipStream_t, const perks_tuning *);
template int baseline3d<double>(double *, const double *, const perks_shape &, int64_t, hipStream_t);
template int plan3d_query<double>(const perks_shape &, const perks_tuning *, perks_stencil_plan *);
}  // namespace perks
