// 2D stencil kernels and launchers instantiated for float.
#include "stencil2d.hpp"
#include "stencil_api.hpp"

namespace perks {
template int run2d_in<float>(float *, const double *, const perks_shape &, int64_t, bool, hipStream_t, void *, size_t);
template int run2d<float>(float *, const double *, const perks_shape &, int64_t, bool, hipStream_t, const perks_tuning *);
template int plan2d_query<float>(const perks_shape &, bool, const perks_tuning *, perks_stencil_plan *);
}  // namespace perks
