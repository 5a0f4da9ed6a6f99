// The register-resident persistent CG solvers (cg_f64_reg, cg_mixed_reg): the
// device code of cg_device.hpp compiled for 8 waves per workgroup, one
// workgroup per CU (two waves per SIMD), so that each wave may use 256
// registers, about 120 of them (FP64) for the r, p and q entries of its
// 2 x CG_RV rows per thread.
#define PERKS_CG_WAVES 8
#include "cg_device.hpp"

namespace perks {

const void *cg_reg_kernel(bool jacobi, bool mixed, int *threads, int *rows_per_thread) {
    *threads = CG_THREADS;
    *rows_per_thread = CG_VT * CG_RV;
    if (mixed)
        return jacobi ? reinterpret_cast<const void *>(&cg_persistent_reg<true, true>)
                      : reinterpret_cast<const void *>(&cg_persistent_reg<false, true>);
    return jacobi ? reinterpret_cast<const void *>(&cg_persistent_reg<true, false>)
                  : reinterpret_cast<const void *>(&cg_persistent_reg<false, false>);
}

}  // namespace perks
