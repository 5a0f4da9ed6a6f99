// Entry points of the per-dtype stencil translation units (explicitly
// instantiated in stencil{2d,3d}_{f32,f64}.hip so they compile in parallel).
#pragma once

#include "common.hpp"

namespace perks {

template <typename T>
int run2d(T *grid, const double *coeffs, const perks_shape &s, int64_t steps, bool box, hipStream_t st,
          const perks_tuning *tu);
template <typename T>
int plan2d_query(const perks_shape &shape, bool box, const perks_tuning *tune, perks_stencil_plan *plan);
// run2d with the default plan, barrier words and face buffers in `mem` (cap
// bytes, device); allocates nothing.
template <typename T>
int run2d_in(T *grid, const double *coeffs, const perks_shape &s, int64_t steps, bool box, hipStream_t st,
             void *mem, size_t cap);

// Temporally blocked 2D radius-1 kernel (perks_tuning.kernel = 3).
template <typename T>
int run2d_tb(T *grid, const double *coeffs, const perks_shape &s, int64_t steps, bool box, hipStream_t st,
             const perks_tuning *tu);
template <typename T>
int plan2d_tb_query(const perks_shape &s, bool box, const perks_tuning *tu, perks_stencil_plan *plan);
template <typename T>
int run2d_tb_batched(T *const *grids, const perks_shape *shapes, int count, const double *coeffs, int64_t steps,
                     bool box, hipStream_t st);
// A batched-stencil plan (perks_stencil_batch_*): its own device memory and
// its launch as a one-node HIP graph.
struct StencilBatchPlan;
template <typename T>
int tb_batch_create(T *const *grids, const perks_shape *shapes, int count, const double *coeffs, int64_t steps,
                    bool box, StencilBatchPlan **out);
int tb_batch_run(StencilBatchPlan *P, hipStream_t st);
int tb_batch_graph(StencilBatchPlan *P, void **graph);
void tb_batch_destroy(StencilBatchPlan *P);

// Radius-2..4 2D stencils: `radius` 2..4 with `box` false (stars) or radius
// 2 with `box` true.
template <typename T>
int run2d_wide(T *grid, const double *coeffs, const perks_shape &s, int64_t steps, int radius, bool box,
               hipStream_t st, const perks_tuning *tu);
template <typename T>
int baseline2d_wide(T *grid, const double *coeffs, const perks_shape &s, int64_t steps, int radius, bool box,
                    hipStream_t st);
template <typename T>
int plan2d_wide_query(const perks_shape &s, int radius, bool box, const perks_tuning *tu, perks_stencil_plan *plan);

// 3D stencils beyond the 7-point star: any radius-1 pattern (`box`) or the
// radius-2 star (streamed through HBM every step).
template <typename T>
int run3d_wide(T *grid, const double *coeffs, const perks_shape &s, int64_t steps, int radius, bool box,
               hipStream_t st, const perks_tuning *tu);
template <typename T>
int baseline3d_wide(T *grid, const double *coeffs, const perks_shape &s, int64_t steps, int radius, bool box,
                    hipStream_t st);
template <typename T>
int plan3d_wide_query(const perks_shape &s, int radius, bool box, const perks_tuning *tu, perks_stencil_plan *plan);

template <typename T>
int run3d(T *grid, const double *coeffs, const perks_shape &s, int64_t steps, hipStream_t st,
          const perks_tuning *tu);
template <typename T>
int baseline3d(T *grid, const double *coeffs, const perks_shape &s, int64_t steps, hipStream_t st);
template <typename T>
int plan3d_query(const perks_shape &s, const perks_tuning *tu, perks_stencil_plan *plan);

}  // namespace perks
