// Host side of the stencil entry points: argument checks, launch planning
// (tile depth, grid size, cached vs streamed tiles) and kernel dispatch.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <new>
#include <vector>

#include "common.hpp"
#include "stencil_api.hpp"

// Scratch of perks_stencil_run_noalloc (barrier words, then face buffers):
// one copy per device, alive until the process ends.  In host code this name
// is a stand-in, not a device address: kernels get the address that
// hipGetSymbolAddress returns for the current device.  It has external
// linkage (in its own namespace): the runtime resolves only exported device
// symbols, and an internal-linkage array is reported as an invalid symbol.
// No kernel names it, so `used` keeps the device compiler from dropping it;
// 256 spare bytes let the host round its address up to 256 bytes whatever
// alignment the code object gives it.
constexpr size_t NOALLOC_BYTES = size_t(32) << 20;
namespace perks_noalloc {
__device__ __attribute__((used)) __align__(256) unsigned char scratch[NOALLOC_BYTES + 256];
}

namespace perks {
namespace {

// Zero fill of n 32-bit words (a kernel, not hipMemsetAsync: stream-ordered
// and safe under graph capture).
__global__ __launch_bounds__(256) void fill_zero_words(unsigned *w, size_t n) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) w[i] = 0u;
}

// Per-device address of `scratch`, looked up on the first call on a device
// (with that device current), when the whole array is also cleared on the
// caller's stream: the barrier and halo words then start at epoch 0, and
// every later call continues the epochs the previous one left there.
std::mutex g_noalloc_mu;
void *g_noalloc_ptr[64];

int noalloc_scratch(hipStream_t st, void **out) {
    int dev = -1;
    PERKS_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return set_error(PERKS_E_HIP, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(perks_noalloc::scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return set_error(PERKS_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        }
        ptr = (void *)(((uintptr_t)ptr + 255) & ~(uintptr_t)255);
        hipLaunchKernelGGL(fill_zero_words, dim3(1024), dim3(256), 0, st, (unsigned *)ptr, NOALLOC_BYTES / 4);
        PERKS_HIP_TRY(hipGetLastError());
        g_noalloc_ptr[dev] = ptr;
    }
    *out = g_noalloc_ptr[dev];
    return PERKS_OK;
}

// Patterns: radius 1 (2D 5-point star, 2D 9-point box, 3D 7-point star),
// the radius-2..4 2D stars and radius-2 2D box, and the radius-2 3D star.
enum Kind { K_2D5 = 0, K_2D9 = 1, K_3D7 = 2, K_W2S = 3, K_W3S = 4, K_W4S = 5, K_W2B = 6, K_3S2 = 7 };

int radius_of(const perks_shape &s) { return s.radius <= 0 ? 1 : s.radius; }
bool is_wide(Kind k) { return k >= K_W2S && k <= K_W2B; }
int wide_radius(Kind k) { return k == K_W2B ? 2 : (int)k - 1; }
bool is_wide3(Kind k) { return k == K_3S2; }

int classify(const double *c, const perks_shape &s, Kind *kind) {
    const int r = radius_of(s);
    if (r > 1 && s.ndim == 3) {
        if (r != 2) return set_error(PERKS_E_UNSUPPORTED, "3D stencils of radius %d are not supported", r);
        const int w = 5;
        for (int dz = 0; dz < w; ++dz)
            for (int dy = 0; dy < w; ++dy)
                for (int dx = 0; dx < w; ++dx) {
                    const int off = (dz != 2) + (dy != 2) + (dx != 2);
                    if (off > 1 && c[(dz * w + dy) * w + dx] != 0.0)
                        return set_error(PERKS_E_UNSUPPORTED, "3D radius-2 weights must form a star");
                }
        *kind = K_3S2;
        return PERKS_OK;
    }
    if (r > 1) {
        const int w = 2 * r + 1;
        bool off_axis = false;
        for (int dy = 0; dy < w; ++dy)
            for (int dx = 0; dx < w; ++dx)
                if (dy != r && dx != r && c[dy * w + dx] != 0.0) off_axis = true;
        if (!off_axis) {
            *kind = (Kind)(K_W2S + (r - 2));
            return PERKS_OK;
        }
        if (r != 2) return set_error(PERKS_E_UNSUPPORTED, "2D boxes of radius %d are not supported (radius 2 is)", r);
        *kind = K_W2B;
        return PERKS_OK;
    }
    if (s.ndim == 2) {
        // [dy][dx]: corners are indices 0, 2, 6, 8
        bool corners = c[0] != 0.0 || c[2] != 0.0 || c[6] != 0.0 || c[8] != 0.0;
        *kind = corners ? K_2D9 : K_2D5;
        return PERKS_OK;
    }
    // 3D: the 7-point star (centre and face neighbours), else the box kernel
    for (int dz = 0; dz < 3; ++dz)
        for (int dy = 0; dy < 3; ++dy)
            for (int dx = 0; dx < 3; ++dx) {
                int off = (dz != 1) + (dy != 1) + (dx != 1);
                if (off > 1 && c[(dz * 3 + dy) * 3 + dx] != 0.0)
                    // the radius-1 box variant of the 3D streamed kernels
                    // (3d27pt, poisson, 3d17pt) passes its small-grid parity
                    // tests but hung once at 256^3 with four workgroups per
                    // CU, cause not found; it stays off until that is understood
                    return set_error(PERKS_E_UNSUPPORTED,
                                     "3D weights outside the 7-point star are not supported at radius 1");
            }
    *kind = K_3D7;
    return PERKS_OK;
}

// True when the caller left every tuning field at zero (the library's choice).
bool untuned(const perks_tuning *tu) {
    return !tu || (tu->waves_per_wg == 0 && tu->wgs_per_cu == 0 && tu->rows_per_lane == 0 &&
                   tu->planes_per_lane == 0 && tu->sync == 0 && tu->max_cached_tiles == 0 && tu->kernel == 0 &&
                   tu->steps_per_sync == 0);
}

// Interior cells from which an untuned 2D radius-1 run takes the radius-2..4
// kernel family.  Measured on MI355X: at 3072^2 that family (grid barrier,
// one register-cached 64 x 24..48 tile per wave) beats the radius-1 kernel
// (point-to-point halo words, LDS rows) in both precisions and both
// patterns; on small grids, whose steps are a few microseconds, the
// point-to-point kernel's neighbour-only waits are cheaper than a device
// barrier.
constexpr int64_t WIDE_FAMILY_MIN_CELLS = int64_t(1) << 20;

// 2D radius-1 patterns may run on the radius-2..4 kernel family
// (perks_tuning.kernel = 2, or untuned on a large grid whose tiles that
// family caches all at once); the per-step baseline always uses that
// family's per-step kernel, the faster of the two per-step kernels.
bool use_wide_family(Kind k, const perks_shape &s, perks_dtype dt, const perks_tuning *tu) {
    if (k != K_2D5 && k != K_2D9) return false;
    if (tu && tu->kernel == 2) return true;
    if (!untuned(tu)) return false;
    const int64_t cells = (s.nx - 2) * (s.ny - 2);
    if (cells < WIDE_FAMILY_MIN_CELLS) return false;
    perks_stencil_plan pl{};
    const bool box = k == K_2D9;
    const int rc = dt == PERKS_F64 ? plan2d_wide_query<double>(s, 1, box, nullptr, &pl)
                                   : plan2d_wide_query<float>(s, 1, box, nullptr, &pl);
    return rc == PERKS_OK && pl.tiles > 0 && pl.cached_tiles == pl.tiles;
}

int check_tuning(const perks_tuning *tu) {
    if (tu && (tu->kernel < 0 || tu->kernel > 3))
        return set_error(PERKS_E_INVAL, "tuning.kernel must be 0, 1, 2 or 3");
    if (tu && tu->steps_per_sync != 0 && tu->kernel != 3)
        return set_error(PERKS_E_INVAL, "tuning.steps_per_sync applies to kernel 3 only");
    return PERKS_OK;
}

// The temporally blocked kernel (2D radius-1 patterns): kernel = 3, and the
// library's choice below WIDE_FAMILY_MIN_CELLS interior cells (measured on
// MI355X at 256^2 .. 1024^2 FP64 and FP32: 1.3-2.6 us per step against 3.1-4.8
// for the point-to-point kernel and 3.4-5.1 for one launch per step), and
// above it when its default plan keeps every tile in registers (3072^2: 8.6
// us per step FP64 and 6.1 FP32 against 10.5 and 7.4 for the radius-2..4
// family).
bool use_tb(Kind k, const perks_shape &s, perks_dtype dt, const perks_tuning *tu) {
    if (k != K_2D5 && k != K_2D9) return false;
    if (tu && tu->kernel == 3) return true;
    if (!untuned(tu)) return false;
    if ((s.nx - 2) * (s.ny - 2) < WIDE_FAMILY_MIN_CELLS) return true;
    perks_stencil_plan pl{};
    const bool box = k == K_2D9;
    const int rc = dt == PERKS_F64 ? plan2d_tb_query<double>(s, box, nullptr, &pl)
                                   : plan2d_tb_query<float>(s, box, nullptr, &pl);
    return rc == PERKS_OK && pl.tiles > 0 && pl.cached_tiles == pl.tiles;
}

int check_common(const void *grid, const double *coeffs, const perks_shape &s, int64_t steps, perks_dtype dt) {
    if (!grid || !coeffs) return set_error(PERKS_E_INVAL, "grid and coeffs must not be NULL");
    if (s.ndim != 2 && s.ndim != 3) return set_error(PERKS_E_INVAL, "ndim must be 2 or 3 (got %d)", s.ndim);
    if (dt != PERKS_F32 && dt != PERKS_F64) return set_error(PERKS_E_INVAL, "dtype must be PERKS_F32 or PERKS_F64");
    if (steps < 0) return set_error(PERKS_E_INVAL, "steps must be >= 0");
    if (s.radius < 0 || s.radius > 4) return set_error(PERKS_E_INVAL, "radius must be 0..4 (got %d)", s.radius);
    const int r = radius_of(s);
    if (s.nx < 2 * r + 1 || s.ny < 2 * r + 1 || (s.ndim == 3 && s.nz < 2 * r + 1))
        return set_error(PERKS_E_INVAL, "every extent must be >= %d (ring of width %d on both sides)", 2 * r + 1, r);
    const int64_t lim = int64_t(1) << 30;
    if (s.nx > lim || s.ny > lim || (s.ndim == 3 && s.nz > lim))
        return set_error(PERKS_E_INVAL, "extent too large");
    const int64_t cells = s.nx * s.ny * (s.ndim == 3 ? s.nz : 1);
    if (cells > (int64_t(1) << 36)) return set_error(PERKS_E_INVAL, "grid too large");
    const int w = 2 * r + 1;
    const int n = s.ndim == 3 ? w * w * w : w * w;
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(coeffs[i])) return set_error(PERKS_E_INVAL, "coeffs must be finite");
    return PERKS_OK;
}

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Tunings the autotuner chose, per (device, pattern, dtype, extents); used by
// perks_stencil_run when the caller passes no tuning.
using TuneKey = std::tuple<int, int, int, int64_t, int64_t, int64_t>;
std::mutex g_tune_mu;
std::map<TuneKey, perks_tuning> g_tuned;

TuneKey tune_key(Kind kind, perks_dtype dt, const perks_shape &s) {
    int dev = -1;
    (void)hipGetDevice(&dev);
    return TuneKey(dev, (int)kind, (int)dt, s.nx, s.ny, s.ndim == 3 ? s.nz : 1);
}

bool tuned_for(Kind kind, perks_dtype dt, const perks_shape &s, perks_tuning *out) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(tune_key(kind, dt, s));
    if (it == g_tuned.end()) return false;
    *out = it->second;
    return true;
}

int run_dispatch(void *grid, const double *coeffs, const perks_shape &shape, int64_t steps, perks_dtype dt,
                 Kind kind, hipStream_t st, const perks_tuning *tune) {
    if (use_tb(kind, shape, dt, tune)) {
        const bool box = kind == K_2D9;
        return dt == PERKS_F64 ? run2d_tb<double>((double *)grid, coeffs, shape, steps, box, st, tune)
                               : run2d_tb<float>((float *)grid, coeffs, shape, steps, box, st, tune);
    }
    if (is_wide(kind) || use_wide_family(kind, shape, dt, tune)) {
        const int r = is_wide(kind) ? wide_radius(kind) : 1;
        const bool box = kind == K_W2B || kind == K_2D9;
        return dt == PERKS_F64 ? run2d_wide<double>((double *)grid, coeffs, shape, steps, r, box, st, tune)
                               : run2d_wide<float>((float *)grid, coeffs, shape, steps, r, box, st, tune);
    }
    if (is_wide3(kind)) {
        return dt == PERKS_F64 ? run3d_wide<double>((double *)grid, coeffs, shape, steps, 2, false, st, tune)
                               : run3d_wide<float>((float *)grid, coeffs, shape, steps, 2, false, st, tune);
    }
    if (shape.ndim == 2) {
        const bool box = kind == K_2D9;
        return dt == PERKS_F64 ? run2d<double>((double *)grid, coeffs, shape, steps, box, st, tune)
                               : run2d<float>((float *)grid, coeffs, shape, steps, box, st, tune);
    }
    return dt == PERKS_F64 ? run3d<double>((double *)grid, coeffs, shape, steps, st, tune)
                           : run3d<float>((float *)grid, coeffs, shape, steps, st, tune);
}

// Checks a batch (2D radius-1 grids of one pattern); box: the 9-point box.
int check_batch(void *const *grids, const perks_shape *shapes, int count, const double *coeffs, int64_t steps,
                perks_dtype dt, bool *box) {
    if (count < 0) return set_error(PERKS_E_INVAL, "count must be >= 0");
    if (count > 0 && (!grids || !shapes)) return set_error(PERKS_E_INVAL, "grids and shapes must not be NULL");
    Kind kind = K_2D5;
    for (int i = 0; i < count; ++i) {
        int rc = check_common(grids[i], coeffs, shapes[i], steps, dt);
        if (rc) return set_error(rc, "grid %d: %s", i, last_error());
        if (shapes[i].ndim != 2) return set_error(PERKS_E_UNSUPPORTED, "batched stencils are 2D");
        if (radius_of(shapes[i]) != 1) return set_error(PERKS_E_UNSUPPORTED, "batched stencils have radius 1");
        rc = classify(coeffs, shapes[i], &kind);
        if (rc) return rc;
    }
    *box = kind == K_2D9;
    return PERKS_OK;
}

}  // namespace
}  // namespace perks

using namespace perks;

extern "C" {

int perks_stencil_run(void *grid, const double *coeffs, perks_shape shape, int64_t steps, perks_dtype dt,
                      void *stream, const perks_tuning *tune) {
    int rc = check_common(grid, coeffs, shape, steps, dt);
    if (rc) return rc;
    rc = check_tuning(tune);
    if (rc) return rc;
    Kind kind;
    rc = classify(coeffs, shape, &kind);
    if (rc) return rc;
    if (steps == 0) return PERKS_OK;
    perks_tuning remembered;
    if (!tune && tuned_for(kind, dt, shape, &remembered)) tune = &remembered;
    return run_dispatch(grid, coeffs, shape, steps, dt, kind, as_stream(stream), tune);
}

int perks_stencil_run_noalloc(void *grid, const double *coeffs, perks_shape shape, int64_t steps, perks_dtype dt,
                              void *stream) {
    int rc = check_common(grid, coeffs, shape, steps, dt);
    if (rc) return rc;
    Kind kind;
    rc = classify(coeffs, shape, &kind);
    if (rc) return rc;
    if (shape.ndim != 2 || (kind != K_2D5 && kind != K_2D9))
        return set_error(PERKS_E_UNSUPPORTED, "perks_stencil_run_noalloc runs 2D radius-1 patterns only");
    if (steps == 0) return PERKS_OK;
    hipStream_t st = as_stream(stream);
    void *mem = nullptr;
    rc = noalloc_scratch(st, &mem);
    if (rc) return rc;
    const bool box = kind == K_2D9;
    return dt == PERKS_F64 ? run2d_in<double>((double *)grid, coeffs, shape, steps, box, st, mem, NOALLOC_BYTES)
                           : run2d_in<float>((float *)grid, coeffs, shape, steps, box, st, mem, NOALLOC_BYTES);
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
        const int r = is_wide(kind) ? wide_radius(kind) : 1;
        const bool box = kind == K_W2B || kind == K_2D9;
        return dt == PERKS_F64 ? baseline2d_wide<double>((double *)grid, coeffs, shape, steps, r, box, st)
                               : baseline2d_wide<float>((float *)grid, coeffs, shape, steps, r, box, st);
    }
    if (is_wide3(kind)) {
        return dt == PERKS_F64 ? baseline3d_wide<double>((double *)grid, coeffs, shape, steps, 2, false, st)
                               : baseline3d_wide<float>((float *)grid, coeffs, shape, steps, 2, false, st);
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
    rc = check_tuning(tune);
    if (rc) return rc;
    memset(plan, 0, sizeof(*plan));
    if (use_tb(kind, shape, dt, tune)) {
        const bool box = kind == K_2D9;
        return dt == PERKS_F64 ? plan2d_tb_query<double>(shape, box, tune, plan)
                               : plan2d_tb_query<float>(shape, box, tune, plan);
    }
    if (is_wide(kind) || use_wide_family(kind, shape, dt, tune)) {
        const int r = is_wide(kind) ? wide_radius(kind) : 1;
        const bool box = kind == K_W2B || kind == K_2D9;
        return dt == PERKS_F64 ? plan2d_wide_query<double>(shape, r, box, tune, plan)
                               : plan2d_wide_query<float>(shape, r, box, tune, plan);
    }
    if (is_wide3(kind)) {
        return dt == PERKS_F64 ? plan3d_wide_query<double>(shape, 2, false, tune, plan)
                               : plan3d_wide_query<float>(shape, 2, false, tune, plan);
    }
    if (shape.ndim == 2)
        return dt == PERKS_F64 ? plan2d_query<double>(shape, kind == K_2D9, tune, plan)
                               : plan2d_query<float>(shape, kind == K_2D9, tune, plan);
    return dt == PERKS_F64 ? plan3d_query<double>(shape, tune, plan) : plan3d_query<float>(shape, tune, plan);
}

int perks_stencil_run_batched(void *const *grids, const perks_shape *shapes, int32_t count, const double *coeffs,
                              int64_t steps, perks_dtype dt, void *stream) {
    bool box = false;
    int rc = check_batch(grids, shapes, count, coeffs, steps, dt, &box);
    if (rc) return rc;
    if (count == 0 || steps == 0) return PERKS_OK;
    hipStream_t st = as_stream(stream);
    return dt == PERKS_F64
               ? run2d_tb_batched<double>(reinterpret_cast<double *const *>(grids), shapes, count, coeffs, steps, box,
                                          st)
               : run2d_tb_batched<float>(reinterpret_cast<float *const *>(grids), shapes, count, coeffs, steps, box, st);
}

// The plan behind perks_stencil_batch: the batched kernel's plan and the
// device it was made on.
struct perks_stencil_batch {
    perks::StencilBatchPlan *plan = nullptr;
    int device = -1;
};

int perks_stencil_batch_create(void *const *grids, const perks_shape *shapes, int32_t count, const double *coeffs,
                               int64_t steps, perks_dtype dt, perks_stencil_batch **plan) {
    if (!plan) return set_error(PERKS_E_INVAL, "plan must not be NULL");
    *plan = nullptr;
    bool box = false;
    int rc = check_batch(grids, shapes, count, coeffs, steps, dt, &box);
    if (rc) return rc;
    auto *B = new (std::nothrow) perks_stencil_batch();
    if (!B) return set_error(PERKS_E_NOMEM, "plan allocation failed");
    (void)hipGetDevice(&B->device);
    if (count > 0) {
        rc = dt == PERKS_F64
                 ? tb_batch_create<double>(reinterpret_cast<double *const *>(grids), shapes, count, coeffs, steps, box,
                                           &B->plan)
                 : tb_batch_create<float>(reinterpret_cast<float *const *>(grids), shapes, count, coeffs, steps, box,
                                          &B->plan);
        if (rc) {
            delete B;
            return rc;
        }
    }
    *plan = B;
    return PERKS_OK;
}

int perks_stencil_batch_run(perks_stencil_batch *plan, void *stream) {
    if (!plan) return set_error(PERKS_E_INVAL, "plan must not be NULL");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != plan->device)
        return set_error(PERKS_E_INVAL, "the plan belongs to device %d", plan->device);
    return plan->plan ? tb_batch_run(plan->plan, as_stream(stream)) : PERKS_OK;
}

int perks_stencil_batch_graph(perks_stencil_batch *plan, void **graph) {
    if (!plan || !graph) return set_error(PERKS_E_INVAL, "plan and graph must not be NULL");
    if (!plan->plan) return set_error(PERKS_E_UNSUPPORTED, "an empty batch has no graph");
    return tb_batch_graph(plan->plan, graph);
}

int perks_stencil_batch_destroy(perks_stencil_batch *plan) {
    if (!plan) return PERKS_OK;
    tb_batch_destroy(plan->plan);
    delete plan;
    return PERKS_OK;
}

// The tuning table as text: a header line, then one line per entry of the
// current device: kind dtype nx ny nz and the eight perks_tuning fields.
int perks_tuning_save(const char *path) {
    if (!path) return set_error(PERKS_E_INVAL, "path must not be NULL");
    int dev = -1;
    (void)hipGetDevice(&dev);
    (void)hipGetLastError();
    std::vector<std::pair<TuneKey, perks_tuning>> rows;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (const auto &kv : g_tuned)
            if (std::get<0>(kv.first) == dev) rows.push_back(kv);
    }
    FILE *f = fopen(path, "w");
    if (!f) return set_error(PERKS_E_INVAL, "cannot open %s for writing", path);
    fprintf(f, "perks-tuning 1\n");
    for (const auto &kv : rows) {
        const perks_tuning &t = kv.second;
        fprintf(f, "%d %d %lld %lld %lld %d %d %d %d %d %d %d %d\n", std::get<1>(kv.first), std::get<2>(kv.first),
                (long long)std::get<3>(kv.first), (long long)std::get<4>(kv.first), (long long)std::get<5>(kv.first),
                t.waves_per_wg, t.wgs_per_cu, t.rows_per_lane, t.planes_per_lane, t.sync, t.max_cached_tiles,
                t.kernel, t.steps_per_sync);
    }
    const bool ok = !ferror(f);
    if (fclose(f) != 0 || !ok) return set_error(PERKS_E_INVAL, "writing %s failed", path);
    return PERKS_OK;
}

int perks_tuning_load(const char *path) {
    if (!path) return set_error(PERKS_E_INVAL, "path must not be NULL");
    FILE *f = fopen(path, "r");
    if (!f) return set_error(PERKS_E_INVAL, "cannot open %s", path);
    int dev = -1;
    (void)hipGetDevice(&dev);
    (void)hipGetLastError();
    char head[32] = {0};
    int version = 0;
    std::vector<std::pair<TuneKey, perks_tuning>> rows;
    bool ok = fscanf(f, "%31s %d", head, &version) == 2 && strcmp(head, "perks-tuning") == 0 && version == 1;
    while (ok) {
        int kind, dt;
        long long nx, ny, nz;
        perks_tuning t{};
        const int n = fscanf(f, "%d %d %lld %lld %lld %d %d %d %d %d %d %d %d", &kind, &dt, &nx, &ny, &nz,
                             &t.waves_per_wg, &t.wgs_per_cu, &t.rows_per_lane, &t.planes_per_lane, &t.sync,
                             &t.max_cached_tiles, &t.kernel, &t.steps_per_sync);
        if (n == EOF) break;
        if (n != 13 || kind < K_2D5 || kind > K_3S2 || (dt != PERKS_F32 && dt != PERKS_F64) || nx < 1 || ny < 1 ||
            nz < 1 || check_tuning(&t) != PERKS_OK) {
            ok = false;
            break;
        }
        rows.emplace_back(TuneKey(dev, kind, dt, nx, ny, nz), t);
    }
    fclose(f);
    if (!ok) return set_error(PERKS_E_INVAL, "%s is not a tuning file of this library (nothing loaded)", path);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto &kv : rows) g_tuned[kv.first] = kv.second;
    return PERKS_OK;
}

int perks_stencil_autotune(const double *coeffs, perks_shape shape, perks_dtype dt, int64_t probe_steps,
                           int32_t remember, void *stream, perks_tuning *best, double *best_gcells) {
    int dummy = 0;
    int rc = check_common(&dummy, coeffs, shape, 1, dt);
    if (rc) return rc;
    if (!best) return set_error(PERKS_E_INVAL, "best must not be NULL");
    if (probe_steps < 1) return set_error(PERKS_E_INVAL, "probe_steps must be >= 1");
    Kind kind;
    rc = classify(coeffs, shape, &kind);
    if (rc) return rc;
    // candidates: the planner's own choice and every forced depth, in each
    // synchronisation mode the kernels offer
    std::vector<perks_tuning> cands;
    auto add = [&](int rows, int planes, int sync, int kernel = 0, int k = 0) {
        perks_tuning t{};
        t.rows_per_lane = rows;
        t.planes_per_lane = planes;
        t.sync = sync;
        t.kernel = kernel;
        t.steps_per_sync = k;
        perks_stencil_plan pl;
        if (perks_stencil_plan_query(coeffs, shape, dt, &t, &pl) == PERKS_OK) cands.push_back(t);
    };
    if (is_wide(kind)) {
        add(0, 0, 0);
        for (int r : {24, 32, 48, 80}) add(r, 0, 1);
    } else if (is_wide3(kind)) {
        add(0, 0, 0);
    } else if (shape.ndim == 2) {
        for (int sync : {2, 1}) {
            add(0, 0, sync);
            for (int r : {8, 16, 32, 48, 64}) add(r, 0, sync);
        }
        // the radius-2..4 kernel family at radius 1
        add(0, 0, 1, 2);
        for (int r : {24, 32, 48, 80}) add(r, 0, 1, 2);
        // temporal blocking (a block's K steps per exchange): on small grids
        // the short tiles; on any grid the tall ones when every tile stays in
        // registers (their blocks would stream otherwise)
        if ((shape.nx - 2) * (shape.ny - 2) < WIDE_FAMILY_MIN_CELLS)
            for (int k : {2, 4, 8})
                for (int h : {8, 16}) add(h, 0, 0, 3, k);
        for (int k : {2, 4})
            for (int h : {32, 56}) {
                perks_tuning t{};
                t.rows_per_lane = h;
                t.kernel = 3;
                t.steps_per_sync = k;
                perks_stencil_plan pl;
                if (perks_stencil_plan_query(coeffs, shape, dt, &t, &pl) == PERKS_OK && pl.tiles > 0 &&
                    pl.cached_tiles == pl.tiles)
                    cands.push_back(t);
            }
    } else {
        add(0, 0, 0);
        for (int pz : {8, 16, 24, 32}) add(0, pz, 0);   // column depths
    }
    if (cands.empty()) return set_error(PERKS_E_UNSUPPORTED, "no candidate plan for this stencil");
    hipStream_t st = as_stream(stream);
    const int64_t cells = shape.nx * shape.ny * (shape.ndim == 3 ? shape.nz : 1);
    const size_t bytes = (size_t)cells * (dt == PERKS_F64 ? 8 : 4);
    void *g = nullptr;
    if (hipMalloc(&g, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(PERKS_E_NOMEM, "autotune: hipMalloc of %zu bytes failed", bytes);
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    double best_t = INFINITY;
    int best_i = -1;
    rc = PERKS_OK;
    do {
        if (hipMemsetAsync(g, 0, bytes, st) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
            hipEventCreate(&e1) != hipSuccess) {
            rc = set_error(PERKS_E_HIP, "autotune: event or memset failed");
            break;
        }
        for (size_t i = 0; i < cands.size(); ++i) {
            rc = run_dispatch(g, coeffs, shape, std::max<int64_t>(1, probe_steps / 4), dt, kind, st, &cands[i]);
            if (rc) break;
            if (hipEventRecord(e0, st) != hipSuccess) { rc = set_error(PERKS_E_HIP, "autotune: event record"); break; }
            rc = run_dispatch(g, coeffs, shape, probe_steps, dt, kind, st, &cands[i]);
            if (rc) break;
            float ms = 0.f;
            if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                rc = set_error(PERKS_E_HIP, "autotune: timing failed");
                break;
            }
            if (ms < best_t) {
                best_t = ms;
                best_i = (int)i;
            }
        }
    } while (false);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(st);
    (void)hipFree(g);
    if (rc) return rc;
    *best = cands[best_i];
    const int r = radius_of(shape);
    const int64_t interior = (shape.nx - 2 * r) * (shape.ny - 2 * r) * (shape.ndim == 3 ? shape.nz - 2 * r : 1);
    if (best_gcells) *best_gcells = (double)interior * probe_steps / (best_t * 1e-3) / 1e9;
    if (remember) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned[tune_key(kind, dt, shape)] = *best;
    }
    return PERKS_OK;
}

}  // extern "C"
