// Host runtime of libperks: error strings, per-device scratch memory, device
// facts.
#include <algorithm>
#include <mutex>
#include <vector>

#include "common.hpp"

namespace perks {

namespace {
thread_local char g_last_error[1024] = "no error";

struct ScratchBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
};
constexpr int kMaxDevices = 64;
ScratchBuf g_scratch[kMaxDevices][SLOT_COUNT];
DeviceFacts g_facts[kMaxDevices];
std::mutex g_mu;
}  // namespace

int set_error(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
    return code;
}

const char *last_error() { return g_last_error; }

void *scratch(int slot, size_t bytes) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices || slot < 0 || slot >= SLOT_COUNT) {
        set_error(PERKS_E_HIP, "scratch: no current HIP device");
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    ScratchBuf &b = g_scratch[dev][slot];
    if (b.bytes >= bytes && b.ptr) return b.ptr;
    if (b.ptr) {
        // the old buffer may still be in use by queued work
        if (hipDeviceSynchronize() != hipSuccess || hipFree(b.ptr) != hipSuccess) {
            set_error(PERKS_E_HIP, "scratch: freeing the old buffer failed");
            return nullptr;
        }
        b.ptr = nullptr;
        b.bytes = 0;
    }
    size_t want = bytes < 4096 ? 4096 : bytes;
    want = (want + 65535) & ~size_t(65535);
    void *p = nullptr;
    if (hipMalloc(&p, want) != hipSuccess) {
        (void)hipGetLastError();
        set_error(PERKS_E_NOMEM, "scratch: hipMalloc of %zu bytes failed", want);
        return nullptr;
    }
    // Barrier words and every other scratch start zeroed; the barrier relies
    // on it (epoch 0), the other slots are fully written before being read.
    if (hipMemset(p, 0, want) != hipSuccess) {
        set_error(PERKS_E_HIP, "scratch: hipMemset failed");
        return nullptr;
    }
    b.ptr = p;
    b.bytes = want;
    return p;
}

int device_facts(DeviceFacts *out) {
    int dev = 0;
    PERKS_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return set_error(PERKS_E_HIP, "device index %d out of range", dev);
    {
        std::lock_guard<std::mutex> lock(g_mu);
        if (g_facts[dev].device == dev) {
            *out = g_facts[dev];
            return PERKS_OK;
        }
    }
    hipDeviceProp_t prop;
    PERKS_HIP_TRY(hipGetDeviceProperties(&prop, dev));
    DeviceFacts f;
    f.device = dev;
    f.cus = prop.multiProcessorCount;
    f.lds_per_cu = (int)prop.maxSharedMemoryPerMultiProcessor;
    f.regs_per_cu = prop.regsPerMultiprocessor;
    f.l2 = prop.l2CacheSize;
    f.hbm = prop.totalGlobalMem;
    snprintf(f.arch, sizeof(f.arch), "%s", prop.gcnArchName);
    std::lock_guard<std::mutex> lock(g_mu);
    g_facts[dev] = f;
    *out = f;
    return PERKS_OK;
}

namespace {
// grid size and barrier words (NULL: the shared ones) of the last persistent
// launch per device
int g_last_wgs[kMaxDevices];
unsigned *g_last_ws[kMaxDevices];
}

void note_persistent_launch(int wgs, unsigned *ws) {
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < kMaxDevices) {
        std::lock_guard<std::mutex> lock(g_mu);
        g_last_wgs[dev] = wgs;
        g_last_ws[dev] = ws;
    }
}

void forget_persistent_launch(unsigned *ws) {
    std::lock_guard<std::mutex> lock(g_mu);
    for (int d = 0; d < kMaxDevices; ++d)
        if (g_last_ws[d] == ws) {
            g_last_wgs[d] = 0;
            g_last_ws[d] = nullptr;
        }
}

int read_barrier_stats(int G, unsigned *ws, hipStream_t st, perks_barrier_stats_t *out) {
    memset(out, 0, sizeof(*out));
    if (G <= 0) return PERKS_OK;
    if (G > SYNC_MAX_WGS) return set_error(PERKS_E_INVAL, "barrier stats: %d workgroups", G);
    if (!ws) ws = (unsigned *)scratch(SLOT_SYNC, SYNC_BYTES);
    if (!ws) return PERKS_E_NOMEM;
    std::vector<unsigned long long> rec((size_t)G * SYNC_STATS_WORDS);
    PERKS_HIP_TRY(hipMemcpyAsync(rec.data(), ws + SYNC_STATS, rec.size() * sizeof(unsigned long long),
                                 hipMemcpyDeviceToHost, st));
    PERKS_HIP_TRY(hipStreamSynchronize(st));
    double wait = 0, total = 0, count = 0, wmax = 0;
    for (int g = 0; g < G; ++g) {
        const unsigned long long *r = &rec[(size_t)g * SYNC_STATS_WORDS];
        wait += (double)r[0];
        total += (double)r[1];
        count += (double)r[2];
        wmax = std::max(wmax, (double)r[0]);
    }
    out->wgs = G;
    out->barriers = (int64_t)(count / G + 0.5);
    out->wait_cycles = wait / G;
    out->max_wait_cycles = wmax;
    out->total_cycles = total / G;
    out->wait_share = total > 0 ? wait / total : 0.0;
    return PERKS_OK;
}

int launch_coop(const void *fn, int wgs, int threads, void *params, hipStream_t st) {
    note_persistent_launch(wgs, nullptr);
    void *args[] = {params};
    hipError_t e = hipLaunchCooperativeKernel(fn, dim3(wgs), dim3(threads), args, 0, st);
    if (e == hipErrorCooperativeLaunchTooLarge) {
        (void)hipGetLastError();
        return set_error(PERKS_E_NOTCORESIDENT, "cooperative launch of %d workgroups x %d threads is too large", wgs,
                         threads);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_error(PERKS_E_HIP, "hipLaunchCooperativeKernel: %s", hipGetErrorString(e));
    }
    return PERKS_OK;
}

}  // namespace perks

extern "C" {

const char *perks_strerror(int code) {
    switch (code) {
        case PERKS_OK: return "success";
        case PERKS_NOT_CONVERGED: return "not converged within maxit";
        case PERKS_BREAKDOWN: return "breakdown (matrix not SPD or non-finite value)";
        case PERKS_E_INVAL: return "invalid argument";
        case PERKS_E_NOMEM: return "out of device memory";
        case PERKS_E_HIP: return "HIP runtime error";
        case PERKS_E_NOTCORESIDENT: return "persistent grid cannot be co-resident";
        case PERKS_E_UNSUPPORTED: return "unsupported configuration";
        default: return "unknown error code";
    }
}

const char *perks_last_error(void) { return perks::last_error(); }

int perks_device_query(perks_device_info *info) {
    if (!info) return perks::set_error(PERKS_E_INVAL, "perks_device_query: info is NULL");
    perks::DeviceFacts f;
    int rc = perks::device_facts(&f);
    if (rc) return rc;
    info->cus = f.cus;
    info->lds_per_cu = f.lds_per_cu;
    info->regs_per_cu = f.regs_per_cu;
    info->l2_bytes = f.l2;
    info->hbm_bytes = (int64_t)f.hbm;
    snprintf(info->arch, sizeof(info->arch), "%s", f.arch);
    return PERKS_OK;
}

int perks_barrier_stats(void *stream, perks_barrier_stats_t *out) {
    if (!out) return perks::set_error(PERKS_E_INVAL, "perks_barrier_stats: out is NULL");
    memset(out, 0, sizeof(*out));
    int dev = 0;
    PERKS_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= perks::kMaxDevices) return perks::set_error(PERKS_E_HIP, "device index out of range");
    int G;
    unsigned *ws;
    {
        std::lock_guard<std::mutex> lock(perks::g_mu);
        G = perks::g_last_wgs[dev];
        ws = perks::g_last_ws[dev];
    }
    return perks::read_barrier_stats(G, ws, (hipStream_t)stream, out);
}

}  // extern "C"
