// Host runtime of libperks: error strings, per-device scratch memory, device
// facts.
#include <mutex>

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

int launch_coop(const void *fn, int wgs, int threads, void *params, hipStream_t st) {
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

}  // extern "C"
