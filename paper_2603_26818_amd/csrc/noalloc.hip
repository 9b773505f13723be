// noalloc.hip -- pfc_step_noalloc: the PFC step for callers that cannot allocate device memory.
//
// pfc_step needs device memory beyond psi and the state: the twiddle tables and one scratch
// spectrum, which the plan's caller-allocated workspace holds.  This variant keeps both in a
// file-scope device array instead (one copy per GPU, held until the process ends), so a call
// allocates nothing.  The kernels and their arguments are those of pfc_step, so the results are
// the same bits.
#include <hip/hip_runtime.h>

#include <mutex>

#include "api_internal.hpp"

namespace {

constexpr size_t kTableBytes = size_t(1) << 20;      // twiddle tables of any supported plan (<= 0.6 MiB)
constexpr size_t kSpectrumBytes = size_t(64) << 20;  // one native spectrum: up to 256^3 FP32
constexpr size_t kScratchBytes = kTableBytes + kSpectrumBytes;
constexpr int kMaxDevices = 64;

// The tables at offset 0, the scratch spectrum at kTableBytes.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Per device: the array's device address (from hipGetSymbolAddress, taken once with the device
// current) and the id of the plan whose tables it holds.
struct DeviceArea {
    char *ptr = nullptr;
    uint64_t tables_of = 0;
};
std::mutex g_mu;
DeviceArea g_area[kMaxDevices];

struct CurrentDevice {
    int prev = -1;
    hipError_t err = hipSuccess;
    explicit CurrentDevice(int dev)
    {
        err = hipGetDevice(&prev);
        if (err == hipSuccess && prev != dev) err = hipSetDevice(dev);
    }
    ~CurrentDevice()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

}  // namespace

extern "C" pfc_status pfc_step_noalloc(pfc_plan *p, void *psi, void *state, int64_t nsteps, void *stream)
{
    pfc_status st = pfc_internal::check_step_args(p, psi, state, nsteps);
    if (st != PFC_OK) return st;
    if (pfc_internal::spectrum_bytes(p) > kSpectrumBytes || pfc_internal::table_bytes(p) > kTableBytes)
        return pfc_internal::report(PFC_ERR_WORKSPACE,
                                    "pfc_step_noalloc: the grid's scratch spectrum exceeds the static 64 MiB "
                                    "(at most 256^3 FP32 or 2^23 FP64 points); use pfc_step with a workspace");
    const int dev = pfc_internal::plan_device(p);
    if (dev >= kMaxDevices) return pfc_internal::report(PFC_ERR_INVALID_ARG, "pfc_step_noalloc: device ordinal >= 64");
    CurrentDevice cd(dev);
    if (cd.err != hipSuccess) return pfc_internal::report(PFC_ERR_HIP, "pfc_step_noalloc: hipSetDevice failed");
    std::lock_guard<std::mutex> lock(g_mu);
    DeviceArea &a = g_area[dev];
    if (!a.ptr) {
        void *addr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !addr)
            return pfc_internal::report(PFC_ERR_HIP, "pfc_step_noalloc: hipGetSymbolAddress of the scratch array failed");
        a.ptr = static_cast<char *>(addr);
    }
    // the step reads the tables and fully writes the spectrum before reading it, so nothing needs
    // clearing; the tables are copied only when another plan's are there
    if (a.tables_of != pfc_internal::plan_id(p)) {
        st = pfc_internal::upload_tables(p, a.ptr, stream);
        if (st != PFC_OK) return st;
        a.tables_of = pfc_internal::plan_id(p);
    }
    return pfc_internal::step_with_buffers(p, psi, state, nsteps, stream, a.ptr, a.ptr + kTableBytes);
}
