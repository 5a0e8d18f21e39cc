// mmm_multiply_noalloc: mmm_multiply with the workspace taken from a
// library-owned device array instead of a caller allocation, for callers
// that cannot allocate device memory (code under stream capture, tight
// serving loops, hosts that forbid allocation on the hot path).
//
// The array lives in this file as a file-scope __device__ variable, so each
// device the library runs on holds its own copy (allocated when the code
// object is loaded there) until the process ends.  Host code never passes
// the array's name to a kernel: in host code that name denotes a host-side
// stand-in.  The device address is obtained once per device, with that
// device current, through hipGetSymbolAddress and kept in a per-device
// table; every later call on that device uses the kept address.
//
// Every method's kernels treat the workspace as uninitialised on entry and
// clear (with fill kernels) whatever must start at zero, so the contents a
// previous call left behind never reach a result.  Calls that overlap in
// time on one device share the array and race: the caller serialises them
// (one stream, or events between streams).
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/mmm.h"
#include "launch.h"

namespace {

constexpr size_t kScratchBytes = (size_t)MMM_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[MMM_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of `scratch` per device, null until looked up

// Device address of this device's scratch array (looked up on the first
// call on the device, with the device current).
mmm_status scratch_for_current_device(void** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return mmm::set_error(MMM_ELAUNCH, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return mmm::set_error(MMM_EUNSUPPORTED, "device %d beyond the scratch table", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return mmm::set_error(MMM_ELAUNCH, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                                  hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return MMM_OK;
}

}  // namespace

extern "C" {

size_t mmm_noalloc_scratch_bytes(void) { return kScratchBytes; }

mmm_status mmm_multiply_noalloc(const double* A, const double* B, double* C, int64_t N, int64_t P, int64_t M,
                                mmm_method method, const mmm_config* cfg, void* stream)
{
    // the size check first: a product whose workspace does not fit is
    // refused before the scratch is looked up or anything is enqueued
    size_t need = 0;
    if (N > 0 && P > 0 && M > 0 && (int)method >= 0 && (int)method < MMM_METHOD_COUNT) {
        need = mmm_workspace_bytes(method, N, P, M, cfg);
        if (need != (size_t)-1 && need > kScratchBytes)
            return mmm::set_error(MMM_EWORKSPACE,
                                  "mmm_multiply_noalloc: this product needs %zu bytes of workspace; the static "
                                  "scratch holds %zu",
                                  need, kScratchBytes);
    }
    // products that need no workspace do not touch the scratch array
    if (need == 0 || need == (size_t)-1) return mmm_multiply(A, B, C, N, P, M, method, cfg, nullptr, 0, stream);
    void* ws = nullptr;
    mmm_status st = scratch_for_current_device(&ws);
    if (st != MMM_OK) return st;
    return mmm_multiply(A, B, C, N, P, M, method, cfg, ws, kScratchBytes, stream);
}

}  // extern "C"
