// noalloc.hip -- pcf_pairwise_lp_noalloc: the L_p / Gram matrix call with its
// workspace (tile plan and packed breakpoint records) in a device array the
// library holds, for callers that cannot allocate device memory.
//
// The array `scratch` is a file-scope device variable: every GPU the library
// runs on holds its own copy, from module load until the process ends. Host
// code never passes the variable itself to a kernel (on the host it is only
// a stand-in); the first call on a device, with that device current, looks
// up the copy's device address with hipGetSymbolAddress and keeps it per
// device. Every call on a device shares that device's array and overwrites
// the plan and records it holds, so calls that overlap on one device (other
// streams, other host threads) race; calls in one stream are ordered.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "pcf.h"
#include "plan.hpp"

namespace pcf {
pcf_status noalloc_fail(pcf_status s, const std::string &msg);
pcf_status noalloc_forward(const pcf_set *X, pcf_kind kind, double p, void *out,
                           int64_t ldo, const pcf_window *w, void *ws,
                           size_t ws_bytes, uint32_t flags, void *stream);
pcf_status noalloc_plan_bytes(const pcf_set *X, const pcf_window *w, int64_t ldo,
                              uint32_t flags, int64_t *bytes);
}  // namespace pcf

using namespace pcf;

namespace {

constexpr size_t kScratchBytes = PCF_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {nullptr};

// Device address of the current device's copy of `scratch` (looked up once
// per device).
pcf_status scratch_address(void **ptr)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return noalloc_fail(PCF_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return noalloc_fail(PCF_EDEVICE, "device index beyond the library's table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return noalloc_fail(PCF_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                                 hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return PCF_OK;
}

}  // namespace

extern "C" pcf_status pcf_pairwise_lp_noalloc(const pcf_set *X, pcf_kind kind, double p,
                                              void *out, int64_t ldo, const pcf_window *w,
                                              uint32_t flags, void *stream)
{
    if (kind != PCF_LP && kind != PCF_LP_POW && kind != PCF_GRAM)
        return noalloc_fail(PCF_EINVAL, "kind must be PCF_LP, PCF_LP_POW or PCF_GRAM");
    if (flags & (PCF_REUSE_PLAN | PCF_RECORDS_PACKED))
        return noalloc_fail(PCF_EINVAL, "the shared scratch keeps no plan between calls: "
                                        "PCF_REUSE_PLAN and PCF_RECORDS_PACKED are refused");
    if (X && X->n > 0) {
        // the plan's exact workspace, checked before any device work
        int64_t need = 0;
        pcf_status st = noalloc_plan_bytes(X, w, ldo, flags, &need);
        if (st != PCF_OK)
            return st;
        if (need > (int64_t)kScratchBytes)
            return noalloc_fail(PCF_ENOMEM,
                                "the call needs " + std::to_string(need) +
                                    " bytes of workspace; the library's scratch holds " +
                                    std::to_string((long long)kScratchBytes) +
                                    " (use pcf_pairwise_lp with a caller workspace)");
    }
    void *ws = nullptr;
    if (X && X->n > 0) {
        pcf_status st = scratch_address(&ws);
        if (st != PCF_OK)
            return st;
    }
    return noalloc_forward(X, kind, p, out, ldo, w, ws, kScratchBytes, flags, stream);
}
