// Search entry point for callers that cannot allocate device memory (code
// that must not call hipMalloc: tight serving loops, harnesses that forbid
// it).  Every buffer of the search (frontier levels, chain queues, hit
// records, sort buffers, counters) is cut from one file-scope device array of
// kScratchBytes; each GPU the library runs on holds its own copy of the array
// until the process ends.
//
// Host code never passes the array's name to a kernel or a copy: on the host
// it is only a stand-in for the symbol.  At the first call on a device, with
// that device current, hipGetSymbolAddress gives the array's address there,
// which is kept per device and is the only way host code reaches it.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "alae_internal.h"

namespace {
constexpr uint64_t kScratchBytes = ALAE_NOALLOC_SCRATCH_BYTES;  // per device
constexpr int kMaxDevices = 64;
}  // namespace

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {

struct DeviceScratch {
    std::mutex mu;                  // calls on one device take turns: they share the array
    bool ready = false;
    uint8_t *ptr = nullptr;         // address of `scratch` on this device
    alae_workspace *ws = nullptr;   // workspace whose buffers all live in that array
};

DeviceScratch g_dev[kMaxDevices];

}  // namespace

extern "C" {

alae_status alae_search_device_noalloc(const alae_index *index, const uint8_t *d_query_codes, size_t m,
                                       const alae_scoring *scoring, int32_t H, const alae_search_opts *opts,
                                       void *stream, uint64_t *d_keys, int32_t *d_scores, size_t capacity,
                                       size_t *hit_count) {
    using namespace alae;
    if (!index || !d_query_codes || !hit_count || (capacity > 0 && (!d_keys || !d_scores))) {
        set_error("alae_search_device_noalloc: null argument");
        return ALAE_E_ARG;
    }
    const int dev = index->device;
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("alae_search_device_noalloc: device %d is outside 0..%d", dev, kMaxDevices - 1);
        return ALAE_E_ARG;
    }
    DeviceScratch &d = g_dev[dev];
    std::lock_guard<std::mutex> lock(d.mu);
    if (!d.ready) {
        hipError_t e = hipSetDevice(dev);
        if (e == hipSuccess) {
            void *p = nullptr;
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e == hipSuccess) d.ptr = static_cast<uint8_t *>(p);
        }
        if (e != hipSuccess || !d.ptr) {
            hipGetLastError();
            set_error("alae_search_device_noalloc: no address for the scratch array on device %d: %s", dev,
                      hipGetErrorString(e));
            return ALAE_E_DEVICE;
        }
        const alae_status st = region_workspace_create(dev, d.ptr, kScratchBytes, &d.ws);
        if (st != ALAE_OK) return st;
        d.ready = true;
    }
    uint64_t cnt = 0;
    const alae_status st = region_search(d.ws, index, d_query_codes, m, scoring, H, opts, stream, d_keys, d_scores,
                                         capacity, &cnt);
    if (st == ALAE_OK || (st == ALAE_E_NOMEM && cnt > capacity)) *hit_count = (size_t)cnt;
    return st;
}

}  // extern "C"
