// nz_static.hip -- nz_sweep_batch_static: the batch sweep run inside a device
// buffer that the library owns for the life of the process, for callers that
// must not allocate device memory (code being captured into a HIP graph, tight
// serving loops, hosts that forbid allocation calls).
//
// The buffer is a file-scope __device__ array.  Host code never passes the
// array's name to a kernel or a copy: on the host that name is only a stand-in
// for the symbol, so the first call on each device looks up the array's device
// address with hipGetSymbolAddress (with that device current) and every later
// use goes through that address.  Each device holds its own copy.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <mutex>

#include "../../include/nz.h"
#include "nz_launch.h"

#define NZ_API extern "C" __attribute__((visibility("default")))

namespace {

constexpr size_t kScratchBytes = NZ_STATIC_SCRATCH_BYTES;

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

struct DeviceScratch {
    uint8_t *ptr = nullptr;   // device address of this device's copy of scratch
    std::mutex call;          // one call at a time uses a device's copy
};

std::mutex g_map_lock;
std::map<int, std::unique_ptr<DeviceScratch>> g_scratch;   // kept until the process ends

int scratch_of(int device, DeviceScratch **out)
{
    std::lock_guard<std::mutex> g(g_map_lock);
    auto &slot = g_scratch[device];
    if (!slot) {
        // the caller made `device` current before asking
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            g_scratch.erase(device);
            return nz::set_error(NZ_EDEVICE, "hipGetSymbolAddress of the static buffer failed");
        }
        if (reinterpret_cast<uintptr_t>(p) % 256) {
            g_scratch.erase(device);
            return nz::set_error(NZ_EDEVICE, "the static buffer is not 256-byte aligned");
        }
        slot.reset(new DeviceScratch);
        slot->ptr = static_cast<uint8_t *>(p);
    }
    *out = slot.get();
    return NZ_OK;
}

}  // namespace

NZ_API int nz_sweep_batch_static(const nz_job *jobs, int32_t njobs, int32_t *d_nstar, int32_t *d_mass,
                                 int32_t *h_backoffs, const nz_tuning *tune, void *stream)
{
    // every size check happens before the first device call
    if (int rc = nz::check_batch_fits(jobs, njobs, tune, kScratchBytes)) return rc;
    int64_t total = 0;
    for (int j = 0; j < njobs; ++j) total += jobs[j].nsamples;
    if (total > 0 && !d_nstar) return nz::set_error(NZ_EINVAL, "n* output is NULL");
    if (total == 0) return nz::run_batch_one_group(jobs, njobs, nullptr, 0, d_nstar, d_mass, h_backoffs, tune,
                                                   static_cast<hipStream_t>(stream));
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return nz::set_error(NZ_EDEVICE, "hipGetDevice failed");
    DeviceScratch *s = nullptr;
    if (int rc = scratch_of(device, &s)) return rc;
    std::lock_guard<std::mutex> g(s->call);
    return nz::run_batch_one_group(jobs, njobs, s->ptr, kScratchBytes, d_nstar, d_mass, h_backoffs, tune,
                                   static_cast<hipStream_t>(stream));
}

NZ_API size_t nz_static_scratch_bytes(void) { return kScratchBytes; }
