// sttsm without allocation: the workspace (X panels, temporaries) and the
// plan's index tables live in one static device array, for callers that
// cannot allocate device memory.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>

#include "abi_util.hpp"
#include "plan.hpp"

using namespace symt;

namespace {

// The array itself.  In host code its name stands for a host-side shadow,
// not a device address: host code uses only the per-device address that
// hipGetSymbolAddress returns.
static __device__ __align__(256) unsigned char scratch[STTSM_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::map<int, char *> g_scratch_ptr;   // device -> address of that device's copy

// Address of the current device's copy of the array, looked up once per
// device (with that device current).
char *scratch_address(std::string *why)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        *why = "hipGetDevice failed";
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) return it->second;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        *why = std::string("hipGetSymbolAddress of the static scratch array failed: ") + hipGetErrorString(e);
        return nullptr;
    }
    g_scratch_ptr[dev] = (char *)ptr;
    return (char *)ptr;
}

}  // namespace

extern "C" int sttsm_noalloc(const bcss_layout *A, const void *A_dev, const void *X_dev, int64_t rs_x, int64_t cs_x,
                             const bcss_layout *C, void *C_dev, int32_t prec, void *stream)
{
    PlanKey key;
    int rc = make_key(A, C, prec, &key);
    if (rc != STTSM_OK) return rc;
    if (!A_dev || !X_dev || !C_dev) return fail(STTSM_EINVAL, "null buffer");
    std::string why;
    const Plan *P = plan_get_host(key, &why);
    if (!P) return fail(STTSM_EINVAL, why);
    const size_t tab_bytes = P->tab_blob.size();   // a multiple of 256
    const size_t need = tab_bytes + P->ws_bytes;
    if (need > STTSM_NOALLOC_SCRATCH_BYTES)
        return fail(STTSM_EINVAL, "sttsm_noalloc: this problem needs " + std::to_string(need) +
                                      " bytes of scratch; the static array holds " +
                                      std::to_string((size_t)STTSM_NOALLOC_SCRATCH_BYTES));
    char *base = scratch_address(&why);
    if (!base) return fail(STTSM_EHIP, why);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // The tables first, then the workspace; the workspace needs no clearing
    // (every byte a level reads, an earlier kernel of the same call wrote).
    if (tab_bytes && hipMemcpyAsync(base, P->tab_blob.data(), tab_bytes, hipMemcpyHostToDevice, s) != hipSuccess)
        return fail(STTSM_EHIP, std::string("plan table copy failed: ") + hipGetErrorString(hipGetLastError()));
    return launch_levels(P, A, A_dev, X_dev, rs_x, cs_x, 0, C_dev, base + tab_bytes, base, s);
}
