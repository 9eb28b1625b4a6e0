// ftlm_lanczos_noalloc: ftlm_lanczos with its workspace in a device array
// that the library holds, for callers that cannot allocate device memory.
//
// The array below is the whole workspace (Lanczos vector blocks, FP64
// partials, chain state, alpha/beta, descriptors). Each GPU the library runs
// on holds its own copy until the process ends. Host code never uses the
// array's name as an address: the name is a host-side stand-in, so the device
// address is looked up once per device with hipGetSymbolAddress and kept.
#include <hip/hip_runtime.h>

#include <mutex>

#include "host.hpp"

namespace {

constexpr size_t kScratchBytes = FTLM_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of `scratch` on each device, once looked up

// The device address of `scratch` on the current device (looked up on the
// first call made with that device current).
int scratch_on_current_device(int* dev_out, void** out) {
    int dev = -1;
    HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return ftlm::fail(FTLM_E_RANGE, "device %d not in [0, %d)", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIP_CHECK(hipGetSymbolAddress(reinterpret_cast<void**>(&p), HIP_SYMBOL(scratch)));
        if (!p) return ftlm::fail(FTLM_E_DEVICE, "no device address for the no-alloc scratch on device %d", dev);
        g_scratch_ptr[dev] = p;
    }
    *dev_out = dev;
    *out = g_scratch_ptr[dev];
    return FTLM_OK;
}

}  // namespace

extern "C" int ftlm_lanczos_noalloc(const ftlm_sector* s, const ftlm_graph* g, uint64_t seed, uint64_t r0, int R,
                                    int M, int dist, int dtype, double* alpha_host, double* beta_host,
                                    int32_t* steps_host, void* stream) {
    using namespace ftlm;
    if (!s || !g || !alpha_host || !beta_host || !steps_host) return fail(FTLM_E_INVALID, "null argument");
    size_t need = 0;
    if (int rc = ftlm_lanczos_workspace_bytes(s, R, dtype, &need)) return rc;
    if (need > kScratchBytes)
        return fail(FTLM_E_RANGE,
                    "R = %d chains of a sector of dimension %llu need %zu bytes of workspace; the no-alloc scratch "
                    "holds %zu",
                    R, (unsigned long long)s->dim, need, kScratchBytes);
    int dev = -1;
    void* work = nullptr;
    if (int rc = scratch_on_current_device(&dev, &work)) return rc;
    // the sector's tables must sit on the device whose scratch is used
    hipPointerAttribute_t attr{};
    HIP_CHECK(hipPointerGetAttributes(&attr, s->table));
    if (attr.device != dev)
        return fail(FTLM_E_INVALID, "sector tables are on device %d, the current device is %d", attr.device, dev);
    return ftlm_lanczos(s, g, seed, r0, R, M, dist, dtype, work, kScratchBytes, alpha_host, beta_host, steps_host,
                        stream);
}
