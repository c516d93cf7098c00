// helm_vcycle_noalloc: the shifted-Laplacian V-cycle of helm_vcycle with its
// scratch (the coarse levels' right-hand sides and corrections, and the
// coarsest level's FP64 polynomial buffers) in a fixed device array of this
// translation unit instead of library-allocated memory, for callers that
// cannot allocate (stream capture, allocation-free serving loops).
#include <mutex>

#include "internal.h"

namespace helm {
namespace {

constexpr size_t SCRATCH_BYTES = 32ull << 20;   // 32 MiB per GPU, held until the process ends
constexpr int MAX_DEVICES = 64;

// The array itself; host code uses only the device address that
// hipGetSymbolAddress returns for it (per device), never the name.
__device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

std::mutex g_scratch_mutex;
void* g_scratch_ptr[MAX_DEVICES] = {nullptr};

int scratch_address(void** out) {
    int dev = 0;
    HELM_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(HELM_EINVAL, "helm_vcycle_noalloc: device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(HELM_EHIP, "helm_vcycle_noalloc: hipGetSymbolAddress(scratch) failed: %s",
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return HELM_OK;
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace
}  // namespace helm

using namespace helm;

extern "C" size_t helm_vcycle_noalloc_max_bytes(void) { return SCRATCH_BYTES; }

extern "C" int helm_vcycle_noalloc(helm_op_t op, const void* f, void* e, int nrhs, void* stream) {
    if (!op || nrhs < 0) return fail(HELM_EINVAL, "helm_vcycle_noalloc: bad arguments");
    if (nrhs == 0) return HELM_OK;
    if (!f || !e) return fail(HELM_EINVAL, "helm_vcycle_noalloc: NULL buffer");
    // layout: per level l >= 1 the right-hand sides then the corrections (c64),
    // then three c128 buffers of the coarsest level
    size_t need = 0;
    size_t off_f[MAX_LEVELS] = {0}, off_e[MAX_LEVELS] = {0};
    for (int l = 1; l < op->nlev; ++l) {
        const size_t b = align256(sizeof(c64) * (size_t)nrhs * op->lv[l].n());
        off_f[l] = need;
        need += b;
        off_e[l] = need;
        need += b;
    }
    const size_t bc = align256(sizeof(c128) * (size_t)nrhs * op->lv[op->nlev - 1].n());
    const size_t off_c = need;
    need += 3 * bc;
    if (need > SCRATCH_BYTES)
        return fail(HELM_EINVAL,
                    "helm_vcycle_noalloc: %d right-hand sides of this grid need %zu bytes of scratch, above the "
                    "fixed %zu (use fewer right-hand sides per call, or helm_vcycle)",
                    nrhs, need, SCRATCH_BYTES);
    void* base = nullptr;
    int rc = scratch_address(&base);
    if (rc) return rc;
    unsigned char* p = (unsigned char*)base;
    MgWork<float> w;
    for (int l = 0; l < MAX_LEVELS; ++l) {
        w.f[l] = l >= 1 && l < op->nlev ? (c64*)(p + off_f[l]) : nullptr;
        w.e[l] = l >= 1 && l < op->nlev ? (c64*)(p + off_e[l]) : nullptr;
    }
    w.ra = (c128*)(p + off_c);
    w.rb = (c128*)(p + off_c + bc);
    w.xw = (c128*)(p + off_c + 2 * bc);
    return launch_vcycle<float>(op, (const c64*)f, nullptr, 0, (c64*)e, nullptr, nrhs, nullptr, 0, w,
                                (hipStream_t)stream);
}
