// noalloc.hip -- kct_project_noalloc: the forward projection b := A x without
// any allocation, for callers that cannot allocate device memory (code under
// HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
//
// kct_project takes a caller-owned workspace for the z-fastest copy of the
// volume that its kernels read.  This entry point uses a fixed device array
// of this file instead, `scratch`, KCT_NOALLOC_SCRATCH_BYTES long, which every
// device the library runs on holds until the process ends.  Its device
// address is looked up once per device (hipGetSymbolAddress, with that device
// current) and kept; the kernels receive that address, never the host-side
// name of the array.  The copy overwrites every element the projector reads,
// so nothing needs clearing between calls.  All calls on one device share the
// array: calls that overlap in time on one device (different streams or host
// threads) race on it.
#include <mutex>

#include "../../include/kct.h"
#include "kct_internal.h"

namespace kct {

void set_error(const std::string &msg);

static __device__ __align__(256) unsigned char scratch[KCT_NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;

// Device address of `scratch` on `device` (which must be the current device),
// looked up on the first call for that device.
static hipError_t scratch_address(int device, void **ptr)
{
    static std::mutex mu;
    static void *addr[NOALLOC_MAX_DEVICES] = {};
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[device] = p;
    }
    *ptr = addr[device];
    return hipSuccess;
}

}  // namespace kct

extern "C" kct_status kct_project_noalloc(kct_geometry h, kct_dtype dtype, const void *x, void *b,
                                          hipStream_t stream)
{
    using namespace kct;
    if (!h) {
        set_error("kct_project_noalloc: geometry is NULL");
        return KCT_ERR_INVALID_ARG;
    }
    int64_t n_vox = 0, n_rays = 0;
    kct_status s = kct_geometry_dims(h, &n_vox, &n_rays);
    if (s != KCT_OK) return s;
    size_t elem = 0;
    switch (dtype) {
    case KCT_F32: elem = 4; break;
    case KCT_BF16:
    case KCT_F16: elem = 2; break;
    case KCT_F64: elem = 8; break;
    default:
        set_error("kct_project_noalloc: unknown storage type");
        return KCT_ERR_UNSUPPORTED;
    }
    if ((size_t)n_vox * elem > KCT_NOALLOC_SCRATCH_BYTES) {
        set_error("kct_project_noalloc: the volume (" + std::to_string((size_t)n_vox * elem) +
                  " bytes in this storage type) exceeds the fixed scratch of " +
                  std::to_string((size_t)KCT_NOALLOC_SCRATCH_BYTES) + " bytes; use kct_project with a workspace");
        return KCT_ERR_WORKSPACE;
    }
    int device = -1;
    if (hipGetDevice(&device) != hipSuccess) {
        set_error("kct_project_noalloc: hipGetDevice failed");
        return KCT_ERR_HIP;
    }
    void *ws = nullptr;
    const hipError_t e = scratch_address(device, &ws);
    if (e != hipSuccess) {
        set_error(std::string("kct_project_noalloc: hipGetSymbolAddress of the scratch array failed: ") +
                  hipGetErrorString(e));
        return KCT_ERR_HIP;
    }
    // the remaining checks (device of the geometry, pointers, alignment) and the
    // launches are kct_project's, with the scratch as its workspace
    return kct_project(h, dtype, x, b, ws, KCT_NOALLOC_SCRATCH_BYTES, stream);
}
