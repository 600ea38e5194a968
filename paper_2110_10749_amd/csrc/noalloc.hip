// The allocation-free entry point: a Stokes layer sum of a surface staged
// into a fixed device array of the library instead of a caller's workspace.
//
// The array lives in device memory of every GPU the library runs on, for the
// life of the process.  In host code its name only stands for the device
// symbol; the device address is taken once per device with
// hipGetSymbolAddress (with that device current) and kept, and only that
// address is handed to kernels.  Every call on one device reuses its array:
// staging rewrites all node data, masks and boxes, the pass kernels write
// every partial slot they later read, and the flags and counters are cleared
// by fill kernels.  Calls that overlap in time on one device race on it.
#include <cmath>
#include <mutex>
#include <string>

#include "solver.h"

namespace sdbie {
namespace {

// the largest surface the array holds, and the source splits of its passes
// (the staged copies, tile masks, Morton keys, source records and partial
// slots of a layer sum of 32768 nodes at 8 splits take 22.9 MB)
constexpr int64_t kStaticMaxNodes = SDBIE_NOALLOC_MAX_NODES;
constexpr int kStaticSplits = 8;
constexpr size_t kStaticScratchBytes = (size_t)24 << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// device address of this device's copy of the array (taken once per device)
void* scratch_address() {
    int dev = 0;
    SDBIE_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) throw Error(SDBIE_ERR_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            throw Error(SDBIE_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

void stokes_layer_apply_static(const sdbie_surface* s, double mu, sdbie_layer layer, const double* dens,
                               double* out, sdbie_precision prec, hipStream_t st) {
    if (!s || !s->x || !s->nrm || !s->w) throw Error(SDBIE_ERR_ARG, "null surface array");
    if (s->n < 1 || s->n > kStaticMaxNodes)
        throw Error(SDBIE_ERR_ARG, "n must lie in [1, " + std::to_string(kStaticMaxNodes) +
                                       "] for the allocation-free layer sum (use a plan for larger surfaces)");
    if (!(std::isfinite(s->delta) && s->delta >= kMinDelta && s->delta <= kMaxCoord))
        throw Error(SDBIE_ERR_ARG, "delta must lie in [1e-15, 1e15]");
    if (layer_workspace_bytes(s->n, kStaticSplits) > kStaticScratchBytes)
        throw Error(SDBIE_ERR_WORKSPACE, "the static scratch array is too small for this surface");
    void* base = scratch_address();
    Plan P;  // host bookkeeping only; every device buffer is carved out of the array
    P.n = s->n;
    P.max_restart = 1;
    P.delta = s->delta;
    double* in = nullptr;
    carve_layer_workspace(P, base, kStaticSplits, &in);
    stage_surface(P, s, st);
    apply_stokes_layer(P, mu, layer, dens, out, prec, st, in);
}

}  // namespace sdbie
