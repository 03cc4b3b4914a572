// C ABI of libedt (declared in include/edt.h): argument validation, workspace
// layout and the launch sequence of one transform.
#include "../../include/edt.h"
#include "edt_internal.h"

#include <math.h>

#include <mutex>

namespace edt {
namespace {

// Workspace of edt_feature_noalloc: every device that runs this code object
// holds its own copy of the array until the process ends.  Host code never
// passes the array's name to a kernel or a copy (on the host it is only a
// stand-in for the device symbol): it looks up the array's device address
// once per device and uses that.
static __device__ __align__(256) uint8_t scratch[EDT_NOALLOC_SCRATCH_BYTES];

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices];  // device address of scratch, per device

// Device address of scratch on the current device, looked up on the first
// call there.
hipError_t scratch_address(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p || (reinterpret_cast<uintptr_t>(p) & 255) != 0) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

__global__ __launch_bounds__(256) void k_sqrt(const int32_t* __restrict__ D,
                                              float* __restrict__ out, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) {
        out[q] = __int_as_float(sqrt_bits(D[q]));
    }
}

}  // namespace

hipError_t launch_sqrt(const int32_t* D, float* out, int64_t n, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    EDT_LAUNCH(k_sqrt, dim3((unsigned)blocks), dim3(256), 0, stream, D, out, n);
    return launch_status();
}

edt_status check_image(const uint8_t* mask, int32_t H, int32_t W, int64_t mask_pitch,
                       int32_t polarity, int32_t metric, int64_t out_pitch) {
    if (H < 1 || W < 1 || H > EDT_MAX_SIDE || W > EDT_MAX_SIDE) return EDT_ERR_TOO_LARGE;
    if (!mask || mask_pitch < W || out_pitch < W) return EDT_ERR_INVALID_ARG;
    if (polarity != EDT_TO_OBJECT && polarity != EDT_TO_BACKGROUND) return EDT_ERR_INVALID_ARG;
    if (metric < 0 || metric > EDT_METRIC_CHAMFER34) return EDT_ERR_INVALID_ARG;
    return EDT_OK;
}

static edt_status run(const uint8_t* mask, int32_t H, int32_t W, int64_t mask_pitch,
                      int32_t polarity, int32_t metric, int32_t* dist, int32_t* feat,
                      int64_t out_pitch, void* workspace, size_t workspace_bytes,
                      void* stream, bool fsq = false) {
    edt_status st = check_image(mask, H, W, mask_pitch, polarity, metric, out_pitch);
    if (st != EDT_OK) return st;
    if (!dist && !feat) return EDT_ERR_INVALID_ARG;
    const Layout L = layout_for(H, W);
    if (!workspace || workspace_bytes < L.total) return EDT_ERR_INVALID_ARG;
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return EDT_ERR_INVALID_ARG;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    Img g;
    g.mask = mask;
    g.mpitch = mask_pitch;
    g.dist = dist;
    g.feat = feat;
    g.opitch = out_pitch;
    g.ws = static_cast<uint8_t*>(workspace);
    g.H = H;
    g.W = W;
    g.pol = polarity;
    g.metric = metric;
    g.fsq = fsq ? 1 : 0;
    return enqueue_single(g, s) == hipSuccess ? EDT_OK : EDT_ERR_DEVICE;
}

hipError_t enqueue_single(const Img& g, hipStream_t stream) {
    hipError_t e = launch_column_pass(g, stream);
    if (e == hipSuccess) e = launch_row_pass(g, g.ws + layout_for(g.H, g.W).slots, stream);
    return e;
}

}  // namespace edt

extern "C" {

int32_t edt_abi_version(void) { return EDT_ABI_VERSION; }

const char* edt_status_string(edt_status s) {
    switch (s) {
        case EDT_OK: return "ok";
        case EDT_ERR_INVALID_ARG: return "invalid argument";
        case EDT_ERR_UNSUPPORTED: return "unsupported metric";
        case EDT_ERR_TOO_LARGE: return "image too large";
        case EDT_ERR_OUT_OF_MEMORY: return "out of memory";
        case EDT_ERR_BUSY: return "busy";
        case EDT_ERR_NOT_READY: return "not ready";
        case EDT_ERR_DEVICE: return "device error";
        default: return "unknown status";
    }
}

size_t edt_workspace_bytes(int32_t H, int32_t W, int32_t want_feature) {
    (void)want_feature;
    if (H < 1 || W < 1 || H > EDT_MAX_SIDE || W > EDT_MAX_SIDE) return 0;
    return edt::layout_for(H, W).total;
}

edt_status edt_sq(const uint8_t* mask, int32_t H, int32_t W, int64_t mask_pitch,
                  int32_t polarity, int32_t metric, int32_t* dist_sq, int64_t out_pitch,
                  void* workspace, size_t workspace_bytes, void* stream) {
    if (!dist_sq) return EDT_ERR_INVALID_ARG;
    return edt::run(mask, H, W, mask_pitch, polarity, metric, dist_sq, nullptr, out_pitch,
                    workspace, workspace_bytes, stream);
}

edt_status edt_feature(const uint8_t* mask, int32_t H, int32_t W, int64_t mask_pitch,
                       int32_t polarity, int32_t metric, int32_t* dist_sq,
                       int32_t* feature, int64_t out_pitch, void* workspace,
                       size_t workspace_bytes, void* stream) {
    if (!feature) return EDT_ERR_INVALID_ARG;
    return edt::run(mask, H, W, mask_pitch, polarity, metric, dist_sq, feature, out_pitch,
                    workspace, workspace_bytes, stream);
}

edt_status edt_feature_noalloc(const uint8_t* mask, int32_t H, int32_t W, int64_t mask_pitch,
                               int32_t polarity, int32_t metric, int32_t* dist_sq,
                               int32_t* feature, int64_t out_pitch, void* stream) {
    if (!feature) return EDT_ERR_INVALID_ARG;
    // the size limit first, so that a refused call touches no device state
    if (H >= 1 && W >= 1 && H <= EDT_MAX_SIDE && W <= EDT_MAX_SIDE &&
        edt::layout_for(H, W).total > (size_t)EDT_NOALLOC_SCRATCH_BYTES)
        return EDT_ERR_TOO_LARGE;
    const edt_status st = edt::check_image(mask, H, W, mask_pitch, polarity, metric, out_pitch);
    if (st != EDT_OK) return st;
    void* ws = nullptr;
    if (edt::scratch_address(&ws) != hipSuccess) return EDT_ERR_DEVICE;
    return edt::run(mask, H, W, mask_pitch, polarity, metric, dist_sq, feature, out_pitch, ws,
                    (size_t)EDT_NOALLOC_SCRATCH_BYTES, stream);
}

edt_status edt_dist_f32(const uint8_t* mask, int32_t H, int32_t W, int64_t mask_pitch,
                        int32_t polarity, float* dist, int32_t* feature, int64_t out_pitch,
                        void* workspace, size_t workspace_bytes, void* stream) {
    if (!dist) return EDT_ERR_INVALID_ARG;
    return edt::run(mask, H, W, mask_pitch, polarity, EDT_METRIC_EUCLIDEAN_SQ,
                    reinterpret_cast<int32_t*>(dist), feature, out_pitch, workspace,
                    workspace_bytes, stream, true);
}

edt_status edt_sqrt_f32(const int32_t* dist_sq, float* dist, int64_t n, void* stream) {
    if (n < 0 || (n > 0 && (!dist_sq || !dist))) return EDT_ERR_INVALID_ARG;
    if (edt::launch_sqrt(dist_sq, dist, n, reinterpret_cast<hipStream_t>(stream)) !=
        hipSuccess)
        return EDT_ERR_DEVICE;
    return EDT_OK;
}

}  // extern "C"
