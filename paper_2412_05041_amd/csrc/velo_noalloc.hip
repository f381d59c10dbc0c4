// velo_noalloc.hip -- the gradient of the learned filter for callers that
// cannot allocate device memory: its per-workgroup partial sums live in a
// file-scope device array instead of a context's workspace.
#include <mutex>

#include "../../include/velo.h"
#include "mlp.h"

using namespace velo;

namespace {

constexpr int kMaxDevices = 64;

// One copy per GPU, held until the process ends.  Host code never passes the
// array's name to a kernel: it is a host-side stand-in, not a device address.
static __device__ __align__(256) float scratch[kMaxGradBlocks * kGradStride];

std::mutex g_mu;
float* g_ptr[kMaxDevices] = {};

int fail(int code, const char* msg) { return set_last_error(code, msg); }

// Device address of `scratch` on the current device, resolved once per device
// (with that device current) and kept.
int scratch_ptr(float** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return fail(VELO_ERR_DEVICE, "hipGetDevice failed");
    if (dev >= kMaxDevices) return fail(VELO_ERR_UNSUPPORTED, "device index above 63");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return fail(VELO_ERR_DEVICE, "hipGetSymbolAddress(scratch) failed");
        g_ptr[dev] = static_cast<float*>(p);
    }
    *out = g_ptr[dev];
    return VELO_OK;
}

}  // namespace

extern "C" {

int velo_mlp_grad_noalloc(int64_t n, const float* d_master, const uint16_t* d_feat, const uint8_t* d_label,
                          float* d_grad, float* d_loss, void* stream) {
    if (n <= 0 || !d_master || !d_feat || !d_label || !d_grad)
        return fail(VELO_ERR_ARG, "velo_mlp_grad_noalloc: n must be > 0 and the arrays non-null");
    const int64_t blocks = mlp_grad_blocks(n);
    if (blocks > (int64_t)kMaxGradBlocks)
        return fail(VELO_ERR_ARG, "velo_mlp_grad_noalloc: more workgroup partials than the scratch holds");
    float* part = nullptr;
    if (int rc = scratch_ptr(&part)) return rc;
    // every partial the reduction reads is written first: nothing to clear
    const hipError_t e =
        launch_mlp_grad_part(d_master, part, n, d_feat, d_label, d_grad, d_loss, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail(VELO_ERR_DEVICE, hipGetErrorString(e));
    return VELO_OK;
}

}  // extern "C"
