// k_mlp.hip -- learned ghost filter kernels (placeholder until the MFMA kernels land).
#include "mlp.h"

namespace velo {

int mlp_init(MlpState& m) {
    if (hipMalloc(&m.d_master, sizeof(float) * kNParam) != hipSuccess) return -1;
    if (hipMalloc(&m.d_norm, sizeof(float) * 2 * kNFeat) != hipSuccess) return -1;
    if (hipMalloc(&m.d_m, sizeof(float) * kNParam) != hipSuccess) return -1;
    if (hipMalloc(&m.d_v, sizeof(float) * kNParam) != hipSuccess) return -1;
    if (hipMalloc(&m.d_grad, sizeof(float) * kNParam) != hipSuccess) return -1;
    if (hipMalloc(&m.d_part, sizeof(float) * kMaxGradBlocks * kGradStride) != hipSuccess) return -1;
    if (hipMemset(m.d_m, 0, sizeof(float) * kNParam) != hipSuccess) return -1;
    if (hipMemset(m.d_v, 0, sizeof(float) * kNParam) != hipSuccess) return -1;
    return 0;
}

void mlp_free(MlpState& m) {
    hipFree(m.d_master);
    hipFree(m.d_norm);
    hipFree(m.d_m);
    hipFree(m.d_v);
    hipFree(m.d_grad);
    hipFree(m.d_part);
    m = MlpState{};
}

hipError_t launch_mlp_accept(const MlpState&, const FindArgs&, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_features(const Params&, const float*, int64_t, const int32_t*, const int32_t*, const uint32_t*,
                           const float*, const float*, uint16_t*, float*, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_mlp_forward(const MlpState&, int64_t, const uint16_t*, float*, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_mlp_grad(MlpState&, int64_t, const uint16_t*, const uint8_t*, float*, float*, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_adam(MlpState&, float, hipStream_t) { return hipErrorNotSupported; }

}  // namespace velo
