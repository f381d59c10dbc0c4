// mlp.h -- learned ghost filter state and launchers (internal to libvelo).
#pragma once

#include "kernels.h"

namespace velo {

constexpr int kNParam = 1441;
constexpr int kNFeat = 10;
// parameter offsets: W1[32][10], b1[32], W2[32][32], b2[32], w3[32], b3
constexpr int oW1 = 0, oB1 = 320, oW2 = 352, oB2 = 1376, oW3 = 1408, oB3 = 1440;

struct MlpState {
    float* d_master = nullptr;  // FP32 master weights [1441]
    float* d_norm = nullptr;    // means[10], sds[10]
    float* d_m = nullptr;       // Adam moments
    float* d_v = nullptr;
    float* d_grad = nullptr;    // [1441]
    float* d_part = nullptr;    // per-block partial gradients [kMaxGradBlocks][kGradStride]
    float* d_loss_part = nullptr;
    int64_t step = 0;
    float beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
    int has_weights = 0;
    uint64_t version = 1;
};

constexpr int kMaxGradBlocks = 1024;
constexpr int kGradStride = 1472;  // 1441 rounded up (+ loss)

int mlp_init(MlpState& m);
void mlp_free(MlpState& m);
hipError_t launch_mlp_accept(const MlpState& m, const FindArgs& a, hipStream_t s);
hipError_t launch_features(const Params& p, const float* norm, int64_t n, const int32_t* trk_hit_off,
                           const int32_t* trk_hit, const uint32_t* trk_planes, const float* clu_x,
                           const float* clu_y, uint16_t* feat, float* feat32, hipStream_t s);
hipError_t launch_standardize(const float* norm, int64_t n, const float* raw, uint16_t* feat, hipStream_t s);
hipError_t launch_mlp_forward(const MlpState& m, int64_t n, const uint16_t* feat, float* logit, hipStream_t s);
hipError_t launch_mlp_grad(MlpState& m, int64_t n, const uint16_t* feat, const uint8_t* label, float* grad,
                           float* loss, hipStream_t s);
// Same gradient with the master weights and the per-block partials
// ([mlp_grad_blocks(n)][kGradStride] FP32, fully written before being read)
// given explicitly; the workgroup count depends on n only.
int64_t mlp_grad_blocks(int64_t n);
hipError_t launch_mlp_grad_part(const float* master, float* part, int64_t n, const uint16_t* feat,
                                const uint8_t* label, float* grad, float* loss, hipStream_t s);
hipError_t launch_adam(MlpState& m, float lr, hipStream_t s);

int find_blocks_per_cu(int threads, int tile, bool seed);

}  // namespace velo
