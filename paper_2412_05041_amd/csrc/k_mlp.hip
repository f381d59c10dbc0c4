// k_mlp.hip -- learned ghost filter: 10 -> 32 -> 32 -> 1 ReLU MLP on BF16 MFMA
// (FP32 accumulation), its training gradient with a fixed-order
// (deterministic) reduction, Adam, and the candidate features.
//
// Orientation: samples run along the MFMA N dimension and the weights are the
// A operand, so a layer's accumulator layout (lane l holds rows 4(l/16)+j,
// column l%16) is exactly the next layer's B operand layout: activations never
// leave registers in the forward pass.  Only the weight-gradient products,
// whose reduction dimension is the sample, go through a small per-wave LDS
// transpose.
//
// The products over the 32 hidden units (the second layer, and its transpose
// in the gradient) are one gfx950 v_mfma_f32_16x16x32_bf16 each: a lane's
// eight K slots hold the units 4g..4g+3 and 16+4g..16+4g+3 of the two 16-unit
// accumulator tiles, in both operands -- a reduction index can be laid out in
// any order the two operands share.  The products over 16 samples and over
// the 10 inputs use v_mfma_f32_16x16x16_bf16.
//
// Rounding: weights, inputs and hidden activations are BF16 (round to nearest
// even); biases are added in FP32 (they initialise the accumulator); the last
// layer is an FP32 dot product.  Gradients treat the BF16 roundings as
// identities; the per-sample gradient factors are rounded to BF16 where they
// enter an MFMA.
#include "fitfeat.h"
#include "mlp.h"

namespace velo {

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16v8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// K = 32: the eight slots of a lane are (lo[0..3], hi[0..3]) in both operands.
__device__ __forceinline__ f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16v8, a), __builtin_bit_cast(bf16v8, b), c, 0,
                                                  0, 0);
}

__device__ __forceinline__ bf16x8 cat(bf16x4 lo, bf16x4 hi) {
    return bf16x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
}

__device__ __forceinline__ short bf(float f) { return (short)f2bf(f); }
__device__ __forceinline__ float rbf(float f) { return bf2f(f2bf(f)); }

// Per-wave register copy of the network (lane l: g = l/16, r = l%16).
struct Net {
    bf16x4 a1[2];     // W1[mt*16 + r][4g + j]        (inputs >= 10 are zero)
    bf16x4 a2[2][2];  // W2[mt*16 + r][kc*16 + 4g + j]
    f32x4 c1[2];      // b1[mt*16 + 4g + j]
    f32x4 c2[2];      // b2[mt*16 + 4g + j]
    float w3[2][4];   // bf16(w3[mt*16 + 4g + j])
    float b3;
};

__device__ __forceinline__ void load_net(const float* w, Net& n) {
    const int l = threadIdx.x % kWave, g = l / 16, r = l % 16;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        const int o = mt * 16 + r;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int i = 4 * g + j;
            n.a1[mt][j] = i < kNFeat ? bf(w[oW1 + o * kNFeat + i]) : (short)0;
            n.a2[mt][0][j] = bf(w[oW2 + o * 32 + i]);
            n.a2[mt][1][j] = bf(w[oW2 + o * 32 + 16 + i]);
            n.c1[mt][j] = w[oB1 + mt * 16 + 4 * g + j];
            n.c2[mt][j] = w[oB2 + mt * 16 + 4 * g + j];
            n.w3[mt][j] = rbf(w[oW3 + mt * 16 + 4 * g + j]);
        }
    }
    n.b3 = w[oB3];
}

struct Fwd {
    f32x4 a1[2], a2[2];   // pre-activations
    bf16x4 h1[2];         // bf16(relu(a1)), B-operand layout (K chunk = mt)
    float h2[2][4];       // bf16(relu(a2)) as float
    float z;              // logit of sample r (same in the 4 lanes of column r)
};

// Forward of 16 samples; x = this lane's 4 inputs of sample r (features 4g..4g+3).
__device__ __forceinline__ void forward16(const Net& n, bf16x4 x, Fwd& f) {
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        f.a1[mt] = mfma16(n.a1[mt], x, n.c1[mt]);
#pragma unroll
        for (int j = 0; j < 4; ++j) f.h1[mt][j] = bf(fmaxf(f.a1[mt][j], 0.0f));
    }
    float part = 0.0f;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        const f32x4 acc = mfma32(cat(n.a2[mt][0], n.a2[mt][1]), cat(f.h1[0], f.h1[1]), n.c2[mt]);
        f.a2[mt] = acc;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            f.h2[mt][j] = rbf(fmaxf(acc[j], 0.0f));
            part = part + n.w3[mt][j] * f.h2[mt][j];
        }
    }
    part = part + __shfl_xor(part, 16, kWave);
    part = part + __shfl_xor(part, 32, kWave);
    f.z = n.b3 + part;
}

__device__ __forceinline__ bf16x4 load_x(const uint16_t* feat, int64_t s, int64_t n) {
    const int g = (threadIdx.x % kWave) / 16;
    bf16x4 x = {0, 0, 0, 0};
    if (s < n) {
        const uint2 v = *reinterpret_cast<const uint2*>(feat + s * 16 + 4 * g);
        x[0] = (short)(v.x & 0xffff);
        x[1] = (short)(v.x >> 16);
        x[2] = (short)(v.y & 0xffff);
        x[3] = (short)(v.y >> 16);
    }
    return x;
}

__global__ __launch_bounds__(256) void k_mlp_forward(const float* master, int64_t n, const uint16_t* feat,
                                                     float* logit) {
    Net net;
    load_net(master, net);
    const int l = threadIdx.x % kWave;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
    const int64_t tiles = (n + 15) / 16;
    for (int64_t t = wave; t < tiles; t += nwaves) {
        const int64_t s = t * 16 + l % 16;
        Fwd f;
        forward16(net, load_x(feat, s, n), f);
        if (l < 16 && s < n) logit[s] = f.z;
    }
}

// Learned decision for every candidate of an event (one workgroup per event).
__global__ __launch_bounds__(256) void k_mlp_accept(FindArgs a) {
    __shared__ int s_out, s_hit, s_fb;
    const int e = blockIdx.x;
    if (e >= a.n_events) return;
    Net net;
    load_net(a.mlp_master, net);
    if (threadIdx.x == 0) { s_out = 0; s_hit = 0; s_fb = 0; }
    __syncthreads();
    const Work& w = a.w;
    const int nc = w.ev_ncand[e];
    const int64_t slot0 = a.clu_off[e * kPlanes];
    const int l = threadIdx.x % kWave, wv = threadIdx.x / kWave;
    int my_out = 0, my_hit = 0, my_fb = 0;
    for (int t = wv; t * 16 < nc; t += blockDim.x / kWave) {
        const int c = t * 16 + l % 16;
        Fwd f;
        forward16(net, load_x(w.cfeat + slot0 * 16, c, nc), f);
        if (l < 16 && c < nc) {
            uint8_t fl = w.cflags[slot0 + c];
            const float z = f.z;
            bool acc;
            if (isnan(z) || fabsf(z) < a.p.logit_band) {
                fl |= TRK_FALLBACK;
                acc = (fl & TRK_PLAIN) != 0;
                ++my_fb;
            } else {
                acc = !(z > 0.0f);
            }
            if (acc) {
                fl |= TRK_ACCEPT;
                ++my_out;
                my_hit += __popc(w.cmask[slot0 + c]);
            }
            w.cflags[slot0 + c] = fl;
            w.clogit[slot0 + c] = z;
        }
    }
    atomicAdd(&s_out, my_out);
    atomicAdd(&s_hit, my_hit);
    atomicAdd(&s_fb, my_fb);
    __syncthreads();
    if (threadIdx.x == 0) {
        w.ev_nout[e] = s_out;
        w.ev_nouthit[e] = s_hit;
        if (s_fb && a.status) {
            atomicAdd(a.status + ST_NFALLBACK, s_fb);
            atomicOr(a.status + kStatusHdr + e, EV_FALLBACK);
        }
    }
}

// ------------------------------------------------------------------ gradient

constexpr int kGradThreads = 256;
constexpr int kGradWaves = kGradThreads / kWave;

// Per-block partial gradient (parameters in the master layout, loss last).
__global__ __launch_bounds__(kGradThreads) void k_mlp_grad(const float* master, int64_t n, const uint16_t* feat,
                                                           const uint8_t* label, float* part, int64_t tiles_per_wave) {
    __shared__ uint16_t s_t[kGradWaves][2][32][16];  // per-wave transposes (gradient factor, h1)
    __shared__ float s_red[kGradWaves][kGradStride];
    Net net;
    load_net(master, net);
    const int l = threadIdx.x % kWave, g = l / 16, r = l % 16, wv = threadIdx.x / kWave;
    // W2^T as A operand: lane holds W2[kc*16 + 4g + j][mt*16 + r]
    bf16x4 a2t[2][2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int kc = 0; kc < 2; ++kc)
#pragma unroll
            for (int j = 0; j < 4; ++j) a2t[mt][kc][j] = bf(master[oW2 + (kc * 16 + 4 * g + j) * 32 + mt * 16 + r]);
    const float inv_n = 1.0f / (float)n;
    f32x4 gw2[2][2], gw1[2];
    float gw3[2][4], gb2[2][4], gb1[2][4], gb3 = 0.0f, loss = 0.0f;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        gw1[mt] = f32x4{0, 0, 0, 0};
#pragma unroll
        for (int kc = 0; kc < 2; ++kc) gw2[mt][kc] = f32x4{0, 0, 0, 0};
#pragma unroll
        for (int j = 0; j < 4; ++j) { gw3[mt][j] = 0.0f; gb2[mt][j] = 0.0f; gb1[mt][j] = 0.0f; }
    }
    const int64_t wave = (int64_t)blockIdx.x * kGradWaves + wv;
    const int64_t nwaves = (int64_t)gridDim.x * kGradWaves;
    for (int64_t it = 0; it < tiles_per_wave; ++it) {
        const int64_t t = wave + it * nwaves;
        const int64_t s0 = t * 16;
        const int64_t s = s0 + r;
        Fwd f;
        forward16(net, load_x(feat, s, n), f);
        const bool valid = s < n;
        const float y = valid ? (label[s] ? 1.0f : 0.0f) : 0.0f;
        const float gz = valid ? (1.0f / (1.0f + expf(-f.z)) - y) * inv_n : 0.0f;
        if (g == 0 && valid) {
            loss += fmaxf(f.z, 0.0f) + log1pf(expf(-fabsf(f.z))) - y * f.z;
            gb3 += gz;
        }
        // output layer and the gradient at a2
        bf16x4 ga2[2];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                gw3[mt][j] += gz * f.h2[mt][j];
                const float v = f.a2[mt][j] > 0.0f ? gz * net.w3[mt][j] : 0.0f;
                gb2[mt][j] += v;
                ga2[mt][j] = bf(v);
            }
        // transpose ga2 and h1 through LDS: row = unit, column = sample
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                s_t[wv][0][mt * 16 + 4 * g + j][r] = (uint16_t)ga2[mt][j];
                s_t[wv][1][mt * 16 + 4 * g + j][r] = (uint16_t)f.h1[mt][j];
            }
        __syncthreads();
        bf16x4 ta[2], th[2];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                ta[mt][j] = (short)s_t[wv][0][mt * 16 + r][4 * g + j];
                th[mt][j] = (short)s_t[wv][1][mt * 16 + r][4 * g + j];
            }
        // dW2[o][i] += sum_s ga2[o][s] h1[i][s]
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int kc = 0; kc < 2; ++kc) gw2[mt][kc] = mfma16(ta[mt], th[kc], gw2[mt][kc]);
        // gradient at h1: W2^T ga2, then at a1
        bf16x4 ga1[2];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
            const f32x4 gh = mfma32(cat(a2t[mt][0], a2t[mt][1]), cat(ga2[0], ga2[1]), f32x4{0, 0, 0, 0});
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float v = f.a1[mt][j] > 0.0f ? gh[j] : 0.0f;
                gb1[mt][j] += v;
                ga1[mt][j] = bf(v);
            }
        }
        __syncthreads();
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int j = 0; j < 4; ++j) s_t[wv][0][mt * 16 + 4 * g + j][r] = (uint16_t)ga1[mt][j];
        __syncthreads();
        // dW1[o][i] += sum_s ga1[o][s] x[s][i]; B operand = x[s0 + 4g + j][i = r]
        bf16x4 xb;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t sj = s0 + 4 * g + j;
            xb[j] = sj < n ? (short)feat[sj * 16 + r] : (short)0;
        }
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
#pragma unroll
            for (int j = 0; j < 4; ++j) ta[mt][j] = (short)s_t[wv][0][mt * 16 + r][4 * g + j];
            gw1[mt] = mfma16(ta[mt], xb, gw1[mt]);
        }
        __syncthreads();
    }
    // reduce the vector accumulators over the 16 sample columns (fixed order)
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int o = 1; o < 16; o <<= 1) {
                gw3[mt][j] += __shfl_xor(gw3[mt][j], o, kWave);
                gb2[mt][j] += __shfl_xor(gb2[mt][j], o, kWave);
                gb1[mt][j] += __shfl_xor(gb1[mt][j], o, kWave);
            }
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        gb3 += __shfl_xor(gb3, o, kWave);
        loss += __shfl_xor(loss, o, kWave);
    }
    float* red = s_red[wv];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int o = mt * 16 + 4 * g + j;
            if (r == 0) {
                red[oW3 + o] = gw3[mt][j];
                red[oB2 + o] = gb2[mt][j];
                red[oB1 + o] = gb1[mt][j];
            }
            if (r < kNFeat) red[oW1 + o * kNFeat + r] = gw1[mt][j];
#pragma unroll
            for (int kc = 0; kc < 2; ++kc) red[oW2 + o * 32 + kc * 16 + r] = gw2[mt][kc][j];
        }
    if (l == 0) {
        red[oB3] = gb3;
        red[kNParam] = loss;
    }
    __syncthreads();
    for (int p = threadIdx.x; p <= kNParam; p += kGradThreads) {
        float s = 0.0f;
        for (int q = 0; q < kGradWaves; ++q) s += s_red[q][p];
        part[(int64_t)blockIdx.x * kGradStride + p] = s;
    }
}

// Fixed-order sum of the per-block partials: for 64 consecutive parameters
// (one per lane), wave w adds the partials of blocks [w*nb/16, (w+1)*nb/16) in
// block order, then wave 0 adds the 16 wave sums in wave order.  The order
// depends only on the number of blocks, so the gradient is reproducible.
constexpr int kRedWaves = 16;
__global__ __launch_bounds__(kRedWaves * kWave) void k_grad_reduce(const float* part, int nblocks, float* grad,
                                                                  float* loss, float inv_n) {
    __shared__ float s_sum[kRedWaves][kWave];
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
    const int p = blockIdx.x * kWave + lane;
    const int b0 = (int)((int64_t)nblocks * wv / kRedWaves), b1 = (int)((int64_t)nblocks * (wv + 1) / kRedWaves);
    float s = 0.0f;
    if (p <= kNParam)
        for (int b = b0; b < b1; ++b) s += part[(int64_t)b * kGradStride + p];
    s_sum[wv][lane] = s;
    __syncthreads();
    if (wv == 0 && p <= kNParam) {
        float t = 0.0f;
        for (int w = 0; w < kRedWaves; ++w) t += s_sum[w][lane];
        if (p < kNParam) grad[p] = t;
        else if (loss) *loss = t * inv_n;
    }
}

__global__ __launch_bounds__(256) void k_adam(float* w, float* m, float* v, const float* g, float lr, float b1,
                                              float b2, float eps, float c1, float c2) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kNParam) return;
    const float gp = g[p];
    const float mp = b1 * m[p] + (1.0f - b1) * gp;
    const float vp = b2 * v[p] + (1.0f - b2) * gp * gp;
    m[p] = mp;
    v[p] = vp;
    w[p] = w[p] - lr * (mp / c1) / (sqrtf(vp / c2) + eps);
}

__global__ __launch_bounds__(256) void k_features(Params p, const float* norm, int64_t n, const int32_t* hit_off,
                                                  const int32_t* hits, const uint32_t* planes, const float* clu_x,
                                                  const float* clu_y, uint16_t* feat, float* feat32) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int32_t* h = hits + hit_off[t];
    const FitResult f = fit_track_hits([&](int, int i) { return h[i]; }, planes[t], clu_x, clu_y, p.z, p.sigma);
    float raw[10];
    raw_features(f, p.sigma, raw);
    if (feat32)
        for (int i = 0; i < 10; ++i) feat32[t * 10 + i] = raw[i];
    if (!feat) return;
    uint16_t fb[16];
    std_features(raw, norm, fb);
    uint4* out = reinterpret_cast<uint4*>(feat + t * 16);
    const uint4* src = reinterpret_cast<const uint4*>(fb);
    out[0] = src[0];
    out[1] = src[1];
}

__global__ __launch_bounds__(256) void k_standardize(const float* norm, int64_t n, const float* raw, uint16_t* feat) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    uint16_t fb[16];
    std_features(raw + t * 10, norm, fb);
    uint4* out = reinterpret_cast<uint4*>(feat + t * 16);
    const uint4* src = reinterpret_cast<const uint4*>(fb);
    out[0] = src[0];
    out[1] = src[1];
}

}  // namespace

hipError_t launch_standardize(const float* norm, int64_t n, const float* raw, uint16_t* feat, hipStream_t s) {
    const int64_t grid = (n + 255) / 256;
    hipLaunchKernelGGL(k_standardize, dim3((unsigned)grid), dim3(256), 0, s, norm, n, raw, feat);
    return hipGetLastError();
}

int mlp_init(MlpState& m) {
    if (hipMalloc(&m.d_master, sizeof(float) * kNParam) != hipSuccess) return -1;
    if (hipMalloc(&m.d_norm, sizeof(float) * 2 * kNFeat) != hipSuccess) return -1;
    if (hipMalloc(&m.d_m, sizeof(float) * kNParam) != hipSuccess) return -1;
    if (hipMalloc(&m.d_v, sizeof(float) * kNParam) != hipSuccess) return -1;
    if (hipMalloc(&m.d_grad, sizeof(float) * kNParam) != hipSuccess) return -1;
    if (hipMalloc(&m.d_part, sizeof(float) * kMaxGradBlocks * kGradStride) != hipSuccess) return -1;
    if (hipMemset(m.d_m, 0, sizeof(float) * kNParam) != hipSuccess) return -1;
    if (hipMemset(m.d_v, 0, sizeof(float) * kNParam) != hipSuccess) return -1;
    if (hipMemset(m.d_master, 0, sizeof(float) * kNParam) != hipSuccess) return -1;
    return 0;
}

void mlp_free(MlpState& m) {
    (void)hipFree(m.d_master);
    (void)hipFree(m.d_norm);
    (void)hipFree(m.d_m);
    (void)hipFree(m.d_v);
    (void)hipFree(m.d_grad);
    (void)hipFree(m.d_part);
    m = MlpState{};
}

hipError_t launch_mlp_accept(const MlpState&, const FindArgs& a, hipStream_t s) {
    if (a.n_events <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_accept, dim3(a.n_events), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_features(const Params& p, const float* norm, int64_t n, const int32_t* trk_hit_off,
                           const int32_t* trk_hit, const uint32_t* trk_planes, const float* clu_x,
                           const float* clu_y, uint16_t* feat, float* feat32, hipStream_t s) {
    const int64_t grid = (n + 255) / 256;
    hipLaunchKernelGGL(k_features, dim3((unsigned)grid), dim3(256), 0, s, p, norm, n, trk_hit_off, trk_hit,
                       trk_planes, clu_x, clu_y, feat, feat32);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const MlpState& m, int64_t n, const uint16_t* feat, float* logit, hipStream_t s) {
    const int64_t tiles = (n + 15) / 16;
    const int64_t grid = std::min<int64_t>(4096, (tiles + 3) / 4);
    hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)std::max<int64_t>(grid, 1)), dim3(256), 0, s, m.d_master, n,
                       feat, logit);
    return hipGetLastError();
}

// Grid size of the gradient depends on n only, so the reduction order (and the
// result) is reproducible bit for bit.
int64_t mlp_grad_blocks(int64_t n) {
    const int64_t tiles = (n + 15) / 16;
    return std::max<int64_t>(1, std::min<int64_t>(kMaxGradBlocks, (tiles + kGradWaves - 1) / kGradWaves));
}

hipError_t launch_mlp_grad_part(const float* master, float* part, int64_t n, const uint16_t* feat,
                                const uint8_t* label, float* grad, float* loss, hipStream_t s) {
    const int64_t tiles = (n + 15) / 16;
    const int64_t blocks = mlp_grad_blocks(n);
    const int64_t nwaves = blocks * kGradWaves;
    const int64_t per_wave = (tiles + nwaves - 1) / nwaves;
    hipLaunchKernelGGL(k_mlp_grad, dim3((unsigned)blocks), dim3(kGradThreads), 0, s, master, n, feat, label, part,
                       per_wave);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_grad_reduce, dim3((kNParam + 1 + kWave - 1) / kWave), dim3(kRedWaves * kWave), 0, s, part,
                       (int)blocks, grad, loss, 1.0f / (float)n);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(MlpState& m, int64_t n, const uint16_t* feat, const uint8_t* label, float* grad,
                           float* loss, hipStream_t s) {
    return launch_mlp_grad_part(m.d_master, m.d_part, n, feat, label, grad, loss, s);
}

hipError_t launch_adam(MlpState& m, float lr, hipStream_t s) {
    const double c1 = 1.0 - std::pow((double)m.beta1, (double)m.step);
    const double c2 = 1.0 - std::pow((double)m.beta2, (double)m.step);
    hipLaunchKernelGGL(k_adam, dim3((kNParam + 255) / 256), dim3(256), 0, s, m.d_master, m.d_m, m.d_v, m.d_grad, lr,
                       m.beta1, m.beta2, m.eps, (float)c1, (float)c2);
    return hipGetLastError();
}

}  // namespace velo
