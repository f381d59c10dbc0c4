// k_kalman.hip -- Kalman fit of VELO track segments (one thread per track).
//
// Each projection (x-z, y-z) is a straight line whose slope takes an
// independent kick of variance ms^2 on every plane the track crosses (the
// parameterised multiple scattering); hits are measured with variance
// sigma^2.  The filter starts from the two most downstream hits (position at
// the second, slope through both, their exact covariance including the kicks
// on the planes between them) and steps plane by plane towards the
// interaction region: at each plane the slope variance grows by ms^2 (the
// segment below a plane differs from the one above it by that plane's kick),
// the state is carried down, and a hit on the plane updates it.  The state
// returned is the one at the most upstream hit.  With ms = 0 this is the
// least-squares line.  All 26 planes are unrolled, so the per-plane state
// stays in registers.
#include "fitfeat.h"
#include "kernels.h"

namespace velo {

namespace {

struct Proj {
    float x, s, cxx, cxs, css, chi2;
};

__device__ __forceinline__ void init_proj(Proj& k, float ua, float ub, float D, float s2, float m2g) {
    k.x = ub;
    k.s = (ua - ub) / D;
    k.cxx = s2;
    k.cxs = -s2 / D;
    k.css = (s2 + s2) / (D * D) + m2g;
    k.chi2 = 0.0f;
}

// slope kick undone, then the state carried down by dz
__device__ __forceinline__ void step_proj(Proj& k, float dz, float m2) {
    k.css = k.css + m2;
    k.x = k.x - k.s * dz;
    const float cxx = k.cxx - dz * k.cxs - dz * k.cxs + dz * dz * k.css;
    const float cxs = k.cxs - dz * k.css;
    k.cxx = cxx;
    k.cxs = cxs;
}

__device__ __forceinline__ void update_proj(Proj& k, float u, float s2) {
    const float r = u - k.x;
    const float S = k.cxx + s2;
    const float kx = k.cxx / S, ks = k.cxs / S;
    k.x = k.x + kx * r;
    k.s = k.s + ks * r;
    const float cxx = k.cxx - kx * k.cxx;
    const float cxs = k.cxs - kx * k.cxs;
    const float css = k.css - ks * k.cxs;
    k.cxx = cxx;
    k.cxs = cxs;
    k.css = css;
    k.chi2 = k.chi2 + r * r / S;
}

__global__ __launch_bounds__(256) void k_kalman(KalmanArgs a) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nt = a.n_tracks ? (int64_t)*a.n_tracks : a.max_tracks;
    if (t >= nt || t >= a.max_tracks) return;
    const uint32_t mask = a.trk_planes[t];
    const int32_t* h = a.trk_hit + a.trk_hit_off[t];
    float x[kPlanes], y[kPlanes], z[kPlanes];
    gather_hits([&](int, int i) { return h[i]; }, mask, a.clu_x, a.clu_y, x, y);
#pragma unroll
    for (int k = 0; k < kPlanes; ++k) z[k] = a.z[k];
    const int n = __popc(mask);
    float4* o = reinterpret_cast<float4*>(a.out + t * 16);
    if (n < 2) {
        o[0] = o[1] = o[2] = o[3] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        return;
    }
    const int la = 31 - __clz(mask);
    const int lb = 31 - __clz(mask & ~(1u << la));
    const int lf = __ffs(mask) - 1;
    const float s2 = a.sigma * a.sigma, m2 = a.ms * a.ms;
    float za = 0.0f, zb = 0.0f, xa = 0.0f, xb = 0.0f, ya = 0.0f, yb = 0.0f;
#pragma unroll
    for (int k = 0; k < kPlanes; ++k) {
        if (k == la) { za = z[k]; xa = x[k]; ya = y[k]; }
        if (k == lb) { zb = z[k]; xb = x[k]; yb = y[k]; }
    }
    const float D = za - zb;
    float g = 0.0f;
#pragma unroll
    for (int q = 1; q < kPlanes - 1; ++q) {
        if (q > lb && q < la) {
            const float w = (za - z[q]) / D;
            g = g + w * w;
        }
    }
    const float m2g = m2 * g;
    Proj px, py;
    init_proj(px, xa, xb, D, s2, m2g);
    init_proj(py, ya, yb, D, s2, m2g);
#pragma unroll
    for (int q = kPlanes - 2; q >= 0; --q) {
        if (q < lb && q >= lf) {
            const float dz = z[q + 1] - z[q];
            step_proj(px, dz, m2);
            step_proj(py, dz, m2);
            if (mask & (1u << q)) {
                update_proj(px, x[q], s2);
                update_proj(py, y[q], s2);
            }
        }
    }
    float zf = 0.0f;
#pragma unroll
    for (int k = 0; k < kPlanes; ++k)
        if (k == lf) zf = z[k];
    o[0] = make_float4(px.x, py.x, px.s, py.s);
    o[1] = make_float4(zf, px.cxx, px.cxs, px.css);
    o[2] = make_float4(py.cxx, py.cxs, py.css, px.chi2 + py.chi2);
    o[3] = make_float4((float)(2 * n - 4), 0.0f, 0.0f, 0.0f);
}

}  // namespace

hipError_t launch_kalman(const KalmanArgs& a, hipStream_t s) {
    if (a.max_tracks <= 0) return hipSuccess;
    const int64_t grid = (a.max_tracks + 255) / 256;
    hipLaunchKernelGGL(k_kalman, dim3((unsigned)grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace velo
