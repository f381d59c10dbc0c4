// k_extrap.hip -- forward extrapolation of VELO states through the magnet.
//
// The first step of forward tracking: each VELO state goes along its straight
// line to the middle of the magnet; there the field is replaced by one change
// of the x slope, kick x (charge / momentum), and the track goes on straight to
// the tracker plane z_t.  Per track: the states at both planes, the window in x
// at z_t that holds every track of momentum >= p_min, and -- given a hit at
// z_t -- the charge / momentum that leads to it and the slope after the kink.
// One thread per track; the VELO state and the result are 32-byte rows, read
// and written as two 16-byte vectors each.
#include "kernels.h"

namespace velo {

namespace {

__global__ __launch_bounds__(256) void k_extrapolate(ExtrapArgs a) {
    const int64_t n = a.n_tracks ? (int64_t)*a.n_tracks : a.max_tracks;
    const int64_t lim = n < a.max_tracks ? n : a.max_tracks;
    const float lever = a.z_t - a.z_mag;
    const float w = a.kick / a.p_min * lever;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < lim; t += (int64_t)gridDim.x * blockDim.x) {
        const float4 p0 = reinterpret_cast<const float4*>(a.par)[2 * t];
        const float4 p1 = reinterpret_cast<const float4*>(a.par)[2 * t + 1];
        const float x0 = p0.x, y0 = p0.y, z0 = p0.z, tx = p0.w, ty = p1.x;
        const float xm = x0 + tx * (a.z_mag - z0);
        const float ym = y0 + ty * (a.z_mag - z0);
        const float xl = xm + tx * lever;
        const float qop = a.x_hit ? ((a.x_hit[t] - xm) / lever - tx) / a.kick : 0.0f;
        float4 o0, o1;
        o0.x = xm;
        o0.y = ym;
        o0.z = xl;
        o0.w = y0 + ty * (a.z_t - z0);
        o1.x = xl - w;
        o1.y = xl + w;
        o1.z = qop;
        o1.w = tx + a.kick * qop;
        reinterpret_cast<float4*>(a.out)[2 * t] = o0;
        reinterpret_cast<float4*>(a.out)[2 * t + 1] = o1;
    }
}

}  // namespace

hipError_t launch_extrapolate(const ExtrapArgs& a, hipStream_t s) {
    if (a.max_tracks <= 0) return hipSuccess;
    const int64_t blocks = (a.max_tracks + 255) / 256;
    const int grid = (int)(blocks < 65536 ? blocks : 65536);
    hipLaunchKernelGGL(k_extrapolate, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace velo
