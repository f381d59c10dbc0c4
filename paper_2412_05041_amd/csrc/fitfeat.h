// fitfeat.h -- the FP32 least-squares straight-line fit and the candidate
// features, shared by the finder's acceptance step, the output/fit kernels and
// the feature kernel so that every caller evaluates the same operations in the
// same order (built without contraction).
//
// Fit over the n hits in plane order, sums as left folds from 0:
//   zr = (sum z)/n, xr = (sum x)/n, yr = (sum y)/n, d_i = z_i - zr,
//   tx = sum d_i (x_i - xr) / sum d_i^2 (likewise ty),
//   r_i = (x_i - xr) - tx d_i (likewise y), chi2 = sum (rx^2 + ry^2) / sigma^2,
//   ndof = 2n - 4.
// Features: chi2/ndof, n, tx, ty, max|rx|/sigma, max|ry|/sigma, first- and
// last-hit squared residual / sigma^2, first and last plane / 25.
#pragma once

#include "common.h"

namespace velo {

struct FitResult {
    float xr, yr, zr, tx, ty, chi2;
    int n, ndof;
    float mrx, mry, r_first, r_last;
    int first, last;
};

// Gathers the coordinates of a track's hits into per-plane registers:
// hit_at(k, i) gives the cluster index of the i-th hit (on plane k).  Two
// rounds of independent loads with no branch between a load and its use, so
// that each round waits once: every plane's hit index (hit_at is called for
// every plane, with i clamped to the last hit, and must be safe to read
// there), then every plane's coordinates, planes off the mask reading the
// first hit's.  Planes off the mask get 0.
template <typename HitAt>
__device__ __forceinline__ void gather_hits(HitAt hit_at, uint32_t mask, const float* clu_x, const float* clu_y,
                                            float* x, float* y) {
    const int n = __popc(mask);
    if (n == 0) {
#pragma unroll
        for (int k = 0; k < kPlanes; ++k) { x[k] = 0.0f; y[k] = 0.0f; }
        return;
    }
    const int first = __ffs(mask) - 1;
    int h[kPlanes];
#pragma unroll
    for (int k = 0; k < kPlanes; ++k) h[k] = hit_at(k, min(__popc(mask & ((1u << k) - 1u)), n - 1));
    int h0 = h[0];
#pragma unroll
    for (int k = 1; k < kPlanes; ++k) h0 = k == first ? h[k] : h0;
#pragma unroll
    for (int k = 0; k < kPlanes; ++k) {
        const bool on = (mask >> k) & 1u;
        const int hk = on ? h[k] : h0;
        const float xv = clu_x[hk];
        const float yv = clu_y[hk];
        x[k] = on ? xv : 0.0f;
        y[k] = on ? yv : 0.0f;
    }
}

// Fit of the gathered hits (planes ascending, left folds from 0).
__device__ __forceinline__ FitResult fit_hits(const float* x, const float* y, uint32_t mask, const float* zp,
                                              float sigma) {
    FitResult f;
    f.first = mask ? __ffs(mask) - 1 : -1;
    f.last = mask ? 31 - __clz(mask) : -1;
    const int n = __popc(mask);
    float sz = 0.0f, sx = 0.0f, sy = 0.0f;
#pragma unroll
    for (int k = 0; k < kPlanes; ++k)
        if (mask & (1u << k)) { sz = sz + zp[k]; sx = sx + x[k]; sy = sy + y[k]; }
    const float fn = (float)n;
    f.zr = sz / fn;
    f.xr = sx / fn;
    f.yr = sy / fn;
    float szz = 0.0f, szx = 0.0f, szy = 0.0f;
#pragma unroll
    for (int k = 0; k < kPlanes; ++k) {
        if (mask & (1u << k)) {
            const float d = zp[k] - f.zr;
            szz = szz + d * d;
            szx = szx + d * (x[k] - f.xr);
            szy = szy + d * (y[k] - f.yr);
        }
    }
    f.tx = szx / szz;
    f.ty = szy / szz;
    float ss = 0.0f;
    f.mrx = 0.0f;
    f.mry = 0.0f;
    f.r_first = 0.0f;
    f.r_last = 0.0f;
#pragma unroll
    for (int k = 0; k < kPlanes; ++k) {
        if (mask & (1u << k)) {
            const float d = zp[k] - f.zr;
            const float rx = (x[k] - f.xr) - f.tx * d;
            const float ry = (y[k] - f.yr) - f.ty * d;
            const float rr = rx * rx + ry * ry;
            ss = ss + rr;
            f.mrx = fmaxf(f.mrx, fabsf(rx));
            f.mry = fmaxf(f.mry, fabsf(ry));
            if (k == f.first) f.r_first = rr;
            f.r_last = rr;
        }
    }
    f.chi2 = ss / (sigma * sigma);
    f.n = n;
    f.ndof = 2 * n - 4;
    return f;
}

template <typename HitAt>
__device__ __forceinline__ FitResult fit_track_hits(HitAt hit_at, uint32_t mask, const float* clu_x,
                                                    const float* clu_y, const float* zp, float sigma) {
    float x[kPlanes], y[kPlanes];
    gather_hits(hit_at, mask, clu_x, clu_y, x, y);
    return fit_hits(x, y, mask, zp, sigma);
}

__device__ __forceinline__ void raw_features(const FitResult& f, float sigma, float* o) {
    const float s2 = sigma * sigma;
    o[0] = f.chi2 / (float)f.ndof;
    o[1] = (float)f.n;
    o[2] = f.tx;
    o[3] = f.ty;
    o[4] = f.mrx / sigma;
    o[5] = f.mry / sigma;
    o[6] = f.r_first / s2;
    o[7] = f.r_last / s2;
    o[8] = (float)f.first / 25.0f;
    o[9] = (float)f.last / 25.0f;
}

// BF16 bit pattern of a float, round to nearest even (NaN stays NaN).
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Standardised BF16 features (10 used, 6 zero) into out[16].
__device__ __forceinline__ void std_features(const float* raw, const float* norm, uint16_t* out) {
#pragma unroll
    for (int i = 0; i < 10; ++i) out[i] = f2bf((raw[i] - norm[i]) / norm[10 + i]);
#pragma unroll
    for (int i = 10; i < 16; ++i) out[i] = 0;
}

}  // namespace velo
