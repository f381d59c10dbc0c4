// k_output.hip -- bookkeeping kernels: workspace reset, largest-first event
// order, per-event scans, CSR compaction of the accepted tracks (with their
// fit parameters, which the acceptance step already computed), and the
// standalone least-squares fit.
#include "fitfeat.h"
#include "kernels.h"

namespace velo {

namespace {

constexpr int kScanThreads = 1024;

__global__ void k_reset(Work w, int n_events, int32_t* status) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (tid < 8) w.counters[tid] = 0;
    if (status) {
        for (int64_t i = tid; i < kStatusHdr + n_events; i += stride) status[i] = 0;
    }
}

// Largest events first (by clusters, log2 buckets): a coarse LPT order for the
// work-stealing finder, in two lists -- events whose planes all fit kp (the
// first LDS tile) into w.order, the others into `big`.  Single workgroup; the
// order inside a bucket is whatever the atomics give -- results never depend
// on it.
__global__ __launch_bounds__(1024) void k_order(Work w, int n_events, const int32_t* clu_off, int kp, int32_t* big,
                                                int big_count) {
    __shared__ int hist[2][33];
    __shared__ int start[2][33];
    if (threadIdx.x < 66) (&hist[0][0])[threadIdx.x] = 0;
    __syncthreads();
    // size class (log2 of the event's clusters) and whether a plane exceeds kp
    auto classify = [&](int e, int* b) {
        const int32_t* o = clu_off + e * kPlanes;
        const int n = o[kPlanes] - o[0];
        *b = 31 - (n > 0 ? 32 - __clz(n) : 0);
        int over = 0;
        for (int k = 0; k < kPlanes; ++k) over |= (o[k + 1] - o[k]) > kp;
        return over;
    };
    for (int e = threadIdx.x; e < n_events; e += blockDim.x) {
        int b;
        const int g = classify(e, &b);
        atomicAdd(&hist[g][b], 1);
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        int s = 0;
        for (int b = 0; b < 33; ++b) { start[threadIdx.x][b] = s; s += hist[threadIdx.x][b]; }
        // k_reset cleared the counters: events for the first tile, and the
        // head of the list the larger ones go to
        w.counters[threadIdx.x == 0 ? 6 : big_count] = s;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < n_events; e += blockDim.x) {
        int b;
        if (classify(e, &b)) big[atomicAdd(&start[1][b], 1)] = e;
        else w.order[atomicAdd(&start[0][b], 1)] = e;
    }
}

// Block-wide exclusive scan of per-event counts into ev_tbase/ev_hbase; also
// trk_off and the totals.  Single workgroup of 1024 threads.
__global__ __launch_bounds__(kScanThreads) void k_scan(Work w, int n_events, int32_t* trk_off,
                                                       int32_t* trk_hit_off, int64_t trk_cap, int32_t* status,
                                                       int emit) {
    __shared__ int64_t s_t[kScanThreads / kWave], s_h[kScanThreads / kWave];
    __shared__ int64_t carry_t, carry_h;
    if (threadIdx.x == 0) { carry_t = 0; carry_h = 0; }
    __syncthreads();
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    for (int base = 0; base < n_events; base += kScanThreads) {
        const int e = base + threadIdx.x;
        const int vt = e < n_events ? (emit ? w.ev_ncand[e] : w.ev_nout[e]) : 0;
        const int vh = e < n_events ? (emit ? w.ev_ncandhit[e] : w.ev_nouthit[e]) : 0;
        int tt, th;
        const int et = wave_excl_scan(vt, &tt);
        const int eh = wave_excl_scan(vh, &th);
        if (lane == 0) { s_t[wid] = tt; s_h[wid] = th; }
        __syncthreads();
        int64_t pt = carry_t, ph = carry_h;
        for (int i = 0; i < wid; ++i) { pt += s_t[i]; ph += s_h[i]; }
        if (e < n_events) {
            w.ev_tbase[e] = (int32_t)(pt + et);
            w.ev_hbase[e] = (int32_t)(ph + eh);
            trk_off[e] = (int32_t)(pt + et);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int i = 0; i < kScanThreads / kWave; ++i) { carry_t += s_t[i]; carry_h += s_h[i]; }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        trk_off[n_events] = (int32_t)carry_t;
        if (carry_t <= trk_cap) trk_hit_off[carry_t] = (int32_t)carry_h;
        if (status) {
            status[ST_NTRK] = (int32_t)carry_t;
            status[ST_NHIT] = (int32_t)carry_h;
        }
    }
}

// Least-squares fit of one track (the acceptance fit, same operations).
// par: x_ref, y_ref, z_ref, tx, ty, chi2, ndof, 0.
__device__ void fit_track(const int32_t* hits, uint32_t mask, const float* clu_x, const float* clu_y,
                          const Params& p, float* par) {
    const FitResult f = fit_track_hits([&](int, int i) { return hits[i]; }, mask, clu_x, clu_y, p.z, p.sigma);
    float4* o = reinterpret_cast<float4*>(par);
    o[0] = make_float4(f.xr, f.yr, f.zr, f.tx);
    o[1] = make_float4(f.ty, f.chi2, (float)f.ndof, 0.0f);
}

// CSR compaction of one event's output tracks (one workgroup per event).
__global__ __launch_bounds__(256) void k_output(OutArgs a) {
    __shared__ int s_wt[256 / kWave], s_wh[256 / kWave];
    __shared__ int carry_t, carry_h;
    const int e = blockIdx.x;
    if (e >= a.n_events) return;
    const Work& w = a.w;
    const int nc = w.ev_ncand[e];
    const int64_t slot0 = a.clu_off[e * kPlanes];
    const int64_t tbase = w.ev_tbase[e], hbase = w.ev_hbase[e];
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    if (threadIdx.x == 0) { carry_t = 0; carry_h = 0; }
    __syncthreads();
    bool overflow = false;
    for (int base = 0; base < nc; base += 256) {
        const int c = base + threadIdx.x;
        int out = 0, nh = 0;
        uint32_t mask = 0;
        uint8_t fl = 0;
        if (c < nc) {
            fl = w.cflags[slot0 + c];
            out = (a.emit_rejected || (fl & TRK_ACCEPT)) ? 1 : 0;
            mask = w.cmask[slot0 + c];
            nh = out ? __popc(mask) : 0;
        }
        int tt, th;
        const int et = wave_excl_scan(out, &tt);
        const int eh = wave_excl_scan(nh, &th);
        if (lane == 0) { s_wt[wid] = tt; s_wh[wid] = th; }
        __syncthreads();
        int pt = carry_t, ph = carry_h;
        for (int i = 0; i < wid; ++i) { pt += s_wt[i]; ph += s_wh[i]; }
        if (out) {
            const int64_t t = tbase + pt + et;
            const int64_t h = hbase + ph + eh;
            if (t < a.trk_cap && h + nh <= a.hit_cap) {
                a.trk_hit_off[t] = (int32_t)h;
                a.trk_planes[t] = mask;
                if (a.trk_flags) a.trk_flags[t] = fl;
                if (a.trk_logit) a.trk_logit[t] = w.clogit[slot0 + c];
                // every plane slot of the candidate (and its fit) is read
                // before the first store, so that the copy waits once
                const int32_t* ch = w.chits + (slot0 + c) * kPlanes;
                int32_t hv[kPlanes];
#pragma unroll
                for (int k = 0; k < kPlanes; ++k) hv[k] = ch[k];
                float4 f0, f1;
                if (a.par) {  // the acceptance step's fit of these hits (same function, same bits)
                    const float4* src = reinterpret_cast<const float4*>(w.cpar + (slot0 + c) * 8);
                    f0 = src[0];
                    f1 = src[1];
                }
                int j = 0;
#pragma unroll
                for (int k = 0; k < kPlanes; ++k)
                    if (mask & (1u << k)) a.trk_hit[h + j++] = hv[k];
                if (a.par) {
                    float4* dst = reinterpret_cast<float4*>(a.par + t * 8);
                    dst[0] = f0;
                    dst[1] = f1;
                }
            } else {
                overflow = true;
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int i = 0; i < 256 / kWave; ++i) { carry_t += s_wt[i]; carry_h += s_wh[i]; }
        }
        __syncthreads();
    }
    if (__syncthreads_or(overflow) && threadIdx.x == 0) set_event_flag(a.status, e, EV_OVERFLOW, 1);
}

__global__ __launch_bounds__(256) void k_fit(FitArgs a) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = a.n_tracks ? (int64_t)*a.n_tracks : a.max_tracks;
    if (t >= n || t >= a.max_tracks) return;
    fit_track(a.trk_hit + a.trk_hit_off[t], a.trk_planes[t], a.clu_x, a.clu_y, a.p, a.par + t * 8);
}

}  // namespace

hipError_t launch_reset(const Work& w, int n_events, int32_t* status, hipStream_t s) {
    const int64_t n = (int64_t)n_events * kPlanes + kStatusHdr + 8;
    const int grid = (int)std::min<int64_t>(1024, (n + 255) / 256);
    hipLaunchKernelGGL(k_reset, dim3(grid), dim3(256), 0, s, w, n_events, status);
    return hipGetLastError();
}

hipError_t launch_order(const Work& w, int n_events, const int32_t* clu_off, int kp, int32_t* big, int big_count,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_order, dim3(1), dim3(1024), 0, s, w, n_events, clu_off, kp, big, big_count);
    return hipGetLastError();
}

hipError_t launch_scan(const OutArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanThreads), 0, s, a.w, a.n_events, a.trk_off, a.trk_hit_off,
                       a.trk_cap, a.status, a.emit_rejected);
    return hipGetLastError();
}

hipError_t launch_output(const OutArgs& a, hipStream_t s) {
    if (a.n_events == 0) return hipSuccess;
    hipLaunchKernelGGL(k_output, dim3(a.n_events), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fit(const FitArgs& a, hipStream_t s) {
    if (a.max_tracks <= 0) return hipSuccess;
    const int64_t grid = (a.max_tracks + 255) / 256;
    hipLaunchKernelGGL(k_fit, dim3((unsigned)grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace velo
