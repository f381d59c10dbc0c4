// k_decode.hip -- decode of the synthetic super-pixel banks into the CSR pixel
// input of the clustering (per (event, plane): pixel ids sorted ascending).
//
// Word = pattern[0:8] | sp_row[8:17] | sp_col[17:27], bits 27..31 zero; pattern
// bit 2*dr + dc is pixel (4*sp_row + dr, 2*sp_col + dc).  A word with a reserved
// bit, an empty pattern or a pixel outside the 1454 x 1454 sensor is
// malformed: it yields nothing and flags its event (bad input).  A pixel
// decoded twice is kept and flags its event.
//
// Three launches: (1) one wave per plane counts the pixels of its valid
// words; (2) one workgroup scans the counts into pix_off; (3) one wave per
// plane sorts its pixels by a counting sort over row buckets (LDS histogram
// -> bucket starts -> scatter) followed by an insertion sort of each bucket
// by id (a lane per bucket): up to kDecCap pixels in LDS with 8-row buckets,
// above that in the output array with one bucket per row.  The order inside
// the counting sort depends on atomics; the result, sorted ids, does not.
#include "kernels.h"

namespace velo {

namespace {

constexpr int kDecCap = 1024;  // pixels of a plane sorted in LDS
constexpr int kRows = kSide;
constexpr int kSmallShift = 3;  // rows per bucket (log2) of a plane sorted in LDS

__device__ __forceinline__ bool word_ok(uint32_t w) {
    const uint32_t pattern = w & 0xffu, spr = (w >> 8) & 0x1ffu, spc = (w >> 17) & 0x3ffu;
    if ((w >> 27) != 0u || pattern == 0u) return false;
    // the highest set row / column offsets must stay on the sensor
    const uint32_t rows = (pattern & 0xc0u) ? 3u : (pattern & 0x30u) ? 2u : (pattern & 0x0cu) ? 1u : 0u;
    const uint32_t col1 = (pattern & 0xaau) ? 1u : 0u;
    return 4u * spr + rows < (uint32_t)kSide && 2u * spc + col1 < (uint32_t)kSide;
}

__global__ __launch_bounds__(kWave) void k_dec_count(DecodeArgs a) {
    const int seg = blockIdx.x;
    if (seg >= a.n_seg) return;
    const int lane = threadIdx.x;
    const int b0 = a.bank_off[seg], b1 = a.bank_off[seg + 1];
    int cnt = 0, bad = 0;
    for (int i = b0 + lane; i < b1; i += kWave) {
        const uint32_t w = a.bank[i];
        if (word_ok(w)) cnt += __popc(w & 0xffu);
        else bad = 1;
    }
    int tot;
    wave_excl_scan(cnt, &tot);
    if (__ballot(bad) != 0ull && lane == 0) set_event_flag(a.status, seg / kPlanes, EV_BAD_INPUT, 2);
    if (lane == 0) a.w.seg_m[seg] = tot;
}

__global__ __launch_bounds__(1024) void k_dec_scan(DecodeArgs a) {
    __shared__ int64_t s_w[1024 / kWave];
    __shared__ int64_t s_carry;
    const int n = a.n_seg;
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    const int per = (n + 1023) / 1024;
    const int b0 = min(n, (int)threadIdx.x * per), b1 = min(n, b0 + per);
    int64_t loc = 0;
    int i = b0;
    for (; i + 8 <= b1; i += 8) {  // 8 counts per load group
        int v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = a.w.seg_m[i + q];
#pragma unroll
        for (int q = 0; q < 8; ++q) loc += v[q];
    }
    for (; i < b1; ++i) loc += a.w.seg_m[i];
    int tot;
    const int ex = wave_excl_scan((int)loc, &tot);
    if (lane == 0) s_w[wid] = tot;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t c = 0;
        for (int q = 0; q < 1024 / kWave; ++q) { const int64_t t = s_w[q]; s_w[q] = c; c += t; }
        s_carry = c;
    }
    __syncthreads();
    int64_t run = s_w[wid] + ex;
    i = b0;
    for (; i + 8 <= b1; i += 8) {
        int v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = a.w.seg_m[i + q];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            a.pix_off[i + q] = (int32_t)run;
            run += v[q];
        }
    }
    for (; i < b1; ++i) {
        a.pix_off[i] = (int32_t)run;
        run += a.w.seg_m[i];
    }
    if (threadIdx.x == 0) {
        a.pix_off[n] = (int32_t)s_carry;
        if (a.status) a.status[ST_NPIX] = (int32_t)s_carry;
    }
}

__global__ __launch_bounds__(kWave) void k_dec_sort(DecodeArgs a) {
    // one LDS buffer: 8-row buckets + the plane's ids (small planes), or the
    // per-row buckets alone (large planes, ids in the output array)
    constexpr int kSmallBuckets = (kRows + (1 << kSmallShift) - 1) >> kSmallShift;
    static_assert(kSmallBuckets + kDecCap <= kRows, "LDS layout");
    __shared__ uint32_t s_buf[kRows];
    uint32_t* s_row = s_buf;
    uint32_t* s_tmp = s_buf + kSmallBuckets;
    const int seg = blockIdx.x;
    if (seg >= a.n_seg) return;
    const int lane = threadIdx.x;
    const int64_t p0 = a.pix_off[seg];
    const int n = a.pix_off[seg + 1] - (int)p0;
    if (n == 0) return;
    if (p0 + n > a.pix_cap) {  // the plane does not fit: offsets only
        if (lane == 0) set_event_flag(a.status, seg / kPlanes, EV_OVERFLOW, 1);
        return;
    }
    const bool in_lds = n <= kDecCap;
    uint32_t* dst = in_lds ? s_tmp : a.pix_id + p0;
    const int shift = in_lds ? kSmallShift : 0;
    const int nb = (kRows + (1 << shift) - 1) >> shift;
    const int b0 = a.bank_off[seg], b1 = a.bank_off[seg + 1];
    for (int r = lane; r < nb; r += kWave) s_row[r] = 0u;
    wave_sync();
    // bucket histogram
    for (int i = b0 + lane; i < b1; i += kWave) {
        const uint32_t w = a.bank[i];
        if (!word_ok(w)) continue;
        const uint32_t spr = (w >> 8) & 0x1ffu;
        for (int bit = 0; bit < 8; ++bit)
            if ((w >> bit) & 1u) atomicAdd(s_row + ((4u * spr + (uint32_t)(bit >> 1)) >> shift), 1u);
    }
    wave_sync();
    // bucket starts: each lane scans a contiguous chunk of buckets
    {
        const int per = (nb + kWave - 1) / kWave;
        const int r0 = min(nb, lane * per), r1 = min(nb, r0 + per);
        uint32_t loc = 0;
        for (int r = r0; r < r1; ++r) loc += s_row[r];
        int tot;
        uint32_t run = (uint32_t)wave_excl_scan((int)loc, &tot);
        for (int r = r0; r < r1; ++r) {
            const uint32_t c = s_row[r];
            s_row[r] = run;
            run += c;
        }
    }
    wave_sync();
    // scatter: s_row[b] becomes the end of bucket b
    for (int i = b0 + lane; i < b1; i += kWave) {
        const uint32_t w = a.bank[i];
        if (!word_ok(w)) continue;
        const uint32_t spr = (w >> 8) & 0x1ffu, spc = (w >> 17) & 0x3ffu;
        for (int bit = 0; bit < 8; ++bit) {
            if (!((w >> bit) & 1u)) continue;
            const uint32_t r = 4u * spr + (uint32_t)(bit >> 1), c = 2u * spc + (uint32_t)(bit & 1);
            const uint32_t pos = atomicAdd(s_row + (r >> shift), 1u);
            dst[pos] = r * (uint32_t)kSide + c;
        }
    }
    if (!in_lds) __threadfence();  // the scattered stores before other lanes read them
    wave_sync();
    // each bucket sorted by id (insertion sort; buckets are short), duplicates flagged
    int dup = 0;
    for (int r = lane; r < nb; r += kWave) {
        const int e = (int)s_row[r], s = r ? (int)s_row[r - 1] : 0;
        for (int i = s + 1; i < e; ++i) {
            const uint32_t v = dst[i];
            int j = i - 1;
            while (j >= s && dst[j] > v) {
                dst[j + 1] = dst[j];
                --j;
            }
            dst[j + 1] = v;
        }
        for (int i = s + 1; i < e; ++i) dup |= dst[i] == dst[i - 1] ? 1 : 0;
    }
    wave_sync();
    if (__ballot(dup) != 0ull && lane == 0) set_event_flag(a.status, seg / kPlanes, EV_BAD_INPUT, 2);
    if (in_lds)
        for (int i = lane; i < n; i += kWave) a.pix_id[p0 + i] = s_tmp[i];
}

}  // namespace

hipError_t launch_decode(const DecodeArgs& a, hipStream_t s) {
    if (a.n_seg <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_dec_count, dim3(a.n_seg), dim3(kWave), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_dec_scan, dim3(1), dim3(1024), 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_dec_sort, dim3(a.n_seg), dim3(kWave), 0, s, a);
    return hipGetLastError();
}

}  // namespace velo
