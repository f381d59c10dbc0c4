// k_cluster.hip -- pixel clustering and azimuth-sorted hit staging.
//
// Four launches: (1) clustering with segment-local numbering, centroids
// parked in the per-pixel scratch, one wave64 workgroup per (event, plane)
// segment of at most 512 pixels; (2) the same for the larger segments, one
// 256-thread workgroup each; (3) exclusive scan of the per-segment cluster
// counts into the cluster offsets; (4) global numbering, centroid output and,
// for the fused pipeline, the azimuth-sorted staging of each segment, one
// wave per segment.
//
// Clustering = 8-connected components of the fired pixels.  Each pixel unites
// with its neighbours of smaller id (same row: id-1; previous row: the three
// ids around id-1454, with the column checked so that rows never wrap).
// Union-find links the larger root under the smaller with atomicMin, so the
// surviving root of a component is its smallest index = smallest pixel id.
// Roots are numbered by a wave prefix sum in index order; integer column/row
// sums give the centroid x = ((float)sum_c / (float)n - 726.5f) * 0.055f.
#include "kernels.h"

namespace velo {

namespace {

constexpr int kCap = 512;                          // pixels of a segment one wave clusters in LDS
constexpr int kBigWaves = 4;                       // waves of a workgroup that clusters one large segment
constexpr int kGroupThreads = kBigWaves * kWave;
constexpr int kGroupCap = kBigWaves * kCap;        // pixels of a segment such a workgroup clusters in LDS
constexpr int kFinalCap = 1024;                    // pixels of a segment the numbering pass keeps in registers
constexpr int kStageCap = 512;                     // clusters of a segment staged from registers and LDS

// Packed per-cluster sums of a segment clustered in LDS, one 64-bit word:
// [sum of columns:26 | pixel count:12 | sum of rows:26].
constexpr int kSumBits = 26, kCntBits = 12;
static_assert(kGroupCap < (1 << kCntBits) && (int64_t)kGroupCap * (kSide - 1) < (1ll << kSumBits),
              "a segment's packed sums fit their fields");
__device__ __forceinline__ unsigned long long pack_pixel(uint32_t c, uint32_t r) {
    return ((unsigned long long)c << (kSumBits + kCntBits)) | (1ull << kSumBits) | (unsigned long long)r;
}
constexpr int kSmallBuckets = 256;   // staging buckets for segments in LDS

template <typename P>
__device__ __forceinline__ int ld_rlx(P* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

template <typename P>
__device__ __forceinline__ int find_root(P* par, int a) {
    int p = ld_rlx(par + a);
    while (p != a) {
        a = p;
        p = ld_rlx(par + a);
    }
    return a;
}

template <typename P>
__device__ __forceinline__ void unite(P* par, int a, int b) {
    while (true) {
        a = find_root(par, a);
        b = find_root(par, b);
        if (a == b) return;
        if (a < b) { const int t = a; a = b; b = t; }
        const int old = atomicMin(par + a, b);
        if (old == a) return;
        a = old;  // a gained a parent meanwhile: unite that parent with b
    }
}

// A pixel id the sensor has: below 1454^2 and outside the central hole.
__device__ __forceinline__ bool valid_pixel(uint32_t id) {
    if (id >= (uint32_t)(kSide * kSide)) return false;
    const int dc = 2 * (int)(id % kSide) - (kSide - 1), dr = 2 * (int)(id / kSide) - (kSide - 1);
    return dc * dc + dr * dr >= kHoleD2;
}

template <typename Id>
__device__ __forceinline__ int lower_bound_u32(const Id* a, int n, uint32_t v) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

template <typename Id, typename P>
__device__ __forceinline__ void unite_neighbours(const Id* ids, P* par, int i) {
    const uint32_t id = ids[i];
    const uint32_t c = id % kSide, r = id / kSide;
    if (c > 0 && i > 0 && ids[i - 1] == id - 1) unite(par, i, i - 1);
    if (r == 0) return;
    const uint32_t lo = id - kSide - (c > 0 ? 1u : 0u);
    const uint32_t hi = id - kSide + (c < kSide - 1 ? 1u : 0u);
    for (int j = lower_bound_u32(ids, i, lo); j < i && ids[j] <= hi; ++j) unite(par, i, j);
}


// Synchronisation and prefix sums of a group of G threads that clusters one
// segment: one wave (lockstep lanes; a fence orders the accesses, no barrier)
// or the whole workgroup.  t: thread index in the group; wsum: per-wave
// totals in LDS (whole-workgroup groups only).
template <int G>
struct Group {
    int t;
    int* wsum;
    __device__ void sync() const {
        if constexpr (G == kWave) wave_sync(); else __syncthreads();
    }
    __device__ bool any(int v) const {
        if constexpr (G == kWave) {
            wave_sync();
            return __ballot(v) != 0ull;
        } else {
            return __syncthreads_or(v) != 0;
        }
    }
    // exclusive prefix sum of v in thread order, and the total (uniform call)
    __device__ int excl_scan(int v, int* total) const {
        int tot;
        const int ex = wave_excl_scan(v, &tot);
        if constexpr (G == kWave) {
            *total = tot;
            return ex;
        } else {
            const int wv = t / kWave;
            if (t % kWave == 0) wsum[wv] = tot;
            __syncthreads();
            int base = 0, all = 0;
#pragma unroll
            for (int q = 0; q < G / kWave; ++q) {
                const int sq = wsum[q];
                base += q < wv ? sq : 0;
                all += sq;
            }
            __syncthreads();
            *total = all;
            return base + ex;
        }
    }
};

// Azimuth-sorted staging of the m clusters of one segment, by (key, index).
// kbuf/tbuf: m-element scratch; hist: nb counters (LDS).  Staged entry g =
// gbase + rank holds x, y, key and the global cluster index gbase + j.
template <int kNb, typename KB, typename TB>
__device__ void stage_segment(const float* cx, const float* cy, int m, int64_t gbase, KB* kbuf, TB* tbuf,
                              uint32_t* hist, const Work& w) {
    constexpr int kShift = kKeyBits - __builtin_ctz(kNb);
    const int lane = threadIdx.x;
    for (int b = lane; b < kNb; b += kWave) hist[b] = 0;
    __syncthreads();
    for (int j = lane; j < m; j += kWave) {
        const int k = phi_key(atan2f(cy[j], cx[j]));
        kbuf[j] = (uint32_t)k;
        atomicAdd(hist + (k >> kShift), 1u);
    }
    __syncthreads();
    {
        constexpr int per = kNb / kWave;
        uint32_t loc[per];
        uint32_t s = 0;
#pragma unroll
        for (int i = 0; i < per; ++i) { loc[i] = hist[lane * per + i]; s += loc[i]; }
        int tot;
        uint32_t run = (uint32_t)wave_excl_scan((int)s, &tot);
#pragma unroll
        for (int i = 0; i < per; ++i) { hist[lane * per + i] = run; run += loc[i]; }
    }
    __syncthreads();
    for (int j = lane; j < m; j += kWave) {
        const uint32_t pos = atomicAdd(hist + (kbuf[j] >> kShift), 1u);
        tbuf[pos] = j;
    }
    __syncthreads();
    // hist[b] is now the end of bucket b
    for (int p = lane; p < m; p += kWave) {
        const int j = tbuf[p];
        const uint32_t kj = kbuf[j];
        const int b = (int)(kj >> kShift);
        const int s = b ? (int)hist[b - 1] : 0, e = (int)hist[b];
        int r = s;
        for (int q = s; q < e; ++q) {
            const int i = tbuf[q];
            const uint32_t ki = kbuf[i];
            r += (ki < kj || (ki == kj && i < j)) ? 1 : 0;
        }
        const int64_t g = gbase + r;
        w.stg[g] = Staged{cx[j], cy[j], (int32_t)(gbase + j), kj};
        w.used[g] = 0;
    }
}

// Clustering of one segment with segment-local numbering by a group of G
// threads, for segments above the LDS capacity: parent and rank arrays and
// the sums in the per-pixel global scratch.  Writes pix_clu = local rank,
// seg_m = cluster count and, at pixel-indexed scratch positions p0 + j, the
// centroid x, y and pixel count of cluster j.  refuse: the scratch cannot
// hold the segment (overflow flag).
template <int G, typename Id, typename P, typename R>
__device__ void cluster_global(const ClusterArgs& a, int seg, int p0, int n, const Id* ids, P* par, R* rnk,
                               int refuse, const Group<G>& g) {
    static_assert(G == kGroupThreads, "the global-memory path runs on the whole workgroup (its phases meet at barriers)");
    const int t = g.t;
    const Work& w = a.w;
    const int e = seg / kPlanes;
    int bad = refuse;
    if (a.validate && !refuse) {
        for (int i = t; i < n; i += G) {
            const uint32_t id = ids[i];
            if (!valid_pixel(id) || (i > 0 && ids[i - 1] >= id)) bad = 1;
        }
    }
    if (g.any(bad)) {
        for (int i = t; i < n; i += G) a.pix_clu[p0 + i] = -1;
        if (t == 0) {
            w.seg_m[seg] = 0;
            set_event_flag(a.status, e, refuse ? EV_OVERFLOW : EV_BAD_INPUT, refuse ? 1 : 2);
        }
        return;
    }
    for (int i = t; i < n; i += G) par[i] = i;
    __syncthreads();
    for (int i = t; i < n; i += G) unite_neighbours(ids, par, i);
    __syncthreads();
    for (int i = t; i < n; i += G) rnk[i] = find_root(par, i);
    __syncthreads();
    // number the roots in index order; par[root] := its rank
    int m = 0;
    for (int c0 = 0; c0 < n; c0 += G) {
        const int i = c0 + t;
        const int isroot = (i < n && rnk[i] == i) ? 1 : 0;
        int tot;
        const int ex = g.excl_scan(isroot, &tot);
        if (isroot) par[i] = m + ex;
        m += tot;
    }
    __syncthreads();
    for (int i = t; i < n; i += G) rnk[i] = par[rnk[i]];
    for (int j = t; j < m; j += G) { w.g_sc[p0 + j] = 0; w.g_sr[p0 + j] = 0; w.g_cnt[p0 + j] = 0; }
    __syncthreads();
    for (int i = t; i < n; i += G) {
        const int rk = rnk[i];
        a.pix_clu[p0 + i] = rk;
        const uint32_t id = ids[i];
        atomicAdd(w.g_sc + p0 + rk, id % kSide);
        atomicAdd(w.g_sr + p0 + rk, id / kSide);
        atomicAdd(w.g_cnt + p0 + rk, 1u);
    }
    __syncthreads();
    for (int j = t; j < m; j += G) {
        const uint32_t sc = w.g_sc[p0 + j], sr = w.g_sr[p0 + j], cnt = w.g_cnt[p0 + j];
        const float fn = (float)cnt;
        // centroid parked in the scratch (same slots as the sums: read before write)
        w.g_sc[p0 + j] = __float_as_uint(((float)sc / fn - 726.5f) * 0.055f);
        w.g_sr[p0 + j] = __float_as_uint(((float)sr / fn - 726.5f) * 0.055f);
        w.g_cnt[p0 + j] = cnt;
    }
    if (t == 0) w.seg_m[seg] = m;
}

// Clustering of a segment in LDS by a group of G threads: one wave (at most
// kCap pixels) or the whole workgroup (at most kGroupCap).  Per-pixel state
// (id, root, rank; pixel i = t + G r) stays in registers; only the ids and the
// union-find parents live in LDS (one word each per pixel of the capacity),
// and once the ranks are known that space holds the packed per-cluster sums.
// Same outputs as cluster_global.
template <int G>
__device__ void cluster_lds(const ClusterArgs& a, int seg, int p0, int n, unsigned long long* s_buf,
                            const Group<G>& g) {
    constexpr int kC = G == kWave ? kCap : kGroupCap;
    constexpr int R = kC / G;
    uint32_t* s_id = reinterpret_cast<uint32_t*>(s_buf);
    int32_t* s_par = reinterpret_cast<int32_t*>(s_id + kC);
    const int t = g.t;
    const Work& w = a.w;
    if (n == 0) {
        if (t == 0) w.seg_m[seg] = 0;
        return;
    }
    // All R loads are issued before the first is used (addresses clamped into
    // the segment), so the group waits for the ids once, not once per row.
    uint32_t id[R];
#pragma unroll
    for (int r = 0; r < R; ++r) id[r] = a.pix_id[p0 + min(t + r * G, n - 1)];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = t + r * G;
        if (i < n) {
            s_id[i] = id[r];
            s_par[i] = i;
        } else {
            id[r] = 0u;
        }
    }
    g.sync();
    int bad = 0;
    if (a.validate) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = t + r * G;
            if (i < n && (!valid_pixel(id[r]) || (i > 0 && s_id[i - 1] >= id[r]))) bad = 1;
        }
    }
    if (g.any(bad)) {
        for (int i = t; i < n; i += G) a.pix_clu[p0 + i] = -1;
        if (t == 0) {
            w.seg_m[seg] = 0;
            set_event_flag(a.status, seg / kPlanes, EV_BAD_INPUT, 2);
        }
        return;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = t + r * G;
        if (i < n) unite_neighbours(s_id, s_par, i);
    }
    g.sync();
    int root[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = t + r * G;
        root[r] = i < n ? find_root(s_par, i) : -1;
    }
    g.sync();
    // number the roots in index order; par[root] := its rank
    int m = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = t + r * G;
        const int isroot = root[r] == i ? 1 : 0;
        int tot;
        const int ex = g.excl_scan(isroot, &tot);
        if (isroot) s_par[i] = m + ex;
        m += tot;
    }
    g.sync();
    int rank[R];
#pragma unroll
    for (int r = 0; r < R; ++r) rank[r] = root[r] >= 0 ? s_par[root[r]] : 0;
    g.sync();
    // ids and parents are dead: the same words hold the packed sums
    unsigned long long* s_sum = s_buf;
    for (int j = t; j < m; j += G) s_sum[j] = 0;
    g.sync();
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = t + r * G;
        if (i < n) {
            a.pix_clu[p0 + i] = rank[r];
            atomicAdd(s_sum + rank[r], pack_pixel(id[r] % kSide, id[r] / kSide));
        }
    }
    g.sync();
    for (int j = t; j < m; j += G) {
        const unsigned long long v = s_sum[j];
        const uint32_t sc = (uint32_t)(v >> (kSumBits + kCntBits));
        const uint32_t cnt = (uint32_t)((v >> kSumBits) & ((1u << kCntBits) - 1u));
        const uint32_t sr = (uint32_t)(v & ((1ull << kSumBits) - 1ull));
        const float fn = (float)cnt;
        w.g_sc[p0 + j] = __float_as_uint(((float)sc / fn - 726.5f) * 0.055f);
        w.g_sr[p0 + j] = __float_as_uint(((float)sr / fn - 726.5f) * 0.055f);
        w.g_cnt[p0 + j] = cnt;
    }
    if (t == 0) w.seg_m[seg] = m;
}

// Counter of the segments k_cluster leaves to k_cluster_big (zeroed with the
// other counters before every clustering).
constexpr int kBigSegCounter = 7;

// One wave per segment of at most kCap pixels; a larger segment (or one the
// scratch refuses) is appended to the list k_cluster_big works through.
__global__ __launch_bounds__(kWave) void k_cluster(ClusterArgs a) {
    __shared__ unsigned long long s_buf[kCap];
    const int seg = blockIdx.x;
    if (seg >= a.n_seg) return;
    const Work& w = a.w;
    const int p0 = a.pix_off[seg];
    const int n = a.pix_off[seg + 1] - p0;
    // the per-pixel scratch covers pixel positions below its capacity
    const int refuse = (int64_t)p0 + n > w.cap_scratch ? 1 : 0;
    if (n <= kCap && !refuse) {
        cluster_lds<kWave>(a, seg, p0, n, s_buf, Group<kWave>{(int)threadIdx.x, nullptr});
    } else if (threadIdx.x == 0) {
        w.seg_big[atomicAdd(w.counters + kBigSegCounter, 1)] = seg;
    }
}

// The segments k_cluster left over, one 256-thread workgroup each (a grid
// smaller than the list takes several in turn): in LDS up to kGroupCap
// pixels, else in global memory.
constexpr int kBigGrid = 1024;
__global__ __launch_bounds__(kGroupThreads) void k_cluster_big(ClusterArgs a) {
    __shared__ unsigned long long s_buf[kGroupCap];
    __shared__ int s_wsum[kBigWaves];
    const Work& w = a.w;
    const int nb = w.counters[kBigSegCounter];
    const Group<kGroupThreads> grp{(int)threadIdx.x, s_wsum};
    for (int q = blockIdx.x; q < nb; q += gridDim.x) {
        const int seg = w.seg_big[q];
        const int p0 = a.pix_off[seg];
        const int n = a.pix_off[seg + 1] - p0;
        const int refuse = (int64_t)p0 + n > w.cap_scratch ? 1 : 0;
        if (n <= kGroupCap && !refuse) {
            cluster_lds<kGroupThreads>(a, seg, p0, n, s_buf, grp);
        } else {
            cluster_global<kGroupThreads>(a, seg, p0, n, a.pix_id + p0, w.g_par + p0, w.g_tmp + p0, refuse, grp);
        }
        __syncthreads();  // the LDS is free for the next segment
    }
}

// Exclusive scan of the segment cluster counts -> clu_off (single workgroup).
// Each thread scans a contiguous chunk, reading it 8 counts at a time so that
// the loads of a group are in flight together.
__global__ __launch_bounds__(1024) void k_scan_seg(ClusterArgs a) {
    __shared__ int64_t s_w[1024 / kWave];
    __shared__ int64_t s_carry;
    const Work& w = a.w;
    const int n = a.n_seg;
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    const int per = (n + 1023) / 1024;
    const int b0 = min(n, (int)threadIdx.x * per), b1 = min(n, b0 + per);
    int64_t loc = 0;
    int i = b0;
    for (; i + 8 <= b1; i += 8) {
        int v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = w.seg_m[i + q];
#pragma unroll
        for (int q = 0; q < 8; ++q) loc += v[q];
    }
    for (; i < b1; ++i) loc += w.seg_m[i];
    int tot;
    // 64-bit chunk sums are small (< 2^31 clusters in a batch): scan them as int
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
        for (int q = 0; q < 8; ++q) v[q] = w.seg_m[i + q];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            a.clu_off[i + q] = (int32_t)run;
            run += v[q];
        }
    }
    for (; i < b1; ++i) {
        a.clu_off[i] = (int32_t)run;
        run += w.seg_m[i];
    }
    if (threadIdx.x == 0) {
        a.clu_off[n] = (int32_t)s_carry;
        if (a.status) {
            a.status[ST_NCLU] = (int32_t)s_carry;
            a.status[ST_NPIX] = a.pix_off[n];
        }
    }
}

// Global numbering, centroid output and (fused pipeline) staging.
// LDS of a staging wave, 4 KB: a segment of at most kStageCap clusters sorts in it
// (keys, 16-bit positions, kSmallBuckets counters); a larger one keeps its
// keys and positions in the per-pixel scratch and its kBuckets counters here.
struct StageLds {
    uint32_t w[kBuckets];
    __device__ uint32_t* keys() { return w; }
    __device__ uint16_t* pos() { return reinterpret_cast<uint16_t*>(w + kStageCap); }
    __device__ uint32_t* hist_small() { return w + kStageCap + kStageCap / 2; }
    static_assert(kStageCap + kStageCap / 2 + kSmallBuckets <= kBuckets, "the small layout fits");
};

// Azimuth-sorted staging by (key, index) of m <= kStageCap clusters whose
// coordinates a wave holds in registers (cluster j = lane + 64 r): bucket
// counts, bucket starts, bucket members, then each cluster's rank among its
// bucket's members.  Staged entry cb + rank holds x, y, key and the global
// cluster index cb + j.
__device__ void stage_regs(const float (&cx)[kStageCap / kWave], const float (&cy)[kStageCap / kWave], int m,
                           int64_t cb, StageLds& lds, const Work& w) {
    constexpr int RM = kStageCap / kWave;
    constexpr int kNb = kSmallBuckets;
    constexpr int kShift = kKeyBits - __builtin_ctz(kNb);
    const int lane = threadIdx.x;
    uint32_t* kbuf = lds.keys();
    uint16_t* tbuf = lds.pos();
    uint32_t* hist = lds.hist_small();
    for (int b = lane; b < kNb; b += kWave) hist[b] = 0;
    __syncthreads();
    uint32_t key[RM];
#pragma unroll
    for (int r = 0; r < RM; ++r) {
        const int j = lane + r * kWave;
        key[r] = 0;
        if (j < m) {
            key[r] = (uint32_t)phi_key(atan2f(cy[r], cx[r]));
            kbuf[j] = key[r];
            atomicAdd(hist + (key[r] >> kShift), 1u);
        }
    }
    __syncthreads();
    {
        constexpr int per = kNb / kWave;
        uint32_t loc[per];
        uint32_t t = 0;
#pragma unroll
        for (int i = 0; i < per; ++i) { loc[i] = hist[lane * per + i]; t += loc[i]; }
        int tot;
        uint32_t run = (uint32_t)wave_excl_scan((int)t, &tot);
#pragma unroll
        for (int i = 0; i < per; ++i) { hist[lane * per + i] = run; run += loc[i]; }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RM; ++r) {
        const int j = lane + r * kWave;
        if (j < m) tbuf[atomicAdd(hist + (key[r] >> kShift), 1u)] = (uint16_t)j;
    }
    __syncthreads();
    // hist[b] is now the end of bucket b
#pragma unroll
    for (int r = 0; r < RM; ++r) {
        const int j = lane + r * kWave;
        if (j < m) {
            const uint32_t kj = key[r];
            const int b = (int)(kj >> kShift);
            const int e = (int)hist[b];
            int rank = b ? (int)hist[b - 1] : 0;
            for (int q = rank; q < e; ++q) {
                const int i = tbuf[q];
                const uint32_t ki = kbuf[i];
                rank += (ki < kj || (ki == kj && i < j)) ? 1 : 0;
            }
            const int64_t g = cb + rank;
            w.stg[g] = Staged{cx[r], cy[r], (int32_t)(cb + j), kj};
            w.used[g] = 0;
        }
    }
}

// Global numbering, centroid output and staging of a segment of at most
// kFinalCap pixels and kStageCap clusters, one wave.  Every global load (the segment's
// local labels and parked centroids) is issued at once into registers, with
// addresses clamped into the segment; the staging then works from registers
// and LDS.  Same outputs as the general loops of k_cluster_final.
__device__ void final_small(const ClusterArgs& a, int seg, int p0, int n, int64_t cb, int m, StageLds& lds) {
    constexpr int R = kFinalCap / kWave;
    constexpr int RM = kStageCap / kWave;
    const int lane = threadIdx.x;
    const Work& w = a.w;
    int32_t lab[R];
    float cx[RM], cy[RM];
    uint32_t cnt[RM];
    if (n > 0) {
#pragma unroll
        for (int r = 0; r < R; ++r) lab[r] = a.pix_clu[p0 + min(lane + r * kWave, n - 1)];
    }
    if (m > 0) {
        const float* tx = reinterpret_cast<const float*>(w.g_sc + p0);
        const float* ty = reinterpret_cast<const float*>(w.g_sr + p0);
#pragma unroll
        for (int r = 0; r < RM; ++r) {
            const int j = min(lane + r * kWave, m - 1);
            cx[r] = tx[j];
            cy[r] = ty[j];
            cnt[r] = w.g_cnt[p0 + j];
        }
    }
    if (n > 0) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = lane + r * kWave;
            if (i < n && lab[r] >= 0) a.pix_clu[p0 + i] = (int32_t)(cb + lab[r]);
        }
    }
    if (m <= 0) return;
    if (cb + m > a.clu_cap) {
        if (lane == 0) set_event_flag(a.status, seg / kPlanes, EV_OVERFLOW, 1);
        return;
    }
#pragma unroll
    for (int r = 0; r < RM; ++r) {
        const int j = lane + r * kWave;
        if (j < m) {
            a.clu_x[cb + j] = cx[r];
            a.clu_y[cb + j] = cy[r];
            if (a.clu_npix) a.clu_npix[cb + j] = (int32_t)cnt[r];
        }
    }
    if (a.stage) stage_regs(cx, cy, m, cb, lds, w);
}

__global__ __launch_bounds__(kWave) void k_cluster_final(ClusterArgs a) {
    __shared__ StageLds s_lds;
    const int seg = blockIdx.x;
    if (seg >= a.n_seg) return;
    const Work& w = a.w;
    const int p0 = a.pix_off[seg];
    const int n = a.pix_off[seg + 1] - p0;
    const int64_t cb = a.clu_off[seg];
    const int m = a.clu_off[seg + 1] - (int)cb;
    // refused in the first pass (m is always >= 0: the test only makes the
    // branch need both offset loads, so that they are in flight together)
    if (((int64_t)p0 + n > w.cap_scratch) | (m < 0)) return;
    if (n <= kFinalCap && m <= kStageCap) {
        final_small(a, seg, p0, n, cb, m, s_lds);
        return;
    }
    for (int i = threadIdx.x; i < n; i += kWave) {
        const int32_t v = a.pix_clu[p0 + i];
        if (v >= 0) a.pix_clu[p0 + i] = (int32_t)(cb + v);
    }
    if (m <= 0) return;
    if (cb + m > a.clu_cap) {
        if (threadIdx.x == 0) set_event_flag(a.status, seg / kPlanes, EV_OVERFLOW, 1);
        return;
    }
    const float* tx = reinterpret_cast<const float*>(w.g_sc + p0);
    const float* ty = reinterpret_cast<const float*>(w.g_sr + p0);
    for (int j = threadIdx.x; j < m; j += kWave) {
        a.clu_x[cb + j] = tx[j];
        a.clu_y[cb + j] = ty[j];
        if (a.clu_npix) a.clu_npix[cb + j] = (int32_t)w.g_cnt[p0 + j];
    }
    if (!a.stage) return;
    if (m <= kStageCap) {
        stage_segment<kSmallBuckets>(tx, ty, m, cb, s_lds.keys(), s_lds.pos(), s_lds.hist_small(), w);
    } else {
        stage_segment<kBuckets>(tx, ty, m, cb, (uint32_t*)(w.g_par + p0), w.g_tmp + p0, s_lds.w, w);
    }
}

// Staging alone (velo_find_tracks on caller-provided clusters): one wave per segment.
__global__ __launch_bounds__(kWave) void k_stage(StageArgs a) {
    __shared__ StageLds s_lds;
    const int seg = blockIdx.x;
    if (seg >= a.n_seg) return;
    const int64_t cb = a.clu_off[seg];
    const int m = a.clu_off[seg + 1] - (int)cb;
    if (m <= 0 || cb + m > a.w.cap_clusters) return;  // the finder flags such events
    if (m <= kStageCap) {
        // coordinates loaded at once into registers (addresses clamped into the segment)
        constexpr int RM = kStageCap / kWave;
        float cx[RM], cy[RM];
#pragma unroll
        for (int r = 0; r < RM; ++r) {
            const int64_t j = cb + min((int)threadIdx.x + r * kWave, m - 1);
            cx[r] = a.clu_x[j];
            cy[r] = a.clu_y[j];
        }
        stage_regs(cx, cy, m, cb, s_lds, a.w);
    } else {
        stage_segment<kBuckets>(a.clu_x + cb, a.clu_y + cb, m, cb, (uint32_t*)(a.w.g_par + cb), a.w.g_tmp + cb,
                                s_lds.w, a.w);
    }
}

}  // namespace

// The counters must be zero (launch_reset), as before every clustering.
hipError_t launch_cluster(const ClusterArgs& a, hipStream_t s) {
    if (a.n_seg <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cluster, dim3(a.n_seg), dim3(kWave), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cluster_big, dim3(a.n_seg < kBigGrid ? a.n_seg : kBigGrid), dim3(kGroupThreads), 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_seg, dim3(1), dim3(1024), 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cluster_final, dim3(a.n_seg), dim3(kWave), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_stage(const StageArgs& a, hipStream_t s) {
    if (a.n_seg <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_stage, dim3(a.n_seg), dim3(kWave), 0, s, a);
    return hipGetLastError();
}

}  // namespace velo
