// common.h -- device-side shared definitions of libvelo (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace velo {

constexpr int kPlanes = 26;
constexpr int kSide = 1454;
// Central hole of a plane: pixel (column c, row r) exists iff
// (2c - 1453)^2 + (2r - 1453)^2 >= kHoleD2 (a 5 mm radius in half-pixel units).
constexpr int kHoleD2 = 33058;
constexpr int kStatusHdr = 8;
// Square grid over the sensor plane for disc searches on crowded planes:
// 0.5 mm cells over [-40, 40] mm in x and y.
constexpr int kGridN = 160;
constexpr int kCells = kGridN * kGridN;
constexpr float kGridInv = 2.0f;
constexpr float kGridOrg = 40.0f;
constexpr int64_t kCellWords = (int64_t)26 * (kCells + 1) + kCells;  // per workgroup
constexpr int kMaxLdsBlocksPerCu = 8;  // bound of the LDS-tile finder's grid
constexpr int kWave = 64;

// Seed-level filter network (10 -> 32 -> 32 -> 1) as the finder reads it: the
// first two weight matrices transposed ([input][unit], so the 32 lanes of a
// half-wave read one row), biases, output weights, the feature normalisation
// (10 means, 10 reciprocal standard deviations) and the rejection threshold.
constexpr int kSeedIn = 10, kSeedH = 32;
constexpr int kSeedW1T = 0, kSeedB1 = kSeedW1T + kSeedIn * kSeedH, kSeedW2T = kSeedB1 + kSeedH,
              kSeedB2 = kSeedW2T + kSeedH * kSeedH, kSeedW3 = kSeedB2 + kSeedH, kSeedB3 = kSeedW3 + kSeedH,
              kSeedNorm = kSeedB3 + 1, kSeedThr = kSeedNorm + 2 * kSeedIn, kSeedFloats = kSeedThr + 1;
constexpr float kSeedZLim = 2000.0f;  // clip of the closest-approach z feature (mm)
constexpr int kKeyBits = 16;          // azimuth key resolution
constexpr int kBuckets = 1024;        // counting-sort buckets of large segments (top 10 key bits)

// Cut set + plane positions, passed by value to every kernel that needs them.
struct Params {
    float t_max, d2_max, s_max, e_max;
    int max_skip;
    float c3, c4, sigma;
    int mode;
    float logit_band;
    float z[kPlanes];
    // conservative search radii derived on the host (pruning only, never decisive)
    float r_seed;   // >= sqrt(d2_max)
    float r_mid;    // >= sqrt(s_max)
    float r_ext;    // >= sqrt(e_max)
};

enum : int { EV_OVERFLOW = 1, EV_BAD_INPUT = 2, EV_LARGE = 4, EV_FALLBACK = 8, EV_TILE2 = 16 };
enum : int { TRK_PLAIN = 1, TRK_LEARNED = 2, TRK_FALLBACK = 4, TRK_ACCEPT = 8 };
enum : int { ST_SEVERITY = 0, ST_NCLU = 1, ST_NTRK = 2, ST_NHIT = 3, ST_NPIX = 4, ST_NLARGE = 5,
             ST_NFALLBACK = 6, ST_MAXCAND = 7 };

// A staged hit: coordinates, global cluster index and azimuth key in one
// 16-byte record, so that a hit is one vector load.
struct __align__(16) Staged {
    float x, y;
    int32_t id;
    uint32_t key;
};

// Device workspace (allocated by velo_reserve).  Per-cluster arrays are indexed
// by global cluster index; per-candidate arrays by candidate slot, where the
// candidates of event e occupy [clu_off[26 e], clu_off[26 e] + n_cand(e)).
struct Work {
    // azimuth-sorted staging of each (event, plane): x, y, key, global cluster index
    struct Staged* stg;   // one 16-byte record per staged position
    uint8_t* used;        // per staged position: hit taken
    // large-event path: each plane's hits again in grid-cell order (x, y and
    // the staged position), and per workgroup the cell starts of all planes
    // of its current event followed by one plane's fill counters
    float* g_gx;
    float* g_gy;
    int32_t* g_gpos;
    int32_t* g_cell;
    // candidates
    int32_t* chits;       // [slot][26] global cluster index of the hit on each plane
    uint32_t* cmask;      // planes bitmask
    uint8_t* cflags;      // TRK_* flags
    float* clogit;
    uint16_t* cfeat;      // [slot][16] BF16 standardised features
    float* cpar;          // [slot][8] the acceptance fit (x, y, z_ref, tx, ty, chi2, ndof, 0)
    // per event
    int32_t* ev_ncand;    // candidates
    int32_t* ev_nout;     // tracks to output
    int32_t* ev_nouthit;  // hits of those tracks
    int32_t* ev_ncandhit; // hits of all candidates (emit_rejected output)
    int32_t* ev_tbase;    // exclusive scans of ev_nout / ev_nouthit
    int32_t* ev_hbase;
    int32_t* order;       // event processing order (largest first)
    int32_t* large;       // events that did not fit the first LDS tile
    int32_t* large2;      // events that did not fit the second LDS tile either
    int32_t* seg_m;       // clusters per (event, plane) segment
    int32_t* seg_big;     // segments the one-wave clustering left to whole workgroups
    int32_t* counters;    // [1] finder events, [2] #large, [3] large-path tickets, [4] second-tile
                          // tickets, [5] #large2, [7] #seg_big, others spare
    // large-event path, per cluster (global cluster index)
    int32_t* g_claim;
    uint64_t* g_slota;
    uint32_t* g_slotb;
    float* g_ttx;         // track state, per candidate slot
    float* g_tty;
    float* g_txb;
    float* g_tyb;
    float* g_dtx;         // downstream end of new tracks
    float* g_dty;
    float* g_dxb;
    float* g_dyb;
    int32_t* g_tkb;       // planes of the two ends (bits 0-7 upstream, 8-15 downstream)
    int32_t* g_enum;      // seed-enumeration scratch, 6 per cluster
    int32_t* g_twant;
    // large-event seed pool: per block of the large kernel
    float* p_q;
    int32_t* p_h;         // [entry][3] staged positions
    uint8_t* p_alive;
    int64_t pool_cap;     // entries per block (its stride in the pool)
    int64_t pool_use;     // entries a block fills before seeding a step in key ranges (<= pool_cap)
    int32_t n_large_blocks;
    // cluster kernel global path scratch, per pixel
    int32_t* g_par;
    uint32_t* g_sc;
    uint32_t* g_sr;
    uint32_t* g_cnt;
    int32_t* g_tmp;
    int64_t cap_clusters, cap_pixels;
    int64_t cap_scratch;  // entries of the per-pixel scratch (max of pixels, clusters)
    int32_t cap_events;
};

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Monotone azimuth key: floor((phi + pi) * 2^16 / (2 pi)), clamped.  Used only
// to order hits for window searches; every decision uses the exact cuts.
__device__ __forceinline__ int phi_key(float phi) {
    const float u = (phi + 3.14159265358979f) * 10430.378350470453f;
    int k = (int)u;
    k = k < 0 ? 0 : k;
    return k > 65535 ? 65535 : k;
}

__device__ __forceinline__ void atomic_max_i32(int32_t* p, int32_t v) { atomicMax(p, v); }

__device__ __forceinline__ void set_event_flag(int32_t* status, int e, int flag, int severity) {
    if (!status) return;
    atomicOr(status + kStatusHdr + e, flag);
    atomicMax(status + ST_SEVERITY, severity);
}

// Synchronisation of the lanes of one wave (they run in lockstep: a fence
// orders the LDS accesses around the point, no workgroup barrier is needed).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Wave-wide exclusive prefix sum of v (wave64).
__device__ __forceinline__ int wave_excl_scan(int v, int* total) {
    int x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int y = __shfl_up(x, o, kWave);
        if (lane_id() >= o) x += y;
    }
    *total = __shfl(x, kWave - 1, kWave);
    return x - v;
}

}  // namespace velo
