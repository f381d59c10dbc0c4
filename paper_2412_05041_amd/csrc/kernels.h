// kernels.h -- kernel argument blocks and host launchers (internal to libvelo).
#pragma once

#include "common.h"

namespace velo {

struct ClusterArgs {
    int n_seg;  // events * 26
    const int32_t* pix_off;
    const uint32_t* pix_id;
    int32_t* pix_clu;
    int32_t* clu_off;
    float* clu_x;
    float* clu_y;
    int32_t* clu_npix;
    int64_t clu_cap;
    int32_t* status;
    int validate;
    int stage;  // also write the azimuth-sorted staging (fused pipeline)
    Work w;
};

struct StageArgs {
    int n_seg;
    const int32_t* clu_off;
    const float* clu_x;
    const float* clu_y;
    Work w;
};

struct FindArgs {
    int n_events;
    const int32_t* clu_off;
    const float* clu_x;
    const float* clu_y;
    int32_t* status;
    Params p;
    Work w;
    const float* mlp_master;  // learned mode: FP32 master weights (device)
    const float* mlp_norm;    // 20 floats
    int64_t clu_limit;        // events whose clusters reach beyond this are not processed
    // LDS-tile admission: an event with more clusters than admit x (the tile's
    // track capacity) goes straight to the next pass (0: planes alone decide)
    float admit;
    // event queue of an LDS-tile pass: events q_in[0 .. n) with n = n_events
    // (q_count < 0) or counters[q_count], taken through counters[q_cursor];
    // events that do not fit go to q_out, counted in counters[q_out_count]
    const int32_t* q_in;
    int q_count, q_cursor, q_out_count;
    int32_t* q_out;
    const float* seed_net;    // seed filter network, kSeedFloats (null: no seed filter)
    float* seed_feat;         // seed emission for training: [seed_cap][10] features (null: off)
    int32_t* seed_hits;       // [seed_cap][3] global cluster indices
    int64_t seed_cap;
    unsigned long long* seed_count;  // candidates seen (may exceed seed_cap)
};

// Forward extrapolation through a single-kink magnet (velo_extrapolate).
struct ExtrapArgs {
    int64_t max_tracks;
    const int32_t* n_tracks;  // device count (nullable: max_tracks)
    const float* par;         // [max_tracks][8] VELO states (x, y, z, tx, ty, ...), 16-byte aligned
    const float* x_hit;       // [max_tracks] x of a hit at z_t (nullable)
    float z_mag, z_t, kick, p_min;
    float* out;               // [max_tracks][8], 16-byte aligned
};

struct OutArgs {
    int n_events;
    const int32_t* clu_off;
    const float* clu_x;
    const float* clu_y;
    int32_t* trk_off;
    int32_t* trk_hit_off;
    int32_t* trk_hit;
    uint32_t* trk_planes;
    uint8_t* trk_flags;
    float* trk_logit;
    float* par;  // fused fit output (nullable)
    int64_t trk_cap, hit_cap;
    int emit_rejected;
    int32_t* status;
    Params p;
    Work w;
};

struct FitArgs {
    int64_t max_tracks;
    const int32_t* n_tracks;  // nullable
    const int32_t* trk_hit_off;
    const int32_t* trk_hit;
    const uint32_t* trk_planes;
    const float* clu_x;
    const float* clu_y;
    float* par;
    Params p;
};

struct KalmanArgs {
    int64_t max_tracks;
    const int32_t* n_tracks;  // nullable
    const int32_t* trk_hit_off;
    const int32_t* trk_hit;
    const uint32_t* trk_planes;
    const float* clu_x;
    const float* clu_y;
    float* out;               // [max_tracks][16]
    float z[kPlanes];
    float sigma;              // measurement error (mm)
    float ms;                 // slope kick per plane crossed (rad)
};

struct DecodeArgs {
    int n_seg;                // events * 26
    const int32_t* bank_off;  // [n_seg + 1] word offsets
    const uint32_t* bank;     // super-pixel words
    int32_t* pix_off;         // [n_seg + 1]
    uint32_t* pix_id;         // [pix_cap]
    int64_t pix_cap;
    int32_t* status;          // nullable
    Work w;                   // seg_m: per-plane pixel counts
};

// launchers (return hipError_t)
hipError_t launch_reset(const Work& w, int n_events, int32_t* status, hipStream_t s);
hipError_t launch_order(const Work& w, int n_events, const int32_t* clu_off, int kp, int32_t* big, int big_count,
                        hipStream_t s);
hipError_t launch_cluster(const ClusterArgs& a, hipStream_t s);
hipError_t launch_stage(const StageArgs& a, hipStream_t s);
// The finder's three passes over the lists k_order made: the configured LDS
// tile over the events that fit it (w.order); the next larger tile (512
// threads per event) over those that did not, and over those that overflowed
// the first tile's track or candidate capacity (w.large; tiles 0 and 1); the
// global-memory finder over what neither took (w.large2).  Plane capacity of
// each tile: tile_planes.
int tile_planes(int tile);
hipError_t launch_finder_first(FindArgs a, int threads, int tile, int grid, hipStream_t s);
hipError_t launch_finder_second(FindArgs a, int tile, int grid, hipStream_t s);
hipError_t launch_finder_large(FindArgs a, hipStream_t s);
constexpr int kSecondPassThreads = 512;
hipError_t launch_accept(const FindArgs& a, hipStream_t s);
hipError_t launch_scan(const OutArgs& a, hipStream_t s);
hipError_t launch_output(const OutArgs& a, hipStream_t s);
hipError_t launch_fit(const FitArgs& a, hipStream_t s);
hipError_t launch_extrapolate(const ExtrapArgs& a, hipStream_t s);
hipError_t launch_kalman(const KalmanArgs& a, hipStream_t s);
hipError_t launch_decode(const DecodeArgs& a, hipStream_t s);

// Records `msg` as this thread's velo_last_error() and returns `code`.
int set_last_error(int code, const char* msg);

}  // namespace velo
