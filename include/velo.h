/* velo.h -- C ABI of the MI355X VELO hot path (libvelo.so).
 *
 * The library reconstructs vertex-detector (VELO) track segments of the first
 * software-trigger stage described in arXiv 2412.05041 (section "HLT1 details
 * and results": a simplified pattern recognition, a fit of the VELO segment
 * only, hits taken by one pass removed before the next, candidates kept when
 * they have enough hits and a low chi2).  The paper does not spell out the
 * steps; the library implements this reading:
 *
 *   velo_cluster      8-connected pixel clusters per (event, plane), numbered by
 *                     smallest pixel id, binary centroid;
 *   velo_find_tracks  triplet seeding on consecutive planes (downstream first),
 *                     greedy claiming by miss distance, plane-by-plane
 *                     extension, chi2 (or learned) acceptance;
 *   velo_fit          least-squares straight-line fit of each track;
 *   velo_pipeline     the three steps in one stream-ordered call (persistent
 *                     work-stealing kernels, captured once in a HIP graph);
 *   velo_mlp_*        the learned ghost filter (10 -> 32 -> 32 -> 1, BF16 MFMA,
 *                     FP32 accumulation) and its on-GPU training step;
 *   velo_seed_*       a learned seed (triplet) filter inside the finder, and the
 *                     emission of seed candidates to train it;
 *   velo_kalman_fit, velo_decode, velo_extrapolate
 *                     a parameterised Kalman fit of the VELO segment, a raw-bank
 *                     decode front end, and the extrapolation through a
 *                     single-kink magnet that forward tracking starts from.
 *
 * Conventions
 *   - Every d_* argument is a DEVICE pointer owned by the caller; it must stay
 *     valid until the work queued on `stream` has finished.  `stream` is a
 *     hipStream_t (NULL = default stream).  Host pointers are named h_*.
 *   - Calls only enqueue work: they never synchronise, except velo_status_read
 *     and velo_autotune, which say so.
 *   - The return value reports argument validation and launch errors only
 *     (VELO_OK or a negative VELO_ERR_*).  Data-dependent problems (capacity
 *     overflow, malformed input) are written asynchronously to d_status:
 *       d_status[0]             worst severity (0 ok, 1 overflow, 2 bad input)
 *       d_status[1..4]          required clusters, tracks, track hits, pixels
 *       d_status[5]             events processed by the large-event path
 *       d_status[6]             tracks decided by the plain-cut fallback
 *       d_status[7]             largest seed-candidate count of one plane step
 *                               on the large-event path (its pool per workgroup
 *                               is min(2^23, max(2^16, 16 * max_clusters /
 *                               max_events)) entries; a step with more
 *                               candidates is seeded in key ranges, each as
 *                               large as the pool: same result, more passes)
 *       d_status[8 + e]         flags of event e (VELO_EV_*)
 *     so d_status holds VELO_STATUS_WORDS(n_events) int32.  On overflow every
 *     offset array is still complete and exact; element arrays are written only
 *     below their capacity.
 *   - A context is used from one host thread and one stream at a time.
 *   - Layouts: events x 26 planes in CSR form.  pix_id = row*1454 + column,
 *     strictly ascending inside an (event, plane) segment.  Cluster and track
 *     indices are global within the batch.
 */
#ifndef VELO_H
#define VELO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VELO_N_PLANES 26
#define VELO_N_SIDE 1454
#define VELO_MLP_NPARAM 1441
#define VELO_MLP_NFEAT 10
#define VELO_FEAT_STRIDE 16
#define VELO_STATUS_HDR 8
#define VELO_STATUS_WORDS(n_events) (VELO_STATUS_HDR + (n_events))

enum velo_error {
    VELO_OK = 0,
    VELO_ERR_ARG = -1,          /* invalid argument (null pointer, negative size, ...) */
    VELO_ERR_NOT_RESERVED = -2, /* velo_reserve was not called or is too small          */
    VELO_ERR_DEVICE = -3,       /* a HIP call failed; see velo_last_error()             */
    VELO_ERR_UNSUPPORTED = -4   /* configuration the library does not implement         */
};

enum velo_event_flag {
    VELO_EV_OVERFLOW = 1,  /* an output or internal capacity was exceeded: no tracks */
    VELO_EV_BAD_INPUT = 2, /* malformed pixel input (validate mode)                   */
    VELO_EV_LARGE_PATH = 4, /* processed by the large-event (global memory) path      */
    VELO_EV_FALLBACK = 8,  /* learned mode: some decision used the plain cut          */
    VELO_EV_SECOND_TILE = 16 /* did not fit the configured LDS tile: next larger tile */
};

enum velo_track_flag {
    VELO_TRK_PLAIN_ACCEPT = 1, /* chi2/ndof cut passed                    */
    VELO_TRK_LEARNED = 2,      /* learned mode was active                 */
    VELO_TRK_FALLBACK = 4,     /* learned mode fell back to the plain cut */
    VELO_TRK_ACCEPT = 8        /* final decision                          */
};

/* Detector geometry.  plane_z strictly ascending (mm, FP32). */
typedef struct velo_geometry {
    int32_t n_planes; /* must be VELO_N_PLANES */
    float plane_z[VELO_N_PLANES];
} velo_geometry;

/* Cut set of the track finder.  All comparisons are FP32, evaluated in the
 * order their expressions are written in (the comments on each field give the
 * quantity), with no fused multiply-add. */
typedef struct velo_cuts {
    float t_max;      /* seed: |tx| <= t_max and |ty| <= t_max                     */
    float d2_max;     /* seed: squared closest approach of its line to the z axis  */
    float s_max;      /* seed: squared miss distance of the middle hit             */
    float e_max;      /* extension: squared miss distance of an added hit          */
    int32_t max_skip; /* planes a track may skip while being extended              */
    float c3;         /* chi2/ndof bound of 3-hit tracks                           */
    float c4;         /* chi2/ndof bound of tracks with >= 4 hits                  */
    float sigma;      /* hit resolution of the fit (mm)                            */
    int32_t mode;     /* 0 plain chi2 cut, 1 learned filter                        */
    float logit_band; /* learned: |logit| < band falls back to the plain cut      */
} velo_cuts;

typedef struct velo_ctx velo_ctx;

/* Creates a context on HIP device `device` (made current for the call).
 * Validates the geometry (ascending z, 26 planes) and cuts (finite, >= 0). */
int velo_create(const velo_geometry* geometry, const velo_cuts* cuts, int device, velo_ctx** out);
void velo_destroy(velo_ctx* ctx);
int velo_set_cuts(velo_ctx* ctx, const velo_cuts* cuts);

/* 1 = check pixel inputs (ids < 1454^2, outside the central hole -- pixel
 * (c, r) exists iff (2c - 1453)^2 + (2r - 1453)^2 >= 33058 --, strictly
 * ascending per segment) and flag VELO_EV_BAD_INPUT instead of clustering
 * malformed segments. */
int velo_set_validate(velo_ctx* ctx, int32_t on);

/* The only call that allocates the internal workspace (velo_create allocates
 * the small network states).  Must be made before any other enqueue and before
 * stream capture; may be repeated to grow.  max_clusters bounds the clusters of
 * a batch (<= max_pixels).  The large-event finder's candidate pool follows
 * the mean event size (max_clusters / max_events), so a repeated call for fewer,
 * larger events lays the workspace out again even when the counts fit (every
 * earlier capacity is kept). */
int velo_reserve(velo_ctx* ctx, int32_t max_events, int64_t max_pixels, int64_t max_clusters);

/* Seed-candidate pool of each workgroup of the large-event finder: at most
 * `entries` candidates of a plane step are held at once (1 <= entries <= the
 * reserved pool, d_status[7]'s description gives its size; 0 = all of it).  A
 * step with more candidates is seeded in ranges of the claiming key (q, h0),
 * each range claimed before the next is enumerated -- the greedy claiming
 * accepts in key order, so the tracks never depend on the pool; smaller pools
 * take more passes over the step.  The overflow remains only if more
 * candidates than the pool holds share one key (q, h0).  velo_reserve resets
 * the pool to all of the reservation. */
int velo_set_large_pool(velo_ctx* ctx, int64_t entries);

/* Routing of events between the finder's passes (performance only: every pass
 * gives the same tracks).  An event whose clusters exceed clusters_per_track x
 * the track capacity of an LDS tile skips that tile and goes straight to the
 * next pass, as an event with a plane larger than the tile does; without the
 * rule such an event would most likely run out of track slots late in its plane
 * walk and be redone.  Collision events create about one candidate track per
 * 15 clusters; the default, 13.5, routes those that would overflow the first
 * tile.  0 turns the rule off (planes alone decide). */
int velo_set_admission(velo_ctx* ctx, float clusters_per_track);

/* Pixel clustering (connected components, 8-neighbourhood).
 *   in : d_pix_off[n_events*26+1] int32, d_pix_id[...] uint32
 *   out: d_pix_clu[n_pix] global cluster index of each pixel,
 *        d_clu_off[n_events*26+1], d_clu_x/d_clu_y[clu_cap] centroid (mm),
 *        d_clu_npix[clu_cap] (nullable) pixels per cluster.
 * Cluster x = ((float)sum_col / (float)n - 726.5f) * 0.055f, likewise y. */
int velo_cluster(velo_ctx* ctx, int32_t n_events, const int32_t* d_pix_off, const uint32_t* d_pix_id,
                 int32_t* d_pix_clu, int32_t* d_clu_off, float* d_clu_x, float* d_clu_y,
                 int32_t* d_clu_npix, int64_t clu_cap, int32_t* d_status, void* stream);

/* Track finding on clusters (CSR per event and plane, as velo_cluster writes).
 *   out: d_trk_off[n_events+1], d_trk_hit_off[trk_cap+1], d_trk_hit[hit_cap]
 *        (global cluster indices, plane ascending), d_trk_planes[trk_cap]
 *        (bit k = hit on plane k), d_trk_flags[trk_cap] (nullable, VELO_TRK_*),
 *        d_trk_logit[trk_cap] (nullable, learned mode).
 * Tracks of an event are in creation order.  emit_rejected = 1 writes every
 * candidate with its flags instead of the accepted tracks only. */
int velo_find_tracks(velo_ctx* ctx, int32_t n_events, const int32_t* d_clu_off, const float* d_clu_x,
                     const float* d_clu_y, int32_t* d_trk_off, int32_t* d_trk_hit_off, int32_t* d_trk_hit,
                     uint32_t* d_trk_planes, uint8_t* d_trk_flags, float* d_trk_logit, int64_t trk_cap,
                     int64_t hit_cap, int32_t emit_rejected, int32_t* d_status, void* stream);

/* Straight-line least-squares fit (x-z and y-z), centred at the hit centroid.
 *   d_n_tracks (nullable): device count of tracks; when given, only that many
 *   (at most max_tracks) are fitted, which keeps the call free of host syncs.
 *   out: d_par[max_tracks][8] = x_ref, y_ref, z_ref, tx, ty, chi2, ndof, 0. */
int velo_fit(velo_ctx* ctx, int64_t max_tracks, const int32_t* d_n_tracks, const int32_t* d_trk_hit_off,
             const int32_t* d_trk_hit, const uint32_t* d_trk_planes, const float* d_clu_x,
             const float* d_clu_y, float* d_par, void* stream);

/* Decode of raw banks (a synthetic super-pixel format: the paper names the
 * persisted raw banks of the detector but not their format) into the CSR
 * pixel input of velo_cluster.  Per (event, plane) a list of 32-bit words, in
 * any order, word = pattern[0:8] | sp_row[8:17] | sp_col[17:27] with bits
 * 27..31 zero; pattern bit 2*dr + dc is the pixel (row 4*sp_row + dr, column
 * 2*sp_col + dc).
 *   d_bank_off[n_events*26+1] word offsets, d_bank words (device).
 *   out: d_pix_off[n_events*26+1], d_pix_id[pix_cap] -- each plane's ids
 *   sorted ascending.  A plane whose ids do not all fit below pix_cap writes
 *   none (its event flagged VELO_EV_OVERFLOW; offsets stay complete).
 * A malformed word (reserved bit, empty pattern, pixel off the sensor) yields
 * no pixel; it and any pixel decoded twice (kept) flag the event
 * VELO_EV_BAD_INPUT.  d_status[4] = total pixels.  Needs velo_reserve for
 * n_events. */
int velo_decode(velo_ctx* ctx, int32_t n_events, const int32_t* d_bank_off, const uint32_t* d_bank,
                int32_t* d_pix_off, uint32_t* d_pix_id, int64_t pix_cap, int32_t* d_status, void* stream);

/* Kalman fit of the VELO segment (the paper's HLT1 fits only the VELO part of
 * a track, with a parameterised Kalman filter -- section "HLT1 details and
 * results"; the parameterisation here is this library's reading): per
 * projection a straight line whose slope takes an independent kick of
 * standard deviation `ms` (rad) on every plane crossed, hits with the
 * context's measurement error sigma.  Started from the two most downstream
 * hits, run plane by plane towards the interaction region; ms = 0 gives the
 * least-squares line.
 *   d_n_tracks (nullable): device count of tracks, as for velo_fit.
 *   out: d_out[max_tracks][16] = x, y, tx, ty, z (state at the most upstream
 *   hit; tx, ty = slopes of the segment just downstream of it), Cxx, Cxt, Ctt,
 *   Cyy, Cyt, Ctt (covariances of the two projections), chi2, ndof, 0, 0, 0.
 * Errors: VELO_ERR_ARG for a negative or non-finite ms, null arrays. */
int velo_kalman_fit(velo_ctx* ctx, int64_t max_tracks, const int32_t* d_n_tracks, const int32_t* d_trk_hit_off,
                    const int32_t* d_trk_hit, const uint32_t* d_trk_planes, const float* d_clu_x,
                    const float* d_clu_y, float ms, float* d_out, void* stream);

/* The whole path (cluster -> find -> fit) in one call.  Output identical to
 * velo_cluster + velo_find_tracks + velo_fit.  The kernels are captured into a
 * HIP graph on first use for a given argument set and replayed afterwards. */
int velo_pipeline(velo_ctx* ctx, int32_t n_events, const int32_t* d_pix_off, const uint32_t* d_pix_id,
                  int32_t* d_pix_clu, int32_t* d_clu_off, float* d_clu_x, float* d_clu_y,
                  int64_t clu_cap, int32_t* d_trk_off, int32_t* d_trk_hit_off, int32_t* d_trk_hit,
                  uint32_t* d_trk_planes, uint8_t* d_trk_flags, float* d_trk_logit, float* d_par,
                  int64_t trk_cap, int64_t hit_cap, int32_t* d_status, void* stream);

/* Stage timing.  With timing on, velo_pipeline runs its kernels eagerly (no
 * graph) with HIP events recorded on `stream` between the stages; after the
 * call velo_last_timing synchronises the stream and returns the durations (ms)
 * of the VELO_N_STAGES stages: reset, cluster+staging, event order, finder
 * (configured LDS tile), finder (events that did not fit it: the next larger
 * LDS tile, then global memory), acceptance (+ learned decision), scan,
 * output+fit. */
#define VELO_N_STAGES 8
int velo_set_timing(velo_ctx* ctx, int32_t on);
int velo_last_timing(velo_ctx* ctx, float* h_ms, int32_t n);

/* Launch configuration of the track finder: threads per event (64, 128, 256, 512)
 * and LDS tile (plane capacity 0: 256, 1: 512, 2: 1024 clusters; events with a
 * larger plane go on to the next tile, then to global memory).  Outputs never
 * depend on it. */
int velo_set_launch(velo_ctx* ctx, int32_t threads, int32_t tile);
int velo_get_launch(velo_ctx* ctx, int32_t* threads, int32_t* tile);

/* Autotuner of the finder's launch (pattern: batches of uneven events in one
 * persistent launch, threads per event and LDS tile chosen by timing).  Times
 * each of the VELO_N_LAUNCH configurations with n_ctx batches in flight, the
 * way a caller that keeps several batches going (one context and stream each)
 * runs them: context i works on streams[i] -- event lists, the finder passes,
 * the plain acceptance, over the clusters given (device inputs, as for
 * velo_find_tracks, read-only and shared) -- all streams concurrently, `reps`
 * batches per context after one warm-up batch; the time per batch is the
 * span from the first to the last batch divided by reps * n_ctx.  The fastest
 * configuration is set on every context.  Synchronises the streams.
 *   ctxs[n_ctx]: distinct contexts on one device, each reserved for n_events
 *     (1 <= n_ctx <= 16); streams[n_ctx]: hipStream_t of each (NULL = default).
 *   cache_path (nullable): a text file, one line per pick ("<key>\t<threads>
 *     <tile> <ms per batch>").  The key names the device (architecture, CU
 *     count), n_events, the clusters per event in quarter-octave buckets,
 *     n_ctx, and a hash of the cuts, plane positions and seed-filter state.  A
 *     line with the same key is applied without timing (h_ms then all -1);
 *     otherwise the pick is appended.
 *   h_ms (nullable): VELO_N_LAUNCH timings, threads-major (64, 128, 256, 512)
 *     then tile.
 * Errors: VELO_ERR_ARG for bad arguments or a cache file that cannot be
 * appended to (the pick is set all the same); on any other error every
 * context keeps the launch it had. */
#define VELO_N_LAUNCH 12
int velo_autotune(velo_ctx* const* ctxs, int32_t n_ctx, int32_t n_events, const int32_t* d_clu_off,
                  const float* d_clu_x, const float* d_clu_y, int32_t reps, const char* cache_path, float* h_ms,
                  void* const* streams);

/* Learned filter.  Parameters: 1441 FP32 master weights in the order
 * W1[32][10], b1[32], W2[32][32], b2[32], w3[32], b3; normalisation: 10 means
 * then 10 standard deviations.  Both are copied (host pointers). */
int velo_mlp_set_weights(velo_ctx* ctx, const float* h_master, const float* h_norm);
int velo_mlp_get_weights(velo_ctx* ctx, float* h_master, float* h_norm);

/* Features of candidates: d_feat[n][16] BF16 bit patterns, standardised
 * ((f - mean) / sd, FP32, round to nearest even), 10 used, 6 zero.  d_feat
 * may be null when d_feat_f32 is given: then only the raw FP32 features are
 * written and no normalisation is needed (collecting training data). */
int velo_features(velo_ctx* ctx, int64_t n_tracks, const int32_t* d_trk_hit_off, const int32_t* d_trk_hit,
                  const uint32_t* d_trk_planes, const float* d_clu_x, const float* d_clu_y,
                  uint16_t* d_feat, float* d_feat_f32 /* nullable [n][10] raw FP32 */, void* stream);

/* Standardisation alone: d_raw[n][10] FP32 features -> d_feat[n][16] BF16, by
 * the same rule as velo_features (used to prepare stored training data). */
int velo_standardize(velo_ctx* ctx, int64_t n, const float* d_raw, uint16_t* d_feat, void* stream);

/* Logits of n feature rows (BF16 MFMA, FP32 accumulation). */
int velo_mlp_forward(velo_ctx* ctx, int64_t n, const uint16_t* d_feat, float* d_logit, void* stream);

/* Gradient of the mean BCE-with-logits loss (label 1 = ghost) w.r.t. the 1441
 * parameters, deterministic (fixed-order reduction).  d_grad[1441] FP32,
 * d_loss (nullable) FP32. */
int velo_mlp_grad(velo_ctx* ctx, int64_t n, const uint16_t* d_feat, const uint8_t* d_label, float* d_grad,
                  float* d_loss, void* stream);

/* One training step: gradient as above, then Adam (beta1, beta2, eps as set
 * by velo_mlp_set_adam; lr given) on the FP32 master weights. */
int velo_mlp_train_step(velo_ctx* ctx, int64_t n, const uint16_t* d_feat, const uint8_t* d_label, float lr,
                        float* d_loss, void* stream);
int velo_mlp_set_adam(velo_ctx* ctx, float beta1, float beta2, float eps);

/* The gradient of velo_mlp_grad for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving or training loops,
 * harnesses that forbid hipMalloc): no context and no allocation of any kind.
 * The weights come as d_master[1441] FP32 (device, the velo_mlp_set_weights
 * order); d_feat, d_label, d_grad and d_loss are as for velo_mlp_grad, and
 * the result is bit-identical to velo_mlp_grad with the same weights.
 * Scratch: the per-workgroup partial sums go to a device array inside the
 * library, 1024 x 1472 FP32 (5.75 MiB), one copy per GPU held until the
 * process ends; the gradient spreads any n over at most 1024 workgroups, so
 * every n >= 1 fits (a computed workgroup count above 1024 would be rejected
 * with VELO_ERR_ARG).  Each partial is written before it is read, so nothing
 * needs clearing between calls.  All calls on one GPU share the array: calls
 * that overlap in time on one GPU (two streams, two threads) race and give
 * wrong gradients; serialise them.  The first call on a device resolves the
 * array's address on it (no stream work).
 * Errors: VELO_ERR_ARG for n <= 0 or null arrays, VELO_ERR_DEVICE for a
 * failed launch (message in velo_last_error). */
int velo_mlp_grad_noalloc(int64_t n, const float* d_master, const uint16_t* d_feat, const uint8_t* d_label,
                          float* d_grad, float* d_loss, void* stream);

/* Optimiser state for checkpoints: master[1441], m[1441], v[1441], step. */
int velo_mlp_get_state(velo_ctx* ctx, float* h_master, float* h_m, float* h_v, int64_t* h_step);
int velo_mlp_set_state(velo_ctx* ctx, const float* h_master, const float* h_m, const float* h_v, int64_t step);

/* Forward extrapolation of VELO states through the magnet -- the first step of
 * forward tracking (section "HLT1 details and results": straight from the
 * VELO to the middle of the magnet, the field replaced there by one change of
 * slope that depends on the track's momentum).  The magnet is the caller's:
 *   z_mag: the plane of the kink (mm); z_t: the tracker plane (mm), > z_mag;
 *   kick: change of the x slope per unit charge / momentum (rad GeV), != 0;
 *   p_min: the smallest momentum the window must hold (GeV), > 0.
 * d_par: [max_tracks][8] states as velo_fit writes them (x, y, z, tx, ty at
 * z; the other three are not read); d_x_hit (nullable): [max_tracks] x of a
 * hit at z_t; d_n_tracks (nullable): device count of tracks, as for velo_fit.
 * d_out: [max_tracks][8] = x, y at z_mag; x of the straight line and y at z_t
 * (no kink in y); x_lo, x_hi = the straight x -+ kick / p_min * (z_t - z_mag);
 * the q/p that takes the track to x_hit (0 without d_x_hit); tx after the kink
 * for that q/p.  FP32.  d_par and d_out 16-byte aligned.
 * Errors: VELO_ERR_ARG for null arrays, misaligned rows or an invalid magnet. */
typedef struct velo_magnet {
    float z_mag, z_t, kick, p_min;
} velo_magnet;
int velo_extrapolate(velo_ctx* ctx, int64_t max_tracks, const int32_t* d_n_tracks, const float* d_par,
                     const float* d_x_hit, const velo_magnet* magnet, float* d_out, void* stream);

/* Seed-level learned filter (a triplet filter: an extension of the simplified
 * pattern recognition that the first trigger stage uses for throughput --
 * section "HLT1 details and results" -- with the track filter's network
 * shape).  Every seed candidate that passes the
 * seed cuts gets ten FP32 features: the middle-hit miss q, the squared
 * transverse distance of the h0-h2 line from the z axis, the z of its closest
 * approach to the axis (clipped to +-2000 mm), h0's squared radius, the squared
 * slope, the squared cosine between h0's radial direction and the slope, the
 * plane k and the cluster counts of planes k, k+1, k+2.  The network runs in
 * FP32 (features standardised as (f - mean) * r, r = 1 / sd rounded to FP32;
 * each unit from its bias, inputs ascending, ReLU; no BF16 rounding); a candidate
 * whose logit exceeds `threshold` is dropped before the claiming, which changes
 * the tracks found.  h_weights: 1441 floats in the track network's order
 * (pass BF16-rounded values to reproduce a BF16-trained network); h_norm: 10
 * means then 10 non-zero standard deviations; both copied (host pointers).
 * h_weights = NULL switches the filter off (the default).  Applies to
 * velo_find_tracks, velo_pipeline and velo_autotune from the next call. */
int velo_seed_filter_set(velo_ctx* ctx, const float* h_weights, const float* h_norm, float threshold);

/* Training emission of seed candidates: from the next finder call on, every
 * candidate reaching the seed filter (all that pass the seed cuts) appends
 * its ten raw features to d_feat [cap][10] (FP32) and its three global cluster
 * indices (planes k, k+1, k+2) to d_hits [cap][3]; *d_count (caller-zeroed
 * device counter) counts all of them, also those beyond `cap`, which are not
 * written.  Order is unspecified, and an event that one finder pass hands on
 * to the next (a capacity it overflowed) may emit some candidates twice.  All NULL
 * switches emission off.  The buffers are caller-owned and must stay valid
 * while emission is on. */
int velo_seed_emit(velo_ctx* ctx, float* d_feat, int32_t* d_hits, int64_t cap, unsigned long long* d_count);

/* Synchronises `stream` and copies `n_words` status words to the host. */
int velo_status_read(velo_ctx* ctx, const int32_t* d_status, int32_t* h_status, int32_t n_words, void* stream);

const char* velo_status_string(int code);
/* Message of the last failing call on this thread ("" if none). */
const char* velo_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* VELO_H */
