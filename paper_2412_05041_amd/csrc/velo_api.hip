// velo_api.hip -- the C ABI of libvelo: context, workspace, argument checks,
// stream-ordered launches and the graph-captured pipeline.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/velo.h"
#include "kernels.h"
#include "mlp.h"

using namespace velo;

namespace {

thread_local std::string g_last_error;

// Clusters per track slot above which an event skips an LDS tile: collision
// events create about one candidate track per 15 clusters (noise included), and
// nearly every one above 13.5 per slot runs out of the first tile's slots.
constexpr float kDefaultAdmit = 13.5f;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define HIP_OK(expr)                                                                  \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail(VELO_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(e_));    \
    } while (0)

struct GraphKey {
    std::vector<uintptr_t> v;
    bool operator==(const GraphKey& o) const { return v == o.v; }
};

}  // namespace

struct velo_ctx {
    int device = 0;
    Params p{};
    int validate = 0;
    int threads = 256, tile = 1;
    int64_t pool_limit = 0;  // velo_set_large_pool (0: the reserved pool)
    float admit = kDefaultAdmit;  // velo_set_admission
    Work w{};
    void* ws = nullptr;
    size_t ws_bytes = 0;
    int n_cu = 0;
    hipStream_t cap_stream = nullptr;
    // graph cache of velo_pipeline
    hipGraphExec_t exec = nullptr;
    GraphKey key;
    uint64_t version = 1;  // bumped by anything that changes captured parameters
    MlpState mlp;
    // seed-level filter (kSeedFloats on the device) and its training emission
    float* d_seed = nullptr;
    int seed_on = 0;
    float* seed_feat = nullptr;
    int32_t* seed_hits = nullptr;
    int64_t seed_cap = 0;
    unsigned long long* seed_count = nullptr;
    // stage timing (eager pipeline)
    int timing = 0;
    hipEvent_t ev[VELO_N_STAGES + 1] = {};
    hipStream_t ev_stream = nullptr;
    int ev_valid = 0;
};

namespace {

int check_ctx(velo_ctx* c) {
    if (!c) return fail(VELO_ERR_ARG, "null context");
    if (!c->ws) return fail(VELO_ERR_NOT_RESERVED, "velo_reserve was not called");
    return VELO_OK;
}

int set_params(velo_ctx* c, const velo_cuts* cu) {
    const float v[] = {cu->t_max, cu->d2_max, cu->s_max, cu->e_max, cu->c3, cu->c4, cu->sigma};
    for (float x : v)
        if (!(x >= 0.0f) || (std::isinf(x) && x != cu->c3 && x != cu->c4))
            return fail(VELO_ERR_ARG, "cuts must be finite and >= 0");
    if (cu->max_skip < 0 || cu->max_skip > 24) return fail(VELO_ERR_ARG, "max_skip out of range");
    if (cu->mode != 0 && cu->mode != 1) return fail(VELO_ERR_ARG, "mode must be 0 or 1");
    if (!(cu->logit_band >= 0.0f)) return fail(VELO_ERR_ARG, "logit_band must be >= 0");
    if (!(cu->sigma > 0.0f)) return fail(VELO_ERR_ARG, "sigma must be > 0");
    Params& p = c->p;
    p.t_max = cu->t_max;
    p.d2_max = cu->d2_max;
    p.s_max = cu->s_max;
    p.e_max = cu->e_max;
    p.max_skip = cu->max_skip;
    p.c3 = cu->c3;
    p.c4 = cu->c4;
    p.sigma = cu->sigma;
    p.mode = cu->mode;
    p.logit_band = cu->logit_band;
    // search radii: generous upper bounds of the cut distances (pruning only)
    p.r_seed = std::sqrt(cu->d2_max) * 1.0001f + 1e-6f;
    p.r_mid = std::sqrt(cu->s_max) * 1.0001f + 1e-6f;
    p.r_ext = std::sqrt(cu->e_max) * 1.0001f + 1e-6f;
    c->version++;
    return VELO_OK;
}

template <typename T>
T* carve(char*& cur, int64_t n) {
    cur = (char*)(((uintptr_t)cur + 255) & ~(uintptr_t)255);
    T* p = (T*)cur;
    cur += sizeof(T) * (size_t)std::max<int64_t>(n, 1);
    return p;
}

// Seed-candidate pool entries per large-event workgroup for a reservation of
// E events and C clusters: from the mean event (16 entries per cluster: noise-
// dominated planes give ~2 candidates per hit pair passing the pair cuts).
int64_t pool_entries(int32_t E, int64_t C) {
    return std::max<int64_t>(1 << 16, std::min<int64_t>(1 << 23, 16 * (C / std::max(E, 1))));
}

size_t layout(Work& w, char* base, int32_t E, int64_t P, int64_t C, int n_cu, int64_t min_pool) {
    char* cur = base;
    const int64_t PX = std::max(P, C);
    w.stg = carve<Staged>(cur, C);
    w.used = carve<uint8_t>(cur, C);
    w.chits = carve<int32_t>(cur, C * kPlanes);
    w.cmask = carve<uint32_t>(cur, C);
    w.cflags = carve<uint8_t>(cur, C);
    w.clogit = carve<float>(cur, C);
    w.cfeat = carve<uint16_t>(cur, C * 16);
    w.cpar = carve<float>(cur, C * 8);
    w.ev_ncand = carve<int32_t>(cur, E);
    w.ev_nout = carve<int32_t>(cur, E);
    w.ev_nouthit = carve<int32_t>(cur, E);
    w.ev_ncandhit = carve<int32_t>(cur, E);
    w.ev_tbase = carve<int32_t>(cur, E);
    w.ev_hbase = carve<int32_t>(cur, E);
    w.order = carve<int32_t>(cur, E);
    w.large = carve<int32_t>(cur, E);
    w.large2 = carve<int32_t>(cur, E);
    w.seg_m = carve<int32_t>(cur, (int64_t)E * kPlanes);
    w.seg_big = carve<int32_t>(cur, (int64_t)E * kPlanes);
    w.counters = carve<int32_t>(cur, 8);
    w.g_claim = carve<int32_t>(cur, C);
    w.g_slota = carve<uint64_t>(cur, C);
    w.g_slotb = carve<uint32_t>(cur, C);
    w.g_ttx = carve<float>(cur, C);
    w.g_tty = carve<float>(cur, C);
    w.g_txb = carve<float>(cur, C);
    w.g_tyb = carve<float>(cur, C);
    w.g_dtx = carve<float>(cur, C);
    w.g_dty = carve<float>(cur, C);
    w.g_dxb = carve<float>(cur, C);
    w.g_dyb = carve<float>(cur, C);
    w.g_tkb = carve<int32_t>(cur, C);
    w.g_twant = carve<int32_t>(cur, C);
    w.g_enum = carve<int32_t>(cur, 6 * C + 8);
    w.g_gx = carve<float>(cur, C);
    w.g_gy = carve<float>(cur, C);
    w.g_gpos = carve<int32_t>(cur, C);
    // global-memory finder: each workgroup owns a seed-candidate pool for one
    // plane step of its current event (pool_entries, or min_pool when larger:
    // a reservation kept for a batch of fewer, larger events); as many
    // workgroups as a pool budget of 8 entries per cluster allows (at most 2
    // per CU, at least 1)
    w.pool_cap = std::max(pool_entries(E, C), min_pool);
    w.pool_use = w.pool_cap;
    const int64_t budget = std::max<int64_t>(1 << 20, std::min<int64_t>(int64_t(1) << 29, 8 * C));
    w.n_large_blocks = (int32_t)std::max<int64_t>(1, std::min<int64_t>(2 * std::max(n_cu, 1), budget / w.pool_cap));
    w.g_cell = carve<int32_t>(cur, kCellWords * w.n_large_blocks);
    const int64_t pool = w.pool_cap * w.n_large_blocks;
    w.p_q = carve<float>(cur, pool);
    w.p_h = carve<int32_t>(cur, pool * 3);
    w.p_alive = carve<uint8_t>(cur, pool);
    w.g_par = carve<int32_t>(cur, PX);
    w.g_sc = carve<uint32_t>(cur, PX);
    w.g_sr = carve<uint32_t>(cur, PX);
    w.g_cnt = carve<uint32_t>(cur, PX);
    w.g_tmp = carve<int32_t>(cur, PX);
    w.cap_clusters = C;
    w.cap_pixels = P;
    w.cap_scratch = PX;
    w.cap_events = E;
    return (size_t)(cur - base) + 256;
}

int grid_for(velo_ctx* c, int n_events, int threads, int tile) {
    const int per_cu = find_blocks_per_cu(threads, std::min(tile, 2), c->seed_on || c->seed_feat);
    const int g = std::max(1, c->n_cu * std::min(std::max(per_cu, 1), kMaxLdsBlocksPerCu));
    return std::max(1, std::min(n_events, g));
}

int mark(velo_ctx* c, int i, hipStream_t s, bool on);

// Event lists for the finder (k_order): events whose planes all fit the
// configured tile, and the others -- for the next larger tile, or (tile 2)
// straight for the global-memory finder.
hipError_t enqueue_order(velo_ctx* c, int E, const int32_t* clu_off, hipStream_t s) {
    return launch_order(c->w, E, clu_off, tile_planes(c->tile), c->tile < 2 ? c->w.large : c->w.large2,
                        c->tile < 2 ? 2 : 5, s);
}

// The finder's passes, in order on the stream: the configured tile, then (tiles
// 0 and 1) the next larger tile over the few events too large for it -- the
// heaviest of the batch, 512 threads each -- then the global-memory finder.
// (Running the second pass beside the first, on a stream of its own, shortens
// one batch but slows batches in flight together: its 81 KB workgroups take the
// LDS the first pass's smaller ones would use.)
int enqueue_finder(velo_ctx* c, const FindArgs& fa, int E, hipStream_t s, bool timed) {
    HIP_OK(launch_finder_first(fa, c->threads, c->tile, grid_for(c, E, c->threads, c->tile), s));
    if (int rc = mark(c, 4, s, timed)) return rc;
    if (c->tile < 2)
        HIP_OK(launch_finder_second(fa, c->tile + 1, grid_for(c, E, kSecondPassThreads, c->tile + 1), s));
    HIP_OK(launch_finder_large(fa, s));
    return mark(c, 5, s, timed);
}

// Enqueue the finder (staging must be in place) and the output compaction.
// Timing mark i (no-op unless the eager timed pipeline is running).
int mark(velo_ctx* c, int i, hipStream_t s, bool on) {
    if (on) HIP_OK(hipEventRecord(c->ev[i], s));
    return VELO_OK;
}

int enqueue_find_out(velo_ctx* c, int32_t E, const int32_t* clu_off, const float* clu_x, const float* clu_y,
                     int32_t* trk_off, int32_t* trk_hit_off, int32_t* trk_hit, uint32_t* trk_planes,
                     uint8_t* trk_flags, float* trk_logit, float* par, int64_t trk_cap, int64_t hit_cap,
                     int32_t emit, int32_t* status, int64_t clu_limit, hipStream_t s, bool timed = false) {
    HIP_OK(enqueue_order(c, E, clu_off, s));
    if (int rc = mark(c, 3, s, timed)) return rc;
    FindArgs fa{};
    fa.n_events = E;
    fa.clu_off = clu_off;
    fa.clu_x = clu_x;
    fa.clu_y = clu_y;
    fa.status = status;
    fa.p = c->p;
    fa.w = c->w;
    fa.mlp_master = c->mlp.d_master;
    fa.mlp_norm = c->mlp.d_norm;
    fa.clu_limit = clu_limit;
    fa.admit = c->admit;
    fa.seed_net = c->seed_on ? c->d_seed : nullptr;
    fa.seed_feat = c->seed_feat;
    fa.seed_hits = c->seed_hits;
    fa.seed_cap = c->seed_cap;
    fa.seed_count = c->seed_count;
    if (int rc = enqueue_finder(c, fa, E, s, timed)) return rc;
    HIP_OK(launch_accept(fa, s));
    if (c->p.mode == 1) HIP_OK(launch_mlp_accept(c->mlp, fa, s));
    if (int rc = mark(c, 6, s, timed)) return rc;
    OutArgs oa{};
    oa.n_events = E;
    oa.clu_off = clu_off;
    oa.clu_x = clu_x;
    oa.clu_y = clu_y;
    oa.trk_off = trk_off;
    oa.trk_hit_off = trk_hit_off;
    oa.trk_hit = trk_hit;
    oa.trk_planes = trk_planes;
    oa.trk_flags = trk_flags;
    oa.trk_logit = trk_logit;
    oa.par = par;
    oa.trk_cap = trk_cap;
    oa.hit_cap = hit_cap;
    oa.emit_rejected = emit;
    oa.status = status;
    oa.p = c->p;
    oa.w = c->w;
    HIP_OK(launch_scan(oa, s));
    if (int rc = mark(c, 7, s, timed)) return rc;
    HIP_OK(launch_output(oa, s));
    if (int rc = mark(c, 8, s, timed)) return rc;
    return VELO_OK;
}

// ---------------------------------------------------------------- autotuner

constexpr int kMaxInFlight = 16;

// Launch state of the contexts being tuned and the timing events: on any exit
// before commit() the contexts get their launches back and the events are freed.
struct TuneScope {
    velo_ctx* const* ctxs;
    int n;
    int th[kMaxInFlight], tl[kMaxInFlight];
    hipEvent_t e0 = nullptr, e1 = nullptr, join[kMaxInFlight] = {};
    bool ok = true, done = false;
    TuneScope(velo_ctx* const* c, int n_) : ctxs(c), n(n_) {
        for (int i = 0; i < n; ++i) { th[i] = c[i]->threads; tl[i] = c[i]->tile; }
        ok = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
        for (int i = 0; ok && i < n; ++i) ok = hipEventCreateWithFlags(&join[i], hipEventDisableTiming) == hipSuccess;
    }
    void commit(int threads, int tile) {
        for (int i = 0; i < n; ++i) {
            ctxs[i]->threads = threads;
            ctxs[i]->tile = tile;
            ctxs[i]->version++;
        }
        done = true;
    }
    ~TuneScope() {
        if (!done)
            for (int i = 0; i < n; ++i) { ctxs[i]->threads = th[i]; ctxs[i]->tile = tl[i]; ctxs[i]->version++; }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        for (int i = 0; i < n; ++i)
            if (join[i]) (void)hipEventDestroy(join[i]);
    }
};

// Stream 0 waits for the work queued so far on the other streams.
hipError_t join_streams(TuneScope& sc, void* const* streams, int n) {
    for (int i = 1; i < n; ++i) {
        hipError_t e = hipEventRecord(sc.join[i], (hipStream_t)streams[i]);
        if (e == hipSuccess) e = hipStreamWaitEvent((hipStream_t)streams[0], sc.join[i], 0);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// One batch of the tuned work on a context: event lists, the finder passes
// and the acceptance (plain cut; it does not depend on the launch).
int enqueue_tune_batch(velo_ctx* c, int32_t E, const int32_t* clu_off, const float* clu_x, const float* clu_y,
                       hipStream_t s) {
    HIP_OK(launch_reset(c->w, E, nullptr, s));
    HIP_OK(enqueue_order(c, E, clu_off, s));
    FindArgs fa{};
    fa.n_events = E;
    fa.clu_off = clu_off;
    fa.clu_x = clu_x;
    fa.clu_y = clu_y;
    fa.status = nullptr;
    fa.p = c->p;
    fa.p.mode = 0;
    fa.w = c->w;
    fa.clu_limit = c->w.cap_clusters;
    fa.admit = c->admit;
    fa.seed_net = c->seed_on ? c->d_seed : nullptr;
    if (int rc = enqueue_finder(c, fa, E, s, false)) return rc;
    HIP_OK(launch_accept(fa, s));
    return VELO_OK;
}

// Cache key: device, batch shape (events; clusters per event in quarter-octave
// buckets), batches in flight, and everything of the context that changes the
// finder's work (cuts, plane positions, seed filter).
std::string tune_key(const hipDeviceProp_t& prop, const velo_ctx* c, int n_ctx, int32_t E, int32_t n_clu) {
    uint64_t h = 1469598103934665603ull;  // FNV-1a over the finder's parameters
    auto mix = [&](const void* p, size_t n) {
        const unsigned char* b = static_cast<const unsigned char*>(p);
        for (size_t i = 0; i < n; ++i) { h ^= b[i]; h *= 1099511628211ull; }
    };
    mix(&c->p, sizeof(Params));
    const int seed = c->seed_on;
    mix(&seed, sizeof(seed));
    const double cpe = (double)n_clu / (double)E;
    const int bucket = cpe > 0.0 ? (int)std::lround(4.0 * std::log2(cpe)) : -1000;
    char buf[256];
    snprintf(buf, sizeof(buf), "%s/%dcu events=%d clu_bucket=%d in_flight=%d params=%016llx", prop.gcnArchName,
             prop.multiProcessorCount, E, bucket, n_ctx, (unsigned long long)h);
    for (char* q = buf; *q; ++q)
        if (*q == '\t' || *q == '\n') *q = ' ';
    return buf;
}

// Cache file: one line per pick, "<key>\t<threads> <tile> <ms>"; the last line
// of a key wins.
bool tune_cache_lookup(const char* path, const std::string& key, int* th, int* tl) {
    FILE* f = fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool hit = false;
    while (fgets(line, sizeof(line), f)) {
        char* tab = strchr(line, '\t');
        if (!tab) continue;
        *tab = 0;
        int a = 0, b = 0;
        if (key == line && sscanf(tab + 1, "%d %d", &a, &b) == 2 && (a == 64 || a == 128 || a == 256 || a == 512) &&
            b >= 0 && b <= 2) {
            *th = a;
            *tl = b;
            hit = true;
        }
    }
    fclose(f);
    return hit;
}

bool tune_cache_append(const char* path, const std::string& key, int th, int tl, float ms) {
    FILE* f = fopen(path, "a");
    if (!f) return false;
    const bool ok = fprintf(f, "%s\t%d %d %.6f\n", key.c_str(), th, tl, ms) > 0;
    return (fclose(f) == 0) && ok;
}

int check_reserved(velo_ctx* c, int32_t E, int64_t clusters) {
    if (E < 0) return fail(VELO_ERR_ARG, "n_events < 0");
    if (E > c->w.cap_events) return fail(VELO_ERR_NOT_RESERVED, "n_events %d > reserved %d", E, c->w.cap_events);
    if (clusters > c->w.cap_clusters)
        return fail(VELO_ERR_NOT_RESERVED, "cluster capacity %lld > reserved %lld", (long long)clusters,
                    (long long)c->w.cap_clusters);
    return VELO_OK;
}

}  // namespace

int velo::set_last_error(int code, const char* msg) {
    g_last_error = msg;
    return code;
}

extern "C" {

const char* velo_last_error(void) { return g_last_error.c_str(); }

const char* velo_status_string(int code) {
    switch (code) {
        case VELO_OK: return "ok";
        case VELO_ERR_ARG: return "invalid argument";
        case VELO_ERR_NOT_RESERVED: return "workspace not reserved or too small";
        case VELO_ERR_DEVICE: return "HIP error";
        case VELO_ERR_UNSUPPORTED: return "unsupported";
        default: return "unknown";
    }
}

int velo_create(const velo_geometry* g, const velo_cuts* cu, int device, velo_ctx** out) {
    if (!g || !cu || !out) return fail(VELO_ERR_ARG, "null argument");
    *out = nullptr;
    if (g->n_planes != kPlanes) return fail(VELO_ERR_ARG, "n_planes must be %d", kPlanes);
    for (int k = 0; k < kPlanes; ++k) {
        if (!std::isfinite(g->plane_z[k])) return fail(VELO_ERR_ARG, "plane_z not finite");
        if (k && !(g->plane_z[k] > g->plane_z[k - 1])) return fail(VELO_ERR_ARG, "plane_z must ascend");
    }
    HIP_OK(hipSetDevice(device));
    velo_ctx* c = new velo_ctx();
    c->device = device;
    for (int k = 0; k < kPlanes; ++k) c->p.z[k] = g->plane_z[k];
    int rc = set_params(c, cu);
    if (rc) { delete c; return rc; }
    hipDeviceProp_t prop;
    hipError_t e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) { delete c; return fail(VELO_ERR_DEVICE, "hipGetDeviceProperties: %s", hipGetErrorString(e)); }
    c->n_cu = prop.multiProcessorCount;
    e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) { delete c; return fail(VELO_ERR_DEVICE, "hipStreamCreate: %s", hipGetErrorString(e)); }
    rc = mlp_init(c->mlp);
    if (rc) { delete c; return fail(VELO_ERR_DEVICE, "MLP state allocation failed"); }
    if (hipMalloc(&c->d_seed, sizeof(float) * kSeedFloats) != hipSuccess) {
        mlp_free(c->mlp);
        delete c;
        return fail(VELO_ERR_DEVICE, "seed filter allocation failed");
    }
    *out = c;
    return VELO_OK;
}

void velo_destroy(velo_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    if (c->exec) (void)hipGraphExecDestroy(c->exec);
    if (c->ws) (void)hipFree(c->ws);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    for (int i = 0; i <= VELO_N_STAGES; ++i)
        if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
    mlp_free(c->mlp);
    if (c->d_seed) (void)hipFree(c->d_seed);
    delete c;
}

int velo_set_cuts(velo_ctx* c, const velo_cuts* cu) {
    if (!c || !cu) return fail(VELO_ERR_ARG, "null argument");
    return set_params(c, cu);
}

int velo_set_validate(velo_ctx* c, int32_t on) {
    if (!c) return fail(VELO_ERR_ARG, "null context");
    c->validate = on ? 1 : 0;
    c->version++;
    return VELO_OK;
}

int velo_set_launch(velo_ctx* c, int32_t threads, int32_t tile) {
    if (!c) return fail(VELO_ERR_ARG, "null context");
    if (threads != 64 && threads != 128 && threads != 256 && threads != 512)
        return fail(VELO_ERR_ARG, "threads must be 64/128/256/512");
    if (tile < 0 || tile > 2) return fail(VELO_ERR_ARG, "tile must be 0..2");
    c->threads = threads;
    c->tile = tile;
    c->version++;
    return VELO_OK;
}

int velo_get_launch(velo_ctx* c, int32_t* threads, int32_t* tile) {
    if (!c || !threads || !tile) return fail(VELO_ERR_ARG, "null argument");
    *threads = c->threads;
    *tile = c->tile;
    return VELO_OK;
}

int velo_reserve(velo_ctx* c, int32_t max_events, int64_t max_pixels, int64_t max_clusters) {
    if (!c) return fail(VELO_ERR_ARG, "null context");
    if (max_events < 0 || max_pixels < 0 || max_clusters < 0 || max_clusters > max_pixels + 1)
        return fail(VELO_ERR_ARG, "bad reserve sizes");
    if (max_pixels >= (int64_t)1 << 31) return fail(VELO_ERR_UNSUPPORTED, "more than 2^31 pixels per batch");
    // the large-event pool follows the mean event size, so a workspace that
    // covers the counts but was laid out for smaller events is laid out again
    const int64_t want_pool = pool_entries(std::max(max_events, 1), std::max<int64_t>(max_clusters, 1));
    if (c->ws && max_events <= c->w.cap_events && max_pixels <= c->w.cap_pixels &&
        max_clusters <= c->w.cap_clusters && want_pool <= c->w.pool_cap) {
        if (c->w.pool_use != c->w.pool_cap) {  // a pool limit ends with any reservation
            c->w.pool_use = c->w.pool_cap;
            c->pool_limit = 0;
            c->version++;
        }
        return VELO_OK;
    }
    int32_t E = std::max(max_events, 1);
    int64_t P = std::max<int64_t>(max_pixels, 1), C = std::max<int64_t>(max_clusters, 1), min_pool = want_pool;
    if (c->ws) {  // keep what the old reservation covered
        E = std::max(E, c->w.cap_events);
        P = std::max(P, c->w.cap_pixels);
        C = std::max(C, c->w.cap_clusters);
        min_pool = std::max(min_pool, c->w.pool_cap);
    }
    HIP_OK(hipSetDevice(c->device));
    if (c->ws) {
        HIP_OK(hipDeviceSynchronize());
        HIP_OK(hipFree(c->ws));
        c->ws = nullptr;
    }
    Work w{};
    const size_t bytes = layout(w, nullptr, E, P, C, c->n_cu, min_pool);
    void* base = nullptr;
    HIP_OK(hipMalloc(&base, bytes));
    layout(w, (char*)base, E, P, C, c->n_cu, min_pool);
    c->w = w;
    c->ws = base;
    c->ws_bytes = bytes;
    c->pool_limit = 0;
    c->version++;
    return VELO_OK;
}

int velo_set_admission(velo_ctx* c, float clusters_per_track) {
    if (!c) return fail(VELO_ERR_ARG, "null context");
    if (!(clusters_per_track >= 0.0f) || !std::isfinite(clusters_per_track))
        return fail(VELO_ERR_ARG, "clusters per track must be finite and >= 0");
    c->admit = clusters_per_track;
    c->version++;
    return VELO_OK;
}

int velo_set_large_pool(velo_ctx* c, int64_t entries) {
    if (int rc = check_ctx(c)) return rc;
    if (entries < 0 || entries > c->w.pool_cap)
        return fail(VELO_ERR_ARG, "pool entries must be 0..%lld (the reserved pool)", (long long)c->w.pool_cap);
    c->w.pool_use = entries ? entries : c->w.pool_cap;
    c->pool_limit = entries;
    c->version++;
    return VELO_OK;
}

int velo_cluster(velo_ctx* c, int32_t E, const int32_t* pix_off, const uint32_t* pix_id, int32_t* pix_clu,
                 int32_t* clu_off, float* clu_x, float* clu_y, int32_t* clu_npix, int64_t clu_cap,
                 int32_t* status, void* stream) {
    if (int rc = check_ctx(c)) return rc;
    if (E < 0 || !pix_off || !clu_off || (E > 0 && (!pix_id && false)) || clu_cap < 0)
        return fail(VELO_ERR_ARG, "bad arguments");
    if (clu_cap > 0 && (!clu_x || !clu_y)) return fail(VELO_ERR_ARG, "null cluster arrays");
    if (int rc = check_reserved(c, E, 0)) return rc;
    hipStream_t s = (hipStream_t)stream;
    HIP_OK(launch_reset(c->w, E, status, s));
    ClusterArgs a{};
    a.n_seg = E * kPlanes;
    a.pix_off = pix_off;
    a.pix_id = pix_id;
    a.pix_clu = pix_clu;
    a.clu_off = clu_off;
    a.clu_x = clu_x;
    a.clu_y = clu_y;
    a.clu_npix = clu_npix;
    a.clu_cap = clu_cap;
    a.status = status;
    a.validate = c->validate;
    a.stage = 0;
    a.w = c->w;
    if (E == 0) {
        HIP_OK(hipMemsetAsync(clu_off, 0, sizeof(int32_t), s));
        return VELO_OK;
    }
    HIP_OK(launch_cluster(a, s));
    return VELO_OK;
}

int velo_find_tracks(velo_ctx* c, int32_t E, const int32_t* clu_off, const float* clu_x, const float* clu_y,
                     int32_t* trk_off, int32_t* trk_hit_off, int32_t* trk_hit, uint32_t* trk_planes,
                     uint8_t* trk_flags, float* trk_logit, int64_t trk_cap, int64_t hit_cap, int32_t emit,
                     int32_t* status, void* stream) {
    if (int rc = check_ctx(c)) return rc;
    if (E < 0 || !clu_off || !trk_off || !trk_hit_off || trk_cap < 0 || hit_cap < 0)
        return fail(VELO_ERR_ARG, "bad arguments");
    if (trk_cap > 0 && (!trk_planes || !trk_hit)) return fail(VELO_ERR_ARG, "null track arrays");
    if (c->p.mode == 1 && !c->mlp.has_weights) return fail(VELO_ERR_ARG, "learned mode needs MLP weights");
    if (int rc = check_reserved(c, E, 0)) return rc;
    hipStream_t s = (hipStream_t)stream;
    HIP_OK(launch_reset(c->w, E, status, s));
    StageArgs sa{E * kPlanes, clu_off, clu_x, clu_y, c->w};
    HIP_OK(launch_stage(sa, s));
    return enqueue_find_out(c, E, clu_off, clu_x, clu_y, trk_off, trk_hit_off, trk_hit, trk_planes, trk_flags,
                            trk_logit, nullptr, trk_cap, hit_cap, emit, status, c->w.cap_clusters, s);
}

int velo_fit(velo_ctx* c, int64_t max_tracks, const int32_t* n_tracks, const int32_t* trk_hit_off,
             const int32_t* trk_hit, const uint32_t* trk_planes, const float* clu_x, const float* clu_y,
             float* par, void* stream) {
    if (!c) return fail(VELO_ERR_ARG, "null context");
    if (max_tracks < 0) return fail(VELO_ERR_ARG, "max_tracks < 0");
    if (max_tracks == 0) return VELO_OK;
    if (!trk_hit_off || !trk_hit || !trk_planes || !clu_x || !clu_y || !par)
        return fail(VELO_ERR_ARG, "null argument");
    FitArgs a{max_tracks, n_tracks, trk_hit_off, trk_hit, trk_planes, clu_x, clu_y, par, c->p};
    HIP_OK(launch_fit(a, (hipStream_t)stream));
    return VELO_OK;
}

int velo_decode(velo_ctx* c, int32_t E, const int32_t* bank_off, const uint32_t* bank, int32_t* pix_off,
                uint32_t* pix_id, int64_t pix_cap, int32_t* status, void* stream) {
    if (int rc = check_ctx(c)) return rc;
    if (E < 0 || pix_cap < 0 || !bank_off || !pix_off || (pix_cap > 0 && !pix_id)) return fail(VELO_ERR_ARG, "bad arguments");
    if (int rc = check_reserved(c, E, 0)) return rc;
    if (E == 0) return VELO_OK;
    hipStream_t s = (hipStream_t)stream;
    HIP_OK(launch_reset(c->w, E, status, s));
    DecodeArgs a{};
    a.n_seg = E * kPlanes;
    a.bank_off = bank_off;
    a.bank = bank;
    a.pix_off = pix_off;
    a.pix_id = pix_id;
    a.pix_cap = pix_cap;
    a.status = status;
    a.w = c->w;
    HIP_OK(launch_decode(a, s));
    return VELO_OK;
}

int velo_kalman_fit(velo_ctx* c, int64_t max_tracks, const int32_t* n_tracks, const int32_t* trk_hit_off,
                    const int32_t* trk_hit, const uint32_t* trk_planes, const float* clu_x, const float* clu_y,
                    float ms, float* out, void* stream) {
    if (!c) return fail(VELO_ERR_ARG, "null context");
    if (max_tracks < 0) return fail(VELO_ERR_ARG, "max_tracks < 0");
    if (!(ms >= 0.0f) || !std::isfinite(ms)) return fail(VELO_ERR_ARG, "ms must be finite and >= 0");
    if (max_tracks == 0) return VELO_OK;
    if (!trk_hit_off || !trk_hit || !trk_planes || !clu_x || !clu_y || !out)
        return fail(VELO_ERR_ARG, "null argument");
    KalmanArgs a{};
    a.max_tracks = max_tracks;
    a.n_tracks = n_tracks;
    a.trk_hit_off = trk_hit_off;
    a.trk_hit = trk_hit;
    a.trk_planes = trk_planes;
    a.clu_x = clu_x;
    a.clu_y = clu_y;
    a.out = out;
    for (int k = 0; k < kPlanes; ++k) a.z[k] = c->p.z[k];
    a.sigma = c->p.sigma;
    a.ms = ms;
    HIP_OK(launch_kalman(a, (hipStream_t)stream));
    return VELO_OK;
}

int velo_extrapolate(velo_ctx* c, int64_t max_tracks, const int32_t* n_tracks, const float* par, const float* x_hit,
                     const velo_magnet* m, float* out, void* stream) {
    if (!c || !m) return fail(VELO_ERR_ARG, "null argument");
    if (max_tracks < 0) return fail(VELO_ERR_ARG, "max_tracks < 0");
    if (!std::isfinite(m->z_mag) || !std::isfinite(m->z_t) || !(m->z_t > m->z_mag))
        return fail(VELO_ERR_ARG, "need finite z_mag < z_t");
    if (!std::isfinite(m->kick) || m->kick == 0.0f) return fail(VELO_ERR_ARG, "kick must be finite and non-zero");
    if (!std::isfinite(m->p_min) || !(m->p_min > 0.0f)) return fail(VELO_ERR_ARG, "p_min must be finite and > 0");
    if (max_tracks == 0) return VELO_OK;
    if (!par || !out) return fail(VELO_ERR_ARG, "null argument");
    if ((reinterpret_cast<uintptr_t>(par) | reinterpret_cast<uintptr_t>(out)) & 15)
        return fail(VELO_ERR_ARG, "par and out rows must be 16-byte aligned");
    ExtrapArgs a{};
    a.max_tracks = max_tracks;
    a.n_tracks = n_tracks;
    a.par = par;
    a.x_hit = x_hit;
    a.z_mag = m->z_mag;
    a.z_t = m->z_t;
    a.kick = m->kick;
    a.p_min = m->p_min;
    a.out = out;
    HIP_OK(launch_extrapolate(a, (hipStream_t)stream));
    return VELO_OK;
}

int velo_pipeline(velo_ctx* c, int32_t E, const int32_t* pix_off, const uint32_t* pix_id, int32_t* pix_clu,
                  int32_t* clu_off, float* clu_x, float* clu_y, int64_t clu_cap, int32_t* trk_off,
                  int32_t* trk_hit_off, int32_t* trk_hit, uint32_t* trk_planes, uint8_t* trk_flags,
                  float* trk_logit, float* par, int64_t trk_cap, int64_t hit_cap, int32_t* status,
                  void* stream) {
    if (int rc = check_ctx(c)) return rc;
    if (E <= 0 || !pix_off || !clu_off || !clu_x || !clu_y || !trk_off || !trk_hit_off || !trk_hit ||
        !trk_planes || clu_cap < 0 || trk_cap < 0 || hit_cap < 0)
        return fail(VELO_ERR_ARG, "bad arguments");
    if (c->p.mode == 1 && !c->mlp.has_weights) return fail(VELO_ERR_ARG, "learned mode needs MLP weights");
    if (int rc = check_reserved(c, E, std::min<int64_t>(clu_cap, c->w.cap_clusters))) return rc;
    if (clu_cap > c->w.cap_clusters)
        return fail(VELO_ERR_NOT_RESERVED, "clu_cap exceeds the reserved cluster capacity");
    hipStream_t s = (hipStream_t)stream;
    if (c->timing) {
        // eager run with events between the stages
        c->ev_valid = 0;
        ClusterArgs a{};
        a.n_seg = E * kPlanes;
        a.pix_off = pix_off;
        a.pix_id = pix_id;
        a.pix_clu = pix_clu;
        a.clu_off = clu_off;
        a.clu_x = clu_x;
        a.clu_y = clu_y;
        a.clu_npix = nullptr;
        a.clu_cap = clu_cap;
        a.status = status;
        a.validate = c->validate;
        a.stage = 1;
        a.w = c->w;
        if (int rc = mark(c, 0, s, true)) return rc;
        HIP_OK(launch_reset(c->w, E, status, s));
        if (int rc = mark(c, 1, s, true)) return rc;
        HIP_OK(launch_cluster(a, s));
        if (int rc = mark(c, 2, s, true)) return rc;
        int rc = enqueue_find_out(c, E, clu_off, clu_x, clu_y, trk_off, trk_hit_off, trk_hit, trk_planes, trk_flags,
                                  trk_logit, par, trk_cap, hit_cap, 0, status, clu_cap, s, true);
        if (rc) return rc;
        c->ev_stream = s;
        c->ev_valid = 1;
        return VELO_OK;
    }
    GraphKey key;
    key.v = {(uintptr_t)E, (uintptr_t)pix_off, (uintptr_t)pix_id, (uintptr_t)pix_clu, (uintptr_t)clu_off,
             (uintptr_t)clu_x, (uintptr_t)clu_y, (uintptr_t)clu_cap, (uintptr_t)trk_off, (uintptr_t)trk_hit_off,
             (uintptr_t)trk_hit, (uintptr_t)trk_planes, (uintptr_t)trk_flags, (uintptr_t)trk_logit,
             (uintptr_t)par, (uintptr_t)trk_cap, (uintptr_t)hit_cap, (uintptr_t)status, (uintptr_t)c->version,
             (uintptr_t)c->mlp.version, (uintptr_t)c->ws};
    if (!(c->exec && key == c->key)) {
        if (c->exec) {
            HIP_OK(hipGraphExecDestroy(c->exec));
            c->exec = nullptr;
        }
        hipStream_t cs = c->cap_stream;
        HIP_OK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        int rc = VELO_OK;
        ClusterArgs a{};
        a.n_seg = E * kPlanes;
        a.pix_off = pix_off;
        a.pix_id = pix_id;
        a.pix_clu = pix_clu;
        a.clu_off = clu_off;
        a.clu_x = clu_x;
        a.clu_y = clu_y;
        a.clu_npix = nullptr;
        a.clu_cap = clu_cap;
        a.status = status;
        a.validate = c->validate;
        a.stage = 1;
        a.w = c->w;
        if (launch_reset(c->w, E, status, cs) != hipSuccess || launch_cluster(a, cs) != hipSuccess)
            rc = fail(VELO_ERR_DEVICE, "launch failed during capture");
        if (!rc)
            rc = enqueue_find_out(c, E, clu_off, clu_x, clu_y, trk_off, trk_hit_off, trk_hit, trk_planes, trk_flags,
                                  trk_logit, par, trk_cap, hit_cap, 0, status, clu_cap, cs);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(cs, &g);
        if (rc) { if (g) (void)hipGraphDestroy(g); return rc; }
        if (e != hipSuccess) return fail(VELO_ERR_DEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&c->exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) { c->exec = nullptr; return fail(VELO_ERR_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e)); }
        c->key = key;
    }
    HIP_OK(hipGraphLaunch(c->exec, s));
    return VELO_OK;
}

int velo_autotune(velo_ctx* const* ctxs, int32_t n_ctx, int32_t E, const int32_t* clu_off, const float* clu_x,
                  const float* clu_y, int32_t reps, const char* cache_path, float* h_ms, void* const* streams) {
    if (!ctxs || n_ctx <= 0 || n_ctx > kMaxInFlight || !streams)
        return fail(VELO_ERR_ARG, "need 1..%d contexts and their streams", kMaxInFlight);
    if (E <= 0 || !clu_off || !clu_x || !clu_y || reps <= 0) return fail(VELO_ERR_ARG, "bad arguments");
    for (int i = 0; i < n_ctx; ++i) {
        if (int rc = check_ctx(ctxs[i])) return rc;
        if (int rc = check_reserved(ctxs[i], E, 0)) return rc;
        if (ctxs[i]->device != ctxs[0]->device) return fail(VELO_ERR_ARG, "contexts on different devices");
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) return fail(VELO_ERR_ARG, "a context appears twice");
    }
    velo_ctx* c0 = ctxs[0];
    HIP_OK(hipSetDevice(c0->device));
    // the batch's shape for the cache key: its cluster count (synchronous read)
    int32_t n_clu = 0;
    HIP_OK(hipMemcpy(&n_clu, clu_off + (int64_t)E * kPlanes, sizeof(int32_t), hipMemcpyDeviceToHost));
    std::string key;
    if (cache_path) {
        hipDeviceProp_t prop;
        HIP_OK(hipGetDeviceProperties(&prop, c0->device));
        key = tune_key(prop, c0, n_ctx, E, n_clu);
        int th = 0, tl = 0;
        if (tune_cache_lookup(cache_path, key, &th, &tl)) {
            for (int i = 0; i < n_ctx; ++i) {
                ctxs[i]->threads = th;
                ctxs[i]->tile = tl;
                ctxs[i]->version++;
            }
            if (h_ms)
                for (int i = 0; i < VELO_N_LAUNCH; ++i) h_ms[i] = -1.0f;
            return VELO_OK;
        }
    }
    TuneScope scope(ctxs, n_ctx);  // restores every launch and frees the events on any early return
    if (!scope.ok) return fail(VELO_ERR_DEVICE, "hipEventCreate failed");
    hipStream_t s0 = (hipStream_t)streams[0];
    // staging once per context; the finder changes only the used flags, which
    // every event resets when its planes are loaded
    for (int i = 0; i < n_ctx; ++i) {
        hipStream_t s = (hipStream_t)streams[i];
        HIP_OK(launch_reset(ctxs[i]->w, E, nullptr, s));
        StageArgs sa{E * kPlanes, clu_off, clu_x, clu_y, ctxs[i]->w};
        HIP_OK(launch_stage(sa, s));
    }
    const int threads[4] = {64, 128, 256, 512};
    float best = 1e30f;
    int bt = c0->threads, bl = c0->tile, idx = 0;
    for (int ti = 0; ti < 4; ++ti) {
        for (int tl = 0; tl < 3; ++tl, ++idx) {
            for (int i = 0; i < n_ctx; ++i) {
                ctxs[i]->threads = threads[ti];
                ctxs[i]->tile = tl;
            }
            // one warm-up batch per context, then reps batches per context, the
            // contexts' streams running concurrently between two joins on stream 0
            for (int r = 0; r <= reps; ++r) {
                if (r == 1) {
                    HIP_OK(join_streams(scope, streams, n_ctx));
                    HIP_OK(hipEventRecord(scope.e0, s0));
                    for (int i = 1; i < n_ctx; ++i) HIP_OK(hipStreamWaitEvent((hipStream_t)streams[i], scope.e0, 0));
                }
                for (int i = 0; i < n_ctx; ++i)
                    if (int rc = enqueue_tune_batch(ctxs[i], E, clu_off, clu_x, clu_y, (hipStream_t)streams[i]))
                        return rc;
            }
            HIP_OK(join_streams(scope, streams, n_ctx));
            HIP_OK(hipEventRecord(scope.e1, s0));
            HIP_OK(hipEventSynchronize(scope.e1));
            float ms = 0.0f;
            HIP_OK(hipEventElapsedTime(&ms, scope.e0, scope.e1));
            ms /= (float)(reps * n_ctx);
            if (h_ms) h_ms[idx] = ms;
            if (ms < best) { best = ms; bt = threads[ti]; bl = tl; }
        }
    }
    scope.commit(bt, bl);
    if (cache_path && !tune_cache_append(cache_path, key, bt, bl, best))
        return fail(VELO_ERR_ARG, "cannot append to the autotune cache %s (launch %d x tile %d was set)", cache_path,
                    bt, bl);
    return VELO_OK;
}

int velo_set_timing(velo_ctx* c, int32_t on) {
    if (!c) return fail(VELO_ERR_ARG, "null context");
    if (on && !c->ev[0]) {
        for (int i = 0; i <= VELO_N_STAGES; ++i) HIP_OK(hipEventCreate(&c->ev[i]));
    }
    c->timing = on ? 1 : 0;
    return VELO_OK;
}

int velo_last_timing(velo_ctx* c, float* h_ms, int32_t n) {
    if (!c || !h_ms || n < 0) return fail(VELO_ERR_ARG, "bad arguments");
    if (!c->ev_valid) return fail(VELO_ERR_ARG, "no timed pipeline call");
    HIP_OK(hipStreamSynchronize(c->ev_stream));
    for (int i = 0; i < n && i < VELO_N_STAGES; ++i) {
        float ms = 0.0f;
        HIP_OK(hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]));
        h_ms[i] = ms;
    }
    return VELO_OK;
}

int velo_status_read(velo_ctx* c, const int32_t* d_status, int32_t* h_status, int32_t n_words, void* stream) {
    if (!c || !d_status || !h_status || n_words < 0) return fail(VELO_ERR_ARG, "bad arguments");
    HIP_OK(hipStreamSynchronize((hipStream_t)stream));
    HIP_OK(hipMemcpy(h_status, d_status, sizeof(int32_t) * (size_t)n_words, hipMemcpyDeviceToHost));
    return VELO_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- learned filter
extern "C" {

int velo_seed_filter_set(velo_ctx* c, const float* h_weights, const float* h_norm, float threshold) {
    if (!c) return fail(VELO_ERR_ARG, "null context");
    if (!h_weights) {
        c->seed_on = 0;
        c->version++;
        return VELO_OK;
    }
    if (!h_norm) return fail(VELO_ERR_ARG, "null normalisation");
    for (int i = 0; i < kSeedIn; ++i)
        if (!(h_norm[kSeedIn + i] != 0.0f)) return fail(VELO_ERR_ARG, "normalisation sd must be non-zero");
    // host layout of the track network: W1 [unit][input], b1, W2 [unit][input], b2, w3, b3
    std::vector<float> d(kSeedFloats);
    for (int o = 0; o < kSeedH; ++o) {
        for (int i = 0; i < kSeedIn; ++i) d[kSeedW1T + i * kSeedH + o] = h_weights[o * kSeedIn + i];
        d[kSeedB1 + o] = h_weights[kSeedIn * kSeedH + o];
        for (int i = 0; i < kSeedH; ++i)
            d[kSeedW2T + i * kSeedH + o] = h_weights[kSeedIn * kSeedH + kSeedH + o * kSeedH + i];
        d[kSeedB2 + o] = h_weights[kSeedIn * kSeedH + kSeedH + kSeedH * kSeedH + o];
        d[kSeedW3 + o] = h_weights[kSeedIn * kSeedH + 2 * kSeedH + kSeedH * kSeedH + o];
    }
    d[kSeedB3] = h_weights[kSeedIn * kSeedH + 3 * kSeedH + kSeedH * kSeedH];
    for (int i = 0; i < kSeedIn; ++i) {
        d[kSeedNorm + i] = h_norm[i];
        d[kSeedNorm + kSeedIn + i] = 1.0f / h_norm[kSeedIn + i];  // FP32, as the network defines it
    }
    d[kSeedThr] = threshold;
    HIP_OK(hipSetDevice(c->device));
    HIP_OK(hipMemcpy(c->d_seed, d.data(), sizeof(float) * kSeedFloats, hipMemcpyHostToDevice));
    c->seed_on = 1;
    c->version++;
    return VELO_OK;
}

int velo_seed_emit(velo_ctx* c, float* d_feat, int32_t* d_hits, int64_t cap, unsigned long long* d_count) {
    if (!c) return fail(VELO_ERR_ARG, "null context");
    if (!d_feat && !d_hits && !d_count) {
        c->seed_feat = nullptr;
        c->seed_hits = nullptr;
        c->seed_cap = 0;
        c->seed_count = nullptr;
        c->version++;
        return VELO_OK;
    }
    if (!d_feat || !d_hits || !d_count || cap < 0) return fail(VELO_ERR_ARG, "seed emission needs all three buffers");
    c->seed_feat = d_feat;
    c->seed_hits = d_hits;
    c->seed_cap = cap;
    c->seed_count = d_count;
    c->version++;
    return VELO_OK;
}

int velo_mlp_set_weights(velo_ctx* c, const float* h_master, const float* h_norm) {
    if (!c || !h_master || !h_norm) return fail(VELO_ERR_ARG, "null argument");
    for (int i = 0; i < kNFeat; ++i)
        if (!(h_norm[kNFeat + i] != 0.0f)) return fail(VELO_ERR_ARG, "normalisation sd must be non-zero");
    HIP_OK(hipMemcpy(c->mlp.d_master, h_master, sizeof(float) * kNParam, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(c->mlp.d_norm, h_norm, sizeof(float) * 2 * kNFeat, hipMemcpyHostToDevice));
    c->mlp.has_weights = 1;
    c->mlp.version++;
    return VELO_OK;
}

int velo_mlp_get_weights(velo_ctx* c, float* h_master, float* h_norm) {
    if (!c || !h_master || !h_norm) return fail(VELO_ERR_ARG, "null argument");
    HIP_OK(hipMemcpy(h_master, c->mlp.d_master, sizeof(float) * kNParam, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(h_norm, c->mlp.d_norm, sizeof(float) * 2 * kNFeat, hipMemcpyDeviceToHost));
    return VELO_OK;
}

int velo_features(velo_ctx* c, int64_t n, const int32_t* trk_hit_off, const int32_t* trk_hit,
                  const uint32_t* trk_planes, const float* clu_x, const float* clu_y, uint16_t* feat,
                  float* feat32, void* stream) {
    if (!c || n < 0) return fail(VELO_ERR_ARG, "bad arguments");
    if (n == 0) return VELO_OK;
    if (!trk_hit_off || !trk_hit || !trk_planes || !clu_x || !clu_y || (!feat && !feat32))
        return fail(VELO_ERR_ARG, "null argument");
    if (feat && !c->mlp.has_weights) return fail(VELO_ERR_ARG, "normalisation not set (velo_mlp_set_weights)");
    HIP_OK(launch_features(c->p, c->mlp.d_norm, n, trk_hit_off, trk_hit, trk_planes, clu_x, clu_y, feat, feat32,
                           (hipStream_t)stream));
    return VELO_OK;
}

int velo_standardize(velo_ctx* c, int64_t n, const float* raw, uint16_t* feat, void* stream) {
    if (!c || n < 0) return fail(VELO_ERR_ARG, "bad arguments");
    if (n == 0) return VELO_OK;
    if (!raw || !feat) return fail(VELO_ERR_ARG, "null argument");
    if (!c->mlp.has_weights) return fail(VELO_ERR_ARG, "normalisation not set (velo_mlp_set_weights)");
    HIP_OK(launch_standardize(c->mlp.d_norm, n, raw, feat, (hipStream_t)stream));
    return VELO_OK;
}

int velo_mlp_forward(velo_ctx* c, int64_t n, const uint16_t* feat, float* logit, void* stream) {
    if (!c || n < 0) return fail(VELO_ERR_ARG, "bad arguments");
    if (n == 0) return VELO_OK;
    if (!feat || !logit) return fail(VELO_ERR_ARG, "null argument");
    if (!c->mlp.has_weights) return fail(VELO_ERR_ARG, "weights not set");
    HIP_OK(launch_mlp_forward(c->mlp, n, feat, logit, (hipStream_t)stream));
    return VELO_OK;
}

int velo_mlp_grad(velo_ctx* c, int64_t n, const uint16_t* feat, const uint8_t* label, float* grad, float* loss,
                  void* stream) {
    if (!c || n <= 0 || !feat || !label || !grad) return fail(VELO_ERR_ARG, "bad arguments");
    if (!c->mlp.has_weights) return fail(VELO_ERR_ARG, "weights not set");
    HIP_OK(launch_mlp_grad(c->mlp, n, feat, label, grad, loss, (hipStream_t)stream));
    return VELO_OK;
}

int velo_mlp_train_step(velo_ctx* c, int64_t n, const uint16_t* feat, const uint8_t* label, float lr, float* loss,
                        void* stream) {
    if (!c || n <= 0 || !feat || !label || !(lr >= 0.0f)) return fail(VELO_ERR_ARG, "bad arguments");
    if (!c->mlp.has_weights) return fail(VELO_ERR_ARG, "weights not set");
    hipStream_t s = (hipStream_t)stream;
    HIP_OK(launch_mlp_grad(c->mlp, n, feat, label, c->mlp.d_grad, loss, s));
    c->mlp.step += 1;
    HIP_OK(launch_adam(c->mlp, lr, s));
    c->mlp.version++;
    return VELO_OK;
}

int velo_mlp_set_adam(velo_ctx* c, float beta1, float beta2, float eps) {
    if (!c || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return fail(VELO_ERR_ARG, "bad Adam parameters");
    c->mlp.beta1 = beta1;
    c->mlp.beta2 = beta2;
    c->mlp.eps = eps;
    return VELO_OK;
}

int velo_mlp_get_state(velo_ctx* c, float* h_master, float* h_m, float* h_v, int64_t* h_step) {
    if (!c || !h_master || !h_m || !h_v || !h_step) return fail(VELO_ERR_ARG, "null argument");
    HIP_OK(hipDeviceSynchronize());
    HIP_OK(hipMemcpy(h_master, c->mlp.d_master, sizeof(float) * kNParam, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(h_m, c->mlp.d_m, sizeof(float) * kNParam, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(h_v, c->mlp.d_v, sizeof(float) * kNParam, hipMemcpyDeviceToHost));
    *h_step = c->mlp.step;
    return VELO_OK;
}

int velo_mlp_set_state(velo_ctx* c, const float* h_master, const float* h_m, const float* h_v, int64_t step) {
    if (!c || !h_master || !h_m || !h_v || step < 0) return fail(VELO_ERR_ARG, "bad arguments");
    HIP_OK(hipDeviceSynchronize());
    HIP_OK(hipMemcpy(c->mlp.d_master, h_master, sizeof(float) * kNParam, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(c->mlp.d_m, h_m, sizeof(float) * kNParam, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(c->mlp.d_v, h_v, sizeof(float) * kNParam, hipMemcpyHostToDevice));
    c->mlp.step = step;
    c->mlp.version++;
    return VELO_OK;
}

}  // extern "C"
