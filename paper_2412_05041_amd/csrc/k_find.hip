// k_find.hip -- track finding: triplet seeding + plane-by-plane extension.
//
// One workgroup owns one event at a time and walks the planes from the most
// downstream one (k = 25) to the most upstream one (k = 0).  At step k:
//   T1  every open track is extended onto plane k: its line (through its two
//       most upstream hits) is evaluated at z_k and the closest unused hit with
//       squared miss distance q <= e_max is wanted (ties: lower hit index); a
//       hit wanted by several tracks goes to the lowest track index.  A track
//       stays open while it has skipped at most max_skip planes.
//   T2  seeds: every triplet (h0 on k, h1 on k+1, h2 on k+2) of unused hits
//       with |tx|,|ty| <= t_max, pointing outward and passing within
//       sqrt(d2_max) of the beam axis, and with middle-hit miss q <= s_max, is a
//       candidate.  Candidates are accepted greedily by (q, h0, h1, h2) when
//       all three hits are still free; accepted seeds become tracks with
//       consecutive indices in that order.
//   T3  the new tracks are extended downstream (planes k+3 .. 25) in lockstep,
//       with the same rule as T1.
// A separate kernel then fits every candidate (least squares, FP32) and accepts
// it when chi2/ndof <= c3 (3 hits) or c4 (plain mode), or writes its features
// for the learned decision.  Every expression follows the oracle's order of
// operations; the device code is built without contraction.
//
// Parallel formulation (identical results):
//   * hits of each plane are staged sorted by azimuth; a candidate search only
//     visits hits whose azimuth lies in a window that provably contains every
//     hit passing the exact cut (plus a margin far above rounding), and the
//     exact FP32 cut then decides;
//   * the planes k .. k+4 sit in an LDS ring, which covers seeding (k .. k+2)
//     and the usual reach of the downstream completion (k+3, k+4);
//   * T1/T3 conflicts: atomicMin of the track index on the wanted hit;
//   * T2 greedy: rounds of "every candidate that holds the smallest key on all
//     three of its hits wins"; the per-hit minimum of the 96-bit key is taken
//     in two phases (64-bit atomicMin of (q, h0), then 32-bit atomicMin of
//     (h1, h2) among the candidates holding that minimum on the hit).  This
//     accepts exactly the candidates the sequential greedy accepts; winners are
//     then ranked by key for their track indices.
#include "fitfeat.h"
#include "kernels.h"

namespace velo {

namespace {

constexpr float kPi = 3.14159265358979f;
constexpr float kTwoPi = 6.28318530717959f;
constexpr int kIntMax = 0x7fffffff;
constexpr int kRing = 5;  // planes k .. k+4 in the window
constexpr int kLutLarge = 4096;  // key buckets of a large-event plane
constexpr float kKeysPerRad = 10430.378350470453f;  // 2^16 / (2 pi)

// Phase timing (a diagnostic build, -DVELO_PHASE_TIMING): per finder pass
// (0: first LDS tile, 1: second tile, 2: global memory) thread 0 of each
// workgroup adds the wall-clock ticks of each phase of a plane step, after a
// barrier: 0 plane load, 1 forwarding, 2 seed enumeration, 3 seed filter +
// claiming, 4 track creation + downstream completion; then 5/6 downstream
// completion steps on ring / non-ring planes, 7 ticks of the latter, 8
// events, 9 ticks of whole events, 10 the part of the plane load that writes
// the ring (LDS-tile passes; slot 0 then holds the next plane's prefetch).
#ifdef VELO_PHASE_TIMING
// 64 copies of the counters, one per workgroup index modulo 64, so that the
// counters' own atomics do not contend (they would hold up every later wait
// on memory of the workgroups adding them); the probe sums the copies.
constexpr int kPhaseSlots = 12, kPhaseCopies = 64;
__device__ unsigned long long g_phase[3][kPhaseCopies][kPhaseSlots];
__device__ __forceinline__ int phase_pass(const FindArgs& a) {
    return a.q_in == a.w.order ? 0 : (a.q_in == a.w.large ? 1 : 2);
}
#define PHASE_T0() uint64_t ph_t = wall_clock64(), ph_t0 = ph_t
#define PHASE(i)                                                        \
    do {                                                                \
        __syncthreads();                                                \
        if (threadIdx.x == 0) {                                         \
            const uint64_t now = wall_clock64();                        \
            atomicAdd(&g_phase[phase_pass(a)][blockIdx.x % kPhaseCopies][i], (unsigned long long)(now - ph_t)); \
            ph_t = now;                                                 \
        }                                                               \
    } while (0)
#define PCOUNT(i, v)                                                    \
    do {                                                                \
        if (threadIdx.x == 0) atomicAdd(&g_phase[phase_pass(a)][blockIdx.x % kPhaseCopies][i], (unsigned long long)(v)); \
    } while (0)
#define PCLOCK() wall_clock64()
#define PHASE_END()                                                     \
    do {                                                                \
        PCOUNT(8, 1);                                                   \
        PCOUNT(9, wall_clock64() - ph_t0);                              \
    } while (0)
#else
#define PHASE_T0() (void)0
#define PHASE(i) (void)0
#define PCOUNT(i, v) (void)0
#define PCLOCK() 0ull
#define PHASE_END() (void)0
#endif

// ---------------------------------------------------------------- storage
// Accessors hide where a workgroup keeps its per-event state: the LDS tile
// (normal events) or global scratch (large events).

// An LDS tile: plane capacity kP, tracks kT, seed candidates per step kC;
// 2^kLB key buckets in the index of a ring plane, 2^kCB in the coarse index
// every plane of the event keeps.
template <int kP, int kT, int kC, int kLB, int kCB>
struct Tile {
    float wx[kRing][kP];
    float wy[kRing][kP];
    uint64_t slota[3][kP];  // seeding planes k, k+1, k+2 (then winner keys)
    uint32_t slotb[3][kP];  // (then winner list, then downstream claims)
    int32_t claim[kP];
    uint16_t wid[kRing][kP];  // plane-local cluster index
    uint16_t wk[kRing][kP];
    uint32_t ubits[kPlanes][(kP + 31) / 32];  // used flags of every plane of the event
    // tracks: upstream end (T1); the downstream end (T3) of a step's new tracks
    // lives in the seeding-slot memory once the seeds are claimed
    float ttx[kT], tty[kT], txb[kT], tyb[kT];
    uint32_t tmask[kT];
    int16_t twant[kT];
    int8_t tkb[kT];
    float cq[kC];
    uint16_t cp[kC][3];
    uint8_t calive[kC];
    uint16_t lut[kRing][(1 << kLB) + 1];     // first position of each key bucket
    uint16_t clut[kPlanes][(1 << kCB) + 1];  // coarse bucket index of every plane of the event
};

struct Scalars {
    int n_tracks, n_cand, n_acc, event, n_pairs;
    int wsum[16];            // per-wave partial sums of block scans
    float z[kPlanes];        // plane positions (lane-indexed reads stay in LDS)
    int wn[kRing];
    int wplane[kRing];       // plane held by each ring slot
    int64_t wg[kRing];       // staged (= cluster) base of the plane in each ring slot
    int64_t cb[kPlanes + 1]; // global cluster offsets of the event's planes
};

template <int kP, int kT, int kC, int kLB, int kCB>
struct LdsStore {
    static constexpr bool kLarge = false;
    Tile<kP, kT, kC, kLB, kCB>* t;
    Scalars* s;
    int64_t slot0;
    int seed_k = 0;
    int dbase = 0;  // first track of the downstream-state window
    int dn = 0;     // its length
    __device__ float X(int sl, int i) const { return t->wx[sl][i]; }
    __device__ float Y(int sl, int i) const { return t->wy[sl][i]; }
    __device__ int K(int sl, int i) const { return t->wk[sl][i]; }
    __device__ int L(int sl, int i) const { return t->wid[sl][i]; }  // plane-local index
    __device__ int64_t ID(int sl, int i) const { return s->wg[sl] + t->wid[sl][i]; }
    __device__ bool UP(int j, int i) const { return (t->ubits[j][i >> 5] >> (i & 31)) & 1u; }
    __device__ void set_UP(int j, int i) { atomicOr(&t->ubits[j][i >> 5], 1u << (i & 31)); }
    // used flag of position i of plane j, held in ring slot sl
    __device__ bool U(int, int j, int i) const { return UP(j, i); }
    __device__ void set_U(int, int j, int i) { set_UP(j, i); }
    __device__ int32_t* claim(int) { return t->claim; }
    __device__ int32_t* claimT(int64_t) { return reinterpret_cast<int32_t*>(&t->slotb[0][0]); }
    __device__ uint64_t* slotA(int role) { return t->slota[role]; }
    __device__ uint32_t* slotB(int role) { return t->slotb[role]; }
    __device__ float& ttx(int i) { return t->ttx[i]; }
    __device__ float& tty(int i) { return t->tty[i]; }
    __device__ float& txb(int i) { return t->txb[i]; }
    __device__ float& tyb(int i) { return t->tyb[i]; }
    __device__ float* dst() const { return reinterpret_cast<float*>(&t->slota[0][0]); }
    __device__ float& dtx(int i) { return dst()[i - dbase]; }
    __device__ float& dty(int i) { return dst()[dn + i - dbase]; }
    __device__ float& dxb(int i) { return dst()[2 * dn + i - dbase]; }
    __device__ float& dyb(int i) { return dst()[3 * dn + i - dbase]; }
    __device__ int tkb(int i) const { return t->tkb[i]; }
    __device__ void set_tkb(int i, int v) { t->tkb[i] = (int8_t)v; }
    __device__ int dkb(int i) const { return reinterpret_cast<const int8_t*>(dst() + 4 * dn)[i - dbase]; }
    __device__ void set_dkb(int i, int v) { reinterpret_cast<int8_t*>(dst() + 4 * dn)[i - dbase] = (int8_t)v; }
    // enumeration scratch (seeding slots are free before the claiming rounds)
    __device__ int32_t* pref() { return reinterpret_cast<int32_t*>(&t->slotb[0][0]); }
    __device__ int32_t* ebuf() { return reinterpret_cast<int32_t*>(&t->slota[0][0]); }
    // h0 of each thread's first seed pair (after the window bounds ebuf holds)
    __device__ int32_t* first_h0() { return ebuf() + 4 * kP; }
    // seed-filter broadcast scratch: 2 x 32 floats for each of a round's (at
    // most 16) candidate groups, in the seeding slots (still free then)
    __device__ float* bcast() { return reinterpret_cast<float*>(&t->slota[0][0]); }
    static_assert(sizeof(uint64_t) * 3 * kP >= sizeof(float) * 2 * 16 * kSeedH, "broadcast scratch fits the slots");
    __device__ uint32_t& tmask(int i) { return t->tmask[i]; }
    __device__ int16_t& twant(int i) { return t->twant[i]; }
    __device__ float& cq(int i) { return t->cq[i]; }
    __device__ int cp(int i, int j) const { return t->cp[i][j]; }
    __device__ void set_cp(int i, int a, int b, int c) {
        t->cp[i][0] = (uint16_t)a; t->cp[i][1] = (uint16_t)b; t->cp[i][2] = (uint16_t)c;
    }
    __device__ uint8_t& calive(int i) { return t->calive[i]; }
    // winner keys and winner list (after the rounds), clear of the downstream
    // state that overlays slota
    __device__ uint64_t* wkey64() { return reinterpret_cast<uint64_t*>(&t->slotb[0][0]); }
    __device__ uint32_t* wtmp() { return &t->slotb[2][0]; }
    __device__ int cap_tracks() const { return kT; }
    __device__ int cap_cand() const { return kC; }
    static constexpr int kPlaneCap = kP;
    static constexpr int kLutN = 1 << kLB;
    static constexpr int kLutShift = kKeyBits - kLB;
    static constexpr int kCoarseN = 1 << kCB;
    static constexpr int kCoarseShift = kKeyBits - kCB;
    __device__ uint16_t* lut(int sl) { return t->lut[sl]; }
};

struct GlobalStore {
    static constexpr bool kLarge = true;
    static constexpr int kPlaneCap = 0;  // planes stay in global memory
    Scalars* s;
    const Work* w;
    int64_t slot0;   // first candidate slot of the event
    int64_t pool0;   // first seed-pool entry of this workgroup
    int cap_t;
    int seed_k = 0;  // plane of h0 during seeding
    const float* seedw = nullptr;  // seed network in LDS, rows [unit][input] (seed variant)
    float* seedh = nullptr;        // per-thread first-layer activations in LDS, [unit][thread]
    __device__ float* bcast() { return seedh; }  // seed-filter broadcast scratch (>= 2 x 16 x 32 floats)
    __device__ float X(int sl, int i) const { return w->stg[s->wg[sl] + i].x; }
    __device__ float Y(int sl, int i) const { return w->stg[s->wg[sl] + i].y; }
    __device__ int K(int sl, int i) const { return (int)w->stg[s->wg[sl] + i].key; }
    __device__ int L(int sl, int i) const { return (int)(w->stg[s->wg[sl] + i].id - s->wg[sl]); }
    __device__ int64_t ID(int sl, int i) const { return w->stg[s->wg[sl] + i].id; }
    __device__ bool U(int sl, int, int i) const { return w->used[s->wg[sl] + i] != 0; }
    __device__ void set_U(int sl, int, int i) { w->used[s->wg[sl] + i] = 1; }
    __device__ int32_t* claim(int sl) { return w->g_claim + s->wg[sl]; }
    __device__ int32_t* claimT(int64_t g) { return w->g_claim + g; }
    __device__ uint64_t* slotA(int role) { return w->g_slota + s->cb[seed_k + role]; }
    __device__ uint32_t* slotB(int role) { return w->g_slotb + s->cb[seed_k + role]; }
    __device__ float& ttx(int i) { return w->g_ttx[slot0 + i]; }
    __device__ float& tty(int i) { return w->g_tty[slot0 + i]; }
    __device__ float& txb(int i) { return w->g_txb[slot0 + i]; }
    __device__ float& tyb(int i) { return w->g_tyb[slot0 + i]; }
    __device__ float& dtx(int i) { return w->g_dtx[slot0 + i]; }
    __device__ float& dty(int i) { return w->g_dty[slot0 + i]; }
    __device__ float& dxb(int i) { return w->g_dxb[slot0 + i]; }
    __device__ float& dyb(int i) { return w->g_dyb[slot0 + i]; }
    __device__ int tkb(int i) const { return w->g_tkb[slot0 + i] & 0xff; }
    __device__ void set_tkb(int i, int v) { w->g_tkb[slot0 + i] = (w->g_tkb[slot0 + i] & ~0xff) | v; }
    __device__ int dkb(int i) const { return (w->g_tkb[slot0 + i] >> 8) & 0xff; }
    __device__ void set_dkb(int i, int v) { w->g_tkb[slot0 + i] = (w->g_tkb[slot0 + i] & ~0xff00) | (v << 8); }
    __device__ uint32_t& tmask(int i) { return w->cmask[slot0 + i]; }
    __device__ int32_t& twant(int i) { return w->g_twant[slot0 + i]; }
    __device__ float& cq(int i) { return w->p_q[pool0 + i]; }
    __device__ int cp(int i, int j) const { return w->p_h[(pool0 + i) * 3 + j]; }
    __device__ void set_cp(int i, int a, int b, int c) {
        int32_t* h = w->p_h + (pool0 + i) * 3;
        h[0] = a; h[1] = b; h[2] = c;
    }
    __device__ uint8_t& calive(int i) { return w->p_alive[pool0 + i]; }
    __device__ uint64_t* wkey64() { return w->g_slota + s->cb[seed_k]; }
    __device__ uint32_t* wtmp() { return w->g_slotb + s->cb[seed_k]; }
    __device__ int cap_tracks() const { return cap_t; }
    __device__ int cap_cand() const { return (int)w->pool_use; }
    int dbase = 0, dn = 0;
    int32_t* cell = nullptr;  // this workgroup's grid cell starts (plane-major)
    __device__ const int32_t* cells(int j) const { return cell + (int64_t)j * (kCells + 1); }
    __device__ int32_t* pref() { return w->g_enum + 6 * s->cb[seed_k]; }
    __device__ int32_t* ebuf() { return w->g_enum + 6 * s->cb[seed_k] + s->cb[seed_k + 1] - s->cb[seed_k] + 1; }
    static constexpr int kLutN = kLutLarge;
    static constexpr int kLutShift = 4;
    uint16_t (*luts)[kLutLarge + 1] = nullptr;  // LDS
    __device__ uint16_t* lut(int sl) { return luts[sl]; }
    uint32_t* hist = nullptr;  // LDS histogram of the key-range seeding
};

// ---------------------------------------------------------------- windows

// Key ranges covering keys [a - m, b + m] on the key circle (a <= b, as plain
// integers possibly outside [0, 65535]).
__device__ __forceinline__ int key_span(int a, int b, int m, int* lo, int* hi) {
    int l = a - m, h = b + m;
    if (h - l >= 65535) { lo[0] = 0; hi[0] = 65535; return 1; }
    if (l < 0) {
        lo[0] = l + 65536; hi[0] = 65535;
        lo[1] = 0; hi[1] = h;
        return 2;
    }
    if (h > 65535) {
        lo[0] = l; hi[0] = 65535;
        lo[1] = 0; hi[1] = h - 65536;
        return 2;
    }
    lo[0] = l; hi[0] = h;
    return 1;
}

// Key ranges covering every key position within asin(R/|E|) of the azimuth of
// E = (ex, ey), from cheap bounds rather than atan2f and asinf:
//   * the azimuth of E: an octant reduction to atan(t), |t| <= 1, evaluated
//     with the odd degree-9 polynomial of Abramowitz & Stegun 4.4.49 (Hastings;
//     |error| about 1e-5 rad) and the hardware reciprocal;
//   * the half-angle: asin(x) <= tan(asin(x)) = R / sqrt(|E|^2 - R^2), from the
//     hardware reciprocal square root, widened by 0.1 %;
// then 1e-4 rad and two keys on each side absorb the polynomial's error, FP32
// rounding, the truncation of the staged keys and their clamp at 65535.  A
// point within 2R of the axis takes the whole circle.
__device__ __forceinline__ int point_window(float ex, float ey, float R, int* lo, int* hi) {
    const float e2 = ex * ex + ey * ey;
    if (!(e2 > 4.0f * R * R)) { lo[0] = 0; hi[0] = 65535; return 1; }
    const float half = R * __builtin_amdgcn_rsqf(e2 - R * R) * 1.001f + 1e-4f;
    const float ax = fabsf(ex), ay = fabsf(ey);
    const float t = fminf(ax, ay) * __builtin_amdgcn_rcpf(fmaxf(ax, ay));
    const float s = t * t;
    float phi = t * (0.9998660f + s * (-0.3302995f + s * (0.1801410f + s * (-0.0851330f + s * 0.0208351f))));
    if (ay > ax) phi = 1.57079633f - phi;
    if (ex < 0.0f) phi = kPi - phi;
    if (ey < 0.0f) phi = -phi;
    const float c = (phi + kPi) * kKeysPerRad;
    const float w = half * kKeysPerRad;
    return key_span((int)floorf(c - w) - 2, (int)ceilf(c + w) + 2, 0, lo, hi);
}

// Grid cell (one axis) of a coordinate; monotone in v, clamped to the grid.
__device__ __forceinline__ int grid_cell1(float v) {
    const float c = floorf((v + kGridOrg) * kGridInv);
    return (int)fminf(fmaxf(c, 0.0f), (float)(kGridN - 1));
}

// Visits every cell-order position whose cell meets the square around the
// disc (c, R); a margin of 1e-3 mm keeps the FP32 bounds outside the disc.
template <class F>
__device__ __forceinline__ void grid_visit(const int32_t* cs, float cx, float cy, float R, F f) {
    const float rm = R + 1e-3f;
    const int ix0 = grid_cell1(cx - rm), ix1 = grid_cell1(cx + rm);
    const int iy0 = grid_cell1(cy - rm), iy1 = grid_cell1(cy + rm);
    for (int iy = iy0; iy <= iy1; ++iy) {
        const int e = cs[iy * kGridN + ix1 + 1];
        for (int q = cs[iy * kGridN + ix0]; q < e; ++q) f(q);
    }
}

template <class KF>
__device__ __forceinline__ int lower_key(KF key, int n, int v) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (key(mid) < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Lower bound through a bucket index: lut[b] = first position whose key
// has bucket >= b, then a short forward scan.
template <int kShift, class KF>
__device__ __forceinline__ int lower_lut(const uint16_t* lut, KF key, int n, int v) {
    int i = lut[v >> kShift];
    while (i < n && key(i) < v) ++i;
    return i;
}

// Visits every position of a key-sorted plane whose key lies in the ranges
// lo[r] .. hi[r], through its bucket index lut (lut[b] = first position whose
// key bucket is >= b): every position of the buckets a range touches, with
// the key test inside, so the ends of a range are not searched for.  A
// position's data (load(i)) is read together with its key, two positions at
// a time, and f(i, data) sees the ones that pass: a visit waits for one round
// of reads per two positions instead of a chain of key reads and data reads.
template <int kShift, class KF, class LF, class F>
__device__ __forceinline__ void visit_lut(const uint16_t* lut, KF key, LF load, int nr, const int* lo, const int* hi,
                                          F f) {
    for (int r = 0; r < nr; ++r) {
        const int i1 = lut[(hi[r] >> kShift) + 1];
        for (int i = lut[lo[r] >> kShift]; i < i1; i += 2) {
            const int j = min(i + 1, i1 - 1);
            const int ka = key(i), kb = key(j);
            const auto da = load(i);
            const auto db = load(j);
            if (ka >= lo[r] && ka <= hi[r]) f(i, da);
            if (j > i && kb >= lo[r] && kb <= hi[r]) f(j, db);
        }
    }
}

// What a window search reads of a staged position besides its key.
struct PosData {
    float x, y;
    int id;
    bool used;
};

// Half-width in keys of the azimuth range subtended by a disc of radius R seen
// at distance r (asin(R/r) plus margins), or -1 when the whole circle is needed.
__device__ __forceinline__ int disc_keys(float R, float r) {
    if (!(r > R * 1.001f + 1e-3f)) return -1;
    return (int)ceilf((asinf(R / r) * 1.0001f + 2e-4f) * kKeysPerRad) + 2;
}

// Best unused hit (q, index) within e_max of (ex, ey) on a staged plane in
// LDS with bucket index lut.
template <int kShift, class KF, class UF, class XF, class YF, class IF>
__device__ __forceinline__ int best_hit(const uint16_t* lut, KF key, UF used, XF xf, YF yf, IF idf, float ex, float ey,
                                        const Params& p) {
    int lo[2], hi[2];
    const int nr = point_window(ex, ey, p.r_ext, lo, hi);
    float bq = 0.0f;
    int bid = kIntMax, want = -1;
    auto load = [&](int i) { return PosData{xf(i), yf(i), idf(i), used(i)}; };
    visit_lut<kShift>(lut, key, load, nr, lo, hi, [&](int i, const PosData& d) {
        if (d.used) return;
        const float dx = d.x - ex;
        const float dy = d.y - ey;
        const float q = dx * dx + dy * dy;
        if (!(q <= p.e_max)) return;
        if (want < 0 || q < bq || (q == bq && d.id < bid)) { want = i; bq = q; bid = d.id; }
    });
    return want;
}

// best_hit on a plane read from global memory through a bucket index: every
// position of the buckets the key ranges touch is visited -- the bounds come
// from the index alone -- and the key test inside keeps exactly the positions
// best_hit visits.  The positions are read four at a time into separate
// registers (the last group's spare reads repeat its last position and are
// skipped), so that a search waits once per group, not once per hit; the
// skip test uses non-short-circuit operators so that each read is used
// unconditionally and stays where it is issued.
template <int kShift, class UF>
__device__ __forceinline__ int best_hit_buckets(const uint16_t* lut, const Staged* plane, UF used, int64_t gbase,
                                                float ex, float ey, const Params& p) {
    constexpr int kB = 4;
    int lo[2], hi[2];
    const int nr = point_window(ex, ey, p.r_ext, lo, hi);
    float bq = 0.0f;
    int bid = kIntMax, want = -1;
    for (int r = 0; r < nr; ++r) {
        const int i0 = lut[lo[r] >> kShift], i1 = lut[(hi[r] >> kShift) + 1];
        for (int b = i0; b < i1; b += kB) {
            Staged h[kB];
#pragma unroll
            for (int u = 0; u < kB; ++u) h[u] = plane[min(b + u, i1 - 1)];
#pragma unroll
            for (int u = 0; u < kB; ++u) {
                const int i = b + u;
                const int k = (int)h[u].key;
                if (((i >= i1) | (k < lo[r]) | (k > hi[r])) || used(i)) continue;
                const float dx = h[u].x - ex;
                const float dy = h[u].y - ey;
                const float q = dx * dx + dy * dy;
                if (!(q <= p.e_max)) continue;
                const int id = (int)(h[u].id - gbase);
                if (want < 0 || q < bq || (q == bq && id < bid)) { want = i; bq = q; bid = id; }
            }
        }
    }
    return want;
}

// best_hit on a plane of the large-event path through its grid (same rule).
__device__ __forceinline__ int best_hit_grid(const Work& w, const int32_t* cs, int64_t g, float ex, float ey,
                                             const Params& p) {
    float bq = 0.0f;
    int bid = kIntMax, want = -1;
    grid_visit(cs, ex, ey, p.r_ext, [&](int q0) {
        const int i = w.g_gpos[g + q0];
        if (w.used[g + i]) return;
        const float dx = w.g_gx[g + q0] - ex;
        const float dy = w.g_gy[g + q0] - ey;
        const float q = dx * dx + dy * dy;
        if (!(q <= p.e_max)) return;
        const int id = (int)(w.stg[g + i].id - g);
        if (want < 0 || q < bq || (q == bq && id < bid)) { want = i; bq = q; bid = id; }
    });
    return want;
}

// ---------------------------------------------------------------- steps

// Block-wide exclusive scan of v[0..n) in place; v[n] = total.  Each thread
// scans a contiguous chunk; chunk sums are combined with a wave scan.
template <int kT, class V>
__device__ void block_excl_scan(V* v, int n, Scalars& sc) {
    const int per = (n + kT - 1) / kT;
    const int b0 = threadIdx.x * per;
    int loc = 0;
    for (int i = b0; i < b0 + per && i < n; ++i) loc += v[i];
    int tot;
    const int ex = wave_excl_scan(loc, &tot);
    const int wv = threadIdx.x / kWave;
    if ((threadIdx.x % kWave) == 0) sc.wsum[wv] = tot;
    __syncthreads();
    int run = ex;
    for (int q = 0; q < wv; ++q) run += sc.wsum[q];
    int total = 0;
    for (int q = 0; q < kT / kWave; ++q) total += sc.wsum[q];
    for (int i = b0; i < b0 + per && i < n; ++i) {
        const int c = v[i];
        v[i] = run;
        run += c;
    }
    if (threadIdx.x == 0) v[n] = total;
    __syncthreads();
}

// Registers holding the first hits of the next plane, loaded one step ahead so
// that the global-memory latency overlaps the current step.  The values stay
// as loaded (the cluster index global) until the plane is written to the
// ring: any arithmetic on them here would wait for the load right away.
struct Prefetch {
    float x[2], y[2];
    int key[2], kprev[2], id[2];
};

template <int kT, int kPF>
__device__ __forceinline__ void prefetch_plane(const Scalars& sc, const FindArgs& a, int k, Prefetch& pf) {
    const int64_t g = sc.cb[k];
    const int n = (int)(sc.cb[k + 1] - g);
#pragma unroll
    for (int r = 0; r < kPF; ++r) {
        const int i = threadIdx.x + r * kT;
        if (i < n) {
            const Staged h = a.w.stg[g + i];
            pf.x[r] = h.x;
            pf.y[r] = h.y;
            pf.key[r] = (int)h.key;
            pf.kprev[r] = i ? (int)a.w.stg[g + i - 1].key : -1;
            pf.id[r] = h.id;
        }
    }
}

// Bucket index entries owned by position i of a key-sorted plane of n hits:
// lut[b] = first position whose key bucket is >= b.
template <int kShift, int kN>
__device__ __forceinline__ void lut_entries(uint16_t* lut, int i, int n, int key, int kprev) {
    const int bi = key >> kShift;
    const int bp = kprev < 0 ? -1 : (kprev >> kShift);
    for (int b = bp + 1; b <= bi; ++b) lut[b] = (uint16_t)i;
    if (i == n - 1)
        for (int b = bi + 1; b <= kN; ++b) lut[b] = (uint16_t)n;
}

// Plane k into ring slot k % kRing (LDS tile): hits, used flags and bucket
// index are written by the thread owning each position (one barrier).  A
// coarse bucket index of the plane is kept for the whole event: it serves the
// downstream completion once the plane has left the ring, as do the used flags
// of every plane, which stay in LDS.
template <int kT, int kPF, class S>
__device__ void load_plane_lds(S& st, const FindArgs& a, int k, const Prefetch& pf) {
    Scalars& sc = *st.s;
    const int sl = k % kRing;
    auto* t = st.t;
    const int64_t g = sc.cb[k];
    const int n = (int)(sc.cb[k + 1] - g);
    constexpr int kShift = S::kLutShift, kN = S::kLutN;
    uint16_t* lut = t->lut[sl];
    uint16_t* clut = t->clut[k];
    for (int wd = threadIdx.x; wd < (n + 31) / 32; wd += kT) t->ubits[k][wd] = 0u;
    auto put = [&](int i, float x, float y, int key, int kprev, int id) {
        t->wx[sl][i] = x;
        t->wy[sl][i] = y;
        t->wk[sl][i] = (uint16_t)key;
        t->wid[sl][i] = (uint16_t)id;
        t->claim[i] = kIntMax;
        lut_entries<kShift, kN>(lut, i, n, key, kprev);
        lut_entries<S::kCoarseShift, S::kCoarseN>(clut, i, n, key, kprev);
    };
#pragma unroll
    for (int r = 0; r < kPF; ++r) {
        const int i = threadIdx.x + r * kT;
        if (i < n) put(i, pf.x[r], pf.y[r], pf.key[r], pf.kprev[r], pf.id[r] - (int)g);
    }
    for (int i = threadIdx.x + kPF * kT; i < n; i += kT) {
        const Staged h = a.w.stg[g + i];
        put(i, h.x, h.y, (int)h.key, (int)a.w.stg[g + i - 1].key, (int)(h.id - g));
    }
    if (n == 0)
        for (int b = threadIdx.x; b <= kN; b += kT) lut[b] = 0;
    if (n == 0)
        for (int b = threadIdx.x; b <= S::kCoarseN; b += kT) clut[b] = 0;
    if (threadIdx.x == 0) {
        sc.wg[sl] = g;
        sc.wn[sl] = n;
        sc.wplane[sl] = k;
        sc.n_cand = 0;  // the step's seed and winner counters
        sc.n_acc = 0;
    }
    __syncthreads();
}

// Plane k for the large path: slot bookkeeping, the bucket index, and the
// plane's grid (a counting sort of its hits by cell; the order inside a cell
// is whatever the atomics give -- every search takes a minimum or collects a
// set, so results never depend on it).  The hits stay in global memory.
template <int kT, class S>
__device__ void load_plane_global(S& st, int k) {
    Scalars& sc = *st.s;
    const Work& w = *st.w;
    const int sl = k % kRing;
    __syncthreads();
    const int64_t g = sc.cb[k];
    const int n = (int)(sc.cb[k + 1] - g);
    if (threadIdx.x == 0) {
        sc.wg[sl] = g;
        sc.wn[sl] = n;
        sc.wplane[sl] = k;
        sc.n_cand = 0;  // the step's seed and winner counters
        sc.n_acc = 0;
    }
    int32_t* cs = st.cell + (int64_t)k * (kCells + 1);
    int32_t* fill = st.cell + (int64_t)kPlanes * (kCells + 1);
    for (int c = threadIdx.x; c < kCells; c += kT) {
        cs[c] = 0;
        fill[c] = 0;
    }
    __syncthreads();
    uint16_t* lut = st.lut(sl);
    constexpr int kShift = S::kLutShift, kN = S::kLutN;
    if (n == 0) {
        for (int b = threadIdx.x; b <= kN; b += kT) lut[b] = 0;
    } else {
        for (int i = threadIdx.x; i < n; i += kT) {
            lut_entries<kShift, kN>(lut, i, n, st.K(sl, i), i ? st.K(sl, i - 1) : -1);
            atomicAdd(cs + grid_cell1(w.stg[g + i].y) * kGridN + grid_cell1(w.stg[g + i].x), 1);
        }
    }
    __syncthreads();
    block_excl_scan<kT>(cs, kCells, sc);
    for (int i = threadIdx.x; i < n; i += kT) {
        const float x = w.stg[g + i].x, y = w.stg[g + i].y;
        const int c = grid_cell1(y) * kGridN + grid_cell1(x);
        const int q = cs[c] + atomicAdd(fill + c, 1);
        w.g_gx[g + q] = x;
        w.g_gy[g + q] = y;
        w.g_gpos[g + q] = i;
    }
    __syncthreads();
}

// T1: extend open tracks onto plane k.
template <int kT, class S>
__device__ void forward(S& st, const FindArgs& a, int k) {
    Scalars& sc = *st.s;
    const int sl = k % kRing;
    const int n = sc.wn[sl];
    const int nt = sc.n_tracks;
    const Params& p = a.p;
    int32_t* claim = st.claim(sl);
    for (int t = threadIdx.x; t < nt; t += kT) {
        int want = -1;
        const int kb = st.tkb(t);
        if (n > 0 && kb - k - 1 <= p.max_skip) {
            const float d = sc.z[k] - sc.z[kb];
            const float ex = st.txb(t) + st.ttx(t) * d;
            const float ey = st.tyb(t) + st.tty(t) * d;
            if constexpr (S::kLarge) {
                want = best_hit_grid(a.w, st.cells(k), sc.wg[sl], ex, ey, p);
            } else {
                const uint16_t* lut = st.lut(sl);
                auto key = [&](int i) { return st.K(sl, i); };
                want = best_hit<S::kLutShift>(lut, key, [&](int i) { return st.U(sl, k, i); },
                                              [&](int i) { return st.X(sl, i); }, [&](int i) { return st.Y(sl, i); },
                                              [&](int i) { return st.L(sl, i); }, ex, ey, p);
            }
            if (want >= 0) atomicMin(claim + want, t);
        }
        st.twant(t) = want;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < nt; t += kT) {
        const int i = st.twant(t);
        if (i >= 0 && claim[i] == t) {
            st.set_U(sl, k, i);
            const float xh = st.X(sl, i), yh = st.Y(sl, i);
            const int kb = st.tkb(t);
            const float dz = sc.z[kb] - sc.z[k];
            st.ttx(t) = (st.txb(t) - xh) / dz;
            st.tty(t) = (st.tyb(t) - yh) / dz;
            st.txb(t) = xh;
            st.tyb(t) = yh;
            st.set_tkb(t, k);
            st.tmask(t) |= 1u << k;
            a.w.chits[(st.slot0 + t) * kPlanes + k] = (int32_t)st.ID(sl, i);
        }
    }
    __syncthreads();
    if constexpr (S::kLarge) {
        // the global claim words of a plane serve T3 later: leave them clear
        // (an LDS tile resets its claim words when the next plane is loaded)
        for (int t = threadIdx.x; t < nt; t += kT) {
            const int i = st.twant(t);
            if (i >= 0) claim[i] = kIntMax;
        }
        __syncthreads();
    }
}

// A pass of the seeding of one plane step restricted to a range of candidate
// keys (large-event path).  The key is the claiming order's first part, (q,
// h0's plane-local index), as one 64-bit integer: q >= 0, so its bit pattern
// orders like its value.  mode 1 counts the keys in [lo, hi] into hist (bin =
// (key - lo) >> shift); mode 2 stores the candidates with keys in [lo, hi] from
// pool entry `base` on.
struct SeedRange {
    int mode;
    uint64_t lo, hi;
    int shift;
    uint32_t* hist;
    int base;
};

// T2 candidate enumeration, load-balanced over (h0, h2) pairs: (A) every
// unused h0 gets its azimuth window on plane k+2 (up to two position ranges);
// (B) a block scan of the window sizes; (C) the pairs are dealt out evenly and
// each surviving pair searches plane k+1 for its middle hit.  Returns false
// (uniformly) on candidate overflow.  rg (large-event path only): a pass
// restricted to a key range; null: every candidate, stored from entry 0.
template <int kT, class S>
__device__ bool enumerate_seeds(S& st, const FindArgs& a, int k, const SeedRange* rg = nullptr) {
    Scalars& sc = *st.s;
    const Params& p = a.p;
    const int s0 = k % kRing, s1 = (k + 1) % kRing, s2 = (k + 2) % kRing;
    const int n0 = sc.wn[s0], n1 = sc.wn[s1], n2 = sc.wn[s2];
    if (n0 == 0 || n1 == 0 || n2 == 0) return true;  // sc.n_cand was cleared with the plane load
    const float dz2 = p.z[k + 2] - p.z[k];
    const float dz1 = p.z[k + 1] - p.z[k];
    const int cap = st.cap_cand();
    auto key1 = [&](int i) { return st.K(s1, i); };
    auto key2 = [&](int i) { return st.K(s2, i); };
    const uint16_t* lut1 = st.lut(s1);
    const uint16_t* lut2 = st.lut(s2);
    auto lower2 = [&](int v) { return lower_lut<S::kLutShift>(lut2, key2, n2, v); };
    int32_t* pref = st.pref();        // [n0 + 1]
    int32_t* eb = st.ebuf();          // a0[n0], b0[n0], a1[n0], b1[n0]
    // (A) windows.  An outward line through h0 passing within D of the axis
    // keeps every later point within asin(D/r0) of h0's azimuth: h2 lies in
    // that wedge.
    auto window = [&](int i0) {
        int cnt = 0, ra0 = 0, rb0 = 0, ra1 = 0, rb1 = 0;
        if (!st.U(s0, k, i0)) {
            const float x0 = st.X(s0, i0), y0 = st.Y(s0, i0);
            const int k0 = st.K(s0, i0);
            const float r0 = sqrtf(x0 * x0 + y0 * y0);
            const int mD = disc_keys(p.r_seed, r0);
            int lo[2], hi[2];
            const int nr = mD < 0 ? (lo[0] = 0, hi[0] = 65535, 1) : key_span(k0, k0, mD, lo, hi);
            ra0 = lower2(lo[0]);
            rb0 = lower2(hi[0] + 1);
            if (nr == 2) {
                ra1 = lower2(lo[1]);
                rb1 = lower2(hi[1] + 1);
            }
            cnt = (rb0 - ra0) + (rb1 - ra1);
        }
        eb[i0] = ra0;
        eb[n0 + i0] = rb0;
        eb[2 * n0 + i0] = ra1;
        eb[3 * n0 + i0] = rb1;
        return cnt;
    };
    if (n0 <= kT) {
        // (A + B) one h0 per thread; the window sizes scanned across the
        // workgroup in registers (wave scans + per-wave totals)
        const int cnt = (int)threadIdx.x < n0 ? window(threadIdx.x) : 0;
        int tot;
        const int ex = wave_excl_scan(cnt, &tot);
        const int wv = threadIdx.x / kWave;
        if ((threadIdx.x % kWave) == 0) sc.wsum[wv] = tot;
        __syncthreads();
        int base = 0, total = 0;
        for (int q = 0; q < kT / kWave; ++q) {
            const int v = sc.wsum[q];
            base += q < wv ? v : 0;
            total += v;
        }
        if ((int)threadIdx.x < n0) pref[threadIdx.x] = base + ex;
        if (threadIdx.x == 0) pref[n0] = total;
        if constexpr (!S::kLarge) {
            // (C) below gives thread t the pairs from t * per on; the h0 whose
            // pairs [base + ex, base + ex + cnt) hold that pair tells t so
            static_assert(S::kLarge || 2 * S::kPlaneCap >= kT, "first_h0 fits the seeding slots");
            const int per = (total + kT - 1) / kT;
            int32_t* first = st.first_h0();
            for (int t = (base + ex + per - 1) / max(per, 1); cnt > 0 && t * per < base + ex + cnt; ++t)
                first[t] = threadIdx.x;
        }
        __syncthreads();
    } else {
        for (int i0 = threadIdx.x; i0 < n0; i0 += kT) pref[i0] = window(i0);
        __syncthreads();
        // (B)
        block_excl_scan<kT>(pref, n0, sc);
    }
    const int np = pref[n0];
    // (C) each thread takes a contiguous run of pairs: its first h0 (marked
    // above, or one search), then a forward walk
    const int per = (np + kT - 1) / kT;
    const int pb = min(np, (int)threadIdx.x * per), pe = min(np, pb + per);
    int i0 = 0;
    if (pb < pe) {
        bool known = false;
        if constexpr (!S::kLarge) {
            if (n0 <= kT) {
                i0 = st.first_h0()[threadIdx.x];
                known = true;
            }
        }
        if (!known) {
            int hi = n0;  // last i0 with pref[i0] <= pb
            while (hi - i0 > 1) {
                const int mid = (i0 + hi) >> 1;
                if (pref[mid] <= pb) i0 = mid; else hi = mid;
            }
        }
    }
    int nxt = pref[i0 + 1];
    // h0's pair offset, window bounds and coordinates, read once per run of
    // its pairs (the loop writes only the candidate arrays)
    int cur = -1, pbase = 0, ra0 = 0, rb0 = 0, ra1 = 0;
    float x0 = 0.0f, y0 = 0.0f;
    for (int pi = pb; pi < pe; ++pi) {
        while (pi >= nxt) nxt = pref[++i0 + 1];
        if (i0 != cur) {
            cur = i0;
            pbase = pref[i0];
            ra0 = eb[i0];
            rb0 = eb[n0 + i0];
            ra1 = eb[2 * n0 + i0];
            x0 = st.X(s0, i0);
            y0 = st.Y(s0, i0);
        }
        const int o = pi - pbase;
        const int len0 = rb0 - ra0;
        const int i2 = o < len0 ? ra0 + o : ra1 + (o - len0);
        if (st.U(s2, k + 2, i2)) continue;
        const float tx = (st.X(s2, i2) - x0) / dz2;
        const float ty = (st.Y(s2, i2) - y0) / dz2;
        if (!(fabsf(tx) <= p.t_max && fabsf(ty) <= p.t_max)) continue;
        if (!(x0 * tx + y0 * ty > 0.0f)) continue;
        const float cr = x0 * ty - y0 * tx;
        if (!(cr * cr <= p.d2_max * (tx * tx + ty * ty))) continue;
        const float ex = x0 + tx * dz1;
        const float ey = y0 + ty * dz1;
        auto try_mid = [&](int i1, float x1, float y1, bool used1) {
            if (used1) return;
            const float dx = x1 - ex;
            const float dy = y1 - ey;
            const float q = dx * dx + dy * dy;
            if (!(q <= p.s_max)) return;
            int base = 0;
            if constexpr (S::kLarge) {
                if (rg) {
                    const uint64_t key = ((uint64_t)__float_as_uint(q) << 32) | (uint32_t)st.L(s0, i0);
                    if (key < rg->lo || key > rg->hi) return;
                    if (rg->mode == 1) {
                        atomicAdd(rg->hist + (int)((key - rg->lo) >> rg->shift), 1u);
                        return;
                    }
                    base = rg->base;
                }
            }
            const int c = base + atomicAdd(&sc.n_cand, 1);
            if (c < cap) {
                st.cq(c) = q;
                st.set_cp(c, i0, i1, i2);
                st.calive(c) = 1;
            }
        };
        if constexpr (S::kLarge) {
            // crowded planes: the disc of radius R_mid around the prediction
            const int64_t g1 = sc.wg[s1];
            grid_visit(st.cells(k + 1), ex, ey, p.r_mid,
                       [&](int q1) {
                           const int i1 = a.w.g_gpos[g1 + q1];
                           try_mid(i1, a.w.g_gx[g1 + q1], a.w.g_gy[g1 + q1], st.U(s1, k + 1, i1));
                       });
        } else {
            // the disc of radius R_mid around the predicted middle point
            int lo1[2], hi1[2];
            const int nr1 = point_window(ex, ey, p.r_mid, lo1, hi1);
            auto load1 = [&](int i1) { return PosData{st.X(s1, i1), st.Y(s1, i1), 0, st.U(s1, k + 1, i1)}; };
            visit_lut<S::kLutShift>(lut1, key1, load1, nr1, lo1, hi1,
                                    [&](int i1, const PosData& d) { try_mid(i1, d.x, d.y, d.used); });
        }
    }
    __syncthreads();
    if constexpr (S::kLarge) {
        if (rg) return rg->base + sc.n_cand <= cap;
        if (threadIdx.x == 0 && a.status) atomicMax(a.status + ST_MAXCAND, sc.n_cand);
    }
    return sc.n_cand <= cap;
}

// Synchronisation of a group of kG threads of a kT-thread workgroup: the whole
// workgroup (barrier) or its first wave alone (lockstep lanes: an LDS fence
// orders the accesses, no barrier needed).
template <int kG, int kT>
__device__ __forceinline__ void group_sync() {
    if constexpr (kG == kT) {
        __syncthreads();
    } else {
        static_assert(kG == kWave, "a sub-group is one wave");
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

template <int kG, int kT>
__device__ __forceinline__ bool group_or(int v) {
    if constexpr (kG == kT) {
        return __syncthreads_or(v) != 0;
    } else {
        group_sync<kG, kT>();
        return __ballot(v) != 0ull;
    }
}

// T2 greedy claiming by rounds of local minima; winners end marked 3.
// Candidate states: 1 alive, 2 won this round, 3 settled winner, 0 dead.  Run
// by a group of kG threads (the workgroup, or its first wave when the
// candidates fit it).  Only the slots of hits that some candidate uses are
// read, so only those are cleared.
template <int kG, int kT, class S>
__device__ void claim_rounds(S& st, int k, int c0, int nc) {
    const int s0 = k % kRing, s1 = (k + 1) % kRing, s2 = (k + 2) % kRing;
    uint64_t* A0 = st.slotA(0);
    uint64_t* A1 = st.slotA(1);
    uint64_t* A2 = st.slotA(2);
    uint32_t* B0 = st.slotB(0);
    uint32_t* B1 = st.slotB(1);
    uint32_t* B2 = st.slotB(2);
    for (int c = c0 + threadIdx.x; c < nc; c += kG) {
        const int i0 = st.cp(c, 0), i1 = st.cp(c, 1), i2 = st.cp(c, 2);
        A0[i0] = ~0ull; A1[i1] = ~0ull; A2[i2] = ~0ull;
        B0[i0] = ~0u; B1[i1] = ~0u; B2[i2] = ~0u;
    }
    group_sync<kG, kT>();
    auto keyA = [&](int c) {
        return ((uint64_t)__float_as_uint(st.cq(c)) << 32) | (uint32_t)st.L(s0, st.cp(c, 0));
    };
    auto keyB = [&](int c) {
        return ((uint32_t)st.L(s1, st.cp(c, 1)) << 16) | (uint32_t)st.L(s2, st.cp(c, 2));
    };
    while (true) {
        for (int c = c0 + threadIdx.x; c < nc; c += kG) {
            if (st.calive(c) != 1) continue;
            const uint64_t kA = keyA(c);
            atomicMin((unsigned long long*)(A0 + st.cp(c, 0)), kA);
            atomicMin((unsigned long long*)(A1 + st.cp(c, 1)), kA);
            atomicMin((unsigned long long*)(A2 + st.cp(c, 2)), kA);
        }
        group_sync<kG, kT>();
        // per hit: among the candidates holding the smallest (q, h0) there,
        // the smallest (h1, h2) -- the per-hit minimum of the full key
        for (int c = c0 + threadIdx.x; c < nc; c += kG) {
            if (st.calive(c) != 1) continue;
            const int i0 = st.cp(c, 0), i1 = st.cp(c, 1), i2 = st.cp(c, 2);
            const uint64_t kA = keyA(c);
            const uint32_t kB = keyB(c);
            if (A0[i0] == kA) atomicMin(B0 + i0, kB);
            if (A1[i1] == kA) atomicMin(B1 + i1, kB);
            if (A2[i2] == kA) atomicMin(B2 + i2, kB);
        }
        group_sync<kG, kT>();
        for (int c = c0 + threadIdx.x; c < nc; c += kG) {
            if (st.calive(c) != 1) continue;
            const int i0 = st.cp(c, 0), i1 = st.cp(c, 1), i2 = st.cp(c, 2);
            const uint64_t kA = keyA(c);
            const uint32_t kB = keyB(c);
            if (A0[i0] == kA && A1[i1] == kA && A2[i2] == kA && B0[i0] == kB && B1[i1] == kB && B2[i2] == kB) {
                st.calive(c) = 2;
                st.set_U(s0, k, i0);
                st.set_U(s1, k + 1, i1);
                st.set_U(s2, k + 2, i2);
            }
        }
        group_sync<kG, kT>();
        int any = 0;
        for (int c = c0 + threadIdx.x; c < nc; c += kG) {
            const uint8_t al = st.calive(c);
            if (al != 1 && al != 2) continue;
            const int i0 = st.cp(c, 0), i1 = st.cp(c, 1), i2 = st.cp(c, 2);
            A0[i0] = ~0ull; A1[i1] = ~0ull; A2[i2] = ~0ull;
            B0[i0] = ~0u; B1[i1] = ~0u; B2[i2] = ~0u;
            if (al == 2) {
                st.calive(c) = 3;
            } else if (st.U(s0, k, i0) || st.U(s1, k + 1, i1) || st.U(s2, k + 2, i2)) {
                st.calive(c) = 0;
            } else {
                any = 1;
            }
        }
        if (!group_or<kG, kT>(any)) break;
    }
}

// Claiming of the candidates [c0, c1) (by the first wave alone when they fit it).
template <int kT, class S>
__device__ void claim_seeds(S& st, const FindArgs&, int k, int c0, int c1) {
    if (kT > kWave && c1 - c0 <= kWave) {
        if (threadIdx.x < kWave) claim_rounds<kWave, kT>(st, k, c0, c1);
        __syncthreads();
    } else {
        claim_rounds<kT, kT>(st, k, c0, c1);
    }
}

// One downstream completion step (plane j) of the tracks [t0, t1), by a group
// of kG threads (the workgroup, or its first wave when the tracks fit it).  The
// plane is read through the accessors given (LDS ring or global staging).
// Returns (uniformly over the group) whether any track was still open.
template <int kG, int kT, class S, class SR, class SF, class XF, class YF, class IF>
__device__ bool complete_plane(S& st, const FindArgs& a, int j, int t0, int t1, int n, int32_t* claimT, SR search,
                               SF set_used, XF xf, YF yf, IF idf, int64_t gbase) {
    const Params& p = a.p;
    if constexpr (!S::kLarge) {
        for (int i = threadIdx.x; i < n; i += kG) claimT[i] = kIntMax;
        group_sync<kG, kT>();
    }
    int active = 0;
    for (int t = t0 + threadIdx.x; t < t1; t += kG) {
        int want = -1;
        const int kb = st.dkb(t);
        if (j - kb - 1 <= p.max_skip) {
            active = 1;
            const float d = st.s->z[j] - st.s->z[kb];
            const float ex = st.dxb(t) + st.dtx(t) * d;
            const float ey = st.dyb(t) + st.dty(t) * d;
            if (n > 0) {
                want = search(ex, ey);
                if (want >= 0) atomicMin(claimT + want, t);
            }
        }
        st.twant(t) = want;
    }
    if (!group_or<kG, kT>(active)) return false;
    for (int t = t0 + threadIdx.x; t < t1; t += kG) {
        const int i = st.twant(t);
        if (i >= 0 && claimT[i] == t) {
            set_used(i);
            const float xh = xf(i), yh = yf(i);
            const int kb = st.dkb(t);
            const float dz = st.s->z[kb] - st.s->z[j];
            st.dtx(t) = (st.dxb(t) - xh) / dz;
            st.dty(t) = (st.dyb(t) - yh) / dz;
            st.dxb(t) = xh;
            st.dyb(t) = yh;
            st.set_dkb(t, j);
            st.tmask(t) |= 1u << j;
            a.w.chits[(st.slot0 + t) * kPlanes + j] = (int32_t)(gbase + idf(i));
        }
    }
    group_sync<kG, kT>();
    if constexpr (S::kLarge) {
        for (int t = t0 + threadIdx.x; t < t1; t += kG) {
            const int i = st.twant(t);
            if (i >= 0) claimT[i] = kIntMax;
        }
        group_sync<kG, kT>();
    }
    return true;
}

// Rank the winners by (q, h0) -- unique among winners since they share no hit --
// create their tracks, then T3.  Returns false on track-capacity overflow.
template <int kT, class S>
__device__ bool create_tracks(S& st, const FindArgs& a, int k) {
    Scalars& sc = *st.s;
    const Params& p = a.p;
    const int s0 = k % kRing, s1 = (k + 1) % kRing, s2 = (k + 2) % kRing;
    const int t0 = sc.n_tracks;
    uint64_t* wkey = st.wkey64();
    uint32_t* wc = st.wtmp();
    // sc.n_acc was cleared with the plane load
    for (int c = threadIdx.x; c < sc.n_cand; c += kT) {
        if (st.calive(c) == 3) {
            st.calive(c) = 0;
            wc[atomicAdd(&sc.n_acc, 1)] = (uint32_t)c;
        }
    }
    __syncthreads();
    const int nw = sc.n_acc;
    if (t0 + nw > st.cap_tracks()) return false;
    if (nw == 0) return true;
    for (int i = threadIdx.x; i < nw; i += kT) {
        const int c = (int)wc[i];
        wkey[i] = ((uint64_t)__float_as_uint(st.cq(c)) << 32) | (uint32_t)st.L(s0, st.cp(c, 0));
    }
    __syncthreads();
    st.dbase = t0;  // downstream state overlays the seeding slots from here on
    st.dn = nw;
    for (int i = threadIdx.x; i < nw; i += kT) {
        const int c = (int)wc[i];
        const uint64_t ki = wkey[i];
        int rk = 0;
        for (int j = 0; j < nw; ++j) rk += wkey[j] < ki ? 1 : 0;
        const int t = t0 + rk;
        const int i0 = st.cp(c, 0), i1 = st.cp(c, 1), i2 = st.cp(c, 2);
        const float x0 = st.X(s0, i0), y0 = st.Y(s0, i0);
        const float x1 = st.X(s1, i1), y1 = st.Y(s1, i1);
        const float x2 = st.X(s2, i2), y2 = st.Y(s2, i2);
        // upstream end: b = h0 (plane k), a = h1 (plane k+1)
        const float dzu = p.z[k + 1] - p.z[k];
        st.ttx(t) = (x1 - x0) / dzu;
        st.tty(t) = (y1 - y0) / dzu;
        st.txb(t) = x0;
        st.tyb(t) = y0;
        st.set_tkb(t, k);
        // downstream end: b = h2 (plane k+2), a = h1 (plane k+1)
        const float dzd = p.z[k + 1] - p.z[k + 2];
        st.dtx(t) = (x1 - x2) / dzd;
        st.dty(t) = (y1 - y2) / dzd;
        st.dxb(t) = x2;
        st.dyb(t) = y2;
        st.set_dkb(t, k + 2);
        st.tmask(t) = 7u << k;
        int32_t* ch = a.w.chits + (st.slot0 + t) * kPlanes;
        ch[k] = (int32_t)st.ID(s0, i0);
        ch[k + 1] = (int32_t)st.ID(s1, i1);
        ch[k + 2] = (int32_t)st.ID(s2, i2);
    }
    if (threadIdx.x == 0) sc.n_tracks = t0 + nw;
    __syncthreads();

    // T3: downstream completion of tracks [t0, t0 + nw), planes k+3 .. 25; by
    // the first wave alone when the new tracks fit it (no workgroup barriers)
    auto t3 = [&](auto grp) {
    constexpr int kG = decltype(grp)::value;
    for (int j = k + 3; j < kPlanes; ++j) {
        bool open;
        if (!S::kLarge && j < k + kRing) {
            const int sl = j % kRing;
            const int nj = sc.wn[sl];
            const uint16_t* lut = st.lut(sl);
            auto key = [&](int i) { return st.K(sl, i); };
            auto xf = [&](int i) { return st.X(sl, i); };
            auto yf = [&](int i) { return st.Y(sl, i); };
            auto idf = [&](int i) { return st.L(sl, i); };
            auto search = [&](float ex, float ey) {
                return best_hit<S::kLutShift>(lut, key, [&](int i) { return st.U(sl, j, i); }, xf, yf, idf, ex, ey,
                                              a.p);
            };
            open = complete_plane<kG, kT>(st, a, j, t0, t0 + nw, nj, st.claimT(0), search,
                                          [&](int i) { st.set_U(sl, j, i); }, xf, yf, idf, sc.wg[sl]);
            PCOUNT(5, 1);
        } else {
            const uint64_t tg = PCLOCK();
            const int64_t g = sc.cb[j];
            const Work& w = a.w;
            const int nj = (int)(sc.cb[j + 1] - g);
            auto key = [&](int i) { return (int)w.stg[g + i].key; };
            auto xf = [&](int i) { return w.stg[g + i].x; };
            auto yf = [&](int i) { return w.stg[g + i].y; };
            auto idf = [&](int i) { return (int)(w.stg[g + i].id - g); };
            if constexpr (S::kLarge) {
                auto search = [&](float ex, float ey) { return best_hit_grid(w, st.cells(j), g, ex, ey, a.p); };
                open = complete_plane<kG, kT>(st, a, j, t0, t0 + nw, nj, st.claimT(g), search,
                                              [&](int i) { w.used[g + i] = 1; }, xf, yf, idf, g);
            } else {
                // a plane that has left the ring: hits from global staging through
                // its coarse bucket index, used flags in LDS
                const uint16_t* clut = st.t->clut[j];
                auto search = [&](float ex, float ey) {
                    return best_hit_buckets<S::kCoarseShift>(clut, w.stg + g, [&](int i) { return st.UP(j, i); }, g,
                                                             ex, ey, a.p);
                };
                open = complete_plane<kG, kT>(st, a, j, t0, t0 + nw, nj, st.claimT(g), search,
                                              [&](int i) { st.set_UP(j, i); }, xf, yf, idf, g);
            }
            PCOUNT(6, 1);
            PCOUNT(7, PCLOCK() - tg);
        }
        if (!open) break;
    }
    };
    if (kT > kWave && nw <= kWave) {
        if (threadIdx.x < kWave) t3(std::integral_constant<int, kWave>{});
        __syncthreads();
    } else {
        t3(std::integral_constant<int, kT>{});
    }
    return true;
}

// Seed-level learned filter and training emission, between enumeration and
// claiming.  Features of candidate c (the ten values of the seed filter, FP32,
// each in one fixed order).
template <class S>
__device__ __forceinline__ void seed_features(S& st, const Params& p, int k, int c, const float* fn, float* f,
                                              int* i0, int* i1, int* i2) {
    const int s0 = k % kRing, s1 = (k + 1) % kRing, s2 = (k + 2) % kRing;
    *i0 = st.cp(c, 0);
    *i1 = st.cp(c, 1);
    *i2 = st.cp(c, 2);
    const float dz2 = p.z[k + 2] - p.z[k];
    const float dz1 = p.z[k + 1] - p.z[k];
    const float x0 = st.X(s0, *i0), y0 = st.Y(s0, *i0);
    const float tx = (st.X(s2, *i2) - x0) / dz2;
    const float ty = (st.Y(s2, *i2) - y0) / dz2;
    const float ex = x0 + tx * dz1;
    const float ey = y0 + ty * dz1;
    const float dx = st.X(s1, *i1) - ex;
    const float dy = st.Y(s1, *i1) - ey;
    const float t2 = tx * tx + ty * ty;
    const float rt = x0 * tx + y0 * ty;
    const float cr = x0 * ty - y0 * tx;
    const float r2 = x0 * x0 + y0 * y0;
    float zc = p.z[k] - rt / t2;
    zc = zc < -kSeedZLim ? -kSeedZLim : (zc > kSeedZLim ? kSeedZLim : zc);
    f[0] = dx * dx + dy * dy;
    f[1] = cr * cr / t2;
    f[2] = zc;
    f[3] = r2;
    f[4] = t2;
    f[5] = rt * rt / (r2 * t2);
    f[6] = fn[0];
    f[7] = fn[1];
    f[8] = fn[2];
    f[9] = fn[3];
}

// The network evaluates in FP32 in one fixed order: features standardised as
// (f - mean) * (1 / sd), each unit starts from its bias and adds weight x input
// for inputs in ascending order, ReLU between layers.  Two layouts of the same
// arithmetic: a group of lanes per candidate (each lane holds one or two
// hidden units, their outputs broadcast to the group through LDS), and -- in
// the large-event finder, whose
// crowded plane steps bring thousands of candidates -- one candidate per lane
// with the weights read from an LDS copy as uniform operands.  A candidate
// whose logit exceeds the threshold dies.
template <int kT, class S>
__device__ void seed_filter(S& st, const FindArgs& a, int k, const float* __restrict__ W, int cb0, int nc) {
    Scalars& sc = *st.s;
    const Params& p = a.p;
    const int s0 = k % kRing, s1 = (k + 1) % kRing, s2 = (k + 2) % kRing;
    const float fn[4] = {(float)k, (float)(sc.cb[k + 1] - sc.cb[k]), (float)(sc.cb[k + 2] - sc.cb[k + 1]),
                         (float)(sc.cb[k + 3] - sc.cb[k + 2])};
    const bool on = W != nullptr;
    auto emit = [&](const float* f, int i0, int i1, int i2) {
        const unsigned long long slot = atomicAdd(a.seed_count, 1ull);
        if (slot < (unsigned long long)a.seed_cap) {
            for (int i = 0; i < kSeedIn; ++i) a.seed_feat[slot * kSeedIn + i] = f[i];
            a.seed_hits[slot * 3] = (int32_t)st.ID(s0, i0);
            a.seed_hits[slot * 3 + 1] = (int32_t)st.ID(s1, i1);
            a.seed_hits[slot * 3 + 2] = (int32_t)st.ID(s2, i2);
        }
    };
    bool per_lane = false;
    if constexpr (S::kLarge) per_lane = on && nc - cb0 >= kT / 4;
    if (per_lane) {
        if constexpr (S::kLarge) {
            const float* sw = st.seedw;
            for (int c = cb0 + threadIdx.x; c < nc; c += kT) {
                float f[kSeedIn];
                int i0, i1, i2;
                seed_features(st, p, k, c, fn, f, &i0, &i1, &i2);
                if (a.seed_feat) emit(f, i0, i1, i2);
                float xs[kSeedIn], h1[kSeedH];
                for (int i = 0; i < kSeedIn; ++i) xs[i] = (f[i] - sw[kSeedNorm + i]) * sw[kSeedNorm + kSeedIn + i];
                // first layer through LDS (a rolled loop keeps the registers
                // for the rest of the finder), read back for the second
                float* hs = st.seedh;
#pragma unroll 1
                for (int o = 0; o < kSeedH; ++o) {
                    float h = sw[kSeedB1 + o];
                    for (int i = 0; i < kSeedIn; ++i) h = h + sw[kSeedW1T + o * kSeedIn + i] * xs[i];
                    hs[o * kT + threadIdx.x] = h > 0.0f ? h : 0.0f;
                }
                for (int o = 0; o < kSeedH; ++o) h1[o] = hs[o * kT + threadIdx.x];
                float z = sw[kSeedB3];
#pragma unroll 1
                for (int o = 0; o < kSeedH; ++o) {
                    float h = sw[kSeedB2 + o];
                    for (int i = 0; i < kSeedH; ++i) h = h + sw[kSeedW2T + o * kSeedH + i] * h1[i];
                    z = z + sw[kSeedW3 + o] * (h > 0.0f ? h : 0.0f);
                }
                if (z > sw[kSeedThr]) st.calive(c) = 0;
            }
        }
    } else {
        // a group of kL lanes per candidate, kU hidden units per lane: half
        // a wave (one unit each) for 512-thread workgroups, a quarter (two
        // each) for smaller ones, so that a round always takes 16 candidates
        constexpr int kL = kT >= 512 ? kSeedH : kSeedH / 2;
        constexpr int kU = kSeedH / kL;
        constexpr int kGroups = kT / kL;
        static_assert(kWave % kL == 0, "a candidate's lanes lie in one wave");
        static_assert(kGroups <= 16, "the broadcast scratch holds 16 groups");
        const int l = threadIdx.x & (kL - 1);
        // this group's 32 activations of each layer, broadcast through LDS
        float* b1 = st.bcast() + (threadIdx.x / kL) * kSeedH;
        float* b2 = b1 + kGroups * kSeedH;
        for (int c0 = cb0; c0 < nc; c0 += kGroups) {
            const int c = c0 + (int)threadIdx.x / kL;
            const bool valid = c < nc;
            // idle groups take a valid candidate and still join the broadcasts
            float f[kSeedIn];
            int i0, i1, i2;
            seed_features(st, p, k, valid ? c : nc - 1, fn, f, &i0, &i1, &i2);
            if (a.seed_feat && valid && l == 0) emit(f, i0, i1, i2);
            if (!on) continue;
            // the per-lane weight rows are re-read each round (L1) rather than
            // held in registers across the loop; the uniform ones come
            // through the scalar cache
            const float* Wl = W;
            asm volatile("" : "+s"(Wl));
            typedef const __attribute__((address_space(1))) float* gptr;
            const gptr Wg = (gptr)Wl;
            float xs[kSeedIn];
            for (int i = 0; i < kSeedIn; ++i) xs[i] = (f[i] - W[kSeedNorm + i]) * W[kSeedNorm + kSeedIn + i];
            for (int u = 0; u < kU; ++u) {  // units l * kU + u
                const int o = l * kU + u;
                float h = Wg[kSeedB1 + o];
                for (int i = 0; i < kSeedIn; ++i) h = h + Wg[kSeedW1T + i * kSeedH + o] * xs[i];
                b1[o] = h > 0.0f ? h : 0.0f;
            }
            group_sync<kWave, kT>();
            float h2[kU];
            for (int u = 0; u < kU; ++u) h2[u] = Wg[kSeedB2 + l * kU + u];
            for (int i = 0; i < kSeedH; ++i) {
                const float x = b1[i];
                for (int u = 0; u < kU; ++u) h2[u] = h2[u] + Wg[kSeedW2T + i * kSeedH + l * kU + u] * x;
            }
            for (int u = 0; u < kU; ++u) b2[l * kU + u] = h2[u] > 0.0f ? h2[u] : 0.0f;
            group_sync<kWave, kT>();
            float z = W[kSeedB3];
            for (int i = 0; i < kSeedH; ++i) z = z + W[kSeedW3 + i] * b2[i];
            if (valid && l == 0 && z > W[kSeedThr]) st.calive(c) = 0;
            group_sync<kWave, kT>();  // the next round rewrites b1 and b2
        }
    }
    __syncthreads();
}

// Seeding of a plane step whose candidates exceed the pool (large-event path):
// the candidates are taken in ascending ranges of the key (q, h0), each range
// as large as the pool holds -- a counting pass into a histogram of the keys
// left finds its upper end, a second pass stores it -- and each range is
// claimed before the next is enumerated.  The greedy claiming accepts in key
// order and a candidate with a taken hit is never accepted, so claiming range
// by range, skipping the hits earlier ranges took, accepts exactly what one
// pass over all candidates accepts.  The winners of every range wait in the
// claim words of planes k, k+1, k+2 (idle while plane k seeds: forwarding onto
// plane k is done and downstream completion starts at k+3; at most one winner
// per h0, so they fit), then go to the front of the pool (q, hits; state 3),
// where create_tracks finds them, and the claim words are cleared again.
// Returns false only when more candidates than the pool holds share one key.
constexpr int kRangeBins = 1024;

template <int kT, bool kSeed, class S>
__device__ bool seed_ranges(S& st, const FindArgs& a, int k, const float* __restrict__ seed_net) {
    Scalars& sc = *st.s;
    const int cap = st.cap_cand();
    uint32_t* hist = st.hist;
    int32_t* wq = st.claimT(sc.cb[k]);        // q bits of winner j
    int32_t* wa = st.claimT(sc.cb[k + 1]);    // h0 | h1 << 16 (staged positions)
    int32_t* wb = st.claimT(sc.cb[k + 2]);    // h2
    const uint64_t kmax = ((uint64_t)__float_as_uint(a.p.s_max) << 32) | 0xffffffffull;
    uint64_t lo = 0;
    if (threadIdx.x == 0) sc.n_acc = 0;  // winners so far
    while (true) {
        // upper end of the range: the largest bin boundary whose keys fit the pool
        uint64_t top = kmax, hi = kmax;
        while (true) {
            int shift = 0;
            while (((top - lo) >> shift) >= (uint64_t)kRangeBins) ++shift;
            for (int b = threadIdx.x; b < kRangeBins; b += kT) hist[b] = 0;
            __syncthreads();
            const SeedRange rc{1, lo, top, shift, hist, 0};
            enumerate_seeds<kT>(st, a, k, &rc);
            // inclusive prefix sums over the bins (one thread: 1024 bins, rare path)
            if (threadIdx.x == 0) {
                uint32_t run = 0;
                int last = -1;
                for (int b = 0; b < kRangeBins; ++b) {
                    run += hist[b];
                    if (run <= (uint32_t)cap) last = b;
                }
                sc.wsum[0] = last;
                sc.wsum[1] = run <= (uint32_t)cap ? 1 : 0;
            }
            __syncthreads();
            const int last = sc.wsum[0];
            const bool all = sc.wsum[1] != 0;
            __syncthreads();
            if (all) { hi = top; break; }
            if (last >= 0) { hi = lo + (((uint64_t)(last + 1)) << shift) - 1; break; }
            if (shift == 0) return false;  // one key alone exceeds the pool
            top = lo + ((uint64_t)1 << shift) - 1;  // the first bin: split it finer
        }
        // store and claim the range [lo, hi]
        if (threadIdx.x == 0) sc.n_cand = 0;
        __syncthreads();
        const SeedRange rs{2, lo, hi, 0, nullptr, 0};
        if (!enumerate_seeds<kT>(st, a, k, &rs)) return false;
        const int nc = sc.n_cand;
        if (nc > 0) {
            if constexpr (kSeed) seed_filter<kT>(st, a, k, seed_net, 0, nc);
            claim_seeds<kT>(st, a, k, 0, nc);
            for (int c = threadIdx.x; c < nc; c += kT) {
                if (st.calive(c) != 3) continue;
                const int j = atomicAdd(&sc.n_acc, 1);
                wq[j] = (int32_t)__float_as_uint(st.cq(c));
                wa[j] = st.cp(c, 0) | (st.cp(c, 1) << 16);
                wb[j] = st.cp(c, 2);
            }
            __syncthreads();
        }
        if (hi >= kmax) break;
        lo = hi + 1;
    }
    // the winners to the front of the pool (fewer than its physical size,
    // which is at least 2^16 entries: one winner per h0 at most), claim words clear
    const int nw = sc.n_acc;
    for (int j = threadIdx.x; j < nw; j += kT) {
        const uint32_t va = (uint32_t)wa[j];
        st.cq(j) = __uint_as_float((uint32_t)wq[j]);
        st.set_cp(j, (int)(va & 0xffffu), (int)(va >> 16), wb[j]);
        st.calive(j) = 3;
        wq[j] = kIntMax;
        wa[j] = kIntMax;
        wb[j] = kIntMax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        sc.n_cand = nw;
        sc.n_acc = 0;
    }
    __syncthreads();
    return true;
}

// Whole event.  Returns false when a capacity was too small (LDS tile: redo on
// the large path; large path: overflow); on true the candidates are final.
template <int kT, bool kSeed, class S>
__device__ bool find_event(S& st, const FindArgs& a, int e, const float* __restrict__ seed_net) {
    Scalars& sc = *st.s;
    if (threadIdx.x == 0) {
        sc.n_tracks = 0;
        for (int i = 0; i < kRing; ++i) { sc.wn[i] = 0; sc.wg[i] = 0; }
    }
    for (int k = threadIdx.x; k <= kPlanes; k += kT) {
        sc.cb[k] = a.clu_off[e * kPlanes + k];
        if (k < kPlanes) sc.z[k] = a.p.z[k];
    }
    __syncthreads();
    PHASE_T0();
    // hits per thread prefetched one plane ahead: as many as a full plane of
    // the tile needs, at most two
    constexpr int kPF = S::kLarge ? 1 : ((S::kPlaneCap + kT - 1) / kT > 2 ? 2 : (S::kPlaneCap + kT - 1) / kT);
    Prefetch pf;
    if constexpr (!S::kLarge) prefetch_plane<kT, kPF>(sc, a, kPlanes - 1, pf);
    for (int k = kPlanes - 1; k >= 0; --k) {
        if constexpr (S::kLarge) {
            load_plane_global<kT>(st, k);
        } else {
            load_plane_lds<kT, kPF>(st, a, k, pf);
            PHASE(10);
            if (k > 0) prefetch_plane<kT, kPF>(sc, a, k - 1, pf);
        }
        PHASE(0);
        if (sc.n_tracks > 0) forward<kT>(st, a, k);
        PHASE(1);
        if (k <= kPlanes - 3) {
            st.seed_k = k;
            if (enumerate_seeds<kT>(st, a, k)) {
                PHASE(2);
                if (sc.n_cand > 0) {
                    if constexpr (kSeed) seed_filter<kT>(st, a, k, seed_net, 0, sc.n_cand);
                    claim_seeds<kT>(st, a, k, 0, sc.n_cand);
                    PHASE(3);
                }
            } else if constexpr (S::kLarge) {
                if (!seed_ranges<kT, kSeed>(st, a, k, seed_net)) return false;
            } else {
                return false;  // the larger tile or the large path redoes the event
            }
            if (sc.n_cand > 0) {
                if (!create_tracks<kT>(st, a, k)) return false;
                PHASE(4);
            }
        }
    }
    const int nt = sc.n_tracks;
    PHASE_END();
    if constexpr (!S::kLarge) {
        for (int t = threadIdx.x; t < nt; t += kT) a.w.cmask[st.slot0 + t] = st.tmask(t);
    }
    if (threadIdx.x == 0) a.w.ev_ncand[e] = nt;
    return true;
}

__device__ __forceinline__ void write_empty(const FindArgs& a, int e, int flag) {
    a.w.ev_ncand[e] = 0;
    set_event_flag(a.status, e, flag, 1);
}

// kSeed: the variant with the seed filter / emission (separate code, so that
// the plain finder keeps its register allocation and occupancy).
// seed_net: the seed network (null: none), a separate read-only argument so that
// its uniform weights load through the scalar cache.
// Waves per SIMD the register allocation must allow: four 256-thread
// workgroups of the first tile share a CU (their LDS fits four times), and
// 512-thread ones need four waves per SIMD to run one workgroup per CU.
template <int kT, int kP>
constexpr int find_waves_per_eu() { return kT >= 512 ? 4 : (kT == 256 && kP <= 256 ? 4 : 1); }

template <int kT, int kP, int kTr, int kC, int kLB, int kCB, bool kSeed>
__global__ __launch_bounds__(kT, (find_waves_per_eu<kT, kP>())) void k_find_lds(FindArgs a,
                                                                               const float* __restrict__ seed_net) {
    __shared__ Tile<kP, kTr, kC, kLB, kCB> tile;
    __shared__ Scalars sc;
    LdsStore<kP, kTr, kC, kLB, kCB> st{&tile, &sc, 0};
    while (true) {
        if (threadIdx.x == 0) {
            const int n = a.q_count < 0 ? a.n_events : a.w.counters[a.q_count];
            const int i = atomicAdd(a.w.counters + a.q_cursor, 1);
            sc.event = i < n ? a.q_in[i] : -1;
        }
        __syncthreads();
        const int e = sc.event;
        if (e < 0) return;
        if (a.q_in == a.w.large && threadIdx.x == 0 && a.status) atomicOr(a.status + kStatusHdr + e, EV_TILE2);
        if (a.clu_off[(e + 1) * kPlanes] > a.clu_limit) {  // clusters not (all) available
            if (threadIdx.x == 0) write_empty(a, e, EV_OVERFLOW);
            __syncthreads();
            continue;
        }
        // admission: every plane must fit the tile, and the event must not be
        // so large that it would likely run out of track slots
        int big = 0;
        for (int k = threadIdx.x; k < kPlanes; k += kT)
            big |= (a.clu_off[e * kPlanes + k + 1] - a.clu_off[e * kPlanes + k]) > kP;
        if (threadIdx.x == 0 && a.admit > 0.0f)
            big |= (float)(a.clu_off[(e + 1) * kPlanes] - a.clu_off[e * kPlanes]) > a.admit * (float)kTr;
        big = __syncthreads_or(big);
        bool ok = false;
        if (!big) {
            st.slot0 = a.clu_off[e * kPlanes];
            ok = find_event<kT, kSeed>(st, a, e, seed_net);
        }
        if (!ok && threadIdx.x == 0) {
            const int i = atomicAdd(a.w.counters + a.q_out_count, 1);
            a.q_out[i] = e;
        }
        __syncthreads();
    }
}

template <int kT, bool kSeed>
__global__ __launch_bounds__(kT) void k_find_large(FindArgs a, const float* __restrict__ seed_net) {
    __shared__ Scalars sc;
    __shared__ uint16_t luts[kRing][kLutLarge + 1];
    __shared__ __align__(16) float seedw[kSeed ? kSeedFloats : 1];
    // the seed filter's activations; the key-range seeding's histogram shares
    // the words (it is used only while no filter runs)
    __shared__ __align__(16) float seedh[kSeed ? (kSeedH * kT > kRangeBins ? kSeedH * kT : kRangeBins) : kRangeBins];
    GlobalStore st{&sc, &a.w, 0, (int64_t)blockIdx.x * a.w.pool_cap, 0};
    st.luts = luts;
    st.hist = reinterpret_cast<uint32_t*>(seedh);
    st.seedh = seedh;
    if constexpr (kSeed) {
        // the seed network with its weight matrices back in [unit][input] rows
        if (seed_net) {
            for (int i = threadIdx.x; i < kSeedFloats; i += kT) {
                float v = seed_net[i];
                if (i < kSeedB1) {
                    const int o = i / kSeedIn, j = i % kSeedIn;
                    v = seed_net[kSeedW1T + j * kSeedH + o];
                } else if (i >= kSeedW2T && i < kSeedB2) {
                    const int o = (i - kSeedW2T) / kSeedH, j = (i - kSeedW2T) % kSeedH;
                    v = seed_net[kSeedW2T + j * kSeedH + o];
                }
                seedw[i] = v;
            }
            st.seedw = seedw;
        }
        __syncthreads();
    }
    st.cell = a.w.g_cell + (int64_t)blockIdx.x * kCellWords;
    const int n_large = a.w.counters[a.q_count];
    while (true) {
        if (threadIdx.x == 0) {
            const int i = atomicAdd(a.w.counters + a.q_cursor, 1);
            sc.event = i < n_large ? a.q_in[i] : -1;
        }
        __syncthreads();
        const int e = sc.event;
        if (e < 0) return;
        const int64_t c0 = a.clu_off[e * kPlanes], c1 = a.clu_off[(e + 1) * kPlanes];
        if (c1 > a.clu_limit) {  // clusters not (all) available
            if (threadIdx.x == 0) write_empty(a, e, EV_OVERFLOW);
            __syncthreads();
            continue;
        }
        int too_big = 0;
        for (int k = threadIdx.x; k < kPlanes; k += kT)
            too_big |= (a.clu_off[e * kPlanes + k + 1] - a.clu_off[e * kPlanes + k]) > 65535;
        too_big = __syncthreads_or(too_big);
        if (threadIdx.x == 0 && a.status) {
            atomicAdd(a.status + ST_NLARGE, 1);
            atomicOr(a.status + kStatusHdr + e, EV_LARGE);
        }
        if (too_big) {
            if (threadIdx.x == 0) write_empty(a, e, EV_OVERFLOW);
            __syncthreads();
            continue;
        }
        for (int64_t i = c0 + threadIdx.x; i < c1; i += kT) {
            a.w.used[i] = 0;
            a.w.g_claim[i] = kIntMax;
            a.w.g_slota[i] = ~0ull;
            a.w.g_slotb[i] = ~0u;
            a.w.cmask[i] = 0;
            a.w.g_tkb[i] = 0;
        }
        st.slot0 = c0;
        st.cap_t = (int)((c1 - c0) / 3 + 1);
        __syncthreads();
        const bool ok = find_event<kT, kSeed>(st, a, e, seed_net);
        if (!ok && threadIdx.x == 0) write_empty(a, e, EV_OVERFLOW);
        __syncthreads();
    }
}

// Acceptance of every candidate of an event (one workgroup per event): FP32
// fit, chi2/ndof cut, features for the learned decision, output counts.
__global__ __launch_bounds__(256) void k_accept(FindArgs a) {
    __shared__ int s_out, s_hit, s_all;
    const int e = blockIdx.x;
    if (e >= a.n_events) return;
    if (threadIdx.x == 0) { s_out = 0; s_hit = 0; s_all = 0; }
    __syncthreads();
    const Params& p = a.p;
    const int nt = a.w.ev_ncand[e];
    const int64_t slot0 = a.clu_off[e * kPlanes];
    int my_out = 0, my_hit = 0, my_all = 0;
    for (int t = threadIdx.x; t < nt; t += blockDim.x) {
        const int64_t slot = slot0 + t;
        const uint32_t mask = a.w.cmask[slot];
        const int32_t* ch = a.w.chits + slot * kPlanes;
        const FitResult f = fit_track_hits([&](int k, int) { return ch[k]; }, mask, a.clu_x, a.clu_y, p.z, p.sigma);
        float4* fo = reinterpret_cast<float4*>(a.w.cpar + slot * 8);  // reused by the output step
        fo[0] = make_float4(f.xr, f.yr, f.zr, f.tx);
        fo[1] = make_float4(f.ty, f.chi2, (float)f.ndof, 0.0f);
        const float lim = f.n == 3 ? p.c3 : p.c4;
        const bool plain = f.chi2 / (float)f.ndof <= lim;
        uint8_t fl = plain ? TRK_PLAIN : 0;
        if (p.mode == 1) {
            float raw[10];
            raw_features(f, p.sigma, raw);
            uint16_t fb[16];
            std_features(raw, a.mlp_norm, fb);
            uint4* out = reinterpret_cast<uint4*>(a.w.cfeat + slot * 16);
            const uint4* src = reinterpret_cast<const uint4*>(fb);
            out[0] = src[0];
            out[1] = src[1];
            fl |= TRK_LEARNED;
        } else if (plain) {
            fl |= TRK_ACCEPT;
        }
        a.w.cflags[slot] = fl;
        my_all += f.n;
        my_out += (fl & TRK_ACCEPT) ? 1 : 0;
        my_hit += (fl & TRK_ACCEPT) ? f.n : 0;
    }
    atomicAdd(&s_out, my_out);
    atomicAdd(&s_hit, my_hit);
    atomicAdd(&s_all, my_all);
    __syncthreads();
    if (threadIdx.x == 0) {
        a.w.ev_nout[e] = s_out;
        a.w.ev_nouthit[e] = s_hit;
        a.w.ev_ncandhit[e] = s_all;
    }
}

bool seed_variant(const FindArgs& a) { return a.seed_net != nullptr || a.seed_feat != nullptr; }

template <int kT, int kP, int kTr, int kC, int kLB, int kCB>
hipError_t launch_lds(const FindArgs& a, int grid, hipStream_t s) {
    if (seed_variant(a))
        hipLaunchKernelGGL((k_find_lds<kT, kP, kTr, kC, kLB, kCB, true>), dim3(grid), dim3(kT), 0, s, a, a.seed_net);
    else
        hipLaunchKernelGGL((k_find_lds<kT, kP, kTr, kC, kLB, kCB, false>), dim3(grid), dim3(kT), 0, s, a, nullptr);
    return hipGetLastError();
}

template <int kT, int kP, int kTr, int kC, int kLB, int kCB>
int occ_lds(bool seed) {
    int n = 0;
    const hipError_t e =
        seed ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_find_lds<kT, kP, kTr, kC, kLB, kCB, true>, kT, 0)
             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_find_lds<kT, kP, kTr, kC, kLB, kCB, false>, kT, 0);
    return e == hipSuccess ? n : 1;
}

}  // namespace

// Tile shapes: (plane capacity, tracks, seed candidates per step, key-index
// bits of a ring plane, of the per-event coarse index).  The first tile is
// sized so that four 256-thread workgroups fit a CU's 160 KB of LDS.
#define VELO_TILES(X, T)                   \
    X(T, 0, 256, 304, 336, 7, 5)           \
    X(T, 1, 512, 640, 640, 8, 6)           \
    X(T, 2, 1024, 1024, 1024, 8, 6)

static hipError_t launch_find_lds(const FindArgs& a, int threads, int tile, int grid, hipStream_t s) {
#define VELO_CASE(T, L, P, TR, C, LB, CB) \
    case T * 4 + L: return launch_lds<T, P, TR, C, LB, CB>(a, grid, s);
    switch (threads * 4 + tile) {
        VELO_TILES(VELO_CASE, 64)
        VELO_TILES(VELO_CASE, 128)
        VELO_TILES(VELO_CASE, 256)
        VELO_TILES(VELO_CASE, 512)
        default: return hipErrorInvalidValue;
    }
#undef VELO_CASE
}

int find_blocks_per_cu(int threads, int tile, bool seed) {
#define VELO_CASE(T, L, P, TR, C, LB, CB) \
    case T * 4 + L: return occ_lds<T, P, TR, C, LB, CB>(seed);
    switch (threads * 4 + tile) {
        VELO_TILES(VELO_CASE, 64)
        VELO_TILES(VELO_CASE, 128)
        VELO_TILES(VELO_CASE, 256)
        VELO_TILES(VELO_CASE, 512)
        default: return 1;
    }
#undef VELO_CASE
}

static hipError_t launch_find_large(const FindArgs& a, hipStream_t s) {
    if (seed_variant(a))
        hipLaunchKernelGGL((k_find_large<256, true>), dim3(a.w.n_large_blocks), dim3(256), 0, s, a, a.seed_net);
    else
        hipLaunchKernelGGL((k_find_large<256, false>), dim3(a.w.n_large_blocks), dim3(256), 0, s, a, nullptr);
    return hipGetLastError();
}

int tile_planes(int tile) {
#define VELO_CASE(T, L, P, TR, C, LB, CB) \
    case L: return P;
    switch (tile) {
        VELO_TILES(VELO_CASE, 0)
        default: return 0;
    }
#undef VELO_CASE
}

hipError_t launch_finder_first(FindArgs a, int threads, int tile, int grid, hipStream_t s) {
    a.q_in = a.w.order;
    a.q_count = 6;
    a.q_cursor = 1;
    // events that overflow the tile's track or candidate capacity join the
    // second pass's list (it starts after this pass), or go to global memory
    a.q_out = tile < 2 ? a.w.large : a.w.large2;
    a.q_out_count = tile < 2 ? 2 : 5;
    return launch_find_lds(a, threads, tile, grid, s);
}

hipError_t launch_finder_second(FindArgs a, int tile, int grid, hipStream_t s) {
    a.q_in = a.w.large;
    a.q_count = 2;
    a.q_cursor = 4;
    a.q_out = a.w.large2;
    a.q_out_count = 5;
    return launch_find_lds(a, kSecondPassThreads, tile, grid, s);
}

hipError_t launch_finder_large(FindArgs a, hipStream_t s) {
    a.q_in = a.w.large2;
    a.q_count = 5;
    a.q_cursor = 3;
    return launch_find_large(a, s);
}

#ifdef VELO_PHASE_TIMING
// out: 3 passes x 12 slots (see g_phase), summed over the copies; reset
// clears them afterwards.
extern "C" int velo_probe_phase(unsigned long long* out, int reset) {
    static unsigned long long buf[3][kPhaseCopies][kPhaseSlots];
    if (hipMemcpyFromSymbol(buf, HIP_SYMBOL(g_phase), sizeof(g_phase)) != hipSuccess) return -1;
    for (int p = 0; p < 3; ++p)
        for (int i = 0; i < kPhaseSlots; ++i) {
            unsigned long long t = 0;
            for (int c = 0; c < kPhaseCopies; ++c) t += buf[p][c][i];
            out[p * kPhaseSlots + i] = t;
        }
    if (reset) {
        static const unsigned long long z[3][kPhaseCopies][kPhaseSlots] = {};
        if (hipMemcpyToSymbol(HIP_SYMBOL(g_phase), z, sizeof(z)) != hipSuccess) return -1;
    }
    return 0;
}
#endif

hipError_t launch_accept(const FindArgs& a, hipStream_t s) {
    if (a.n_events <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_accept, dim3(a.n_events), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace velo
