// velo_oracle.cpp -- plain, slow CPU oracle of the VELO hot path.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
// this file; only the test-suite, the smoke check and the CPU-baseline leg of the
// benchmark do.  It shares no source with the HIP library.
//
// What the paper (arXiv 2412.05041, section "HLT1 details and results") fixes:
//   * the first trigger stage reconstructs vertex-detector track segments with a
//     simplified pattern recognition and fits only the VELO segment;
//   * hits taken by one pass are removed before the next pass runs;
//   * a candidate is kept when it has enough hits and a low enough chi2.
// The paper does not describe the clustering, the seeding, the extension or the
// fit.  The steps below are this project's reading, written out in the plainest
// possible form: connected-component clustering, greedy triplet seeding with hit
// claiming, plane-by-plane extension, a least-squares straight-line fit, and a
// small MLP ghost filter.  Every choice has a strict tie-break so the output is
// unique.
//
// FP rules: IEEE binary32/64, round to nearest even, every expression evaluated
// in the written order, no contraction (built with -ffp-contract=off, SSE math).
//
// Parity pins live in tests/test_oracle_*.py (library routines, closed forms,
// brute force on tiny inputs, invariants).

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

constexpr int kPlanes = 26;
constexpr int kSide = 1454;

// ---------------------------------------------------------------------------
// Clustering: 8-connected components of the fired pixels of one (event, plane).
// Representative = smallest pixel id; clusters are numbered by representative;
// centroid from the integer column/row sums (binary hits, no charge).
// ---------------------------------------------------------------------------

int uf_find(std::vector<int>& p, int a) {
    while (p[a] != a) a = p[a];
    return a;
}

void uf_union(std::vector<int>& p, int a, int b) {
    a = uf_find(p, a);
    b = uf_find(p, b);
    if (a == b) return;
    if (a < b) p[b] = a; else p[a] = b;
}

}  // namespace

extern "C" {

// Clusters every (event, plane) segment of the CSR pixel input.
// pix_off[E*26+1], pix_id[n_pix] ascending within a segment.
// Outputs: pix_clu[n_pix] global cluster index, clu_off[E*26+1],
// clu_x/clu_y/clu_npix[n_clu] (caller sizes them to n_pix).  Returns n_clu.
long long vo_cluster(int n_events, const int32_t* pix_off, const uint32_t* pix_id,
                     int32_t* pix_clu, int32_t* clu_off, float* clu_x, float* clu_y,
                     int32_t* clu_npix) {
    long long n_clu = 0;
    clu_off[0] = 0;
    for (int s = 0; s < n_events * kPlanes; ++s) {
        const int a = pix_off[s], b = pix_off[s + 1], n = b - a;
        const uint32_t* ids = pix_id + a;
        std::vector<int> parent(n);
        for (int i = 0; i < n; ++i) parent[i] = i;
        for (int i = 0; i < n; ++i) {
            const int c = int(ids[i] % kSide), r = int(ids[i] / kSide);
            for (int dr = -1; dr <= 1; ++dr)
                for (int dc = -1; dc <= 1; ++dc) {
                    if (dr == 0 && dc == 0) continue;
                    const int cc = c + dc, rr = r + dr;
                    if (cc < 0 || cc >= kSide || rr < 0 || rr >= kSide) continue;
                    const uint32_t nid = uint32_t(rr) * kSide + uint32_t(cc);
                    const uint32_t* it = std::lower_bound(ids, ids + n, nid);
                    if (it != ids + n && *it == nid) uf_union(parent, i, int(it - ids));
                }
        }
        // representative = smallest index (= smallest id) of each component
        std::vector<int> rep(n, -1);
        for (int i = 0; i < n; ++i) {
            const int root = uf_find(parent, i);
            if (rep[root] < 0 || i < rep[root]) rep[root] = i;
        }
        std::vector<int> reps;
        for (int i = 0; i < n; ++i)
            if (uf_find(parent, i) == i) reps.push_back(rep[i]);
        std::sort(reps.begin(), reps.end());
        std::vector<long long> sc(reps.size(), 0), sr(reps.size(), 0), cnt(reps.size(), 0);
        for (int i = 0; i < n; ++i) {
            const int rp = rep[uf_find(parent, i)];
            const int ord = int(std::lower_bound(reps.begin(), reps.end(), rp) - reps.begin());
            pix_clu[a + i] = int32_t(n_clu + ord);
            sc[ord] += ids[i] % kSide;
            sr[ord] += ids[i] / kSide;
            cnt[ord] += 1;
        }
        for (size_t j = 0; j < reps.size(); ++j) {
            const float fn = float(cnt[j]);
            clu_x[n_clu + j] = (float(sc[j]) / fn - 726.5f) * 0.055f;
            clu_y[n_clu + j] = (float(sr[j]) / fn - 726.5f) * 0.055f;
            if (clu_npix) clu_npix[n_clu + j] = int32_t(cnt[j]);
        }
        n_clu += (long long)reps.size();
        clu_off[s + 1] = int32_t(n_clu);
    }
    return n_clu;
}

// Cut set of the track finder (all FP32 except the integers).
struct vo_cuts {
    float t_max;      // |tx|,|ty| bound of a seed
    float d2_max;     // squared distance of closest approach of a seed line to the z axis
    float s_max;      // squared miss distance of the middle seed hit
    float e_max;      // squared miss distance of an extension hit
    int max_skip;     // planes a track may skip while being extended
    float c3;         // chi2/ndof bound, 3-hit tracks
    float c4;         // chi2/ndof bound, >= 4 hits
    float sigma;      // hit resolution (mm) of the fit
    int mode;         // 0 plain, 1 learned
    float logit_band; // learned: |logit| < band falls back to the plain cut
};

// Seed-level learned filter: a network of the track filter's shape (10 -> 32
// -> 32 -> 1) applied to every seed candidate before the claiming.
struct vo_seed_net {
    const float* w;     // 1441 FP32 weights, the track network's layout
    const float* norm;  // 10 means then 10 standard deviations of the features
    float threshold;    // a candidate whose logit exceeds this is dropped
};

}  // extern "C"

namespace {

// ---------------------------------------------------------------------------
// Straight-line least-squares fit in x-z and y-z, centred at the hit centroid.
// FP32 version (used by the acceptance step) and FP64 version (the reference
// the device fit is compared against).
// ---------------------------------------------------------------------------

template <typename T>
struct FitOut {
    T xr, yr, zr, tx, ty, chi2;
    int ndof;
    T rx[kPlanes], ry[kPlanes];
};

template <typename T>
FitOut<T> ls_fit(int n, const T* x, const T* y, const T* z, T sigma) {
    FitOut<T> f;
    T sz = 0, sx = 0, sy = 0;
    for (int i = 0; i < n; ++i) { sz = sz + z[i]; sx = sx + x[i]; sy = sy + y[i]; }
    const T fn = T(n);
    f.zr = sz / fn;
    f.xr = sx / fn;
    f.yr = sy / fn;
    T szz = 0, szx = 0, szy = 0;
    for (int i = 0; i < n; ++i) {
        const T d = z[i] - f.zr;
        szz = szz + d * d;
        szx = szx + d * (x[i] - f.xr);
        szy = szy + d * (y[i] - f.yr);
    }
    f.tx = szx / szz;
    f.ty = szy / szz;
    T s = 0;
    for (int i = 0; i < n; ++i) {
        const T d = z[i] - f.zr;
        f.rx[i] = (x[i] - f.xr) - f.tx * d;
        f.ry[i] = (y[i] - f.yr) - f.ty * d;
        s = s + (f.rx[i] * f.rx[i] + f.ry[i] * f.ry[i]);
    }
    f.chi2 = s / (sigma * sigma);
    f.ndof = 2 * n - 4;
    return f;
}

// ---------------------------------------------------------------------------
// BF16 helpers and the MLP ghost filter: 10 features -> 32 -> 32 -> 1, ReLU.
// Weights and activations are rounded to BF16 (round to nearest even); sums
// are taken in FP64 here and rounded to FP32 once.
// ---------------------------------------------------------------------------

constexpr int kIn = 10, kH = 32;
constexpr int oW1 = 0, oB1 = oW1 + kH * kIn, oW2 = oB1 + kH, oB2 = oW2 + kH * kH,
              oW3 = oB2 + kH, oB3 = oW3 + kH, kNParam = oB3 + 1;
static_assert(kNParam == 1441, "parameter count");

uint16_t to_bf16(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return uint16_t((u >> 16) | 0x40);  // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}

float from_bf16(uint16_t h) {
    const uint32_t u = uint32_t(h) << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

float rbf(float f, int on) { return on ? from_bf16(to_bf16(f)) : f; }

struct MlpTrace {
    double x[kIn], a1[kH], h1[kH], a2[kH], h2[kH], z;
};

// Forward pass of one sample.  `x` are the (already BF16) standardized features.
void mlp_forward(const float* w, const float* xin, int round_on, MlpTrace& t) {
    for (int i = 0; i < kIn; ++i) t.x[i] = xin[i];
    for (int o = 0; o < kH; ++o) {
        double acc = w[oB1 + o];
        for (int i = 0; i < kIn; ++i) acc += double(rbf(w[oW1 + o * kIn + i], round_on)) * t.x[i];
        t.a1[o] = round_on ? double(float(acc)) : acc;
        t.h1[o] = t.a1[o] > 0 ? t.a1[o] : 0.0;
        if (round_on) t.h1[o] = rbf(float(t.h1[o]), 1);
    }
    for (int o = 0; o < kH; ++o) {
        double acc = w[oB2 + o];
        for (int i = 0; i < kH; ++i) acc += double(rbf(w[oW2 + o * kH + i], round_on)) * t.h1[i];
        t.a2[o] = round_on ? double(float(acc)) : acc;
        t.h2[o] = t.a2[o] > 0 ? t.a2[o] : 0.0;
        if (round_on) t.h2[o] = rbf(float(t.h2[o]), 1);
    }
    double acc = w[oB3];
    for (int i = 0; i < kH; ++i) acc += double(rbf(w[oW3 + i], round_on)) * t.h2[i];
    t.z = round_on ? double(float(acc)) : acc;
}

struct Feat {
    float f[kIn];
};

// The ten candidate features, all FP32, from the FP32 fit of the candidate.
Feat features(int n, const float* x, const float* y, const float* z, int first_plane,
              int last_plane, float sigma) {
    const FitOut<float> f = ls_fit<float>(n, x, y, z, sigma);
    const float s2 = sigma * sigma;
    float mrx = 0.0f, mry = 0.0f;
    for (int i = 0; i < n; ++i) {
        mrx = std::max(mrx, std::fabs(f.rx[i]));
        mry = std::max(mry, std::fabs(f.ry[i]));
    }
    Feat o;
    o.f[0] = f.chi2 / float(f.ndof);
    o.f[1] = float(n);
    o.f[2] = f.tx;
    o.f[3] = f.ty;
    o.f[4] = mrx / sigma;
    o.f[5] = mry / sigma;
    o.f[6] = (f.rx[0] * f.rx[0] + f.ry[0] * f.ry[0]) / s2;
    o.f[7] = (f.rx[n - 1] * f.rx[n - 1] + f.ry[n - 1] * f.ry[n - 1]) / s2;
    o.f[8] = float(first_plane) / 25.0f;
    o.f[9] = float(last_plane) / 25.0f;
    return o;
}

// ---------------------------------------------------------------------------
// Track finding for one event.
// ---------------------------------------------------------------------------

struct Track {
    int hit[kPlanes];  // event-local hit index per plane, -1 if none
};

int first_plane(const Track& t) {
    for (int k = 0; k < kPlanes; ++k) if (t.hit[k] >= 0) return k;
    return -1;
}
int last_plane(const Track& t) {
    for (int k = kPlanes - 1; k >= 0; --k) if (t.hit[k] >= 0) return k;
    return -1;
}
// next plane with a hit strictly above / below k
int plane_above(const Track& t, int k) {
    for (int j = k + 1; j < kPlanes; ++j) if (t.hit[j] >= 0) return j;
    return -1;
}
int plane_below(const Track& t, int k) {
    for (int j = k - 1; j >= 0; --j) if (t.hit[j] >= 0) return j;
    return -1;
}

struct EventIn {
    int base[kPlanes + 1];  // event-local index range of each plane
    const float* x;         // event-local arrays
    const float* y;
    const float* z;         // plane z
};

// Best unused hit on plane k for the prediction (ex, ey): minimum (q, h) with q <= e_max.
int best_hit(const EventIn& ev, const std::vector<char>& used, int k, float ex, float ey,
             float e_max) {
    int bh = -1;
    float bq = 0.0f;
    for (int h = ev.base[k]; h < ev.base[k + 1]; ++h) {
        if (used[h]) continue;
        const float dx = ev.x[h] - ex;
        const float dy = ev.y[h] - ey;
        const float q = dx * dx + dy * dy;
        if (!(q <= e_max)) continue;
        if (bh < 0 || q < bq || (q == bq && h < bh)) { bh = h; bq = q; }
    }
    return bh;
}

// Line through hits a (plane ka) and b (plane kb), evaluated on plane k.
void predict(const EventIn& ev, int a, int ka, int b, int kb, int k, float& ex, float& ey) {
    const float dzab = ev.z[ka] - ev.z[kb];
    const float tx = (ev.x[a] - ev.x[b]) / dzab;
    const float ty = (ev.y[a] - ev.y[b]) / dzab;
    const float d = ev.z[k] - ev.z[kb];
    ex = ev.x[b] + tx * d;
    ey = ev.y[b] + ty * d;
}

struct Seed {
    float q;
    int h0, h1, h2;
};

struct StepStats {
    long long pair_tests = 0, triplet_tests = 0, candidates = 0, rejected = 0;
};

// ---------------------------------------------------------------------------
// Seed-level learned filter (a project extension in the spirit of the paper's
// remark that the first stage simplifies its pattern recognition for
// throughput).  Ten FP32 features of a seed (h0, h1, h2) on planes k, k+1,
// k+2, each written in one fixed order:
//   0  q, the squared miss of h1 from the line through h0 and h2 (the seed cut)
//   1  squared transverse distance of that line from the z axis
//   2  z where the line passes closest to the z axis, clipped to +-2000 mm
//   3  squared radius of h0
//   4  squared slope tx^2 + ty^2
//   5  squared cosine between h0's radial direction and the slope direction
//   6  k;  7, 8, 9  number of clusters on planes k, k+1, k+2
// ---------------------------------------------------------------------------

constexpr float kSeedZLim = 2000.0f;

void seed_features(const EventIn& ev, int k, int h0, int h1, int h2, float* f) {
    const float x0 = ev.x[h0], y0 = ev.y[h0];
    const float dz2 = ev.z[k + 2] - ev.z[k];
    const float dz1 = ev.z[k + 1] - ev.z[k];
    const float tx = (ev.x[h2] - x0) / dz2;
    const float ty = (ev.y[h2] - y0) / dz2;
    const float ex = x0 + tx * dz1;
    const float ey = y0 + ty * dz1;
    const float dx = ev.x[h1] - ex;
    const float dy = ev.y[h1] - ey;
    const float t2 = tx * tx + ty * ty;
    const float rt = x0 * tx + y0 * ty;
    const float cr = x0 * ty - y0 * tx;
    const float r2 = x0 * x0 + y0 * y0;
    float zc = ev.z[k] - rt / t2;
    zc = zc < -kSeedZLim ? -kSeedZLim : (zc > kSeedZLim ? kSeedZLim : zc);
    f[0] = dx * dx + dy * dy;
    f[1] = cr * cr / t2;
    f[2] = zc;
    f[3] = r2;
    f[4] = t2;
    f[5] = rt * rt / (r2 * t2);
    f[6] = float(k);
    f[7] = float(ev.base[k + 1] - ev.base[k]);
    f[8] = float(ev.base[k + 2] - ev.base[k + 1]);
    f[9] = float(ev.base[k + 3] - ev.base[k + 2]);
}

// The seed network in FP32: standardise as (f - mean) * r with r = 1 / sd
// rounded to FP32, then each unit starts from its bias and adds weight x input
// for inputs in ascending order; ReLU between layers.
float seed_logit(const vo_seed_net& sn, const float* f) {
    const float* w = sn.w;
    float xs[kIn], h1[kH], h2[kH];
    for (int i = 0; i < kIn; ++i) {
        const float r = 1.0f / sn.norm[kIn + i];
        xs[i] = (f[i] - sn.norm[i]) * r;
    }
    for (int o = 0; o < kH; ++o) {
        float a = w[oB1 + o];
        for (int i = 0; i < kIn; ++i) a = a + w[oW1 + o * kIn + i] * xs[i];
        h1[o] = a > 0.0f ? a : 0.0f;
    }
    for (int o = 0; o < kH; ++o) {
        float a = w[oB2 + o];
        for (int i = 0; i < kH; ++i) a = a + w[oW2 + o * kH + i] * h1[i];
        h2[o] = a > 0.0f ? a : 0.0f;
    }
    float z = w[oB3];
    for (int i = 0; i < kH; ++i) z = z + w[oW3 + i] * h2[i];
    return z;
}

std::vector<Track> find_event(const EventIn& ev, const vo_cuts& c, const vo_seed_net* sn, StepStats& st,
                              int dbg_step, std::vector<Seed>* dbg_cands) {
    const int n = ev.base[kPlanes];
    std::vector<char> used(n, 0);
    std::vector<Track> tr;
    for (int k = kPlanes - 1; k >= 0; --k) {
        // forwarding of existing tracks onto plane k
        const int nt = int(tr.size());
        std::vector<int> want(nt, -1);
        for (int t = 0; t < nt; ++t) {
            const int kb = first_plane(tr[t]);
            if (kb - k - 1 > c.max_skip) continue;
            const int ka = plane_above(tr[t], kb);
            float ex, ey;
            predict(ev, tr[t].hit[ka], ka, tr[t].hit[kb], kb, k, ex, ey);
            want[t] = best_hit(ev, used, k, ex, ey, c.e_max);
        }
        std::vector<int> owner(n, -1);
        for (int t = 0; t < nt; ++t)
            if (want[t] >= 0 && owner[want[t]] < 0) owner[want[t]] = t;
        for (int t = 0; t < nt; ++t)
            if (want[t] >= 0 && owner[want[t]] == t) { tr[t].hit[k] = want[t]; used[want[t]] = 1; }

        if (k > kPlanes - 3) continue;
        // seeding on planes k, k+1, k+2
        const float dz2 = ev.z[k + 2] - ev.z[k];
        const float dz1 = ev.z[k + 1] - ev.z[k];
        std::vector<Seed> cand;
        for (int h0 = ev.base[k]; h0 < ev.base[k + 1]; ++h0) {
            if (used[h0]) continue;
            const float x0 = ev.x[h0], y0 = ev.y[h0];
            for (int h2 = ev.base[k + 2]; h2 < ev.base[k + 3]; ++h2) {
                if (used[h2]) continue;
                ++st.pair_tests;
                const float tx = (ev.x[h2] - x0) / dz2;
                const float ty = (ev.y[h2] - y0) / dz2;
                if (!(std::fabs(tx) <= c.t_max && std::fabs(ty) <= c.t_max)) continue;
                if (!(x0 * tx + y0 * ty > 0.0f)) continue;
                const float cr = x0 * ty - y0 * tx;
                if (!(cr * cr <= c.d2_max * (tx * tx + ty * ty))) continue;
                const float ex = x0 + tx * dz1;
                const float ey = y0 + ty * dz1;
                for (int h1 = ev.base[k + 1]; h1 < ev.base[k + 2]; ++h1) {
                    if (used[h1]) continue;
                    ++st.triplet_tests;
                    const float dx = ev.x[h1] - ex;
                    const float dy = ev.y[h1] - ey;
                    const float q = dx * dx + dy * dy;
                    if (q <= c.s_max) cand.push_back({q, h0, h1, h2});
                }
            }
        }
        st.candidates += (long long)cand.size();
        if (sn) {
            // the seed filter: drop the candidates the network calls fake
            size_t m = 0;
            for (const Seed& s : cand) {
                float f[kIn];
                seed_features(ev, k, s.h0, s.h1, s.h2, f);
                if (seed_logit(*sn, f) > sn->threshold) ++st.rejected;
                else cand[m++] = s;
            }
            cand.resize(m);
        }
        std::sort(cand.begin(), cand.end(), [](const Seed& a, const Seed& b) {
            if (a.q != b.q) return a.q < b.q;
            if (a.h0 != b.h0) return a.h0 < b.h0;
            if (a.h1 != b.h1) return a.h1 < b.h1;
            return a.h2 < b.h2;
        });
        if (dbg_cands && dbg_step == k) *dbg_cands = cand;
        if (dbg_cands && dbg_step == -2) dbg_cands->insert(dbg_cands->end(), cand.begin(), cand.end());
        const int first_new = int(tr.size());
        for (const Seed& s : cand) {
            if (used[s.h0] || used[s.h1] || used[s.h2]) continue;
            used[s.h0] = used[s.h1] = used[s.h2] = 1;
            Track t;
            for (int j = 0; j < kPlanes; ++j) t.hit[j] = -1;
            t.hit[k] = s.h0;
            t.hit[k + 1] = s.h1;
            t.hit[k + 2] = s.h2;
            tr.push_back(t);
        }
        // downstream completion of the new tracks, plane by plane
        const int last_new = int(tr.size());
        for (int j = k + 3; j < kPlanes; ++j) {
            std::vector<int> w(last_new - first_new, -1);
            for (int t = first_new; t < last_new; ++t) {
                const int kb = last_plane(tr[t]);
                if (j - kb - 1 > c.max_skip) continue;
                const int ka = plane_below(tr[t], kb);
                float ex, ey;
                predict(ev, tr[t].hit[ka], ka, tr[t].hit[kb], kb, j, ex, ey);
                w[t - first_new] = best_hit(ev, used, j, ex, ey, c.e_max);
            }
            std::vector<int> own(n, -1);
            for (int t = first_new; t < last_new; ++t) {
                const int h = w[t - first_new];
                if (h >= 0 && own[h] < 0) own[h] = t;
            }
            for (int t = first_new; t < last_new; ++t) {
                const int h = w[t - first_new];
                if (h >= 0 && own[h] == t) { tr[t].hit[j] = h; used[h] = 1; }
            }
        }
    }
    return tr;
}

// Kalman filter of one projection (x or y) of a straight VELO track whose
// slope receives an independent kick of variance ms2 at every plane it
// crosses (the parameterised multiple-scattering noise), measurements of
// variance sigma2.  pl[0..n) are the hit planes ascending, u[] the measured
// coordinates, zp[] the plane positions.  The filter runs from the most
// downstream hit towards the interaction region and returns the state at the
// most upstream hit: position, slope of the segment just downstream of it,
// their covariance, and the chi2 of the measurements after the first two.
template <typename T>
struct KalState { T x, s, cxx, cxs, css, chi2; };

template <typename T>
KalState<T> kalman_1d(int n, const int* pl, const T* u, const T* zp, T sigma2, T ms2) {
    KalState<T> k{};
    if (n < 2) return k;
    // start at the second most downstream hit b from the two most downstream
    // hits (a, b): slope (u_a - u_b) / D; the kicks on the planes strictly
    // between them move u_a by kick * (z_a - z_q)
    const int a = n - 1, b = n - 2;
    const T D = zp[pl[a]] - zp[pl[b]];
    T g = T(0);
    for (int q = pl[b] + 1; q < pl[a]; ++q) {
        const T w = (zp[pl[a]] - zp[q]) / D;
        g = g + w * w;
    }
    k.x = u[b];
    k.s = (u[a] - u[b]) / D;
    k.cxx = sigma2;
    k.cxs = -sigma2 / D;
    k.css = (sigma2 + sigma2) / (D * D) + ms2 * g;
    k.chi2 = T(0);
    int p = pl[b];
    for (int i = b - 1; i >= 0; --i) {
        // one plane at a time towards the next hit: undo the kick of plane p
        // (the slope below p differs from the one above it by that kick), then
        // carry the position down with that slope
        while (p > pl[i]) {
            const T dz = zp[p] - zp[p - 1];
            k.css = k.css + ms2;
            k.x = k.x - k.s * dz;
            const T cxx = k.cxx - dz * k.cxs - dz * k.cxs + dz * dz * k.css;
            const T cxs = k.cxs - dz * k.css;
            k.cxx = cxx;
            k.cxs = cxs;
            --p;
        }
        // measurement update
        const T r = u[i] - k.x;
        const T S = k.cxx + sigma2;
        const T kx = k.cxx / S, ks = k.cxs / S;
        k.x = k.x + kx * r;
        k.s = k.s + ks * r;
        const T cxx = k.cxx - kx * k.cxx;
        const T cxs = k.cxs - kx * k.cxs;
        const T css = k.css - ks * k.cxs;
        k.cxx = cxx;
        k.cxs = cxs;
        k.css = css;
        k.chi2 = k.chi2 + r * r / S;
    }
    return k;
}

template <typename T>
void kalman_track(int n, const int* pl, const T* x, const T* y, const T* zp, T sigma, T ms, double* o) {
    const T s2 = sigma * sigma, m2 = ms * ms;
    const KalState<T> kx = kalman_1d<T>(n, pl, x, zp, s2, m2);
    const KalState<T> ky = kalman_1d<T>(n, pl, y, zp, s2, m2);
    o[0] = kx.x; o[1] = ky.x; o[2] = kx.s; o[3] = ky.s; o[4] = n > 0 ? zp[pl[0]] : T(0);
    o[5] = kx.cxx; o[6] = kx.cxs; o[7] = kx.css;
    o[8] = ky.cxx; o[9] = ky.cxs; o[10] = ky.css;
    o[11] = kx.chi2 + ky.chi2;
    o[12] = 2 * n - 4;
    o[13] = o[14] = o[15] = 0.0;
}

}  // namespace

extern "C" {

// Decode of super-pixel banks into the CSR pixel input (the synthetic raw-bank
// format: word = pattern[0:8] | sp_row[8:17] | sp_col[17:27], bits 27..31
// zero; pattern bit 2*dr + dc is pixel (4*sp_row + dr, 2*sp_col + dc)).
// A word with a reserved bit set, an empty pattern, or a set bit outside the
// 1454 x 1454 sensor is malformed: it yields no pixel and flags its event (2).
// A pixel id decoded twice is kept (twice) and flags its event (2).  Each
// plane's ids are written sorted ascending.  pix_off[E*26+1]; pix_id holds
// up to pix_cap ids: a plane whose ids would not all fit writes none of them
// and flags its event 1 (the offsets stay complete).  Returns the total pixel
// count.
long long vo_decode(int n_events, const int32_t* bank_off, const uint32_t* bank, int32_t* pix_off,
                    uint32_t* pix_id, long long pix_cap, int32_t* flags) {
    const int n_seg = n_events * kPlanes;
    for (int e = 0; e < n_events; ++e) flags[e] = 0;
    long long total = 0;
    pix_off[0] = 0;
    for (int sgi = 0; sgi < n_seg; ++sgi) {
        const int e = sgi / kPlanes;
        std::vector<uint32_t> ids;
        for (int wi = bank_off[sgi]; wi < bank_off[sgi + 1]; ++wi) {
            const uint32_t w = bank[wi];
            const uint32_t pattern = w & 0xffu, spr = (w >> 8) & 0x1ffu, spc = (w >> 17) & 0x3ffu;
            bool ok = (w >> 27) == 0 && pattern != 0;
            std::vector<uint32_t> mine;
            for (int bit = 0; bit < 8 && ok; ++bit) {
                if (!((pattern >> bit) & 1u)) continue;
                const uint32_t r = 4 * spr + (uint32_t)(bit >> 1), c = 2 * spc + (uint32_t)(bit & 1);
                if (r >= (uint32_t)kSide || c >= (uint32_t)kSide) ok = false;
                else mine.push_back(r * (uint32_t)kSide + c);
            }
            if (!ok) { flags[e] = 2; continue; }
            ids.insert(ids.end(), mine.begin(), mine.end());
        }
        std::sort(ids.begin(), ids.end());
        for (size_t i = 1; i < ids.size(); ++i)
            if (ids[i] == ids[i - 1]) flags[e] = 2;
        if (total + (long long)ids.size() <= pix_cap) {
            for (size_t i = 0; i < ids.size(); ++i) pix_id[total + (long long)i] = ids[i];
        } else if (flags[e] == 0) {
            flags[e] = 1;
        }
        total += (long long)ids.size();
        pix_off[sgi + 1] = (int32_t)total;
    }
    return total;
}

// Kalman fits (x and y projections) of n_tracks CSR tracks, slope noise `ms`
// (rad per plane crossed), measurement error `sigma`.  FP64 or FP32.
// out[t*16 + {0..15}] = x, y, tx, ty, z (state at the most upstream hit),
// Cxx, Cxt, Ctt (x projection), Cyy, Cyt, Ctt (y), chi2, ndof, 0, 0, 0.
void vo_kalman(long long n_tracks, const int32_t* trk_hit_off, const int32_t* trk_hit,
               const uint32_t* trk_planes, const float* clu_x, const float* clu_y,
               const float* plane_z, float sigma, float ms, int fp64, double* out) {
    double zd[kPlanes];
    for (int k = 0; k < kPlanes; ++k) zd[k] = plane_z[k];
    for (long long t = 0; t < n_tracks; ++t) {
        const int a = trk_hit_off[t], n = trk_hit_off[t + 1] - a;
        int pl[kPlanes];
        double xd[kPlanes], yd[kPlanes];
        float xf[kPlanes], yf[kPlanes];
        int i = 0;
        for (int k = 0; k < kPlanes && i < n; ++k) {
            if (!((trk_planes[t] >> k) & 1u)) continue;
            const int h = trk_hit[a + i];
            pl[i] = k;
            xf[i] = clu_x[h]; yf[i] = clu_y[h];
            xd[i] = xf[i]; yd[i] = yf[i];
            ++i;
        }
        if (fp64) kalman_track<double>(n, pl, xd, yd, zd, double(sigma), double(ms), out + 16 * t);
        else kalman_track<float>(n, pl, xf, yf, plane_z, sigma, ms, out + 16 * t);
    }
}

// Straight-line fits of n_tracks CSR tracks.  FP64 (`fp64`=1) or FP32 (`fp64`=0).
// par[t*8 + {0..7}] = x_ref, y_ref, z_ref, tx, ty, chi2, ndof, 0 (as double).
void vo_fit(long long n_tracks, const int32_t* trk_hit_off, const int32_t* trk_hit,
            const uint32_t* trk_planes, const float* clu_x, const float* clu_y,
            const float* plane_z, float sigma, int fp64, double* par) {
    for (long long t = 0; t < n_tracks; ++t) {
        const int a = trk_hit_off[t], n = trk_hit_off[t + 1] - a;
        double xd[kPlanes], yd[kPlanes], zd[kPlanes];
        float xf[kPlanes], yf[kPlanes], zf[kPlanes];
        int i = 0;
        for (int k = 0; k < kPlanes && i < n; ++k) {
            if (!((trk_planes[t] >> k) & 1u)) continue;
            const int h = trk_hit[a + i];
            xf[i] = clu_x[h]; yf[i] = clu_y[h]; zf[i] = plane_z[k];
            xd[i] = xf[i]; yd[i] = yf[i]; zd[i] = zf[i];
            ++i;
        }
        double* p = par + 8 * t;
        if (fp64) {
            const FitOut<double> f = ls_fit<double>(n, xd, yd, zd, double(sigma));
            p[0] = f.xr; p[1] = f.yr; p[2] = f.zr; p[3] = f.tx; p[4] = f.ty; p[5] = f.chi2;
            p[6] = f.ndof;
        } else {
            const FitOut<float> f = ls_fit<float>(n, xf, yf, zf, sigma);
            p[0] = f.xr; p[1] = f.yr; p[2] = f.zr; p[3] = f.tx; p[4] = f.ty; p[5] = f.chi2;
            p[6] = f.ndof;
        }
        p[7] = 0.0;
    }
}

// Learned-filter parameters seen by the oracle's acceptance step.
struct vo_mlp {
    const float* master;  // 1441 FP32 master weights
    const float* norm;    // 10 means then 10 standard deviations
};

// Per-candidate flags
enum { VO_PLAIN_ACCEPT = 1, VO_LEARNED = 2, VO_FALLBACK = 4, VO_ACCEPT = 8 };

// Track finding over all events.  Inputs: cluster CSR (clu_off[E*26+1], clu_x,
// clu_y), plane_z[26].  Outputs (caller-sized: tracks <= n_clu/3+1, hits <= n_clu):
// trk_off[E+1], trk_hit_off[T+1], trk_hit[H] (global cluster index, plane
// ascending), trk_planes[T] bitmask, trk_flags[T], trk_logit[T] (nullable),
// trk_feat[T*10] (nullable, the FP32 features).  emit_rejected=1 outputs every
// candidate.  seed (nullable): the seed-level filter.  stats (nullable): pair
// tests, triplet tests, seed candidates, seeds dropped by the seed filter.
// Returns the number of tracks written.
long long vo_find_tracks(int n_events, const int32_t* clu_off, const float* clu_x,
                         const float* clu_y, const float* plane_z, const vo_cuts* cuts,
                         const vo_mlp* mlp, const vo_seed_net* seed, int emit_rejected, int32_t* trk_off,
                         int32_t* trk_hit_off, int32_t* trk_hit, uint32_t* trk_planes,
                         uint8_t* trk_flags, float* trk_logit, float* trk_feat,
                         long long* stats, int dbg_event, int dbg_step, float* dbg_cand,
                         long long* dbg_ncand) {
    long long T = 0, H = 0;
    trk_off[0] = 0;
    trk_hit_off[0] = 0;
    StepStats st;
    for (int e = 0; e < n_events; ++e) {
        const int g0 = clu_off[e * kPlanes];
        EventIn ev;
        for (int k = 0; k <= kPlanes; ++k) ev.base[k] = clu_off[e * kPlanes + k] - g0;
        ev.x = clu_x + g0;
        ev.y = clu_y + g0;
        ev.z = plane_z;
        std::vector<Seed> dc;
        const bool dbg = dbg_cand && e == dbg_event;  // dbg_step -2: every step's candidates
        std::vector<Track> tr = find_event(ev, *cuts, seed, st, dbg ? dbg_step : -1, dbg ? &dc : nullptr);
        if (dbg) {
            for (size_t i = 0; i < dc.size(); ++i) {
                dbg_cand[4 * i] = dc[i].q;
                dbg_cand[4 * i + 1] = float(dc[i].h0);
                dbg_cand[4 * i + 2] = float(dc[i].h1);
                dbg_cand[4 * i + 3] = float(dc[i].h2);
            }
            *dbg_ncand = (long long)dc.size();
        }
        for (const Track& t : tr) {
            float x[kPlanes], y[kPlanes], z[kPlanes];
            int hs[kPlanes], n = 0;
            uint32_t mask = 0;
            for (int k = 0; k < kPlanes; ++k) {
                if (t.hit[k] < 0) continue;
                x[n] = ev.x[t.hit[k]];
                y[n] = ev.y[t.hit[k]];
                z[n] = plane_z[k];
                hs[n] = t.hit[k];
                mask |= 1u << k;
                ++n;
            }
            const FitOut<float> f = ls_fit<float>(n, x, y, z, cuts->sigma);
            const float lim = n == 3 ? cuts->c3 : cuts->c4;
            const bool plain = f.chi2 / float(f.ndof) <= lim;
            uint8_t flags = plain ? VO_PLAIN_ACCEPT : 0;
            bool acc = plain;
            float logit = 0.0f;
            const Feat ft = features(n, x, y, z, first_plane(t), last_plane(t), cuts->sigma);
            if (cuts->mode == 1 && mlp) {
                float xs[kIn];
                for (int i = 0; i < kIn; ++i)
                    xs[i] = rbf((ft.f[i] - mlp->norm[i]) / mlp->norm[kIn + i], 1);
                MlpTrace tc;
                mlp_forward(mlp->master, xs, 1, tc);
                logit = float(tc.z);
                flags |= VO_LEARNED;
                if (std::isnan(logit) || std::fabs(logit) < cuts->logit_band) {
                    flags |= VO_FALLBACK;
                } else {
                    acc = !(logit > 0.0f);
                }
            }
            if (acc) flags |= VO_ACCEPT;
            if (!acc && !emit_rejected) continue;
            trk_planes[T] = mask;
            trk_flags[T] = flags;
            if (trk_logit) trk_logit[T] = logit;
            if (trk_feat) for (int i = 0; i < kIn; ++i) trk_feat[T * kIn + i] = ft.f[i];
            for (int i = 0; i < n; ++i) trk_hit[H + i] = g0 + hs[i];
            H += n;
            ++T;
            trk_hit_off[T] = int32_t(H);
        }
        trk_off[e + 1] = int32_t(T);
    }
    if (stats) {
        stats[0] = st.pair_tests;
        stats[1] = st.triplet_tests;
        stats[2] = st.candidates;
        stats[3] = st.rejected;
    }
    return T;
}

// Forward extrapolation of VELO states through the magnet (the first step of
// forward tracking in section "HLT1 details and results": a straight line from
// the VELO to the middle of the magnet, the field replaced by a single change
// of slope there, proportional to charge / momentum).  FP64 closed form.
// par[t*8 + {0..4}] = x, y, z, tx, ty of the VELO state (the fit's output);
// x_hit (nullable) = x of a hit at z_t.  out[t*8 + {0..7}] = x, y at z_mag;
// x of the straight line and y at z_t; the x window at z_t holding every track
// with momentum >= p_min (x_lin -+ kick / p_min * (z_t - z_mag)); the q/p that
// leads to x_hit (0 without hits); the slope after the kink for that q/p.
void vo_extrapolate(long long n, const float* par, const float* x_hit, double z_mag, double z_t, double kick,
                    double p_min, double* out) {
    for (long long t = 0; t < n; ++t) {
        const float* p = par + 8 * t;
        const double x0 = p[0], y0 = p[1], z0 = p[2], tx = p[3], ty = p[4];
        const double xm = x0 + tx * (z_mag - z0);
        const double ym = y0 + ty * (z_mag - z0);
        const double lever = z_t - z_mag;
        const double xl = xm + tx * lever;
        const double w = kick / p_min * lever;
        const double qop = x_hit ? ((double(x_hit[t]) - xm) / lever - tx) / kick : 0.0;
        double* o = out + 8 * t;
        o[0] = xm;
        o[1] = ym;
        o[2] = xl;
        o[3] = y0 + ty * (z_t - z0);
        o[4] = xl - w;
        o[5] = xl + w;
        o[6] = qop;
        o[7] = tx + kick * qop;
    }
}

// Seed features of given triplets: hits[n][3] are global cluster indices on
// planes k, k+1, k+2 of one event.  Returns 0, or -1 (nothing written past the
// offending row) when a triplet is not on three consecutive planes of one event.
int vo_seed_features(long long n, const int32_t* hits, int n_events, const int32_t* clu_off,
                     const float* clu_x, const float* clu_y, const float* plane_z, float* feat) {
    const int32_t* end = clu_off + n_events * kPlanes + 1;
    for (long long t = 0; t < n; ++t) {
        const int32_t* h = hits + 3 * t;
        const long long s = (long long)(std::upper_bound(clu_off, end, h[0]) - clu_off) - 1;
        if (s < 0 || s >= (long long)n_events * kPlanes) return -1;
        const int e = int(s / kPlanes), k = int(s % kPlanes);
        if (k > kPlanes - 3) return -1;
        const int32_t* o = clu_off + e * kPlanes;
        if (!(h[1] >= o[k + 1] && h[1] < o[k + 2] && h[2] >= o[k + 2] && h[2] < o[k + 3])) return -1;
        EventIn ev;
        for (int j = 0; j <= kPlanes; ++j) ev.base[j] = o[j] - o[0];
        ev.x = clu_x + o[0];
        ev.y = clu_y + o[0];
        ev.z = plane_z;
        seed_features(ev, k, h[0] - o[0], h[1] - o[0], h[2] - o[0], feat + kIn * t);
    }
    return 0;
}

// Logits of the seed network for given raw features [n][10].
void vo_seed_logit(long long n, const float* feat, const vo_seed_net* sn, float* out) {
    for (long long t = 0; t < n; ++t) out[t] = seed_logit(*sn, feat + kIn * t);
}

// Standardised BF16 features of given FP32 features (row-major [n][10]) -> [n][16].
void vo_standardize(long long n, const float* feat, const float* norm, uint16_t* out) {
    for (long long t = 0; t < n; ++t)
        for (int i = 0; i < 16; ++i)
            out[t * 16 + i] = i < kIn ? to_bf16((feat[t * kIn + i] - norm[i]) / norm[kIn + i]) : 0;
}

// MLP forward of n samples given BF16 inputs [n][16]; round_on=0 gives the
// FP64 network without any BF16 rounding (used for finite-difference checks).
void vo_mlp_forward(long long n, const uint16_t* xb, const float* master, int round_on,
                    double* logit) {
    for (long long t = 0; t < n; ++t) {
        float x[kIn];
        for (int i = 0; i < kIn; ++i) x[i] = from_bf16(xb[t * 16 + i]);
        MlpTrace tc;
        mlp_forward(master, x, round_on, tc);
        logit[t] = tc.z;
    }
}

// Mean binary cross-entropy with logits and its gradient w.r.t. the 1441
// parameters.  Rounding (round_on=1) follows the BF16 forward; derivatives of
// the rounding steps are taken as 1.  With round_on=0 and FP64 inputs
// (xd != nullptr) this is the exact gradient of the unrounded network.
double vo_mlp_loss_grad(long long n, const uint16_t* xb, const double* xd, const uint8_t* label,
                        const float* master, const double* master_d, int round_on,
                        double* grad) {
    for (int i = 0; i < kNParam; ++i) grad[i] = 0.0;
    std::vector<double> wd(kNParam);
    for (int i = 0; i < kNParam; ++i)
        wd[i] = master_d ? master_d[i] : double(rbf(master[i], round_on));
    // biases are never rounded
    for (int i = 0; i < kH; ++i) {
        wd[oB1 + i] = master_d ? master_d[oB1 + i] : master[oB1 + i];
        wd[oB2 + i] = master_d ? master_d[oB2 + i] : master[oB2 + i];
    }
    wd[oB3] = master_d ? master_d[oB3] : master[oB3];
    double loss = 0.0;
    const double inv = 1.0 / double(n);
    for (long long t = 0; t < n; ++t) {
        double x[kIn], a1[kH], h1[kH], a2[kH], h2[kH];
        for (int i = 0; i < kIn; ++i) x[i] = xd ? xd[t * kIn + i] : from_bf16(xb[t * 16 + i]);
        for (int o = 0; o < kH; ++o) {
            double acc = wd[oB1 + o];
            for (int i = 0; i < kIn; ++i) acc += wd[oW1 + o * kIn + i] * x[i];
            a1[o] = round_on ? double(float(acc)) : acc;
            h1[o] = a1[o] > 0 ? a1[o] : 0.0;
            if (round_on) h1[o] = rbf(float(h1[o]), 1);
        }
        for (int o = 0; o < kH; ++o) {
            double acc = wd[oB2 + o];
            for (int i = 0; i < kH; ++i) acc += wd[oW2 + o * kH + i] * h1[i];
            a2[o] = round_on ? double(float(acc)) : acc;
            h2[o] = a2[o] > 0 ? a2[o] : 0.0;
            if (round_on) h2[o] = rbf(float(h2[o]), 1);
        }
        double z = wd[oB3];
        for (int i = 0; i < kH; ++i) z += wd[oW3 + i] * h2[i];
        if (round_on) z = double(float(z));
        const double y = label[t] ? 1.0 : 0.0;
        // softplus(z) - y*z, evaluated stably
        loss += (z > 0 ? z : 0.0) + std::log1p(std::exp(-std::fabs(z))) - y * z;
        const double gz = (1.0 / (1.0 + std::exp(-z)) - y) * inv;
        grad[oB3] += gz;
        double ga2[kH];
        for (int i = 0; i < kH; ++i) {
            grad[oW3 + i] += gz * h2[i];
            ga2[i] = a2[i] > 0 ? gz * wd[oW3 + i] : 0.0;
        }
        double ga1[kH];
        for (int i = 0; i < kH; ++i) ga1[i] = 0.0;
        for (int o = 0; o < kH; ++o) {
            grad[oB2 + o] += ga2[o];
            for (int i = 0; i < kH; ++i) {
                grad[oW2 + o * kH + i] += ga2[o] * h1[i];
                ga1[i] += wd[oW2 + o * kH + i] * ga2[o];
            }
        }
        for (int o = 0; o < kH; ++o) {
            const double g = a1[o] > 0 ? ga1[o] : 0.0;
            grad[oB1 + o] += g;
            for (int i = 0; i < kIn; ++i) grad[oW1 + o * kIn + i] += g * x[i];
        }
    }
    return loss * inv;
}

// One Adam step on FP64 state (bias-corrected, step counted from 1).
void vo_adam(int n, double* w, double* m, double* v, const double* g, int step, double lr,
             double b1, double b2, double eps) {
    const double c1 = 1.0 - std::pow(b1, step), c2 = 1.0 - std::pow(b2, step);
    for (int i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        w[i] -= lr * (m[i] / c1) / (std::sqrt(v[i] / c2) + eps);
    }
}

uint16_t vo_to_bf16(float f) { return to_bf16(f); }

}  // extern "C"
