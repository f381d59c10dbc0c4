"""Truth matching of reconstructed tracks against the generator's MC truth.

Evaluation only (host, numpy): it scores outputs, it never produces them.

Definitions (this project's reading; the paper prints no efficiency or ghost
rate for this path):
  * cluster truth = the MC id holding most of the cluster's pixels (tie -> the
    lower id; noise, -1, never beats a real id);
  * an MC track is reconstructible when it is the truth of clusters on >= 3
    distinct planes;
  * a reconstructed track is a ghost unless >= 70 % of its hits carry one MC id
    (exactly 70 % is not a ghost);
  * efficiency = reconstructible MC tracks matched by >= 1 non-ghost track,
    divided by the reconstructible ones; ghost rate = ghosts / tracks; clone
    rate = surplus non-ghost matches / non-ghost tracks.
"""
from __future__ import annotations

import numpy as np

N_PLANES = 26


def cluster_truth(pix_clu, pix_mc, n_clu):
    """MC id per cluster (event-local MC index, -1 noise)."""
    pix_clu = np.asarray(pix_clu, np.int64)
    mc = np.asarray(pix_mc, np.int64)
    if pix_clu.size == 0:
        return np.full(n_clu, -1, np.int64)
    # distinct (cluster, id) pairs with their pixel counts; noise ranks last
    noise_px = mc < 0
    pri = np.where(noise_px, mc.max(initial=0) + 1, mc)
    o = np.lexsort((pri, pix_clu))
    c_s, p_s = pix_clu[o], pri[o]
    new = np.ones(c_s.size, bool)
    new[1:] = (c_s[1:] != c_s[:-1]) | (p_s[1:] != p_s[:-1])
    start = np.flatnonzero(new)
    cnt = np.diff(np.append(start, c_s.size))
    clu, pr, noise = c_s[start], p_s[start], noise_px[o][start]
    # order per cluster: real before noise, more pixels first, lower id first
    order = np.lexsort((pr, -cnt, noise, clu))
    clu_o = clu[order]
    first = np.ones(clu_o.size, bool)
    first[1:] = clu_o[1:] != clu_o[:-1]
    best = order[first]
    truth = np.full(n_clu, -1, np.int64)
    truth[clu[best]] = np.where(noise[best], -1, pr[best])
    return truth


def label_tracks(trk_hit_off, trk_hit, clu_truth, frac=0.7):
    """Per track: (matched MC id or -1, is_ghost).  MC ids are event-local."""
    trk_hit_off = np.asarray(trk_hit_off, np.int64)
    T = trk_hit_off.size - 1
    if T == 0:
        return np.zeros(0, np.int64), np.zeros(0, bool)
    n = np.diff(trk_hit_off)
    tid = np.repeat(np.arange(T), n)
    t = clu_truth[np.asarray(trk_hit, np.int64)]
    real = t >= 0
    key = tid[real] * (np.int64(1) << 32) + t[real]
    u, cnt = np.unique(key, return_counts=True)
    tk = u >> 32
    mk = u & ((np.int64(1) << 32) - 1)
    order = np.lexsort((mk, -cnt, tk))
    tk_o = tk[order]
    first = np.ones(tk_o.size, bool)
    first[1:] = tk_o[1:] != tk_o[:-1]
    best = order[first]
    best_mc = np.full(T, -1, np.int64)
    best_cnt = np.zeros(T, np.int64)
    best_mc[tk[best]] = mk[best]
    best_cnt[tk[best]] = cnt[best]
    # ghost iff best_cnt / n < frac, evaluated exactly in integers: 10*cnt < 7*n
    num, den = int(round(frac * 10)), 10
    ghost = best_cnt * den < num * n
    return np.where(ghost, -1, best_mc), ghost


def eff_ghost(batch, pix_clu, clu_off, trk_off, trk_hit_off, trk_hit):
    """Efficiency, ghost rate and clone rate of a reconstructed batch."""
    E = batch.n_events
    n_clu = int(clu_off[-1])
    truth_local = cluster_truth(pix_clu, batch.pix_mc, n_clu)
    # globalise MC ids by event
    clu_off = np.asarray(clu_off, np.int64)
    clu_ev = np.repeat(np.arange(E), np.diff(clu_off[::N_PLANES]))
    clu_plane = np.repeat(np.tile(np.arange(N_PLANES), E), np.diff(clu_off))
    mc_base = np.asarray(batch.trk_off, np.int64)
    truth = np.where(truth_local >= 0, truth_local + mc_base[clu_ev], -1)
    n_mc = int(batch.trk_off[-1])
    # reconstructible: truth on >= 3 distinct planes
    real = truth >= 0
    pk = np.unique(truth[real] * N_PLANES + clu_plane[real])
    planes_per_mc = np.bincount(pk // N_PLANES, minlength=n_mc)
    recon = planes_per_mc >= 3
    mc, ghost = label_tracks(trk_hit_off, trk_hit, truth)
    T = mc.size
    good = mc >= 0
    matched = np.zeros(n_mc, bool)
    matched[mc[good]] = True
    n_rec = int(recon.sum())
    eff = float((matched & recon).sum()) / n_rec if n_rec else float("nan")
    ghost_rate = float(ghost.sum()) / T if T else 0.0
    n_good = int(good.sum())
    clone = float(n_good - np.unique(mc[good]).size) / n_good if n_good else 0.0
    return dict(efficiency=eff, ghost_rate=ghost_rate, clone_rate=clone, n_tracks=T,
                n_reconstructible=n_rec, n_ghost=int(ghost.sum()))


def candidate_labels(batch, pix_clu, clu_off, trk_hit_off, trk_hit):
    """Training labels for candidates: 1 = ghost (< 70 % of hits from one MC track)."""
    E = batch.n_events
    n_clu = int(clu_off[-1])
    truth_local = cluster_truth(pix_clu, batch.pix_mc, n_clu)
    clu_off = np.asarray(clu_off, np.int64)
    clu_ev = np.repeat(np.arange(E), np.diff(clu_off[::N_PLANES]))
    truth = np.where(truth_local >= 0, truth_local + np.asarray(batch.trk_off, np.int64)[clu_ev], -1)
    _, ghost = label_tracks(trk_hit_off, trk_hit, truth)
    return ghost.astype(np.uint8)
