"""Seed-level learned filter: seed collection, labels, evaluation.

The finder emits every seed candidate that passes the seed cuts (its ten FP32
features and its three cluster indices, velo_seed_emit); a seed is genuine
(label 0) when its three clusters carry the same MC particle, fake (label 1)
otherwise.  The network has the track filter's shape and is trained by the same
BF16 MFMA kernels (velo_mlp_train_step); the finder then evaluates it in FP32
with BF16-rounded weights and drops seeds whose logit exceeds a threshold.
Everything numeric runs in libvelo's kernels; this module moves data and keeps
score.
"""
from __future__ import annotations

import os
import time

import numpy as np
import torch

from . import gen, metrics, velo

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "configs", "seed_default.npz")


def bf16_round(w: np.ndarray) -> np.ndarray:
    """FP32 values rounded to the nearest BF16 (ties to even), as FP32."""
    return torch.from_numpy(np.ascontiguousarray(w, np.float32)).to(torch.bfloat16).float().numpy()


def load_default():
    """(weights, norm, threshold) of the committed seed network."""
    d = np.load(WEIGHTS, allow_pickle=False)
    return d["weights"].astype(np.float32), d["norm"].astype(np.float32), float(d["threshold"])


def labels(batch: gen.Batch, pix_clu: np.ndarray, clu_off: np.ndarray, hits: np.ndarray) -> np.ndarray:
    """1 = fake seed (its clusters do not all carry one MC particle)."""
    n_clu = int(clu_off[-1])
    mc = metrics.cluster_truth(pix_clu, batch.pix_mc, n_clu)
    m0, m1, m2 = mc[hits[:, 0]], mc[hits[:, 1]], mc[hits[:, 2]]
    return (~((m0 >= 0) & (m0 == m1) & (m0 == m2))).astype(np.uint8)


def collect(v: velo.Velo, batch: gen.Batch, cap: int):
    """Raw features, fake labels and cluster triplets of every seed candidate of
    the plain finder on a batch."""
    off, ids = velo.to_device(batch)
    v.reserve(batch.n_events, batch.n_pix, batch.n_pix)
    c = v.cluster(off, ids, with_npix=False)
    n_clu = int(c["clu_off"][-1].item())
    buf = v.seed_emit(cap)
    try:
        v.find_tracks(c["clu_off"], c["clu_x"], c["clu_y"], n_clu=n_clu)
        torch.cuda.synchronize()
    finally:
        v.seed_emit(0)
    m = min(int(buf["count"][0].item()), cap)
    hits = buf["hits"][:m].cpu().numpy().astype(np.int64)
    raw = buf["feat"][:m].cpu().numpy()
    lab = labels(batch, c["pix_clu"][:batch.n_pix].cpu().numpy(), c["clu_off"].cpu().numpy(), hits)
    return raw, lab, hits


def reconstruct(v: velo.Velo, batch: gen.Batch, cut: dict, net=None, reps: int = 0):
    """Efficiency / ghost / clone rates of the pipeline with the seed filter
    `net` = (weights, norm, threshold) or without it (None); with reps > 0 also
    events/s over that many graph replays."""
    v.set_cuts(cut)
    if net is None:
        v.seed_filter_set(None)
    else:
        v.seed_filter_set(*net)
    off, ids = velo.to_device(batch)
    v.reserve(batch.n_events, batch.n_pix, batch.n_pix)
    bufs = v.pipeline_buffers(batch.n_events, batch.n_pix)
    v.pipeline(off, ids, bufs)
    st = v.read_status(bufs["status"])
    T, H = int(st[2]), int(st[3])
    m = metrics.eff_ghost(batch, bufs["pix_clu"][:batch.n_pix].cpu().numpy(), bufs["clu_off"].cpu().numpy(),
                          bufs["trk_off"].cpu().numpy(), bufs["trk_hit_off"][:T + 1].cpu().numpy(),
                          bufs["trk_hit"][:H].cpu().numpy())
    m["severity"] = int(st[0])
    if reps > 0:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            v.pipeline(off, ids, bufs)
        torch.cuda.synchronize()
        m["events_per_s"] = reps * batch.n_events / (time.perf_counter() - t0)
    v.seed_filter_set(None)
    return m
