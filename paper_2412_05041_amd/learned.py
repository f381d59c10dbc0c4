"""Learned ghost filter: dataset collection, on-GPU training and evaluation.

Everything numeric runs in libvelo's kernels (candidate finding, features, MLP
forward/backward, Adam); this module only moves data and keeps score.

Workloads: (1) the learned-filter configuration, candidates from the
single-vertex generator (20 straight tracks per event, no scattering, no
noise) found with loose windows (x3 on the default distances); (2) candidates
of the nominal generator (pile-up, 1 mrad scattering, noise) found with the
scattering cut set, ~0.6 % of them ghosts, ghosts weighted 4:1 in the loss.
Every candidate is emitted with or without the chi2 cut; label 1 = ghost (< 70
% of the hits from one MC track).  The network (10 -> 32 -> 32 -> 1, BF16
weights/activations, FP32 accumulation) is trained with Adam on batches of
65536 candidates and compared with the plain chi2 cut on the same candidates
of independent test events.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np
import torch

from . import gen, metrics, velo

HERE = os.path.dirname(os.path.abspath(__file__))
CFG = os.path.join(HERE, "configs")
WEIGHTS = os.path.join(CFG, "mlp_default.npz")
# the network trained on candidates of the nominal generator (pile-up,
# scattering, noise; the scattering cut set), ghosts weighted 4:1
NOMINAL_WEIGHTS = os.path.join(CFG, "mlp_nominal.npz")
DEFAULT_BAND = math.log(0.6 / 0.4)  # |sigmoid(z) - 0.5| < 0.1  <=>  |z| < ln(0.6/0.4)
N_PARAM = 1441
BATCH = 65536


def cuts(name: str) -> dict:
    return json.load(open(os.path.join(CFG, f"cuts_{name}.json")))


def he_uniform(seed: int = 1004) -> np.ndarray:
    """He-uniform initial weights (biases zero) in the master layout."""
    rng = np.random.default_rng(seed)
    w = np.zeros(N_PARAM, np.float32)
    w[0:320] = rng.uniform(-1, 1, 320) * math.sqrt(6.0 / 10)
    w[352:1376] = rng.uniform(-1, 1, 1024) * math.sqrt(6.0 / 32)
    w[1408:1440] = rng.uniform(-1, 1, 32) * math.sqrt(6.0 / 32)
    return w


def load_default_weights(path: str = WEIGHTS):
    d = np.load(path, allow_pickle=False)
    return d["master"].astype(np.float32), d["norm"].astype(np.float32)


def candidates(v: velo.Velo, batch: gen.Batch, with_labels=True):
    """All track candidates of a batch (emit_rejected) with raw FP32 features,
    plain-cut decisions and (optionally) ghost labels."""
    off, ids = velo.to_device(batch)
    c = v.cluster(off, ids, with_npix=False)
    n_clu = int(c["clu_off"][-1].item())
    t = v.find_tracks(c["clu_off"], c["clu_x"], c["clu_y"], n_clu=n_clu, emit_rejected=True)
    T = int(t["trk_off"][-1].item())
    raw = v.features(t["trk_hit_off"], t["trk_hit"], t["trk_planes"], c["clu_x"], c["clu_y"], T, raw=True,
                     standardised=False)
    out = dict(raw=raw[:T].cpu().numpy(), plain=(t["trk_flags"][:T].cpu().numpy() & velo.TRK_PLAIN_ACCEPT) != 0)
    if with_labels:
        H = int(t["trk_hit_off"][T].item())
        out["label"] = metrics.candidate_labels(batch, c["pix_clu"][:batch.n_pix].cpu().numpy(),
                                                c["clu_off"].cpu().numpy(), t["trk_hit_off"][:T + 1].cpu().numpy(),
                                                t["trk_hit"][:H].cpu().numpy())
    return out


def collect(v: velo.Velo, workload: gen.Workload, n_target: int, chunk_events: int = 20000, log=None):
    """Candidates from successive generator batches until n_target are collected."""
    raws, labs, plains = [], [], []
    n, i = 0, 0
    while n < n_target:
        b = gen.generate(workload.with_events(chunk_events, workload.seed + 7919 * i))
        v.reserve(b.n_events, b.n_pix, b.n_pix)
        d = candidates(v, b)
        raws.append(d["raw"])
        labs.append(d["label"])
        plains.append(d["plain"])
        n += len(d["label"])
        i += 1
        if log:
            log(f"chunk {i}: {n} candidates")
    return np.concatenate(raws)[:n_target], np.concatenate(labs)[:n_target], np.concatenate(plains)[:n_target]


def normalisation(raw: np.ndarray) -> np.ndarray:
    mu = raw.mean(0)
    sd = raw.std(0)
    sd = np.where(sd > 1e-6, sd, 1.0)
    return np.concatenate([mu, sd]).astype(np.float32)


def standardise(v: velo.Velo, raw: np.ndarray) -> torch.Tensor:
    """BF16 standardised features (library rule) of raw FP32 features."""
    t = torch.from_numpy(np.ascontiguousarray(raw, np.float32)).to(v.device)
    return v.standardize(t, raw.shape[0])


def train(v: velo.Velo, feat: torch.Tensor, label: torch.Tensor, epochs: int, lr: float = 1e-3,
          batch: int = BATCH, log=None):
    """Adam on the FP32 master weights held by the context; returns the epoch losses."""
    n = feat.shape[0]
    losses = []
    loss = torch.zeros(1, dtype=torch.float32, device=v.device)
    for ep in range(epochs):
        tot, cnt = 0.0, 0
        for s0 in range(0, n - batch + 1, batch):
            v.mlp_train_step(feat[s0:s0 + batch], label[s0:s0 + batch], lr, n=batch, loss=loss)
            tot += float(loss.item())
            cnt += 1
        losses.append(tot / max(cnt, 1))
        if log:
            log(f"epoch {ep}: loss {losses[-1]:.5f}")
    return losses


def evaluate(v: velo.Velo, batch: gen.Batch, base_cuts: dict, band: float):
    """Efficiency / ghost rate of the plain cut and of the learned filter on the
    same candidates (pipeline outputs in both modes)."""
    res = {}
    off, ids = velo.to_device(batch)
    v.reserve(batch.n_events, batch.n_pix, batch.n_pix)
    for mode in ("plain", "learned"):
        v.set_cuts(dict(base_cuts, mode=0 if mode == "plain" else 1, logit_band=band))
        bufs = v.pipeline_buffers(batch.n_events, batch.n_pix)
        v.pipeline(off, ids, bufs)
        st = v.read_status(bufs["status"])
        T, H = int(st[2]), int(st[3])
        m = metrics.eff_ghost(batch, bufs["pix_clu"][:batch.n_pix].cpu().numpy(), bufs["clu_off"].cpu().numpy(),
                              bufs["trk_off"].cpu().numpy(), bufs["trk_hit_off"][:T + 1].cpu().numpy(),
                              bufs["trk_hit"][:H].cpu().numpy())
        m["fallback_tracks"] = int(st[6])
        res[mode] = m
    v.set_cuts(dict(base_cuts, mode=0))
    return res
