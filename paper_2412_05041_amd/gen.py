"""Seeded synthetic VELO events: the input generator shared by the HIP path and the oracle.

This module produces inputs only.  It holds none of the method's arithmetic (no
clustering, no track finding, no fit): it draws collisions, propagates straight
tracks through a fixed set of pixel planes and writes the fired pixel ids as
CSR arrays, together with the Monte-Carlo truth needed to score the output.

Physics context from the paper (arXiv 2412.05041):
  * the vertex detector is an array of silicon pixel planes around the
    interaction region (section "Detector");
  * the acceptance is 2 < eta < 5, z points downstream along the beam and y up
    (section "Detector");
  * Run-3 pile-up is mu = 5 (section "Introduction").
Everything else (plane positions, pixel pitch, the hole, cluster shapes, noise,
scattering) is a synthetic stand-in for the paper's LHCb data, which is not
available; the recipe is stated in the workload definitions below.

Layout of a batch (all numpy, host side):
  pix_off  int32 [E*26+1]  CSR offsets per (event, plane)
  pix_id   uint32 [n_pix]  pixel id r*1454+c, strictly ascending within (event, plane)
  pix_mc   int32 [n_pix]   MC track index within the event, -1 for noise
  trk_off  int32 [E+1]     CSR offsets of MC tracks per event
  plus MC track parameters for diagnostics.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

N_PLANES = 26
N_SIDE = 1454            # 80 mm / 55 um = 1454.5 -> 1454 pixels per side
PITCH = 0.055            # mm
HOLE_D2 = 33058          # pixel exists iff (2c-1453)^2 + (2r-1453)^2 >= HOLE_D2 (5 mm radius)
Z_FIRST, Z_LAST = -300.0, 750.0
GEOMETRY_SEED = 0


def plane_z(seed: int = GEOMETRY_SEED) -> np.ndarray:
    """FP32 plane positions: first/last fixed, inner planes at the nominal 42 mm pitch
    with a seeded uniform jitter of +-10 mm (computed in FP64, rounded once)."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(-10.0, 10.0, size=N_PLANES - 2)
    z = np.empty(N_PLANES, np.float64)
    z[0], z[-1] = Z_FIRST, Z_LAST
    z[1:-1] = Z_FIRST + 42.0 * np.arange(1, N_PLANES - 1) + u
    return z.astype(np.float32)


def pixel_exists(c, r):
    c = np.asarray(c, np.int64)
    r = np.asarray(r, np.int64)
    inside = (c >= 0) & (c < N_SIDE) & (r >= 0) & (r < N_SIDE)
    d2 = (2 * c - (N_SIDE - 1)) ** 2 + (2 * r - (N_SIDE - 1)) ** 2
    return inside & (d2 >= HOLE_D2)


def n_existing_pixels() -> int:
    c = np.arange(N_SIDE)
    d = (2 * c - (N_SIDE - 1)) ** 2
    return int((d[:, None] + d[None, :] >= HOLE_D2).sum())


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic workload.  `tracks` selects the multiplicity model."""
    name: str
    n_events: int
    seed: int
    tracks: str                 # "fixed", "pv_poisson", "lognormal", "uniform"
    n_tracks: int = 20          # fixed / lognormal base
    pv_mean: float = 5.0        # pv_poisson
    trk_per_pv: float = 40.0    # pv_poisson
    trk_lo: int = 2000          # uniform
    trk_hi: int = 30000         # uniform
    ln_sigma: float = 0.7       # lognormal occupancy scale
    ln_clip: tuple = (0.2, 5.0)
    ms_sigma: float = 0.0       # rad, slope kick per projection after each plane crossed
    noise_p: float = 0.0        # per-pixel noise probability per plane
    hit_eff: float = 0.98

    def with_events(self, n: int, seed: int | None = None) -> "Workload":
        return dataclasses.replace(self, n_events=n, seed=self.seed if seed is None else seed)


# Noise for the nominal workload: the literal 0.1 %/pixel would give ~56k noise
# pixels per event, which contradicts the stated ~3k clusters/event.  The nominal
# workload instead calibrates p so that the mean cluster count is ~3000 per event
# (signal alone gives ~2.1k); "nominal_literal_noise" keeps the literal figure.
NOMINAL_NOISE_P = 1.6e-5

WORKLOADS = {
    "tiny": Workload("tiny", 100, 1001, "fixed", n_tracks=20),
    "nominal": Workload("nominal", 1000, 1002, "pv_poisson", ms_sigma=1e-3, noise_p=NOMINAL_NOISE_P),
    "nominal_literal_noise": Workload("nominal_literal_noise", 1000, 1002, "pv_poisson",
                                      ms_sigma=1e-3, noise_p=1e-3),
    "uneven": Workload("uneven", 4096, 1003, "lognormal", n_tracks=20),
    "learned_train": Workload("learned_train", 20000, 1004, "fixed", n_tracks=20),
    "learned_test": Workload("learned_test", 5000, 2004, "fixed", n_tracks=20),
    "heavy_ion": Workload("heavy_ion", 128, 1005, "uniform", ms_sigma=1e-3, noise_p=3e-3),
}


@dataclasses.dataclass
class Batch:
    n_events: int
    pix_off: np.ndarray     # int32 [E*26+1]
    pix_id: np.ndarray      # uint32
    pix_mc: np.ndarray      # int32
    trk_off: np.ndarray     # int32 [E+1]  MC tracks per event
    trk_param: np.ndarray   # float64 [T, 5]  vx, vy, vz, tx0, ty0
    plane_z: np.ndarray     # float32 [26]

    @property
    def n_pix(self) -> int:
        return int(self.pix_off[-1])

    def event_slice(self, e0: int, e1: int) -> "Batch":
        """Events [e0, e1) as a batch of their own (offsets rebased)."""
        p0, p1 = int(self.pix_off[e0 * N_PLANES]), int(self.pix_off[e1 * N_PLANES])
        t0, t1 = int(self.trk_off[e0]), int(self.trk_off[e1])
        return Batch(e1 - e0,
                     (self.pix_off[e0 * N_PLANES:e1 * N_PLANES + 1] - p0).astype(np.int32),
                     self.pix_id[p0:p1].copy(), self.pix_mc[p0:p1].copy(),
                     (self.trk_off[e0:e1 + 1] - t0).astype(np.int32),
                     self.trk_param[t0:t1].copy(), self.plane_z)


def _tracks_per_event(w: Workload, rng: np.random.Generator):
    """Per event: number of PVs and tracks per PV (list of arrays)."""
    E = w.n_events
    if w.tracks == "fixed":
        return [np.array([w.n_tracks])] * E
    if w.tracks == "lognormal":
        s = np.clip(rng.lognormal(0.0, w.ln_sigma, size=E), *w.ln_clip)
        n = np.maximum(1, np.rint(w.n_tracks * s).astype(np.int64))
        return [np.array([k]) for k in n]
    if w.tracks == "uniform":
        n = rng.integers(w.trk_lo, w.trk_hi + 1, size=E)
        return [np.array([k]) for k in n]
    if w.tracks == "pv_poisson":
        npv = rng.poisson(w.pv_mean, size=E)
        return [rng.poisson(w.trk_per_pv, size=k) for k in npv]
    raise ValueError(w.tracks)


def _signal_pixels(w, rng, zs, ev_of_trk, vtx, kin):
    """Propagate tracks; return (key, mc) arrays of fired pixels for these tracks.

    key = (event*26 + plane) << 22 | pixel id ; mc = track index within its event.
    """
    T = ev_of_trk.shape[0]
    tx = kin[:, 0].copy()
    ty = kin[:, 1].copy()
    x = vtx[:, 0].copy()
    y = vtx[:, 1].copy()
    zprev = vtx[:, 2].copy()
    keys, mcs = [], []
    mc_local = kin[:, 2].astype(np.int64)
    for k in range(N_PLANES):
        zk = float(zs[k])
        act = zk > zprev  # forward tracks only cross planes downstream of the vertex
        dz = np.where(act, zk - zprev, 0.0)
        x = x + tx * dz
        y = y + ty * dz
        zprev = np.where(act, zk, zprev)
        u = x / PITCH + 727.0
        v = y / PITCH + 727.0
        c = np.floor(u).astype(np.int64)
        r = np.floor(v).astype(np.int64)
        ok = act & pixel_exists(c, r) & (rng.random(T) < w.hit_eff)
        size = rng.integers(1, 4, size=T)
        fu = u - c
        fv = v - r
        idx = np.nonzero(ok)[0]
        cs = [c[idx]]
        rs = [r[idx]]
        ts = [idx]
        i2 = idx[size[idx] >= 2]
        cs.append(c[i2] + np.where(fu[i2] >= 0.5, 1, -1))
        rs.append(r[i2])
        ts.append(i2)
        i3 = idx[size[idx] == 3]
        cs.append(c[i3])
        rs.append(r[i3] + np.where(fv[i3] >= 0.5, 1, -1))
        ts.append(i3)
        cc = np.concatenate(cs)
        rr = np.concatenate(rs)
        tt = np.concatenate(ts)
        keep = pixel_exists(cc, rr)
        cc, rr, tt = cc[keep], rr[keep], tt[keep]
        pid = rr * N_SIDE + cc
        keys.append(((ev_of_trk[tt] * N_PLANES + k) << 22) | pid)
        mcs.append(mc_local[tt])
        if w.ms_sigma > 0.0:  # scattering kick after the plane is crossed
            tx = tx + np.where(act, rng.normal(0.0, w.ms_sigma, size=T), 0.0)
            ty = ty + np.where(act, rng.normal(0.0, w.ms_sigma, size=T), 0.0)
    return np.concatenate(keys), np.concatenate(mcs)


def _noise_pixels(w, rng, e0, e1, n_exist):
    """Binomial(#pixels, p) distinct uniformly drawn existing pixels per (event, plane)."""
    if w.noise_p <= 0.0:
        return np.zeros(0, np.int64)
    ne = (e1 - e0) * N_PLANES
    counts = rng.binomial(n_exist, w.noise_p, size=ne)
    out = []
    total = int(counts.sum())
    if total == 0:
        return np.zeros(0, np.int64)
    seg = np.repeat(np.arange(ne, dtype=np.int64), counts)
    # draw with rejection of hole/duplicates, topping up the shortfall
    want = counts.copy()
    have = np.zeros(ne, np.int64)
    chosen = np.zeros(0, np.int64)
    todo_seg = seg
    while todo_seg.size:
        ids = rng.integers(0, N_SIDE * N_SIDE, size=todo_seg.size)
        ok = pixel_exists(ids % N_SIDE, ids // N_SIDE)
        cand = ((todo_seg + e0 * N_PLANES) << 22) | ids
        cand = cand[ok]
        chosen = np.unique(np.concatenate([chosen, cand]))
        have = np.bincount((chosen >> 22) - e0 * N_PLANES, minlength=ne)
        short = np.maximum(want - have, 0)
        todo_seg = np.repeat(np.arange(ne, dtype=np.int64), short)
    # trim any overshoot per segment (keep the first `want` in id order)
    segs = (chosen >> 22) - e0 * N_PLANES
    start = np.searchsorted(segs, np.arange(ne))
    rank = np.arange(chosen.size) - start[segs]
    out = chosen[rank < want[segs]]
    return out


def generate(w: Workload, max_tracks_per_chunk: int = 300_000) -> Batch:
    """Generate a batch for workload `w` (deterministic in w.seed)."""
    rng = np.random.default_rng(w.seed)
    zs = plane_z()
    E = w.n_events
    per_ev = _tracks_per_event(w, rng)
    n_trk = np.array([int(a.sum()) for a in per_ev], np.int64)
    trk_off = np.zeros(E + 1, np.int64)
    np.cumsum(n_trk, out=trk_off[1:])
    n_exist = n_existing_pixels()

    all_keys, all_mc, params = [], [], []
    e0 = 0
    while e0 < E:
        e1 = e0 + 1
        while e1 < E and trk_off[e1 + 1] - trk_off[e0] <= max_tracks_per_chunk:
            e1 += 1
        T = int(trk_off[e1] - trk_off[e0])
        ev_of_trk = np.repeat(np.arange(e0, e1, dtype=np.int64), n_trk[e0:e1])
        # one vertex per PV, tracks of a PV share it
        vtx = np.empty((T, 3))
        pos = 0
        pv_sizes = np.concatenate([per_ev[e] for e in range(e0, e1)]) if T else np.zeros(0, np.int64)
        npv = pv_sizes.size
        pv = np.column_stack([rng.normal(0, 0.04, npv), rng.normal(0, 0.04, npv), rng.normal(0, 50.0, npv)])
        vtx = np.repeat(pv, pv_sizes, axis=0) if npv else np.zeros((0, 3))
        eta = rng.uniform(2.0, 5.0, T)
        phi = rng.uniform(0.0, 2 * math.pi, T)
        th = 2.0 * np.arctan(np.exp(-eta))
        t = np.tan(th)
        mc_local = np.arange(T) - (trk_off[ev_of_trk] - trk_off[e0])
        kin = np.column_stack([t * np.cos(phi), t * np.sin(phi), mc_local])
        params.append(np.column_stack([vtx, kin[:, :2]]))
        k_sig, m_sig = _signal_pixels(w, rng, zs, ev_of_trk, vtx, kin)
        k_noi = _noise_pixels(w, rng, e0, e1, n_exist)
        all_keys.append(k_sig)
        all_mc.append(m_sig)
        all_keys.append(k_noi)
        all_mc.append(np.full(k_noi.size, -1, np.int64))
        e0 = e1

    keys = np.concatenate(all_keys) if all_keys else np.zeros(0, np.int64)
    mc = np.concatenate(all_mc) if all_mc else np.zeros(0, np.int64)
    # duplicates: a real MC id beats noise; among real ids the lower wins
    pri = np.where(mc < 0, np.int64(1) << 40, mc)
    order = np.lexsort((pri, keys))
    keys, mc = keys[order], mc[order]
    first = np.ones(keys.size, bool)
    first[1:] = keys[1:] != keys[:-1]
    keys, mc = keys[first], mc[first]
    seg = keys >> 22
    pix_off = np.searchsorted(seg, np.arange(E * N_PLANES + 1)).astype(np.int64)
    if pix_off[-1] >= 2**31:
        raise ValueError("batch too large for int32 offsets")
    return Batch(E, pix_off.astype(np.int32), (keys & ((1 << 22) - 1)).astype(np.uint32),
                 mc.astype(np.int32), trk_off.astype(np.int32),
                 np.concatenate(params) if params else np.zeros((0, 5)), zs)


# ---------------------------------------------------------------- raw banks
# A synthetic front-end format (the paper names the persisted "raw banks" but
# gives no format; this one is this project's): per (event, plane) a list of
# 32-bit super-pixel words, each a 2-column x 4-row pixel block --
#   bits  0..7   hit pattern, bit (2 * row_offset + column_offset)
#   bits  8..16  super-pixel row    = row >> 2     (0..363)
#   bits 17..26  super-pixel column = column >> 1  (0..726)
#   bits 27..31  zero
# in arbitrary order within the plane (here: a seeded shuffle).

SP_ROWS = (N_SIDE + 3) // 4
SP_COLS = (N_SIDE + 1) // 2


def raw_banks(b: Batch, seed: int = 0):
    """Encode a batch's pixels as super-pixel words: (bank_off int32 [E*26+1], bank uint32)."""
    rng = np.random.default_rng(seed)
    n_seg = b.n_events * N_PLANES
    seg = np.repeat(np.arange(n_seg, dtype=np.int64), np.diff(b.pix_off.astype(np.int64)))
    ids = b.pix_id.astype(np.int64)
    r, c = ids // N_SIDE, ids % N_SIDE
    spkey = (seg << 20) | ((r >> 2) << 10) | (c >> 1)
    bit = np.left_shift(1, (r & 3) * 2 + (c & 1))
    order = np.argsort(spkey, kind="stable")
    sk, bt = spkey[order], bit[order]
    first = np.ones(sk.size, bool)
    first[1:] = sk[1:] != sk[:-1]
    starts = np.flatnonzero(first)
    keys = sk[starts]
    pattern = np.bitwise_or.reduceat(bt, starts) if starts.size else np.zeros(0, np.int64)
    wseg = keys >> 20
    words = pattern | (((keys >> 10) & 0x3ff) << 8) | ((keys & 0x3ff) << 17)
    shuffle = np.lexsort((rng.random(words.size), wseg))
    words, wseg = words[shuffle], wseg[shuffle]
    bank_off = np.searchsorted(wseg, np.arange(n_seg + 1)).astype(np.int32)
    return bank_off, words.astype(np.uint32)


def hand_event(tracks, plane_list=None, zs=None, noise=()):
    """Build a one-event batch from explicit straight tracks (tests).

    tracks: list of (x0, y0, tx, ty) with x = x0 + tx*z; each hit is a single pixel
    containing the crossing; plane_list optionally restricts the planes per track.
    noise: iterable of (plane, c, r) extra pixels.
    """
    zs = plane_z() if zs is None else zs
    keys, mcs = [], []
    for i, (x0, y0, tx, ty) in enumerate(tracks):
        planes = range(N_PLANES) if plane_list is None or plane_list[i] is None else plane_list[i]
        for k in planes:
            z = float(zs[k])
            c = int(math.floor((x0 + tx * z) / PITCH + 727.0))
            r = int(math.floor((y0 + ty * z) / PITCH + 727.0))
            if pixel_exists(c, r):
                keys.append((k << 22) | (r * N_SIDE + c))
                mcs.append(i)
    for (k, c, r) in noise:
        keys.append((k << 22) | (r * N_SIDE + c))
        mcs.append(-1)
    return from_keys(keys, mcs, len(tracks), zs)


def from_keys(keys, mcs, n_mc, zs=None, n_events=1):
    """Batch from (event*26+plane)<<22|id keys (duplicates resolved as in generate)."""
    zs = plane_z() if zs is None else zs
    keys = np.asarray(keys, np.int64)
    mc = np.asarray(mcs, np.int64)
    pri = np.where(mc < 0, np.int64(1) << 40, mc)
    order = np.lexsort((pri, keys))
    keys, mc = keys[order], mc[order]
    first = np.ones(keys.size, bool)
    first[1:] = keys[1:] != keys[:-1]
    keys, mc = keys[first], mc[first]
    pix_off = np.searchsorted(keys >> 22, np.arange(n_events * N_PLANES + 1)).astype(np.int32)
    n_mc = np.atleast_1d(n_mc)
    trk_off = np.concatenate([[0], np.cumsum(n_mc)]).astype(np.int32)
    return Batch(n_events, pix_off, (keys & ((1 << 22) - 1)).astype(np.uint32), mc.astype(np.int32),
                 trk_off, np.zeros((int(trk_off[-1]), 5)), zs)


def concat(batches) -> Batch:
    """Concatenate batches event-wise."""
    offs, ids, mcs, toffs, params = [np.zeros(1, np.int64)], [], [], [np.zeros(1, np.int64)], []
    p = t = 0
    for b in batches:
        offs.append(b.pix_off[1:].astype(np.int64) + p)
        toffs.append(b.trk_off[1:].astype(np.int64) + t)
        ids.append(b.pix_id)
        mcs.append(b.pix_mc)
        params.append(b.trk_param)
        p += b.n_pix
        t += int(b.trk_off[-1])
    return Batch(sum(b.n_events for b in batches), np.concatenate(offs).astype(np.int32),
                 np.concatenate(ids).astype(np.uint32), np.concatenate(mcs).astype(np.int32),
                 np.concatenate(toffs).astype(np.int32), np.concatenate(params), batches[0].plane_z)
