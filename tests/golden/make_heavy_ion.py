"""Writes the oracle's result on one heavy-ion-like event as a golden file.

The oracle needs minutes to an hour for an event of this size, so its result is
stored: SHA-256 digests of every output array (the GPU tests recompute them
from the device outputs), the counts, and the FP64 fit of a sample of the
tracks.  Only the oracle and the seeded input generator are called; the seed
network, when asked for, is read from the committed weights file with numpy.

    python tests/golden/make_heavy_ion.py
        heavy_ion_oracle.json: the first seed from 5000 upwards whose event has
        at most 2600 tracks (about 1 CPU minute; the noise, about 6k clusters
        per plane, is at full strength)
    python tests/golden/make_heavy_ion.py --min-tracks 15000 --out heavy_ion_15k_oracle.json
    python tests/golden/make_heavy_ion.py --min-tracks 15000 --seed-filter \\
        --out heavy_ion_15k_seed_oracle.json
        the first seed from 5000 upwards whose event has at least 15000 tracks,
        without and with the seed-level filter (tens of CPU minutes each)

Event: the heavy-ion workload (single vertex, tracks uniform in [2000, 30000],
0.3 % per-pixel noise, 1 mrad scattering), cut set `cuts_ms`.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.abspath(os.path.join(HERE, "..", ".."))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2412_05041_amd import gen  # noqa: E402

FIT_STRIDE = 97  # every 97th track's FP64 fit is stored
SEED_NET = os.path.join(ROOT, "paper_2412_05041_amd", "configs", "seed_default.npz")


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def pick_seed(min_tracks, max_tracks):
    for seed in range(5000, 5200):
        b = gen.generate(gen.WORKLOADS["heavy_ion"].with_events(1, seed))
        if min_tracks <= int(b.trk_off[-1]) <= max_tracks:
            return seed, b
    raise RuntimeError("no seed found")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--min-tracks", type=int, default=0)
    ap.add_argument("--max-tracks", type=int, default=2600)
    ap.add_argument("--seed-filter", action="store_true", help="run the oracle with the committed seed network")
    ap.add_argument("--out", default="heavy_ion_oracle.json")
    a = ap.parse_args()
    max_tracks = a.max_tracks if a.min_tracks == 0 else max(a.max_tracks, 30000)
    seed, b = pick_seed(a.min_tracks, max_tracks)
    cut = json.load(open(os.path.join(ROOT, "paper_2412_05041_amd", "configs", "cuts_ms.json")))
    net = None
    if a.seed_filter:
        d = np.load(SEED_NET, allow_pickle=False)
        net = (d["weights"].astype(np.float32), d["norm"].astype(np.float32), float(d["threshold"]))
    print(f"seed {seed}: {int(b.trk_off[-1])} MC tracks, {b.n_pix} pixels", flush=True)
    t0 = time.time()
    c = oracle.cluster(b.pix_off, b.pix_id)
    t = oracle.find_tracks(c["clu_off"], c["clu_x"], c["clu_y"], b.plane_z, cut, seed=net)
    par = oracle.fit(t["trk_hit_off"], t["trk_hit"], t["trk_planes"], c["clu_x"], c["clu_y"], b.plane_z, cut["sigma"])
    dt = time.time() - t0
    T = len(t["trk_planes"])
    sample = list(range(0, T, FIT_STRIDE))
    out = {
        "what": "oracle result on one heavy-ion-like event (cuts_ms), digests of the output arrays",
        "workload": "heavy_ion", "seed": seed, "n_events": 1, "cuts": "ms",
        "seed_filter": "configs/seed_default.npz" if net is not None else None,
        "n_pix": b.n_pix, "n_mc_tracks": int(b.trk_off[-1]),
        "n_clusters": int(c["clu_off"][-1]), "n_tracks": T, "n_hits": int(t["trk_hit_off"][-1]),
        "max_plane_clusters": int(np.diff(c["clu_off"]).max()),
        "stats": {"pair_tests": int(t["stats"][0]), "triplet_tests": int(t["stats"][1]),
                  "seed_candidates": int(t["stats"][2]), "seeds_dropped": int(t["stats"][3])},
        "sha256": {
            "clu_off": digest(c["clu_off"].astype(np.int32)),
            "pix_clu": digest(c["pix_clu"].astype(np.int32)),
            "clu_x": digest(c["clu_x"].astype(np.float32)),
            "clu_y": digest(c["clu_y"].astype(np.float32)),
            "trk_off": digest(t["trk_off"].astype(np.int32)),
            "trk_hit_off": digest(t["trk_hit_off"].astype(np.int32)),
            "trk_hit": digest(t["trk_hit"].astype(np.int32)),
            "trk_planes": digest(t["trk_planes"].astype(np.uint32)),
            "trk_flags": digest(t["trk_flags"].astype(np.uint8)),
        },
        "fit_sample": {"tracks": sample, "par64": [[float(v) for v in par[i, :7]] for i in sample]},
        "oracle_seconds": round(dt, 1),
    }
    json.dump(out, open(os.path.join(HERE, a.out), "w"), indent=1)
    print(json.dumps({k: out[k] for k in out if k not in ("sha256", "fit_sample")}), flush=True)


if __name__ == "__main__":
    main()
