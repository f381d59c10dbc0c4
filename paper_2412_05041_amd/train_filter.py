"""Train the learned ghost filter on the GPU and evaluate it against the plain cut.

    python -m paper_2412_05041_amd.train_filter [--candidates 2000000] [--max-epochs 50]
    python -m paper_2412_05041_amd.train_filter --workload nominal --ghost-weight 4 \
        --out configs/mlp_nominal.npz

Steps (all arithmetic in libvelo's kernels):
  1. candidates of generator events found with the workload's cut set, every
     candidate emitted, FP32 features from the feature kernel, ghost labels
     from the MC truth.  Default: the single-vertex generator (20 straight
     tracks, seeds from 1004) with the loose cut set; `--workload nominal`:
     the nominal generator (pile-up, scattering, noise; seeds from 1004) with
     the scattering cut set, whose candidates hold ~0.6 % ghosts;
  2. normalisation (mean, sd) of the training features;
  3. He-uniform initial weights (seed 1004), Adam (lr 1e-3) on batches of
     65536, early stopping on the validation loss (10 % of the candidates).
     `--ghost-weight w` repeats every ghost of the training split w times (a
     class weight of w: the loss then counts each ghost w times);
  4. test events (seed 2004): efficiency and ghost rate of the plain chi2 cut and
     of the learned decision on the same candidates, and events/s of both.
Writes the weights + normalisation (configs/mlp_default.npz by default) and a
JSON report.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from . import gen, learned, velo


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def events_per_s(v, batch, reps=10):
    off, ids = velo.to_device(batch)
    bufs = v.pipeline_buffers(batch.n_events, batch.n_pix)
    v.pipeline(off, ids, bufs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        v.pipeline(off, ids, bufs)
    torch.cuda.synchronize()
    return reps * batch.n_events / (time.perf_counter() - t0)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--candidates", type=int, default=2_000_000)
    ap.add_argument("--max-epochs", type=int, default=50)
    ap.add_argument("--patience", type=int, default=4)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--test-events", type=int, default=5000)
    ap.add_argument("--out", default=learned.WEIGHTS)
    ap.add_argument("--report", default="learned_report.json")
    ap.add_argument("--workload", choices=["learned", "nominal"], default="learned")
    ap.add_argument("--ghost-weight", type=int, default=1)
    args = ap.parse_args()

    if args.workload == "nominal":
        base = learned.cuts("ms")
        train_w, chunk = gen.WORKLOADS["nominal"].with_events(1000, 1004), 1000
        test_w = gen.WORKLOADS["nominal"].with_events(args.test_events, 2004)
    else:
        base = learned.cuts("loose")
        train_w, chunk = gen.WORKLOADS["learned_train"], 20000
        test_w = gen.WORKLOADS["learned_test"].with_events(args.test_events)
    loose = base
    zs = gen.plane_z()
    v = velo.Velo(zs, base)
    t0 = time.time()
    raw, lab, plain = learned.collect(v, train_w, args.candidates, chunk_events=chunk, log=log)
    log(f"collected {len(lab)} candidates ({lab.mean():.4%} ghosts) in {time.time() - t0:.1f}s")
    n_val = len(lab) // 10
    norm = learned.normalisation(raw[:-n_val])
    rng = np.random.default_rng(1004)
    tr_raw, tr_lab = raw[:-n_val], lab[:-n_val]
    if args.ghost_weight > 1:  # class weight: every ghost w times
        g = np.flatnonzero(tr_lab)
        extra = np.repeat(g, args.ghost_weight - 1)
        tr_raw = np.concatenate([tr_raw, tr_raw[extra]])
        tr_lab = np.concatenate([tr_lab, tr_lab[extra]])
    perm = rng.permutation(len(tr_lab))
    v.mlp_set_weights(learned.he_uniform(1004), norm)
    f_tr = learned.standardise(v, tr_raw[perm])
    y_tr = torch.from_numpy(tr_lab[perm].astype(np.uint8)).to(v.device)
    va_raw, va_lab = raw[-n_val:], lab[-n_val:]
    if args.ghost_weight > 1:  # the validation loss with the same class weight
        extra = np.repeat(np.flatnonzero(va_lab), args.ghost_weight - 1)
        va_raw = np.concatenate([va_raw, va_raw[extra]])
        va_lab = np.concatenate([va_lab, va_lab[extra]])
    f_va = learned.standardise(v, va_raw)
    y_va = torch.from_numpy(va_lab.astype(np.uint8)).to(v.device)

    best, best_state, bad, hist = float("inf"), None, 0, []
    for ep in range(args.max_epochs):
        tl = learned.train(v, f_tr, y_tr, 1, lr=args.lr)[0]
        _, vl = v.mlp_grad(f_va, y_va, len(va_lab))
        vl = float(vl.item())
        hist.append((tl, vl))
        log(f"epoch {ep}: train {tl:.5f} val {vl:.5f}")
        if vl < best - 1e-6:
            best, best_state, bad = vl, v.mlp_get_state(), 0
        else:
            bad += 1
            if bad >= args.patience:
                break
    v.mlp_set_state(*best_state)
    master, _ = v.mlp_get_weights()
    np.savez(args.out, master=master, norm=norm)
    log(f"saved {args.out}")

    # evaluation on independent events
    report = dict(workload=args.workload, ghost_weight=args.ghost_weight,
                  train_candidates=int(len(lab) - n_val), val_candidates=int(n_val),
                  ghost_fraction=float(lab.mean()), epochs=len(hist), best_val_loss=best,
                  loss_history=hist)
    test = gen.generate(test_w)
    for band_name, band in (("band0", 0.0), ("band_default", learned.DEFAULT_BAND)):
        r = learned.evaluate(v, test, loose, band)
        report[f"learned_test_{band_name}"] = r
        log(band_name, json.dumps(r))
    v.set_cuts(dict(loose, mode=0))
    report["events_per_s_plain"] = events_per_s(v, test)
    v.set_cuts(dict(loose, mode=1, logit_band=0.0))
    report["events_per_s_learned"] = events_per_s(v, test)
    nominal = gen.generate(gen.WORKLOADS["nominal"].with_events(200, 9202))
    report["nominal_ms_band_default"] = learned.evaluate(v, nominal, learned.cuts("ms"), learned.DEFAULT_BAND)
    os.makedirs(os.path.dirname(args.report) or ".", exist_ok=True)
    json.dump(report, open(args.report, "w"), indent=1)
    print(json.dumps({k: report[k] for k in report if k != "loss_history"}), flush=True)


if __name__ == "__main__":
    main()
