"""Train the seed-level filter on the GPU and measure what it gains.

    python -m paper_2412_05041_amd.train_seed_filter [--nominal-events 6000] [--noise-events 40]

Steps (all arithmetic in libvelo's kernels):
  1. seed candidates of the plain finder (ms cut set) on training events of two
     kinds: nominal occupancy (seeds from 3001) and the literal 0.1 % per-pixel
     noise of the nominal configuration (seeds from 3501); the finder emits each
     candidate's ten FP32 features, labels come from the MC truth (fake = the
     three clusters do not share one particle);
  2. normalisation (mean, sd) of the training features, He-uniform initial
     weights (seed 3001), Adam (lr 1e-3) on batches of 65536 with the BF16 MFMA
     training kernels, early stopping on the validation loss (10 %);
  3. threshold: the logits of the genuine validation seeds give the cuts that
     keep 99 % ... 99.99 % of them; for each, the finder with the filter
     reconstructs validation events of both kinds, and the cut with the best
     noisy-event efficiency among those that keep the nominal efficiency within
     0.2 % of the plain method and the noisy-event ghost rate below one third is
     kept;
  4. independent test events (seeds from 4001): efficiency, ghost and clone
     rates and events/s with and without the filter, nominal, noisy and
     heavy-ion.
Writes configs/seed_default.npz (BF16-rounded weights, normalisation,
threshold) and a JSON report.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from . import gen, learned, seeds, velo


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def gather(v, workload, n_events, chunk, seed0):
    raws, labs = [], []
    for i, e0 in enumerate(range(0, n_events, chunk)):
        b = gen.generate(workload.with_events(min(chunk, n_events - e0), seed0 + i))
        raw, lab, _ = seeds.collect(v, b, cap=max(b.n_pix * 2, 1 << 16))
        raws.append(raw)
        labs.append(lab)
        log(f"{workload.name} chunk {i}: {len(lab)} seeds, {lab.mean():.3%} fake")
    return np.concatenate(raws), np.concatenate(labs)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--nominal-events", type=int, default=6000)
    ap.add_argument("--noise-events", type=int, default=40)
    ap.add_argument("--max-epochs", type=int, default=60)
    ap.add_argument("--patience", type=int, default=5)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--out", default=seeds.WEIGHTS)
    ap.add_argument("--report", default="seed_report.json")
    args = ap.parse_args()

    cut = learned.cuts("ms")
    zs = gen.plane_z()
    nominal, noisy = gen.WORKLOADS["nominal"], gen.WORKLOADS["nominal_literal_noise"]
    v = velo.Velo(zs, cut)
    t0 = time.time()
    r1, l1 = gather(v, nominal, args.nominal_events, 2000, 3001)
    r2, l2 = gather(v, noisy, args.noise_events, 10, 3501)
    raw, lab = np.concatenate([r1, r2]), np.concatenate([l1, l2])
    rng = np.random.default_rng(3001)
    perm = rng.permutation(len(lab))
    raw, lab = raw[perm], lab[perm]
    log(f"collected {len(lab)} seeds ({lab.mean():.3%} fake) in {time.time() - t0:.1f}s")

    n_val = len(lab) // 10
    norm = learned.normalisation(raw[n_val:])
    tr = velo.Velo(zs, cut)  # the training context (its MLP state)
    tr.mlp_set_weights(learned.he_uniform(3001), norm)
    f_tr = learned.standardise(tr, raw[n_val:])
    y_tr = torch.from_numpy(lab[n_val:].astype(np.uint8)).to(tr.device)
    f_va = learned.standardise(tr, raw[:n_val])
    y_va = torch.from_numpy(lab[:n_val].astype(np.uint8)).to(tr.device)
    best, best_state, bad, hist = float("inf"), None, 0, []
    for ep in range(args.max_epochs):
        tl = learned.train(tr, f_tr, y_tr, 1, lr=args.lr)[0]
        _, vl = tr.mlp_grad(f_va, y_va, n_val)
        vl = float(vl.item())
        hist.append((tl, vl))
        log(f"epoch {ep}: train {tl:.5f} val {vl:.5f}")
        if vl < best - 1e-6:
            best, best_state, bad = vl, tr.mlp_get_state(), 0
        else:
            bad += 1
            if bad >= args.patience:
                break
    tr.mlp_set_state(*best_state)
    master, _ = tr.mlp_get_weights()
    weights = seeds.bf16_round(master)

    # threshold scan on validation events
    z_va = tr.mlp_forward(f_va, n_val).cpu().numpy()[:n_val]
    genuine = z_va[lab[:n_val] == 0]
    val_nom = gen.generate(nominal.with_events(300, 3901))
    val_noise = gen.generate(noisy.with_events(6, 3902))
    base_nom = seeds.reconstruct(v, val_nom, cut)
    base_noise = seeds.reconstruct(v, val_noise, cut)
    scan = []
    for keep in (0.99, 0.995, 0.998, 0.999, 0.9995, 0.9998, 0.9999):
        thr = float(np.quantile(genuine, keep))
        net = (weights, norm, thr)
        a = seeds.reconstruct(v, val_nom, cut, net)
        b = seeds.reconstruct(v, val_noise, cut, net)
        scan.append(dict(keep=keep, threshold=thr, nominal=a, noisy=b))
        log(f"keep {keep}: thr {thr:.3f} nominal eff {a['efficiency']:.4f} ghost {a['ghost_rate']:.4f} | "
            f"noisy eff {b['efficiency']:.4f} ghost {b['ghost_rate']:.4f}")
    ok = [s for s in scan if s["nominal"]["efficiency"] >= base_nom["efficiency"] - 0.002
          and s["noisy"]["ghost_rate"] < 1.0 / 3.0] or scan[:1]
    chosen = max(ok, key=lambda s: s["noisy"]["efficiency"])
    np.savez(args.out, weights=weights, norm=norm, threshold=np.float32(chosen["threshold"]))
    log(f"saved {args.out} (threshold {chosen['threshold']:.4f}, keep {chosen['keep']})")

    # independent test events
    net = (weights, norm, chosen["threshold"])
    report = dict(train_seeds=int(len(lab) - n_val), val_seeds=int(n_val), fake_fraction=float(lab.mean()),
                  epochs=len(hist), best_val_loss=best, loss_history=hist, threshold=chosen["threshold"],
                  keep_genuine=chosen["keep"], validation=dict(plain_nominal=base_nom, plain_noisy=base_noise,
                                                               scan=scan))
    tests = {"nominal": (nominal.with_events(1000, 4001), 20), "noisy": (noisy.with_events(40, 4002), 3),
             "heavy_ion": (gen.WORKLOADS["heavy_ion"].with_events(4, 4003), 1)}
    for name, (w, reps) in tests.items():
        b = gen.generate(w)
        p = seeds.reconstruct(v, b, cut, None, reps=reps)
        s = seeds.reconstruct(v, b, cut, net, reps=reps)
        report[f"test_{name}"] = dict(plain=p, seed_filter=s)
        log(f"test {name}: plain {json.dumps(p)}\n    seed  {json.dumps(s)}")
    os.makedirs(os.path.dirname(args.report) or ".", exist_ok=True)
    json.dump(report, open(args.report, "w"), indent=1)
    print(json.dumps({k: report[k] for k in report if k not in ("loss_history", "validation")}), flush=True)


if __name__ == "__main__":
    main()
