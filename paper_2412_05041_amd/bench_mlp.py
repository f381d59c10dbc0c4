"""Throughput of the learned filter's MLP kernels on one GPU.

    python -m paper_2412_05041_amd.bench_mlp [--samples 2097152] [--reps 20]

Times the BF16 MFMA forward (velo_mlp_forward) over `samples` candidates and
the training step (velo_mlp_train_step: forward, backward, deterministic
gradient reduction, Adam) on batches of 65536, with HIP events on the launch
stream.  Work per sample: forward 2 x (10*32 + 32*32 + 32) = 2752 FLOP (the
10->32 layer padded to 16 inputs on the MFMA: 2 x (16*32 + 32*32 + 32) = 3136
issued); backward ~4864 FLOP.  Prints one JSON line with the achieved TFLOP/s
and the fraction of the MI355X dense BF16 peak (2.5 PFLOP/s).
"""
from __future__ import annotations

import argparse
import json

import numpy as np
import torch

from . import velo

BF16_PEAK_TFLOPS = 2500.0
FWD_FLOP = 2 * (10 * 32 + 32 * 32 + 32)
BWD_FLOP = 4864


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--samples", type=int, default=1 << 21)
    ap.add_argument("--batch", type=int, default=65536)
    ap.add_argument("--reps", type=int, default=20)
    args = ap.parse_args()
    rng = np.random.default_rng(1)
    v = velo.Velo(np.linspace(-300, 750, 26).astype(np.float32), dict(
        t_max=0.4, d2_max=9.0, s_max=0.09, e_max=0.25, max_skip=1, c3=4.0, c4=16.0,
        sigma=float(np.float32(0.055 / np.sqrt(12.0))), mode=0, logit_band=0.0))
    w = np.zeros(1441, np.float32)
    w[:1440] = rng.normal(0, 0.3, 1440)
    v.mlp_set_weights(w, np.concatenate([np.zeros(10), np.ones(10)]).astype(np.float32))
    raw = torch.from_numpy(rng.normal(0, 1, (args.samples, 10)).astype(np.float32)).to(v.device)
    feat = v.standardize(raw, args.samples)
    label = torch.from_numpy((rng.random(args.samples) < 0.1).astype(np.uint8)).to(v.device)
    loss = torch.zeros(1, dtype=torch.float32, device=v.device)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    v.mlp_forward(feat, args.samples)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.reps):
        v.mlp_forward(feat, args.samples)
    e1.record()
    torch.cuda.synchronize()
    fwd_ms = e0.elapsed_time(e1) / args.reps

    B = args.batch
    v.mlp_train_step(feat[:B], label[:B], 1e-3, n=B, loss=loss)
    torch.cuda.synchronize()
    nb = args.samples // B
    e0.record()
    for r in range(args.reps):
        i = (r % nb) * B
        v.mlp_train_step(feat[i:i + B], label[i:i + B], 1e-3, n=B, loss=loss)
    e1.record()
    torch.cuda.synchronize()
    step_ms = e0.elapsed_time(e1) / args.reps

    fwd_tf = args.samples * FWD_FLOP / (fwd_ms * 1e-3) / 1e12
    step_tf = B * (FWD_FLOP + BWD_FLOP) / (step_ms * 1e-3) / 1e12
    print(json.dumps({
        "forward": {"samples": args.samples, "ms": fwd_ms, "samples_per_s": args.samples / (fwd_ms * 1e-3),
                    "TFLOPs": fwd_tf, "frac_bf16_peak": fwd_tf / BF16_PEAK_TFLOPS},
        "train_step": {"batch": B, "ms": step_ms, "samples_per_s": B / (step_ms * 1e-3),
                       "TFLOPs": step_tf, "frac_bf16_peak": step_tf / BF16_PEAK_TFLOPS},
        "peak_TFLOPs": BF16_PEAK_TFLOPS,
    }), flush=True)


if __name__ == "__main__":
    main()
