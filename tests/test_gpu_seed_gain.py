"""What the trained seed-level filter gains over the plain method (committed weights).

The network in configs/seed_default.npz was trained on the GPU by the library's
own kernels (paper_2412_05041_amd/train_seed_filter.py) on the seeds of
nominal-occupancy events and of events with the literal 0.1 % per-pixel noise.
On independent events it must keep the nominal efficiency (>= plain - 0.5 %)
without adding ghosts, and on the noisy events -- where greedy claiming lets
noise triplets take the hits of real tracks -- raise the efficiency by more
than five points and cut the ghost rate from above 90 % to below 50 %.
"""
import os
import sys

import pytest

from gpu_helpers import cuts
from paper_2412_05041_amd import gen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    from paper_2412_05041_amd import seeds, velo
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(seeds.WEIGHTS):
        pytest.skip("no trained seed weights")
    return seeds, velo, seeds.load_default()


def compare(ctx, workload, n, seed):
    seeds, velo, net = ctx
    cut = cuts("ms")
    b = gen.generate(gen.WORKLOADS[workload].with_events(n, seed))
    v = velo.Velo(b.plane_z, cut)
    p = seeds.reconstruct(v, b, cut)
    s = seeds.reconstruct(v, b, cut, net)
    print(f"[seed gain] {workload}: plain {p['efficiency']:.4f}/{p['ghost_rate']:.4f}  "
          f"filtered {s['efficiency']:.4f}/{s['ghost_rate']:.4f}", file=sys.stderr, flush=True)
    assert p["severity"] == 0 and s["severity"] == 0
    return p, s


def test_nominal_efficiency_kept(ctx):
    p, s = compare(ctx, "nominal", 300, 9301)
    assert s["efficiency"] >= p["efficiency"] - 0.005
    assert s["ghost_rate"] <= p["ghost_rate"]


def test_noisy_events_gain(ctx):
    p, s = compare(ctx, "nominal_literal_noise", 10, 9302)
    assert p["ghost_rate"] > 0.9
    assert s["efficiency"] > p["efficiency"] + 0.05
    assert s["ghost_rate"] < 0.5
