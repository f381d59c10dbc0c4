"""GPU parity of the large-event finder's key-range seeding: a plane step with
more seed candidates than the workgroup's pool is seeded in ascending ranges of
the claiming key (q, h0), each claimed before the next is enumerated.  With the
pool cut down to a few hundred entries, literal-noise events (the large-event
path: thousands of clusters per plane, ~1.5k candidates per step) go through
many ranges per step; their tracks must equal the oracle's bit for bit, without
and with the seed-level filter, and equal those of the full pool."""
import json
import os
import sys

import numpy as np
import pytest

import oracle
from gpu_helpers import assert_tracks_equal, cuts, np_
from paper_2412_05041_amd import gen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def velo_mod():
    from paper_2412_05041_amd import velo
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return velo


def seed_net():
    d = np.load(os.path.join(ROOT, "paper_2412_05041_amd", "configs", "seed_default.npz"), allow_pickle=False)
    return d["weights"].astype(np.float32), d["norm"].astype(np.float32), float(d["threshold"])


@pytest.fixture(scope="module")
def noisy():
    b = gen.generate(gen.WORKLOADS["nominal_literal_noise"].with_events(3, 71))
    c = oracle.cluster(b.pix_off, b.pix_id)
    return b, c


@pytest.mark.parametrize("with_seed_filter", [False, True])
def test_range_seeding_matches_oracle(velo_mod, noisy, with_seed_filter):
    b, c = noisy
    cut = cuts("ms")
    net = seed_net() if with_seed_filter else None
    t = oracle.find_tracks(c["clu_off"], c["clu_x"], c["clu_y"], b.plane_z, cut, seed=net)
    v = velo_mod.Velo(b.plane_z, cut)
    if net is not None:
        v.seed_filter_set(*net)
    v.reserve(b.n_events, b.n_pix, b.n_pix)
    off, ids = velo_mod.to_device(b)
    results = []
    for pool in (0, 4096, 300, 64):
        say(f"[ranges] seed_filter={with_seed_filter} pool={pool}")
        v.set_large_pool(pool)
        bufs = v.pipeline_buffers(b.n_events, b.n_pix)
        v.pipeline(off, ids, bufs)
        torch.cuda.synchronize()
        st = v.read_status(bufs["status"])
        assert st[0] == 0, st[:8]
        assert st[5] == b.n_events  # every event on the large-event path
        if pool:
            assert st[7] > pool  # some step had more candidates than the pool: ranges were used
        assert_tracks_equal(bufs, t)
        T = int(np_(bufs["trk_off"])[-1])
        results.append(np_(bufs["trk_hit"], int(np_(bufs["trk_hit_off"], T + 1)[-1])))
    assert all(np.array_equal(results[0], r) for r in results[1:])
    with pytest.raises(velo_mod.VeloError):
        v.set_large_pool(-1)
    v.close()
