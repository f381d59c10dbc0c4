"""Several batches in flight, as the benchmark runs them: four contexts, each
with its own batch, buffers and HIP stream, their pipelines (replayed graphs)
interleaved so that all four run at once.  Every batch's clusters and tracks
must equal the oracle's for that batch, bit for bit: no context may see
another's work.
"""
import sys

import pytest

from gpu_helpers import assert_clusters_equal, assert_tracks_equal, cuts, oracle_run
from paper_2412_05041_amd import gen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

LANES = 4
EVENTS = 64


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def velo_mod():
    from paper_2412_05041_amd import velo
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return velo


@pytest.mark.parametrize("launch", [(256, 0), (512, 1)])
def test_four_batches_in_flight_match_their_oracles(velo_mod, launch):
    cut = cuts("ms")
    batches = [gen.generate(gen.WORKLOADS["nominal"].with_events(EVENTS, 7100 + k)) for k in range(LANES)]
    lanes = []
    for b in batches:
        v = velo_mod.Velo(b.plane_z, cut)
        v.reserve(b.n_events, b.n_pix, b.n_pix)
        v.set_launch(*launch)
        off, ids = velo_mod.to_device(b)
        lanes.append(dict(v=v, b=b, off=off, ids=ids, bufs=v.pipeline_buffers(b.n_events, b.n_pix),
                          stream=torch.cuda.Stream()))
    torch.cuda.synchronize()
    say(f"[in flight] {LANES} contexts x {EVENTS} nominal events, launch {launch}")
    cur = torch.cuda.current_stream()
    for L in lanes:
        L["stream"].wait_stream(cur)
    for k in range(3 * LANES):  # three replays per lane, all lanes in flight
        L = lanes[k % LANES]
        with torch.cuda.stream(L["stream"]):
            L["v"].pipeline(L["off"], L["ids"], L["bufs"])
    for L in lanes:
        cur.wait_stream(L["stream"])
    torch.cuda.synchronize()
    for k, L in enumerate(lanes):
        b = L["b"]
        c, t = oracle_run(b, cut)
        assert L["v"].read_status(L["bufs"]["status"])[0] == 0, k
        assert_clusters_equal(L["bufs"], c, b.n_pix)
        assert_tracks_equal(L["bufs"], t)
    for L in lanes:
        L["v"].close()
