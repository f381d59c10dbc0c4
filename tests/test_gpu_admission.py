"""GPU checks of the finder's event routing (velo_set_admission): an event whose
clusters exceed the ratio x an LDS tile's track capacity skips that tile.  The
routing never changes a track: on a nominal batch whose largest events overflow
the first tile, the tracks equal the oracle's bit for bit with the default
ratio, with the rule off (those events then run out of track slots mid-event
and are redone by the second tile) and with a ratio so small that every
non-empty event skips both tiles for the global-memory path."""
import sys

import numpy as np
import pytest

from gpu_helpers import assert_clusters_equal, assert_tracks_equal, cuts, oracle_run
from paper_2412_05041_amd import gen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def setup():
    from paper_2412_05041_amd import velo
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    b = gen.generate(gen.WORKLOADS["nominal"].with_events(64, 515))
    cut = cuts("ms")
    c, t = oracle_run(b, cut)
    return velo, b, cut, c, t


@pytest.mark.parametrize("ratio", [None, 0.0, 1e-3])
def test_routing_keeps_the_tracks(setup, ratio):
    velo, b, cut, c, t = setup
    say(f"[admission] ratio {ratio}")
    v = velo.Velo(b.plane_z, cut)
    v.set_launch(256, 0)
    if ratio is not None:
        v.set_admission(ratio)
    v.reserve(b.n_events, b.n_pix, b.n_pix)
    off, ids = velo.to_device(b)
    bufs = v.pipeline_buffers(b.n_events, b.n_pix)
    v.pipeline(off, ids, bufs)
    torch.cuda.synchronize()
    st = v.read_status(bufs["status"])
    assert st[0] == 0, st[:8]
    assert_clusters_equal(bufs, c, b.n_pix)
    assert_tracks_equal(bufs, t, check_flags=True)
    ev = st[8:8 + b.n_events]
    second = (ev & velo.EV_SECOND_TILE) != 0
    ncl = np.diff(c["clu_off"][::26])
    if ratio is None or ratio == 0.0:
        # the batch holds events too large for the first tile, and they were redone
        assert second.sum() >= 3
        assert st[5] == 0
    else:
        assert st[5] == int((ncl > 0).sum())
        assert np.all(((ev & velo.EV_LARGE_PATH) != 0) == (ncl > 0))
    v.close()


def test_bad_ratio_rejected(setup):
    velo, b, cut, c, t = setup
    v = velo.Velo(b.plane_z, cut)
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(velo.VeloError):
            v.set_admission(bad)
    v.close()
