"""GPU failure handling, forced from the host: output capacities too small for
the tracks or their hits, and a learned filter whose weights are NaN.

* Track or hit capacity overflow: the call still succeeds; d_status reports
  severity 1 and the required track and hit counts (exact), trk_off is
  complete and equal to the oracle's, every track written below the
  capacities equals the oracle's track, and exactly the events with a track
  that did not fit are flagged VELO_EV_OVERFLOW.
* NaN weights: every logit is NaN, so every decision falls back to the plain
  chi2 cut: the tracks equal the oracle's plain-method tracks bit for bit,
  every track carries the fallback flag, and d_status[6] counts them all.
"""
import sys

import numpy as np
import pytest

from gpu_helpers import assert_tracks_equal, cuts, np_, oracle_run
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
    b = gen.generate(gen.WORKLOADS["nominal"].with_events(40, 4242))
    cut = cuts("ms")
    c, t = oracle_run(b, cut)
    return velo, b, cut, c, t


def check_capacity(velo, b, cut, c, t, trk_cap, hit_cap):
    v = velo.Velo(b.plane_z, cut)
    v.reserve(b.n_events, b.n_pix, b.n_pix)
    off, ids = velo.to_device(b)
    gc = v.cluster(off, ids, with_npix=False)
    n_clu = int(c["clu_off"][-1])
    g = v.find_tracks(gc["clu_off"], gc["clu_x"], gc["clu_y"], n_clu=n_clu, trk_cap=trk_cap, hit_cap=hit_cap)
    torch.cuda.synchronize()
    st = v.read_status(g["status"])
    T, H = len(t["trk_planes"]), int(t["trk_hit_off"][-1])
    assert st[0] == 1 and st[2] == T and st[3] == H, st[:8]
    assert np.array_equal(np_(g["trk_off"]), t["trk_off"])
    hoff = t["trk_hit_off"].astype(np.int64)
    fits = (np.arange(T) < trk_cap) & (hoff[1:] <= hit_cap)
    n_fit = int(fits.sum())
    assert n_fit > 0 and fits[:n_fit].all()  # the tracks that fit are a prefix
    assert np.array_equal(np_(g["trk_hit_off"], n_fit), t["trk_hit_off"][:n_fit])
    assert np.array_equal(np_(g["trk_planes"], n_fit, np.uint32), t["trk_planes"][:n_fit])
    h_fit = int(hoff[n_fit])
    assert np.array_equal(np_(g["trk_hit"], h_fit), t["trk_hit"][:h_fit])
    # events flagged: those with a track that did not fit
    ev_of = np.repeat(np.arange(b.n_events), np.diff(t["trk_off"]))
    want = np.zeros(b.n_events, bool)
    want[ev_of[~fits]] = True
    got = (st[8:8 + b.n_events] & velo.EV_OVERFLOW) != 0
    assert np.array_equal(got, want)
    v.close()


def test_track_capacity_overflow(setup):
    velo, b, cut, c, t = setup
    T = len(t["trk_planes"])
    say(f"[failures] track capacity {T // 2} of {T}")
    check_capacity(velo, b, cut, c, t, T // 2, int(t["trk_hit_off"][-1]) + 10)


def test_hit_capacity_overflow(setup):
    velo, b, cut, c, t = setup
    H = int(t["trk_hit_off"][-1])
    say(f"[failures] hit capacity {H // 3} of {H}")
    check_capacity(velo, b, cut, c, t, len(t["trk_planes"]) + 10, H // 3)


def test_nan_weights_fall_back_to_the_plain_cut(setup):
    velo, b, cut, c, t = setup
    say("[failures] NaN network weights")
    v = velo.Velo(b.plane_z, dict(cut, mode=1, logit_band=0.0))
    norm = np.concatenate([np.zeros(10), np.ones(10)]).astype(np.float32)
    v.mlp_set_weights(np.full(velo.N_PARAM, np.nan, np.float32), norm)
    v.reserve(b.n_events, b.n_pix, b.n_pix)
    off, ids = velo.to_device(b)
    bufs = v.pipeline_buffers(b.n_events, b.n_pix)
    v.pipeline(off, ids, bufs)
    torch.cuda.synchronize()
    st = v.read_status(bufs["status"])
    assert st[0] == 0, st[:8]
    assert_tracks_equal(bufs, t)
    T = len(t["trk_planes"])
    fl = np_(bufs["trk_flags"], T)
    assert np.all(fl & velo.TRK_FALLBACK) and np.all(fl & velo.TRK_LEARNED)
    # every candidate's decision fell back: at least every output track
    assert st[6] >= T
    has = np.diff(t["trk_off"]) > 0
    assert np.all((st[8:8 + b.n_events][has] & velo.EV_FALLBACK) != 0)
    v.close()
