"""GPU parity on a heavy-ion-like event, against the oracle's stored result.

The oracle needs about a minute for this event (7.6k clusters on its fullest
plane, 0.3 % noise), so tests/golden/make_heavy_ion.py stored SHA-256 digests
of its output arrays; the device outputs must hash to the same values, through
the three-call path and through the fused pipeline.  The event is too large for
any LDS tile, so it runs on the global-memory finder.  The FP32 device fit is
checked against the oracle's FP64 fit of the (identical) tracks.
"""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

from gpu_helpers import assert_fit_close, cuts, np_
from paper_2412_05041_amd import gen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "heavy_ion_oracle.json")))


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


@pytest.fixture(scope="module")
def event():
    from paper_2412_05041_amd import velo
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    b = gen.generate(gen.WORKLOADS[GOLD["workload"]].with_events(GOLD["n_events"], GOLD["seed"]))
    assert b.n_pix == GOLD["n_pix"]
    return velo, b


def check_digests(arrays):
    bad = [k for k, a in arrays.items() if digest(a) != GOLD["sha256"][k]]
    assert not bad, f"arrays differing from the oracle: {bad}"


def test_three_call_path(event):
    velo, b = event
    print(f"[heavy] seed {GOLD['seed']}: {b.n_pix} pixels", file=sys.stderr, flush=True)
    cut = cuts(GOLD["cuts"])
    v = velo.Velo(b.plane_z, cut)
    v.reserve(b.n_events, b.n_pix, b.n_pix)
    off, ids = velo.to_device(b)
    c = v.cluster(off, ids, with_npix=False)
    n_clu = int(c["clu_off"][-1].item())
    assert n_clu == GOLD["n_clusters"]
    t = v.find_tracks(c["clu_off"], c["clu_x"], c["clu_y"], n_clu=n_clu)
    torch.cuda.synchronize()
    st = v.read_status(t["status"])
    assert st[0] == 0, st[:8]
    T = int(t["trk_off"][-1].item())
    H = int(t["trk_hit_off"][T].item())
    assert (T, H) == (GOLD["n_tracks"], GOLD["n_hits"])
    check_digests({
        "clu_off": np_(c["clu_off"]), "pix_clu": np_(c["pix_clu"], b.n_pix),
        "clu_x": np_(c["clu_x"], n_clu), "clu_y": np_(c["clu_y"], n_clu),
        "trk_off": np_(t["trk_off"]), "trk_hit_off": np_(t["trk_hit_off"], T + 1), "trk_hit": np_(t["trk_hit"], H),
        "trk_planes": np_(t["trk_planes"], T, np.uint32), "trk_flags": np_(t["trk_flags"], T),
    })
    par = np_(v.fit(t["trk_hit_off"], t["trk_hit"], t["trk_planes"], c["clu_x"], c["clu_y"], n_tracks=T), T)
    tr = dict(trk_hit_off=np_(t["trk_hit_off"], T + 1), trk_hit=np_(t["trk_hit"], H),
              trk_planes=np_(t["trk_planes"], T, np.uint32))
    cc = dict(clu_x=np_(c["clu_x"], n_clu), clu_y=np_(c["clu_y"], n_clu))
    p64 = assert_fit_close(par, tr, cc, b.plane_z, cut["sigma"])
    # the stored sample of the oracle's FP64 fit pins the fit independently
    idx = GOLD["fit_sample"]["tracks"]
    assert np.allclose(p64[idx, :7], np.array(GOLD["fit_sample"]["par64"]), rtol=1e-12, atol=1e-9)


def test_fused_pipeline(event):
    velo, b = event
    cut = cuts(GOLD["cuts"])
    v = velo.Velo(b.plane_z, cut)
    v.reserve(b.n_events, b.n_pix, b.n_pix)
    off, ids = velo.to_device(b)
    bufs = v.pipeline_buffers(b.n_events, b.n_pix)
    for _ in range(2):  # second call replays the captured graph
        v.pipeline(off, ids, bufs)
        torch.cuda.synchronize()
        st = v.read_status(bufs["status"])
        assert st[0] == 0, st[:8]
        n_clu, T, H = int(st[1]), int(st[2]), int(st[3])
        assert (n_clu, T, H) == (GOLD["n_clusters"], GOLD["n_tracks"], GOLD["n_hits"])
        check_digests({
            "clu_off": np_(bufs["clu_off"]), "pix_clu": np_(bufs["pix_clu"], b.n_pix),
            "clu_x": np_(bufs["clu_x"], n_clu), "clu_y": np_(bufs["clu_y"], n_clu),
            "trk_off": np_(bufs["trk_off"]), "trk_hit_off": np_(bufs["trk_hit_off"], T + 1),
            "trk_hit": np_(bufs["trk_hit"], H), "trk_planes": np_(bufs["trk_planes"], T, np.uint32),
            "trk_flags": np_(bufs["trk_flags"], T),
        })


def test_context_first_reserved_for_many_small_events(event):
    """A context reserved for 1000 nominal-size events, then for this one event:
    the counts fit the old workspace, but its large-event candidate pool was
    sized for small events, so velo_reserve must lay it out again."""
    velo, b = event
    cut = cuts(GOLD["cuts"])
    v = velo.Velo(b.plane_z, cut)
    v.reserve(1000, 6_000_000, 6_000_000)
    v.reserve(b.n_events, b.n_pix, b.n_pix)
    off, ids = velo.to_device(b)
    c = v.cluster(off, ids, with_npix=False)
    n_clu = int(c["clu_off"][-1].item())
    t = v.find_tracks(c["clu_off"], c["clu_x"], c["clu_y"], n_clu=n_clu)
    torch.cuda.synchronize()
    st = v.read_status(t["status"])
    assert st[0] == 0, st[:8]
    T = int(t["trk_off"][-1].item())
    H = int(t["trk_hit_off"][T].item())
    assert (T, H) == (GOLD["n_tracks"], GOLD["n_hits"])
    check_digests({"trk_hit_off": np_(t["trk_hit_off"], T + 1), "trk_hit": np_(t["trk_hit"], H),
                   "trk_planes": np_(t["trk_planes"], T, np.uint32)})
