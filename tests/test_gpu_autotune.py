"""GPU checks of the library's autotuner (velo_autotune): with two batches in
flight on their own contexts and streams it picks the fastest of the timed
launches, sets it on both contexts, and the pipeline then still gives the
oracle's tracks bit for bit; its text cache reproduces the pick without timing;
a bad call leaves every launch as it was."""
import ctypes as C
import sys

import numpy as np
import pytest

from gpu_helpers import assert_clusters_equal, assert_tracks_equal, cuts, oracle_run
from paper_2412_05041_amd import gen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

THREADS = (64, 128, 256, 512)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def velo_mod():
    from paper_2412_05041_amd import velo
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return velo


def test_autotune_in_flight_pick_cache_and_parity(velo_mod, tmp_path):
    say("[autotune] two contexts in flight, nominal 96 events")
    b = gen.generate(gen.WORKLOADS["nominal"].with_events(96, 61))
    cut = cuts("ms")
    c, t = oracle_run(b, cut)
    ctxs = [velo_mod.Velo(b.plane_z, cut) for _ in range(2)]
    for v in ctxs:
        v.reserve(b.n_events, b.n_pix, b.n_pix)
        v.set_launch(64, 2)
    off, ids = velo_mod.to_device(b)
    gc = ctxs[0].cluster(off, ids, with_npix=False)
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream() for _ in ctxs]
    cache = str(tmp_path / "tune.txt")
    ms, launch = velo_mod.autotune(ctxs, gc["clu_off"], gc["clu_x"], gc["clu_y"], reps=2, cache=cache,
                                   streams=streams)
    assert len(ms) == velo_mod.N_LAUNCH and min(ms) > 0
    i = int(np.argmin(ms))
    assert launch == (THREADS[i // 3], i % 3), (launch, ms)
    assert all(v.get_launch() == launch for v in ctxs)
    # the cache gives the same pick without timing
    for v in ctxs:
        v.set_launch(64, 2)
    ms2, launch2 = velo_mod.autotune(ctxs, gc["clu_off"], gc["clu_x"], gc["clu_y"], reps=2, cache=cache,
                                     streams=streams)
    assert launch2 == launch and all(x == -1.0 for x in ms2)
    assert all(v.get_launch() == launch for v in ctxs)
    assert open(cache).read().count("\n") == 1
    # both contexts with the tuned launch: oracle tracks bit for bit
    for v in ctxs:
        bufs = v.pipeline_buffers(b.n_events, b.n_pix)
        v.pipeline(off, ids, bufs)
        torch.cuda.synchronize()
        assert v.read_status(bufs["status"])[0] == 0
        assert_clusters_equal(bufs, c, b.n_pix)
        assert_tracks_equal(bufs, t)
    # bad calls: rejected before any work, launches unchanged
    lib = velo_mod.lib()
    hs = (C.c_void_p * 2)(ctxs[0].h.value, ctxs[0].h.value)
    ss = (C.c_void_p * 2)(streams[0].cuda_stream, streams[1].cuda_stream)
    p = lambda x: C.c_void_p(x.data_ptr())
    rc = lib.velo_autotune(hs, 2, b.n_events, p(gc["clu_off"]), p(gc["clu_x"]), p(gc["clu_y"]), 2, None, None, ss)
    assert rc == -1 and b"twice" in lib.velo_last_error()
    rc = lib.velo_autotune(hs, 0, b.n_events, p(gc["clu_off"]), p(gc["clu_x"]), p(gc["clu_y"]), 2, None, None, ss)
    assert rc == -1
    assert all(v.get_launch() == launch for v in ctxs)
    for v in ctxs:
        v.close()
