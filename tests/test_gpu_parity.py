"""GPU parity: the HIP path through the C ABI vs the CPU oracle.

Clusters (ids, offsets, centroid bits) and tracks (CSR hit lists, plane masks,
flags) must be bit-identical; the FP32 fit must agree with the FP64 oracle fit
to 1e-5 of each quantity's natural scale.
"""
import sys

import numpy as np
import pytest

from gpu_helpers import (assert_clusters_equal, assert_fit_close, assert_tracks_equal, cuts, np_,
                         oracle_run)
from paper_2412_05041_amd import gen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def velo_mod():
    from paper_2412_05041_amd import velo
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return velo


WORKLOADS = [
    ("tiny", None, "default"),
    ("nominal", None, "ms"),
    ("uneven", None, "default"),
    ("nominal_literal_noise", 20, "ms"),
]


def make(name, n):
    w = gen.WORKLOADS[name]
    return gen.generate(w if n is None else w.with_events(n))


@pytest.mark.parametrize("name,n,cutname", WORKLOADS)
def test_three_call_path_matches_oracle(velo_mod, name, n, cutname):
    say(f"[parity] three-call {name} n={n}")
    b = make(name, n)
    cut = cuts(cutname)
    c, t = oracle_run(b, cut)
    v = velo_mod.Velo(b.plane_z, cut)
    v.reserve(b.n_events, b.n_pix, b.n_pix)
    off, ids = velo_mod.to_device(b)
    gc = v.cluster(off, ids)
    torch.cuda.synchronize()
    st = v.read_status(gc["status"])
    assert st[0] == 0 and st[1] == int(c["clu_off"][-1]) and st[4] == b.n_pix
    assert_clusters_equal(gc, c, b.n_pix)
    n_clu = int(c["clu_off"][-1])
    gt = v.find_tracks(gc["clu_off"], gc["clu_x"], gc["clu_y"], n_clu=n_clu)
    torch.cuda.synchronize()
    st = v.read_status(gt["status"])
    assert st[0] == 0, st[:8]
    assert_tracks_equal(gt, t)
    T = len(t["trk_planes"])
    par = v.fit(gt["trk_hit_off"], gt["trk_hit"], gt["trk_planes"], gc["clu_x"], gc["clu_y"], n_tracks=T)
    assert_fit_close(np_(par, T), t, c, b.plane_z, cut["sigma"])
    say(f"[parity] {name}: {b.n_events} events, {n_clu} clusters, {T} tracks, large={st[5]}")


@pytest.mark.parametrize("name,n,cutname", WORKLOADS[:3])
def test_pipeline_matches_oracle_and_replays(velo_mod, name, n, cutname):
    say(f"[parity] pipeline {name}")
    b = make(name, n)
    cut = cuts(cutname)
    c, t = oracle_run(b, cut)
    v = velo_mod.Velo(b.plane_z, cut)
    v.reserve(b.n_events, b.n_pix, b.n_pix)
    off, ids = velo_mod.to_device(b)
    bufs = v.pipeline_buffers(b.n_events, b.n_pix)
    first = None
    for rep in range(3):  # first call captures the graph, later calls replay it
        for k in ("trk_hit", "trk_planes", "clu_x"):
            bufs[k].fill_(-7)
        v.pipeline(off, ids, bufs)
        torch.cuda.synchronize()
        st = v.read_status(bufs["status"])
        assert st[0] == 0, st[:8]
        assert_clusters_equal(bufs, c, b.n_pix)
        assert_tracks_equal(bufs, t, check_flags=True)
        T = len(t["trk_planes"])
        if first is None:
            first = np_(bufs["par"], T).copy()
            assert_fit_close(first, t, c, b.plane_z, cut["sigma"])
        else:
            assert np.array_equal(np_(bufs["par"], T), first)


@pytest.mark.parametrize("name,n,cutname", WORKLOADS[:2])
def test_three_calls_on_pipeline_buffers(velo_mod, name, n, cutname):
    """velo_cluster -> velo_find_tracks -> velo_fit on the pipeline's buffers,
    with the fit's track count read on the device: the oracle's outputs."""
    say(f"[parity] three-call {name}")
    b = make(name, n)
    cut = cuts(cutname)
    c, t = oracle_run(b, cut)
    v = velo_mod.Velo(b.plane_z, cut)
    v.reserve(b.n_events, b.n_pix, b.n_pix)
    off, ids = velo_mod.to_device(b)
    bufs = v.pipeline_buffers(b.n_events, b.n_pix)
    v.three_call(off, ids, bufs)
    torch.cuda.synchronize()
    assert v.read_status(bufs["status_clu"])[0] == 0
    assert v.read_status(bufs["status"])[0] == 0
    assert_clusters_equal(dict(bufs, clu_npix=None), c, b.n_pix)
    assert_tracks_equal(bufs, t, check_flags=True)
    T = len(t["trk_planes"])
    assert_fit_close(np_(bufs["par"], T), t, c, b.plane_z, cut["sigma"])


def test_emit_rejected_candidates_and_flags(velo_mod):
    b = make("nominal", 60)
    cut = cuts("ms")
    c, t = oracle_run(b, cut, emit_rejected=True)
    v = velo_mod.Velo(b.plane_z, cut)
    v.reserve(b.n_events, b.n_pix, b.n_pix)
    off, ids = velo_mod.to_device(b)
    gc = v.cluster(off, ids)
    gt = v.find_tracks(gc["clu_off"], gc["clu_x"], gc["clu_y"], emit_rejected=True)
    torch.cuda.synchronize()
    assert_tracks_equal(gt, t, check_flags=True)
    assert np.any((t["trk_flags"] & 8) == 0)  # some candidates rejected


@pytest.mark.parametrize("threads", [64, 128, 256, 512])
@pytest.mark.parametrize("tile", [0, 1, 2])
def test_every_launch_configuration_gives_identical_tracks(velo_mod, threads, tile):
    say(f"[parity] launch threads={threads} tile={tile}")
    b = make("nominal", 120)
    cut = cuts("ms")
    c, t = oracle_run(b, cut)
    v = velo_mod.Velo(b.plane_z, cut)
    v.set_launch(threads, tile)
    v.reserve(b.n_events, b.n_pix, b.n_pix)
    off, ids = velo_mod.to_device(b)
    bufs = v.pipeline_buffers(b.n_events, b.n_pix)
    v.pipeline(off, ids, bufs)
    torch.cuda.synchronize()
    st = v.read_status(bufs["status"])
    assert st[0] == 0
    assert_tracks_equal(bufs, t, check_flags=True)
    if tile == 0:  # planes above 256 hits went through the second (512) tile
        assert np.any(st[8:8 + b.n_events] & velo_mod.EV_SECOND_TILE)


@pytest.fixture(scope="module")
def dense():
    w = gen.Workload("dense", 2, 4321, "uniform", trk_lo=1500, trk_hi=2500, ms_sigma=1e-3, noise_p=5e-4)
    b = gen.generate(w)
    cut = cuts("ms")
    c, t = oracle_run(b, cut)
    return b, cut, c, t


@pytest.mark.parametrize("tile", [1, 2])
def test_large_event_path_on_dense_events(velo_mod, dense, tile):
    # tile 1: the second LDS pass refuses them too; tile 2: straight to global memory
    say(f"[parity] dense events (large path), tile {tile}")
    b, cut, c, t = dense
    v = velo_mod.Velo(b.plane_z, cut)
    v.set_launch(512, tile)
    v.reserve(b.n_events, b.n_pix, b.n_pix)
    off, ids = velo_mod.to_device(b)
    bufs = v.pipeline_buffers(b.n_events, b.n_pix)
    v.pipeline(off, ids, bufs)
    torch.cuda.synchronize()
    st = v.read_status(bufs["status"])
    assert st[0] == 0 and st[5] == 2, st[:8]
    assert_clusters_equal(bufs, c, b.n_pix)
    assert_tracks_equal(bufs, t, check_flags=True)


def test_edge_cases_empty_and_sparse_events(velo_mod):
    # event 0 empty, event 1 a single pixel, event 2 one plane only, event 3 a normal event
    e3 = make("tiny", 1)
    keys = [(1 * 26 + 5) << 22 | 1000, (2 * 26 + 7) << 22 | 5000, (2 * 26 + 7) << 22 | 5001]
    keys += [int((3 * 26) << 22) + int(k) for k in (((np.repeat(np.arange(26), np.diff(e3.pix_off)).astype(np.int64)) << 22) | e3.pix_id.astype(np.int64))]
    b = gen.from_keys(keys, [0] * len(keys), [0, 0, 0, 20], n_events=4)
    cut = cuts("default")
    c, t = oracle_run(b, cut)
    v = velo_mod.Velo(b.plane_z, cut)
    v.reserve(b.n_events, b.n_pix, b.n_pix)
    off, ids = velo_mod.to_device(b)
    bufs = v.pipeline_buffers(b.n_events, b.n_pix)
    v.pipeline(off, ids, bufs)
    torch.cuda.synchronize()
    assert_clusters_equal(bufs, c, b.n_pix)
    assert_tracks_equal(bufs, t)
    assert np_(bufs["trk_off"]).tolist()[:4] == [0, 0, 0, 0]


def test_cluster_capacity_overflow_reports_required_size(velo_mod):
    b = make("tiny", 10)
    cut = cuts("default")
    c, _ = oracle_run(b, cut)
    v = velo_mod.Velo(b.plane_z, cut)
    v.reserve(b.n_events, b.n_pix, b.n_pix)
    off, ids = velo_mod.to_device(b)
    gc = v.cluster(off, ids, clu_cap=50)
    torch.cuda.synchronize()
    st = v.read_status(gc["status"])
    assert st[0] == 1 and st[1] == int(c["clu_off"][-1])
    assert np.array_equal(np_(gc["clu_off"]), c["clu_off"])  # offsets complete and exact


def test_validate_mode_flags_malformed_segments(velo_mod):
    b = make("tiny", 3)
    ids = b.pix_id.copy()
    s = b.pix_off[26 + 15]  # event 1, plane 15: swap two ids
    assert b.pix_off[26 + 16] - s >= 2
    ids[s], ids[s + 1] = ids[s + 1], ids[s]
    # event 2: one pixel moved into the central hole, between its neighbours'
    # ids so that the segment stays strictly ascending
    hole = np.array([r * 1454 + c for r in range(630, 824) for c in range(630, 824)
                     if (2 * c - 1453) ** 2 + (2 * r - 1453) ** 2 < 33058])
    moved = False
    for p in range(26):
        lo, hi = b.pix_off[2 * 26 + p], b.pix_off[2 * 26 + p + 1]
        for i in range(lo + 1, hi - 1):
            inside = hole[(hole > ids[i - 1]) & (hole < ids[i + 1])]
            if inside.size:
                ids[i] = inside[0]
                moved = True
                break
        if moved:
            break
    assert moved
    b.pix_id = ids
    v = velo_mod.Velo(b.plane_z, cuts("default"))
    v.set_validate(True)
    v.reserve(b.n_events, b.n_pix, b.n_pix)
    off, idt = velo_mod.to_device(b)
    gc = v.cluster(off, idt)
    torch.cuda.synchronize()
    st = v.read_status(gc["status"])
    assert st[0] == 2 and st[8 + 1] & 2 and st[8 + 2] & 2 and not (st[8] & 2)
