"""GPU seed-level filter (velo_seed_filter_set / velo_seed_emit) against the oracle.

Bit-exact: the emitted seed candidates of the plain finder are the oracle's
candidates of every step, with the oracle's FP32 features; with a network
switched on, the tracks (CSR hit lists, plane masks, flags) equal the oracle's
run with the same network, on the LDS-tile path (every launch configuration),
the large-event path and the graph-captured pipeline, and switching the filter
off and on again gives the plain and the filtered oracle results in turn.  With
the learned track filter on as well, the candidates stay bit-exact and the
acceptance decisions agree away from the band edge.

The network is a fixed He-uniform draw with fixed feature scales; its
threshold is the 70 % quantile of the oracle's own logits on the oracle's
candidates, so that about a third of the seeds is dropped.
"""
import sys

import numpy as np
import pytest

import oracle
from gpu_helpers import assert_tracks_equal, cuts, np_
from paper_2412_05041_amd import gen, learned

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

# fixed feature scales (means, standard deviations) of the ten seed features
NORM = np.array([0.05, 0.3, 0.0, 300.0, 0.02, 0.9, 12.0, 100.0, 100.0, 100.0,
                 0.1, 0.5, 300.0, 300.0, 0.03, 0.1, 7.0, 100.0, 100.0, 100.0], np.float32)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def velo_mod():
    from paper_2412_05041_amd import velo
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return velo


def make(name, n, seed=None):
    w = gen.WORKLOADS[name]
    return gen.generate(w if n is None else w.with_events(n, seed if seed is not None else w.seed))


def oracle_candidates(c, plane_z, cut, events):
    """The plain oracle's seed candidates of every step of the given events, as global triplets."""
    rows = []
    for e in events:
        t = oracle.find_tracks(c["clu_off"], c["clu_x"], c["clu_y"], plane_z, cut, dbg_event=e, dbg_step=-2)
        rows.append(t["dbg_cand"][:, 1:].astype(np.int64) + int(c["clu_off"][e * 26]))
    return np.concatenate(rows) if rows else np.zeros((0, 3), np.int64)


def network(c, plane_z, cut):
    w = learned.he_uniform(2024)
    h = oracle_candidates(c, plane_z, cut, range(min(3, (c["clu_off"].size - 1) // 26)))
    f = oracle.seed_features(h, c["clu_off"], c["clu_x"], c["clu_y"], plane_z)
    z = oracle.seed_logit(f, (w, NORM, 0.0))
    return w, NORM, float(np.quantile(z, 0.7))


def gpu_tracks(v, b, velo_mod, emit_cap=0):
    off, ids = velo_mod.to_device(b)
    gc = v.cluster(off, ids)
    buf = v.seed_emit(emit_cap) if emit_cap else None
    gt = v.find_tracks(gc["clu_off"], gc["clu_x"], gc["clu_y"], n_clu=b.n_pix)
    torch.cuda.synchronize()
    if emit_cap:
        v.seed_emit(0)
    return gc, gt, buf


@pytest.mark.parametrize("name,n,cutname", [("tiny", 40, "default"), ("nominal", 30, "ms")])
def test_emitted_candidates_are_the_oracle_candidates(velo_mod, name, n, cutname):
    say(f"[seed] emission {name}")
    b = make(name, n)
    cut = cuts(cutname)
    c = oracle.cluster(b.pix_off, b.pix_id)
    ref = oracle_candidates(c, b.plane_z, cut, range(b.n_events))
    v = velo_mod.Velo(b.plane_z, cut)
    v.reserve(b.n_events, b.n_pix, b.n_pix)
    gc, gt, buf = gpu_tracks(v, b, velo_mod, emit_cap=len(ref) + 1000)
    assert v.read_status(gt["status"])[0] == 0
    m = int(buf["count"][0].item())
    assert m == len(ref)
    hits = np_(buf["hits"], m).astype(np.int64)
    feat = np_(buf["feat"], m)
    o = np.lexsort(hits.T[::-1])
    r = np.lexsort(ref.T[::-1])
    assert np.array_equal(hits[o], ref[r])
    f_ref = oracle.seed_features(ref[r], c["clu_off"], c["clu_x"], c["clu_y"], b.plane_z)
    assert np.array_equal(feat[o].view(np.int32), f_ref.view(np.int32))


CASES = [("tiny", None, "default"), ("nominal", 200, "ms"), ("uneven", 600, "default"),
         ("nominal_literal_noise", 2, "ms")]


@pytest.mark.parametrize("name,n,cutname", CASES)
def test_filtered_tracks_match_oracle(velo_mod, name, n, cutname):
    say(f"[seed] filter {name} n={n}")
    b = make(name, n)
    cut = cuts(cutname)
    c = oracle.cluster(b.pix_off, b.pix_id)
    net = network(c, b.plane_z, cut)
    t = oracle.find_tracks(c["clu_off"], c["clu_x"], c["clu_y"], b.plane_z, cut, seed=net)
    plain = oracle.find_tracks(c["clu_off"], c["clu_x"], c["clu_y"], b.plane_z, cut)
    assert t["stats"][3] > 0
    v = velo_mod.Velo(b.plane_z, cut)
    v.reserve(b.n_events, b.n_pix, b.n_pix)
    v.seed_filter_set(*net)
    gc, gt, _ = gpu_tracks(v, b, velo_mod)
    st = v.read_status(gt["status"])
    assert st[0] == 0, st[:8]
    assert_tracks_equal(gt, t, check_flags=True)
    if name == "nominal_literal_noise":
        assert st[5] == b.n_events  # the large-event path ran
    say(f"[seed] {name}: {len(t['trk_planes'])} tracks (plain {len(plain['trk_planes'])}), "
        f"{t['stats'][3]} of {t['stats'][2]} seeds dropped")


@pytest.mark.parametrize("threads", [64, 128, 256, 512])
@pytest.mark.parametrize("tile", [0, 1, 2])
def test_every_launch_configuration_with_the_filter(velo_mod, threads, tile):
    b = make("nominal", 60, 77)
    cut = cuts("ms")
    c = oracle.cluster(b.pix_off, b.pix_id)
    net = network(c, b.plane_z, cut)
    t = oracle.find_tracks(c["clu_off"], c["clu_x"], c["clu_y"], b.plane_z, cut, seed=net)
    v = velo_mod.Velo(b.plane_z, cut)
    v.reserve(b.n_events, b.n_pix, b.n_pix)
    v.set_launch(threads, tile)
    v.seed_filter_set(*net)
    gc, gt, _ = gpu_tracks(v, b, velo_mod)
    assert v.read_status(gt["status"])[0] == 0
    assert_tracks_equal(gt, t, check_flags=True)


def test_pipeline_switches_the_filter(velo_mod):
    say("[seed] pipeline toggle")
    b = make("nominal", 100, 78)
    cut = cuts("ms")
    c = oracle.cluster(b.pix_off, b.pix_id)
    net = network(c, b.plane_z, cut)
    t_f = oracle.find_tracks(c["clu_off"], c["clu_x"], c["clu_y"], b.plane_z, cut, seed=net)
    t_p = oracle.find_tracks(c["clu_off"], c["clu_x"], c["clu_y"], b.plane_z, cut)
    v = velo_mod.Velo(b.plane_z, cut)
    v.reserve(b.n_events, b.n_pix, b.n_pix)
    off, ids = velo_mod.to_device(b)
    bufs = v.pipeline_buffers(b.n_events, b.n_pix)
    for on, ref in ((True, t_f), (True, t_f), (False, t_p), (True, t_f)):
        v.seed_filter_set(*net) if on else v.seed_filter_set(None)
        bufs["trk_hit"].fill_(-7)
        v.pipeline(off, ids, bufs)
        torch.cuda.synchronize()
        assert v.read_status(bufs["status"])[0] == 0
        assert_tracks_equal(bufs, ref, check_flags=True)


def test_seed_filter_with_the_learned_acceptance(velo_mod):
    """Both networks at once: the seed filter decides which candidates exist
    (bit-exact), the BF16 track network then decides acceptance (logits within
    the track network's tolerance, decisions equal away from the band edge)."""
    b = make("nominal", 40, 51)
    cut = dict(cuts("ms"), mode=1, logit_band=0.1)
    c = oracle.cluster(b.pix_off, b.pix_id)
    seed = network(c, b.plane_z, cuts("ms"))
    rng = np.random.default_rng(52)
    master = rng.normal(0, 0.5, 1441).astype(np.float32)
    norm = np.concatenate([[50, 8, 0, 0, 5, 5, 5, 5, 0.6, 0.8],
                           [100, 4, 0.1, 0.1, 5, 5, 10, 10, 0.2, 0.2]]).astype(np.float32)
    t = oracle.find_tracks(c["clu_off"], c["clu_x"], c["clu_y"], b.plane_z, cut, mlp=(master, norm),
                           emit_rejected=True, seed=seed)
    assert t["stats"][3] > 0
    v = velo_mod.Velo(b.plane_z, cut)
    v.mlp_set_weights(master, norm)
    v.seed_filter_set(*seed)
    v.reserve(b.n_events, b.n_pix, b.n_pix)
    off, ids = velo_mod.to_device(b)
    gc = v.cluster(off, ids)
    gt = v.find_tracks(gc["clu_off"], gc["clu_x"], gc["clu_y"], emit_rejected=True)
    torch.cuda.synchronize()
    T = len(t["trk_planes"])
    H = int(t["trk_hit_off"][-1])
    assert np.array_equal(np_(gt["trk_off"]), t["trk_off"])
    assert np.array_equal(np_(gt["trk_hit"], H), t["trk_hit"])
    assert np.array_equal(np_(gt["trk_planes"], T, np.uint32), t["trk_planes"])
    z, zo = np_(gt["trk_logit"], T), t["trk_logit"]
    assert np.all(np.abs(z - zo) <= 2e-2 * np.maximum(1.0, np.abs(zo)))
    sure = np.abs(zo) > 0.1 + 2e-2
    assert np.array_equal(np_(gt["trk_flags"], T)[sure] & 0x0f, t["trk_flags"][sure] & 0x0f)
