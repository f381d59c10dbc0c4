"""GPU decode of the synthetic super-pixel banks (velo_decode) against the oracle.

Bit-exact: offsets, sorted pixel ids and the per-event flags (bad input,
overflow) on generated banks (LDS path and, for heavy-ion planes above 1024
pixels, the global path), on banks with malformed words and duplicates, and
under a capacity limit.  End to end: decoded pixels through the pipeline give
the tracks of the original pixels.
"""
import sys

import numpy as np
import pytest

import oracle
from gpu_helpers import cuts, np_
from paper_2412_05041_amd import gen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

EV_OVERFLOW, EV_BAD_INPUT = 1, 2


@pytest.fixture(scope="module")
def velo_mod():
    from paper_2412_05041_amd import velo
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return velo


def run(velo_mod, off, bank, E, cap):
    v = velo_mod.Velo(gen.plane_z(), cuts("default"))
    v.reserve(E, max(cap, 1), max(cap, 1))
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    out = v.decode(d(off), d(bank.view(np.int32)), cap)
    st = v.read_status(out["status"])
    return out, st


def compare(velo_mod, off, bank, E, cap=None):
    cap = 8 * bank.size if cap is None else cap
    out, st = run(velo_mod, off, bank, E, cap)
    po, pid, flags, total = oracle.decode(off, bank, E, pix_cap=cap)
    assert np.array_equal(np_(out["pix_off"]), po)
    assert st[4] == total
    ev = st[8:8 + E]
    assert np.array_equal(ev & (EV_OVERFLOW | EV_BAD_INPUT), flags)
    # the planes that were written (the oracle writes the same ones)
    g = np_(out["pix_id"], None, np.uint32)
    for s in range(E * 26):
        a, b = po[s], po[s + 1]
        if b <= cap:
            assert np.array_equal(g[a:b], pid[a:b]), f"plane {s}"
    return out, st


@pytest.mark.parametrize("name,n", [("tiny", None), ("nominal", None), ("heavy_ion", 2)])
def test_decode_generated_banks(velo_mod, name, n):
    print(f"[decode] {name}", file=sys.stderr, flush=True)
    w = gen.WORKLOADS[name]
    b = gen.generate(w if n is None else w.with_events(n, 91))
    off, bank = gen.raw_banks(b, seed=11)
    out, st = compare(velo_mod, off, bank, b.n_events)
    assert st[0] == 0
    assert np.array_equal(np_(out["pix_id"], b.n_pix, np.uint32), b.pix_id)
    if name == "heavy_ion":
        assert np.diff(b.pix_off).max() > 1024  # the global-memory sort ran


def test_decode_malformed_and_duplicates(velo_mod):
    rng = np.random.default_rng(3)
    E = 4
    words = []
    off = np.zeros(E * 26 + 1, np.int32)
    for s in range(E * 26):
        k = int(rng.integers(0, 30))
        pat = rng.integers(0, 256, k)
        spr = rng.integers(0, 366, k)   # a few rows beyond the sensor
        spc = rng.integers(0, 729, k)   # and columns
        extra = (rng.random(k) < 0.02).astype(np.int64)
        wds = pat | (spr << 8) | (spc << 17) | (extra << 27)
        if s % 7 == 0 and k:
            wds = np.concatenate([wds, wds[:1]])  # a repeated word: duplicate pixels
        words.append(wds)
        off[s + 1] = off[s] + len(wds)
    bank = np.concatenate(words).astype(np.uint32)
    out, st = compare(velo_mod, off, bank, E)
    assert st[0] == 2


def test_decode_capacity(velo_mod):
    b = gen.generate(gen.WORKLOADS["nominal"].with_events(6, 5))
    off, bank = gen.raw_banks(b, seed=2)
    out, st = compare(velo_mod, off, bank, 6, cap=b.n_pix - 100)
    assert st[0] == 1


def test_decoded_pixels_give_the_same_tracks(velo_mod):
    b = gen.generate(gen.WORKLOADS["nominal"].with_events(100, 19))
    off, bank = gen.raw_banks(b, seed=4)
    out, st = run(velo_mod, off, bank, b.n_events, b.n_pix)
    assert st[0] == 0
    cut = cuts("ms")
    v = velo_mod.Velo(b.plane_z, cut)
    v.reserve(b.n_events, b.n_pix, b.n_pix)
    ref_off, ref_ids = velo_mod.to_device(b)
    r = v.pipeline_buffers(b.n_events, b.n_pix)
    v.pipeline(ref_off, ref_ids, r)
    ref = {k: np_(r[k]).copy() for k in ("trk_off", "trk_hit_off", "trk_hit", "trk_planes")}
    g = v.pipeline_buffers(b.n_events, b.n_pix)
    v.pipeline(out["pix_off"], out["pix_id"][:b.n_pix], g)
    torch.cuda.synchronize()
    T = int(ref["trk_off"][-1])
    H = int(ref["trk_hit_off"][T])
    assert T > 0
    for k, n in (("trk_off", None), ("trk_hit_off", T + 1), ("trk_hit", H), ("trk_planes", T)):
        assert np.array_equal(np_(g[k], n), ref[k][:n] if n is not None else ref[k]), k
