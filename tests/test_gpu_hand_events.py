"""GPU vs oracle on hand-built cluster events and on tie-heavy events.

The hand-built events of the oracle's pins (cut boundaries, claiming order,
missing planes) run through velo_find_tracks on explicit cluster coordinates.
Tie-heavy events put every hit on a coarse grid so that many seed candidates
have bit-equal miss distances: the tie-breaks by hit index must agree.
"""
import numpy as np
import pytest

import oracle
from gpu_helpers import assert_tracks_equal, cuts, np_
from paper_2412_05041_amd import gen

import test_oracle_find as hand

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ZS = gen.plane_z()


@pytest.fixture(scope="module")
def velo_mod():
    from paper_2412_05041_amd import velo
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return velo


def run_both(velo_mod, off, x, y, cut, emit=True):
    t = oracle.find_tracks(off, x, y, ZS, cut, emit_rejected=emit)
    v = velo_mod.Velo(ZS, cut)
    E = (off.size - 1) // 26
    n = max(int(off[-1]), 1)
    v.reserve(E, n, n)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    g = v.find_tracks(d(off), d(x), d(y), n_clu=int(off[-1]), emit_rejected=emit)
    torch.cuda.synchronize()
    st = v.read_status(g["status"])
    assert st[0] == 0, st[:8]
    return g, t


HAND = [
    lambda: hand.line_hits((20.0, 5.0), (0.04, 0.01), [k for k in range(8, 26) if k != 15]),
    lambda: hand.line_hits((20.0, 5.0), (0.04, 0.01), [k for k in range(8, 26) if k not in (15, 16)]),
    lambda: hand.doca_line(2.9),
    lambda: hand.doca_line(3.1),
    lambda: hand.three_hit_line((20.0, 0.0), (0.39, 0.0)),
    lambda: hand.three_hit_line((20.0, 0.0), (-0.05, 0.0)),
]


@pytest.mark.parametrize("i", range(len(HAND)))
def test_hand_events(velo_mod, i):
    off, x, y, _ = hand.event_from_hits(HAND[i]())
    g, t = run_both(velo_mod, off, x, y, cuts("default"))
    assert_tracks_equal(g, t, check_flags=True)


def test_equal_miss_distance_tie_break(velo_mod):
    k, zv = 12, -400.0
    z = [float(ZS[k + i]) for i in range(3)]
    A = [(k + i, 0.003 * (z[i] - z[1]), 0.05 * (z[i] - zv)) for i in range(3)]
    B = [(kk, -xx, yy) for (kk, xx, yy) in A]
    for hits in ([A[0], B[0], A[1], A[2], B[2]], [B[0], A[0], A[1], B[2], A[2]]):
        off, x, y, _ = hand.event_from_hits(hits)
        g, t = run_both(velo_mod, off, x, y, cuts("default"))
        assert_tracks_equal(g, t, check_flags=True)


def tie_event(seed, per_plane=60):
    """Hits in a narrow wedge on a 1/8 mm grid, planes 32 mm apart: the line
    midpoints are exact and thousands of seed candidates tie exactly on (q, h0)."""
    rng = np.random.default_rng(seed)
    zs = (np.arange(26) * 32.0 - 300.0).astype(np.float32)
    hits = set()
    for k in range(26):
        for _ in range(per_plane):
            r = rng.uniform(8, 8 + 0.02 * (zs[k] + 300.0) + 2)
            ph = rng.uniform(0.3, 0.5)
            hits.add((k, float(np.round(r * np.cos(ph) * 8) / 8), float(np.round(r * np.sin(ph) * 8) / 8)))
    hits = sorted(hits)
    off = np.zeros(27, np.int32)
    for k, _, _ in hits:
        off[k + 1:] += 1
    return zs, off, np.array([h[1] for h in hits], np.float32), np.array([h[2] for h in hits], np.float32)


@pytest.mark.parametrize("seed", range(4))
def test_exact_tie_heavy_events(velo_mod, seed):
    zs, off, x, y = tie_event(seed)
    cut = dict(cuts("default"), s_max=0.5, d2_max=25.0)
    t = oracle.find_tracks(off, x, y, zs, cut, emit_rejected=True)
    v = velo_mod.Velo(zs, cut)
    n = int(off[-1])
    v.reserve(1, n, n)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    g = v.find_tracks(d(off), d(x), d(y), n_clu=n, emit_rejected=True)
    torch.cuda.synchronize()
    assert v.read_status(g["status"])[0] == 0
    assert_tracks_equal(g, t, check_flags=True)
    assert len(t["trk_planes"]) > 100
