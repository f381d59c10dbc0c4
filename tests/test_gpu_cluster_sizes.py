"""Clustering at the segment sizes where the device changes method.

A segment of at most 512 pixels is clustered by one wave in LDS, a larger one
by a 256-thread workgroup: in LDS up to 2048 pixels, through global memory
above.  One batch holds segments on both sides of each boundary, scattered
small clusters and solid blocks (one component of 512, 2048 and 3000 pixels,
the largest pixel counts and coordinate sums each method packs); pixel labels,
offsets, centroid bits and pixel counts must equal the oracle's.  Validate
mode must flag malformed segments of both large-segment methods, and only
their events.
"""
import sys

import numpy as np
import pytest

import oracle
from gpu_helpers import assert_clusters_equal, cuts
from paper_2412_05041_amd import gen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SIDE = gen.N_SIDE
SIZES = [0, 1, 2, 63, 64, 65, 511, 512, 513, 700, 1023, 1024, 2047, 2048, 2049, 3000, 6000]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def velo_mod():
    from paper_2412_05041_amd import velo
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return velo


def scattered(rng, n, avoid_row=None):
    """n distinct sensor pixel ids (ascending) made of small 8-connected
    clusters of 1-4 pixels at random places."""
    ids = set()
    offs = [(0, 1), (1, 0), (1, 1), (1, -1)]
    while len(ids) < n:
        c, r = int(rng.integers(0, SIDE)), int(rng.integers(0, SIDE))
        k = int(rng.integers(1, 5))
        cand = [(c, r)] + [(c + dc, r + dr) for dc, dr in offs[: k - 1]]
        for cc, rr in cand:
            if avoid_row is not None and rr == avoid_row:
                continue
            if gen.pixel_exists(cc, rr) and len(ids) < n:
                ids.add(rr * SIDE + cc)
    return np.array(sorted(ids), np.uint32)


def block(c0, r0, w, h):
    """A solid w x h block of pixels (one component)."""
    return np.array(sorted(r * SIDE + c for r in range(r0, r0 + h) for c in range(c0, c0 + w)), np.uint32)


def batch(segments):
    """Events x 26 planes from a list of per-segment id arrays (padded with
    empty planes to whole events)."""
    n_ev = (len(segments) + 25) // 26
    segs = list(segments) + [np.zeros(0, np.uint32)] * (n_ev * 26 - len(segments))
    off = np.zeros(len(segs) + 1, np.int32)
    off[1:] = np.cumsum([s.size for s in segs])
    return n_ev, off, np.concatenate(segs).astype(np.uint32)


def run(velo_mod, n_ev, off, ids, validate=False):
    v = velo_mod.Velo(gen.plane_z(), cuts("default"))
    v.set_validate(validate)
    v.reserve(n_ev, int(off[-1]), int(off[-1]))
    d_off = torch.from_numpy(off).cuda()
    d_ids = torch.from_numpy(ids.view(np.int32)).cuda()
    g = v.cluster(d_off, d_ids)
    torch.cuda.synchronize()
    return g, v.read_status(g["status"])


def test_segments_across_the_method_boundaries_match_the_oracle(velo_mod):
    rng = np.random.default_rng(2412)
    segs = [scattered(rng, n) for n in SIZES]
    segs += [block(100, 100, 32, 16),   # one 512-pixel component: the one-wave path
             block(100, 100, 64, 32),   # one 2048-pixel component: the workgroup in LDS
             block(100, 100, 60, 50)]   # one 3000-pixel component: the workgroup through global memory
    n_ev, off, ids = batch(segs)
    say("segment sizes", [int(s.size) for s in segs])
    g, st = run(velo_mod, n_ev, off, ids)
    assert st[0] == 0, st[:8]
    c = oracle.cluster(off, ids)
    assert_clusters_equal(g, c, int(off[-1]))
    # the solid blocks are single clusters of their full size
    n_clu = np.diff(c["clu_off"])
    for k, s in enumerate(segs[len(SIZES):]):
        seg = len(SIZES) + k
        assert n_clu[seg] == 1 and c["clu_npix"][c["clu_off"][seg]] == s.size


def hole_segment(rng, n):
    """n ascending valid ids with one pixel replaced by a pixel of the central
    hole, keeping the order strict."""
    row = SIDE // 2
    base = scattered(rng, n - 3, avoid_row=row)
    left, mid, right = row * SIDE + 600, row * SIDE + 610, row * SIDE + 860
    assert gen.pixel_exists(600, row) and gen.pixel_exists(610, row) and gen.pixel_exists(860, row)
    ids = np.array(sorted(set(base.tolist()) | {left, mid, right}), np.uint32)
    i = int(np.searchsorted(ids, mid))
    ids[i] = row * SIDE + SIDE // 2  # inside the hole, between left and right
    assert not gen.pixel_exists(SIDE // 2, row)
    assert np.all(np.diff(ids.astype(np.int64)) > 0)
    return ids


@pytest.mark.parametrize("n", [700, 2600])
def test_validate_mode_flags_large_malformed_segments(velo_mod, n):
    rng = np.random.default_rng(n)
    swapped = scattered(rng, n)
    swapped[[n // 2, n // 2 + 1]] = swapped[[n // 2 + 1, n // 2]]
    segs = [np.zeros(0, np.uint32)] * 26 * 3
    segs[0 * 26 + 7] = swapped                  # event 0: order broken
    segs[1 * 26 + 12] = hole_segment(rng, n)    # event 1: a pixel in the hole
    segs[2 * 26 + 3] = scattered(rng, n)        # event 2: valid
    n_ev, off, ids = batch(segs)
    g, st = run(velo_mod, n_ev, off, ids, validate=True)
    assert st[0] == 2, st[:8]
    assert st[8 + 0] & 2 and st[8 + 1] & 2 and not (st[8 + 2] & 2), st[8:11]
    # the valid event is clustered as the oracle clusters it
    c = oracle.cluster(off[2 * 26:3 * 26 + 1] - off[2 * 26], ids[off[2 * 26]:off[3 * 26]])
    lo, hi = int(off[2 * 26]), int(off[3 * 26])
    d_clu = g["pix_clu"][lo:hi].cpu().numpy()
    c0 = int(g["clu_off"][2 * 26].item())
    assert np.array_equal(d_clu - c0, c["pix_clu"])
