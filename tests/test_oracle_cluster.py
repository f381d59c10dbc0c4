"""Pins of the oracle's clustering: 8-connected components of the fired pixels.

The clustering has a plain definition (connected components under
8-connectivity, clusters numbered by their smallest pixel id, binary centroid),
so the pins are a library routine (scipy.ndimage.label), a brute-force
all-pairs union-find, closed-form centroids and hand-built edge cases.
"""
import numpy as np
import pytest
from scipy import ndimage

import oracle
from paper_2412_05041_amd import gen

N = gen.N_SIDE


def one_plane_batch(ids, plane=0):
    ids = np.unique(np.asarray(ids, np.int64))
    off = np.zeros(27, np.int32)
    off[plane + 1:] = ids.size
    return off, ids.astype(np.uint32)


def clusters_as_sets(ids, pix_clu):
    out = {}
    for i, c in zip(ids, pix_clu):
        out.setdefault(int(c), set()).add(int(i))
    return out


@pytest.mark.parametrize("seed,fill", [(1, 0.05), (2, 0.15), (3, 0.3)])
def test_matches_scipy_label_8conn(seed, fill):
    rng = np.random.default_rng(seed)
    h, w = 48, 64
    r0, c0 = 100, 1380  # crop touching the right sensor edge (c = 1453)
    img = rng.random((h, w)) < fill
    img[:, c0 + w - N:] = False if c0 + w > N else img[:, c0 + w - N:]
    rr, cc = np.nonzero(img)
    ok = cc + c0 < N
    rr, cc = rr[ok], cc[ok]
    ids = (rr + r0) * N + (cc + c0)
    off, ids_u = one_plane_batch(ids)
    out = oracle.cluster(off, ids_u)
    lab, nlab = ndimage.label(img, structure=np.ones((3, 3), int))
    # same partition
    ref = {}
    for r, c in zip(rr, cc):
        ref.setdefault(int(lab[r, c]), set()).add(int((r + r0) * N + c + c0))
    got = clusters_as_sets(ids_u, out["pix_clu"])
    assert sorted(map(sorted, got.values())) == sorted(map(sorted, ref.values()))
    assert out["clu_off"][-1] == len(ref)
    # numbering by smallest pixel id
    mins = [min(got[k]) for k in sorted(got)]
    assert mins == sorted(mins)
    # centroid from integer sums, 3 FP32 ops
    for k in sorted(got):
        px = np.array(sorted(got[k]))
        sc, sr, n = int((px % N).sum()), int((px // N).sum()), px.size
        ex = (np.float32(sc) / np.float32(n) - np.float32(726.5)) * np.float32(0.055)
        ey = (np.float32(sr) / np.float32(n) - np.float32(726.5)) * np.float32(0.055)
        assert out["clu_x"][k] == ex and out["clu_y"][k] == ey
        assert out["clu_npix"][k] == n


def brute_components(ids):
    ids = list(ids)
    parent = list(range(len(ids)))

    def f(a):
        while parent[a] != a:
            a = parent[a]
        return a
    for i in range(len(ids)):
        for j in range(len(ids)):
            ci, ri, cj, rj = ids[i] % N, ids[i] // N, ids[j] % N, ids[j] // N
            if i != j and max(abs(ci - cj), abs(ri - rj)) == 1:
                a, b = f(i), f(j)
                if a != b:
                    parent[max(a, b)] = min(a, b)
    comp = {}
    for i in range(len(ids)):
        comp.setdefault(f(i), set()).add(ids[i])
    return sorted(map(sorted, comp.values()))


@pytest.mark.parametrize("seed", range(5))
def test_matches_bruteforce_union_find(seed):
    rng = np.random.default_rng(100 + seed)
    r = rng.integers(700, 712, 40)
    c = rng.integers(0, 12, 40)  # left edge, c = 0 included
    ids = np.unique(r * N + c)
    off, ids_u = one_plane_batch(ids, plane=7)
    out = oracle.cluster(off, ids_u)
    got = sorted(map(sorted, clusters_as_sets(ids_u, out["pix_clu"]).values()))
    assert got == brute_components(ids_u.tolist())


def test_row_wrap_is_not_adjacency():
    # (c=1453, r=5) and (c=0, r=6) have consecutive ids but are far apart
    a, b = 5 * N + 1453, 6 * N + 0
    off, ids = one_plane_batch([a, b])
    out = oracle.cluster(off, ids)
    assert out["clu_off"][-1] == 2
    # and (c=1453, r=5) with (c=1452, r=6) is a diagonal neighbour
    off, ids = one_plane_batch([a, 6 * N + 1452])
    assert oracle.cluster(off, ids)["clu_off"][-1] == 1


def test_diagonal_and_l_shape():
    # diagonal chain -> one cluster; L-shape -> one cluster; a knight's move -> two
    diag = [10 * N + 10, 11 * N + 11, 12 * N + 12]
    ell = [20 * N + 30, 21 * N + 30, 22 * N + 30, 22 * N + 31]
    knight = [40 * N + 40, 41 * N + 42]
    off, ids = one_plane_batch(diag + ell + knight)
    out = oracle.cluster(off, ids)
    assert out["clu_off"][-1] == 4
    assert list(out["clu_npix"]) == [3, 4, 1, 1]


def test_single_pixel_centroid_closed_form():
    for (c, r) in [(0, 0), (1453, 1453), (726, 727), (100, 1200)]:
        off, ids = one_plane_batch([r * N + c])
        out = oracle.cluster(off, ids)
        assert out["clu_x"][0] == (np.float32(c) - np.float32(726.5)) * np.float32(0.055)
        assert out["clu_y"][0] == (np.float32(r) - np.float32(726.5)) * np.float32(0.055)
    # two pixels side by side: half-pixel shift, exact
    off, ids = one_plane_batch([300 * N + 800, 300 * N + 801])
    out = oracle.cluster(off, ids)
    assert out["clu_x"][0] == np.float32((800.5 - 726.5) * 0.055) or \
        out["clu_x"][0] == (np.float32(800.5) - np.float32(726.5)) * np.float32(0.055)


def test_hole_boundary_pixels_cluster_normally():
    # pixels right at the hole boundary, (2c-1453)^2 + (2r-1453)^2 in {33058, ...}
    pts = []
    for c in range(600, 860):
        for r in range(600, 860):
            d2 = (2 * c - 1453) ** 2 + (2 * r - 1453) ** 2
            if 33058 <= d2 < 33058 + 600:
                pts.append(r * N + c)
    assert gen.pixel_exists(np.array(pts) % N, np.array(pts) // N).all()
    off, ids = one_plane_batch(pts)
    out = oracle.cluster(off, ids)
    got = sorted(map(sorted, clusters_as_sets(ids, out["pix_clu"]).values()))
    assert got == brute_components(ids.tolist())


def test_multi_event_offsets_and_global_numbering():
    b = gen.generate(gen.WORKLOADS["tiny"].with_events(7, 77))
    out = oracle.cluster(b.pix_off, b.pix_id)
    co = out["clu_off"]
    assert co[0] == 0 and np.all(np.diff(co) >= 0)
    # every pixel labelled with a cluster of its own (event, plane) segment
    seg = np.repeat(np.arange(7 * 26), np.diff(b.pix_off))
    assert np.all(out["pix_clu"] >= co[seg]) and np.all(out["pix_clu"] < co[seg + 1])
    # sum of cluster sizes = number of pixels
    assert out["clu_npix"].sum() == b.n_pix
    # no two clusters 8-adjacent (maximality), every cluster connected
    for s in range(7 * 26):
        ids = b.pix_id[b.pix_off[s]:b.pix_off[s + 1]]
        lab = out["pix_clu"][b.pix_off[s]:b.pix_off[s + 1]]
        got = sorted(map(sorted, clusters_as_sets(ids, lab).values()))
        assert got == brute_components(ids.tolist())


def test_empty_planes_and_empty_batch():
    off = np.zeros(27, np.int32)
    out = oracle.cluster(off, np.zeros(0, np.uint32))
    assert out["clu_off"][-1] == 0
