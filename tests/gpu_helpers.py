"""Shared helpers of the GPU tests: run the oracle and the HIP path on one batch."""
import json
import os

import numpy as np

import oracle
from paper_2412_05041_amd import gen

CFG = os.path.join(os.path.dirname(__file__), "..", "paper_2412_05041_amd", "configs")
HOLE_RADIUS_MM = 5.0


def cuts(name):
    return json.load(open(os.path.join(CFG, f"cuts_{name}.json")))


def oracle_run(b, cut, emit_rejected=False):
    c = oracle.cluster(b.pix_off, b.pix_id)
    t = oracle.find_tracks(c["clu_off"], c["clu_x"], c["clu_y"], b.plane_z, cut, emit_rejected=emit_rejected)
    return c, t


def np_(t, n=None, dtype=None):
    a = t.detach().cpu().numpy()
    if n is not None:
        a = a[:n]
    if dtype is not None:
        a = a.view(dtype)
    return a


def assert_clusters_equal(gpu, c, n_pix):
    n_clu = int(c["clu_off"][-1])
    assert np.array_equal(np_(gpu["clu_off"]), c["clu_off"]), "clu_off"
    assert np.array_equal(np_(gpu["pix_clu"], n_pix), c["pix_clu"]), "pix_clu"
    assert np.array_equal(np_(gpu["clu_x"], n_clu, np.int32), c["clu_x"].view(np.int32)), "clu_x bits"
    assert np.array_equal(np_(gpu["clu_y"], n_clu, np.int32), c["clu_y"].view(np.int32)), "clu_y bits"
    if gpu.get("clu_npix") is not None:
        assert np.array_equal(np_(gpu["clu_npix"], n_clu), c["clu_npix"]), "clu_npix"


def assert_tracks_equal(gpu, t, check_flags=False):
    T = len(t["trk_planes"])
    H = int(t["trk_hit_off"][-1])
    assert np.array_equal(np_(gpu["trk_off"]), t["trk_off"]), "trk_off"
    assert np.array_equal(np_(gpu["trk_hit_off"], T + 1), t["trk_hit_off"]), "trk_hit_off"
    assert np.array_equal(np_(gpu["trk_hit"], H), t["trk_hit"]), "trk_hit"
    assert np.array_equal(np_(gpu["trk_planes"], T, np.uint32), t["trk_planes"]), "trk_planes"
    if check_flags:
        assert np.array_equal(np_(gpu["trk_flags"], T), t["trk_flags"]), "trk_flags"


def track_scales(t, c):
    """Natural scales of a track's fit: the largest hit radius (positions) and
    the largest hit offset from the centroid over the z span (slopes)."""
    off = np.asarray(t["trk_hit_off"], np.int64)
    T = off.size - 1
    if T == 0:
        return np.zeros(0), np.zeros(0), np.zeros(0, np.int64), np.zeros(0, np.int64)
    hx = c["clu_x"][t["trk_hit"]].astype(np.float64)
    hy = c["clu_y"][t["trk_hit"]].astype(np.float64)
    rmax = np.maximum.reduceat(np.hypot(hx, hy), off[:-1])
    n = np.diff(off)
    cx = np.add.reduceat(hx, off[:-1]) / n
    cy = np.add.reduceat(hy, off[:-1]) / n
    dev = np.maximum.reduceat(np.hypot(hx - np.repeat(cx, n), hy - np.repeat(cy, n)), off[:-1])
    planes = np.asarray(t["trk_planes"], np.int64)
    first = np.array([int(m & -m).bit_length() - 1 for m in planes])
    last = np.array([int(m).bit_length() - 1 for m in planes])
    return rmax, dev, first, last


def assert_fit_close(par32, t, c, plane_z, sigma):
    """FP32 device fit vs the FP64 oracle fit, 1e-5 relative to the state:
    x_ref, y_ref (the FP64 line at the device's z_ref) within 1e-5 of
    max(|(x, y)|, 5 mm) -- 5 mm, the hole radius, is the smallest distance of a
    hit from the axis and so the smallest magnitude the FP32 sums of hit
    coordinates work at (a noise-made track can pass the axis at its centroid);
    tx, ty within 1e-5 of |(tx, ty)|; z_ref within 1e-5 of the largest |z| of its
    planes (a mean of plane positions that may straddle z = 0); ndof exact.
    chi2 within 1e-3 of max(chi2, 1): it sums squared residuals of ~0.01 mm
    taken between coordinates of ~10 mm, so FP32 rounding of the coordinates
    alone moves it by ~1e-4 relative -- 1e-5 is out of reach of any FP32 fit.
    The device fit must also equal the oracle's FP32 fit (same operations,
    same order) bit for bit."""
    p64 = oracle.fit(t["trk_hit_off"], t["trk_hit"], t["trk_planes"], c["clu_x"], c["clu_y"], plane_z, sigma)
    p32o = oracle.fit(t["trk_hit_off"], t["trk_hit"], t["trk_planes"], c["clu_x"], c["clu_y"], plane_z, sigma,
                      fp64=False).astype(np.float32)
    assert np.array_equal(par32[:, :7].view(np.int32), p32o[:, :7].view(np.int32)), "FP32 fit bits"
    p = par32.astype(np.float64)
    _, _, first, last = track_scales(t, c)
    x64 = p64[:, 0] + p64[:, 3] * (p[:, 2] - p64[:, 2])
    y64 = p64[:, 1] + p64[:, 4] * (p[:, 2] - p64[:, 2])
    pscale = np.maximum(np.hypot(x64, y64), HOLE_RADIUS_MM)
    tscale = np.hypot(p64[:, 3], p64[:, 4])
    assert np.all(np.abs(p[:, 0] - x64) <= 1e-5 * pscale), "x_ref"
    assert np.all(np.abs(p[:, 1] - y64) <= 1e-5 * pscale), "y_ref"
    zscale = np.maximum(np.abs(plane_z[first]), np.abs(plane_z[last])).astype(np.float64)
    assert np.all(np.abs(p[:, 2] - p64[:, 2]) <= 1e-5 * zscale), "z_ref"
    assert np.all(np.abs(p[:, 3] - p64[:, 3]) <= 1e-5 * tscale), "tx"
    assert np.all(np.abs(p[:, 4] - p64[:, 4]) <= 1e-5 * tscale), "ty"
    assert np.all(np.abs(p[:, 5] - p64[:, 5]) <= 1e-3 * np.maximum(p64[:, 5], 1.0)), "chi2"
    assert np.array_equal(p[:, 6], p64[:, 6]), "ndof"
    return p64
