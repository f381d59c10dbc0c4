"""Pins of the oracle's straight-line fit (least squares in x-z and y-z).

The fit has a closed form, so the pins are numpy.polyfit / lstsq on the same
points, exact lines (zero residual) and a hand-computed chi2.
"""
import numpy as np
import pytest

import oracle
from paper_2412_05041_amd import gen

ZS = gen.plane_z()
SIG = np.float32(0.055 / np.sqrt(12.0))


def tracks_from_points(pts):
    """pts: list of (planes, x, y) -> CSR arrays with hits indexing clu_x/clu_y."""
    xs, ys, off, hits, masks = [], [], [0], [], []
    for planes, x, y in pts:
        order = np.argsort(planes)
        for i in order:
            hits.append(len(xs))
            xs.append(x[i])
            ys.append(y[i])
        off.append(len(hits))
        masks.append(sum(1 << int(p) for p in planes))
    return (np.array(off, np.int32), np.array(hits, np.int32), np.array(masks, np.uint32),
            np.array(xs, np.float32), np.array(ys, np.float32))


@pytest.mark.parametrize("seed", range(4))
def test_fp64_fit_matches_polyfit(seed):
    rng = np.random.default_rng(seed)
    pts = []
    for _ in range(50):
        n = rng.integers(3, 27)
        planes = np.sort(rng.choice(26, n, replace=False))
        z = ZS[planes].astype(np.float64)
        x = (rng.normal(0, 10) + rng.normal(0, 0.1) * z + rng.normal(0, 0.05, n)).astype(np.float32)
        y = (rng.normal(0, 10) + rng.normal(0, 0.1) * z + rng.normal(0, 0.05, n)).astype(np.float32)
        pts.append((planes, x, y))
    off, hits, masks, cx, cy = tracks_from_points(pts)
    par = oracle.fit(off, hits, masks, cx, cy, ZS, SIG, fp64=True)
    for t, (planes, x, y) in enumerate(pts):
        z = ZS[planes].astype(np.float64)
        xd, yd = x.astype(np.float64), y.astype(np.float64)
        px = np.polyfit(z, xd, 1)
        py = np.polyfit(z, yd, 1)
        zr = par[t, 2]
        assert zr == pytest.approx(z.mean(), rel=1e-12, abs=1e-9)
        assert par[t, 3] == pytest.approx(px[0], rel=1e-9, abs=1e-12)
        assert par[t, 4] == pytest.approx(py[0], rel=1e-9, abs=1e-12)
        assert par[t, 0] == pytest.approx(np.polyval(px, zr), rel=1e-9, abs=1e-9)
        assert par[t, 1] == pytest.approx(np.polyval(py, zr), rel=1e-9, abs=1e-9)
        res = np.concatenate([xd - np.polyval(px, z), yd - np.polyval(py, z)])
        assert par[t, 5] == pytest.approx((res ** 2).sum() / float(SIG) ** 2, rel=1e-7, abs=1e-9)
        assert par[t, 6] == 2 * len(planes) - 4


def test_exact_line_has_zero_chi2_fp64():
    planes = np.arange(5, 20)
    z = ZS[planes].astype(np.float64)
    # x, y exactly representable on a line: choose slopes that are powers of two
    x = (1.0 + 0.125 * (z - z.mean())).astype(np.float32)
    y = (-3.0 + 0.0625 * (z - z.mean())).astype(np.float32)
    off, hits, masks, cx, cy = tracks_from_points([(planes, x, y)])
    par = oracle.fit(off, hits, masks, cx, cy, ZS, SIG, fp64=True)
    assert par[0, 5] < 1e-6
    assert par[0, 3] == pytest.approx(0.125, rel=1e-6)
    assert par[0, 4] == pytest.approx(0.0625, rel=1e-6)


def test_hand_chi2_three_points():
    # points at +-e about the line x = 0, y = 0 on three planes; closed form chi2
    planes = np.array([3, 4, 5])
    e = 0.01
    x = np.array([e, -2 * e, e], np.float32)  # fits exactly a residual pattern when z symmetric
    y = np.zeros(3, np.float32)
    off, hits, masks, cx, cy = tracks_from_points([(planes, x, y)])
    par = oracle.fit(off, hits, masks, cx, cy, ZS, SIG, fp64=True)
    z = ZS[planes].astype(np.float64)
    A = np.column_stack([np.ones(3), z])
    sol, res, *_ = np.linalg.lstsq(A, x.astype(np.float64), rcond=None)
    assert par[0, 5] == pytest.approx(res[0] / float(SIG) ** 2, rel=1e-9)
    assert par[0, 6] == 2


def test_fp32_fit_close_to_fp64():
    rng = np.random.default_rng(9)
    pts = []
    for _ in range(200):
        n = rng.integers(3, 27)
        planes = np.sort(rng.choice(26, n, replace=False))
        z = ZS[planes].astype(np.float64)
        x = (rng.uniform(-30, 30) + rng.uniform(-0.2, 0.2) * z).astype(np.float32)
        y = (rng.uniform(-30, 30) + rng.uniform(-0.2, 0.2) * z).astype(np.float32)
        pts.append((planes, x, y))
    off, hits, masks, cx, cy = tracks_from_points(pts)
    p64 = oracle.fit(off, hits, masks, cx, cy, ZS, SIG, fp64=True)
    p32 = oracle.fit(off, hits, masks, cx, cy, ZS, SIG, fp64=False)
    # position of the fitted line at the FP32 reference z
    x64 = p64[:, 0] + p64[:, 3] * (p32[:, 2] - p64[:, 2])
    y64 = p64[:, 1] + p64[:, 4] * (p32[:, 2] - p64[:, 2])
    scale = np.hypot(x64, y64)
    assert np.all(np.abs(p32[:, 0] - x64) <= 1e-5 * np.maximum(scale, 1.0))
    assert np.all(np.abs(p32[:, 1] - y64) <= 1e-5 * np.maximum(scale, 1.0))
    tscale = np.hypot(p64[:, 3], p64[:, 4])
    assert np.all(np.abs(p32[:, 3] - p64[:, 3]) <= 1e-5 * tscale)
    assert np.all(np.abs(p32[:, 4] - p64[:, 4]) <= 1e-5 * tscale)
