"""Oracle Kalman fit (straight VELO segment, multiple-scattering slope noise).

Pins, each independent of the filter's recursion:
  * zero noise: the filter is the least-squares line -- its state at the most
    upstream hit equals the oracle's LS fit evaluated there (slope, position,
    chi2), and its covariance equals the LS closed forms
    Var(t) = s^2/Szz, Var(x(z_f)) = s^2 (1/n + (z_f - zbar)^2/Szz),
    Cov = s^2 (z_f - zbar)/Szz;
  * with noise: a Kalman filter of a linear Gaussian model is generalised
    least squares -- numpy GLS over the whole track (measurement covariance
    sigma^2 I + ms^2 B B^T, B the kick lever arms) gives the same state,
    covariance and chi2;
  * FP32 close to FP64; covariances positive definite.
"""
import numpy as np
import pytest

import oracle
from paper_2412_05041_amd import gen

ZS = gen.plane_z().astype(np.float64)
SIGMA = float(np.float32(0.055 / np.sqrt(12.0)))


def one_track(planes, x, y):
    planes = np.asarray(planes)
    off = np.array([0, len(planes)], np.int32)
    hits = np.arange(len(planes), dtype=np.int32)
    mask = np.array([int(sum(1 << int(k) for k in planes))], np.uint32)
    return off, hits, mask, np.asarray(x, np.float32), np.asarray(y, np.float32)


def gls(planes, u, sigma, ms):
    """State (position at the first hit, slope just downstream of it), its
    covariance and the chi2, by generalised least squares over all hits."""
    planes = np.asarray(planes)
    z = ZS[planes]
    zf = z[0]
    n = len(planes)
    A = np.stack([np.ones(n), z - zf], 1)
    kicks = list(range(planes[0] + 1, planes[-1]))
    B = np.zeros((n, max(len(kicks), 1)))
    for i in range(n):
        for j, q in enumerate(kicks):
            if planes[0] < q < planes[i]:
                B[i, j] = z[i] - ZS[q]
    V = sigma ** 2 * np.eye(n) + ms ** 2 * B @ B.T
    Vi = np.linalg.inv(V)
    cov = np.linalg.inv(A.T @ Vi @ A)
    th = cov @ A.T @ Vi @ u
    r = u - A @ th
    return th, cov, float(r @ Vi @ r)


def random_tracks(rng, count, min_hits=3):
    out = []
    for _ in range(count):
        n = int(rng.integers(min_hits, 12))
        planes = np.sort(rng.choice(26, n, replace=False))
        x0, y0 = rng.uniform(-30, 30, 2)
        tx, ty = rng.uniform(-0.2, 0.2, 2)
        z = ZS[planes]
        x = (x0 + tx * (z - z[0]) + rng.normal(0, 0.05, n)).astype(np.float32)
        y = (y0 + ty * (z - z[0]) + rng.normal(0, 0.05, n)).astype(np.float32)
        out.append((planes, x, y))
    return out


@pytest.mark.parametrize("seed", range(3))
def test_zero_noise_is_the_least_squares_line(seed):
    rng = np.random.default_rng(seed)
    for planes, x, y in random_tracks(rng, 40):
        off, hits, mask, cx, cy = one_track(planes, x, y)
        k = oracle.kalman(off, hits, mask, cx, cy, ZS.astype(np.float32), SIGMA, 0.0)[0]
        f = oracle.fit(off, hits, mask, cx, cy, ZS.astype(np.float32), SIGMA)[0]
        zf = ZS[planes[0]]
        assert k[4] == zf
        assert np.isclose(k[2], f[3], rtol=1e-9, atol=1e-12) and np.isclose(k[3], f[4], rtol=1e-9, atol=1e-12)
        assert np.isclose(k[0], f[0] + f[3] * (zf - f[2]), rtol=1e-9, atol=1e-9)
        assert np.isclose(k[1], f[1] + f[4] * (zf - f[2]), rtol=1e-9, atol=1e-9)
        assert np.isclose(k[11], f[5], rtol=1e-8, atol=1e-9)
        assert k[12] == f[6] == 2 * len(planes) - 4
        z = ZS[planes]
        zbar, szz, n, s2 = z.mean(), ((z - z.mean()) ** 2).sum(), len(planes), SIGMA ** 2
        for c0 in (5, 8):  # x and y projections
            assert np.isclose(k[c0 + 2], s2 / szz, rtol=1e-9)
            assert np.isclose(k[c0], s2 * (1.0 / n + (zf - zbar) ** 2 / szz), rtol=1e-9)
            assert np.isclose(k[c0 + 1], s2 * (zf - zbar) / szz, rtol=1e-8, atol=1e-15)


@pytest.mark.parametrize("ms", [1e-4, 1e-3, 5e-3])
def test_noise_equals_generalised_least_squares(ms):
    rng = np.random.default_rng(int(ms * 1e5))
    for planes, x, y in random_tracks(rng, 40):
        off, hits, mask, cx, cy = one_track(planes, x, y)
        k = oracle.kalman(off, hits, mask, cx, cy, ZS.astype(np.float32), SIGMA, ms)[0]
        chi2 = 0.0
        for u, c0, xi, ti in ((cx, 5, 0, 2), (cy, 8, 1, 3)):
            th, cov, c2 = gls(planes, u.astype(np.float64), SIGMA, float(np.float32(ms)))
            assert np.isclose(k[xi], th[0], rtol=1e-9, atol=1e-9)
            assert np.isclose(k[ti], th[1], rtol=1e-8, atol=1e-11)
            assert np.isclose(k[c0], cov[0, 0], rtol=1e-7)
            assert np.isclose(k[c0 + 1], cov[0, 1], rtol=1e-6, atol=1e-14)
            assert np.isclose(k[c0 + 2], cov[1, 1], rtol=1e-7)
            chi2 += c2
        assert np.isclose(k[11], chi2, rtol=1e-7, atol=1e-9)


def test_fp32_close_to_fp64_and_positive_definite():
    rng = np.random.default_rng(9)
    tr = random_tracks(rng, 200)
    for planes, x, y in tr:
        off, hits, mask, cx, cy = one_track(planes, x, y)
        k64 = oracle.kalman(off, hits, mask, cx, cy, ZS.astype(np.float32), SIGMA, 1e-3)[0]
        k32 = oracle.kalman(off, hits, mask, cx, cy, ZS.astype(np.float32), SIGMA, 1e-3, fp64=False)[0]
        for c0 in (5, 8):
            assert k64[c0] > 0 and k64[c0 + 2] > 0 and k64[c0] * k64[c0 + 2] > k64[c0 + 1] ** 2
        assert abs(k32[0] - k64[0]) <= 1e-5 * max(abs(k64[0]), 1.0)
        assert abs(k32[2] - k64[2]) <= 1e-4 * max(abs(k64[2]), 1e-3)
        assert np.allclose(k32[5:11], k64[5:11], rtol=1e-3)


def test_two_hit_track_is_its_initialisation():
    planes, x, y = [4, 7], [1.0, 1.5], [2.0, 2.2]
    off, hits, mask, cx, cy = one_track(planes, x, y)
    k = oracle.kalman(off, hits, mask, cx, cy, ZS.astype(np.float32), SIGMA, 1e-3)[0]
    D = ZS[7] - ZS[4]
    assert k[0] == np.float32(1.0) and np.isclose(k[2], (np.float32(1.5) - np.float32(1.0)) / D)
    assert k[11] == 0.0 and k[12] == 0
