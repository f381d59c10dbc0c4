"""Oracle of the forward extrapolation through a single-kink magnet.

Pins: a hand-worked example; a track of q/p = 0 follows its straight line and
gets q/p 0 back; hits built from the two-segment picture (straight to z_mag,
then the kinked slope) give back the q/p they were built with, and q/p =
+-1/p_min lands exactly on the window edges; the same line given at another
z gives the same outputs.
"""
import numpy as np

import oracle

ZM, ZT, KICK, PMIN = 5000.0, 8000.0, 1.0, 2.0


def states(n, seed):
    rng = np.random.default_rng(seed)
    p = np.zeros((n, 8), np.float32)
    p[:, 0] = rng.uniform(-40, 40, n)
    p[:, 1] = rng.uniform(-40, 40, n)
    p[:, 2] = rng.uniform(-300, 750, n)
    p[:, 3] = rng.uniform(-0.3, 0.3, n)
    p[:, 4] = rng.uniform(-0.3, 0.3, n)
    return p


def test_hand_example():
    p = np.array([[1, 2, 0, 0.01, 0.02, 0, 0, 0]], np.float32)
    o = oracle.extrapolate(p, np.array([81.0 + 3000.0 * 0.25], np.float32), ZM, ZT, KICK, PMIN)[0]
    tx = float(np.float32(0.01))
    ty = float(np.float32(0.02))
    assert np.isclose(o[0], 1 + tx * 5000) and np.isclose(o[1], 2 + ty * 5000)
    assert np.isclose(o[2], 1 + tx * 8000) and np.isclose(o[3], 2 + ty * 8000)
    assert np.isclose(o[4], o[2] - 1500) and np.isclose(o[5], o[2] + 1500)
    # x_hit 750 mm beyond x = 81: slope change 0.25 over 3000 mm, q/p = 0.25 / kick
    assert np.isclose(o[6], (81.0 + 750.0 - o[2]) / 3000.0, rtol=1e-6)
    assert np.isclose(o[7], tx + o[6])


def segments_hit(p, qop):
    """x at z_t of the two-segment trajectory, float64."""
    x0, z0, tx = p[:, 0].astype(np.float64), p[:, 2].astype(np.float64), p[:, 3].astype(np.float64)
    x_at_mag = x0 + tx * (ZM - z0)
    return x_at_mag + (tx + KICK * qop) * (ZT - ZM)


def test_round_trip_and_window_edges():
    p = states(500, 1)
    rng = np.random.default_rng(2)
    qop = rng.uniform(-1 / PMIN, 1 / PMIN, 500)
    xh = segments_hit(p, qop).astype(np.float32)
    o = oracle.extrapolate(p, xh, ZM, ZT, KICK, PMIN)
    # x_hit is rounded to FP32: |dq| <= ulp(x_hit) / (lever * kick)
    tol = np.abs(xh).astype(np.float64) * 2.0 ** -23 / (ZT - ZM) / KICK * 2
    assert np.all(np.abs(o[:, 6] - qop) <= tol + 1e-12)
    for sign, col in ((1.0, 5), (-1.0, 4)):
        edge = segments_hit(p, np.full(500, sign / PMIN))
        assert np.allclose(o[:, col], edge, rtol=1e-12, atol=1e-9)


def test_straight_track():
    p = states(200, 3)
    xl = segments_hit(p, np.zeros(200))
    o = oracle.extrapolate(p, None, ZM, ZT, KICK, PMIN)
    assert np.allclose(o[:, 2], xl, rtol=1e-12, atol=1e-9)
    assert np.all(o[:, 6] == 0) and np.array_equal(o[:, 7], p[:, 3].astype(np.float64))
    # y has no kink
    y = p[:, 1].astype(np.float64) + p[:, 4].astype(np.float64) * (ZT - p[:, 2].astype(np.float64))
    assert np.allclose(o[:, 3], y, rtol=1e-12, atol=1e-9)


def test_state_given_at_another_z():
    p = states(100, 4).astype(np.float64)
    q = p.copy()
    q[:, 2] = 0.0  # the same line described at z = 0
    q[:, 0] = p[:, 0] - p[:, 3] * p[:, 2]
    q[:, 1] = p[:, 1] - p[:, 4] * p[:, 2]
    # exact in FP32 inputs only approximately: compare within the rounding of the moved origin
    a = oracle.extrapolate(p.astype(np.float32), None, ZM, ZT, KICK, PMIN)
    b = oracle.extrapolate(q.astype(np.float32), None, ZM, ZT, KICK, PMIN)
    assert np.allclose(a[:, :6], b[:, :6], rtol=0, atol=1e-3)
