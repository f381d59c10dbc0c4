"""CPU checks of the GPU's parallel formulation (host re-statements, no device).

1. Greedy claiming by rounds of local minima -- the rule the finder kernel runs
   with two-phase atomicMin -- accepts exactly the candidates of the sequential
   greedy over (q, h0, h1, h2).
2. The azimuth-key windows used to prune searches contain every hit that passes
   the exact FP32 cut (brute force over random geometry, float32 arithmetic).
"""
import math

import numpy as np
import pytest

f32 = np.float32


def sequential_greedy(cands):
    used, acc = set(), []
    for c in sorted(cands):
        q, h0, h1, h2 = c
        hs = (("a", h0), ("b", h1), ("c", h2))
        if any(h in used for h in hs):
            continue
        used.update(hs)
        acc.append(c)
    return acc


def rounds_of_local_minima(cands):
    alive = {i: c for i, c in enumerate(cands)}
    used, acc, rounds = set(), [], 0
    while alive:
        rounds += 1
        slot_a, slot_b = {}, {}
        for c in alive.values():  # phase A: (q, h0) min on every hit
            for h in (("a", c[1]), ("b", c[2]), ("c", c[3])):
                slot_a[h] = min(slot_a.get(h, (math.inf, 0)), (c[0], c[1]))
        for c in alive.values():  # phase B: (h1, h2) among the holders of each hit's phase-A minimum
            for h in (("a", c[1]), ("b", c[2]), ("c", c[3])):
                if slot_a[h] == (c[0], c[1]):
                    slot_b[h] = min(slot_b.get(h, (math.inf, 0)), (c[2], c[3]))
        winners = []
        for i, c in alive.items():
            hs = (("a", c[1]), ("b", c[2]), ("c", c[3]))
            if all(slot_a[h] == (c[0], c[1]) for h in hs) and all(slot_b.get(h) == (c[2], c[3]) for h in hs):
                winners.append(i)
        assert winners, "a round must make progress"
        for i in winners:
            c = alive.pop(i)
            used.update((("a", c[1]), ("b", c[2]), ("c", c[3])))
            acc.append(c)
        for i in [i for i, c in alive.items() if (("a", c[1]) in used or ("b", c[2]) in used or ("c", c[3]) in used)]:
            alive.pop(i)
    return sorted(acc), rounds


@pytest.mark.parametrize("seed", range(40))
def test_rounds_equal_sequential_greedy(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 300))
    pool = int(rng.integers(2, 40))
    qs = rng.integers(0, 6, n).astype(float) if seed % 3 == 0 else rng.random(n)  # many exact ties
    cands = sorted({(float(qs[i]), int(rng.integers(pool)), int(rng.integers(pool)), int(rng.integers(pool)))
                    for i in range(n)})
    acc, _ = rounds_of_local_minima(cands)
    assert acc == sorted(sequential_greedy(cands))


# ---------------------------------------------------------------- key windows

KEYS_PER_RAD = f32(10430.378350470453)
PI = f32(3.14159265358979)


def phi_key(x, y):
    u = (np.arctan2(y, x).astype(f32) + PI) * KEYS_PER_RAD
    return np.clip(u.astype(np.int64), 0, 65535)


def disc_keys(R, r):
    """Half-width in keys of asin(R/r) plus margins (None = whole circle)."""
    if not (r > R * 1.001 + 1e-3):
        return None
    return int(math.ceil((math.asin(R / r) * 1.0001 + 2e-4) * float(KEYS_PER_RAD))) + 2


def in_span(k, a, b, m):
    if m is None:
        return True
    lo, hi = a - m, b + m
    return any(lo <= kk <= hi for kk in (k, k - 65536, k + 65536))


def test_seed_windows_contain_every_passing_triplet():
    rng = np.random.default_rng(7)
    D2, S, TMAX = f32(9.0), f32(0.09), f32(0.4)
    R_seed, R_mid = math.sqrt(9.0) * 1.0001 + 1e-6, math.sqrt(0.09) * 1.0001 + 1e-6
    dz1, dz2 = f32(41.5), f32(84.2)
    n = 400000
    # h0 anywhere outside 5 mm; h2 = h0 + t dz2 + jitter (mostly near-pointing lines)
    r0 = rng.uniform(5.0, 40.0, n)
    ph0 = rng.uniform(-math.pi, math.pi, n)
    x0 = (r0 * np.cos(ph0)).astype(f32)
    y0 = (r0 * np.sin(ph0)).astype(f32)
    ang = ph0 + rng.normal(0, 0.25, n)
    tt = rng.uniform(0.0, 0.45, n)
    x2 = (x0 + tt * np.cos(ang) * float(dz2) + rng.normal(0, 0.3, n)).astype(f32)
    y2 = (y0 + tt * np.sin(ang) * float(dz2) + rng.normal(0, 0.3, n)).astype(f32)
    tx = (x2 - x0) / dz2
    ty = (y2 - y0) / dz2
    ok = (np.abs(tx) <= TMAX) & (np.abs(ty) <= TMAX) & (x0 * tx + y0 * ty > 0)
    cr = x0 * ty - y0 * tx
    ok &= cr * cr <= D2 * (tx * tx + ty * ty)
    idx = np.nonzero(ok)[0]
    assert idx.size > 10000
    k0 = phi_key(x0[idx], y0[idx])
    k2 = phi_key(x2[idx], y2[idx])
    ex = x0[idx] + tx[idx] * dz1
    ey = y0[idx] + ty[idx] * dz1
    # middle hits on the boundary of the S3 disc (and inside)
    a1 = rng.uniform(0, 2 * math.pi, idx.size)
    rr = np.sqrt(rng.uniform(0, 1, idx.size)) * 0.3
    x1 = (ex + rr * np.cos(a1)).astype(f32)
    y1 = (ey + rr * np.sin(a1)).astype(f32)
    dx, dy = x1 - ex, y1 - ey
    s3 = dx * dx + dy * dy <= S
    k1 = phi_key(x1, y1)
    for j in range(idx.size):
        rj = math.sqrt(float(x0[idx[j]]) ** 2 + float(y0[idx[j]]) ** 2)
        mD = disc_keys(R_seed, rj)
        assert in_span(int(k2[j]), int(k0[j]), int(k0[j]), mD), j
        if s3[j]:
            kd = int(k2[j]) - int(k0[j])
            kd = kd - 65536 if kd > 32767 else (kd + 65536 if kd < -32768 else kd)
            m1 = disc_keys(R_mid, rj)
            assert in_span(int(k1[j]), int(k0[j]) + min(kd, 0), int(k0[j]) + max(kd, 0), m1), j




def point_windows(ex, ey, R):
    """The extension and middle-hit windows as the finder bounds them (FP32,
    vectorised): the azimuth of E from an octant reduction and the odd
    degree-9 polynomial of Abramowitz & Stegun 4.4.49, the half-angle from
    R / sqrt(|E|^2 - R^2) >= asin(R/|E|) widened by 0.1 %, then 1e-4 rad and
    two keys on each side.  The hardware reciprocal square root is taken one
    part in 2^22 low (it may round either way).  Returns (lo, hi, whole)."""
    ex, ey, R = np.asarray(ex, f32), np.asarray(ey, f32), f32(R)
    e2 = ex * ex + ey * ey
    whole = ~(e2 > f32(4.0) * R * R)
    rsq = (f32(1.0) / np.sqrt(np.maximum(e2 - R * R, f32(1e-30)))).astype(f32) * f32(1.0 - 2.0 ** -22)
    half = R * rsq * f32(1.001) + f32(1e-4)
    ax, ay = np.abs(ex), np.abs(ey)
    t = np.minimum(ax, ay) * (f32(1.0) / np.maximum(np.maximum(ax, ay), f32(1e-30)))
    sq = t * t
    phi = t * (f32(0.9998660) + sq * (f32(-0.3302995) + sq * (f32(0.1801410) + sq * (f32(-0.0851330)
                                                                                   + sq * f32(0.0208351)))))
    phi = np.where(ay > ax, f32(1.57079633) - phi, phi)
    phi = np.where(ex < 0, PI - phi, phi)
    phi = np.where(ey < 0, -phi, phi)
    c = (phi + PI) * KEYS_PER_RAD
    w = half * KEYS_PER_RAD
    lo = np.floor(c - w).astype(np.int64) - 2
    hi = np.ceil(c + w).astype(np.int64) + 2
    return lo, hi, whole


@pytest.mark.parametrize("cut", ["e_max", "s_max"])
def test_point_windows_contain_every_hit_passing_the_cut(cut):
    """Every hit within the FP32 cut of a predicted point E (extension: e_max;
    middle hit: s_max) has its azimuth key inside the window around E."""
    rng = np.random.default_rng(11 if cut == "e_max" else 12)
    q_max = f32(0.25) if cut == "e_max" else f32(0.09)
    R = math.sqrt(float(q_max)) * 1.0001 + 1e-6  # the radius the host gives the kernels
    n = 400000
    rE = np.concatenate([rng.uniform(2 * R, 3 * R, n // 4), rng.uniform(3 * R, 45.0, n - n // 4)])
    aE = rng.uniform(-math.pi, math.pi, n)
    # a quarter exactly on the axes and octant diagonals, where the reduction switches
    aE[: n // 4] = rng.choice(np.arange(-4, 5) * (math.pi / 4), n // 4)
    ex = (rE * np.cos(aE)).astype(f32)
    ey = (rE * np.sin(aE)).astype(f32)
    rr = np.where(rng.random(n) < 0.3, math.sqrt(float(q_max)), math.sqrt(float(q_max)) * np.sqrt(rng.random(n)))
    ah = rng.uniform(0, 2 * math.pi, n)
    hx = (ex + rr * np.cos(ah)).astype(f32)
    hy = (ey + rr * np.sin(ah)).astype(f32)
    dx, dy = hx - ex, hy - ey
    passing = dx * dx + dy * dy <= q_max
    assert passing.sum() > n // 2
    lo, hi, whole = point_windows(ex, ey, R)
    k = phi_key(hx, hy)
    inside = whole | ((lo <= k) & (k <= hi)) | ((lo <= k - 65536) & (k - 65536 <= hi)) | \
        ((lo <= k + 65536) & (k + 65536 <= hi))
    bad = np.nonzero(passing & ~inside)[0]
    assert bad.size == 0, (bad[:5], ex[bad[:5]], ey[bad[:5]], hx[bad[:5]], hy[bad[:5]])

def grid_cell1(v):
    """Cell of a coordinate as the kernels compute it (FP32): 0.5 mm cells over [-40, 40] mm."""
    c = np.floor((np.asarray(v, f32) + f32(40.0)) * f32(2.0))
    return np.clip(c, 0, 159).astype(np.int64)


def test_grid_disc_search_contains_every_hit_in_the_disc():
    """The crowded-plane searches visit the cells meeting the square around the
    disc (centre +- (R + 1e-3)); every hit within R of the centre must lie in one."""
    rng = np.random.default_rng(3)
    n = 200000
    cx = rng.uniform(-41, 41, n).astype(f32)
    cy = rng.uniform(-41, 41, n).astype(f32)
    R = rng.choice([0.3, 0.5, 0.66], n).astype(f32)
    ang = rng.uniform(0, 2 * math.pi, n)
    rr = R * np.sqrt(rng.uniform(0, 1, n))
    rr = np.where(rng.random(n) < 0.2, R, rr)  # many exactly on the rim
    hx = (cx + rr * np.cos(ang)).astype(f32)
    hy = (cy + rr * np.sin(ang)).astype(f32)
    dx, dy = hx - cx, hy - cy
    inside = dx * dx + dy * dy <= R * R
    rm = R + f32(1e-3)
    ix, iy = grid_cell1(hx), grid_cell1(hy)
    ok = (grid_cell1(cx - rm) <= ix) & (ix <= grid_cell1(cx + rm)) & (grid_cell1(cy - rm) <= iy) & (iy <= grid_cell1(cy + rm))
    assert inside.sum() > 100000
    assert np.all(ok[inside])
