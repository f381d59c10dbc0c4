"""Oracle of the seed-level learned filter (the triplet filter applied before claiming).

Pins, none of which re-types the oracle's formulas:
  * features against float64 geometry derived another way: the point of
    closest approach to the z axis from the vertex of the exact quadratic
    r^2(z) sampled at three z, the angle term from atan2, the middle miss from
    linear interpolation between h0 and h2, plane counts from the offsets;
  * on straight tracks the closest-approach z of a true seed lands on the MC
    vertex;
  * the logit against a float64 forward pass of the same network, and a
    hand-built network whose logit is a known piecewise-linear function;
  * in the finder: an infinite threshold changes nothing, a network that
    rejects everything leaves no track, and at the first seeding step a
    closest-approach window drops exactly the candidates outside it.
"""
import numpy as np
import pytest

import oracle
from paper_2412_05041_amd import gen, learned, metrics

N_PARAM = 1441
oW1, oB1, oW2, oB2, oW3, oB3 = 0, 320, 352, 1376, 1408, 1440


@pytest.fixture(scope="module")
def tiny():
    b = gen.generate(gen.WORKLOADS["tiny"].with_events(6, 31))
    c = oracle.cluster(b.pix_off, b.pix_id)
    return b, c


@pytest.fixture(scope="module")
def nominal():
    b = gen.generate(gen.WORKLOADS["nominal"].with_events(2, 33))
    c = oracle.cluster(b.pix_off, b.pix_id)
    return b, c


def step_candidates(c, plane_z, cut, e, k, seed=None):
    """Seed candidates of event e at seeding step k as global triplets (q, h0, h1, h2)."""
    t = oracle.find_tracks(c["clu_off"], c["clu_x"], c["clu_y"], plane_z, cut, dbg_event=e, dbg_step=k, seed=seed)
    d = t["dbg_cand"]
    g0 = int(c["clu_off"][e * 26])
    return d[:, 0], d[:, 1:].astype(np.int64) + g0


def all_candidates(c, plane_z, cut, n_events):
    hs = []
    for e in range(n_events):
        for k in range(24):
            _, h = step_candidates(c, plane_z, cut, e, k)
            hs.append(h)
    return np.concatenate(hs)


def reference_features(h, c, plane_z):
    """float64 features derived without the oracle's expressions."""
    x = c["clu_x"].astype(np.float64)
    y = c["clu_y"].astype(np.float64)
    off = c["clu_off"]
    s = np.searchsorted(off, h[:, 0], side="right") - 1
    k = s % 26
    z = plane_z.astype(np.float64)
    z0, z1, z2 = z[k], z[k + 1], z[k + 2]
    x0, y0, x1, y1, x2, y2 = x[h[:, 0]], y[h[:, 0]], x[h[:, 1]], y[h[:, 1]], x[h[:, 2]], y[h[:, 2]]
    # middle miss: linear interpolation between h0 and h2 at z1
    u = (z1 - z0) / (z2 - z0)
    q = (x1 - (x0 + u * (x2 - x0))) ** 2 + (y1 - (y0 + u * (y2 - y0))) ** 2
    # r^2(z) is an exact quadratic: sample it at z0, z2 and 2 z2 - z0, take the vertex
    def r2(zz):
        w = (zz - z0) / (z2 - z0)
        return (x0 + w * (x2 - x0)) ** 2 + (y0 + w * (y2 - y0)) ** 2
    za, zb, zc_ = z0, z2, 2 * z2 - z0
    ra, rb, rc = r2(za), r2(zb), r2(zc_)
    d = z2 - z0
    a2 = (ra - 2 * rb + rc) / (2 * d * d)
    a1 = (rb - ra) / d - a2 * (za + zb)
    zmin = -a1 / (2 * a2)
    dmin = r2(zmin)
    tx, ty = (x2 - x0) / (z2 - z0), (y2 - y0) / (z2 - z0)
    ang = np.arctan2(y0, x0) - np.arctan2(ty, tx)
    n = np.diff(off)
    base = s - k  # slot of plane 0 of the event
    return dict(q=q, d2=dmin, zc=np.clip(zmin, -2000, 2000), r2=x0 ** 2 + y0 ** 2, t2=tx ** 2 + ty ** 2,
                cos2=np.cos(ang) ** 2, k=k, n0=n[base + k], n1=n[base + k + 1], n2=n[base + k + 2])


def test_features_against_independent_geometry(nominal):
    b, c = nominal
    cut = learned.cuts("loose")
    h = all_candidates(c, b.plane_z, cut, b.n_events)
    assert len(h) > 100
    f = oracle.seed_features(h, c["clu_off"], c["clu_x"], c["clu_y"], b.plane_z).astype(np.float64)
    r = reference_features(h, c, b.plane_z)
    scale = r["r2"]  # the coordinates' squared size bounds the rounding of the quadratic terms
    assert np.allclose(f[:, 0], r["q"], rtol=1e-4, atol=1e-6 * scale.max())
    assert np.all(np.abs(f[:, 1] - r["d2"]) <= 1e-4 * r["d2"] + 1e-5 * scale)
    # zc: conditioning ~ r0 / t2 (a nearly beam-parallel line makes it ill-posed)
    tol_z = 1e-3 + 1e-5 * np.sqrt(scale) / np.sqrt(r["t2"]) * 50
    assert np.all(np.abs(f[:, 2] - r["zc"]) <= tol_z)
    assert np.allclose(f[:, 3], r["r2"], rtol=1e-6)
    assert np.allclose(f[:, 4], r["t2"], rtol=1e-5)
    assert np.allclose(f[:, 5], r["cos2"], rtol=1e-4, atol=1e-5)
    assert np.array_equal(f[:, 6], r["k"])
    assert np.array_equal(f[:, 7], r["n0"]) and np.array_equal(f[:, 8], r["n1"]) and np.array_equal(f[:, 9], r["n2"])


def test_true_seed_points_at_its_vertex(tiny):
    b, c = tiny
    cut = learned.cuts("default")
    h = all_candidates(c, b.plane_z, cut, b.n_events)
    n_clu = int(c["clu_off"][-1])
    mc = metrics.cluster_truth(c["pix_clu"], b.pix_mc, n_clu)
    ev = (np.searchsorted(c["clu_off"], h[:, 0], side="right") - 1) // 26
    m0, m1, m2 = mc[h[:, 0]], mc[h[:, 1]], mc[h[:, 2]]
    true = (m0 >= 0) & (m0 == m1) & (m0 == m2)
    assert true.sum() > 50
    f = oracle.seed_features(h[true], c["clu_off"], c["clu_x"], c["clu_y"], b.plane_z)
    vz = b.trk_param[b.trk_off[ev[true]] + m0[true], 2]
    dz = np.abs(f[:, 2] - vz)
    # extrapolating a two-plane lever arm back to the vertex: mm-scale in z
    assert np.median(dz) < 3.0 and np.quantile(dz, 0.95) < 30.0
    # and the transverse distance is sub-mm (the vertex spread is 0.04 mm)
    assert np.quantile(f[:, 1], 0.95) < 0.5 ** 2


def forward64(w, norm, f):
    w = w.astype(np.float64)
    xs = (f.astype(np.float64) - norm[:10]) / norm[10:]
    h1 = np.maximum(xs @ w[oW1:oB1].reshape(32, 10).T + w[oB1:oW2], 0)
    h2 = np.maximum(h1 @ w[oW2:oB2].reshape(32, 32).T + w[oB2:oW3], 0)
    return h2 @ w[oW3:oB3] + w[oB3]


def test_logit_against_float64_forward(tiny):
    b, c = tiny
    rng = np.random.default_rng(5)
    w = learned.he_uniform(7)
    w[oB1:oW2] = rng.normal(0, 0.1, 32)
    w[oB2:oW3] = rng.normal(0, 0.1, 32)
    w[oB3] = 0.3
    h = all_candidates(c, b.plane_z, learned.cuts("loose"), b.n_events)
    f = oracle.seed_features(h, c["clu_off"], c["clu_x"], c["clu_y"], b.plane_z)
    norm = np.concatenate([f.mean(0), f.std(0) + 1e-3]).astype(np.float32)
    z = oracle.seed_logit(f, (w, norm, 0.0)).astype(np.float64)
    ref = forward64(w, norm.astype(np.float64), f)
    # FP32 accumulation error bound: a few ulps of the sum of |terms| per layer
    mag = np.abs(ref) + 10.0
    assert np.all(np.abs(z - ref) <= 1e-5 * mag)
    assert np.std(ref) > 0.1  # the network is not degenerate


def window_net(L):
    """logit = relu(zc - L) + relu(-zc - L) on raw features (norm 0 / 1)."""
    w = np.zeros(N_PARAM, np.float32)
    w[oW1 + 0 * 10 + 2] = 1.0
    w[oW1 + 1 * 10 + 2] = -1.0
    w[oB1 + 0] = -L
    w[oB1 + 1] = -L
    w[oW2 + 0 * 32 + 0] = 1.0
    w[oW2 + 1 * 32 + 1] = 1.0
    w[oW3 + 0] = 1.0
    w[oW3 + 1] = 1.0
    norm = np.concatenate([np.zeros(10), np.ones(10)]).astype(np.float32)
    return w, norm


def test_hand_built_network_is_piecewise_linear(tiny):
    b, c = tiny
    h = all_candidates(c, b.plane_z, learned.cuts("loose"), b.n_events)
    f = oracle.seed_features(h, c["clu_off"], c["clu_x"], c["clu_y"], b.plane_z)
    L = np.float32(60.0)
    w, norm = window_net(L)
    z = oracle.seed_logit(f, (w, norm, 0.0))
    zc = f[:, 2]
    exp = np.maximum(zc - L, np.float32(0)) + np.maximum(-zc - L, np.float32(0))
    assert np.array_equal(z, exp.astype(np.float32))
    assert (exp > 0).any() and (exp == 0).any()


def test_infinite_threshold_changes_nothing(tiny):
    b, c = tiny
    cut = learned.cuts("ms")
    plain = oracle.find_tracks(c["clu_off"], c["clu_x"], c["clu_y"], b.plane_z, cut)
    w = learned.he_uniform(3)
    norm = np.concatenate([np.zeros(10), np.ones(10)]).astype(np.float32)
    t = oracle.find_tracks(c["clu_off"], c["clu_x"], c["clu_y"], b.plane_z, cut, seed=(w, norm, np.inf))
    for key in ("trk_off", "trk_hit_off", "trk_hit", "trk_planes", "trk_flags"):
        assert np.array_equal(t[key], plain[key]), key
    assert t["stats"][3] == 0 and np.array_equal(t["stats"][:3], plain["stats"][:3])


def test_reject_all_leaves_no_track(tiny):
    b, c = tiny
    w = np.zeros(N_PARAM, np.float32)
    w[oB3] = 1.0
    norm = np.concatenate([np.zeros(10), np.ones(10)]).astype(np.float32)
    t = oracle.find_tracks(c["clu_off"], c["clu_x"], c["clu_y"], b.plane_z, learned.cuts("ms"), seed=(w, norm, 0.0))
    assert t["trk_off"][-1] == 0
    assert t["stats"][2] > 0 and t["stats"][3] == t["stats"][2]


def test_window_drops_exactly_the_candidates_outside(tiny):
    b, c = tiny
    cut = learned.cuts("loose")
    L = 60.0
    w, norm = window_net(L)
    checked = 0
    for e in range(b.n_events):
        q0, h0 = step_candidates(c, b.plane_z, cut, e, 23)
        q1, h1 = step_candidates(c, b.plane_z, cut, e, 23, seed=(w, norm, 0.0))
        zc = reference_features(h0, c, b.plane_z)["zc"]
        inside = np.abs(zc) <= L
        margin = np.abs(np.abs(zc) - L) > 1e-3  # away from the edge, where FP32 could round either way
        keep = {tuple(r) for r in h1.tolist()}
        for r, ins, m in zip(h0.tolist(), inside, margin):
            if m:
                assert (tuple(r) in keep) == bool(ins)
                checked += 1
        assert keep <= {tuple(r) for r in h0.tolist()}
        assert len(h1) < len(h0) or not (~inside).any()
    assert checked > 50
