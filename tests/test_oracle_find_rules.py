"""Pins of the finder's finer rules: which hits predict, how ties and conflicts
are broken, the chi2/ndof acceptance, the candidate features and the learned
decision.

Exact straight lines cannot tell these rules apart (any two hits of a line give
the same prediction), so every event here is built so that a plausible
mistake changes the result:
  * kinked tracks (the slope changes at one plane) with a decoy hit placed
    exactly where a prediction through the wrong pair of hits would land;
  * mirror-symmetric hits whose miss distances are equal bit for bit, so only
    the index tie-break decides;
  * lines with a gap on the last planes, whose most downstream hit only the
    downstream completion can attach;
  * two seeds of one step that want the same downstream hit;
  * 3-, 4- and 5-hit tracks with a chosen chi2/ndof (from numpy lstsq) on
    either side of c3 and c4;
  * the ten candidate features against lstsq residuals;
  * hand-built networks whose logit is a known function of one feature.
"""
import math

import numpy as np
import pytest

import oracle
from test_oracle_find import CUTS, ZS, as_input_positions, event_from_hits, line_hits, run, tracks_of

torch = pytest.importorskip("torch")

SIGMA = CUTS["sigma"]
Z = [float(z) for z in ZS]


def flat_line(planes, x0=15.0, t=0.04):
    """A line in the x-z plane (every y exactly 0), outward along +x."""
    return line_hits((x0, 0.0), (t, 0.0), planes)


def plane_hits(out, orig, hits, track):
    """{plane: input position} of one output track."""
    return {hits[orig[h]][0]: orig[h] for h in tracks_of(out)[track]}


# ------------------------------------------------ which pair of hits predicts

def test_forwarding_predicts_through_the_two_most_upstream_hits():
    # seed on planes 23-25 (y = 0); the hit on plane 22 is displaced by d, so
    # the track kinks there.  On plane 21 one hit continues the kinked line
    # (the line through the hits on 22 and 23); a decoy sits where the line
    # through the hits on 22 and 25 would predict.  Both lie inside the window
    # of either prediction: only the choice of the pair decides.
    d = 0.45
    hits = flat_line([23, 24, 25])
    x22, x21 = hits[0][1] + 0.04 * (Z[22] - Z[23]), hits[0][1] + 0.04 * (Z[21] - Z[23])
    hits.append((22, x22, d))
    good = d * (Z[23] - Z[21]) / (Z[23] - Z[22])
    decoy = d * (Z[25] - Z[21]) / (Z[25] - Z[22])
    assert abs(good - decoy) > 0.2 and (good - decoy) ** 2 < CUTS["e_max"]
    hits += [(21, x21, decoy), (21, x21, good)]
    out, orig = run(hits, emit_rejected=True)  # a kinked track: its chi2 is not the point
    assert len(tracks_of(out)) == 1
    assert plane_hits(out, orig, hits, 0) == {25: 2, 24: 1, 23: 0, 22: 3, 21: 5}


def test_downstream_completion_predicts_through_the_two_most_downstream_hits():
    # seed on planes 10-12 (y = 0), planes 13 and 15 empty (so nothing else can
    # seed); the hit on 14 is displaced by d.  On plane 16 one hit continues the
    # line through the hits on 12 and 14; a decoy sits on the line through the
    # hits on 10 and 14.
    d = 0.45
    hits = flat_line([10, 11, 12])
    x = lambda k: 15.0 + 0.04 * (Z[k] - Z[10])
    hits.append((14, x(14), d))
    good = d * (Z[16] - Z[12]) / (Z[14] - Z[12])
    decoy = d * (Z[16] - Z[10]) / (Z[14] - Z[10])
    assert abs(good - decoy) > 0.19 and (good - decoy) ** 2 < CUTS["e_max"]
    hits += [(16, x(16), decoy), (16, x(16), good)]
    out, orig = run(hits, emit_rejected=True)
    assert len(tracks_of(out)) == 1
    assert plane_hits(out, orig, hits, 0) == {10: 0, 11: 1, 12: 2, 14: 3, 16: 5}


# ------------------------------------------- equal miss distance: lower index

@pytest.mark.parametrize("first", [+1.0, -1.0])
def test_forwarding_tie_goes_to_the_lower_hit_index(first):
    # track in y = 0; on plane 19 two hits at y = +-0.2 above and below its
    # prediction: their miss distances are equal bit for bit
    hits = [(19, 15.0 + 0.04 * (Z[19] - Z[20]), first * 0.2), (19, 15.0 + 0.04 * (Z[19] - Z[20]), -first * 0.2)]
    hits += flat_line(list(range(20, 26)))
    out, orig = run(hits, emit_rejected=True)
    assert len(tracks_of(out)) == 1
    assert plane_hits(out, orig, hits, 0)[19] == 0


@pytest.mark.parametrize("first", [+1.0, -1.0])
def test_completion_tie_goes_to_the_lower_hit_index(first):
    # seed on planes 10-12 in y = 0, plane 13 empty, two mirror hits on plane 14
    x14 = 15.0 + 0.04 * (Z[14] - Z[10])
    hits = flat_line([10, 11, 12]) + [(14, x14, first * 0.2), (14, x14, -first * 0.2)]
    out, orig = run(hits, emit_rejected=True)
    assert len(tracks_of(out)) == 1
    assert plane_hits(out, orig, hits, 0)[14] == 3


def mirror_triplets(k=12, s=0.003, ty=0.05, zv=-400.0):
    """Two seeds mirrored in x that share the middle hit (x = 0 on plane k+1):
    bit-equal miss distances, so the tie-break after q decides."""
    A = [(k + i, s * (Z[k + i] - Z[k + 1]), ty * (Z[k + i] - zv)) for i in range(3)]
    B = [(kk, -xx, yy) for (kk, xx, yy) in A]
    assert A[1][1] == 0.0
    return A, B


def test_seed_tie_breaks_on_h0_when_h0_and_h2_orders_disagree():
    A, B = mirror_triplets()
    # A has the lower h0 but the higher h2
    hits = [A[0], B[0], A[1], B[2], A[2]]
    out, orig = run(hits, emit_rejected=True)
    assert as_input_positions(out, orig) == [[0, 2, 4]]
    # and the other way round: B has the lower h0 and the higher h2
    hits = [B[0], A[0], A[1], A[2], B[2]]
    out, orig = run(hits, emit_rejected=True)
    assert as_input_positions(out, orig) == [[0, 2, 4]]


def test_equal_key_seeds_are_created_in_h0_order_not_h1_order():
    # two disjoint mirror seeds (x -> -x, no shared hit): equal q, so creation
    # order (the track index) follows h0.  Here h0 and h1 orders disagree.
    k, zv, ty = 12, -400.0, 0.05
    A = [(k + i, 2.0 + 0.01 * (Z[k + i] - zv), ty * (Z[k + i] - zv)) for i in range(3)]
    B = [(kk, -xx, yy) for (kk, xx, yy) in A]
    hits = [A[0], B[0], B[1], A[1], A[2], B[2]]
    out, orig = run(hits, emit_rejected=True)
    assert as_input_positions(out, orig) == [[0, 3, 4], [1, 2, 5]]


# ---------------------------------------------- gaps on the downstream planes

def test_hit_beyond_a_gap_on_the_last_planes_comes_from_completion():
    # plane 24 missing: no seed can use plane 25, and forwarding only moves
    # upstream, so only the downstream completion can attach the plane-25 hit
    planes = [k for k in range(10, 26) if k != 24]
    out, orig = run(line_hits((20.0, 5.0), (0.04, 0.01), planes))
    assert as_input_positions(out, orig) == [list(range(len(planes)))]
    assert int(out["trk_planes"][0]) == sum(1 << k for k in planes)


def test_completion_stops_at_a_gap_wider_than_max_skip():
    planes = [k for k in range(10, 26) if k not in (23, 24)]
    out, orig = run(line_hits((20.0, 5.0), (0.04, 0.01), planes))
    assert as_input_positions(out, orig) == [list(range(len(planes) - 1))]
    planes = [k for k in range(10, 26) if k != 24]
    out, orig = run(line_hits((20.0, 5.0), (0.04, 0.01), planes), cuts=dict(CUTS, max_skip=0))
    assert as_input_positions(out, orig) == [list(range(len(planes) - 1))]


def test_completion_conflict_goes_to_the_lowest_track_index():
    # two radial seeds on planes 10-12 (y = 0, slopes 0.04 and 0.05) converge
    # towards plane 14 (plane 13 empty), where one hit lies closer to seed B's
    # prediction.  Seed A has the smaller miss distance, so it becomes track 0
    # although its hits have the higher indices, and the shared hit goes to
    # track 0.
    xa = lambda k: 15.0 + 0.04 * (Z[k] - Z[14])
    xb = lambda k: 15.2 + 0.05 * (Z[k] - Z[14])
    A = [(k, xa(k), 0.0) for k in (10, 11, 12)]
    B = [(k, xb(k), 0.0) for k in (10, 11, 12)]
    B[0] = (10, B[0][1], 0.1)  # B's seed misses its middle hit by ~0.04 mm
    H = (14, 15.15, 0.0)       # 0.05 mm from B's prediction, 0.15 from A's
    hits = B + A + [H]
    out, orig = run(hits, emit_rejected=True)
    assert as_input_positions(out, orig) == [[3, 4, 5, 6], [0, 1, 2]]
    # without the conflict (A absent) B takes the hit: the rule decided above
    out, orig = run(B + [H], emit_rejected=True)
    assert as_input_positions(out, orig) == [[0, 1, 2, 3]]


# ------------------------------------------------------- chi2/ndof acceptance

def lstsq_chi2(z, x, y):
    """chi2 of the straight-line least-squares fits x(z), y(z) (numpy lstsq)."""
    A = np.stack([np.ones_like(z), z], 1)
    s = 0.0
    for u in (x, y):
        c = np.linalg.lstsq(A, u, rcond=None)[0]
        r = u - A @ c
        s += float(r @ r)
    return s / SIGMA ** 2


def track_with_chi2(planes, pattern, target):
    """Hits of an outward line on `planes` with y offsets a * pattern, a chosen
    so that chi2/ndof (FP64 lstsq on the FP32 coordinates) is `target`."""
    base = line_hits((12.0, 4.0), (0.03, 0.01), planes)
    z = np.array([Z[k] for k in planes])
    p = np.asarray(pattern, float)

    def hits_for(a):
        return [(k, np.float32(x), np.float32(y + a * pi)) for (k, x, y), pi in zip(base, p)]

    def chi2(h):
        return lstsq_chi2(z, np.array([v[1] for v in h], float), np.array([v[2] for v in h], float))

    ndof = 2 * len(planes) - 4
    a = 0.1
    for _ in range(3):  # chi2 is quadratic in a up to the FP32 rounding of the hits
        a *= math.sqrt(target * ndof / chi2(hits_for(a)))
    h = hits_for(a)
    return [(k, float(x), float(y)) for k, x, y in h], chi2(h) / ndof


PATTERNS = {3: [0, 1, 0], 4: [1, 0, 0, -0.5], 5: [1, 0, 0, 0, -1]}


@pytest.mark.parametrize("n,target", [(3, 2.0), (3, 5.0), (3, 10.0), (4, 3.0), (4, 10.0), (4, 20.0),
                                      (5, 14.0), (5, 20.0)])
def test_plain_acceptance_is_chi2_per_ndof_against_c3_or_c4(n, target):
    planes = list(range(10, 10 + n))
    hits, chi2_ndof = track_with_chi2(planes, PATTERNS[n], target)
    assert abs(chi2_ndof - target) < 1e-3 * target
    lim = CUTS["c3"] if n == 3 else CUTS["c4"]
    want = chi2_ndof <= lim
    allc, orig = run(hits, emit_rejected=True)
    assert as_input_positions(allc, orig) == [list(range(n))]  # the candidate holds every hit
    assert bool(allc["trk_flags"][0] & oracle.FLAG_PLAIN) == want
    assert bool(allc["trk_flags"][0] & oracle.FLAG_ACCEPT) == want
    acc, _ = run(hits)
    assert len(tracks_of(acc)) == int(want)


# ------------------------------------------------------------------ features

def lstsq_features(planes, hits):
    z = np.array([Z[k] for k in planes])
    x = np.array([h[1] for h in hits], float)
    y = np.array([h[2] for h in hits], float)
    A = np.stack([np.ones_like(z), z], 1)
    cx = np.linalg.lstsq(A, x, rcond=None)[0]
    cy = np.linalg.lstsq(A, y, rcond=None)[0]
    rx, ry = x - A @ cx, y - A @ cy
    n = len(planes)
    chi2 = float(rx @ rx + ry @ ry) / SIGMA ** 2
    return np.array([chi2 / (2 * n - 4), n, cx[1], cy[1],
                     np.abs(rx).max() / SIGMA, np.abs(ry).max() / SIGMA,
                     (rx[0] ** 2 + ry[0] ** 2) / SIGMA ** 2, (rx[-1] ** 2 + ry[-1] ** 2) / SIGMA ** 2,
                     planes[0] / 25.0, planes[-1] / 25.0])


@pytest.mark.parametrize("planes,ox,oy", [
    ([10, 11, 12], [0.0, 0.05, 0.0], [0.0, -0.02, 0.0]),
    ([14, 15, 16, 17], [0.06, 0.0, 0.0, -0.01], [0.0, 0.0, 0.03, 0.0]),
    ([3, 4, 5, 6, 7], [0.0, 0.02, 0.0, 0.0, 0.08], [0.04, 0.0, -0.01, 0.0, 0.0]),
    ([17, 18, 19, 21], [0.01, 0.0, 0.0, 0.07], [0.0, 0.05, 0.0, 0.0]),
])
def test_candidate_features_match_lstsq_residuals(planes, ox, oy):
    base = line_hits((-9.0, 14.0), (-0.02, 0.035), planes)
    hits = [(k, float(np.float32(x + a)), float(np.float32(y + b))) for (k, x, y), a, b in zip(base, ox, oy)]
    out, orig = run(hits, emit_rejected=True)
    assert as_input_positions(out, orig) == [list(range(len(planes)))]
    want = lstsq_features(planes, hits)
    got = out["trk_feat"][0].astype(np.float64)
    # FP32 fit against FP64 lstsq: residuals of ~0.05 mm on ~10 mm coordinates
    assert np.allclose(got, want, rtol=2e-3, atol=2e-3), (got, want)
    assert got[1] == len(planes) and got[8] == np.float32(planes[0] / 25.0) and got[9] == np.float32(planes[-1] / 25.0)


# ---------------------------------------------------- learned decision (hand)

oW1, oB1, oW2, oB2, oW3, oB3 = 0, 320, 352, 1376, 1408, 1440


def passthrough_net(feature):
    """Weights whose logit equals the standardised, BF16-rounded input
    `feature`: h1 = (relu(x), relu(-x)), h2 = h1, z = h2[0] - h2[1]."""
    w = np.zeros(1441, np.float32)
    w[oW1 + 0 * 10 + feature] = 1.0
    w[oW1 + 1 * 10 + feature] = -1.0
    w[oW2 + 0 * 32 + 0] = 1.0
    w[oW2 + 1 * 32 + 1] = 1.0
    w[oW3 + 0], w[oW3 + 1] = 1.0, -1.0
    return w


def hand_track(n, chi2_ndof):
    planes = list(range(10, 10 + n))
    pat = {3: [0, 1, 0], 4: [1, 0, 0, -0.5], 5: [1, 0, 0, 0, -1], 6: [1, 0, 0, 0, 0, -1]}[n]
    return track_with_chi2(planes, pat, chi2_ndof)[0]


# n, chi2/ndof of the track, plain decision, logit = 2 (n - 4), expected flags
WINDOW_CASES = [
    (3, 8.0, False, -2.0, "learned-accept"),  # |z| = band exactly: the network decides
    (4, 30.0, False, 0.0, "fallback"),        # |z| < band: the plain cut decides (reject)
    (5, 2.0, True, 2.0, "learned-reject"),
    (6, 2.0, True, 4.0, "learned-reject"),
]


@pytest.mark.parametrize("n,chi2_ndof,plain,z,kind", WINDOW_CASES)
def test_learned_decision_window_network(n, chi2_ndof, plain, z, kind):
    # feature 1 is the hit count; standardised with mean 4, sd 0.5 it becomes
    # 2 (n - 4), exact in BF16, and the network passes it through: ghost iff
    # z > 0, plain cut when |z| < band (2.0)
    norm = np.array([0.0] * 10 + [1.0] * 10, np.float32)
    norm[1], norm[11] = 4.0, 0.5
    cuts = dict(CUTS, mode=1, logit_band=2.0)
    hits = hand_track(n, chi2_ndof)
    out, orig = run(hits, cuts=cuts, emit_rejected=True, mlp=(passthrough_net(1), norm))
    assert as_input_positions(out, orig) == [list(range(n))]
    f = int(out["trk_flags"][0])
    assert out["trk_logit"][0] == np.float32(z)
    assert bool(f & oracle.FLAG_PLAIN) == plain
    assert f & oracle.FLAG_LEARNED
    assert bool(f & oracle.FLAG_FALLBACK) == (kind == "fallback")
    accept = {"learned-accept": True, "learned-reject": False, "fallback": plain}[kind]
    assert bool(f & oracle.FLAG_ACCEPT) == accept
    kept, _ = run(hits, cuts=cuts, mlp=(passthrough_net(1), norm))
    assert len(tracks_of(kept)) == int(accept)


def test_learned_input_is_the_bf16_rounding_of_the_standardised_feature():
    # the pass-through network on the slope tx: the logit is the standardised
    # feature rounded to BF16 (nearest even), checked against torch's rounding.
    # Then the first layer's biases are set to -+ that rounded value: the
    # network computes relu(x - b) - relu(b - x), exactly 0 when the input was
    # rounded before the first layer, and nonzero (the rounding error) when
    # the unrounded feature reached it.
    norm = np.array([0.0] * 10 + [1.0] * 10, np.float32)
    norm[2], norm[12] = 0.01, 0.003
    cuts = dict(CUTS, mode=1, logit_band=0.0)
    for planes, s in (([10, 11, 12], 0.0371), ([15, 16, 17, 18], 0.0213), ([4, 5, 6], 0.0289)):
        hits = line_hits((10.0, 2.0), (s, 0.004), planes)
        out, _ = run(hits, cuts=cuts, emit_rejected=True, mlp=(passthrough_net(2), norm))
        f = np.float32(out["trk_feat"][0, 2])
        xs = (f - norm[2]) / norm[12]
        want = np.float32(torch.tensor([float(xs)], dtype=torch.float32).to(torch.bfloat16).float().item())
        assert out["trk_logit"][0] == want
        assert want != np.float32(xs)  # the rounding is visible in these cases
        for b, z0 in ((want, True), (np.float32(xs), False)):
            w = passthrough_net(2)
            w[oB1 + 0], w[oB1 + 1] = -b, b
            out, _ = run(hits, cuts=cuts, emit_rejected=True, mlp=(w, norm))
            assert (out["trk_logit"][0] == 0.0) == z0


def test_rounded_gradient_uses_the_rounded_hidden_activation():
    # one live path: b1[0] = 1 + 2^-10 (FP32; its BF16 rounding is 1.0 by the
    # format), W2[0][0] = W3[0] = 1, input 0.  Forward: h1 = 1.0, h2 = 1.0,
    # z = 1; with label 0 the straight-through gradient of W2[0][0] is
    # sigmoid(1) * h1 = sigmoid(1) exactly, of b1[0] sigmoid(1), of W3[0]
    # sigmoid(1) * h2.
    w = np.zeros(1441, np.float32)
    w[oB1] = np.float32(1.0 + 2.0 ** -10)
    w[oW2] = 1.0
    w[oW3] = 1.0
    xb = np.zeros((1, 16), np.uint16)
    loss, g = oracle.mlp_loss_grad(np.zeros(1, np.uint8), master=w, xb=xb, round_on=True)
    sig = 1.0 / (1.0 + math.exp(-1.0))
    assert loss == pytest.approx(math.log1p(math.exp(1.0)), rel=1e-14)
    assert g[oW2] == pytest.approx(sig, rel=1e-14)
    assert g[oB1] == pytest.approx(sig, rel=1e-14)
    assert g[oW3] == pytest.approx(sig, rel=1e-14)
    # unrounded, the same path carries 1 + 2^-10 all the way to the logit
    z = 1.0 + 2.0 ** -10
    loss, g = oracle.mlp_loss_grad(np.zeros(1, np.uint8), master=w, xb=xb, round_on=False)
    sz = 1.0 / (1.0 + math.exp(-z))
    assert g[oW2] == pytest.approx(sz * z, rel=1e-14)
    assert g[oW3] == pytest.approx(sz * z, rel=1e-14)


def test_rounded_gradient_uses_the_rounded_second_hidden_activation():
    # the live path starts at the second layer: b2[0] = 1 + 2^-10 (its BF16
    # rounding is 1.0 by the format), W3[0] = 1, everything else 0.  Forward:
    # h2 = 1.0, z = 1; the straight-through gradient of W3[0] is
    # sigmoid(1) * h2 = sigmoid(1), of b2[0] sigmoid(1).
    w = np.zeros(1441, np.float32)
    w[oB2] = np.float32(1.0 + 2.0 ** -10)
    w[oW3] = 1.0
    xb = np.zeros((1, 16), np.uint16)
    loss, g = oracle.mlp_loss_grad(np.zeros(1, np.uint8), master=w, xb=xb, round_on=True)
    sig = 1.0 / (1.0 + math.exp(-1.0))
    assert loss == pytest.approx(math.log1p(math.exp(1.0)), rel=1e-14)
    assert g[oW3] == pytest.approx(sig, rel=1e-14)
    assert g[oB2] == pytest.approx(sig, rel=1e-14)
    z = 1.0 + 2.0 ** -10
    loss, g = oracle.mlp_loss_grad(np.zeros(1, np.uint8), master=w, xb=xb, round_on=False)
    assert g[oW3] == pytest.approx(z / (1.0 + math.exp(-z)), rel=1e-14)


@pytest.mark.parametrize("first", [+1.0, -1.0])
def test_seed_tie_after_h0_breaks_on_h1(first):
    # h0 and h2 in y = 0, so the prediction on plane k+1 has y = 0 exactly; two
    # middle hits at the same x and y = +-d: bit-equal q with the same h0, so
    # the lower h1 index takes the seed
    k, d = 12, 0.2
    x = lambda j: 15.0 + 0.04 * (Z[j] - Z[k])
    hits = [(k, x(k), 0.0), (k + 1, x(k + 1), first * d), (k + 1, x(k + 1), -first * d), (k + 2, x(k + 2), 0.0)]
    out, orig = run(hits, emit_rejected=True)
    assert as_input_positions(out, orig) == [[0, 1, 3]]


@pytest.mark.parametrize("first", [+1.0, -1.0])
def test_seed_tie_after_h1_breaks_on_h2(first):
    # h0 and h1 in y = 0; two last hits at the same x and y = +-d give slopes
    # ty = +-d / dz2 (exact negatives) and so bit-equal middle misses with the
    # same h0 and h1: the lower h2 index takes the seed
    k, d = 12, 0.2
    x = lambda j: 15.0 + 0.04 * (Z[j] - Z[k])
    hits = [(k, x(k), 0.0), (k + 1, x(k + 1), 0.0), (k + 2, x(k + 2), first * d), (k + 2, x(k + 2), -first * d)]
    out, orig = run(hits, emit_rejected=True)
    assert as_input_positions(out, orig) == [[0, 1, 2]]


# ------------------------------------------------- cuts are inclusive (<=)

def test_middle_hit_cut_keeps_a_miss_equal_to_s_max():
    # the candidate's own q (the finder's debug output) as the cut: kept; one
    # ulp below: dropped
    hits = line_hits((20.0, 0.0), (0.05, 0.0), [10, 11, 12], z0=Z[11])
    hits[1] = (11, hits[1][1], hits[1][2] + 0.17)
    out = run(hits, emit_rejected=True, dbg_event=0, dbg_step=10)[0]
    assert len(out["dbg_cand"]) == 1
    q = np.float32(out["dbg_cand"][0, 0])
    assert len(tracks_of(run(hits, cuts=dict(CUTS, s_max=float(q)), emit_rejected=True)[0])) == 1
    below = float(np.nextafter(q, np.float32(0)))
    assert len(tracks_of(run(hits, cuts=dict(CUTS, s_max=below), emit_rejected=True)[0])) == 0


def test_extension_cut_keeps_a_miss_equal_to_e_max():
    # seed on planes 20-22, one hit on plane 19 off the line; its miss q from
    # the prediction through the hits on 20 and 21, in FP32 as a line
    # extrapolation: the cut at q keeps it, one ulp below drops it
    hits = line_hits((20.0, 0.0), (0.05, 0.0), [20, 21, 22])
    z = np.float32(Z)
    x19 = 20.0 + 0.05 * (Z[19] - Z[20])
    hits.append((19, x19, 0.33))
    f = np.float32
    (_, xa, ya), (_, xb, yb) = hits[1], hits[0]
    tx = (f(xa) - f(xb)) / (z[21] - z[20])
    ty = (f(ya) - f(yb)) / (z[21] - z[20])
    ex = f(xb) + tx * (z[19] - z[20])
    ey = f(yb) + ty * (z[19] - z[20])
    dx, dy = f(x19) - ex, f(0.33) - ey
    q = dx * dx + dy * dy
    got = as_input_positions(*run(hits, cuts=dict(CUTS, e_max=float(q)), emit_rejected=True))
    assert got == [[0, 1, 2, 3]]
    below = float(np.nextafter(q, f(0)))
    got = as_input_positions(*run(hits, cuts=dict(CUTS, e_max=below), emit_rejected=True))
    assert got == [[0, 1, 2]]


@pytest.mark.parametrize("axis", [0, 1])
@pytest.mark.parametrize("t,found", [(0.39, True), (0.41, False)])
def test_seed_slope_bound_applies_to_each_axis(axis, t, found):
    # a radial line along x or along y; the other slope is 0
    p = [0.0, 0.0]
    p[axis] = 20.0
    s = [0.0, 0.0]
    s[axis] = t
    out, _ = run(line_hits(tuple(p), tuple(s), [10, 11, 12], z0=Z[11]))
    assert (len(tracks_of(out)) == 1) == found


# ------------------------------------- seed feature: the closest-approach clip

def test_seed_closest_approach_z_is_clipped_to_2000_mm():
    # a radial line of slope 0.004 at radius 20 mm passes the axis 5000 mm
    # upstream of its first plane: the feature reads -2000; with the slope
    # reversed the line passes it 5000 mm downstream: +2000 (the features are
    # defined for any triplet, the seed cuts aside); a line meeting the axis
    # at z = -100 mm reads that z
    def feat(x0, t):
        hits = [(k, x0 + t * (Z[k] - Z[10]), 0.0) for k in (10, 11, 12)]
        off, x, y, _ = event_from_hits(hits)
        f = oracle.seed_features(np.array([[0, 1, 2]]), off, x, y, ZS)
        return f[0]
    assert feat(20.0, 0.004)[2] == np.float32(-2000.0)
    assert feat(20.0, -0.004)[2] == np.float32(2000.0)
    assert abs(feat(20.0, 20.0 / (Z[10] + 100.0))[2] - (-100.0)) < 1e-2
