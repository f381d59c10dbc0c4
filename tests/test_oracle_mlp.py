"""Pins of the oracle's MLP ghost filter (10 -> 32 -> 32 -> 1, ReLU, BCE loss).

Pins: central finite differences of the unrounded FP64 network (the textbook
definition of the gradient), hand weights with known outputs, the BF16 rounding
rule on values whose rounding is fixed by the format, and the first Adam step's
closed form.
"""
import numpy as np
import pytest

import oracle

oW1, oB1, oW2, oB2, oW3, oB3 = 0, 320, 352, 1376, 1408, 1440


def test_bf16_rounding_rule():
    # 1.0 is exact; 1 + 2^-8 is a tie -> even (1.0); 1 + 3*2^-8 is a tie -> even (1 + 2^-6)
    assert oracle.to_bf16(1.0) == 0x3F80
    assert oracle.to_bf16(1.0 + 2.0 ** -8) == 0x3F80
    assert oracle.to_bf16(1.0 + 3 * 2.0 ** -8) == 0x3F82
    assert oracle.to_bf16(1.0 + 2.0 ** -8 + 2.0 ** -20) == 0x3F81
    assert oracle.to_bf16(-2.0) == 0xC000
    assert oracle.to_bf16(0.0) == 0x0000
    assert oracle.to_bf16(float("inf")) == 0x7F80


def f2bf(a):
    a = np.asarray(a, np.float32)
    return np.array([oracle.to_bf16(float(v)) for v in a.ravel()], np.uint16).reshape(a.shape)


def test_zero_weights_give_output_bias():
    w = np.zeros(1441, np.float32)
    w[oB3] = 0.625
    w[oB1:oB1 + 32] = 3.0
    x = np.zeros((5, 16), np.uint16)
    x[:, :10] = f2bf(np.random.default_rng(0).normal(size=(5, 10)))
    assert np.all(oracle.mlp_forward(x, w) == 0.625)


def test_hand_weights_known_output():
    # h1[o] = relu(x[o]) for o < 10 (identity block), h2 = h1, logit = sum h2 - 1
    w = np.zeros(1441, np.float32)
    for o in range(10):
        w[oW1 + o * 10 + o] = 1.0
        w[oW2 + o * 32 + o] = 1.0
        w[oW3 + o] = 1.0
    w[oB3] = -1.0
    xs = np.array([[0.5, -1.0, 2.0, 0.25, 0, 0, 0, 0, 0, 3.0]], np.float32)
    x = np.zeros((1, 16), np.uint16)
    x[:, :10] = f2bf(xs)
    assert oracle.mlp_forward(x, w)[0] == pytest.approx(0.5 + 2.0 + 0.25 + 3.0 - 1.0, abs=0)


def test_gradient_matches_central_finite_differences():
    rng = np.random.default_rng(3)
    n = 64
    xd = rng.normal(size=(n, 10))
    lab = (rng.random(n) < 0.4).astype(np.uint8)
    wd = rng.normal(0, 0.4, 1441)
    _, g = oracle.mlp_loss_grad(lab, xd=xd, master_d=wd, round_on=False)
    h = 1e-6
    idx = np.concatenate([rng.choice(1441, 60, replace=False), [oB3, oW3, oB1, oW1, oB2]])
    for i in idx:
        wp, wm = wd.copy(), wd.copy()
        wp[i] += h
        wm[i] -= h
        lp, _ = oracle.mlp_loss_grad(lab, xd=xd, master_d=wp, round_on=False)
        lm, _ = oracle.mlp_loss_grad(lab, xd=xd, master_d=wm, round_on=False)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_loss_closed_form_at_zero_logit():
    # all-zero weights: logit = 0 -> loss = ln 2, d loss / d b3 = mean(0.5 - y)
    lab = np.array([1, 0, 0, 1, 1], np.uint8)
    _, g0 = oracle.mlp_loss_grad(lab, xd=np.zeros((5, 10)), master_d=np.zeros(1441), round_on=False)
    loss, _ = oracle.mlp_loss_grad(lab, xd=np.zeros((5, 10)), master_d=np.zeros(1441), round_on=False)
    assert loss == pytest.approx(np.log(2.0), rel=1e-15)
    assert g0[oB3] == pytest.approx(np.mean(0.5 - lab), rel=1e-15)


def test_rounded_forward_equals_unrounded_on_representable_values():
    # integer weights/inputs with small integer activations: every BF16 rounding
    # step is exact, so the rounded and unrounded networks agree exactly
    rng = np.random.default_rng(5)
    w = np.zeros(1441, np.float32)
    w[oW1:oW1 + 320] = rng.integers(-1, 2, 320)
    w[oB1:oB1 + 32] = rng.integers(-2, 3, 32)
    for o in range(32):
        cols = rng.choice(32, 3, replace=False)
        w[oW2 + o * 32 + cols] = rng.choice([-1.0, 1.0], 3)
    w[oB2:oB2 + 32] = rng.integers(-2, 3, 32)
    w[oW3:oW3 + 32] = rng.integers(-1, 2, 32)
    w[oB3] = 0.5
    xs = rng.integers(-1, 2, (16, 10)).astype(np.float32)
    x = np.zeros((16, 16), np.uint16)
    x[:, :10] = f2bf(xs)
    r = oracle.mlp_forward(x, w, round_on=True)
    u = oracle.mlp_forward(x, w, round_on=False)
    assert np.array_equal(r, u)
    assert np.any(r != 0.5)


def test_adam_first_step_closed_form():
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    w = np.zeros(4)
    m = np.zeros(4)
    v = np.zeros(4)
    oracle.adam(w, m, v, g, 1, lr=1e-3)
    # bias-corrected first step: w -= lr * g / (|g| + eps)
    assert np.allclose(w, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)


def test_standardisation_divides_by_the_sd_and_rounds_to_bf16():
    # values whose standardisation is exact: (3 - 1) / 0.5 = 4, (1 - 0) / 4 =
    # 0.25, (-2 - 2) / 8 = -0.5; then ones whose BF16 rounding is fixed by the
    # format: (1 + 2^-8 - 0) / 1 ties to 1.0, (1 + 3 * 2^-8) / 1 to 1 + 2^-6
    norm = np.array([1.0, 0.0, 2.0, 0.0, 0.0, 0, 0, 0, 0, 0] + [0.5, 4.0, 8.0, 1.0, 1.0, 1, 1, 1, 1, 1],
                    np.float32)
    feat = np.array([[3.0, 1.0, -2.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 0, 0, 0, 0, 0]], np.float32)
    out = oracle.standardize(feat, norm)
    assert out.shape == (1, 16)
    assert list(out[0, :5]) == [0x4080, 0x3E80, 0xBF00, 0x3F80, 0x3F82]
    assert np.all(out[0, 10:] == 0)
