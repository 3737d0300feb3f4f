"""Pins of the oracle of the learned start/preconditioner network: the hand
backward pass against central finite differences of the loss, the 3x3
circular convolution against a direct double loop, and the zero network's
prediction (the previous mean and the previous diagonal estimate)."""
import numpy as np

from oracle import learned as L


def _sample(H=7, W=6, seed=0, channels=(4, 5, 3, 2)):
    rng = np.random.default_rng(seed)
    theta = rng.standard_normal(L.n_params(channels)) * 0.4
    feats = rng.standard_normal((channels[0], H, W))
    mu_p = rng.standard_normal((H, W))
    d = np.exp(rng.uniform(0, 3, (H, W)))
    aux = np.stack([mu_p, d, np.exp(rng.uniform(-2, 2, (H, W)))])
    targets = np.stack([mu_p * rng.uniform(0.5, 1.5, (H, W)), np.exp(rng.uniform(-1, 1, (H, W))) / d])
    return theta, feats, aux, targets, channels


def test_conv3_matches_direct_loop():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((3, 5, 4))
    w = rng.standard_normal((2, 3, 3, 3))
    b = rng.standard_normal(2)
    out = L.conv3(x, w, b)
    H, W = 5, 4
    ref = np.zeros((2, H, W))
    for co in range(2):
        for u in range(H):
            for v in range(W):
                acc = b[co]
                for ci in range(3):
                    for ky in range(3):
                        for kx in range(3):
                            acc += w[co, ci, ky, kx] * x[ci, (u + ky - 1) % H, (v + kx - 1) % W]
                ref[co, u, v] = acc
    np.testing.assert_allclose(out, ref, rtol=1e-13, atol=1e-13)


def test_backward_matches_finite_differences():
    theta, feats, aux, targets, ch = _sample()
    Lv, g = L.backward(theta, feats, aux, targets, ch)
    assert np.isclose(Lv, L.loss(theta, feats, aux, targets, ch))
    rng = np.random.default_rng(2)
    idx = rng.choice(theta.size, 40, replace=False)
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (L.loss(tp, feats, aux, targets, ch) - L.loss(tm, feats, aux, targets, ch)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_zero_network_predicts_previous_mean_and_diagonal():
    # the untrained network (zero last layer) reproduces the non-learned warm
    # start: mu_prev, and s_prev wherever s_prev d lies in [0.05, 20]
    H, W = 6, 5
    rng = np.random.default_rng(3)
    alpha = np.exp(rng.uniform(-2, 8, H * W))
    mu = rng.standard_normal(H * W)
    d = 100.0 * 0.8 + alpha
    s = np.exp(rng.uniform(-1.5, 1.5, H * W)) / d
    s[:3] = [1e-4 / d[0], -1.0 / d[1], 50.0 / d[2]]  # below, negative, above the clip
    feats, aux = L.features(alpha, mu, s, 100.0, 0.8, H, W)
    out, _ = L.forward(np.zeros(L.n_params()), feats)
    mu_hat, d_hat = L.predict(out, aux)
    np.testing.assert_allclose(mu_hat, mu.reshape(H, W))
    ref = s.copy()
    ref[:3] = [0.05 / d[0], 0.05 / d[1], 20.0 / d[2]]
    np.testing.assert_allclose(d_hat, ref.reshape(H, W), rtol=1e-14)


def test_untrained_network_loss_is_one_per_term():
    # each loss term is normalised by the untrained network's own error, so a
    # zero network scores A / (A + f M) + LAMBDA_D T / (T + f n): 1 + LAMBDA_D
    # up to the normaliser floor f (A = sum (mu_prev - mu_t)^2, M = sum mu_t^2,
    # T = sum of the squared log targets, n pixels)
    theta, feats, aux, targets, ch = _sample()
    theta = np.zeros_like(theta)
    Lv = L.loss(theta, feats, aux, targets, ch)
    mu_p, d, sb = aux
    A = np.sum((mu_p - targets[0]) ** 2)
    M = np.sum(targets[0] ** 2)
    T = np.sum(np.log(np.clip(targets[1] * d, 0.05, 20.0) / sb) ** 2)
    f, n = L.NORM_FLOOR, mu_p.size
    assert abs(Lv - (A / (A + f * M) + L.LAMBDA_D * T / (T + f * n))) < 1e-12, Lv
    assert abs(Lv - (1.0 + L.LAMBDA_D)) < 0.01


def test_features_hand_computed_2x2():
    # a 2 x 2 grid worked by hand: beta ||h||^2 = 2 * 0.5 = 1, so d = 1 + alpha
    # = [[2, 4], [8, 2]]; every clip bound is hit once
    import math
    alpha = np.array([1.0, 3.0, 7.0, 1.0])
    alpha_prev = np.array([1.0, 1.0, 7.0, 15.0])      # d_prev = [[2, 2], [8, 16]]
    mu = np.array([2.0, 0.0, -2.0, 0.0])              # rms = sqrt(8 / 4) = sqrt(2)
    s = np.array([0.5, 1e-6, 0.25, 100.0])            # s d = [[1, 4e-6], [2, 200]]
    f, aux = L.features(alpha, mu, s, 2.0, 0.5, 2, 2, alpha_prev=alpha_prev)
    r2 = math.sqrt(2.0)
    ln = math.log
    want_f = [
        [[0.5, 0.75], [0.875, 0.5]],                                # alpha / d
        [[2.0 / r2, 0.0], [-2.0 / r2, 0.0]],                        # mu / rms
        [[0.0, ln(1e-3) / 3.0], [ln(2.0) / 3.0, ln(200.0) / 3.0]],  # log clip(s d, 1e-3, 1e3) / 3
        [[ln(2.0) / 10, ln(4.0) / 10], [ln(8.0) / 10, ln(2.0) / 10]],  # log(d / (beta ||h||^2)) / 10
        [[0.0, ln(0.5) / 10], [0.0, ln(8.0) / 10]],                 # clip(log(d_prev / d)) / 10
    ]
    want_aux = [[[2.0, 0.0], [-2.0, 0.0]], [[2.0, 4.0], [8.0, 2.0]], [[1.0, 0.05], [2.0, 20.0]]]
    np.testing.assert_allclose(f, np.array(want_f), rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(aux, np.array(want_aux), rtol=1e-14, atol=1e-15)
    # the clip of log(d_prev / d) at +-10: a move of more than e^10
    f2, _ = L.features(np.array([1e6]), np.array([1.0]), np.array([1.0]), 1.0, 1.0, 1, 1,
                       alpha_prev=np.array([1e-9]))
    assert f2[4, 0, 0] == -1.0
    # a zero mean has rms 1 by definition (no division by zero)
    f3, _ = L.features(alpha, np.zeros(4), s, 2.0, 0.5, 2, 2)
    assert np.all(f3[1] == 0.0) and np.all(f3[4] == 0.0)
