"""Float64 CPU oracle of the learned warm start.

TEST INFRASTRUCTURE ONLY: used by ``tests/`` (gradient checks of the GPU
training kernels); never by the HIP product path.

This part is not in the paper.  It is a small fully convolutional network on
the image grid of a convolution dictionary.  From the state before EM
iteration t, it predicts a start for the CG solve of that E-step, which runs
preconditioned by the Jacobi diagonal of A.  The solve's own stop rule then
judges the prediction (Sec. 3.2).

Definitions (shared with the GPU kernels by specification, not by code):

* features (5 channels) from alpha_t, alpha_{t-1}, mu_{t-1}, s_{t-1}, with the
  diagonal d = beta ||h||^2 + alpha_t of A (d_prev likewise from alpha_{t-1}):
    f0 = alpha_t / d
    f1 = mu_{t-1} / rms(mu_{t-1})          (rms over the image; 1 if it is 0)
    f2 = log(clip(s_{t-1} d, 1e-3, 1e3)) / 3
    f3 = log(d / (beta ||h||^2)) / 10
    f4 = clip(log(d_prev / d), -10, 10) / 10   (how far the last M-step moved A;
         mu_t - mu_{t-1} solves A_t e = (alpha_{t-1} - alpha_t) mu_{t-1})
  aux (3 channels): mu_{t-1}, d, sb = clip(s_{t-1} d, 0.05, 20).
* network: four 3x3 convolutions with circular padding, 5 -> 32 -> 32 -> 32 -> 2
  channels, ReLU after the first three; out[co][u][v] = b[co] +
  sum_{ci,ky,kx} w[co][ci][ky][kx] x[ci][(u+ky-1) mod H][(v+kx-1) mod W].
* prediction: mu_hat = mu_{t-1} (1 + tanh(o0)),  d_hat = exp(clip(o1, -10, 10)) sb / d;
  the solve starts from X0 = [d_hat (.) p_k | mu_hat] with M^-1 = 1/d (the
  Jacobi diagonal; d_hat estimates diag(Sigma), which as a preconditioner
  needs more iterations).  All-zero output gives mu_hat = mu_{t-1} and
  d_hat = clip(s_{t-1} d, 0.05, 20) / d, i.e. the previous iterate, the
  non-learned warm start: the network learns corrections to it.
* loss against the E-step's result (mu_t, s_t), each term relative to the
  untrained network's (the previous iterate's), with tgt = log(clip(s_t d,
  0.05, 20) / sb) and f = NORM_FLOOR:
    L = sum (mu_hat - mu_t)^2 / (sum (mu_{t-1} - mu_t)^2 + f sum mu_t^2)
        + LAMBDA_D * sum (o1 - tgt)^2 / (sum tgt^2 + f HW).
* parameters, flattened: for each layer w (Cout x Cin x 3 x 3, row-major),
  then b (Cout).

The backward pass below is written out by hand.  The tests pin it against
central finite differences of ``loss``.
"""
from __future__ import annotations

import numpy as np

CHANNELS = (5, 32, 32, 32, 2)
LAMBDA_D = 0.1
NORM_FLOOR = 1e-4  # changes below 1% of the mean count as converged (bounds the weights)


def param_shapes(channels=CHANNELS):
    out = []
    for ci, co in zip(channels[:-1], channels[1:]):
        out.append(((co, ci, 3, 3), (co,)))
    return out


def unflatten(theta: np.ndarray, channels=CHANNELS):
    layers, k = [], 0
    for ws, bs in param_shapes(channels):
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        layers.append((theta[k:k + nw].reshape(ws), theta[k + nw:k + nw + nb].reshape(bs)))
        k += nw + nb
    assert k == theta.size
    return layers


def n_params(channels=CHANNELS):
    return sum(int(np.prod(ws)) + int(np.prod(bs)) for ws, bs in param_shapes(channels))


def _shifted(x, ky, kx):
    # xs[c][u][v] = x[c][(u + ky - 1) mod H][(v + kx - 1) mod W]
    return np.roll(x, shift=(-(ky - 1), -(kx - 1)), axis=(1, 2))


def conv3(x, w, b):
    """3x3 cross-correlation with circular padding: [Cin,H,W] -> [Cout,H,W]."""
    out = np.broadcast_to(b[:, None, None], (w.shape[0],) + x.shape[1:]).astype(np.float64).copy()
    for ky in range(3):
        for kx in range(3):
            out += np.einsum("oc,chw->ohw", w[:, :, ky, kx], _shifted(x, ky, kx))
    return out


def features(alpha, mu_prev, s_prev, beta, hh, H, W, alpha_prev=None):
    """(feats [5,H,W], aux [3,H,W]) from the state before an E-step
    (alpha_prev: the previous E-step's alpha; None means unchanged)."""
    alpha = np.asarray(alpha, np.float64).reshape(H, W)
    ap = alpha if alpha_prev is None else np.asarray(alpha_prev, np.float64).reshape(H, W)
    mu = np.asarray(mu_prev, np.float64).reshape(H, W)
    s = np.asarray(s_prev, np.float64).reshape(H, W)
    d = beta * hh + alpha
    rms = float(np.sqrt(np.mean(mu * mu)))
    rms = rms if rms > 0.0 else 1.0
    f = np.stack([alpha / d, mu / rms, np.log(np.clip(s * d, 1e-3, 1e3)) / 3.0,
                  np.log(d / (beta * hh)) / 10.0,
                  np.clip(np.log((beta * hh + ap) / d), -10.0, 10.0) / 10.0])
    return f, np.stack([mu, d, np.clip(s * d, 0.05, 20.0)])


def forward(theta, feats, channels=CHANNELS):
    """Network output [2,H,W] and the activations needed by ``backward``."""
    layers = unflatten(np.asarray(theta, np.float64), channels)
    acts, zs = [np.asarray(feats, np.float64)], []
    x = acts[0]
    for i, (w, b) in enumerate(layers):
        z = conv3(x, w, b)
        zs.append(z)
        x = np.maximum(z, 0.0) if i + 1 < len(layers) else z
        acts.append(x)
    return x, (acts, zs)


def predict(out, aux):
    """(mu_hat, d_hat) from the network output and aux = [mu_prev, d, sb]."""
    mu_hat = aux[0] * (1.0 + np.tanh(out[0]))
    d_hat = np.exp(np.clip(out[1], -10.0, 10.0)) * aux[2] / aux[1]
    return mu_hat, d_hat


def loss_and_grad_out(out, aux, targets):
    """Loss L and dL/d(out) for targets = [mu_t, s_t].  Each term is
    normalised by the same term of the untrained network (the non-learned
    warm start), so L < 1 + LAMBDA_D means a better start than the previous
    iterate, in early and late EM iterations alike."""
    mu_p, d, sb = aux
    mu_t, s_t = targets
    th = np.tanh(out[0])
    e = mu_p * (1.0 + th) - mu_t
    n = out[0].size
    nrm_mu = float(np.sum((mu_p - mu_t) ** 2)) + NORM_FLOOR * float(np.sum(mu_t * mu_t))
    nrm_mu = nrm_mu if nrm_mu > 0.0 else 1.0
    tgt = np.log(np.clip(s_t * d, 0.05, 20.0) / sb)
    nrm_d = float(np.sum(tgt * tgt)) + NORM_FLOOR * n
    r = out[1] - tgt
    L = float(np.sum(e * e)) / nrm_mu + LAMBDA_D * float(np.sum(r * r)) / nrm_d
    g = np.stack([2.0 * e * mu_p * (1.0 - th * th) / nrm_mu, 2.0 * LAMBDA_D * r / nrm_d])
    return L, g


def loss(theta, feats, aux, targets, channels=CHANNELS):
    out, _ = forward(theta, feats, channels)
    return loss_and_grad_out(out, aux, targets)[0]


def backward(theta, feats, aux, targets, channels=CHANNELS):
    """(L, dL/dtheta flattened in the parameter order)."""
    theta = np.asarray(theta, np.float64)
    layers = unflatten(theta, channels)
    out, (acts, zs) = forward(theta, feats, channels)
    L, g = loss_and_grad_out(out, aux, targets)
    grads = []
    for i in range(len(layers) - 1, -1, -1):
        w, b = layers[i]
        x = acts[i]
        gw = np.zeros_like(w)
        for ky in range(3):
            for kx in range(3):
                gw[:, :, ky, kx] = np.einsum("ohw,chw->oc", g, _shifted(x, ky, kx))
        gb = g.sum(axis=(1, 2))
        grads.append((gw, gb))
        if i > 0:
            gx = np.zeros_like(x)
            for ky in range(3):
                for kx in range(3):
                    gx += np.roll(np.einsum("oc,ohw->chw", w[:, :, ky, kx], g), shift=(ky - 1, kx - 1), axis=(1, 2))
            g = gx * (zs[i - 1] > 0.0)
    grads.reverse()
    return L, np.concatenate([np.concatenate([gw.ravel(), gb.ravel()]) for gw, gb in grads])
