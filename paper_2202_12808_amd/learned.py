"""Training and evaluation driver of the learned form (convolution
dictionaries): collects CoFEM's own EM iterates as training samples and runs
the library's training kernels over them.  Every step of the arithmetic runs
in libcofem.so; this module only orders the calls."""
from __future__ import annotations


def collect_samples(make_ctx, seeds, em_iters, net):
    """Samples (feats, aux, targets) from EM iterations 2..em_iters of one
    context per seed.  make_ctx(seed) returns a convolution CoFEM context (a
    warm-started, Jacobi-preconditioned one gives converged targets)."""
    import torch
    samples = []
    for seed in seeds:
        with make_ctx(seed) as g:
            g.em_step(1)
            for _ in range(2, em_iters + 1):
                feats, aux = g.features(net)
                g.em_step(1)
                mu, s, _ = g.posterior()
                samples.append((feats, aux, torch.stack([mu, s]).contiguous()))
    return samples


def train(net, samples, epochs, lr=1e-3, seed=0):
    """Adam over the samples for `epochs` passes (shuffled each epoch);
    returns the mean loss of each epoch (before each step)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    history = []
    for _ in range(epochs):
        losses = [net.train_step(*samples[i], lr=lr) for i in rng.permutation(len(samples))]
        history.append(float(np.mean(losses)))
    return history


def mean_loss(net, samples):
    import numpy as np
    return float(np.mean([net.loss_grad(*s)[0] for s in samples]))
