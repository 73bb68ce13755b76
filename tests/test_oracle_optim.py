"""Pins of the optimiser-step and split-sampling oracle (CPU)."""
import math

import numpy as np
import torch

import scenegen
from oracle import optim as OP
from oracle import render4d as O


def _rand_groups(rng, n, k):
    shapes = dict(means4=(n, 4), log_scales4=(n, 4), q_left=(n, 4), q_right=(n, 4), opacity_logit=(n,),
                  coeffs=(n, k, 3))
    return {g: rng.normal(size=shapes[g]) for g in OP.GROUPS}


def test_adam_matches_torch_optim_adam():
    """Three steps against torch.optim.Adam (an independent implementation),
    one optimiser per group with its own learning rate."""
    rng = np.random.default_rng(3)
    n, k = 50, 9
    p0 = _rand_groups(rng, n, k)
    lr = [1.6e-4, 5e-3, 1e-3, 1e-3, 5e-2, 2.5e-3]
    tens = {g: torch.tensor(p0[g], dtype=torch.float64, requires_grad=True) for g in OP.GROUPS}
    opts = [torch.optim.Adam([tens[g]], lr=lr[i], betas=(0.9, 0.999), eps=1e-15) for i, g in enumerate(OP.GROUPS)]
    p, m = dict(p0), {g: np.zeros_like(p0[g]) for g in OP.GROUPS}
    v = {g: np.zeros_like(p0[g]) for g in OP.GROUPS}
    for step in (1, 2, 3):
        grads = _rand_groups(rng, n, k)
        for g, o in zip(OP.GROUPS, opts):
            o.zero_grad()
            tens[g].grad = torch.tensor(grads[g])
            o.step()
        p, m, v = OP.adam_step(p, grads, m, v, step, lr, 0.9, 0.999, 1e-15)
        for g in OP.GROUPS:
            assert np.allclose(p[g], tens[g].detach().numpy(), rtol=1e-13, atol=1e-15), (g, step)


def test_adam_first_step_is_signed_learning_rate():
    """From zero moments the first step moves every entry by lr * g / (|g| + eps)."""
    rng = np.random.default_rng(4)
    p0 = _rand_groups(rng, 10, 3)
    g0 = _rand_groups(rng, 10, 3)
    zero = {g: np.zeros_like(p0[g]) for g in OP.GROUPS}
    lr = [0.1, 0.2, 0.3, 0.4, 0.5, 0.6]
    p1, _, _ = OP.adam_step(p0, g0, zero, zero, 1, lr, 0.9, 0.999, 1e-8)
    for i, g in enumerate(OP.GROUPS):
        exp = p0[g] - lr[i] * g0[g] / (np.abs(g0[g]) + 1e-8)
        assert np.allclose(p1[g], exp, rtol=1e-12, atol=1e-14)


def test_split_sample_identity_rotation_scales_the_draws():
    sc = scenegen.random_scene(31, 4)
    sc.q_left[:] = [1, 0, 0, 0]
    sc.q_right[:] = [1, 0, 0, 0]
    z = np.random.default_rng(32).normal(size=(4, 4))
    x = OP.split_sample(sc, np.arange(4), z)
    exp = sc.means4.astype(np.float64) + np.exp(sc.log_scales4.astype(np.float64)) * z
    assert np.allclose(x, exp, rtol=1e-14, atol=1e-15)


def test_split_samples_have_the_primitive_covariance():
    """200k draws of one rotated, anisotropic primitive: the sample mean and
    covariance match mu and Sigma = R S S^T R^T within sampling error."""
    sc = scenegen.random_scene(33, 1)
    sc.log_scales4[:] = [[math.log(0.3), math.log(0.1), math.log(0.05), math.log(0.2)]]
    rng = np.random.default_rng(34)
    z = rng.normal(size=(200_000, 4))
    x = OP.split_sample(sc, np.zeros(200_000, np.int64), z)
    cov = O.covariance_4d(torch.as_tensor(sc.log_scales4, dtype=torch.float64),
                          torch.as_tensor(sc.q_left, dtype=torch.float64),
                          torch.as_tensor(sc.q_right, dtype=torch.float64))[0].numpy()
    emp = np.cov(x.T)
    scale = np.sqrt(np.outer(np.diag(cov), np.diag(cov)))
    assert np.abs(emp - cov).max() <= 0.02 * scale.max()
    assert np.abs(x.mean(0) - sc.means4[0]).max() <= 5 * math.sqrt(cov.diagonal().max() / 200_000)
