"""FP64 CPU oracle of the training-step tail: the Adam update of the
primitive parameters and the 4D split sampling.

TEST INFRASTRUCTURE ONLY: only the test suite may import this module; the
product path never calls it. It shares no code with the HIP implementation.

Passages followed (Yang et al., ICLR 2024):
  * Sec. 4.2: training takes the optimiser settings of 3D Gaussian Splatting,
    i.e. Adam (Kingma & Ba) with a learning rate per parameter group.
  * Sec. 3.3 "Densification in spacetime" and the ablation of Sec. 4.4:
    a split primitive's new positions are drawn from its complete 4D
    Gaussian N(mu, Sigma), Sigma = (R S)(R S)^T.
Reading: a sample is mu + R S z with z ~ N(0, I_4) supplied by the caller
(any square root of Sigma gives the same distribution; R S is the one the
representation defines).
"""
from __future__ import annotations

from typing import Dict, Sequence

import numpy as np
import torch

from oracle import render4d as O

GROUPS = ("means4", "log_scales4", "q_left", "q_right", "opacity_logit", "coeffs")


def adam_step(params: Dict[str, np.ndarray], grads: Dict[str, np.ndarray], m: Dict[str, np.ndarray],
              v: Dict[str, np.ndarray], step: int, lr: Sequence[float], beta1: float, beta2: float,
              eps: float):
    """One Adam step, written out from its definition, per group g:
    m = b1 m + (1 - b1) g; v = b2 v + (1 - b2) g^2;
    p -= lr_g * (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).
    Returns new (params, m, v) as float64 arrays; inputs are not modified."""
    bc1 = 1.0 - beta1 ** step
    bc2 = 1.0 - beta2 ** step
    out_p, out_m, out_v = {}, {}, {}
    for gi, name in enumerate(GROUPS):
        p = np.asarray(params[name], np.float64)
        g = np.asarray(grads[name], np.float64)
        mm = beta1 * np.asarray(m[name], np.float64) + (1.0 - beta1) * g
        vv = beta2 * np.asarray(v[name], np.float64) + (1.0 - beta2) * g * g
        out_p[name] = p - lr[gi] * (mm / bc1) / (np.sqrt(vv / bc2) + eps)
        out_m[name] = mm
        out_v[name] = vv
    return out_p, out_m, out_v


def split_sample(scene, idx: np.ndarray, z: np.ndarray) -> np.ndarray:
    """New 4D positions mu_i + R_i S_i z_k for the primitives idx[k] and the
    standard-normal draws z[k] ([K, 4]). Returns float64 [K, 4]."""
    p = O.params_from_scene(scene)
    i = torch.as_tensor(np.asarray(idx, np.int64))
    R = O.rotation_4d(p["q_left"][i], p["q_right"][i])
    s = torch.exp(p["log_scales4"][i])
    zz = torch.as_tensor(np.asarray(z, np.float64))
    return (p["means4"][i] + torch.einsum("kij,kj->ki", R, s * zz)).numpy()
