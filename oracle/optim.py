"""One optimisation step of UBS (Sec. 4.5, "Optimization and Implementation"):
the loss regularisers, an Adam update per parameter group, and the spatial
noise injection.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``): plain float64 numpy,
written from the paper, used to check the HIP kernel.

The loss of Sec. 4.5 adds lambda_o sum_i |o_i| + lambda_Sigma sum_i ||s_i||_1
to the reconstruction terms, so the parameter gradient gains
  d/d o_i          = lambda_o sign(o_i)          (opacity stored activated)
  d/d log s_{i,k}  = lambda_Sigma exp(log s_{i,k})  (s = exp(log s) > 0).
Training uses Adam with the learning rates of Sec. 5.1 (positions 1.6e-4,
opacity 5e-2, scales 5e-3, every other parameter 1e-3) and the spatial means
then receive lambda_eps * epsilon, epsilon given by the caller (the noise
the method draws is an input here).  Readings (the paper is silent): the
noise is added after the Adam step; Adam's betas (0.9, 0.999) and epsilon
(1e-15) are the conventional ones; nothing is clamped.
"""
from __future__ import annotations

import numpy as np

from .preprocess import field_slices

PAPER_LR = {"mu_x": 1.6e-4, "o": 5e-2, "log_s": 5e-3, "other": 1e-3}
LAMBDA_O = 0.01
LAMBDA_S = 0.01
LAMBDA_EPS = 1.0


def row_groups(dim: int, rot: int) -> list:
    """Learning-rate group of every parameter row: 'mu_x', 'o', 'log_s' or
    'other'."""
    sl = field_slices(dim, rot)
    F = max(s.stop for s in sl.values())
    groups = ["other"] * F
    for name in ("mu_x", "o"):
        for r in range(sl[name].start, sl[name].stop):
            groups[r] = name
    for r in range(sl["log_s_x"].start, sl["log_s_x"].stop):
        groups[r] = "log_s"
    return groups


def regulariser_value(params: np.ndarray, dim: int, rot: int, lambda_o: float,
                      lambda_s: float) -> float:
    """lambda_o sum |o| + lambda_Sigma sum ||s||_1 with s = exp(log s)."""
    sl = field_slices(dim, rot)
    P = np.asarray(params, dtype=np.float64)
    return float(lambda_o * np.abs(P[sl["o"]]).sum() + lambda_s * np.exp(P[sl["log_s_x"]]).sum())


def regulariser_grad(params: np.ndarray, dim: int, rot: int, lambda_o: float,
                     lambda_s: float) -> np.ndarray:
    """Gradient of regulariser_value with respect to params (sign(0) = 0)."""
    sl = field_slices(dim, rot)
    P = np.asarray(params, dtype=np.float64)
    G = np.zeros_like(P)
    G[sl["o"]] = lambda_o * np.sign(P[sl["o"]])
    G[sl["log_s_x"]] = lambda_s * np.exp(P[sl["log_s_x"]])
    return G


def adam_step(params, dparams, m, v, step: int, dim: int, rot: int, lr=None,
              beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-15,
              lambda_o: float = LAMBDA_O, lambda_s: float = LAMBDA_S,
              lambda_eps: float = LAMBDA_EPS, noise=None):
    """One step; returns (params, m, v) as new float64 arrays.

    g = dparams + regulariser gradient; per row with its group's rate lr:
      m <- beta1 m + (1 - beta1) g,  v <- beta2 v + (1 - beta2) g^2,
      p <- p - lr * (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps);
    then mu_x <- mu_x + lambda_eps * noise (noise [3][n], or None)."""
    lr = dict(PAPER_LR if lr is None else lr)
    P = np.array(params, dtype=np.float64)
    M = np.array(m, dtype=np.float64)
    V = np.array(v, dtype=np.float64)
    g = np.asarray(dparams, dtype=np.float64) + regulariser_grad(P, dim, rot, lambda_o, lambda_s)
    M = beta1 * M + (1.0 - beta1) * g
    V = beta2 * V + (1.0 - beta2) * g * g
    m_hat = M / (1.0 - beta1 ** step)
    v_hat = V / (1.0 - beta2 ** step)
    rate = np.array([lr[grp] for grp in row_groups(dim, rot)])[:, None]
    P = P - rate * m_hat / (np.sqrt(v_hat) + eps)
    if noise is not None:
        sl = field_slices(dim, rot)
        P[sl["mu_x"]] += lambda_eps * np.asarray(noise, dtype=np.float64)
    return P, M, V
