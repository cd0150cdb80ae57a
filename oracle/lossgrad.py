"""VMC loss-gradient estimator (Sec. IV.A, loss-gradient equation), oracle side.

G = 2 E[(E_loc - L) grad_theta log|psi|], estimated over the W_f walkers whose
local energy is finite: L is their mean local energy (float64, unclipped) and
G = (2 / W_f) sum_w (E_w - L) grad_theta log|psi_w|.  The gradient is taken by
reverse-mode autograd of the surrogate S(theta) = (2/W_f) sum_w g_w
log|psi_w(theta)| with g_w = E_w - L frozen, so only first derivatives of
log|psi| with respect to the parameters appear.
"""
from __future__ import annotations

import numpy as np
import torch

from .ansatz import logpsi


def surrogate(theta, r, weights, system, ans):
    """S(theta) = sum_w weights_w log|psi_w(theta)| (torch scalar)."""
    _, lp = logpsi(torch.as_tensor(r), theta, system, ans)
    return (torch.as_tensor(weights) * lp).sum()


def loss_grad(r, e_loc, params, system, ans, chunk=256):
    """Returns (G [P] numpy float64, mean local energy, number of finite walkers)."""
    e = np.asarray(e_loc, dtype=np.float64)
    ok = np.isfinite(e)
    nf = int(ok.sum())
    if nf == 0:
        return np.zeros_like(np.asarray(params, dtype=np.float64)), float("nan"), 0
    e_mean = float(np.mean(e[ok]))
    wts = np.where(ok, 2.0 * (np.where(ok, e, 0.0) - e_mean) / nf, 0.0)
    r = np.asarray(r, dtype=np.float64)
    G = np.zeros(np.asarray(params).shape[0])
    for s in range(0, r.shape[0], chunk):
        sel = ok[s:s + chunk]
        if not sel.any():
            continue
        theta = torch.tensor(np.asarray(params, dtype=np.float64), requires_grad=True)
        S = surrogate(theta, r[s:s + chunk][sel], wts[s:s + chunk][sel], system, ans)
        G += torch.autograd.grad(S, theta)[0].numpy()
    return G, e_mean, nf
