"""One random-walk Metropolis step (Sec. V, Metropolis sampler), oracle side.

All electrons move at once: r' = r + tau * xi with xi ~ N(0, 1) per
coordinate.  The proposal is accepted when log(u) < 2 (log|psi(r')| -
log|psi(r)|), i.e. with probability min(1, |psi(r')|^2 / |psi(r)|^2); the
comparison is strict and taken in float64, so u = 0 always accepts and a
proposal with log|psi| = -inf or NaN is always rejected.  The noise xi and the
uniforms u are inputs; log|psi(r)| of the current state is an input too (it
is cached by the caller, not recomputed).
"""
from __future__ import annotations

import numpy as np
import torch

from .ansatz import logpsi


def metropolis_step(r, logpsi_cur, noise, u, step, params, system, ans, chunk=256):
    """Returns (r_new, logpsi_new, accepted) as numpy arrays."""
    r = np.asarray(r, dtype=np.float64)
    prop = r + np.float64(step) * np.asarray(noise, dtype=np.float64)
    theta = torch.as_tensor(np.asarray(params, dtype=np.float64))
    lp_new = []
    with torch.no_grad():
        for s in range(0, r.shape[0], chunk):
            lp_new.append(logpsi(torch.as_tensor(prop[s:s + chunk]), theta, system, ans)[1].numpy())
    lp_prop = np.concatenate(lp_new)
    with np.errstate(divide="ignore", invalid="ignore"):
        acc = np.log(np.asarray(u, dtype=np.float64)) < 2.0 * (lp_prop - np.asarray(logpsi_cur))
    r_new = np.where(acc[:, None, None], prop, r)
    lp_out = np.where(acc, lp_prop, logpsi_cur)
    return r_new, lp_out, acc.astype(np.uint8), lp_prop
