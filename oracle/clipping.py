"""Clipped local energies for the loss gradient (Sec. IV.D, gradient clipping), oracle side.

The window is centred at the median mu of the finite local energies and its half-width is
sigma = width x (mean absolute deviation of the finite local energies from mu).  Two shapes:

  hard: E -> min(max(E, mu - sigma), mu + sigma);
  soft: E unchanged inside the window; outside, mu +- sigma (1 + log(|E - mu| / sigma)), which
        joins the window edge continuously with slope 1 and then grows logarithmically (the
        paper names a logarithmic soft scheme without its formula; this form is the reading).

Non-finite local energies pass through unchanged (the loss gradient excludes them); with no
finite value, or sigma = 0, every value passes through unchanged.  Clipped values only enter
the loss gradient, never an energy estimate.
"""
from __future__ import annotations

import numpy as np


def clip_local_energy(e_loc, width=5.0, mode="hard"):
    e = np.asarray(e_loc, dtype=np.float64)
    out = e.copy()
    fin = np.isfinite(e)
    if not fin.any():
        return out
    x = e[fin]
    mu = np.median(x)
    sigma = width * np.mean(np.abs(x - mu))
    if not sigma > 0:
        return out
    if mode == "hard":
        out[fin] = np.minimum(np.maximum(x, mu - sigma), mu + sigma)
    elif mode == "soft":
        dev = np.abs(x - mu)
        far = dev > sigma
        y = x.copy()
        y[far] = mu + np.sign(x[far] - mu) * sigma * (1.0 + np.log(dev[far] / sigma))
        out[fin] = y
    else:
        raise ValueError(mode)
    return out
