"""One random-walk Metropolis step (Sec. V, Metropolis sampler) and one
Metropolis-adjusted Langevin step (Sec. V, Langevin sampler), oracle side.

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


def logpsi_and_grad(r, params, system, ans, chunk=256):
    """log|psi| and its gradient over the electron coordinates by one reverse pass (numpy float64,
    [W], [W, N, 3]); the gradient is NaN where log|psi| is not finite."""
    r = np.asarray(r, dtype=np.float64)
    theta = torch.as_tensor(np.asarray(params, dtype=np.float64))
    lps, grads = [], []
    for s in range(0, r.shape[0], chunk):
        x = torch.as_tensor(r[s:s + chunk]).clone().requires_grad_(True)
        lp = logpsi(x, theta, system, ans)[1]
        g = torch.autograd.grad(lp.sum(), x, allow_unused=True)[0]
        g = torch.zeros_like(x) if g is None else g
        bad = ~torch.isfinite(lp)
        g = torch.where(bad[:, None, None], torch.full_like(g, float("nan")), g)
        lps.append(lp.detach().numpy())
        grads.append(g.detach().numpy())
    return np.concatenate(lps), np.concatenate(grads)


def drift_damping_a(zd):
    """Damping strength a(Z d) of the drift limit of Umrigar, Nightingale and Runge (J. Chem. Phys.
    99, 2865 (1993)) with its angular term at its mean: a = 1/2 + (Z d)^2 / (10 (4 + (Z d)^2)), so
    a = 1/2 on a nucleus and a -> 3/5 far from it."""
    zd2 = np.asarray(zd, dtype=np.float64) ** 2
    return 0.5 + zd2 / (10.0 * (4.0 + zd2))


def langevin_drift(r, grad, tau, system, damp=True):
    """Drift velocity D(r) of the Langevin proposal r' = r + tau D(r) + sqrt(tau) xi, [W, N, 3].

    Without damping D = grad log|psi|.  With damping (the step-size correction near nuclei that the
    paper takes from Hermann et al.; its form is not printed there, this is the reading used here),
    each electron's v = grad_i log|psi| is shortened as
        v_bar = v * 2 / (1 + sqrt(1 + 2 a |v|^2 tau))      (the same as (sqrt(1 + 2x) - 1) / x, x = a|v|^2 tau)
    with a = drift_damping_a(Z d) for its nearest nucleus (charge Z, distance d, lowest index on
    ties), and then capped so that the drift step tau |v_bar| does not exceed d."""
    r = np.asarray(r, dtype=np.float64)
    g = np.asarray(grad, dtype=np.float64)
    if not damp:
        return g.copy()
    R, Z = system.R(), system.Z()
    dist = np.linalg.norm(r[:, :, None, :] - R[None, None], axis=-1)  # [W, N, M]
    idx = np.argmin(dist, axis=-1)
    d = np.take_along_axis(dist, idx[..., None], -1)[..., 0]
    a = drift_damping_a(Z[idx] * d)
    v2 = (g * g).sum(-1)
    vb = g * (2.0 / (1.0 + np.sqrt(1.0 + 2.0 * a * v2 * tau)))[..., None]
    step_len = tau * np.linalg.norm(vb, axis=-1)
    with np.errstate(divide="ignore", invalid="ignore"):
        cap = np.where(step_len > d, d / step_len, 1.0)
    return vb * cap[..., None]


def mala_log_accept(lp_cur, drift_cur, lp_prop, drift_prop, noise, step):
    """log of the Metropolis-Hastings acceptance ratio of a Langevin proposal.

    Target |psi|^2 = exp(2 l); proposal r' = r + eps^2 D(r) + eps xi (overdamped Langevin with time
    step tau = eps^2, eps = step), so q(x | y) = N(x; y + eps^2 D(y), eps^2).  With
    r' - r - eps^2 D = eps xi and r - r' - eps^2 D' = -eps (xi + eps (D + D')):
        log a = 2 (l' - l) + |xi|^2 / 2 - |xi + eps (D + D')|^2 / 2."""
    xi = np.asarray(noise, dtype=np.float64)
    W = xi.shape[0]
    xi = xi.reshape(W, -1)
    g = np.asarray(drift_cur, dtype=np.float64).reshape(W, -1)
    gp = np.asarray(drift_prop, dtype=np.float64).reshape(W, -1)
    back = xi + np.float64(step) * (g + gp)
    return 2.0 * (np.asarray(lp_prop) - np.asarray(lp_cur)) + 0.5 * (xi * xi).sum(1) - 0.5 * (back * back).sum(1)


def mala_step(r, logpsi_cur, grad_cur, noise, u, step, params, system, ans, damp=True, chunk=256):
    """One Metropolis-adjusted Langevin step (Sec. V, Langevin sampler), oracle side.

    All electrons move at once: r' = (r + eps^2 D(r)) + eps xi with eps = step, tau = eps^2,
    xi ~ N(0, 1) per coordinate and D the (damped) drift of langevin_drift; the proposal is
    accepted when log(u) < log a (mala_log_accept), strictly and in float64, so a non-finite
    log|psi(r')| or gradient rejects.  The gradient at the current state is an input (cached by
    the caller with log|psi|).  Returns (r_new, logpsi_new, grad_new, accepted, r_proposed)."""
    r = np.asarray(r, dtype=np.float64)
    g = np.asarray(grad_cur, dtype=np.float64)
    eps = np.float64(step)
    tau = eps * eps
    with np.errstate(divide="ignore", invalid="ignore"):
        drift = langevin_drift(r, g, tau, system, damp)
        prop = (r + tau * drift) + eps * np.asarray(noise, dtype=np.float64)
    lp_prop, g_prop = logpsi_and_grad(prop, params, system, ans, chunk)
    with np.errstate(divide="ignore", invalid="ignore"):
        drift_prop = langevin_drift(prop, g_prop, tau, system, damp)
        la = mala_log_accept(logpsi_cur, drift, lp_prop, drift_prop, noise, step)
        acc = np.log(np.asarray(u, dtype=np.float64)) < la
    r_new = np.where(acc[:, None, None], prop, r)
    lp_out = np.where(acc, lp_prop, logpsi_cur)
    g_out = np.where(acc[:, None, None], g_prop, g)
    return r_new, lp_out, g_out, acc.astype(np.uint8), prop
