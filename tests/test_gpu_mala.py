"""Langevin (MALA) step of the HIP path (through the C ABI) against the FP64 oracle.

Replay parity: both sides start each step from the GPU's state; acceptance decisions must agree
except where |log u - log a| is below a margin set by the precision; for agreeing walkers the
positions, log|psi| and gradients must match.  The gradient at the proposal comes from the reverse
pass (qmc_logpsi_grad's path).  H2 (256 walkers of the small workload) and the
N2-sized ansatz on a walker subset, with and without the drift damping near nuclei.
"""
import numpy as np
import pytest
import torch

import oracle
import qmc_inputs as qi
from tests.gpu_common import dev, host, rel_err

pytestmark = pytest.mark.gpu


def _q():
    from paper_2307_14123_amd import qmc
    return qmc


def _oracle_log_accept(r, lp, g, prop, noise, step, s, a, p, damp):
    tau = step * step
    D = oracle.langevin_drift(r, g, tau, s, damp)
    lpp, gp = oracle.logpsi_and_grad(prop, p, s, a)
    Dp = oracle.langevin_drift(prop, gp, tau, s, damp)
    return oracle.mala_log_accept(lp, D, lpp, Dp, noise, step)


def _replay(k, W, prec, damp, step, n_steps, margin, tol_r, tol_lp, tol_g):
    s, a, p, r = qi.workload_inputs(k, W)
    q = _q()
    plan = q.Plan([s], [W], a, prec)
    P = dev(p, torch.float64 if prec == "fp64" else torch.float32)
    R = dev(r)
    out = plan.local_energy(P, R)
    lp, G = out["logpsi"], out["grad"]
    torch.cuda.synchronize()
    lp0, g0 = oracle.logpsi_and_grad(r, p, s, a)
    assert rel_err(host(lp), lp0).max() < tol_lp
    assert np.abs(host(G).reshape(r.shape) - g0).max() / max(1.0, np.abs(g0).max()) < tol_g
    noise = qi.make_noise(n_steps, W, s.n_elec, 11)
    u = qi.make_uniforms(n_steps, W, 12)
    n_acc = 0
    for t in range(n_steps):
        r_o, lp_o, g_o = host(R).reshape(r.shape).copy(), host(lp).copy(), host(G).reshape(r.shape).copy()
        acc = plan.mala_step(P, R, lp, G, dev(noise[t]), dev(u[t]), step, damp=damp)
        torch.cuda.synchronize()
        r2, lp2, g2, acc_o, prop = oracle.mala_step(r_o, lp_o, g_o, noise[t], u[t], step, p, s, a, damp=damp)
        la = _oracle_log_accept(r_o, lp_o, g_o, prop, noise[t], step, s, a, p, damp)
        acc_g = host(acc).astype(bool)
        same = acc_g == acc_o.astype(bool)
        close = np.abs(np.log(u[t]) - la) < margin
        assert (same | close).all(), f"step {t}: decisions differ beyond the margin"
        ok = same
        Rg = host(R).reshape(r.shape)
        np.testing.assert_allclose(Rg[ok], r2[ok], rtol=tol_r, atol=tol_r)
        assert rel_err(host(lp)[ok], lp2[ok]).max() < tol_lp
        Gg = host(G).reshape(r.shape)
        gerr = np.abs(Gg[ok] - g2[ok]).reshape(ok.sum(), -1).max(1) / np.maximum(
            1.0, np.abs(g2[ok]).reshape(ok.sum(), -1).max(1))
        assert gerr.max() < tol_g
        n_acc += int(acc_g.sum())
    frac = n_acc / (W * n_steps)
    print(f"[mala {prec} damp={damp}] acceptance {frac:.3f}", flush=True)
    assert 0.05 < frac < 0.999


@pytest.mark.parametrize("damp", [False, True])
def test_mala_replay_h2_fp64(damp):
    _replay(0, 256, "fp64", damp, 0.4, 3, 1e-8, 1e-12, 1e-10, 1e-8)


def test_mala_replay_n2_subset_fp64():
    _replay(1, 40, "fp64", True, 0.15, 2, 1e-8, 1e-12, 1e-10, 1e-8)


def test_mala_replay_n2_subset_fp32():
    # float32 network: log|psi| to ~1e-5 relative, gradients to ~1e-3 of their largest component
    _replay(1, 40, "fp32", True, 0.15, 2, 5e-2, 1e-4, 1e-4, 5e-3)


def test_mala_zero_step_keeps_state():
    """step = 0 proposes the current positions: every walker accepts, the positions keep every bit,
    and log|psi| and the gradient become those of the reverse pass at the same positions (equal to
    the jet forward's to rounding)."""
    s, a, p, r = qi.workload_inputs(0, 16)
    q = _q()
    plan = q.Plan([s], [16], a, "fp64")
    P, R = dev(p), dev(r)
    out = plan.local_energy(P, R)
    lp, G = out["logpsi"].clone(), out["grad"].clone()
    g_before, lp_before = host(G).copy(), host(lp).copy()
    acc = plan.mala_step(P, R, lp, G, dev(np.ones((16, 2, 3))), dev(np.full(16, 0.5)), 0.0)
    lp_rev, g_rev = plan.logpsi_grad(P, R)
    torch.cuda.synchronize()
    assert np.all(host(acc) == 1)
    np.testing.assert_array_equal(host(R).reshape(r.shape), r)
    np.testing.assert_array_equal(host(G), host(g_rev))
    np.testing.assert_array_equal(host(lp), host(lp_rev))
    np.testing.assert_allclose(host(G), g_before, rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(host(lp), lp_before, rtol=1e-12, atol=1e-12)
