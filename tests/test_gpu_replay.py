"""Metropolis replay of the N2-sized workload in the configuration the benchmark runs (Sec. V).

Ten random-walk steps of size 0.2 bohr on all 4096 walkers with the float32 autotuned plan; the
oracle replays the first 256 walkers step by step from the GPU's state, on the same noise and
uniforms.  Decisions may differ only where |log u - 2 (l' - l)| is below the margin
delta = 2 x the float32 log|psi| bound at the proposal (max(2e-4, 1e-7 alpha), alpha the oracle's
amplification of the orbital-matrix rounding); every such flip is counted and printed, any other
difference fails.
After each step the oracle is re-synchronised to the GPU's walkers.
"""
import numpy as np
import pytest
import torch

import oracle
import qmc_inputs as qi
from tests.gpu_common import dev, host
from tests.test_gpu_parity import amplification, fp32_logpsi_bound

pytestmark = pytest.mark.gpu


def test_n2_metropolis_replay_fp32_ten_steps():
    from paper_2307_14123_amd import qmc
    wl = qi.workload(1)
    s, a, p, r = qi.workload_inputs(1)
    W, n_steps, tau, n_check = r.shape[0], wl.metropolis_steps or 10, wl.step_size, 256
    noise = qi.make_noise(n_steps, W, s.n_elec, qi.seed(1, 2))
    u = qi.make_uniforms(n_steps, W, qi.seed(1, 3))
    plan = qmc.Plan([s], [W], a, "fp32", autotune=True)
    P, R = dev(p, torch.float32), dev(r)
    lp, _ = plan.logpsi(P, R)
    torch.cuda.synchronize()
    pr = p.astype(np.float32).astype(np.float64)
    flips = 0
    accepted = 0
    for t in range(n_steps):
        r_before = host(R).reshape(r.shape)[:n_check].copy()
        lp_before = host(lp)[:n_check].copy()
        print(f"[n2 replay fp32] step {t}", flush=True)
        acc = host(plan.metropolis_step(P, R, lp, dev(noise[t]), dev(u[t]), tau))[:n_check]
        torch.cuda.synchronize()
        r_o, lp_o, acc_o, prop = oracle.metropolis_step(r_before, lp_before, noise[t][:n_check], u[t][:n_check],
                                                        tau, pr, s, a)
        alpha = amplification(r_before + tau * noise[t][:n_check], p, s, a)
        delta = 2.0 * fp32_logpsi_bound(alpha)
        with np.errstate(divide="ignore", invalid="ignore"):
            margin = np.abs(np.log(u[t][:n_check]) - 2.0 * (prop - lp_before))
        differ = acc != acc_o
        assert np.all(margin[differ] < delta[differ]), (t, np.nonzero(differ & (margin >= delta)))
        flips += int(differ.sum())
        accepted += int(acc.sum())
        # accepted walkers: the GPU's new log|psi| is the proposal's, within the float32 bound
        lp_now = host(lp)[:n_check]
        same = ~differ & (acc == 1)
        assert np.all(np.abs(lp_now[same] - prop[same]) <= fp32_logpsi_bound(alpha[same]))
        # positions follow the decision exactly (the proposal r + tau xi is formed in float64)
        r_now = host(R).reshape(r.shape)[:n_check]
        np.testing.assert_array_equal(r_now[~differ], r_o[~differ])
    print(f"[n2 replay fp32] {n_steps} steps x {n_check} walkers: acceptance {accepted / (n_steps * n_check):.3f}, "
          f"within-margin flips {flips}", flush=True)
