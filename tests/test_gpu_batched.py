"""Batched molecules of different sizes in one plan.

* Concurrent execution (one stream per molecule, forked from and joined to the
  caller's stream) gives the same local energies, Metropolis moves and loss
  gradients, bit for bit, as the molecules run one after another: the kernels
  and their reduction orders are the same.
* The FP64 concurrent plan matches the oracle on every molecule.
* The local energy and loss gradient of a concurrent plan, captured into one
  graph, replay correctly three times in a row with eager work in between.
* Autotuned GEMM tiles (K-step, tile height, persistent grid) change no bit of
  the results, since every candidate sums each output in the same order.

Molecules are taken from the seeded batch generator (2-6 nuclei, Z in
{1, 3, 6, 7, 8}, neutral) at 4-22 electrons, with ragged walker counts.
"""
import numpy as np
import pytest
import torch

import oracle
import qmc_inputs as qi
from tests.gpu_common import dev, host
from tests.test_gpu_parity import flagged

pytestmark = pytest.mark.gpu


def _q():
    from paper_2307_14123_amd import qmc
    return qmc


def _batch(targets, walkers, seed=4004):
    mols = qi.make_molecules(seed, targets)
    a = qi.BATCH_ANSATZ
    params = [qi.make_params(s, a, 700 + k) for k, s in enumerate(mols)]
    pos = [qi.make_walkers(s, w, 800 + k) for k, (s, w) in enumerate(zip(mols, walkers))]
    return mols, a, params, pos


def _cat(xs):
    return np.concatenate([np.ravel(x) for x in xs])


def _step(plan, P, R, noise, u):
    out = plan.local_energy(P, R)
    g, em = plan.loss_grad(P, R, out["e_loc"])
    r2 = R.clone()
    lp = out["logpsi"].clone()
    acc = plan.metropolis_step(P, r2, lp, noise, u, 0.2)
    torch.cuda.synchronize()
    res = {k: host(v) for k, v in out.items()}
    res.update(grad_params=host(g), e_mean=host(em), r_new=host(r2), lp_new=host(lp), acc=host(acc))
    return res


def test_concurrent_matches_sequential_bitwise():
    targets, walkers = [4, 9, 14, 22], [24, 16, 20, 12]
    mols, a, params, pos = _batch(targets, walkers)
    q = _q()
    P = dev(_cat(params), torch.float32)
    R = dev(_cat(pos))
    W = sum(walkers)
    noise = dev(np.random.default_rng(901).standard_normal(R.numel()))
    u = dev(np.random.default_rng(902).random(W))
    seq = _step(q.Plan(mols, walkers, a, "fp32"), P, R, noise, u)
    con = _step(q.Plan(mols, walkers, a, "fp32", concurrent=True), P, R, noise, u)
    for k in seq:
        np.testing.assert_array_equal(con[k], seq[k], err_msg=k)
    assert np.all(np.isfinite(seq["e_loc"]))
    print(f"[concurrent vs sequential] {len(mols)} molecules, {W} walkers: bitwise equal", flush=True)


def test_concurrent_langevin_and_gradient_bitwise():
    """The reverse-pass gradient and a Langevin step over a concurrent plan equal the same calls on
    one plan per molecule (each molecule's walkers and outputs at its offsets)."""
    targets, walkers = [4, 9, 14], [12, 20, 8]
    mols, a, params, pos = _batch(targets, walkers)
    q = _q()
    con = q.Plan(mols, walkers, a, "fp32", concurrent=True)
    P, R = dev(_cat(params), torch.float32), dev(_cat(pos))
    lp, g = con.logpsi_grad(P, R)
    W = sum(walkers)
    noise = np.random.default_rng(903).standard_normal(R.numel())
    u = np.random.default_rng(904).random(W)
    R2, lp2, g2 = R.clone(), lp.clone(), g.clone()
    acc = con.mala_step(P, R2, lp2, g2, dev(noise), dev(u), 0.1)
    torch.cuda.synchronize()
    w0, x0 = 0, 0
    for m, p, r, w in zip(mols, params, pos, walkers):
        one = q.Plan([m], [w], a, "fp32")
        Pm, Rm = dev(p, torch.float32), dev(r)
        lpm, gm = one.logpsi_grad(Pm, Rm)
        n3 = w * m.n_elec * 3
        accm = one.mala_step(Pm, Rm, lpm, gm, dev(noise[x0:x0 + n3]), dev(u[w0:w0 + w]), 0.1)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(host(acc)[w0:w0 + w], host(accm))
        np.testing.assert_array_equal(host(R2)[x0:x0 + n3], host(Rm).ravel())
        np.testing.assert_array_equal(host(lp2)[w0:w0 + w], host(lpm))
        np.testing.assert_array_equal(host(g2)[x0:x0 + n3], host(gm))
        w0 += w
        x0 += n3


def test_concurrent_fp64_matches_oracle():
    targets, walkers = [4, 9], [6, 5]
    mols, a, params, pos = _batch(targets, walkers)
    q = _q()
    plan = q.Plan(mols, walkers, a, "fp64", concurrent=True)
    out = plan.local_energy(dev(_cat(params)), dev(_cat(pos)))
    torch.cuda.synchronize()
    e = host(out["e_loc"])
    w0 = 0
    for s, p, r, w in zip(mols, params, pos, walkers):
        ref = oracle.local_energy(r, p, s, a)
        ok = ~flagged(r, p, s, a)
        scale = np.maximum.reduce([np.abs(ref["e_loc"]), 0.5 * np.abs(ref["lap"]),
                                   0.5 * (ref["grad"] ** 2).sum((1, 2)), np.ones(w)])
        err = (np.abs(e[w0:w0 + w] - ref["e_loc"]) / scale)[ok]
        print(f"[concurrent fp64 N={s.n_up + s.n_down}] max rel E_L err {err.max():.3e}", flush=True)
        assert ok.sum() >= w // 2 and err.max() < 1e-10
        w0 += w


def test_graph_replays_match_eager():
    targets, walkers = [4, 14, 22], [32, 16, 24]
    mols, a, params, pos = _batch(targets, walkers)
    q = _q()
    plan = q.Plan(mols, walkers, a, "fp32", concurrent=True)
    P = dev(_cat(params), torch.float32)
    R = dev(_cat(pos))
    step = q.GraphStep(plan, P, R)
    rng = np.random.default_rng(903)
    for k in range(3):
        newr = _cat(pos) + 0.1 * rng.standard_normal(R.numel())
        R.copy_(dev(newr))
        step.replay()
        torch.cuda.synchronize()
        got = {n: host(t).copy() for n, t in step.out.items()}
        # eager work between replays, on the same plan and workspace
        ref = plan.local_energy(P, R)
        g, em = plan.loss_grad(P, R, ref["e_loc"])
        torch.cuda.synchronize()
        for n in ("logpsi", "sign", "grad", "lap", "e_loc"):
            np.testing.assert_array_equal(got[n], host(ref[n]), err_msg=f"replay {k}: {n}")
        np.testing.assert_array_equal(got["param_grad"], host(g), err_msg=f"replay {k}: param_grad")
        np.testing.assert_array_equal(got["e_mean"], host(em), err_msg=f"replay {k}: e_mean")
    print(f"[graph] 3 replays of E_L + loss gradient over {len(mols)} molecules equal eager", flush=True)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_autotuned_tiles_bitwise(precision):
    targets, walkers = [7, 17], [40, 24]
    mols, a, params, pos = _batch(targets, walkers)
    q = _q()
    dt = torch.float64 if precision == "fp64" else torch.float32
    P = dev(_cat(params), dt)
    R = dev(_cat(pos))
    W = sum(walkers)
    noise = dev(np.random.default_rng(904).standard_normal(R.numel()))
    u = dev(np.random.default_rng(905).random(W))
    tuned = q.Plan(mols, walkers, a, precision, autotune=True)
    tiles = tuned.tiles()
    print(f"[autotune {precision}] tiles per molecule (jet, value, edge, backward): {tiles}", flush=True)
    assert all(t > 0 for row in tiles for t in row)
    ref = _step(q.Plan(mols, walkers, a, precision), P, R, noise, u)
    got = _step(tuned, P, R, noise, u)
    for k in ref:
        np.testing.assert_array_equal(got[k], ref[k], err_msg=k)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_workload_molecules_vs_oracle(precision):
    """Four molecules of the 16-molecule batch (4, 17, 29 and 42 electrons: the smallest and the
    largest, spin blocks of 2 to 21 electrons, both aggregation kernels), 2 walkers each, in one
    concurrent plan: local energies and the loss gradient against the oracle (float64: 1e-10 of
    the largest E_L addend and normwise; float32: the amplification-scaled bounds)."""
    from tests.test_gpu_parity import amplification, fp32_eloc_bound, fp32_grad_bound
    wl = qi.workload(4)
    a = wl.ansatz
    idx = [0, 5, 10, 15]
    mols = [wl.systems[k] for k in idx]
    assert [m.n_elec for m in mols] == [4, 17, 29, 42]
    params = [qi.make_params(m, a, qi.seed(4, 10 + k)) for k, m in zip(idx, mols)]
    pos = [qi.make_walkers(m, 2, qi.seed(4, 40 + k)) for k, m in zip(idx, mols)]
    q = _q()
    plan = q.Plan(mols, [2] * 4, a, precision, concurrent=True)
    P, R = dev(_cat(params), plan.param_dtype), dev(_cat(pos))
    out = plan.local_energy(P, R)
    g, em = plan.loss_grad(P, R, out["e_loc"])
    torch.cuda.synchronize()
    e = host(out["e_loc"])
    G = host(g).astype(np.float64)
    p0 = 0
    for k, (s, p, r) in enumerate(zip(mols, params, pos)):
        pr = p.astype(np.float32).astype(np.float64) if precision == "fp32" else p
        ref = oracle.local_energy(r, pr, s, a)
        scale = np.maximum.reduce([np.abs(ref["e_loc"]), 0.5 * np.abs(ref["lap"]),
                                   0.5 * (ref["grad"] ** 2).sum((1, 2)), np.ones(2)])
        err = np.abs(e[2 * k:2 * k + 2] - ref["e_loc"]) / scale
        Gref, em_ref, _ = oracle.loss_grad(r, e[2 * k:2 * k + 2], pr, s, a)
        n = len(p)
        gerr = np.linalg.norm(G[p0:p0 + n] - Gref) / np.linalg.norm(Gref)
        alpha = amplification(r, p, s, a)
        print(f"[batch {precision} N={s.n_elec}] E_L/scale {err.max():.3e} (alpha {alpha.max():.3g}), "
              f"loss gradient {gerr:.3e}, E mean {host(em)[k]:.6f} vs {em_ref:.6f}", flush=True)
        if precision == "fp64":
            assert err.max() < 1e-10 and gerr < 1e-10
        else:
            assert np.all(err <= fp32_eloc_bound(alpha)) and gerr < fp32_grad_bound(alpha)
        p0 += n


def test_large_spin_blocks_fp32_vs_oracle():
    """The float32 jet aggregation's register form for large spin blocks, against the oracle: 17 + 17
    electrons (20 sender slots, two receivers per thread) and 26 + 26 electrons (32 slots, one receiver
    per thread), each with its receiver groups split over several blocks, in one concurrent plan;
    local energies within the amplification-scaled float32 bound and the loss gradient within its
    bound (oracle at the float32-rounded parameters)."""
    from tests.test_gpu_parity import amplification, fp32_eloc_bound, fp32_grad_bound
    wl = qi.workload(4)
    a = wl.ansatz
    big = qi.System((20.0, 18.0, 14.0), ((0.0, 0.0, 0.0), (3.1, 0.4, -0.6), (-1.2, 2.9, 1.5)), 26, 26)
    mols = [wl.systems[12], big]
    assert [(m.n_up, m.n_down) for m in mols] == [(17, 17), (26, 26)]
    nw = [2, 2]  # (one walker would give E_L - mean = 0: a zero loss gradient)
    params = [qi.make_params(m, a, qi.seed(4, 90 + k)) for k, m in enumerate(mols)]
    pos = [qi.make_walkers(m, n, qi.seed(4, 95 + k)) for k, (m, n) in enumerate(zip(mols, nw))]
    q = _q()
    plan = q.Plan(mols, nw, a, "fp32", concurrent=True)
    P, R = dev(_cat(params), plan.param_dtype), dev(_cat(pos))
    out = plan.local_energy(P, R)
    g, _ = plan.loss_grad(P, R, out["e_loc"])
    torch.cuda.synchronize()
    e = host(out["e_loc"])
    G = host(g).astype(np.float64)
    w0 = p0 = 0
    for s, p, r, n in zip(mols, params, pos, nw):
        pr = p.astype(np.float32).astype(np.float64)
        ref = oracle.local_energy(r, pr, s, a)
        scale = np.maximum.reduce([np.abs(ref["e_loc"]), 0.5 * np.abs(ref["lap"]),
                                   0.5 * (ref["grad"] ** 2).sum((1, 2)), np.ones(n)])
        err = np.abs(e[w0:w0 + n] - ref["e_loc"]) / scale
        Gref, _, _ = oracle.loss_grad(r, e[w0:w0 + n], pr, s, a)
        gerr = np.linalg.norm(G[p0:p0 + len(p)] - Gref) / np.linalg.norm(Gref)
        alpha = amplification(r, p, s, a)
        print(f"[large spin {s.n_up}/{s.n_down} fp32] E_L/scale {err.max():.3e} (alpha {alpha.max():.3g}), "
              f"loss gradient {gerr:.3e}", flush=True)
        assert np.all(err <= fp32_eloc_bound(alpha)) and gerr < fp32_grad_bound(alpha)
        w0 += n
        p0 += len(p)
