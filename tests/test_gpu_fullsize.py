"""Parity at the benchmark sizes and across walker chunks, through the C ABI.

* N2-sized ansatz at its full 4096 walkers, in the plan the benchmark times (float32, autotuned
  tiles: persistent grids and multi-tile edge-filter waves are active at this size) and in float64:
  value-mode log|psi| of every walker against the oracle's numpy forward, and E_L, grad log|psi|
  and the Laplacian of a seeded 48-walker sample of the 4096-walker local energy against the oracle.
* Plans whose walkers are split into chunks (a cap of 7 walkers on 23: three full chunks and a
  ragged one): local energy, log|psi|, the reverse-pass gradient, the loss gradient, a Metropolis and
  a Langevin step against the oracle, and per-walker outputs bit-identical to the unchunked plan.
* The C4H4-sized system at 8192 walkers in float32 (16 chunks of 512): walkers from the first and
  the last chunk against the oracle.

Bounds per walker, with alpha the oracle's amplification of the orbital-matrix rounding into
log|psi| (sum over determinants of |c_p D_p / psi| times the matrices' condition numbers): float32
log|psi| within max(2e-4, 1e-7 alpha), E_L within max(2e-5, 1e-8 alpha) of its largest addend;
float64 within 1e-10, except walkers with alpha above 1e5 (rounding floor 1e-16 alpha), which are
counted and held to 1e-15 alpha.
"""
import numpy as np
import pytest
import torch

import oracle
import qmc_inputs as qi
from tests.gpu_common import dev, host, rel_err, report
from tests.test_gpu_parity import (FP64_ALPHA_FLAG, amplification, cancellation, flagged, fp32_eloc_bound,
                                    fp32_grad_bound, fp32_logpsi_bound)

pytestmark = pytest.mark.gpu


def _q():
    from paper_2307_14123_amd import qmc
    return qmc


def _scale(ref):
    return np.maximum.reduce([np.abs(ref["e_loc"]), 0.5 * np.abs(ref["lap"]),
                              0.5 * (ref["grad"] ** 2).reshape(len(ref["e_loc"]), -1).sum(1),
                              np.ones_like(ref["e_loc"])])


def _print_high_alpha(name, alpha, err, kappa):
    """The count of walkers with alpha >= 2000 and the ten closest to their bound."""
    hi = np.nonzero(alpha >= 2000.0)[0]
    print(f"[{name}] walkers with alpha >= 2000: {len(hi)}", flush=True)
    ratio = err / fp32_logpsi_bound(alpha)
    for w in hi[np.argsort(-ratio[hi])][:10]:
        print(f"[{name}]   walker {w}: alpha {alpha[w]:.3g} (kappa {kappa[w]:.1f}), error {err[w]:.3e}, "
              f"bound {fp32_logpsi_bound(alpha[w]):.3e}", flush=True)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_n2_full_size_parity(prec):
    s, a, p, r = qi.workload_inputs(1)
    W = r.shape[0]
    assert W == 4096
    q = _q()
    print(f"[n2 full {prec}] plan over {W} walkers (autotune={prec == 'fp32'})", flush=True)
    plan = q.Plan([s], [W], a, prec, autotune=(prec == "fp32"))
    P, R = dev(p, plan.param_dtype), dev(r)
    lp, sg = plan.logpsi(P, R)
    out = plan.local_energy(P, R)
    torch.cuda.synchronize()
    print(f"[n2 full {prec}] tiles {plan.tiles()} chunks {plan.chunk_walkers()}", flush=True)
    pr = p.astype(np.float32).astype(np.float64) if prec == "fp32" else p
    ref_s, ref_l = oracle.logpsi_np(r, pr, s, a)
    lp_h, sg_h = host(lp), host(sg)
    err = np.abs(lp_h - ref_l)
    alpha = amplification(r, p, s, a)
    kappa = cancellation(r, p, s, a)
    bad = flagged(r, p, s, a) | (alpha > FP64_ALPHA_FLAG)
    if prec == "fp64":
        rel = err / np.maximum(1.0, np.abs(ref_l))
        print(f"[n2 full fp64] log|psi| max rel err {rel[~bad].max():.3e} over {int((~bad).sum())} walkers; "
              f"flagged {int(bad.sum())} max {rel[bad].max() if bad.any() else 0:.3e}", flush=True)
        assert rel[~bad].max() < 1e-10
        assert np.all(sg_h[~bad] == ref_s[~bad])
        assert np.all(rel[bad] <= 1e-15 * np.maximum(alpha[bad], FP64_ALPHA_FLAG))
    else:
        bound = fp32_logpsi_bound(alpha)
        print(f"[n2 full fp32] log|psi| max err {err.max():.3e}, max err/bound {(err / bound).max():.3f}, "
              f"p50 {np.median(err):.2e}", flush=True)
        _print_high_alpha("n2 full fp32", alpha, err, kappa)
        assert np.all(err <= bound)
        # the sign decides nothing in float32 where the terms cancel to the rounding: check it away from that
        keep = kappa < 1e3
        assert np.all(sg_h[keep] == ref_s[keep])
    # a seeded sample of the full-size local energy against the serial-Laplacian oracle
    idx = np.sort(np.random.default_rng(1999).choice(W, 48, replace=False))
    ref = oracle.local_energy(r[idx], pr, s, a)
    got = {k: host(v) for k, v in out.items()}
    e = np.abs(got["e_loc"][idx] - ref["e_loc"]) / _scale(ref)
    g = got["grad"].reshape(W, -1)[idx]
    gr = ref["grad"].reshape(48, -1)
    gn = np.linalg.norm(g - gr, axis=1) / np.maximum(np.linalg.norm(gr, axis=1), 1.0)
    le = rel_err(got["lap"][idx], ref["lap"], floor=1.0)
    okw = ~bad[idx]
    report(f"n2 full {prec} sample 48", (got["e_loc"][idx] - ref["e_loc"]) * 1e3)
    report(f"n2 full {prec} sample 48 unflagged", ((got["e_loc"][idx] - ref["e_loc"]) * 1e3)[okw])
    # the error on the scale max(|E_L|, 1 Ha) as well as on the largest addend of E_L
    e_own = np.abs(got["e_loc"][idx] - ref["e_loc"]) / np.maximum(np.abs(ref["e_loc"]), 1.0)
    print(f"[n2 full {prec}] sample: E_L/scale {e.max():.3e}, E_L/max(|E_L|,1) over unflagged {e_own[okw].max():.3e}, "
          f"grad {gn.max():.3e}, lap {le.max():.3e}", flush=True)
    al = alpha[idx]
    print(f"[n2 full {prec}] sample: {int((~okw).sum())} flagged walkers (alpha {al[~okw]})", flush=True)
    if prec == "fp64":
        assert e[okw].max() < 1e-10 and gn[okw].max() < 1e-10 and le[okw].max() < 1e-10
        assert np.all(e[~okw] <= 1e-15 * al[~okw]) and np.all(gn[~okw] <= 1e-15 * al[~okw])
    else:
        assert np.all(e <= fp32_eloc_bound(al))
        assert np.all(np.abs(got["logpsi"][idx] - ref["logpsi"]) <= fp32_logpsi_bound(al))


CHUNK_SYS = qi.System((3.0, 1.0, 2.0), ((0.0, 0.0, 0.0), (1.6, 0.2, -0.3), (-0.5, 1.4, 0.9)), 4, 2)
CHUNK_ANS = qi.Ansatz(n_rbf=8, rbf_dmax=7.0, init_layers=2, width=40, mp_layers=2, n_det=3, n_env=3)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_chunked_plan(prec):
    """23 walkers in chunks of at most 7 (7 + 7 + 7 + 2): every operation's chunk loop against the
    oracle, and per-walker outputs bit-identical to the same plan without chunks."""
    s, a = CHUNK_SYS, CHUNK_ANS
    W = 23
    p = qi.make_params(s, a, 81)
    r = qi.make_walkers(s, W, 82)
    q = _q()
    plan = q.Plan([s], [W], a, prec, max_chunk_walkers=7)
    whole = q.Plan([s], [W], a, prec)
    assert plan.chunk_walkers() == [7] and whole.chunk_walkers() == [W]
    P, R = dev(p, plan.param_dtype), dev(r)
    print(f"[chunked {prec}] local energy, log|psi|, reverse-pass gradient", flush=True)
    out = plan.local_energy(P, R)
    out_w = whole.local_energy(P, R)
    lp, sg = plan.logpsi(P, R)
    lpg, grd = plan.logpsi_grad(P, R)
    torch.cuda.synchronize()
    for k in ("logpsi", "sign", "grad", "lap", "e_loc"):
        np.testing.assert_array_equal(host(out[k]), host(out_w[k]), err_msg=k)
    pr = p.astype(np.float32).astype(np.float64) if prec == "fp32" else p
    ref = oracle.local_energy(r, pr, s, a)
    e = np.abs(host(out["e_loc"]) - ref["e_loc"]) / _scale(ref)
    alpha = amplification(r, p, s, a)
    lpo, go = oracle.logpsi_and_grad(r, pr, s, a)
    gn = np.linalg.norm(host(grd).reshape(W, -1) - go.reshape(W, -1), axis=1) / np.maximum(
        np.linalg.norm(go.reshape(W, -1), axis=1), 1.0)
    print(f"[chunked {prec}] E_L/scale {e.max():.3e}, log|psi| value {np.abs(host(lp) - ref['logpsi']).max():.3e}, "
          f"reverse grad {gn.max():.3e}, max alpha {alpha.max():.3g}", flush=True)
    if prec == "fp64":
        assert e.max() < 1e-10
        assert rel_err(host(lp), ref["logpsi"]).max() < 1e-10
        assert rel_err(host(lpg), ref["logpsi"]).max() < 1e-10
        assert gn.max() < 1e-10
    else:
        assert np.all(e <= fp32_eloc_bound(alpha))
        assert np.all(np.abs(host(lp) - ref["logpsi"]) <= fp32_logpsi_bound(alpha))
        assert np.all(gn <= 1e-3 * np.maximum(1.0, alpha / 2000.0))
    assert np.all(host(sg) == ref["sign"])
    # loss gradient accumulated over the four chunks
    print(f"[chunked {prec}] loss gradient", flush=True)
    g, em = plan.loss_grad(P, R, out["e_loc"])
    gw, emw = whole.loss_grad(P, R, out["e_loc"])
    torch.cuda.synchronize()
    assert plan.loss_grad_finite_counts() == [W]
    Gref, em_ref, nf = oracle.loss_grad(r, host(out["e_loc"]), pr, s, a)
    gerr = np.linalg.norm(host(g) - Gref) / np.linalg.norm(Gref)
    werr = np.linalg.norm(host(g) - host(gw)) / np.linalg.norm(host(gw))
    print(f"[chunked {prec}] loss gradient vs oracle {gerr:.3e}, vs unchunked {werr:.3e}", flush=True)
    assert host(em)[0] == host(emw)[0]
    if prec == "fp64":
        assert gerr < 1e-10 and werr < 1e-13
    else:
        assert gerr < fp32_grad_bound(alpha) and werr < 1e-6
    # a Metropolis and a Langevin step across the chunks, replayed by the oracle
    print(f"[chunked {prec}] Metropolis and Langevin steps", flush=True)
    noise = qi.make_noise(2, W, s.n_elec, 83)
    u = qi.make_uniforms(2, W, 84)
    L = lp.clone()
    Rm = R.clone()
    acc = host(plan.metropolis_step(P, Rm, L, dev(noise[0]), dev(u[0]), 0.3))
    Lw = lp.clone()
    Rw = R.clone()
    accw = host(whole.metropolis_step(P, Rw, Lw, dev(noise[0]), dev(u[0]), 0.3))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(acc, accw)
    np.testing.assert_array_equal(host(Rm), host(Rw))
    np.testing.assert_array_equal(host(L), host(Lw))
    r_o, lp_o, acc_o, prop = oracle.metropolis_step(r, host(lp), noise[0], u[0], 0.3, pr, s, a)
    margin = np.abs(np.log(u[0]) - 2 * (prop - host(lp)))
    delta = 2e-9 if prec == "fp64" else 2 * fp32_logpsi_bound(amplification(r + 0.3 * noise[0], p, s, a))
    assert np.all((acc == acc_o) | (margin < delta))
    print(f"[chunked {prec}] Metropolis accepted {int(acc.sum())}/{W}, within-margin flips {int((acc != acc_o).sum())}",
          flush=True)
    G0 = grd.clone()
    Lm = lp.clone()
    Rl = R.clone()
    accm = host(plan.mala_step(P, Rl, Lm, G0, dev(noise[1]), dev(u[1]), 0.1, damp=True))
    G1 = grd.clone()
    Lm1 = lp.clone()
    Rl1 = R.clone()
    accm1 = host(whole.mala_step(P, Rl1, Lm1, G1, dev(noise[1]), dev(u[1]), 0.1, damp=True))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(accm, accm1)
    np.testing.assert_array_equal(host(Rl), host(Rl1))
    np.testing.assert_array_equal(host(G0), host(G1))
    print(f"[chunked {prec}] Langevin accepted {int(accm.sum())}/{W}", flush=True)


def test_c4h4_8192_fp32_first_and_last_chunk():
    s, a, p, r = qi.workload_inputs(3)
    W = r.shape[0]
    assert W == 8192
    q = _q()
    plan = q.Plan([s], [W], a, "fp32")
    wc = plan.chunk_walkers()[0]
    assert W // wc >= 3, "the full-size plan must run several chunks"
    print(f"[c4h4 8192 fp32] chunks of {wc}", flush=True)
    P, R = dev(p, plan.param_dtype), dev(r)
    lp, sg = plan.logpsi(P, R)
    out = plan.local_energy(P, R)
    torch.cuda.synchronize()
    pr = p.astype(np.float32).astype(np.float64)
    # log|psi| (value rows) of 32 walkers at each end, and E_L of 3 walkers at each end
    ends = np.r_[0:32, W - 32:W]
    ref_s, ref_l = oracle.logpsi_np(r[ends], pr, s, a)
    alpha = amplification(r[ends], p, s, a)
    err = np.abs(host(lp)[ends] - ref_l)
    print(f"[c4h4 8192 fp32] value log|psi| max err {err.max():.3e}, max err/bound "
          f"{(err / fp32_logpsi_bound(alpha)).max():.3f}", flush=True)
    _print_high_alpha("c4h4 8192 fp32", alpha, err, cancellation(r[ends], p, s, a))
    assert np.all(err <= fp32_logpsi_bound(alpha))
    few = np.r_[0:3, W - 3:W]
    ref = oracle.local_energy(r[few], pr, s, a)
    got = host(out["e_loc"])[few]
    e = np.abs(got - ref["e_loc"]) / _scale(ref)
    report("c4h4 8192 fp32 first/last chunk", (got - ref["e_loc"]) * 1e3)
    print(f"[c4h4 8192 fp32] E_L/scale {e.max():.3e}", flush=True)
    af = amplification(r[few], p, s, a)
    assert np.all(e <= fp32_eloc_bound(af))
    assert np.all(np.abs(host(out["logpsi"])[few] - ref["logpsi"]) <= fp32_logpsi_bound(af))
