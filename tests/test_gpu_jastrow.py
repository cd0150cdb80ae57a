"""Learnable Jastrow factor exp(J), J = eta(sum_i f_i) (Sec. III.D), on the GPU against the FP64
oracle, with the electron-electron cusp factor on as well: local energies, gradients and Laplacians
(FP64 to 1e-10 of the largest addend, FP32 to 2e-5), value-mode log|psi|, and the loss gradient
including the Jastrow parameters (FP64 to 1e-10 normwise; FP32 to 2e-3)."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
import qmc_inputs as qi
from tests.gpu_common import dev, host, rel_err
from tests.test_gpu_parity import (_compare_fp64, _run_le, amplification, check_fp32_logpsi, fp32_eloc_bound,
                                    fp32_grad_bound)

pytestmark = pytest.mark.gpu


def _q():
    from paper_2307_14123_amd import qmc
    return qmc


def _normwise(g, ref):
    return float(np.linalg.norm(g - ref) / max(np.linalg.norm(ref), 1e-300))


def _n2(W, **kw):
    s, a, p, r = qi.workload_inputs(1, W)
    a = dataclasses.replace(a, jastrow=1, **kw)
    return s, a, qi.make_params(s, a, qi.seed(1, 0)), r


def test_h2_fp64_jastrow():
    s, a, p, r = qi.workload_inputs(0)
    a = dataclasses.replace(a, jastrow=1, ee_cusp=1.0)
    _compare_fp64("h2 jastrow fp64 256", s, a, qi.make_params(s, a, qi.seed(0, 0)), r)


def test_n2_subset_fp64_jastrow():
    s, a, p, r = _n2(24, ee_cusp=0.5)
    _compare_fp64("n2 jastrow fp64 24", s, a, p, r)


def test_ragged_molecule_fp64_jastrow():
    s = qi.System((3.0, 1.0, 2.0), ((0.0, 0.0, 0.0), (1.6, 0.2, -0.3), (-0.5, 1.4, 0.9)), 4, 2)
    a = qi.Ansatz(n_rbf=8, rbf_dmax=7.0, init_layers=2, width=40, mp_layers=2, n_det=3, n_env=3, jastrow=1)
    p = qi.make_params(s, a, 41)
    r = qi.make_walkers(s, 37, 42)
    _compare_fp64("ragged jastrow fp64 37", s, a, p, r)


def test_n2_subset_fp32_jastrow():
    s, a, p, r = _n2(24, ee_cusp=0.5)
    ref = oracle.local_energy(r, p, s, a)
    got = _run_le(s, a, p, r, "fp32")
    scale = np.maximum.reduce([np.abs(ref["e_loc"]), 0.5 * np.abs(ref["lap"]),
                               0.5 * (ref["grad"] ** 2).sum((1, 2)), np.ones_like(ref["e_loc"])])
    e = np.abs(got["e_loc"] - ref["e_loc"]) / scale
    print(f"[n2 jastrow fp32] max rel E_L err {e.max():.3e}", flush=True)
    alpha = amplification(r, p, s, a)
    assert np.all(e <= fp32_eloc_bound(alpha))
    check_fp32_logpsi("n2 jastrow fp32", got["logpsi"], ref["logpsi"], alpha)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 2e-3)])
def test_loss_grad_with_jastrow(prec, tol):
    s, a, p, r = _n2(16, ee_cusp=0.5)
    q = _q()
    plan = q.Plan([s], [16], a, prec)
    P, R = dev(p, plan.param_dtype), dev(r)
    out = plan.local_energy(P, R)
    lp, _ = plan.logpsi(P, R)
    g, em = plan.loss_grad(P, R, out["e_loc"])
    torch.cuda.synchronize()
    # float32: the value forward and the jet forward agree to the float32 value-mode bar, scaled by
    # each walker's amplification alpha; the loss gradient to 2e-3 scaled by the largest one
    alpha = amplification(r, p, s, a)
    if prec == "fp32":
        check_fp32_logpsi("jastrow fp32 value vs jet", host(lp), host(out["logpsi"]), alpha)
        tol = fp32_grad_bound(alpha)
    else:
        assert rel_err(host(lp), host(out["logpsi"])).max() < 1e-12
    Gref, em_ref, nf = oracle.loss_grad(r, host(out["e_loc"]), p, s, a)
    G = host(g).astype(np.float64)
    err = _normwise(G, Gref)
    jerr = _normwise(G[-(a.width * a.width + 2 * a.width + 1):], Gref[-(a.width * a.width + 2 * a.width + 1):])
    print(f"[loss grad jastrow {prec}] normwise rel err {err:.3e}, Jastrow block {jerr:.3e}", flush=True)
    assert err < tol and jerr < tol
