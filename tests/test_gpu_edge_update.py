"""Edge-feature update f_e^l = tanh(f_e^(l-1) Ve^l + ce^l) in every interaction layer after the
first (Sec. III.A, edge update), on the GPU against the FP64 oracle: local energies with gradients
and Laplacians (FP64 to 1e-10 of the largest addend, FP32 to 2e-5), the loss gradient including
the update weights (FP64 to 1e-10 normwise, FP32 to 2e-3), and the position gradient of the
reverse pass (FP64 to 1e-10).  Three and four interaction layers exercise two and three chained
updates; the N2 ansatz (width 128, K 16) runs on a walker subset."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
import qmc_inputs as qi
from oracle.layout import param_shapes
from tests.gpu_common import dev, host, rel_err
from tests.test_gpu_parity import (_compare_fp64, _run_le, amplification, check_fp32_logpsi, fp32_eloc_bound,
                                    fp32_grad_bound)

pytestmark = pytest.mark.gpu

RAGGED = qi.System((3.0, 1.0, 2.0), ((0.0, 0.0, 0.0), (1.6, 0.2, -0.3), (-0.5, 1.4, 0.9)), 4, 2)
RAGGED_ANS = qi.Ansatz(n_rbf=8, rbf_dmax=7.0, init_layers=2, width=40, mp_layers=3, n_det=3, n_env=3,
                       edge_update=1)


def _q():
    from paper_2307_14123_amd import qmc
    return qmc


def _n2(W, **kw):
    s, a, p, r = qi.workload_inputs(1, W)
    a = dataclasses.replace(a, edge_update=1, **kw)
    return s, a, qi.make_params(s, a, qi.seed(1, 0)), r


def _update_slices(s, a):
    """Index ranges of the Ve/ce blocks in the parameter blob."""
    out, off = [], 0
    for name, shp in param_shapes(s, a).items():
        n = int(np.prod(shp))
        if name.endswith(".Ve") or name.endswith(".ce"):
            out.append(slice(off, off + n))
        off += n
    return out


def _normwise(g, ref):
    return float(np.linalg.norm(g - ref) / max(np.linalg.norm(ref), 1e-300))


def test_ragged_molecule_fp64_edge_update():
    p = qi.make_params(RAGGED, RAGGED_ANS, 81)
    _compare_fp64("ragged edge update fp64 37", RAGGED, RAGGED_ANS, p, qi.make_walkers(RAGGED, 37, 82))


def test_n2_subset_fp64_edge_update():
    s, a, p, r = _n2(24)
    _compare_fp64("n2 edge update fp64 24", s, a, p, r)


def test_n2_subset_fp32_edge_update():
    s, a, p, r = _n2(24, jastrow=1, ee_cusp=0.5)
    ref = oracle.local_energy(r, p, s, a)
    got = _run_le(s, a, p, r, "fp32")
    scale = np.maximum.reduce([np.abs(ref["e_loc"]), 0.5 * np.abs(ref["lap"]),
                               0.5 * (ref["grad"] ** 2).sum((1, 2)), np.ones_like(ref["e_loc"])])
    e = np.abs(got["e_loc"] - ref["e_loc"]) / scale
    print(f"[n2 edge update fp32] max rel E_L err {e.max():.3e}", flush=True)
    alpha = amplification(r, p, s, a)
    assert np.all(e <= fp32_eloc_bound(alpha))
    check_fp32_logpsi("n2 edge update fp32", got["logpsi"], ref["logpsi"], alpha)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 2e-3)])
def test_loss_grad_with_edge_update(prec, tol):
    """Every walker, float32 bounds scaled with the amplification alpha: a walker whose determinant
    terms cancel strongly (one of this 16-walker draw sums to 1/1460 of their absolute sum) has a
    float32 log|psi| and gradient that move by 1e-4..1e-3 with any change of rounding order."""
    s, a, p, r = _n2(16)
    alpha = amplification(r, p, s, a)
    q = _q()
    plan = q.Plan([s], [16], a, prec)
    P, R = dev(p, plan.param_dtype), dev(r)
    out = plan.local_energy(P, R)
    lp, _ = plan.logpsi(P, R)
    g, em = plan.loss_grad(P, R, out["e_loc"])
    torch.cuda.synchronize()
    # float32: the value forward and the jet forward round in different orders through the chained
    # updates (the float32 value-mode bar, 2e-4, against each other and the oracle)
    if prec == "fp64":
        assert rel_err(host(lp), host(out["logpsi"])).max() < 1e-12
    else:
        check_fp32_logpsi("edge update fp32 value vs jet", host(lp), host(out["logpsi"]), alpha)
        check_fp32_logpsi("edge update fp32 value vs oracle", host(lp), oracle.logpsi_and_grad(r, p, s, a)[0], alpha)
        tol = fp32_grad_bound(alpha)
    Gref, em_ref, nf = oracle.loss_grad(r, host(out["e_loc"]), p, s, a)
    G = host(g).astype(np.float64)
    sl = _update_slices(s, a)
    assert len(sl) == 2 * 3 * (a.mp_layers - 1)
    uerr = _normwise(np.concatenate([G[x] for x in sl]), np.concatenate([Gref[x] for x in sl]))
    err = _normwise(G, Gref)
    print(f"[loss grad edge update {prec}] normwise rel err {err:.3e}, update blocks {uerr:.3e}", flush=True)
    assert err < tol and uerr < tol


def test_ragged_loss_grad_fp64_edge_update():
    p = qi.make_params(RAGGED, RAGGED_ANS, 83)
    r = qi.make_walkers(RAGGED, 21, 84)
    plan = _q().Plan([RAGGED], [21], RAGGED_ANS, "fp64")
    P, R = dev(p), dev(r)
    out = plan.local_energy(P, R)
    g, em = plan.loss_grad(P, R, out["e_loc"])
    torch.cuda.synchronize()
    Gref, em_ref, nf = oracle.loss_grad(r, host(out["e_loc"]), p, RAGGED, RAGGED_ANS)
    err = _normwise(host(g), Gref)
    print(f"[ragged loss grad edge update fp64] normwise rel err {err:.3e}", flush=True)
    assert err < 1e-10


@pytest.mark.parametrize("which", ["ragged", "n2"])
def test_reverse_position_gradient_edge_update(which):
    if which == "ragged":
        s, a = RAGGED, RAGGED_ANS
        p, r = qi.make_params(s, a, 85), qi.make_walkers(s, 29, 86)
    else:
        s, a, p, r = _n2(12)
    plan = _q().Plan([s], [r.shape[0]], a, "fp64")
    lp, g = plan.logpsi_grad(dev(p), dev(r))
    torch.cuda.synchronize()
    lp0, g0 = oracle.logpsi_and_grad(r, p, s, a)
    W = r.shape[0]
    ge = (np.abs(host(g).reshape(W, -1) - g0.reshape(W, -1)).max(1) /
          np.maximum(np.abs(g0.reshape(W, -1)).max(1), 1.0)).max()
    print(f"[logpsi_grad edge update {which} fp64] log|psi| {rel_err(host(lp), lp0).max():.2e}, "
          f"gradient {ge:.2e}", flush=True)
    assert rel_err(host(lp), lp0).max() < 1e-10 and ge < 1e-10
