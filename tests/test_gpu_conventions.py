"""The numerical conventions of the boundary on the HIP path, through the C ABI.

* psi = 0 (c = (1, -1) on two identical determinants, Sec. II.C / III.E): sign 0, log|psi| = -inf
  and a NaN local energy and Laplacian, in the value and the jet forwards.
* The loss gradient (Sec. IV.A) leaves walkers with a non-finite local energy out of the mean and
  of the estimator, and reports how many entered it in the workspace header.
* An exactly coincident electron pair (the potential is singular there) gives a NaN local energy.
* Metropolis (Sec. V): the comparison log u < 2 (l' - l) is strict and in float64, so u = 0 accepts
  any finite proposal, and a proposal with log|psi'| = -inf is rejected even at u = 0.
Each case is compared with the oracle, which pins the same conventions on the CPU.
"""
import numpy as np
import pytest
import torch

import oracle
import qmc_inputs as qi
from oracle.layout import unpack
from tests.gpu_common import dev, host, rel_err

pytestmark = pytest.mark.gpu

SYS = qi.System((3.0, 1.0, 2.0), ((0.0, 0.0, 0.0), (1.6, 0.2, -0.3), (-0.5, 1.4, 0.9)), 4, 2)
ANS = qi.Ansatz(n_rbf=8, rbf_dmax=7.0, init_layers=1, width=24, mp_layers=2, n_det=2, n_env=2)


def _q():
    from paper_2307_14123_amd import qmc
    return qmc


def _cancelling_params(seed):
    """Determinant 1 a copy of determinant 0, c = (1, -1): psi = 0 at every position."""
    p = qi.make_params(SYS, ANS, seed)
    P = unpack(p, SYS, ANS)
    for sp, n in (("up", SYS.n_up), ("down", SYS.n_down)):
        P[f"orb.{sp}.W"][:, n:2 * n] = P[f"orb.{sp}.W"][:, 0:n]
        P[f"orb.{sp}.b"][n:2 * n] = P[f"orb.{sp}.b"][0:n]
        P[f"orb.{sp}.pi"][1] = P[f"orb.{sp}.pi"][0]
        P[f"orb.{sp}.sigma"][1] = P[f"orb.{sp}.sigma"][0]
    P["c"][:] = [1.0, -1.0]
    return p


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_zero_psi_sign_logpsi_and_nan_energy(prec):
    p = _cancelling_params(71)
    r = qi.make_walkers(SYS, 19, 72)
    st, lt = oracle.logpsi(torch.as_tensor(r), torch.as_tensor(p), SYS, ANS)
    assert np.all(st.numpy() == 0) and np.all(np.isneginf(lt.numpy()))
    q = _q()
    plan = q.Plan([SYS], [19], ANS, prec)
    P, R = dev(p, plan.param_dtype), dev(r)
    lp, sg = plan.logpsi(P, R)
    out = plan.local_energy(P, R)
    g, em = plan.loss_grad(P, R, out["e_loc"])
    torch.cuda.synchronize()
    for name, s_, l_ in (("value", host(sg), host(lp)), ("jet", host(out["sign"]), host(out["logpsi"]))):
        assert np.all(s_ == 0), name
        assert np.all(np.isneginf(l_)), name
    assert np.all(np.isnan(host(out["e_loc"])))
    assert np.all(np.isnan(host(out["lap"])))
    # no walker enters the loss gradient: mean NaN, zero gradient, count 0
    assert np.isnan(host(em)[0])
    assert np.all(host(g) == 0)
    assert plan.loss_grad_finite_counts() == [0]


def test_loss_grad_excludes_non_finite_walkers():
    """NaN and +-inf local energies are left out of the mean and the estimator: the result equals
    the oracle's estimator over the finite walkers only, and the header counts them."""
    p = qi.make_params(SYS, ANS, 73)
    r = qi.make_walkers(SYS, 23, 74)
    q = _q()
    plan = q.Plan([SYS], [23], ANS, "fp64")
    P, R = dev(p), dev(r)
    e = host(plan.local_energy(P, R)["e_loc"]).copy()
    bad = np.array([1, 4, 5, 17, 22])
    e[bad] = [np.nan, np.inf, -np.inf, np.nan, np.inf]
    g, em = plan.loss_grad(P, R, dev(e))
    torch.cuda.synchronize()
    ok = np.isfinite(e)
    Gref, em_ref, nf = oracle.loss_grad(r[ok], e[ok], p, SYS, ANS)
    assert nf == 23 - len(bad)
    assert plan.loss_grad_finite_counts() == [nf]
    assert abs(host(em)[0] - em_ref) <= 1e-12 * abs(em_ref)
    err = np.linalg.norm(host(g) - Gref) / np.linalg.norm(Gref)
    print(f"[loss grad with {len(bad)} non-finite walkers] normwise rel err {err:.2e}", flush=True)
    assert err < 1e-10


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_coincident_pair_gives_nan_energy(prec):
    """An exactly coincident electron pair (opposite spins in walker 0, same spin in walker 1) gives
    E_L = NaN; the remaining walker is ordinary, and the opposite-spin walker's log|psi| is finite and
    matches the oracle's (which also gives NaN there).  The same-spin walker has psi = 0 in exact
    arithmetic (two equal rows) and is checked on the GPU only: the oracle's autograd through an
    exactly singular matrix raises."""
    s, a, p, r = qi.workload_inputs(1, 3)
    r = r.copy()
    r[0, 8] = r[0, 1]          # up electron 1 and down electron 8
    r[1, 2] = r[1, 1]          # up electrons 1 and 2
    ref = oracle.local_energy(r[[0, 2]], p, s, a)
    assert np.isnan(ref["e_loc"][0]) and np.isfinite(ref["e_loc"][1])
    ref = {k: v[[0, 0, 1]] for k, v in ref.items()}
    q = _q()
    plan = q.Plan([s], [3], a, prec)
    out = plan.local_energy(dev(p, plan.param_dtype), dev(r))
    torch.cuda.synchronize()
    e = host(out["e_loc"])
    assert np.isnan(e[0]) and np.isnan(e[1]) and np.isfinite(e[2])
    from tests.test_gpu_parity import amplification, fp32_logpsi_bound
    tol = 1e-10 if prec == "fp64" else float(fp32_logpsi_bound(amplification(r[[0]], p, s, a))[0])
    assert abs(host(out["logpsi"])[0] - ref["logpsi"][0]) <= tol * max(1.0, abs(ref["logpsi"][0]))


def test_metropolis_u_zero_and_minus_inf_proposal():
    """u = 0 accepts a finite proposal even against a far more likely current state; a proposal with
    log|psi'| = -inf (psi = 0 everywhere) is rejected even at u = 0; a current state with
    log|psi| = +inf rejects everything.  Decisions equal the oracle's."""
    q = _q()
    s, a, p, r = qi.workload_inputs(0, 6)
    plan = q.Plan([s], [6], a, "fp64")
    P, R = dev(p), dev(r)
    lp0 = host(plan.logpsi(P, R)[0])
    noise = qi.make_noise(1, 6, s.n_elec, 2)[0]
    lp_in = lp0.copy()
    lp_in[0] += 1e3            # u = 0 must still accept
    lp_in[1] = np.inf          # -inf < -inf is false: reject
    lp_in[2] += 1e3            # u > 0 rejects against a state e^2000 times more likely
    u = np.array([0.0, 0.0, 0.5, 0.0, 1e-300, 0.3])
    L = dev(lp_in)
    acc = host(plan.metropolis_step(P, R, L, dev(noise), dev(u), 0.2))
    torch.cuda.synchronize()
    _, _, acc_o, _ = oracle.metropolis_step(r, lp_in, noise, u, 0.2, p, s, a)
    assert acc[0] == 1 and acc[1] == 0 and acc[2] == 0 and acc[3] == 1
    np.testing.assert_array_equal(acc, acc_o)
    # psi = 0 at every proposal: log|psi'| = -inf is rejected for every u, state unchanged
    pz = _cancelling_params(75)
    rz = qi.make_walkers(SYS, 5, 76)
    plan_z = q.Plan([SYS], [5], ANS, "fp64")
    Rz = dev(rz)
    Lz = dev(np.zeros(5))
    nz = qi.make_noise(1, 5, SYS.n_elec, 77)[0]
    uz = np.array([0.0, 0.0, 0.1, 0.9, 1e-300])
    accz = host(plan_z.metropolis_step(dev(pz), Rz, Lz, dev(nz), dev(uz), 0.3))
    torch.cuda.synchronize()
    _, _, acc_oz, prop_z = oracle.metropolis_step(rz, np.zeros(5), nz, uz, 0.3, pz, SYS, ANS)
    assert np.all(np.isneginf(prop_z))
    assert np.all(accz == 0) and np.all(acc_oz == 0)
    np.testing.assert_array_equal(host(Rz).reshape(rz.shape), rz)
    np.testing.assert_array_equal(host(Lz), np.zeros(5))
