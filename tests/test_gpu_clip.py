"""Clipped local energies (Sec. IV.D) on the GPU against the oracle: per system of a two-system
plan (ragged, odd and even walker counts, heavy tails, ties, NaN and inf), hard and soft shapes,
in place, a 100,000-walker system, and the loss gradient from clipped energies (FP64 to 1e-10)."""
import numpy as np
import pytest
import torch

import oracle
import qmc_inputs as qi
from tests.gpu_common import dev, host

pytestmark = pytest.mark.gpu


def _q():
    from paper_2307_14123_amd import qmc
    return qmc


def _energies(n, seed, ties=False):
    rng = np.random.default_rng(seed)
    e = rng.standard_cauchy(n) * 0.5 - 1.2
    if ties:
        e = np.round(e, 1)
    e[rng.choice(n, max(1, n // 20), replace=False)] = np.nan
    e[rng.choice(n, 2, replace=False)] = np.inf
    return e


def _check(got, ref, e):
    fin = np.isfinite(ref)
    assert np.array_equal(np.isnan(got), np.isnan(ref)) and np.array_equal(got[~fin & ~np.isnan(ref)],
                                                                            ref[~fin & ~np.isnan(ref)])
    np.testing.assert_allclose(got[fin], ref[fin], rtol=1e-13, atol=1e-13)
    same = fin & (ref == e)
    assert np.sum(got[same] != e[same]) <= 2  # a value within rounding of the window edge may flip


@pytest.mark.parametrize("mode", ["hard", "soft"])
@pytest.mark.parametrize("counts,ties", [((37, 64), False), ((64, 37), True), ((1, 2), False)])
def test_clip_two_systems(mode, counts, ties):
    s1, a, _, _ = qi.workload_inputs(0, 4)
    s2 = qi.System((3.0, 1.0), ((0.0, 0.0, 0.0), (1.6, 0.2, -0.3)), 2, 2)
    plan = _q().Plan([s1, s2], list(counts), a, "fp64")
    if counts == (1, 2):
        e1, e2 = np.array([3.5]), np.array([np.nan, -2.0])
    else:
        e1, e2 = _energies(counts[0], 5 + counts[0], ties), _energies(counts[1], 7 + counts[1], ties)
    E = dev(np.concatenate([e1, e2]))
    for width in (0.5, 5.0):
        got = host(plan.clip_local_energy(E, width, mode))
        torch.cuda.synchronize()
        _check(got[:counts[0]], oracle.clip_local_energy(e1, width, mode), e1)
        _check(got[counts[0]:], oracle.clip_local_energy(e2, width, mode), e2)
    E2 = E.clone()
    plan.clip_local_energy(E2, 2.0, mode, out=E2)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host(E2), host(plan.clip_local_energy(E, 2.0, mode)))


def test_clip_many_walkers():
    s, a, _, _ = qi.workload_inputs(0, 4)
    n = 100_000
    plan = _q().Plan([s], [n], a, "fp64")
    e = _energies(n, 3)
    got = host(plan.clip_local_energy(dev(e), 5.0, "hard"))
    torch.cuda.synchronize()
    _check(got, oracle.clip_local_energy(e, 5.0, "hard"), e)


def test_loss_grad_from_clipped_energies():
    s, a, p, r = qi.workload_inputs(2, 16)
    q = _q()
    plan = q.Plan([s], [16], a, "fp64")
    P, R = dev(p), dev(r)
    e = plan.local_energy(P, R)["e_loc"]
    ec = plan.clip_local_energy(e, 1.0, "hard")
    g, em = plan.loss_grad(P, R, ec)
    torch.cuda.synchronize()
    ec_ref = oracle.clip_local_energy(host(e), 1.0, "hard")
    np.testing.assert_allclose(host(ec), ec_ref, rtol=1e-13, atol=1e-13)
    Gref, em_ref, _ = oracle.loss_grad(r, ec_ref, p, s, a)
    err = np.linalg.norm(host(g) - Gref) / np.linalg.norm(Gref)
    print(f"[clipped loss grad fp64] normwise rel err {err:.3e}", flush=True)
    assert err < 1e-10 and abs(host(em)[0] - em_ref) < 1e-12 * abs(em_ref)
