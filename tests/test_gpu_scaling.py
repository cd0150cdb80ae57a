"""The largest systems of the system-size sweep (Sec. VI, scaling) against the FP64 oracle: a 45-electron
atom (23 up, 22 down: one nucleus, the largest spin blocks) and a 44-atom hydrogen chain (the most
nuclei), the N2-sized ansatz at random init, on two walkers each.  FP64 plans to 1e-9 relative, FP32
plans to 1e-4 relative (local energies are O(10^3) Ha here at random init)."""
import functools

import numpy as np
import pytest
import torch

import oracle
import qmc_inputs as qi
from tests.gpu_common import dev, host, rel_err

pytestmark = pytest.mark.gpu

SYSTEMS = {"atom45": lambda: qi.atom(45), "chain44": lambda: qi.hydrogen_chain(44)}


@functools.lru_cache(maxsize=None)
def _case(name):
    s = SYSTEMS[name]()
    a = qi.SCALING_ANSATZ
    p = qi.make_params(s, a, 9000 + s.n_nuc)
    r = qi.make_walkers(s, 2, 9100 + s.n_nuc)
    ref = oracle.local_energy(r, p, s, a, chunk=2)
    return s, a, p, r, ref


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("fp32", 1e-4)])
@pytest.mark.parametrize("name", sorted(SYSTEMS))
def test_sweep_extremes_local_energy(name, prec, tol):
    from paper_2307_14123_amd import qmc
    s, a, p, r, ref = _case(name)
    print(f"[scaling parity] {name} {prec}", flush=True)
    plan = qmc.Plan([s], [2], a, prec)
    P = dev(p, torch.float64 if prec == "fp64" else torch.float32)
    out = plan.local_energy(P, dev(r))
    torch.cuda.synchronize()
    e = host(out["e_loc"])
    lp = host(out["logpsi"])
    assert np.all(np.isfinite(e))
    assert rel_err(lp, ref["logpsi"]).max() < tol
    assert rel_err(e, ref["e_loc"]).max() < tol, (e, ref["e_loc"])
