"""Mixed precision on the cyclobutadiene-sized system (4 C + 4 H, 14 up + 14
down electrons, width 256, 32 determinants): embedding GEMMs with bf16
operands and float32 accumulation (everywhere, or only in the value-row
forwards: bf16v), determinants and the energy combination in float64.  E_L is compared with the FP64 oracle on a walker subset and the
error is reported in mHa, beside the float32 plan on the same walkers."""
import numpy as np
import pytest
import torch

import oracle
import qmc_inputs as qi
from tests.gpu_common import dev, host, report
from tests.test_gpu_parity import flagged

pytestmark = pytest.mark.gpu


def _run(s, a, p, r, precision):
    from paper_2307_14123_amd import qmc
    plan = qmc.Plan([s], [r.shape[0]], a, precision)
    out = plan.local_energy(dev(p, plan.param_dtype), dev(r))
    torch.cuda.synchronize()
    return {k: host(v) for k, v in out.items()}


@pytest.fixture(scope="module")
def c4h4_case():
    wl = qi.workload(3)
    s, a = wl.systems[0], wl.ansatz
    p = qi.make_params(s, a, qi.seed(3, 0))
    r = qi.make_walkers(s, wl.walkers, qi.seed(3, 1))[:6]
    p32 = p.astype(np.float32).astype(np.float64)
    ref = oracle.local_energy(r, p32, s, a, chunk=3)
    ok = ~flagged(r, p32, s, a)
    scale = np.maximum.reduce([np.abs(ref["e_loc"]), 0.5 * np.abs(ref["lap"]),
                               0.5 * (ref["grad"] ** 2).sum((1, 2)), np.ones_like(ref["e_loc"])])
    return s, a, p, r, ref, ok, scale


@pytest.mark.parametrize("precision,rel_bound", [("fp32", 2e-5), ("bf16", 5e-2), ("bf16v", 2e-5)])
def test_c4h4_precision_vs_oracle(c4h4_case, precision, rel_bound):
    s, a, p, r, ref, ok, scale = c4h4_case
    got = _run(s, a, p, r, precision)
    err = (got["e_loc"] - ref["e_loc"]) * 1e3
    report(f"c4h4 {precision} {len(r)} walkers", err[ok])
    rel = np.abs(err[ok]) * 1e-3 / scale[ok]
    print(f"[c4h4 {precision}] max error relative to the largest E_L addend {rel.max():.2e}; "
          f"log|psi| max abs err {np.abs(got['logpsi'] - ref['logpsi'])[ok].max():.2e}", flush=True)
    assert np.all(got["sign"][ok] == ref["sign"][ok])
    assert rel.max() < rel_bound


def test_c4h4_bf16_value_rows_logpsi(c4h4_case):
    """bf16v: the value-row forward (log|psi| for Metropolis and the loss gradient) takes bf16
    operands, so its log|psi| carries bf16 rounding (bounded like the bf16 plan's), while the local
    energy above keeps the float32 bound; the loss gradient stays within 5e-2 normwise."""
    from paper_2307_14123_amd import qmc
    s, a, p, r, ref, ok, scale = c4h4_case
    plan = qmc.Plan([s], [r.shape[0]], a, "bf16v")
    P, R = dev(p, plan.param_dtype), dev(r)
    lp, sg = plan.logpsi(P, R)
    g, _ = plan.loss_grad(P, R, dev(ref["e_loc"]))
    torch.cuda.synchronize()
    err = np.abs(host(lp) - ref["logpsi"])[ok]
    p32 = p.astype(np.float32).astype(np.float64)
    Gref = oracle.loss_grad(r, ref["e_loc"], p32, s, a)[0]
    gerr = np.linalg.norm(host(g).astype(np.float64) - Gref) / np.linalg.norm(Gref)
    print(f"[c4h4 bf16v] value-row log|psi| max abs err {err.max():.2e}; loss gradient normwise {gerr:.2e}",
          flush=True)
    assert np.all(host(sg)[ok] == ref["sign"][ok])
    assert err.max() < 5e-2 * max(1.0, np.abs(ref["logpsi"]).max()) and gerr < 5e-2


def test_c4h4_fp32_three_piece_gemms(c4h4_case):
    """The float32 plan with autotuned tiles: at width 256 the tuner may choose the three-piece bf16
    form of the float32 GEMMs (operands split into three bf16 pieces, six products accumulated in
    float32 on the bf16 matrix cores).  When it does, the local energies keep the float32 bound against
    the oracle (2e-5 of the largest addend, as the plain float32 plan above) and the loss gradient the
    amplification-scaled float32 bound."""
    from paper_2307_14123_amd import qmc
    from tests.test_gpu_parity import amplification, fp32_grad_bound
    s, a, p, r, ref, ok, scale = c4h4_case
    plan = qmc.Plan([s], [r.shape[0]], a, "fp32", autotune=True)
    tiles = plan.tiles()[0]
    print(f"[c4h4 fp32 autotuned] tiles {tiles} (bit 3 = three-piece bf16 form)", flush=True)
    if not any(t > 0 and ((t - 1) & 8) for t in tiles):
        pytest.skip(f"the tuner kept the float32 MFMA form for every GEMM class on this device: {tiles}")
    P, R = dev(p, plan.param_dtype), dev(r)
    out = plan.local_energy(P, R)
    g, _ = plan.loss_grad(P, R, dev(ref["e_loc"]))
    torch.cuda.synchronize()
    e = host(out["e_loc"])
    rel = np.abs(e - ref["e_loc"])[ok] / scale[ok]
    p32 = p.astype(np.float32).astype(np.float64)
    Gref = oracle.loss_grad(r, ref["e_loc"], p32, s, a)[0]
    gerr = np.linalg.norm(host(g).astype(np.float64) - Gref) / np.linalg.norm(Gref)
    alpha = amplification(r, p, s, a)
    print(f"[c4h4 fp32 autotuned] E_L max error relative to the largest addend {rel.max():.2e}; "
          f"loss gradient normwise {gerr:.2e} (bound {fp32_grad_bound(alpha):.2e})", flush=True)
    assert np.all(host(out["sign"])[ok] == ref["sign"][ok])
    assert rel.max() < 2e-5
    assert gerr < fp32_grad_bound(alpha)
