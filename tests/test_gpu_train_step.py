"""The optimizer step of a training iteration (qmc_sgd_update) after a loss
gradient: params - lr * grad computed in float64 and rounded to the io dtype,
bit for bit against the same expression on the host, for both io dtypes."""
import numpy as np
import pytest
import torch

import qmc_inputs as qi
from tests.gpu_common import dev, host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_sgd_update_after_loss_grad(precision):
    from paper_2307_14123_amd import qmc
    s, a, p, r = qi.workload_inputs(1, 16)
    plan = qmc.Plan([s], [16], a, precision)
    P = dev(p, plan.param_dtype)
    R = dev(r)
    e = plan.local_energy(P, R)["e_loc"]
    g, _ = plan.loss_grad(P, R, e)
    before = host(P).copy()
    gh = host(g).copy()
    lr = 3e-3
    plan.sgd_update(P, g, lr)
    torch.cuda.synchronize()
    want = (before.astype(np.float64) - lr * gh.astype(np.float64)).astype(before.dtype)
    np.testing.assert_array_equal(host(P), want)
    assert np.abs(gh).max() > 0
