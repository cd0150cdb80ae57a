"""FP64 CPU oracle for the VMC local-energy hot path (test infrastructure only).

This package is the independent reference that the HIP path is checked
against.  Only the tests, the smoke check and the CPU-baseline leg of the
benchmark may import it; the product path never does.  It shares no code with
the HIP library: it follows the paper's equations directly, in float64, with
torch CPU autograd for derivatives (the paper's own reverse-then-serial route
for the Laplacian, Appendix A.2) and an independent numpy forward.

Modules
-------
layout     -- unpack the flat parameter blob into named tensors
ansatz     -- log|psi| and sign (torch, differentiable)
npforward  -- log|psi| and sign (numpy only, for finite differences)
energy     -- potential, local energy (serial autograd Laplacian)
sampling   -- one random-walk Metropolis step and one Langevin (MALA) step
clipping   -- clipped local energies for the loss gradient
lossgrad   -- the VMC loss-gradient estimator
slater     -- local energy of a Slater determinant of given analytic orbitals
"""
from .layout import unpack, param_shapes, param_count
from .ansatz import ee_cusp, logpsi
from .clipping import clip_local_energy
from .npforward import logpsi_np
from .energy import potential, local_energy
from .sampling import drift_damping_a, langevin_drift, logpsi_and_grad, mala_log_accept, mala_step, metropolis_step
from .lossgrad import loss_grad, surrogate

__all__ = [
    "unpack", "param_shapes", "param_count", "logpsi", "logpsi_np", "potential",
    "local_energy", "metropolis_step", "mala_step", "mala_log_accept", "langevin_drift", "drift_damping_a",
    "logpsi_and_grad", "loss_grad", "surrogate", "ee_cusp", "clip_local_energy",
]
