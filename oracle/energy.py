"""Potential and local energy (oracle side, torch float64 on the CPU).

* V follows the molecular Hamiltonian (Sec. II.A): electron-nucleus attraction
  and electron-electron repulsion.  The printed Hamiltonian omits the
  nucleus-nucleus repulsion; it is added as a constant when include_vnn is set,
  which gives total energies.
* E_loc = -1/2 sum_i (Delta_i log|psi| + |grad_i log|psi||^2) + V, the
  log-domain form of the local energy (Sec. IV.B).
* The derivatives follow the paper's own route (Appendix A.2): the gradient
  from one reverse pass, then the diagonal of the Hessian one coordinate at a
  time (serial over the 3N coordinates), each entry by differentiating one
  gradient component again.
"""
from __future__ import annotations

import numpy as np
import torch

from .ansatz import logpsi


def nuclear_repulsion(system) -> float:
    Z = np.asarray(system.charges, dtype=np.float64)
    R = np.asarray(system.coords, dtype=np.float64).reshape(-1, 3)
    v = 0.0
    for I in range(len(Z)):
        for J in range(I):
            v += Z[I] * Z[J] / np.linalg.norm(R[I] - R[J])
    return float(v)


def potential(r, system, include_vnn=1, include_vee=True):
    """V(r) for r [W, N, 3] (numpy or torch float64) -> same kind, shape [W]."""
    as_np = isinstance(r, np.ndarray)
    rt = torch.as_tensor(r, dtype=torch.float64)
    Z = torch.as_tensor(np.asarray(system.charges, dtype=np.float64))
    R = torch.as_tensor(np.asarray(system.coords, dtype=np.float64).reshape(-1, 3))
    N = rt.shape[1]
    v = torch.zeros(rt.shape[0], dtype=torch.float64)
    for i in range(N):
        for I in range(len(Z)):
            v = v - Z[I] / torch.linalg.norm(rt[:, i] - R[I], dim=-1)
        if include_vee:
            for j in range(i):
                v = v + 1.0 / torch.linalg.norm(rt[:, i] - rt[:, j], dim=-1)
    if include_vnn:
        v = v + nuclear_repulsion(system)
    return v.numpy() if as_np else v


def grad_lap_serial(fn, r):
    """Gradient and Laplacian of the scalar-per-walker fn at r [B, N, 3].

    One reverse pass for the gradient; then, serially for each of the 3N
    coordinates c, d(grad_c)/d r_c by a further reverse pass."""
    r = r.detach().clone().requires_grad_(True)
    out = fn(r)
    val = out[1] if isinstance(out, tuple) else out
    g = torch.autograd.grad(val.sum(), r, create_graph=True)[0]
    B, N, _ = r.shape
    gflat = g.reshape(B, 3 * N)
    lap = torch.zeros(B, dtype=torch.float64)
    for c in range(3 * N):
        hc = torch.autograd.grad(gflat[:, c].sum(), r, retain_graph=True, allow_unused=True)[0]
        if hc is not None:
            lap = lap + hc.reshape(B, 3 * N)[:, c]
    return out, g.detach(), lap.detach()


def local_energy(r, params, system, ans, chunk=32, threads=None):
    """Per-walker sign, log|psi|, grad log|psi| [W,N,3], Laplacian, V and E_loc.

    r: numpy [W, N, 3]; params: numpy flat blob.  Returns a dict of numpy arrays."""
    if threads is not None:
        torch.set_num_threads(int(threads))
    r = np.asarray(r, dtype=np.float64)
    theta = torch.as_tensor(np.asarray(params, dtype=np.float64))
    W = r.shape[0]
    res = {k: [] for k in ("sign", "logpsi", "grad", "lap", "v", "e_loc")}
    for s in range(0, W, chunk):
        rc = torch.as_tensor(r[s:s + chunk])
        (sg, lp), g, lap = grad_lap_serial(lambda x: logpsi(x, theta, system, ans), rc)
        v = potential(rc, system, ans.include_vnn)
        e = -0.5 * (lap + (g ** 2).sum((1, 2))) + v
        res["sign"].append(sg.detach().numpy())
        res["logpsi"].append(lp.detach().numpy())
        res["grad"].append(g.numpy())
        res["lap"].append(lap.numpy())
        res["v"].append(v.numpy())
        res["e_loc"].append(e.detach().numpy())
    return {k: np.concatenate(v) for k, v in res.items()}
