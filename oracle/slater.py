"""Local energy of one Slater determinant per spin built from given analytic
orbitals (oracle side), used to pin the determinant-Laplacian machinery.

psi = det[phi_k(r_a)]_up * det[phi_k(r_a)]_down (spin-factorised determinant,
Sec. III.C), E_loc as in Sec. IV.B with the same serial autograd Laplacian as
the full ansatz.  Also provides the hydrogenic orbitals 1s, 2s, 2p of a
nucleus of charge Z at the origin, whose Slater determinants are exact
eigenfunctions of the non-interacting Hamiltonian (the hydrogenic case of
Sec. II.B).
"""
from __future__ import annotations

import torch

from .energy import grad_lap_serial


def hydrogenic(name: str, Z: float):
    """Unnormalised hydrogenic orbital as a function of r [..., 3]."""
    def radius(x):
        return torch.sqrt((x ** 2).sum(-1))
    if name == "1s":
        return lambda x: torch.exp(-Z * radius(x))
    if name == "2s":
        return lambda x: (1.0 - Z * radius(x) / 2.0) * torch.exp(-Z * radius(x) / 2.0)
    axis = {"2px": 0, "2py": 1, "2pz": 2}[name]
    return lambda x: x[..., axis] * torch.exp(-Z * radius(x) / 2.0)


def slater_logpsi(r, orbs_up, orbs_down):
    """(sign, log|psi|) of det[up orbitals] * det[down orbitals] at r [B, N, 3]."""
    nu = len(orbs_up)
    sign = torch.ones(r.shape[0], dtype=torch.float64)
    logabs = torch.zeros(r.shape[0], dtype=torch.float64)
    for orbs, sl in ((orbs_up, slice(0, nu)), (orbs_down, slice(nu, None))):
        if not orbs:
            continue
        x = r[:, sl]
        A = torch.stack([o(x) for o in orbs], dim=-1)     # [B, a(electron), k(orbital)]
        s, l = torch.linalg.slogdet(A)
        sign = sign * s
        logabs = logabs + l
    return sign, logabs


def slater_local_energy(r, orbs_up, orbs_down, Z, include_vee=False):
    """Kinetic + e-n (+ optional e-e) local energy for one nucleus at the origin."""
    r = torch.as_tensor(r, dtype=torch.float64)
    _, g, lap = grad_lap_serial(lambda x: slater_logpsi(x, orbs_up, orbs_down), r)
    v = -Z * (1.0 / torch.sqrt((r ** 2).sum(-1))).sum(-1)
    if include_vee:
        N = r.shape[1]
        for i in range(N):
            for j in range(i):
                v = v + 1.0 / torch.linalg.norm(r[:, i] - r[:, j], dim=-1)
    return (-0.5 * (lap + (g ** 2).sum((1, 2))) + v).numpy(), g.numpy(), lap.numpy()


def slater_jets(r, orbs_up, orbs_down):
    """Orbital-matrix jets for a kernel-level check of the determinant stage.

    Returns, per spin block, A [B, n, n], dA [B, 3N, n, n] (derivative of every
    entry with respect to every coordinate) and lapA [B, n, n] (sum of second
    derivatives over all coordinates), all by autograd in float64."""
    r = torch.as_tensor(r, dtype=torch.float64)
    B, N, _ = r.shape
    nu = len(orbs_up)
    out = []
    for orbs, lo in ((orbs_up, 0), (orbs_down, nu)):
        n = len(orbs)
        if n == 0:
            out.append(None)
            continue
        A = torch.zeros(B, n, n, dtype=torch.float64)
        dA = torch.zeros(B, 3 * N, n, n, dtype=torch.float64)
        lapA = torch.zeros(B, n, n, dtype=torch.float64)
        for a in range(n):
            for k, o in enumerate(orbs):
                x = r.detach().clone().requires_grad_(True)
                val = o(x[:, lo + a])
                g = torch.autograd.grad(val.sum(), x, create_graph=True)[0].reshape(B, 3 * N)
                lap = torch.zeros(B, dtype=torch.float64)
                for c in range(3 * (lo + a), 3 * (lo + a) + 3):
                    lap = lap + torch.autograd.grad(g[:, c].sum(), x, retain_graph=True)[0].reshape(B, 3 * N)[:, c]
                A[:, a, k] = val.detach()
                dA[:, :, a, k] = g.detach()
                lapA[:, a, k] = lap
        out.append((A, dA, lapA))
    return out
