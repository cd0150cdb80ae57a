"""log|psi| and sign of the graph-network ansatz, in torch float64 (oracle side).

Differentiable with respect to both the electron positions and the parameter
blob, so that the local energy and the loss gradient can be taken with plain
autograd.  Each step cites the passage of the paper it follows:

* Gaussian radial basis of pairwise distances: one of the edge featurisations
  listed under "Edge features" (Sec. III.A); centres k*dmax/(K-1), width
  dmax/(K-1).
* Electron node initialisation: second case of the electron-initialisation
  equation (Sec. III.A, node features), fed with e-n distance features plus the
  mean same-spin and opposite-spin e-e features, followed by tanh layers.
* Interaction layers: graph convolution m = sum_j w(f_ij) * h(f_j)
  normalised by the edge count (Sec. III.A, message generation), nuclei as
  nodes with one trainable vector per nucleus, combined by concatenation and
  added to a residual (third case of the embedding-update equation).  Edge
  features are reused in every layer (first case of the edge-update equation).
* Orbitals: kappa is one linear map per spin (many-body orbital equation,
  Sec. III.B) times isotropic exponential envelopes (envelope equation with
  alpha = 1 and Sigma = sigma * I).
* Spin-factorised determinants (Sec. III.C) combined with coefficients c_p
  (generalised Slater determinant equation, Sec. II.C) in the log domain via
  slogdet and the log-sum-exp identity (Sec. III.E).
"""
from __future__ import annotations

import numpy as np
import torch

from .layout import unpack


def rbf(d: torch.Tensor, K: int, dmax: float) -> torch.Tensor:
    """Gaussian basis rho_k(d) = exp(-((d - mu_k)/s)^2) on the last axis."""
    mu = torch.arange(K, dtype=d.dtype) * (dmax / (K - 1))
    s = dmax / (K - 1)
    return torch.exp(-(((d[..., None] - mu) / s) ** 2))


def _spin(system):
    N = system.n_up + system.n_down
    spin = torch.tensor([0] * system.n_up + [1] * system.n_down)
    same = spin[:, None] == spin[None, :]
    eye = torch.eye(N, dtype=torch.bool)
    return (same & ~eye).to(torch.float64), (~same).to(torch.float64)


def _mlp_filter(rho, U1, a1, U2, a2):
    """Edge filter w(d) = tanh(rho(d) U1 + a1) U2 + a2."""
    return torch.tanh(rho @ U1 + a1) @ U2 + a2


def embedding(r, P, system, ans):
    """Final electron embeddings f_i [B, N, D] and the e-n distances [B, N, M]."""
    dt = torch.float64
    R = torch.as_tensor(np.asarray(system.coords, dtype=np.float64).reshape(-1, 3), dtype=dt)
    B, N, _ = r.shape
    M = R.shape[0]
    K, dmax = ans.n_rbf, ans.rbf_dmax
    # distances; the diagonal is padded with 1 so that no gradient passes through |0|
    diff_ee = r[:, :, None, :] - r[:, None, :, :]
    d_ee = torch.sqrt((diff_ee ** 2).sum(-1) + torch.eye(N, dtype=dt))
    d_en = torch.sqrt(((r[:, :, None, :] - R[None, None, :, :]) ** 2).sum(-1))
    mask_same, mask_opp = _spin(system)
    n_same = mask_same.sum(1).clamp(min=1.0)          # [N]
    n_opp = mask_opp.sum(1).clamp(min=1.0)
    rho_ee = rbf(d_ee, K, dmax)                        # [B, N, N, K]
    rho_en = rbf(d_en, K, dmax)                        # [B, N, M, K]
    x = torch.cat([
        rho_en.reshape(B, N, M * K),
        (mask_same[None, :, :, None] * rho_ee).sum(2) / n_same[None, :, None],
        (mask_opp[None, :, :, None] * rho_ee).sum(2) / n_opp[None, :, None],
    ], dim=-1)
    f = torch.tanh(x @ P["init.W1"] + P["init.b1"])
    for l in range(2, ans.init_layers + 1):
        f = torch.tanh(f @ P[f"init.W{l}"] + P[f"init.b{l}"])
    # edge features per edge type: the radial basis, or with ans.edge_update its update
    # f_e^l = tanh(f_e^(l-1) Ve^l + ce^l) in every layer after the first (Sec. III.A, edge update)
    fe = {"same": rho_ee, "opp": rho_ee, "nuc": rho_en}
    for l in range(ans.mp_layers):
        w = {}
        for t in ("same", "opp", "nuc"):
            if getattr(ans, "edge_update", 0) and l >= 1:
                fe[t] = torch.tanh(fe[t] @ P[f"mp{l}.{t}.Ve"] + P[f"mp{l}.{t}.ce"])
            w[t] = _mlp_filter(fe[t], P[f"mp{l}.{t}.U1"], P[f"mp{l}.{t}.a1"],
                               P[f"mp{l}.{t}.U2"], P[f"mp{l}.{t}.a2"])
        h = f @ P[f"mp{l}.Wh"] + P[f"mp{l}.bh"]         # [B, N, D] sender features
        m_same = (mask_same[None, :, :, None] * w["same"] * h[:, None, :, :]).sum(2) / n_same[None, :, None]
        m_opp = (mask_opp[None, :, :, None] * w["opp"] * h[:, None, :, :]).sum(2) / n_opp[None, :, None]
        m_nuc = (w["nuc"] * P[f"mp{l}.Y"][None, None, :, :]).sum(2) / M
        m = torch.cat([m_same, m_opp, m_nuc], dim=-1)
        f = f + torch.tanh(m @ P[f"mp{l}.Wg"] + P[f"mp{l}.bg"])
    return f, d_en


def orbital_matrices(r, P, system, ans, emb=None):
    """A^{sigma,p} per spin: list of [B, n_det, n_sigma, n_sigma] tensors (emb: the embedding's
    output when already computed).  With ans.full_det (Sec. III.C, full-determinant equation) every
    spin's orbital map gives N orbitals, the rows of both spins form one N x N matrix per p, and the
    list is [A (B, n_det, N, N), None]."""
    f, d_en = embedding(r, P, system, ans) if emb is None else emb
    B = r.shape[0]
    full = bool(getattr(ans, "full_det", 0))
    N = system.n_up + system.n_down
    out = []
    start = 0
    for s, n in (("up", system.n_up), ("down", system.n_down)):
        if n == 0:
            out.append(None)
            continue
        no = N if full else n                                    # orbitals per determinant
        fs = f[:, start:start + n]                               # [B, n(a), D]
        phi = (fs @ P[f"orb.{s}.W"] + P[f"orb.{s}.b"])           # [B, a, p*no + k]
        phi = phi.reshape(B, n, ans.n_det, no).permute(0, 2, 1, 3)  # [B, p, a, k]
        pi = P[f"orb.{s}.pi"]                                    # [p, k, I, beta]
        sg = P[f"orb.{s}.sigma"]
        d = d_en[:, start:start + n]                             # [B, a, I]
        env = (pi[None, :, None, :, :, :] *
               torch.exp(-sg[None, :, None, :, :, :] * d[:, None, :, None, :, None])).sum((-1, -2))
        out.append(phi * env)                                    # [B, p, a, k]
        start += n
    if full:
        return [torch.cat([A for A in out if A is not None], dim=2), None]
    return out


def combine(logdets, signs, c):
    """psi = sum_p c_p det_p in the log domain: returns (sign psi, log|psi|).

    Log-sum-exp identity (Sec. III.E) with the shift taken over the
    determinant logs, so that c_p enters linearly (c_p = 0 drops a term and
    keeps a finite derivative with respect to c_p)."""
    mx = logdets.max(dim=1, keepdim=True).values.detach()
    mx = torch.where(torch.isfinite(mx), mx, torch.zeros_like(mx))
    S = (c[None, :] * signs * torch.exp(logdets - mx)).sum(1)
    return torch.sign(S), mx[:, 0] + torch.log(torch.abs(S))


def ee_cusp(r, system, alpha):
    """Fixed electron-electron cusp factor exp(gamma) (Sec. III.D, electron-cusp equation).

    Read as gamma = sum_{i<j} -c_ij alpha^2 / (alpha + r_ij), c_ij = 1/4 for same-spin and 1/2 for
    opposite-spin pairs: its slope at r_ij = 0 is c_ij for every alpha (Kato's electron-electron
    cusps), and alpha is the length over which it acts.  As printed, -alpha c / (1 + alpha r) has
    slope alpha^2 c at coalescence, which meets the cusp condition only at alpha = 1; the two forms
    agree there."""
    N = r.shape[1]
    i, j = torch.triu_indices(N, N, 1)
    d = torch.linalg.vector_norm(r[:, i] - r[:, j], dim=-1)                     # [B, pairs]
    same = (i < system.n_up) == (j < system.n_up)
    c = torch.where(same, torch.tensor(0.25, dtype=r.dtype), torch.tensor(0.5, dtype=r.dtype))
    return (-c * alpha * alpha / (alpha + d)).sum(-1)


def jastrow(f, P):
    """Learnable Jastrow exponent (Sec. III.D, learnable-Jastrow equation): J = eta(sum_i f_i) with
    eta read as a two-layer MLP, tanh(x W1 + b1) W2 + b2 (one hidden layer of the embedding width,
    scalar output).  Summing over electrons makes J symmetric under every permutation."""
    x = f.sum(1)                                                     # [B, D]
    return (torch.tanh(x @ P["jas.W1"] + P["jas.b1"]) @ P["jas.W2"] + P["jas.b2"])[:, 0]


def logpsi(r, params, system, ans):
    """(sign, log|psi|) for walkers r [B, N, 3] (torch float64); with ans.ee_cusp = alpha > 0 the
    fixed electron-electron cusp factor (ee_cusp) multiplies psi, and with ans.jastrow = 1 the
    learnable factor exp(J) (jastrow)."""
    P = unpack(params, system, ans)
    emb = embedding(r, P, system, ans)
    mats = orbital_matrices(r, P, system, ans, emb)
    B = r.shape[0]
    logdet = torch.zeros(B, ans.n_det, dtype=torch.float64)
    sign = torch.ones(B, ans.n_det, dtype=torch.float64)
    for A in mats:
        if A is None:          # empty spin block: determinant of a 0x0 matrix is 1
            continue
        s, l = torch.linalg.slogdet(A)
        logdet = logdet + l
        sign = sign * s
    sg, lp = combine(logdet, sign, P["c"])
    alpha = float(getattr(ans, "ee_cusp", 0.0))
    if alpha > 0 and r.shape[1] > 1:
        lp = lp + ee_cusp(r, system, alpha)
    if getattr(ans, "jastrow", 0):
        lp = lp + jastrow(emb[0], P)
    return sg, lp
