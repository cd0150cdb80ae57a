"""Independent numpy float64 forward of log|psi| (no autograd).

Written separately from the torch forward, electron by electron and pair by
pair, so that the two cross-check each other; it also backs the
finite-difference tests of the gradient and Laplacian.  Same passages as the
torch forward: radial basis and node initialisation (Sec. III.A), graph
convolution with mean normalisation and concatenation update (Sec. III.A),
orbitals times isotropic envelopes (Sec. III.B), spin-factorised determinants
(Sec. III.C), log-sum-exp over determinants (Sec. III.E), optional fixed
electron-electron cusp factor and learnable Jastrow factor (Sec. III.D).
"""
from __future__ import annotations

import numpy as np

from .layout import unpack


def _rho(d, K, dmax):
    s = dmax / (K - 1)
    return np.stack([np.exp(-((d - k * s) / s) ** 2) for k in range(K)], axis=-1)


def _norm(v):
    return np.sqrt(v[..., 0] ** 2 + v[..., 1] ** 2 + v[..., 2] ** 2)


def logpsi_np(r, params, system, ans):
    """(sign, log|psi|) for r [W, N, 3] (numpy float64)."""
    r = np.asarray(r, dtype=np.float64)
    P = {k: np.asarray(v) for k, v in unpack(np.asarray(params, dtype=np.float64), system, ans).items()}
    W, N, _ = r.shape
    Z = np.asarray(system.charges, dtype=np.float64)
    R = np.asarray(system.coords, dtype=np.float64).reshape(-1, 3)
    M = len(Z)
    K, dmax, D = ans.n_rbf, ans.rbf_dmax, ans.width
    spin = [0] * system.n_up + [1] * system.n_down

    den = [[_norm(r[:, i] - R[I]) for I in range(M)] for i in range(N)]
    dee = [[(_norm(r[:, i] - r[:, j]) if i != j else None) for j in range(N)] for i in range(N)]

    feats = []
    for i in range(N):
        parts = [_rho(den[i][I], K, dmax) for I in range(M)]
        same = [j for j in range(N) if j != i and spin[j] == spin[i]]
        opp = [j for j in range(N) if spin[j] != spin[i]]
        for group in (same, opp):
            if group:
                parts.append(sum(_rho(dee[i][j], K, dmax) for j in group) / len(group))
            else:
                parts.append(np.zeros((W, K)))
        feats.append(np.concatenate(parts, axis=-1))
    f = [np.tanh(x @ P["init.W1"] + P["init.b1"]) for x in feats]
    for l in range(2, ans.init_layers + 1):
        f = [np.tanh(fi @ P[f"init.W{l}"] + P[f"init.b{l}"]) for fi in f]

    def filt(l, t, d):
        x = _rho(d, K, dmax)
        if getattr(ans, "edge_update", 0):
            for lu in range(1, l + 1):  # the edge features' updates up to layer l
                x = np.tanh(x @ P[f"mp{lu}.{t}.Ve"] + P[f"mp{lu}.{t}.ce"])
        hid = np.tanh(x @ P[f"mp{l}.{t}.U1"] + P[f"mp{l}.{t}.a1"])
        return hid @ P[f"mp{l}.{t}.U2"] + P[f"mp{l}.{t}.a2"]

    for l in range(ans.mp_layers):
        h = [fj @ P[f"mp{l}.Wh"] + P[f"mp{l}.bh"] for fj in f]
        new_f = []
        for i in range(N):
            same = [j for j in range(N) if j != i and spin[j] == spin[i]]
            opp = [j for j in range(N) if spin[j] != spin[i]]
            ms = np.zeros((W, D))
            for j in same:
                ms += filt(l, "same", dee[i][j]) * h[j]
            if same:
                ms /= len(same)
            mo = np.zeros((W, D))
            for j in opp:
                mo += filt(l, "opp", dee[i][j]) * h[j]
            if opp:
                mo /= len(opp)
            mn = np.zeros((W, D))
            for I in range(M):
                mn += filt(l, "nuc", den[i][I]) * P[f"mp{l}.Y"][I]
            mn /= M
            m = np.concatenate([ms, mo, mn], axis=-1)
            new_f.append(f[i] + np.tanh(m @ P[f"mp{l}.Wg"] + P[f"mp{l}.bg"]))
        f = new_f

    ndet = ans.n_det
    logdet = np.zeros((W, ndet))
    sign = np.ones((W, ndet))
    blocks = (("up", list(range(system.n_up))), ("down", list(range(system.n_up, N))))
    full = bool(getattr(ans, "full_det", 0))
    Afull = np.zeros((W, ndet, N, N)) if full else None
    for s, idx in blocks:
        n = len(idx)
        if n == 0:
            continue
        no = N if full else n                                      # orbitals per determinant
        Wo, bo = P[f"orb.{s}.W"], P[f"orb.{s}.b"]
        pi, sg = P[f"orb.{s}.pi"], P[f"orb.{s}.sigma"]
        A = np.zeros((W, ndet, n, no))
        for a, i in enumerate(idx):
            phi = f[i] @ Wo + bo                                   # [W, ndet*no]
            for p in range(ndet):
                for k in range(no):
                    env = np.zeros(W)
                    for I in range(M):
                        for b in range(ans.n_env):
                            env += pi[p, k, I, b] * np.exp(-sg[p, k, I, b] * den[i][I])
                    A[:, p, a, k] = phi[:, p * no + k] * env
        if full:
            Afull[:, :, idx[0]:idx[0] + n, :] = A                 # rows of this spin block
            continue
        sg_, ld = np.linalg.slogdet(A)
        logdet += ld
        sign *= sg_
    if full:
        sign, logdet = np.linalg.slogdet(Afull)
    c = P["c"]
    mx = np.max(logdet, axis=1)
    mx = np.where(np.isfinite(mx), mx, 0.0)
    S = np.sum(c[None, :] * sign * np.exp(logdet - mx[:, None]), axis=1)
    alpha = float(getattr(ans, "ee_cusp", 0.0))
    gamma = np.zeros(W)
    if getattr(ans, "jastrow", 0):
        # learnable Jastrow exponent eta(sum_i f_i) (Sec. III.D)
        fsum = sum(f)
        gamma += (np.tanh(fsum @ P["jas.W1"] + P["jas.b1"]) @ P["jas.W2"])[:, 0] + P["jas.b2"][0]
    if alpha > 0:
        # fixed electron-electron cusp factor exp(gamma) (Sec. III.D), pair by pair
        for i in range(N):
            for j in range(i + 1, N):
                c_ij = 0.25 if spin[i] == spin[j] else 0.5
                gamma += -c_ij * alpha * alpha / (alpha + dee[i][j])
    with np.errstate(divide="ignore"):
        return np.sign(S), mx + np.log(np.abs(S)) + gamma
