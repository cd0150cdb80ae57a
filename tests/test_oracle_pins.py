"""Pins of the FP64 oracle against closed forms, invariants and finite differences.

Each test fixes the oracle to something other than itself: exact solutions of
hydrogenic problems (Sec. II.B), the Kato cusp behaviour of exponential
envelopes, the antisymmetry and equivariance requirements (Sec. II.A, II.C),
invariances of a distance-only embedding, an independent numpy forward, and
central finite differences of that numpy forward.
"""
import dataclasses
import math
import os

import numpy as np
import pytest
import torch

import oracle
import qmc_inputs as qi
from oracle.layout import unpack
from oracle.slater import hydrogenic, slater_local_energy

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SMALL = qi.Ansatz(n_rbf=6, rbf_dmax=6.0, init_layers=1, width=12, mp_layers=2, n_det=3, n_env=2)


def _closed_form_count(system, ans):
    """Parameter count of the pinned blob, written as one closed formula."""
    M, K, D, L0, L = system.n_nuc, ans.n_rbf, ans.width, ans.init_layers, ans.mp_layers
    per_layer = 3 * (K * D + D + D * D + D) + D * D + D + M * D + 3 * D * D + D
    orb = sum(D * ans.n_det * n + ans.n_det * n + 2 * ans.n_det * n * M * ans.n_env
              for n in (system.n_up, system.n_down) if n > 0)
    return (M + 2) * K * D + D + (L0 - 1) * (D * D + D) + L * per_layer + orb + ans.n_det


def test_param_count_formula():
    expected = {0: 3235, 1: 532848, 2: 532848, 3: 2286752}
    for k, n in expected.items():
        wl = qi.workload(k)
        s = wl.systems[0]
        assert oracle.param_count(s, wl.ansatz) == n
        assert _closed_form_count(s, wl.ansatz) == n
        assert qi.param_count(s, wl.ansatz) == n
    for s in qi.workload(4).systems:
        a = qi.BATCH_ANSATZ
        assert oracle.param_count(s, a) == _closed_form_count(s, a) == qi.param_count(s, a)


def test_batched_molecules_are_neutral_and_spread():
    mols = qi.workload(4).systems
    assert [m.n_elec for m in mols] == qi.BATCH_TARGETS
    for m in mols:
        assert 2 <= m.n_nuc <= 6
        assert sum(m.charges) == m.n_elec
        assert set(m.charges) <= {1.0, 3.0, 6.0, 7.0, 8.0}
        assert m.n_up == (m.n_elec + 1) // 2
        R = m.R()
        for I in range(m.n_nuc):
            for J in range(I):
                assert np.linalg.norm(R[I] - R[J]) >= 1.5 - 1e-12


def _one_center_params(system, ans, sigma, rng=None):
    """Embedding weights arbitrary, orbital map zero, bias 1: psi = prod of envelopes."""
    n = oracle.param_count(system, ans)
    p = rng.standard_normal(n) * 0.3 if rng is not None else np.zeros(n)
    P = unpack(p, system, ans)
    for s, nel in (("up", system.n_up), ("down", system.n_down)):
        if nel == 0:
            continue
        P[f"orb.{s}.W"][:] = 0.0
        P[f"orb.{s}.b"][:] = 1.0
        P[f"orb.{s}.pi"][:] = 0.0
        P[f"orb.{s}.pi"][:, :, 0, 0] = 1.0
        P[f"orb.{s}.sigma"][:] = 1.0
        P[f"orb.{s}.sigma"][:, :, 0, 0] = sigma
    P["c"][:] = 0.0
    P["c"][0] = 1.0
    return p


def _random_points(n, N, seed, scale=1.5):
    return np.random.default_rng(seed).standard_normal((n, N, 3)) * scale


def test_hydrogen_atom_exact():
    """psi = exp(-r) is the hydrogen ground state: E_L = -1/2 for every r."""
    H = qi.System((1.0,), ((0.0, 0.0, 0.0),), 1, 0)
    p = _one_center_params(H, SMALL, 1.0, np.random.default_rng(1))
    r = _random_points(12, 1, 2)
    res = oracle.local_energy(r, p, H, SMALL)
    np.testing.assert_allclose(res["e_loc"], -0.5, rtol=0, atol=1e-12)


@pytest.mark.parametrize("Z,sigma", [(1.0, 0.7), (1.0, 1.6), (2.0, 1.3), (3.0, 3.0)])
def test_kato_cusp_closed_form(Z, sigma):
    """exp(-sigma r) around charge Z: E_L = -sigma^2/2 + (sigma - Z)/r exactly; the
    1/r divergence cancels only at sigma = Z (Kato's electron-nucleus cusp)."""
    sys1 = qi.System((Z,), ((0.3, -0.2, 0.1),), 1, 0)
    p = _one_center_params(sys1, SMALL, sigma, np.random.default_rng(3))
    r = _random_points(10, 1, 4) + np.array([0.3, -0.2, 0.1])
    rad = np.linalg.norm(r[:, 0] - np.array([0.3, -0.2, 0.1]), axis=-1)
    res = oracle.local_energy(r, p, sys1, SMALL)
    exact = -sigma ** 2 / 2 + (sigma - Z) / rad
    np.testing.assert_allclose(res["e_loc"], exact, rtol=1e-12, atol=1e-12)
    # separately: grad log psi = -sigma * unit vector, Laplacian = -2 sigma / r
    np.testing.assert_allclose(res["lap"], -2 * sigma / rad, rtol=1e-12)
    np.testing.assert_allclose((res["grad"] ** 2).sum((1, 2)), sigma ** 2, rtol=1e-12)


@pytest.mark.parametrize("Z", [2.0, 3.0])
def test_helium_like_product_state(Z):
    """1s^2 with exponent Z: E_L = -Z^2 + 1/r12 exactly (electron repulsion on)."""
    He = qi.System((Z,), ((0.0, 0.0, 0.0),), 1, 1)
    p = _one_center_params(He, SMALL, Z, np.random.default_rng(5))
    r = _random_points(10, 2, 6)
    res = oracle.local_energy(r, p, He, SMALL)
    r12 = np.linalg.norm(r[:, 0] - r[:, 1], axis=-1)
    np.testing.assert_allclose(res["e_loc"], -Z ** 2 + 1 / r12, rtol=1e-12)


@pytest.mark.parametrize("Z,alpha", [(2.0, 1.0), (2.0, 0.4), (3.0, 2.5)])
def test_helium_like_product_state_with_ee_cusp(Z, alpha):
    """1s^2 times exp(gamma(r12)), gamma = -alpha^2 / (2 (alpha + r12)): by hand,
    E_L = -Z^2 + 1/r12 - gamma'' - 2 gamma'/r12 - gamma'^2 + Z gamma' (u1 - u2) . e12, with u the unit
    vectors of the electrons and e12 that of r1 - r2."""
    He = qi.System((Z,), ((0.0, 0.0, 0.0),), 1, 1)
    a = dataclasses.replace(SMALL, ee_cusp=alpha)
    p = _one_center_params(He, a, Z, np.random.default_rng(5))
    r = _random_points(10, 2, 6)
    res = oracle.local_energy(r, p, He, a)
    d = r[:, 0] - r[:, 1]
    r12 = np.linalg.norm(d, axis=-1)
    e12 = d / r12[:, None]
    u1 = r[:, 0] / np.linalg.norm(r[:, 0], axis=-1)[:, None]
    u2 = r[:, 1] / np.linalg.norm(r[:, 1], axis=-1)[:, None]
    g1 = 0.5 * alpha ** 2 / (alpha + r12) ** 2
    g2 = -alpha ** 2 / (alpha + r12) ** 3
    exact = -Z ** 2 + 1 / r12 - g2 - 2 * g1 / r12 - g1 ** 2 + Z * g1 * ((u1 - u2) * e12).sum(-1)
    np.testing.assert_allclose(res["e_loc"], exact, rtol=1e-11, atol=1e-11)


def test_ee_cusp_removes_the_coalescence_divergence():
    """Kato: with the cusp factor the local energy of two opposite-spin electrons stays finite as
    they meet (the kinetic -2 gamma'(0) / r12 cancels +1/r12); without it E_L grows as 1/r12.  The
    slopes at coalescence are 1/4 (same spin) and 1/2 (opposite spin) for any alpha."""
    He = qi.System((2.0,), ((0.0, 0.0, 0.0),), 1, 1)
    mid = np.array([0.4, -0.3, 0.5])
    axis = np.array([0.6, 0.0, 0.8])
    for alpha in (0.5, 1.0, 3.0):
        a = dataclasses.replace(SMALL, ee_cusp=alpha)
        p = _one_center_params(He, a, 2.0, np.random.default_rng(8))
        e = []
        for eps in (1e-3, 1e-5, 1e-7):
            r = np.stack([mid + 0.5 * eps * axis, mid - 0.5 * eps * axis])[None]
            e.append(oracle.local_energy(r, p, He, a)["e_loc"][0])
        assert abs(e[2] - e[1]) < 1e-3 and abs(e[1] - e[0]) < 1e-1
        e_plain = oracle.local_energy(r, _one_center_params(He, SMALL, 2.0, np.random.default_rng(8)), He,
                                      SMALL)["e_loc"][0]
        assert e_plain > 1e6
        for n_up, c in ((2, 0.25), (1, 0.5)):
            s2 = qi.System((1.0,), ((0.0, 0.0, 0.0),), n_up, 2 - n_up)
            for eps in (1e-6,):
                x = torch.as_tensor(np.array([[mid, mid + eps * axis]]))
                x0 = torch.as_tensor(np.array([[mid, mid]]))
                slope = (oracle.ee_cusp(x, s2, alpha) - oracle.ee_cusp(x0, s2, alpha)).item() / eps
                assert abs(slope - c) < 1e-5


def test_constant_jastrow_shifts_log_psi_only():
    """With W1 = 0 the Jastrow exponent is the constant tanh(b1) W2 + b2: log|psi| shifts by it and
    the local energy, gradient and Laplacian do not change."""
    s = _small_system()
    p = qi.make_params(s, SMALL_JAS, 31)
    P = unpack(p, s, SMALL_JAS)
    P["jas.W1"][:] = 0.0
    P["jas.b1"][:] = np.linspace(-1, 1, SMALL_JAS.width)
    P["jas.b2"][:] = 0.3
    shift = float(np.tanh(P["jas.b1"]) @ P["jas.W2"][:, 0] + 0.3)
    p0 = p[:oracle.param_count(s, SMALL_CUSP)]
    r = qi.make_walkers(s, 4, 32)
    a = oracle.local_energy(r, p, s, SMALL_JAS)
    b = oracle.local_energy(r, p0, s, SMALL_CUSP)
    np.testing.assert_allclose(a["logpsi"] - b["logpsi"], shift, rtol=0, atol=1e-12)
    np.testing.assert_allclose(a["e_loc"], b["e_loc"], rtol=1e-12, atol=1e-10)
    np.testing.assert_allclose(a["grad"], b["grad"], rtol=1e-12, atol=1e-12)


def _full_from_factorized(pf, s, af, afull):
    """Full-determinant parameters whose N x N matrices are block diagonal with the factorized
    ansatz's spin blocks: the up map fills orbitals 0..n_up-1, the down map orbitals n_up..N-1, every
    other orbital has zero weights, bias and envelope."""
    N = s.n_up + s.n_down
    Pf = unpack(pf, s, af)
    pfull = np.zeros(oracle.param_count(s, afull))
    Pn = unpack(pfull, s, afull)
    for name, v in Pf.items():
        if not name.startswith("orb."):
            Pn[name][...] = v
    Pn["orb.up.sigma"][...] = 1.0
    Pn["orb.down.sigma"][...] = 1.0
    for sp, n, k0 in (("up", s.n_up, 0), ("down", s.n_down, s.n_up)):
        for p in range(af.n_det):
            Pn[f"orb.{sp}.W"][:, p * N + k0:p * N + k0 + n] = Pf[f"orb.{sp}.W"][:, p * n:(p + 1) * n]
            Pn[f"orb.{sp}.b"][p * N + k0:p * N + k0 + n] = Pf[f"orb.{sp}.b"][p * n:(p + 1) * n]
            Pn[f"orb.{sp}.pi"][p, k0:k0 + n] = Pf[f"orb.{sp}.pi"][p]
            Pn[f"orb.{sp}.sigma"][p, k0:k0 + n] = Pf[f"orb.{sp}.sigma"][p]
    return pfull


def test_full_determinant_reduces_to_factorized_for_block_diagonal_matrices():
    """Block-diagonal full matrices give det A = det A_up det A_down (Sec. III.C), so the full-
    determinant ansatz reproduces the spin-factorized one: log|psi|, sign and E_L."""
    s = _small_system()
    pf = qi.make_params(s, SMALL, 51)
    pf[-SMALL.n_det:] = [1.0, -0.7, 0.4]
    pfull = _full_from_factorized(pf, s, SMALL, SMALL_FULL)
    r = qi.make_walkers(s, 5, 52)
    a = oracle.local_energy(r, pf, s, SMALL)
    b = oracle.local_energy(r, pfull, s, SMALL_FULL)
    np.testing.assert_array_equal(a["sign"], b["sign"])
    np.testing.assert_allclose(b["logpsi"], a["logpsi"], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(b["e_loc"], a["e_loc"], rtol=1e-9, atol=1e-9)


def test_full_determinant_generalized_laplace_expansion():
    """det of the full matrix = sum over n_up-subsets S of the orbitals of eps_S det A[up, S]
    det A[down, complement], eps_S the sign of the permutation (S, complement), by brute force."""
    import itertools
    from oracle.ansatz import orbital_matrices
    s = qi.System((3.0, 1.0), ((0.0, 0.0, 0.0), (1.6, 0.2, -0.3)), 2, 2)
    a = dataclasses.replace(SMALL, n_det=1, full_det=1)
    p = qi.make_params(s, a, 53)
    P = unpack(p, s, a)
    P["c"][:] = 1.0
    r = qi.make_walkers(s, 6, 54)
    A = orbital_matrices(torch.as_tensor(r), unpack(torch.as_tensor(p), s, a), s, a)[0][:, 0].numpy()
    N, nu = 4, 2
    det = np.zeros(len(r))
    for S in itertools.combinations(range(N), nu):
        Sb = [k for k in range(N) if k not in S]
        perm = list(S) + Sb
        inv = sum(1 for x in range(N) for y in range(x + 1, N) if perm[x] > perm[y])
        det += (-1) ** inv * np.linalg.det(A[:, :nu][:, :, list(S)]) * np.linalg.det(A[:, nu:][:, :, Sb])
    sg, lp = oracle.logpsi(torch.as_tensor(r), torch.as_tensor(p), s, a)
    np.testing.assert_allclose(np.log(np.abs(det)), lp.numpy(), rtol=1e-12, atol=1e-12)
    np.testing.assert_array_equal(np.sign(det), sg.numpy())


def _golden_hydrogenic():
    rows = []
    with open(os.path.join(GOLDEN, "hydrogenic_energies.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                Z, up, dn, e = line.split()
                rows.append((float(Z), up.split(","), dn.split(","), float(e)))
    return rows


@pytest.mark.parametrize("Z,up,dn,energy", _golden_hydrogenic())
def test_noninteracting_hydrogenic_slater(Z, up, dn, energy):
    """Slater determinants of hydrogenic orbitals: kinetic + e-n energy is the
    constant sum of -Z^2/(2n^2); pins the determinant-Laplacian route."""
    ou = [hydrogenic(o, Z) for o in up]
    od = [hydrogenic(o, Z) for o in dn]
    r = _random_points(6, len(up) + len(dn), 7, scale=1.0 / Z)
    e, _, _ = slater_local_energy(r, ou, od, Z)
    np.testing.assert_allclose(e, energy, rtol=1e-10)


def _golden_potential():
    rows = []
    with open(os.path.join(GOLDEN, "potential_points.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                name, nuc, el, vnn, v = [x.strip() for x in line.split("|")]
                nuc = [list(map(float, x.split())) for x in nuc.split(";")]
                el = [list(map(float, x.split())) for x in el.split(";")]
                rows.append((name, nuc, el, int(vnn), float(v)))
    return rows


@pytest.mark.parametrize("name,nuc,el,vnn,v", _golden_potential())
def test_potential_hand_values(name, nuc, el, vnn, v):
    N = len(el)
    s = qi.System(tuple(n[0] for n in nuc), tuple(tuple(n[1:]) for n in nuc), N, 0)
    got = oracle.potential(np.array([el]), s, vnn)
    assert abs(got[0] - v) < 1e-14 * max(1.0, abs(v))


def test_nuclear_repulsion_constants():
    from oracle.energy import nuclear_repulsion
    assert abs(nuclear_repulsion(qi.H2) - 1 / 1.4) < 1e-15
    assert abs(nuclear_repulsion(qi.N2) - 49 / 2.068) < 1e-13


def _small_system():
    return qi.System((3.0, 1.0, 2.0), ((0.0, 0.0, 0.0), (1.6, 0.2, -0.3), (-0.5, 1.4, 0.9)), 3, 2)


SMALL_CUSP = dataclasses.replace(SMALL, ee_cusp=0.7)
SMALL_JAS = dataclasses.replace(SMALL, ee_cusp=0.7, jastrow=1)
SMALL_FULL = dataclasses.replace(SMALL, full_det=1)
SMALL_EDGE = dataclasses.replace(SMALL, edge_update=1)


def test_torch_and_numpy_forwards_agree():
    s = _small_system()
    for ans in (SMALL_CUSP, SMALL_JAS, SMALL_FULL, SMALL_EDGE):
        p = qi.make_params(s, ans, 13)
        r = qi.make_walkers(s, 5, 14)
        st, lt = oracle.logpsi(torch.as_tensor(r), torch.as_tensor(p), s, ans)
        sn, ln = oracle.logpsi_np(r, p, s, ans)
        np.testing.assert_allclose(lt.numpy(), ln, rtol=1e-12, atol=1e-12)
        assert np.all(st.numpy() == sn)
    for k in (0, 1):
        s, a, p, r = qi.workload_inputs(k, 6)
        st, lt = oracle.logpsi(torch.as_tensor(r), torch.as_tensor(p), s, a)
        sn, ln = oracle.logpsi_np(r, p, s, a)
        np.testing.assert_allclose(lt.numpy(), ln, rtol=1e-12, atol=1e-12)
        assert np.all(st.numpy() == sn)
    s = _small_system()
    p = qi.make_params(s, SMALL, 11)
    r = qi.make_walkers(s, 7, 12)
    st, lt = oracle.logpsi(torch.as_tensor(r), torch.as_tensor(p), s, SMALL)
    sn, ln = oracle.logpsi_np(r, p, s, SMALL)
    np.testing.assert_allclose(lt.numpy(), ln, rtol=1e-12, atol=1e-12)


def test_single_determinant_matches_numpy_slogdet():
    """One determinant per spin with c = 1: log|psi| = sum of numpy slogdets."""
    from oracle.ansatz import orbital_matrices
    s = _small_system()
    a = qi.Ansatz(n_rbf=6, rbf_dmax=6.0, init_layers=1, width=12, mp_layers=1, n_det=1, n_env=2)
    p = qi.make_params(s, a, 13)
    r = qi.make_walkers(s, 5, 14)
    mats = orbital_matrices(torch.as_tensor(r), unpack(torch.as_tensor(p), s, a), s, a)
    ref = sum(np.linalg.slogdet(A.numpy()[:, 0])[1] for A in mats)
    sgn = np.prod([np.linalg.slogdet(A.numpy()[:, 0])[0] for A in mats], axis=0)
    st, lt = oracle.logpsi(torch.as_tensor(r), torch.as_tensor(p), s, a)
    np.testing.assert_allclose(lt.numpy(), ref, rtol=1e-13)
    assert np.all(st.numpy() == sgn)


def test_cancelling_determinants_give_zero_psi():
    """c = (1, -1) on two identical determinants: psi = 0 -> sign 0, log|psi| = -inf."""
    s = _small_system()
    a = qi.Ansatz(n_rbf=6, rbf_dmax=6.0, init_layers=1, width=12, mp_layers=1, n_det=2, n_env=2)
    p = qi.make_params(s, a, 15)
    P = unpack(p, s, a)
    for sp, n in (("up", s.n_up), ("down", s.n_down)):
        Wo = P[f"orb.{sp}.W"]
        Wo[:, n:2 * n] = Wo[:, 0:n]
        P[f"orb.{sp}.b"][n:2 * n] = P[f"orb.{sp}.b"][0:n]
        P[f"orb.{sp}.pi"][1] = P[f"orb.{sp}.pi"][0]
        P[f"orb.{sp}.sigma"][1] = P[f"orb.{sp}.sigma"][0]
    P["c"][:] = [1.0, -1.0]
    r = qi.make_walkers(s, 4, 16)
    st, lt = oracle.logpsi(torch.as_tensor(r), torch.as_tensor(p), s, a)
    assert np.all(st.numpy() == 0) and np.all(np.isneginf(lt.numpy()))
    res = oracle.local_energy(r, p, s, a)
    assert np.all(np.isnan(res["e_loc"]))


@pytest.mark.parametrize("ans", [SMALL, SMALL_JAS, SMALL_FULL, SMALL_EDGE],
                         ids=["plain", "cusp_jastrow", "full_det", "edge_update"])
def test_same_spin_exchange_antisymmetry(ans):
    s = _small_system()
    p = qi.make_params(s, ans, 17)
    r = qi.make_walkers(s, 5, 18)
    base = oracle.local_energy(r, p, s, ans)
    for (i, j) in ((0, 2), (3, 4)):
        rs = r.copy()
        rs[:, [i, j]] = rs[:, [j, i]]
        sw = oracle.local_energy(rs, p, s, ans)
        assert np.all(sw["sign"] == -base["sign"])
        np.testing.assert_allclose(sw["logpsi"], base["logpsi"], rtol=1e-13, atol=1e-13)
        np.testing.assert_allclose(sw["e_loc"], base["e_loc"], rtol=1e-11, atol=1e-11)
        g = base["grad"].copy()
        g[:, [i, j]] = g[:, [j, i]]
        np.testing.assert_allclose(sw["grad"], g, rtol=1e-11, atol=1e-12)


def test_translation_and_rotation_invariance():
    s = _small_system()
    p = qi.make_params(s, SMALL, 19)
    r = qi.make_walkers(s, 4, 20)
    base = oracle.local_energy(r, p, s, SMALL)
    q, _ = np.linalg.qr(np.random.default_rng(21).standard_normal((3, 3)))
    shift = np.array([0.7, -1.1, 2.3])
    R2 = tuple(tuple(float(x) for x in (q @ np.array(c) + shift)) for c in s.coords)
    s2 = qi.System(s.charges, R2, s.n_up, s.n_down)
    r2 = r @ q.T + shift
    moved = oracle.local_energy(r2, p, s2, SMALL)
    np.testing.assert_allclose(moved["logpsi"], base["logpsi"], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(moved["e_loc"], base["e_loc"], rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(moved["lap"], base["lap"], rtol=1e-10, atol=1e-10)


def _fd_grad_lap(r, p, s, a, h):
    """Central differences of the numpy forward: gradient and Laplacian."""
    W, N, _ = r.shape
    l0 = oracle.logpsi_np(r, p, s, a)[1]
    g = np.zeros((W, N, 3))
    lap = np.zeros(W)
    for i in range(N):
        for x in range(3):
            rp = r.copy(); rp[:, i, x] += h
            rm = r.copy(); rm[:, i, x] -= h
            lpp = oracle.logpsi_np(rp, p, s, a)[1]
            lmm = oracle.logpsi_np(rm, p, s, a)[1]
            g[:, i, x] = (lpp - lmm) / (2 * h)
            lap += (lpp - 2 * l0 + lmm) / h ** 2
    return g, lap


@pytest.mark.parametrize("ans", [SMALL, SMALL_CUSP, SMALL_JAS, SMALL_FULL, SMALL_EDGE],
                         ids=["plain", "ee_cusp", "jastrow", "full_det", "edge_update"])
def test_gradient_and_laplacian_vs_finite_differences(ans):
    s = _small_system()
    p = qi.make_params(s, ans, 23)
    r = qi.make_walkers(s, 4, 24)
    res = oracle.local_energy(r, p, s, ans)
    h = 2e-3
    g1, l1 = _fd_grad_lap(r, p, s, ans, h)
    g2, l2 = _fd_grad_lap(r, p, s, ans, h / 2)
    g = (4 * g2 - g1) / 3          # Richardson extrapolation of O(h^2) schemes
    lap = (4 * l2 - l1) / 3
    scale = np.abs(res["grad"]).max()
    assert np.abs(g - res["grad"]).max() < 1e-7 * max(scale, 1.0)
    np.testing.assert_allclose(lap, res["lap"], rtol=2e-6, atol=2e-6 * np.abs(res["lap"]).max())


@pytest.mark.parametrize("ans", [SMALL, SMALL_JAS, SMALL_EDGE], ids=["plain", "jastrow", "edge_update"])
def test_loss_gradient_vs_finite_differences_of_surrogate(ans):
    """FD (h = 1e-5, float64) of S(theta) = sum_w g_w log|psi_w(theta)| with the
    weights frozen, on sampled parameters (with the Jastrow: the last 64 too), against the autograd
    estimator."""
    s = _small_system()
    p = qi.make_params(s, ans, 25)
    r = qi.make_walkers(s, 6, 26)
    e = oracle.local_energy(r, p, s, ans)["e_loc"]
    G, e_mean, nf = oracle.loss_grad(r, e, p, s, ans)
    assert nf == 6 and abs(e_mean - e.mean()) < 1e-14 * abs(e_mean) + 1e-14
    wts = 2 * (e - e.mean()) / len(e)
    idx = np.random.default_rng(27).choice(len(p), 64, replace=False)
    if ans.jastrow:
        idx = np.concatenate([idx, np.arange(len(p) - 64, len(p))])
    if ans.edge_update:  # every parameter of one edge update
        off = 0
        for name, v in unpack(p, s, ans).items():
            if name == "mp1.opp.Ve":
                idx = np.concatenate([idx, off + np.arange(v.size)])
            off += v.size
    h = 1e-5
    for k in idx:
        pp = p.copy(); pp[k] += h
        pm = p.copy(); pm[k] -= h
        fd = (np.sum(wts * oracle.logpsi_np(r, pp, s, ans)[1]) -
              np.sum(wts * oracle.logpsi_np(r, pm, s, ans)[1])) / (2 * h)
        assert abs(fd - G[k]) < 1e-7 * max(1.0, np.abs(G).max())


def test_loss_gradient_zero_variance_hydrogen():
    """For the exact H-atom state every local energy equals -1/2, so G = 0."""
    H = qi.System((1.0,), ((0.0, 0.0, 0.0),), 1, 0)
    p = _one_center_params(H, SMALL, 1.0, np.random.default_rng(28))
    r = _random_points(16, 1, 29)
    e = oracle.local_energy(r, p, H, SMALL)["e_loc"]
    G, _, _ = oracle.loss_grad(r, e, p, H, SMALL)
    assert np.abs(G).max() < 1e-12


@pytest.mark.slow
def test_loss_gradient_unbiased_hydrogen_closed_form():
    """H atom with psi = exp(-sigma r), exact samples r ~ |psi|^2 (radius Gamma(3, 1/(2 sigma)),
    uniform direction): E[G_sigma] = sigma - 1 = d/dsigma (sigma^2/2 - sigma)."""
    H = qi.System((1.0,), ((0.0, 0.0, 0.0),), 1, 0)
    a = qi.Ansatz(n_rbf=4, rbf_dmax=6.0, init_layers=1, width=4, mp_layers=0, n_det=1, n_env=1)
    sigma = 1.4
    p = _one_center_params(H, a, sigma)
    names = list(oracle.param_shapes(H, a).keys())
    off = 0
    for nm, shp in oracle.param_shapes(H, a).items():
        if nm == "orb.up.sigma":
            break
        off += int(np.prod(shp))
    rng = np.random.default_rng(30)
    nb, per = 20, 2000
    ests = []
    for b in range(nb):
        rad = rng.gamma(3.0, 1.0 / (2 * sigma), per)
        v = rng.standard_normal((per, 3))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        r = (rad[:, None] * v)[:, None, :]
        e = -sigma ** 2 / 2 + (sigma - 1.0) / rad
        G, _, _ = oracle.loss_grad(r, e, p, H, a, chunk=per)
        ests.append(G[off])
    ests = np.array(ests)
    mean = ests.mean()
    err = ests.std(ddof=1) / math.sqrt(nb)     # non-overlapping batch means (Sec. V.A)
    assert abs(mean - (sigma - 1.0)) < 4 * err + 0.01 * (1.0 / per)
    assert "orb.up.sigma" in names


def test_metropolis_zero_step_accepts_everything():
    s, a, p, r = qi.workload_inputs(0, 8)
    lp = oracle.logpsi_np(r, p, s, a)[1]
    noise = qi.make_noise(1, 8, s.n_elec, 2)[0]
    u = qi.make_uniforms(1, 8, 3)[0]
    r2, lp2, acc, _ = oracle.metropolis_step(r, lp, noise, u, 0.0, p, s, a)
    assert np.all(acc == 1) and np.all(r2 == r)
    np.testing.assert_allclose(lp2, lp, rtol=1e-13)


def test_metropolis_rejects_nan_and_accepts_u_zero():
    s, a, p, r = qi.workload_inputs(0, 4)
    lp = oracle.logpsi_np(r, p, s, a)[1]
    noise = qi.make_noise(1, 4, s.n_elec, 2)[0]
    u = np.array([0.0, 0.0, 0.999999, 0.5])
    lp_in = lp.copy()
    lp_in[1] = np.inf            # current state infinitely likely -> proposal rejected unless u = 0
    r2, lp2, acc, prop = oracle.metropolis_step(r, lp_in, noise, u, 0.5, p, s, a)
    assert acc[0] == 1           # log 0 = -inf < anything finite
    assert acc[1] == 0           # -inf < -inf is false


@pytest.mark.slow
def test_metropolis_hydrogen_mean_radius():
    """Sampling |exp(-r)|^2 with the random-walk Metropolis step gives <r> = 3/2."""
    H = qi.System((1.0,), ((0.0, 0.0, 0.0),), 1, 0)
    a = qi.Ansatz(n_rbf=4, rbf_dmax=6.0, init_layers=1, width=4, mp_layers=0, n_det=1, n_env=1)
    p = _one_center_params(H, a, 1.0)
    W = 1000
    r = _random_points(W, 1, 31, scale=1.0)
    lp = oracle.logpsi_np(r, p, H, a)[1]
    rng = np.random.default_rng(32)
    rs = []
    for t in range(400):
        r, lp, acc, _ = oracle.metropolis_step(r, lp, rng.standard_normal((W, 1, 3)), rng.random(W), 0.6, p, H, a, chunk=W)
        if t >= 100:
            rs.append(np.linalg.norm(r[:, 0], axis=-1))
    rs = np.array(rs)                    # [steps, W]
    per_walker = rs.mean(0)
    mean = per_walker.mean()
    err = per_walker.std(ddof=1) / math.sqrt(W)
    assert abs(mean - 1.5) < 4 * err


def _gauss_logq(x, y, gy, eps):
    """log N(x; y + eps^2 gy, eps^2 I) up to the common constant, written out from the definition."""
    d = (x - y - eps * eps * gy).reshape(x.shape[0], -1)
    return -(d * d).sum(1) / (2.0 * eps * eps)


@pytest.mark.parametrize("damp", [False, True])
def test_mala_acceptance_is_the_hastings_ratio(damp):
    """The closed form of the Langevin acceptance equals log pi(r') - log pi(r) + log q(r | r') -
    log q(r' | r) with pi = |psi|^2 and Gaussian drift proposals, evaluated from the positions."""
    s, a, p, r = qi.workload_inputs(0, 16)
    lp, g = oracle.logpsi_and_grad(r, p, s, a)
    xi = qi.make_noise(1, 16, s.n_elec, 7)[0]
    for eps in (0.05, 0.3):
        D = oracle.langevin_drift(r, g, eps * eps, s, damp)
        prop = (r + eps * eps * D) + eps * xi
        lpp, gp = oracle.logpsi_and_grad(prop, p, s, a)
        Dp = oracle.langevin_drift(prop, gp, eps * eps, s, damp)
        ref = 2.0 * (lpp - lp) + _gauss_logq(r, prop, Dp, eps) - _gauss_logq(prop, r, D, eps)
        got = oracle.mala_log_accept(lp, D, lpp, Dp, xi, eps)
        np.testing.assert_allclose(got, ref, rtol=1e-9, atol=1e-9)
        r2, _, _, _, prop2 = oracle.mala_step(r, lp, g, xi, np.full(16, 0.5), eps, p, s, a, damp=damp)
        np.testing.assert_array_equal(prop2, prop)


def test_drift_damping_limits():
    """The damping keeps small drifts, bounds large ones by sqrt(2 tau / a) and by the distance to
    the nearest nucleus, and a takes its published end values (1/2 on the nucleus, 3/5 far away)."""
    assert oracle.drift_damping_a(0.0) == 0.5
    assert abs(oracle.drift_damping_a(1e8) - 0.6) < 1e-12
    H2 = qi.System((1.0, 1.0), ((0.0, 0.0, -0.7), (0.0, 0.0, 0.7)), 1, 1)
    rng = np.random.default_rng(5)
    r = rng.normal(size=(64, 2, 3)) * 2.0
    tau = 0.04
    tiny = rng.normal(size=r.shape) * 1e-4
    r_far = r + np.array([0.0, 0.0, 50.0])
    np.testing.assert_allclose(oracle.langevin_drift(r_far, tiny, tau, H2), tiny, rtol=1e-8)
    big = rng.normal(size=r.shape) * 1e3
    D = oracle.langevin_drift(r, big, tau, H2)
    d = np.linalg.norm(r[:, :, None] - H2.R()[None, None], axis=-1).min(-1)
    step = tau * np.linalg.norm(D, axis=-1)
    assert np.all(step <= d * (1 + 1e-14))
    assert np.all(step <= np.sqrt(2 * tau / 0.5) * (1 + 1e-14))
    cos = (D * big).sum(-1) / (np.linalg.norm(D, axis=-1) * np.linalg.norm(big, axis=-1))
    np.testing.assert_allclose(cos, 1.0, rtol=1e-12)
    # an electron on a nucleus does not drift; far from the cap, the shortening factor is the
    # (sqrt(1 + 2x) - 1) / x of the published limit
    r0 = np.zeros((1, 2, 3))
    r0[0, 0] = H2.R()[0]
    r0[0, 1] = (0.0, 3.0, 0.0)
    v = np.array([[[1.0, 2.0, 0.0], [0.3, 0.0, 0.0]]])
    D0 = oracle.langevin_drift(r0, v, tau, H2)
    assert np.all(D0[0, 0] == 0.0)
    dn = math.sqrt(9 + 0.49)
    a1 = 0.5 + dn ** 2 / (10 * (4 + dn ** 2))
    x = a1 * 0.09 * tau
    np.testing.assert_allclose(D0[0, 1], v[0, 1] * (math.sqrt(1 + 2 * x) - 1) / x, rtol=1e-12)


def test_mala_gradient_matches_finite_differences():
    """The reverse-pass gradient the Langevin drift uses agrees with central differences of log|psi|."""
    s, a, p, r = qi.workload_inputs(0, 4)
    _, g = oracle.logpsi_and_grad(r, p, s, a)
    h = 1e-5
    for c in range(3):
        rp, rm = r.copy(), r.copy()
        rp[:, 1, c] += h
        rm[:, 1, c] -= h
        fd = (oracle.logpsi_np(rp, p, s, a)[1] - oracle.logpsi_np(rm, p, s, a)[1]) / (2 * h)
        np.testing.assert_allclose(g[:, 1, c], fd, rtol=1e-6, atol=1e-7)


def test_mala_zero_step_accepts_everything_and_rejects_nan():
    s, a, p, r = qi.workload_inputs(0, 8)
    lp, g = oracle.logpsi_and_grad(r, p, s, a)
    xi = qi.make_noise(1, 8, s.n_elec, 2)[0]
    u = qi.make_uniforms(1, 8, 3)[0]
    r2, lp2, g2, acc, _ = oracle.mala_step(r, lp, g, xi, u, 0.0, p, s, a)
    assert np.all(acc == 1) and np.all(r2 == r)
    np.testing.assert_allclose(lp2, lp, rtol=1e-13)
    gbad = g.copy()
    gbad[2] = np.nan
    _, _, _, acc2, _ = oracle.mala_step(r, lp, gbad, xi, np.zeros(8), 0.1, p, s, a)
    assert acc2[2] == 0 and np.all(np.delete(acc2, 2) == 1)


@pytest.mark.slow
@pytest.mark.parametrize("damp", [False, True])
def test_mala_hydrogen_mean_radius(damp):
    """Sampling |exp(-r)|^2 with the Langevin step gives <r> = 3/2, with and without damping."""
    H = qi.System((1.0,), ((0.0, 0.0, 0.0),), 1, 0)
    a = qi.Ansatz(n_rbf=4, rbf_dmax=6.0, init_layers=1, width=4, mp_layers=0, n_det=1, n_env=1)
    p = _one_center_params(H, a, 1.0)
    W = 1000
    r = _random_points(W, 1, 41, scale=1.0)
    lp, g = oracle.logpsi_and_grad(r, p, H, a, chunk=W)
    rng = np.random.default_rng(42)
    rs = []
    for t in range(300):
        r, lp, g, acc, _ = oracle.mala_step(r, lp, g, rng.standard_normal((W, 1, 3)), rng.random(W), 0.5, p, H, a,
                                            damp=damp, chunk=W)
        if t >= 100:
            rs.append(np.linalg.norm(r[:, 0], axis=-1))
    per_walker = np.array(rs).mean(0)
    mean = per_walker.mean()
    err = per_walker.std(ddof=1) / math.sqrt(W)
    assert abs(mean - 1.5) < 4 * err


def _golden_clipping():
    rows = []
    with open(os.path.join(GOLDEN, "clipping_example.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                w, x, y = line.split("|")
                rows.append((float(w), np.array(x.split(), dtype=float), np.array(y.split(), dtype=float)))
    return rows


@pytest.mark.parametrize("width,x,y", _golden_clipping())
def test_hard_clipping_hand_example(width, x, y):
    got = oracle.clip_local_energy(x, width, "hard")
    np.testing.assert_allclose(got, y, rtol=1e-14, atol=1e-14)


def test_clipping_window_statistics_by_brute_force():
    """Median by sorting in plain Python (odd and even counts, non-finite values excluded), the
    window, and the soft shape's continuity, unit slope at the edge, odd symmetry and logarithmic
    growth."""
    rng = np.random.default_rng(77)
    for n in (1, 2, 7, 8, 101, 256):
        x = rng.standard_cauchy(n) * 3 - 40
        x_in = np.concatenate([x, [np.nan, np.inf, -np.inf]])
        srt = sorted(float(v) for v in x)
        med = srt[n // 2] if n % 2 else 0.5 * (srt[n // 2 - 1] + srt[n // 2])
        mad = sum(abs(float(v) - med) for v in x) / n
        for width in (0.5, 5.0):
            sig = width * mad
            hard = oracle.clip_local_energy(x_in, width, "hard")
            soft = oracle.clip_local_energy(x_in, width, "soft")
            assert np.isnan(hard[n]) and hard[n + 1] == np.inf and hard[n + 2] == -np.inf
            inside = np.abs(x - med) <= sig
            np.testing.assert_array_equal(hard[:n][inside], x[inside])
            np.testing.assert_array_equal(soft[:n][inside], x[inside])
            np.testing.assert_allclose(hard[:n][~inside], med + np.sign(x[~inside] - med) * sig, rtol=1e-13)
            assert np.all(np.abs(soft[:n] - med) >= np.abs(hard[:n] - med) - 1e-12)
            assert np.all(np.diff(soft[:n][np.argsort(x)]) >= 0)
    # soft shape around mu = 0, sigma = 1 (values 0 and +-1 fix the median and deviation)
    base = np.array([-1.0, 0.0, 1.0] * 50)
    for t in (1.0 + 1e-9, 2.0, 4.0, 8.0):
        v = oracle.clip_local_energy(np.concatenate([base, [t, -t]]), 1.0, "soft")[-2:]
        mad = (100 + 2 * t) / 152
        assert abs(v[0] + v[1]) < 1e-12
        if t > 1.5:
            assert abs(v[0] - mad * (1 + math.log(t / mad))) < 1e-12
    # just outside the edge: t = sigma (1 + e) with sigma = (100 + 2 t) / 152 solved for t
    e = 1e-7
    t = (100 / 152) * (1 + e) / (1 - 2 * (1 + e) / 152)
    a = oracle.clip_local_energy(np.concatenate([base, [t, -t]]), 1.0, "soft")[-2]
    assert abs(a - t) < 1e-12  # continuous, unit slope at the edge


def test_clipping_degenerate_cases():
    assert np.all(np.isnan(oracle.clip_local_energy(np.array([np.nan, np.nan]), 5.0)))
    x = np.full(6, -1.25)
    np.testing.assert_array_equal(oracle.clip_local_energy(x, 5.0, "soft"), x)


def test_zero_edge_updates_match_zeroed_filter_inputs():
    """Edge updates with Ve = 0 and ce = 0 map every later edge feature to tanh(0) = 0, so the
    ansatz equals the plain one whose later layers have U1 = 0 (their filters see only the bias)."""
    s = _small_system()
    pe = qi.make_params(s, SMALL_EDGE, 33)
    Pe = unpack(pe, s, SMALL_EDGE)
    for l in range(1, SMALL.mp_layers):
        for t in ("same", "opp", "nuc"):
            Pe[f"mp{l}.{t}.Ve"][:] = 0.0
            Pe[f"mp{l}.{t}.ce"][:] = 0.0
    r = qi.make_walkers(s, 4, 34)
    a = oracle.logpsi_np(r, pe, s, SMALL_EDGE)[1]
    # the same parameters without the updates, U1 = 0 in the later layers
    p0 = np.concatenate([Pe[k].ravel() for k in Pe if not k.endswith((".Ve", ".ce"))])
    P0 = unpack(p0, s, SMALL)
    for l in range(1, SMALL.mp_layers):
        for t in ("same", "opp", "nuc"):
            P0[f"mp{l}.{t}.U1"][:] = 0.0
    b = oracle.logpsi_np(r, p0, s, SMALL)[1]
    np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-13)


def test_coincident_pair_gives_nan_local_energy():
    """At an exactly coincident electron pair the Coulomb potential is singular and E_L is undefined:
    the oracle returns NaN there and an ordinary value elsewhere (opposite-spin pairs: a same-spin
    pair makes two rows of a matrix equal, and autograd through an exactly singular matrix raises)."""
    s, a, p, r = qi.workload_inputs(0, 3)
    r = r.copy()
    r[0, 1] = r[0, 0]
    res = oracle.local_energy(r, p, s, a)
    assert np.isnan(res["e_loc"][0]) and np.all(np.isfinite(res["e_loc"][1:]))
    assert np.isfinite(res["logpsi"][0])
    s, a, p, r = qi.workload_inputs(1, 2)
    r = r.copy()
    r[0, 8] = r[0, 1]
    res = oracle.local_energy(r, p, s, a)
    assert np.isnan(res["e_loc"][0]) and np.isfinite(res["e_loc"][1])
