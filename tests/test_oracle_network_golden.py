"""Pins of the oracle's network reading against a hand-worked example and closed forms.

tests/golden/tiny_network.txt evaluates a 3-electron, 2-nucleus instance of the
ansatz step by step by hand: the radial basis, the electron initialisation with
its same-spin / opposite-spin means (Sec. III.A, node features), the filters,
mean-normalised messages and the residual concatenation update (Sec. III.A,
message generation and embedding update), orbitals times envelopes (Sec.
III.B), the spin-factorised determinants (Sec. III.C) and the signed sum over
determinants (Sec. II.C, log domain Sec. III.E).  The example has two
same-spin electrons (divisor N_up - 1 = 1), a down electron averaging over two
opposite-spin partners (divisor 2), a same-spin mean over nothing (0), two
nuclei (divisor M = 2) and two determinants of opposite sign, so a wrong
divisor, a swapped concatenation block, a missing residual or a dropped sign
changes the result.
"""
import math
import os

import numpy as np
import pytest
import torch

import oracle
import qmc_inputs as qi
from oracle import ansatz as oa
from oracle.layout import param_shapes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "tiny_network.txt")


def _load():
    sysd, ansd, pos, params, rho, f1, A, logdet = {}, {}, [], {}, [], {}, {}, {}
    exp = {}
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            key = tok[0]
            if key == "system":
                sysd[tok[1]] = [float(v) for v in tok[2:]]
            elif key == "ansatz":
                ansd[tok[1]] = float(tok[2])
            elif key == "position":
                pos.append([float(v) for v in tok[1:]])
            elif key == "param":
                params[tok[1]] = [float(v) for v in tok[2:]]
            elif key == "rho":
                rho.append([float(v) for v in tok[1:]])
            elif key == "f1":
                f1[int(tok[1])] = [float(v) for v in tok[2:]]
            elif key == "A":
                A[(tok[1], int(tok[2]), int(tok[3]), int(tok[4]))] = float(tok[5])
            elif key == "logdet":
                logdet[int(tok[1])] = (float(tok[2]), float(tok[3]))
            else:
                exp[key] = float(tok[1])
    nuc = sysd["coords"]
    system = qi.System(charges=tuple(sysd["charges"]),
                       coords=tuple(tuple(nuc[3 * i:3 * i + 3]) for i in range(len(sysd["charges"]))),
                       n_up=int(sysd["spins"][0]), n_down=int(sysd["spins"][1]))
    ans = qi.Ansatz(n_rbf=int(ansd["n_rbf"]), rbf_dmax=ansd["rbf_dmax"], init_layers=int(ansd["init_layers"]),
                    width=int(ansd["width"]), mp_layers=int(ansd["mp_layers"]), n_det=int(ansd["n_det"]),
                    n_env=int(ansd["n_env"]))
    shapes = param_shapes(system, ans)
    assert list(shapes) == list(params), "golden parameters must be listed in blob order"
    blob = []
    for name, shape in shapes.items():
        assert len(params[name]) == int(np.prod(shape)), name
        blob += params[name]
    return system, ans, np.asarray([pos]), np.asarray(blob), rho, f1, A, logdet, exp


TOL = 1e-13


def test_golden_radial_basis():
    system, ans, *_ , rho, f1, A, logdet, exp = _load()
    for row in rho:
        d, vals = row[0], row[1:]
        got = oa.rbf(torch.tensor([d], dtype=torch.float64), ans.n_rbf, ans.rbf_dmax)[0].numpy()
        np.testing.assert_allclose(got, vals, rtol=0, atol=TOL)


def test_golden_embedding_and_orbitals():
    system, ans, r, blob, rho, f1, A, logdet, exp = _load()
    P = oracle.unpack(torch.tensor(blob), system, ans)
    f, _ = oa.embedding(torch.tensor(r), P, system, ans)
    for i, v in f1.items():
        np.testing.assert_allclose(f[0, i].numpy(), v, rtol=0, atol=TOL)
    mats = oa.orbital_matrices(torch.tensor(r), P, system, ans)
    for (s, p, a, k), v in A.items():
        got = float(mats[0 if s == "up" else 1][0, p, a, k])
        assert abs(got - v) <= TOL, (s, p, a, k, got, v)


def test_golden_logpsi_both_forwards():
    system, ans, r, blob, rho, f1, A, logdet, exp = _load()
    s_t, l_t = oracle.logpsi(torch.tensor(r), torch.tensor(blob), system, ans)
    s_n, l_n = oracle.logpsi_np(r, blob, system, ans)
    assert abs(float(l_t[0]) - exp["logpsi"]) <= TOL
    assert abs(float(l_n[0]) - exp["logpsi"]) <= TOL
    assert float(s_t[0]) == exp["sign"] and float(s_n[0]) == exp["sign"]


def test_golden_signed_determinant_sum():
    """The log-domain combination on the example's two determinants of opposite sign."""
    system, ans, r, blob, rho, f1, A, logdet, exp = _load()
    ld = torch.tensor([[logdet[0][0], logdet[1][0]]], dtype=torch.float64)
    sg = torch.tensor([[logdet[0][1], logdet[1][1]]], dtype=torch.float64)
    c = torch.tensor(blob[-2:], dtype=torch.float64)
    s, l = oa.combine(ld, sg, c)
    assert float(s[0]) == exp["sign"]
    assert abs(float(l[0]) - exp["logpsi"]) <= TOL


@pytest.mark.parametrize("K,dmax", [(2, 2.0), (16, 8.0), (5, 3.0)])
def test_rbf_centre_and_width(K, dmax):
    """rho_k(mu_k) = 1 and rho_k(mu_k +- s) = 1/e for every k (centres k dmax/(K-1), width
    dmax/(K-1))."""
    s = dmax / (K - 1)
    for k in range(K):
        mu = k * s
        d = torch.tensor([mu, mu + s, mu - s], dtype=torch.float64)
        v = oa.rbf(d, K, dmax)[:, k].numpy()
        np.testing.assert_allclose(v, [1.0, math.exp(-1.0), math.exp(-1.0)], rtol=1e-15, atol=0)


@pytest.mark.parametrize("lds,sgs,c,sign,lp", [
    # 2 - 1.5 = 0.5
    ([math.log(2.0), math.log(3.0)], [1.0, -1.0], [1.0, 0.5], 1.0, math.log(0.5)),
    # -2 + 3 * 0.25 = -1.25
    ([math.log(2.0), math.log(3.0)], [-1.0, 1.0], [1.0, 0.25], -1.0, math.log(1.25)),
    # three terms: 1e-300 scale, e^-700 (log shift needed), sum 4e + ... : 5 - 2 - 1 = 2 at scale e^-700
    ([-700.0 + math.log(5.0), -700.0 + math.log(2.0), -700.0], [1.0, -1.0, -1.0], [1.0, 1.0, 1.0], 1.0,
     -700.0 + math.log(2.0)),
    # c_p = 0 drops its term; a negative coefficient flips the sign
    ([0.0, 10.0], [1.0, 1.0], [-2.0, 0.0], -1.0, math.log(2.0)),
])
def test_combine_signed_terms(lds, sgs, c, sign, lp):
    s, l = oa.combine(torch.tensor([lds], dtype=torch.float64), torch.tensor([sgs], dtype=torch.float64),
                      torch.tensor(c, dtype=torch.float64))
    assert float(s[0]) == sign
    assert abs(float(l[0]) - lp) <= 1e-12 * max(1.0, abs(lp))
