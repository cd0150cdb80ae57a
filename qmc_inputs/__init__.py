"""Seeded synthetic inputs shared by the HIP path's tests/benchmarks and the oracle.

This module holds no arithmetic of the method: it only defines the benchmark
systems (nuclear charges and positions, spin counts), the ansatz
hyper-parameters, and draws walkers, parameter blobs, Metropolis noise and
uniforms from numpy PCG64 generators with fixed seeds.  Everything is float64
on the host; callers cast or copy as they need.

Seeds: for workload k in 0..4, seed = 1000*k + j with j = 0 parameters,
1 walkers, 2 proposal noise, 3 uniforms, 4 molecules.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence, Tuple

import numpy as np


@dataclasses.dataclass(frozen=True)
class System:
    """A molecule: nuclear charges Z[M], positions R[M][3] (bohr), spin counts.

    Electrons 0..n_up-1 are spin-up, the rest spin-down (Sec. II.B spin
    convention)."""

    charges: Tuple[float, ...]
    coords: Tuple[Tuple[float, float, float], ...]
    n_up: int
    n_down: int

    @property
    def n_nuc(self) -> int:
        return len(self.charges)

    @property
    def n_elec(self) -> int:
        return self.n_up + self.n_down

    def R(self) -> np.ndarray:
        return np.asarray(self.coords, dtype=np.float64).reshape(self.n_nuc, 3)

    def Z(self) -> np.ndarray:
        return np.asarray(self.charges, dtype=np.float64)


@dataclasses.dataclass(frozen=True)
class Ansatz:
    """Hyper-parameters of the graph-network ansatz (Sec. III)."""

    n_rbf: int = 16          # K Gaussian radial basis functions
    rbf_dmax: float = 8.0    # centres spread on [0, dmax] bohr
    init_layers: int = 1     # L0 tanh layers of the electron-node initialisation
    width: int = 128         # D embedding width
    mp_layers: int = 4       # L message-passing interaction layers
    n_det: int = 16          # determinants
    n_env: int = 8           # envelope exponents per nucleus and orbital
    include_vnn: int = 1     # add the constant nuclear repulsion to V
    ee_cusp: float = 0.0     # length alpha of the fixed electron-electron cusp factor (0: none)
    jastrow: int = 0         # 1: learnable Jastrow factor exp(J), J an MLP of the summed embeddings
    full_det: int = 0        # 1: one N x N determinant per p over both spins (N orbitals per spin map)
    edge_update: int = 0     # 1: edge features updated in every interaction layer after the first


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    index: int
    systems: Tuple[System, ...]
    ansatz: Ansatz
    walkers: int
    precision: str           # "fp64" | "fp32" | "bf16"
    metropolis_steps: int = 0
    step_size: float = 0.2


# --------------------------------------------------------------------------
# Parameter layout (table only: names, shapes, initialisation kind).
# Order and shapes follow the pinned parameter blob: matrices stored [in][out].
# --------------------------------------------------------------------------

def param_table(system: System, ans: Ansatz) -> List[Tuple[str, Tuple[int, ...], str, int]]:
    """List of (name, shape, init-kind, fan_in) in blob order."""
    M, K, D = system.n_nuc, ans.n_rbf, ans.width
    out: List[Tuple[str, Tuple[int, ...], str, int]] = []
    out.append(("init.W1", ((M + 2) * K, D), "w", (M + 2) * K))
    out.append(("init.b1", (D,), "zero", 0))
    for l in range(2, ans.init_layers + 1):
        out.append((f"init.W{l}", (D, D), "w", D))
        out.append((f"init.b{l}", (D,), "zero", 0))
    for l in range(ans.mp_layers):
        for t in ("same", "opp", "nuc"):
            out.append((f"mp{l}.{t}.U1", (K, D), "w", K))
            out.append((f"mp{l}.{t}.a1", (D,), "zero", 0))
            out.append((f"mp{l}.{t}.U2", (D, D), "w", D))
            out.append((f"mp{l}.{t}.a2", (D,), "zero", 0))
            if ans.edge_update and l >= 1:
                out.append((f"mp{l}.{t}.Ve", (K, K), "w", K))
                out.append((f"mp{l}.{t}.ce", (K,), "zero", 0))
        out.append((f"mp{l}.Wh", (D, D), "w", D))
        out.append((f"mp{l}.bh", (D,), "zero", 0))
        out.append((f"mp{l}.Y", (M, D), "normal", 0))
        out.append((f"mp{l}.Wg", (3 * D, D), "w", 3 * D))
        out.append((f"mp{l}.bg", (D,), "zero", 0))
    for s, n in (("up", system.n_up), ("down", system.n_down)):
        if n == 0:
            continue
        P = ans.n_det
        no = system.n_up + system.n_down if ans.full_det else n  # orbitals per determinant
        out.append((f"orb.{s}.W", (D, P * no), "w", D))
        out.append((f"orb.{s}.b", (P * no,), "zero", 0))
        out.append((f"orb.{s}.pi", (P, no, M, ans.n_env), "one", 0))
        out.append((f"orb.{s}.sigma", (P, no, M, ans.n_env), "sigma", 0))
    out.append(("c", (ans.n_det,), "one", 0))
    if ans.jastrow:
        out.append(("jas.W1", (D, D), "w", D))
        out.append(("jas.b1", (D,), "zero", 0))
        out.append(("jas.W2", (D, 1), "w", D))
        out.append(("jas.b2", (1,), "zero", 0))
    return out


def param_count(system: System, ans: Ansatz) -> int:
    return int(sum(int(np.prod(s)) for _, s, _, _ in param_table(system, ans)))


def make_params(system: System, ans: Ansatz, seed: int) -> np.ndarray:
    """Random-init parameter blob (float64), drawn tensor by tensor in blob order.

    Weights ~ N(0, 1/fan_in), biases 0, nuclear vectors Y ~ N(0, 1),
    envelope weights pi = 1, exponents sigma ~ U[0.5, 2], coefficients c = 1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for _, shape, kind, fan_in in param_table(system, ans):
        n = int(np.prod(shape))
        if kind == "w":
            parts.append(rng.standard_normal(n) / math.sqrt(fan_in))
        elif kind == "normal":
            parts.append(rng.standard_normal(n))
        elif kind == "zero":
            parts.append(np.zeros(n))
        elif kind == "one":
            parts.append(np.ones(n))
        elif kind == "sigma":
            parts.append(rng.uniform(0.5, 2.0, n))
        else:  # pragma: no cover
            raise ValueError(kind)
    return np.concatenate(parts).astype(np.float64)


def make_walkers(system: System, n_walkers: int, seed: int) -> np.ndarray:
    """Walkers r[W][N][3]: each electron at a uniformly chosen nucleus plus N(0, 1) per coordinate."""
    rng = np.random.Generator(np.random.PCG64(seed))
    R = system.R()
    idx = rng.integers(0, system.n_nuc, (n_walkers, system.n_elec))
    return R[idx] + rng.standard_normal((n_walkers, system.n_elec, 3))


def make_noise(n_steps: int, n_walkers: int, n_elec: int, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((n_steps, n_walkers, n_elec, 3))


def make_uniforms(n_steps: int, n_walkers: int, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.random((n_steps, n_walkers))


def make_molecules(seed: int, targets: Sequence[int]) -> List[System]:
    """Synthetic neutral molecules with 2-6 nuclei of Z in {1,3,6,7,8}.

    For each target electron count N: redraw (M, Z) until sum Z = N; place the
    first nucleus at the origin and every next one at distance U[1.5, 3] bohr in a
    uniform random direction from a uniformly chosen placed nucleus, rejecting
    placements closer than 1.5 bohr to any placed nucleus."""
    rng = np.random.Generator(np.random.PCG64(seed))
    zs = np.array([1, 3, 6, 7, 8])
    mols = []
    for n in targets:
        while True:
            m = int(rng.integers(2, 7))
            Z = zs[rng.integers(0, len(zs), m)]
            if int(Z.sum()) == n:
                break
        pos = [np.zeros(3)]
        while len(pos) < m:
            base = pos[int(rng.integers(0, len(pos)))]
            v = rng.standard_normal(3)
            v /= np.linalg.norm(v)
            cand = base + rng.uniform(1.5, 3.0) * v
            if all(np.linalg.norm(cand - p) >= 1.5 for p in pos):
                pos.append(cand)
        mols.append(System(tuple(float(z) for z in Z),
                           tuple(tuple(float(x) for x in p) for p in pos),
                           (n + 1) // 2, n // 2))
    return mols


# --------------------------------------------------------------------------
# The five workloads
# --------------------------------------------------------------------------

H2 = System((1.0, 1.0), ((0.0, 0.0, 0.7), (0.0, 0.0, -0.7)), 1, 1)
N2 = System((7.0, 7.0), ((0.0, 0.0, 1.034), (0.0, 0.0, -1.034)), 7, 7)


def _c4h4() -> System:
    cs = [(1.45, 1.25), (1.45, -1.25), (-1.45, 1.25), (-1.45, -1.25)]
    coords = [(x, y, 0.0) for x, y in cs]
    for x, y in cs:
        n = math.hypot(x, y)
        coords.append((x + 2.05 * x / n, y + 2.05 * y / n, 0.0))
    return System((6.0,) * 4 + (1.0,) * 4, tuple(coords), 14, 14)


C4H4 = _c4h4()
BATCH_TARGETS = [4, 7, 9, 12, 14, 17, 19, 22, 24, 27, 29, 32, 34, 37, 39, 42]

H2_ANSATZ = Ansatz(init_layers=2, width=32, mp_layers=0, n_det=1, n_env=4)
N2_ANSATZ = Ansatz(init_layers=1, width=128, mp_layers=4, n_det=16, n_env=8)
C4H4_ANSATZ = Ansatz(init_layers=1, width=256, mp_layers=4, n_det=32, n_env=8)
BATCH_ANSATZ = Ansatz(init_layers=1, width=128, mp_layers=4, n_det=8, n_env=8)


def workload(k: int) -> Workload:
    if k == 0:
        return Workload("h2_fp64", 0, (H2,), H2_ANSATZ, 256, "fp64")
    if k == 1:
        return Workload("n2_fp32", 1, (N2,), N2_ANSATZ, 4096, "fp32", 10, 0.2)
    if k == 2:
        return Workload("n2_grad", 2, (N2,), N2_ANSATZ, 4096, "fp32")
    if k == 3:
        return Workload("c4h4_bf16", 3, (C4H4,), C4H4_ANSATZ, 8192, "bf16")
    if k == 4:
        return Workload("batched16", 4, tuple(make_molecules(4004, BATCH_TARGETS)),
                        BATCH_ANSATZ, 1024, "fp32")
    raise ValueError(k)


# --------------------------------------------------------------------------
# System-size sweep (Sec. VI, scaling): atoms and hydrogen chains up to 45 electrons
# --------------------------------------------------------------------------

SCALING_ATOMS = (2, 4, 6, 10, 14, 18, 24, 30, 36, 45)
SCALING_CHAINS = (2, 4, 6, 10, 14, 18, 24, 30, 36, 44)
SCALING_WALKERS = 2000
SCALING_ANSATZ = N2_ANSATZ


def atom(Z: int) -> System:
    """A neutral atom of charge Z at the origin with the smallest spin polarisation
    (n_up = ceil(Z / 2))."""
    return System((float(Z),), ((0.0, 0.0, 0.0),), (Z + 1) // 2, Z // 2)


def hydrogen_chain(n: int, spacing: float = 1.8) -> System:
    """n hydrogen atoms equally spaced (bohr) on the z axis, centred on the origin, neutral,
    n_up = ceil(n / 2)."""
    z0 = -0.5 * spacing * (n - 1)
    return System((1.0,) * n, tuple((0.0, 0.0, z0 + spacing * i) for i in range(n)), (n + 1) // 2, n // 2)


def seed(k: int, j: int) -> int:
    return 1000 * k + j


def workload_inputs(k: int, n_walkers: int | None = None, system_index: int = 0):
    """(system, ansatz, params, walkers) for one system of workload k.

    For the batched workload every molecule gets its own parameter and walker
    streams (seed offset by 100 * system index)."""
    wl = workload(k)
    sysm = wl.systems[system_index]
    off = 100 * system_index
    W = wl.walkers if n_walkers is None else n_walkers
    params = make_params(sysm, wl.ansatz, seed(k, 0) + off)
    r = make_walkers(sysm, W, seed(k, 1) + off)
    return sysm, wl.ansatz, params, r
