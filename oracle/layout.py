"""Parameter blob of the ansatz, unpacked into named arrays (oracle side).

The blob is one flat vector; each tensor is stored row-major, matrices as
[in][out] so that a layer computes y = x W + b.  Order: the electron-node
initialisation MLP (Sec. III.A, node features, second case of the electron
initialisation equation), then per interaction layer the three edge filters
w (same-spin, opposite-spin, electron-nucleus), the sender map h, the nuclear
node vectors and the update g (graph-convolution and embedding-update
equations), then per spin the orbital map kappa and the isotropic envelope
weights/exponents (Sec. III.B), then the determinant coefficients c_p
(generalised Slater determinant equation, Sec. II.C).
"""
from __future__ import annotations

from collections import OrderedDict

import numpy as np


def param_shapes(system, ans):
    M, K, D = len(system.charges), ans.n_rbf, ans.width
    shapes = OrderedDict()
    shapes["init.W1"] = ((M + 2) * K, D)
    shapes["init.b1"] = (D,)
    for l in range(2, ans.init_layers + 1):
        shapes[f"init.W{l}"] = (D, D)
        shapes[f"init.b{l}"] = (D,)
    for l in range(ans.mp_layers):
        for t in ("same", "opp", "nuc"):
            shapes[f"mp{l}.{t}.U1"] = (K, D)
            shapes[f"mp{l}.{t}.a1"] = (D,)
            shapes[f"mp{l}.{t}.U2"] = (D, D)
            shapes[f"mp{l}.{t}.a2"] = (D,)
            if getattr(ans, "edge_update", 0) and l >= 1:
                shapes[f"mp{l}.{t}.Ve"] = (K, K)
                shapes[f"mp{l}.{t}.ce"] = (K,)
        shapes[f"mp{l}.Wh"] = (D, D)
        shapes[f"mp{l}.bh"] = (D,)
        shapes[f"mp{l}.Y"] = (M, D)
        shapes[f"mp{l}.Wg"] = (3 * D, D)
        shapes[f"mp{l}.bg"] = (D,)
    for s, n in (("up", system.n_up), ("down", system.n_down)):
        if n > 0:
            # full determinant: every spin's orbital map gives all N orbitals of each determinant
            no = system.n_up + system.n_down if getattr(ans, "full_det", 0) else n
            shapes[f"orb.{s}.W"] = (D, ans.n_det * no)
            shapes[f"orb.{s}.b"] = (ans.n_det * no,)
            shapes[f"orb.{s}.pi"] = (ans.n_det, no, M, ans.n_env)
            shapes[f"orb.{s}.sigma"] = (ans.n_det, no, M, ans.n_env)
    shapes["c"] = (ans.n_det,)
    if getattr(ans, "jastrow", 0):
        D = ans.width
        shapes["jas.W1"] = (D, D)
        shapes["jas.b1"] = (D,)
        shapes["jas.W2"] = (D, 1)
        shapes["jas.b2"] = (1,)
    return shapes


def param_count(system, ans) -> int:
    return int(sum(int(np.prod(s)) for s in param_shapes(system, ans).values()))


def unpack(blob, system, ans):
    """Views of the blob (numpy array or torch tensor) keyed by tensor name."""
    out = OrderedDict()
    off = 0
    for name, shape in param_shapes(system, ans).items():
        n = int(np.prod(shape))
        out[name] = blob[off:off + n].reshape(shape)
        off += n
    if off != blob.shape[0]:
        raise ValueError(f"parameter blob has {blob.shape[0]} entries, layout needs {off}")
    return out
