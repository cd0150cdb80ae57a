"""ctypes binding of libqmc.so (argument marshalling only).

Every computation runs in the HIP library; torch provides device memory and
the current stream.  The functions raise if the library is not built or a
call returns an error status: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqmc.so")

QMC_FP64, QMC_FP32, QMC_BF16_MIXED, QMC_BF16_VALUE = 0, 1, 2, 3
PRECISIONS = {"fp64": QMC_FP64, "fp32": QMC_FP32, "bf16": QMC_BF16_MIXED, "bf16v": QMC_BF16_VALUE}
OP_LOGPSI, OP_LOCAL_ENERGY, OP_METROPOLIS, OP_LOGPSI_VJP, OP_LOSS_GRAD, OP_MALA, OP_LOGPSI_GRAD = range(7)
PLAN_CONCURRENT_SYSTEMS, PLAN_AUTOTUNE = 1, 2


class QmcSystem(ctypes.Structure):
    _fields_ = [("n_nuc", ctypes.c_int32), ("charges", ctypes.POINTER(ctypes.c_double)),
                ("coords", ctypes.POINTER(ctypes.c_double)), ("n_up", ctypes.c_int32),
                ("n_down", ctypes.c_int32)]


class QmcAnsatz(ctypes.Structure):
    _fields_ = [("version", ctypes.c_int32), ("n_rbf", ctypes.c_int32), ("rbf_dmax", ctypes.c_double),
                ("init_layers", ctypes.c_int32), ("width", ctypes.c_int32), ("mp_layers", ctypes.c_int32),
                ("n_det", ctypes.c_int32), ("n_env", ctypes.c_int32), ("include_vnn", ctypes.c_int32),
                ("ee_cusp", ctypes.c_double), ("jastrow", ctypes.c_int32), ("full_det", ctypes.c_int32),
                ("edge_update", ctypes.c_int32)]


_lib = None


def lib():
    """Load libqmc.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, sz, i32, i64, dp = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    L.qmc_param_count.restype = i64
    L.qmc_param_count.argtypes = [ctypes.POINTER(QmcSystem), ctypes.POINTER(QmcAnsatz)]
    L.qmc_plan_create.restype = i32
    L.qmc_plan_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(QmcSystem), i32, ctypes.POINTER(i64),
                                  ctypes.POINTER(QmcAnsatz), i32, ctypes.c_uint32]
    L.qmc_plan_create_ex.restype = i32
    L.qmc_plan_create_ex.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(QmcSystem), i32, ctypes.POINTER(i64),
                                     ctypes.POINTER(QmcAnsatz), i32, ctypes.c_uint32, i64]
    L.qmc_plan_chunk_walkers.restype = i32
    L.qmc_plan_chunk_walkers.argtypes = [vp, i32, ctypes.POINTER(i64)]
    L.qmc_plan_destroy.restype = i32
    L.qmc_plan_destroy.argtypes = [vp]
    L.qmc_workspace_size.restype = i32
    L.qmc_workspace_size.argtypes = [vp, i32, ctypes.POINTER(sz)]
    L.qmc_plan_info.restype = i32
    L.qmc_plan_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.qmc_logpsi.restype = i32
    L.qmc_logpsi.argtypes = [vp, vp, dp, dp, dp, vp, sz, vp]
    L.qmc_local_energy.restype = i32
    L.qmc_local_energy.argtypes = [vp, vp, dp, dp, dp, dp, dp, dp, vp, sz, vp]
    L.qmc_metropolis_step.restype = i32
    L.qmc_metropolis_step.argtypes = [vp, vp, dp, dp, dp, dp, ctypes.c_double, vp, vp, sz, vp]
    L.qmc_logpsi_grad.restype = i32
    L.qmc_logpsi_grad.argtypes = [vp, vp, dp, dp, dp, vp, sz, vp]
    L.qmc_mala_step.restype = i32
    L.qmc_mala_step.argtypes = [vp, vp, dp, dp, dp, dp, dp, ctypes.c_double, i32, vp, vp, sz, vp]
    L.qmc_logpsi_vjp.restype = i32
    L.qmc_logpsi_vjp.argtypes = [vp, vp, dp, dp, vp, vp, sz, vp]
    L.qmc_loss_grad.restype = i32
    L.qmc_loss_grad.argtypes = [vp, vp, dp, dp, vp, dp, vp, sz, vp]
    L.qmc_det_jets.restype = i32
    L.qmc_det_jets.argtypes = [i64, i32, i32, dp, dp, dp, dp, dp, vp]
    L.qmc_sgd_update.restype = i32
    L.qmc_sgd_update.argtypes = [i32, vp, vp, i64, ctypes.c_double, vp]
    L.qmc_measure_peaks.restype = i32
    L.qmc_measure_peaks.argtypes = [vp, sz, ctypes.POINTER(ctypes.c_double), vp]
    L.qmc_profile_enable.restype = i32
    L.qmc_profile_enable.argtypes = [i32]
    L.qmc_profile_report.restype = i32
    L.qmc_profile_report.argtypes = [ctypes.c_char_p, sz, i32]
    L.qmc_plan_tiles.restype = i32
    L.qmc_plan_tiles.argtypes = [vp, i32, ctypes.POINTER(i32)]
    L.qmc_status_str.restype = ctypes.c_char_p
    L.qmc_status_str.argtypes = [i32]
    L.qmc_clip_local_energy.restype = i32
    L.qmc_clip_local_energy.argtypes = [vp, dp, dp, ctypes.c_double, i32, vp]
    L.qmc_last_error.restype = ctypes.c_char_p
    L.qmc_last_error.argtypes = []
    _lib = L
    return L


class QmcError(RuntimeError):
    pass


def _check(status: int, what: str):
    if status != 0:
        msg = f"{what}: {lib().qmc_status_str(status).decode()}"
        if status == 4:  # QMC_ERR_HIP: name the failing launch
            msg += f" ({lib().qmc_last_error().decode()})"
        raise QmcError(msg)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def make_ansatz(ans) -> QmcAnsatz:
    return QmcAnsatz(1, ans.n_rbf, float(ans.rbf_dmax), ans.init_layers, ans.width, ans.mp_layers, ans.n_det,
                     ans.n_env, ans.include_vnn, float(getattr(ans, "ee_cusp", 0.0)),
                     int(getattr(ans, "jastrow", 0)), int(getattr(ans, "full_det", 0)),
                     int(getattr(ans, "edge_update", 0)))


class _SysHolder:
    """Keeps the host arrays of a qmc_system alive while the library copies them."""

    def __init__(self, system):
        Z = [float(z) for z in system.charges]
        R = [float(x) for c in system.coords for x in c]
        self.Z = (ctypes.c_double * len(Z))(*Z)
        self.R = (ctypes.c_double * len(R))(*R)
        self.s = QmcSystem(len(Z), self.Z, self.R, system.n_up, system.n_down)


def param_count(system, ans) -> int:
    h = _SysHolder(system)
    a = make_ansatz(ans)
    return int(lib().qmc_param_count(ctypes.byref(h.s), ctypes.byref(a)))


class Plan:
    """A plan over one or several systems; methods take device tensors.

    concurrent: run every system on its own stream of the plan (fork/join with
    the current stream), so that a multi-system batch shares the device and
    captures into one graph.  autotune: time the GEMM tile candidates of every
    system at creation and keep the fastest.  max_chunk_walkers: process each
    system's walkers in chunks of at most this many (0 = the library's own
    choice)."""

    def __init__(self, systems: Sequence, walkers: Sequence[int], ans, precision: str = "fp64",
                 concurrent: bool = False, autotune: bool = False, max_chunk_walkers: int = 0):
        self.systems = list(systems)
        self.walkers = [int(w) for w in walkers]
        self.ans = ans
        self.precision = precision
        holders = [_SysHolder(s) for s in self.systems]
        arr = (QmcSystem * len(holders))(*[h.s for h in holders])
        wps = (ctypes.c_int64 * len(self.walkers))(*self.walkers)
        a = make_ansatz(ans)
        handle = ctypes.c_void_p(0)
        flags = (PLAN_CONCURRENT_SYSTEMS if concurrent else 0) | (PLAN_AUTOTUNE if autotune else 0)
        _check(lib().qmc_plan_create_ex(ctypes.byref(handle), arr, len(holders), wps, ctypes.byref(a),
                                        PRECISIONS[precision], flags, int(max_chunk_walkers)),
               "qmc_plan_create_ex")
        self.handle = handle
        tw, tp, tpos = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().qmc_plan_info(self.handle, ctypes.byref(tw), ctypes.byref(tp), ctypes.byref(tpos)),
               "qmc_plan_info")
        self.total_walkers, self.total_params, self.total_positions = tw.value, tp.value, tpos.value
        self.param_dtype = torch.float64 if precision == "fp64" else torch.float32
        self._ws = {}

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.qmc_plan_destroy(h)
            self.handle = None

    def tiles(self):
        """Per system: GEMM tile choice of the (jet, value, edge, backward) classes (0 = default)."""
        out = []
        for k in range(len(self.systems)):
            t = (ctypes.c_int32 * 4)()
            _check(lib().qmc_plan_tiles(self.handle, k, t), "qmc_plan_tiles")
            out.append(tuple(int(x) for x in t))
        return out

    def chunk_walkers(self):
        """Per system: walkers per chunk (the last chunk holds the remainder)."""
        out = []
        for k in range(len(self.systems)):
            w = ctypes.c_int64()
            _check(lib().qmc_plan_chunk_walkers(self.handle, k, ctypes.byref(w)), "qmc_plan_chunk_walkers")
            out.append(int(w.value))
        return out

    def workspace_bytes(self, op: int) -> int:
        b = ctypes.c_size_t()
        _check(lib().qmc_workspace_size(self.handle, op, ctypes.byref(b)), "qmc_workspace_size")
        return int(b.value)

    def workspace(self, op: int, device="cuda"):
        """One workspace shared by all operations (calls are ordered on the stream), grown on demand."""
        n = self.workspace_bytes(op)
        ws = self._ws.get("shared")
        if ws is None or ws.numel() < n:
            self._ws.pop("shared", None)
            ws = torch.empty(n, dtype=torch.uint8, device=device)
            self._ws["shared"] = ws
        return ws

    def _check_inputs(self, params, r):
        if params.dtype != self.param_dtype or params.numel() != self.total_params or not params.is_contiguous():
            raise ValueError("params: wrong dtype, size or layout")
        if r.dtype != torch.float64 or r.numel() != self.total_positions or not r.is_contiguous():
            raise ValueError("r: expected contiguous float64 [W][N][3] positions")
        if not (params.is_cuda and r.is_cuda):
            raise ValueError("params and r must be device tensors")

    def logpsi(self, params, r, out=None):
        """(log|psi| [W], sign [W]); out: optional (logpsi, sign) float64 device tensors to write
        (sign may be None)."""
        self._check_inputs(params, r)
        W = self.total_walkers
        if out is None:
            lp = torch.empty(W, dtype=torch.float64, device=r.device)
            sg = torch.empty(W, dtype=torch.float64, device=r.device)
        else:
            lp, sg = out
            if lp.dtype != torch.float64 or lp.numel() != W or not lp.is_contiguous():
                raise ValueError("out logpsi: expected contiguous float64 [W]")
            if sg is not None and (sg.dtype != torch.float64 or sg.numel() != W or not sg.is_contiguous()):
                raise ValueError("out sign: expected contiguous float64 [W]")
        ws = self.workspace(OP_LOGPSI)
        _check(lib().qmc_logpsi(self.handle, _ptr(params), _ptr(r), _ptr(lp), _ptr(sg), _ptr(ws), ws.numel(),
                                _stream()), "qmc_logpsi")
        return lp, sg

    def local_energy(self, params, r, out=None):
        self._check_inputs(params, r)
        W = self.total_walkers
        dev = r.device
        if out is None:
            out = {"logpsi": torch.empty(W, dtype=torch.float64, device=dev),
                   "sign": torch.empty(W, dtype=torch.float64, device=dev),
                   "grad": torch.empty(self.total_positions, dtype=torch.float64, device=dev),
                   "lap": torch.empty(W, dtype=torch.float64, device=dev),
                   "e_loc": torch.empty(W, dtype=torch.float64, device=dev)}
        ws = self.workspace(OP_LOCAL_ENERGY)
        _check(lib().qmc_local_energy(self.handle, _ptr(params), _ptr(r), _ptr(out.get("logpsi")),
                                      _ptr(out.get("sign")), _ptr(out.get("grad")), _ptr(out.get("lap")),
                                      _ptr(out["e_loc"]), _ptr(ws), ws.numel(), _stream()), "qmc_local_energy")
        return out

    def metropolis_step(self, params, r, logpsi, noise, u, step, accepted=None):
        """In place on r and logpsi; returns the uint8 acceptance flags."""
        self._check_inputs(params, r)
        W = self.total_walkers
        if noise.dtype != torch.float64 or noise.numel() != self.total_positions or not noise.is_contiguous():
            raise ValueError("noise: expected float64 like r")
        if u.dtype != torch.float64 or u.numel() != W or logpsi.dtype != torch.float64 or logpsi.numel() != W:
            raise ValueError("u/logpsi: expected float64 [W]")
        if accepted is None:
            accepted = torch.empty(W, dtype=torch.uint8, device=r.device)
        ws = self.workspace(OP_METROPOLIS)
        _check(lib().qmc_metropolis_step(self.handle, _ptr(params), _ptr(r), _ptr(logpsi), _ptr(noise), _ptr(u),
                                         float(step), _ptr(accepted), _ptr(ws), ws.numel(), _stream()),
               "qmc_metropolis_step")
        return accepted

    def logpsi_grad(self, params, r):
        """log|psi| [W] and its gradient over the positions [W*N*3] by one reverse pass (no Laplacian)."""
        self._check_inputs(params, r)
        lp = torch.empty(self.total_walkers, dtype=torch.float64, device=r.device)
        g = torch.empty(self.total_positions, dtype=torch.float64, device=r.device)
        ws = self.workspace(OP_LOGPSI_GRAD)
        _check(lib().qmc_logpsi_grad(self.handle, _ptr(params), _ptr(r), _ptr(lp), _ptr(g), _ptr(ws), ws.numel(),
                                     _stream()), "qmc_logpsi_grad")
        return lp, g

    def mala_step(self, params, r, logpsi, grad, noise, u, step, damp=True, accepted=None):
        """One Langevin step, in place on r, logpsi and grad (grad log|psi| of the current state, e.g.
        local_energy(...)["grad"]); returns the uint8 acceptance flags."""
        self._check_inputs(params, r)
        W = self.total_walkers
        for name, t in (("noise", noise), ("grad", grad)):
            if t.dtype != torch.float64 or t.numel() != self.total_positions or not t.is_contiguous():
                raise ValueError(f"{name}: expected contiguous float64 like r")
        if u.dtype != torch.float64 or u.numel() != W or logpsi.dtype != torch.float64 or logpsi.numel() != W:
            raise ValueError("u/logpsi: expected float64 [W]")
        if accepted is None:
            accepted = torch.empty(W, dtype=torch.uint8, device=r.device)
        ws = self.workspace(OP_MALA)
        _check(lib().qmc_mala_step(self.handle, _ptr(params), _ptr(r), _ptr(logpsi), _ptr(grad), _ptr(noise),
                                   _ptr(u), float(step), int(bool(damp)), _ptr(accepted), _ptr(ws), ws.numel(),
                                   _stream()), "qmc_mala_step")
        return accepted

    def clip_local_energy(self, e_loc, width=5.0, mode="hard", out=None):
        """Clipped local energies for the loss gradient (per system: median-centred window of half-width
        width x mean absolute deviation); mode "hard" or "soft" (logarithmic)."""
        if e_loc.dtype != torch.float64 or e_loc.numel() != self.total_walkers or not e_loc.is_contiguous():
            raise ValueError("e_loc: expected contiguous float64 [W]")
        out = torch.empty_like(e_loc) if out is None else out
        if out.dtype != torch.float64 or out.numel() != self.total_walkers or not out.is_contiguous():
            raise ValueError("out: expected contiguous float64 [W]")
        _check(lib().qmc_clip_local_energy(self.handle, _ptr(e_loc), _ptr(out), float(width),
                                           {"hard": 0, "soft": 1}[mode], _stream()), "qmc_clip_local_energy")
        return out

    def logpsi_vjp(self, params, r, cotangent):
        self._check_inputs(params, r)
        g = torch.empty_like(params)
        ws = self.workspace(OP_LOGPSI_VJP)
        _check(lib().qmc_logpsi_vjp(self.handle, _ptr(params), _ptr(r), _ptr(cotangent), _ptr(g), _ptr(ws),
                                    ws.numel(), _stream()), "qmc_logpsi_vjp")
        return g

    def loss_grad(self, params, r, e_loc, grad=None, e_mean=None):
        self._check_inputs(params, r)
        g = torch.empty_like(params) if grad is None else grad
        em = torch.empty(len(self.systems), dtype=torch.float64, device=r.device) if e_mean is None else e_mean
        if g.dtype != params.dtype or g.numel() != params.numel() or em.numel() != len(self.systems):
            raise ValueError("grad / e_mean: wrong dtype or size")
        ws = self.workspace(OP_LOSS_GRAD)
        _check(lib().qmc_loss_grad(self.handle, _ptr(params), _ptr(r), _ptr(e_loc), _ptr(g), _ptr(em), _ptr(ws),
                                   ws.numel(), _stream()), "qmc_loss_grad")
        return g, em

    def loss_grad_finite_counts(self):
        """Per system, the number of walkers with a finite local energy that entered the last loss
        gradient (the workspace header written by qmc_loss_grad; read after that call)."""
        ws = self._ws["shared"]
        return ws[:8 * len(self.systems)].view(torch.int64).cpu().tolist()

    def sgd_update(self, params, grad, lr: float):
        """params -= lr * grad on the device (the optimizer step of a training iteration)."""
        if params.dtype != self.param_dtype or params.numel() != self.total_params or not params.is_contiguous():
            raise ValueError("params: wrong dtype, size or layout")
        if grad.dtype != params.dtype or grad.numel() != params.numel() or not grad.is_contiguous():
            raise ValueError("grad: wrong dtype or size")
        if not (params.is_cuda and grad.is_cuda):
            raise ValueError("params and grad must be device tensors")
        _check(lib().qmc_sgd_update(PRECISIONS[self.precision], _ptr(params), _ptr(grad), params.numel(), float(lr),
                                    _stream()), "qmc_sgd_update")


class GraphStep:
    """Local energies and the loss gradient of a plan captured into one graph.

    Inputs (params, r) and outputs (self.out: logpsi, sign, grad, lap, e_loc,
    param_grad, e_mean) are static tensors; write new positions into r and call
    replay().  With a concurrent plan the graph holds one branch per system."""

    def __init__(self, plan: Plan, params, r, warmup: int = 1):
        self.plan, self.params, self.r = plan, params, r
        W, dev = plan.total_walkers, r.device
        self.out = {"logpsi": torch.empty(W, dtype=torch.float64, device=dev),
                    "sign": torch.empty(W, dtype=torch.float64, device=dev),
                    "grad": torch.empty(plan.total_positions, dtype=torch.float64, device=dev),
                    "lap": torch.empty(W, dtype=torch.float64, device=dev),
                    "e_loc": torch.empty(W, dtype=torch.float64, device=dev),
                    "param_grad": torch.empty_like(params),
                    "e_mean": torch.empty(len(plan.systems), dtype=torch.float64, device=dev)}
        # workspaces are allocated by the warm-up, outside the capture
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(warmup):
                self._body()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._body()

    def _body(self):
        o = self.out
        self.plan.local_energy(self.params, self.r, out=o)
        self.plan.loss_grad(self.params, self.r, o["e_loc"], grad=o["param_grad"], e_mean=o["e_mean"])

    def replay(self):
        self.graph.replay()


def det_jets(jets, n: int, n_tan: int):
    """Determinant stage on given matrix jets [n_mat][n_tan+2][n][n] (float64 device)."""
    if jets.dtype != torch.float64 or not jets.is_contiguous() or not jets.is_cuda:
        raise ValueError("jets: expected contiguous float64 device tensor")
    nmat = jets.numel() // ((n_tan + 2) * n * n)
    dev = jets.device
    ld = torch.empty(nmat, dtype=torch.float64, device=dev)
    sg = torch.empty(nmat, dtype=torch.float64, device=dev)
    g = torch.empty(max(nmat * n_tan, 1), dtype=torch.float64, device=dev)
    lap = torch.empty(nmat, dtype=torch.float64, device=dev)
    _check(lib().qmc_det_jets(nmat, n, n_tan, _ptr(jets), _ptr(ld), _ptr(sg), _ptr(g), _ptr(lap), _stream()),
           "qmc_det_jets")
    return ld, sg, g[:nmat * n_tan].reshape(nmat, n_tan), lap


def measure_peaks(scratch_bytes: int = 1 << 30) -> dict:
    """Achievable device peaks from qmc_measure_peaks, on a scratch tensor allocated here:
    {"fp32_mfma", "bf16_mfma", "fp64_mfma"} in TFLOP/s and "copy" in GB/s (read + write)."""
    buf = torch.empty(scratch_bytes // 4, dtype=torch.float32, device="cuda")
    out = (ctypes.c_double * 4)()
    _check(lib().qmc_measure_peaks(_ptr(buf), buf.numel() * 4, out, _stream()), "qmc_measure_peaks")
    del buf
    return {"fp32_mfma": out[0], "bf16_mfma": out[1], "fp64_mfma": out[2], "copy": out[3]}


def profile_enable(on: bool = True):
    """Time every kernel launch with HIP events on its own stream."""
    _check(lib().qmc_profile_enable(1 if on else 0), "qmc_profile_enable")


def profile_report(reset: bool = True):
    """{kernel name: (launches, total ms)} for the launches recorded since the last reset."""
    buf = ctypes.create_string_buffer(1 << 16)
    _check(lib().qmc_profile_report(buf, len(buf), 1 if reset else 0), "qmc_profile_report")
    out = {}
    for line in buf.value.decode().splitlines():
        name, n, ms = line.rsplit(" ", 2)
        out[name] = (int(n), float(ms))
    return out


class LogPsi(torch.autograd.Function):
    """log|psi| of every walker as a differentiable function of the parameters.

    Forward: qmc_logpsi.  Backward: the hand-written vector-Jacobian product
    qmc_logpsi_vjp (positions get no gradient)."""

    @staticmethod
    def forward(ctx, params, r, plan):
        lp, _ = plan.logpsi(params, r)
        ctx.plan = plan
        ctx.save_for_backward(params, r)
        return lp

    @staticmethod
    def backward(ctx, g):
        params, r = ctx.saved_tensors
        grad = ctx.plan.logpsi_vjp(params, r, g.to(torch.float64).contiguous())
        return grad, None, None


def logpsi_autograd(plan, params, r):
    return LogPsi.apply(params, r, plan)
