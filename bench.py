"""Benchmark of the VMC hot path on one MI355X.

One step = one VMC training iteration over one batch of walkers: 10
random-walk Metropolis steps (each a full log|psi| evaluation of the
proposals), the local energy with exact gradient and Laplacian, clipping of
the local energies, the loss gradient, the gradient-descent update of the
parameters, and log|psi| of the walkers under the updated parameters (the
state the next iteration's Metropolis steps compare against).  Workload: the N2-sized system (two
Z=7 nuclei 2.068 bohr apart, 7 up + 7 down electrons, 4096 walkers, 4
message-passing layers of width 128, 16 determinants, 8 envelope exponents),
float32 jets with float64 determinants.  Inputs are seeded, synthetic and
resident on the GPU before the timed region.

The step is captured into one HIP graph after the warm-up steps; the timed
region replays it K times between HIP events on the launch stream.  An eager
pass over the same K steps, with HIP events around every launch, gives the
per-kernel times and the roofline of the dominant kernel.

Prints one JSON line.  `value` = walkers passed through the whole step per
second; the local-energy-only rate, the error of E_L against the FP64 oracle
(on the seeded network, restored after the timed steps), the roofline of the
dominant kernel, the measured device peaks and the oracle's own throughput on
the host cores are reported beside it.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp32_mfma": 157.3e12, "fp64_mfma": 78.6e12, "bf16_mfma": 2.5e15, "hbm": 8.0e12,
        # float32 exponentials: 256 compute units x 4 SIMDs x 4 lanes per clock (quarter rate) x 2.4 GHz
        "exp_f32": 256 * 4 * 4 * 2.4e9}


def algorithmic_model(s, a, elem_bytes, n_mc, with_grad, fused_edges):
    """Algorithmic work of one bench step per kernel family (FLOP or bytes summed
    over all launches of that family in the step), without padding rows or
    structurally zero rows.

    Jets carry R1 = 3N + 2 rows per electron (value, 3N tangents, Laplacian);
    edge filters carry 3 rows per pair (value, first and second derivative).
    fused_edges: the edge filters run in edge_mlp_kernel (float32, width 128)
    instead of two GEMM launches each."""
    N, M, K, D, L, L0, nd = s.n_elec, s.n_nuc, a.n_rbf, a.width, a.mp_layers, a.init_layers, a.n_det
    T = 3 * N
    R1 = T + 2
    Rj = N * R1
    P = [s.n_up * (s.n_up - 1) // 2 + s.n_down * (s.n_down - 1) // 2, s.n_up * s.n_down, N * M]
    nsq = s.n_up ** 2 + s.n_down ** 2
    eb = elem_bytes
    # forward with jets (local energy)
    # h and the electron-message part of g over all jet rows; the nuclear message has 5 nonzero
    # jet rows per electron (value, own coordinates, Laplacian)
    node_jet = (2 * Rj * ((M + 2) * K * D + (L0 - 1) * D * D) + L * 2 * Rj * 3 * D * D + L * 2 * N * 5 * D * D
                + 2 * R1 * D * nd * nsq)
    edge_jet = L * sum(P) * 3 * 2 * (K * D + D * D)
    # value rows: one log|psi| (Metropolis proposal, stashed forward of the backward)
    node_val = 2 * N * ((M + 2) * K * D + (L0 - 1) * D * D) + L * 2 * N * 4 * D * D + 2 * D * nd * nsq
    edge_val = L * sum(P) * 2 * (K * D + D * D)
    # data cotangents of the backward (x_bar = y_bar W^T), weight gradients (W_bar = x^T y_bar)
    val_bwd = 2 * D * nd * nsq + L * (2 * N * 3 * D * D + 2 * N * D * D + sum(P) * 2 * D * D) + (L0 - 1) * 2 * N * D * D
    wgrad = node_val + edge_val
    # value forwards per step: the Metropolis proposals, the loss gradient's stashed forward and, after
    # the parameter update, log|psi| of the walkers under the new parameters
    n_val = n_mc + (2 if with_grad else 0)
    m = {
        "gemm_kernel<jet>": ("mfma", node_jet),
        "gemm_kernel<val>": ("mfma", n_val * node_val + (0 if fused_edges else n_val * edge_val)
                             + (val_bwd if with_grad else 0)),
        "wgrad_kernel": ("mfma", wgrad if with_grad else 0),
        # HBM-bound kernels: bytes of jets read and written
        "aggregate_kernel": ("hbm", L * eb * (N * R1 * D + N * R1 * 2 * D + (P[0] + P[1]) * 3 * D)),
        "det_kernel<jet>": ("hbm", eb * nd * R1 * nsq + 8 * 2 * nd * (T + 3)),
        "envelope_kernel<jet>": ("hbm", 2 * eb * nd * R1 * nsq),
    }
    if eb == 4:
        # value rows: one exponential per (electron, orbital, nucleus, exponent) and log|psi|
        m["envelope_kernel<val>"] = ("alu", n_val * nd * nsq * M * a.n_env)
    if fused_edges:
        m["edge_mlp_kernel<jet>"] = ("mfma", edge_jet)
        m["edge_mlp_kernel<val>"] = ("mfma", n_val * edge_val)
    else:
        m["gemm_kernel<edge>"] = ("mfma", edge_jet)
    return m


# source file of each kernel family (a stored traffic measurement is used only while it is unchanged)
FAMILY_SOURCE = {"gemm_kernel": "gemm.hip", "edge_mlp_kernel": "edge.hip", "aggregate_kernel": "ops.hip",
                 "det_kernel": "ops.hip", "envelope_kernel": "ops.hip", "wgrad_kernel": "backward.hip"}


def stored_traffic(family, workload, precision):
    """HBM bytes per launch of a kernel family from a committed counter summary
    (profiles/traffic_<family>_<workload>_<precision>.txt, FETCH_SIZE and
    WRITE_SIZE scaled by a plain copy of known size), or None when there is none
    or the family's source changed since the counters were taken."""
    import hashlib
    tag = family.replace("<", "_").replace(">", "")
    path = os.path.join(ROOT, "profiles", f"traffic_{tag}_{workload}_{precision}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    src = os.path.join(ROOT, "paper_2307_14123_amd", "csrc", FAMILY_SOURCE.get(family.split("<")[0], ""))
    if not os.path.isfile(src) or kv.get("source_sha256") != hashlib.sha256(open(src, "rb").read()).hexdigest():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def dist(ms):
    """median, p10 and p90 of per-repetition times (ms) from HIP events on the launch stream"""
    v = np.asarray(ms, dtype=np.float64)
    return {"median": float(np.median(v)), "p10": float(np.percentile(v, 10)), "p90": float(np.percentile(v, 90)),
            "n": int(v.size)}


def environment():
    """GPU name, ROCm and driver versions, and the clock / power state rocm-smi reports."""
    import subprocess
    import torch
    env = {"gpu": torch.cuda.get_device_name(0), "torch": torch.__version__}
    for key, path in (("rocm", "/opt/rocm/.info/version"), ("amdgpu_driver", "/sys/module/amdgpu/version")):
        try:
            with open(path) as f:
                env[key] = f.read().strip()
        except OSError:
            pass
    # rocm-smi is a script started through env: skip it under a profiler, whose preloaded library would
    # make that hop an exec of a process holding the GPU
    if "rocprof" in os.environ.get("LD_PRELOAD", "") or any(k.startswith("ROCPROF") for k in os.environ):
        env["rocm_smi"] = "skipped under a profiler"
        return env
    try:
        res = subprocess.run(["rocm-smi", "--showclocks", "--showpower"], capture_output=True, text=True, timeout=30)
        keep = [ln.strip() for ln in res.stdout.splitlines()
                if any(t in ln for t in ("sclk", "mclk", "fclk", "Power", "power")) and "====" not in ln]
        env["rocm_smi"] = keep[:12]
    except (OSError, subprocess.SubprocessError):
        pass
    return env


def kernel_family(name):
    if name.startswith("gemm_kernel"):
        return "gemm_kernel<" + name.rstrip(">").split(",")[-1] + ">"
    if name.startswith("wgrad_kernel"):
        return "wgrad_kernel"
    return name


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="n2", choices=["n2", "c4h4", "h2", "batched", "scaling", "precision"],
                    help="n2: the headline workload; c4h4 / h2: the precision and small FP64 systems; "
                         "batched: 16 molecules (4-42 electrons) in one graph vs per-molecule launches; "
                         "scaling: train-step time of atoms and hydrogen chains up to 45 electrons; "
                         "precision: C4H4-sized local energies in the fp32, bf16v and bf16 plans against the "
                         "oracle on --cpu-walkers walkers (64 by default)")
    ap.add_argument("--walkers", type=int, default=None)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64", "bf16", "bf16v"],
                    help="bf16v: bf16 operands in the value-row forwards only (local-energy jets in float32)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-walkers", type=int, default=None,
                    help="oracle sample size (160 for n2, 64 for precision)")
    ap.add_argument("--jastrow", action="store_true", help="add the learnable Jastrow factor to the ansatz")
    ap.add_argument("--ee-cusp", type=float, default=0.0, help="alpha of the electron-electron cusp factor (0: none)")
    ap.add_argument("--full-det", action="store_true", help="one N x N determinant per p over both spins")
    ap.add_argument("--edge-update", action="store_true",
                    help="update the edge features in every interaction layer after the first")
    ap.add_argument("--no-sub-records", action="store_true",
                    help="skip the fp64_form / c4h4 / batched sub-records of the default n2 line")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with a plain 256 MiB device copy, the reference for traffic counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (walkers would be sharded "
              "across GPUs with one all-reduce of the loss gradient).", file=sys.stderr)
        sys.exit(2)

    import torch
    import qmc_inputs as qi
    from paper_2307_14123_amd import qmc

    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "scaling":
        return bench_scaling(args)
    if args.workload == "precision":
        return bench_precision(args)
    k = {"n2": 1, "c4h4": 3, "h2": 0}[args.workload]
    wl = qi.workload(k)
    s, a = wl.systems[0], wl.ansatz
    if args.jastrow or args.ee_cusp > 0 or args.full_det or args.edge_update:
        import dataclasses
        a = dataclasses.replace(a, jastrow=int(args.jastrow), ee_cusp=float(args.ee_cusp), full_det=int(args.full_det),
                                edge_update=int(args.edge_update))
    W = args.walkers or wl.walkers
    n_mc, tau = 10, 0.2
    params = qi.make_params(s, a, qi.seed(k, 0))
    r0 = qi.make_walkers(s, W, qi.seed(k, 1))
    noise = qi.make_noise(n_mc, W, s.n_elec, qi.seed(k, 2))
    uni = qi.make_uniforms(n_mc, W, qi.seed(k, 3))

    dev = torch.device("cuda", 0)
    # GEMM tiles chosen by timing the candidates on the device at plan creation (outside the timed region)
    plan = qmc.Plan([s], [W], a, args.precision, autotune=True)
    P = torch.as_tensor(params, dtype=plan.param_dtype, device=dev).contiguous()
    R = torch.as_tensor(r0, device=dev).contiguous()
    NOISE = torch.as_tensor(noise, device=dev).contiguous()
    U = torch.as_tensor(uni, device=dev).contiguous()
    lp, _ = plan.logpsi(P, R)
    out = {"logpsi": torch.empty(W, dtype=torch.float64, device=dev),
           "sign": torch.empty(W, dtype=torch.float64, device=dev),
           "grad": torch.empty(W * s.n_elec * 3, dtype=torch.float64, device=dev),
           "lap": torch.empty(W, dtype=torch.float64, device=dev),
           "e_loc": torch.empty(W, dtype=torch.float64, device=dev)}
    acc = torch.empty(W, dtype=torch.uint8, device=dev)
    for op in (qmc.OP_LOGPSI, qmc.OP_LOCAL_ENERGY, qmc.OP_METROPOLIS, qmc.OP_MALA):
        plan.workspace(op)  # the shared workspace reaches its size before any capture
    has_grad = True
    try:
        plan.loss_grad(P, R, out["e_loc"])
    except qmc.QmcError:
        has_grad = False
    torch.cuda.synchronize()

    G = torch.empty_like(P)
    EM = torch.empty(1, dtype=torch.float64, device=dev)
    EC = torch.empty(W, dtype=torch.float64, device=dev)  # clipped local energies for the gradient
    clip_width = 5.0
    P_init = P.clone()  # the seeded network, restored after the timed steps have updated it
    # plain gradient descent; its cost does not depend on lr, kept small so that the network stays near its
    # seeded initialisation over the warm-up and timed steps
    lr = 1e-8

    def step():
        for t in range(n_mc):
            plan.metropolis_step(P, R, lp, NOISE[t], U[t], tau, accepted=acc)
        plan.local_energy(P, R, out=out)
        if has_grad:
            plan.clip_local_energy(out["e_loc"], clip_width, "hard", out=EC)
            plan.loss_grad(P, R, EC, grad=G, e_mean=EM)
            plan.sgd_update(P, G, lr)
            # the sampler follows psi under the updated parameters: the next step's Metropolis
            # comparisons need log|psi| of the current walkers under them
            plan.logpsi(P, R, out=(lp, None))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # The whole step captured into one HIP graph: the same kernels in the same order, without the
    # gaps between launches.  Falls back to eager steps if capture fails.
    graph, graph_err = None, None
    try:
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            step()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            step()
        g.replay()  # untimed
        torch.cuda.synchronize()
        graph = g
    except Exception as e:  # noqa: BLE001 - reported in the bench line
        graph_err = repr(e)[:200]

    def timed(run, n):
        """n repetitions of run() between HIP events on the launch stream; (wall ms per rep, event ms list)"""
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(n + 1)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev[0].record()
        for i in range(n):
            run()
            ev[i + 1].record()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / n, [ev[i].elapsed_time(ev[i + 1]) for i in range(n)]

    # timed region: K steps (graph replays when captured)
    ms_step, step_ms = timed(graph.replay if graph is not None else step, args.steps)
    # the same K steps eagerly with HIP events around every launch: per-kernel times and rooflines
    qmc.profile_enable(True)
    qmc.profile_report(reset=True)
    ms_eager, eager_ms = timed(step, args.steps)
    prof = qmc.profile_report(reset=True)
    qmc.profile_enable(False)
    P.copy_(P_init)
    torch.cuda.synchronize()

    # local energy alone (one graph per evaluation when it captures): at least 50 repetitions or 1 s
    # (at most 60), each between two HIP events
    def le_eager():
        plan.local_energy(P, R, out=out)

    le_run = le_eager
    if graph is not None:
        try:
            gl = torch.cuda.CUDAGraph()
            with torch.cuda.graph(gl):
                le_eager()
            gl.replay()
            torch.cuda.synchronize()
            le_run = gl.replay
        except Exception:  # noqa: BLE001 - eager local energies then
            le_run = le_eager
    est, _ = timed(le_run, 1)
    reps = int(min(60, max(50 if est < 20 else 1, args.steps, math.ceil(1000.0 / max(est, 1e-3)))))
    ms_le, le_ms = timed(le_run, reps)

    # Langevin steps alone (the gradient-informed sampler), from the state the local energy left:
    # drift proposal, jet forward at the proposal (log|psi| and its gradient), Hastings acceptance;
    # n_mc steps per repetition with the step's noise streams
    mala_eps = 0.1
    Rm, LPm, Gm = R.clone(), out["logpsi"].clone(), out["grad"].clone()
    ACCm = torch.empty((n_mc, W), dtype=torch.uint8, device=dev)

    def mala_eager():
        for t in range(n_mc):
            plan.mala_step(P, Rm, LPm, Gm, NOISE[t], U[t], mala_eps, accepted=ACCm[t])

    mala_eager()
    torch.cuda.synchronize()
    mala_run, mala_launch = mala_eager, "eager"
    if graph is not None:
        try:
            gm = torch.cuda.CUDAGraph()
            with torch.cuda.graph(gm):
                mala_eager()
            gm.replay()
            torch.cuda.synchronize()
            mala_run, mala_launch = gm.replay, f"one HIP graph per {n_mc} steps"
        except Exception:  # noqa: BLE001 - eager steps then
            pass
    ms_mala, mala_ms = timed(mala_run, 3)
    mala_acc = float(ACCm.double().mean().item())

    # Metropolis steps alone, for the comparison with the Langevin step (same walkers, same count)
    Rq, LPq = R.clone(), out["logpsi"].clone()

    def metro_eager():
        for t in range(n_mc):
            plan.metropolis_step(P, Rq, LPq, NOISE[t], U[t], tau, accepted=ACCm[t])

    metro_eager()
    torch.cuda.synchronize()
    metro_run = metro_eager
    if graph is not None:
        try:
            gq = torch.cuda.CUDAGraph()
            with torch.cuda.graph(gq):
                metro_eager()
            gq.replay()
            torch.cuda.synchronize()
            metro_run = gq.replay
        except Exception:  # noqa: BLE001 - eager steps then
            pass
    ms_metro, _ = timed(metro_run, 3)
    peaks = qmc.measure_peaks()

    eb = 8 if args.precision == "fp64" else 4
    fused = args.precision == "fp32" and a.width in (128, 256) and a.n_rbf <= 16
    model = algorithmic_model(s, a, eb, n_mc, has_grad, fused)
    fam = {}
    for k, (nl, ms) in prof.items():
        f = kernel_family(k)
        n0, m0 = fam.get(f, (0, 0.0))
        fam[f] = (n0 + nl, m0 + ms)
    # dominant kernel family by total time in the timed region
    name, (nl, tot_ms) = max(fam.items(), key=lambda kv: kv[1][1])
    gemm_dtype = {"fp32": "fp32_mfma", "fp64": "fp64_mfma", "bf16": "bf16_mfma", "bf16v": "fp32_mfma"}[args.precision]
    roof = None
    if name in model:
        bound, work_per_walker = model[name]
        per_launch = work_per_walker * W * args.steps / nl
        avg_s = tot_ms / nl * 1e-3
        if bound == "mfma":
            pk = PEAK["fp32_mfma"] if (name == "gemm_kernel<val>" or name == "wgrad_kernel") and args.precision == "bf16" \
                else PEAK[gemm_dtype]
            roof = {"bound": "mfma", "achieved": per_launch / avg_s / 1e12, "peak": pk / 1e12, "unit": "TFLOP/s"}
        elif bound == "alu":
            roof = {"bound": "alu", "achieved": per_launch / avg_s / 1e9, "peak": PEAK["exp_f32"] / 1e9,
                    "unit": "Gexp/s"}
        else:
            roof = {"bound": "hbm", "achieved": per_launch / avg_s / 1e9, "peak": PEAK["hbm"] / 1e9, "unit": "GB/s"}
        roof["frac"] = roof["achieved"] / roof["peak"]
        roof["traffic"] = stored_traffic(name, args.workload, args.precision)
        mkey = {"mfma": gemm_dtype if roof["peak"] == PEAK[gemm_dtype] / 1e12 else "fp32_mfma", "hbm": "copy"}
        pm = peaks.get(mkey.get(bound, ""))
        if pm:
            roof["peak_measured"] = pm
            roof["frac_measured"] = roof["achieved"] / pm
        roof["kernel"] = name
        roof["launches_per_step"] = nl / args.steps
        roof["avg_launch_ms"] = tot_ms / nl
    others = {}
    for f, (n1, ms1) in fam.items():
        if f in model and model[f][1] > 0:
            bound, wpw = model[f]
            per = wpw * W * args.steps / (ms1 * 1e-3)
            others[f] = {"bound": bound, "achieved": per / (1e12 if bound == "mfma" else 1e9),
                         "unit": {"mfma": "TFLOP/s", "alu": "Gexp/s"}.get(bound, "GB/s"),
                         "ms_per_step": ms1 / args.steps}

    res = {
        "metric": "walker local energies/sec at stated mHa error vs FP64 oracle; VMC train step ms",
        "value": W / (ms_step * 1e-3),
        "unit": "walkers/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32+f64", "fp64": "f64", "bf16": "bf16+f32+f64", "bf16v": "bf16+f32+f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": {"n2": "N2-sized: 2 x Z=7 at 2.068 bohr, 7 up + 7 down",
                                "c4h4": "C4H4-sized: 4 C + 4 H, 14 up + 14 down",
                                "h2": "H2: 2 x Z=1 at 1.4 bohr, 1 up + 1 down"}[args.workload] + f", {W} walkers, "
                               f"{a.mp_layers} message-passing layers width {a.width}, {a.n_det} dets, "
                               f"{a.n_env} envelope exponents"
                               + (", learnable Jastrow" if a.jastrow else "")
                               + (f", e-e cusp factor alpha {a.ee_cusp}" if a.ee_cusp > 0 else "")
                               + (", full determinants" if a.full_det else "")
                               + (", edge-feature updates" if a.edge_update else "")
                               + f"; step = {n_mc} Metropolis steps (tau {tau}) + "
                               f"local energy" + (" + clipping (median +- 5 mean absolute deviations) + loss "
                                                  "gradient + gradient-descent update (lr 1e-8) + log|psi| under "
                                                  "the updated parameters" if has_grad else ""),
                   "walkers": W, "electrons": s.n_elec, "precision": args.precision, "tiles": plan.tiles()[0],
                   "chunk_walkers": plan.chunk_walkers()[0],
                   "loss_gradient_in_step": has_grad,
                   "step_vs_plain_definition": ("adds clipping of the local energies before the loss gradient "
                                                "(0.13 ms) and the log|psi| refresh after the update (one value "
                                                "forward) to 10 Metropolis steps + local energy + loss gradient "
                                                "+ update" if has_grad else "no loss gradient")},
        "e_loc_per_s": W / (ms_le * 1e-3),
        "e_loc_ms": ms_le,
        "step_ms_events": dist(step_ms),
        "step_launch": "one HIP graph per step" if graph is not None else f"eager (graph capture failed: {graph_err})",
        "step_ms_eager_events": dist(eager_ms),
        "kernel_timing": "HIP events around every launch, in an eager pass over the same steps",
        "e_loc_ms_events": dist(le_ms),
        "mala_step": {"ms": ms_mala / n_mc, "walkers_per_s": W * n_mc / (ms_mala * 1e-3),
                      "events_ms_per_repetition": dist(mala_ms), "steps_per_repetition": n_mc,
                      "launch": mala_launch, "step_size": mala_eps, "damped_drift": True,
                      "acceptance_last_repetition": mala_acc,
                      "metropolis_step_ms": ms_metro / n_mc},
        "roofline": roof,
        "measured_peaks": {"fp32_mfma_tflops": peaks["fp32_mfma"], "bf16_mfma_tflops": peaks["bf16_mfma"],
                           "fp64_mfma_tflops": peaks["fp64_mfma"], "copy_gbs": peaks["copy"]},
        "env": environment(),
        "kernel_rooflines": others,
        "kernels_ms_per_step": {k: round(v[1] / args.steps, 3) for k, v in sorted(prof.items(), key=lambda kv: -kv[1][1])},
    }

    if not args.no_cpu_baseline:
        import oracle
        torch.set_num_threads(os.cpu_count() or 1)
        nw = min(args.cpu_walkers or 160, W) if args.workload == "n2" else min(8, W)
        pc = P_init.double().cpu().numpy()

        def cpu_step(nw_):
            """the step on the first nw_ walkers with the float64 oracle; (positions, E_L dict, part times)"""
            rs_ = r0[:nw_].copy()
            t = [time.perf_counter()]
            lp_c = oracle.logpsi_np(rs_, pc, s, a)[1]
            for tt in range(n_mc):
                rs_, lp_c, _, _ = oracle.metropolis_step(rs_, lp_c, noise[tt, :nw_], uni[tt, :nw_], tau, pc, s, a)
            t.append(time.perf_counter())
            ref_ = oracle.local_energy(rs_, pc, s, a, chunk=16)
            t.append(time.perf_counter())
            if has_grad:
                gc = oracle.loss_grad(rs_, oracle.clip_local_energy(ref_["e_loc"], clip_width, "hard"), pc, s, a)[0]
                _ = pc - lr * gc  # the gradient-descent update of the step
            t.append(time.perf_counter())
            return rs_, ref_, [t[1] - t[0], t[2] - t[1], t[3] - t[2]]

        rs, ref, parts = cpu_step(nw)
        tc = sum(parts)
        try:
            with open("/proc/cpuinfo") as f:
                cpu_model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), None)
        except OSError:
            cpu_model = None
        res["cpu_baseline"] = {"value": nw / tc, "unit": "walkers/s", "cores": torch.get_num_threads(),
                               "kind": "oracle",
                               "sample": f"{nw} of the {W} walkers through the same step (float64 CPU oracle: "
                                         f"serial autograd Laplacian), {tc:.1f} s",
                               "cpu_model": cpu_model, "os_cpu_count": os.cpu_count(),
                               "e_loc_per_s": nw / parts[1], "metropolis_10_steps_s": parts[0],
                               "loss_grad_s": parts[2]}
        # the same oracle on one thread, on a smaller sample
        torch.set_num_threads(1)
        n1 = min(8, nw)
        _, _, parts1 = cpu_step(n1)
        torch.set_num_threads(os.cpu_count() or 1)
        res["cpu_baseline_1thread"] = {"value": n1 / sum(parts1), "unit": "walkers/s", "cores": 1,
                                       "e_loc_per_s": n1 / parts1[1],
                                       "sample": f"{n1} walkers, {sum(parts1):.1f} s"}
        # error of the GPU local energy on the same sample positions, from the timed (autotuned) plan
        # itself: the sample is written into the first walkers of the full batch
        R.view(W, s.n_elec, 3)[:nw] = torch.as_tensor(rs, device=dev)
        plan.local_energy(P, R, out=out)
        torch.cuda.synchronize()
        err = np.abs(out["e_loc"][:nw].cpu().numpy() - ref["e_loc"]) * 1e3
        res["e_loc_err_mha_vs_fp64_oracle"] = {"p50": float(np.median(err)), "p99": float(np.percentile(err, 99)),
                                               "max": float(err.max()), "walkers": nw,
                                               "plan": f"the timed plan ({W} walkers, tiles {plan.tiles()[0]}), "
                                                       f"sample in its first {nw} walkers"}
    if args.workload == "n2" and args.precision == "fp32" and not args.no_sub_records and not (
            a.jastrow or a.ee_cusp > 0 or a.full_det or a.edge_update):
        # the comparison forms, each with its own plan, freed before the next
        del plan
        plan = None
        torch.cuda.empty_cache()
        res["fp64_form"] = fp64_form_record(s, a, W, params, r0, dev)
        torch.cuda.empty_cache()
        res["c4h4"] = c4h4_record(dev, with_oracle=not args.no_cpu_baseline)
        torch.cuda.empty_cache()
        res["batched"] = batched_record(qi.workload(4).walkers, "fp32", 2, 1, dev)
        torch.cuda.empty_cache()
    if args.copy_calibration:
        x = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
    print(json.dumps(res))


def _event_reps(fn, reps):
    """one untimed call, then reps calls each between two HIP events on the launch stream (ms list)"""
    import torch
    fn()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record()
    for i in range(reps):
        fn()
        ev[i + 1].record()
    torch.cuda.synchronize()
    return [ev[i].elapsed_time(ev[i + 1]) for i in range(reps)]


def fp64_form_record(s, a, W, params, r0, dev, reps=10):
    """Local energies per second of the plain float64 GPU form (every stage in float64, autotuned
    tiles) on the same walkers, the comparison form for the float32 plan."""
    import torch
    from paper_2307_14123_amd import qmc
    plan = qmc.Plan([s], [W], a, "fp64", autotune=True)
    P = torch.as_tensor(params, dtype=torch.float64, device=dev).contiguous()
    R = torch.as_tensor(r0, device=dev).contiguous()
    out = plan.local_energy(P, R)
    ms = _event_reps(lambda: plan.local_energy(P, R, out=out), reps)
    d = dist(ms)
    rec = {"e_loc_per_s": W / (d["median"] * 1e-3), "e_loc_ms_events": d, "walkers": W,
           "tiles": plan.tiles()[0], "precision": "fp64"}
    del plan, P, R, out
    return rec


def c4h4_record(dev, with_oracle=True, reps=3, n_err=4):
    """C4H4-sized system at 8192 walkers (width 256, 32 determinants): local-energy time in the float32
    plan and in the plan with bf16 operands in the value-row forwards (bf16v), each on its own
    autotuned plan, and the E_L error of both against the float64 oracle on a few walkers written into
    the first rows of the full batch."""
    import torch
    import oracle
    import qmc_inputs as qi
    from paper_2307_14123_amd import qmc
    s, a, p, r = qi.workload_inputs(3)
    W = r.shape[0]
    ref = oracle.local_energy(r[:n_err], p.astype(np.float32).astype(np.float64), s, a) if with_oracle else None
    rec = {"walkers": W, "electrons": s.n_elec, "width": a.width, "dets": a.n_det}
    for prec in ("fp32", "bf16v"):
        plan = qmc.Plan([s], [W], a, prec, autotune=True)
        P = torch.as_tensor(p, dtype=torch.float32, device=dev).contiguous()
        R = torch.as_tensor(r, device=dev).contiguous()
        out = plan.local_energy(P, R)
        ms = _event_reps(lambda: plan.local_energy(P, R, out=out), reps)
        d = dist(ms)
        lp, _ = plan.logpsi(P, R)
        torch.cuda.synchronize()
        e = {"e_loc_ms_events": d, "e_loc_per_s": W / (d["median"] * 1e-3), "tiles": plan.tiles()[0],
             "chunk_walkers": plan.chunk_walkers()[0]}
        if ref is not None:
            err = np.abs(out["e_loc"][:n_err].cpu().numpy() - ref["e_loc"]) * 1e3
            e["e_loc_err_mha_vs_fp64_oracle"] = {"max": float(err.max()), "p50": float(np.median(err)),
                                                 "walkers": n_err}
            e["value_logpsi_max_abs_err"] = float(np.abs(lp[:n_err].cpu().numpy() - ref["logpsi"]).max())
        rec[prec] = e
        del plan, P, R, out, lp
        torch.cuda.empty_cache()
    return rec


def batched_record(W, prec, steps, warmup, dev, packing_bound=False):
    """16 molecules x W walkers: local energy + loss gradient of the whole batch as one graph launch
    (a concurrent, autotuned plan: one stream per molecule inside the graph) against per-molecule
    launches (one plan per molecule, run one after another).

    packing_bound: also time every molecule alone at 8 W walkers, where its kernels fill the device.
    No single launch that packs the molecules' tiles together can process a molecule's W walkers
    faster than a full device does (per walker), so sum_m t_m(8 W) / 8 is a lower bound on the
    batch's time in any grouped launch, and (per-molecule time) / that bound caps its speed-up."""
    import torch
    import qmc_inputs as qi
    from paper_2307_14123_amd import qmc

    wl = qi.workload(4)
    mols, a = list(wl.systems), wl.ansatz
    params = [qi.make_params(m, a, qi.seed(4, 10 + k)) for k, m in enumerate(mols)]
    pos = [qi.make_walkers(m, W, qi.seed(4, 40 + k)) for k, m in enumerate(mols)]
    dt = torch.float64 if prec == "fp64" else torch.float32

    def timed(fn, reps):
        return float(np.sum(_event_reps(fn, reps)) / reps)

    # per-molecule launches: one single-system plan per molecule, eager, one after another
    per_mol = []
    for m, p, r in zip(mols, params, pos):
        plan = qmc.Plan([m], [W], a, prec)
        Pm = torch.as_tensor(p, dtype=dt, device=dev)
        Rm = torch.as_tensor(r, device=dev).contiguous()
        o = plan.local_energy(Pm, Rm)

        def one():
            plan.local_energy(Pm, Rm, out=o)
            plan.loss_grad(Pm, Rm, o["e_loc"])
        per_mol.append(timed(one, max(2, steps)))
        del plan, o
        torch.cuda.empty_cache()
    ms_per_mol = float(sum(per_mol))
    full = []
    if packing_bound:
        for m, p, r in zip(mols, params, pos):
            W8 = 8 * W
            plan = qmc.Plan([m], [W8], a, prec)
            Pm = torch.as_tensor(p, dtype=dt, device=dev)
            Rm = torch.as_tensor(np.concatenate([r] * 8).ravel(), device=dev).contiguous()
            o = plan.local_energy(Pm, Rm)

            def one8():
                plan.local_energy(Pm, Rm, out=o)
                plan.loss_grad(Pm, Rm, o["e_loc"])
            full.append(timed(one8, 2) / 8)
            print(f"[batched] {m.n_up + m.n_down} electrons: {per_mol[len(full) - 1]:.2f} ms at {W} walkers, "
                  f"{full[-1]:.2f} ms per {W} at {W8}", file=sys.stderr, flush=True)
            del plan, o, Rm
            torch.cuda.empty_cache()

    # the batch: one plan, concurrent molecules, autotuned tiles
    t0 = time.perf_counter()
    plan = qmc.Plan(mols, [W] * len(mols), a, prec, concurrent=True, autotune=True)
    t_tune = time.perf_counter() - t0
    P = torch.as_tensor(np.concatenate(params), dtype=dt, device=dev)
    R = torch.as_tensor(np.concatenate([r.ravel() for r in pos]), device=dev).contiguous()
    o = plan.local_energy(P, R)

    def eager():
        plan.local_energy(P, R, out=o)
        plan.loss_grad(P, R, o["e_loc"])
    ms_eager = timed(eager, max(2, steps))
    # one profiled eager pass for the per-kernel split
    qmc.profile_enable(True)
    qmc.profile_report(reset=True)
    eager()
    torch.cuda.synchronize()
    prof = qmc.profile_report(reset=True)
    qmc.profile_enable(False)
    g = qmc.GraphStep(plan, P, R)
    for _ in range(warmup):
        g.replay()
    ms_graph = timed(g.replay, steps)
    rec = {"electrons": [m.n_up + m.n_down for m in mols], "walkers_each": W, "width": a.width, "dets": a.n_det,
           "step": "local energy + loss gradient of every molecule",
           "batched_graph_ms": ms_graph, "batched_eager_ms": ms_eager, "per_molecule_ms": ms_per_mol,
           "per_molecule_ms_each": [round(x, 3) for x in per_mol],
           "speedup_graph_vs_per_molecule": ms_per_mol / ms_graph, "autotune_s": t_tune, "tiles": plan.tiles(),
           **({"full_device_ms_each_per_W": [round(x, 3) for x in full],
               "packed_lower_bound_ms": float(sum(full)),
               "grouped_launch_speedup_cap": ms_per_mol / float(sum(full))} if full else {}),
           "kernels_ms_eager_pass": {k: round(v[1], 3) for k, v in sorted(prof.items(), key=lambda kv: -kv[1][1])[:12]}}
    del g, plan, P, R, o
    return rec


def bench_precision(args):
    """C4H4-sized system (28 electrons, width 256, 32 determinants) at 8192 walkers: the local energy in
    the float32 plan, the plan with bf16 operands in the value-row forwards (bf16v: the local-energy jets
    stay float32) and the plan with bf16 operands in every embedding GEMM (bf16), each autotuned; E_L of
    an oracle sample (written into the first walkers of the full batch) against the float64 oracle on
    the float32-rounded parameters, and the value-row log|psi| that Metropolis uses."""
    import torch
    import oracle
    import qmc_inputs as qi
    from paper_2307_14123_amd import qmc
    s, a, p, r = qi.workload_inputs(3)
    W = r.shape[0]
    nw = min(args.cpu_walkers or 64, W)
    pr = p.astype(np.float32).astype(np.float64)
    torch.set_num_threads(os.cpu_count() or 1)
    t0 = time.perf_counter()
    parts = []
    for i in range(0, nw, 16):
        parts.append(oracle.local_energy(r[i:min(i + 16, nw)], pr, s, a, chunk=16))
        print(f"[precision] oracle walkers {i}..{min(i + 16, nw) - 1} done", file=sys.stderr, flush=True)
    ref = {k: np.concatenate([q[k] for q in parts]) for k in parts[0]}
    t_or = time.perf_counter() - t0
    print(f"[precision] oracle on {nw} walkers: {t_or:.1f} s", file=sys.stderr, flush=True)
    scale = np.maximum.reduce([np.abs(ref["e_loc"]), 0.5 * np.abs(ref["lap"]),
                               0.5 * (ref["grad"] ** 2).sum((1, 2)), np.ones(nw)])
    dev = torch.device("cuda", 0)
    rows = {}
    for prec in ("fp32", "bf16v", "bf16"):
        plan = qmc.Plan([s], [W], a, prec, autotune=True)
        P = torch.as_tensor(p, dtype=torch.float32, device=dev).contiguous()
        R = torch.as_tensor(r, device=dev).contiguous()
        out = plan.local_energy(P, R)
        ms = _event_reps(lambda: plan.local_energy(P, R, out=out), max(2, args.steps))
        lp, _ = plan.logpsi(P, R)
        lpt = _event_reps(lambda: plan.logpsi(P, R, out=(lp, None)), max(2, args.steps))
        torch.cuda.synchronize()
        e = out["e_loc"][:nw].cpu().numpy()
        err = np.abs(e - ref["e_loc"]) * 1e3
        rel = np.abs(e - ref["e_loc"]) / scale
        lerr = np.abs(lp[:nw].cpu().numpy() - ref["logpsi"])
        rows[prec] = {"e_loc_ms_events": dist(ms), "e_loc_per_s": W / (np.median(ms) * 1e-3),
                      "logpsi_ms_events": dist(lpt), "tiles": plan.tiles()[0],
                      "e_loc_err_mha": {"p50": float(np.median(err)), "p99": float(np.percentile(err, 99)),
                                        "max": float(err.max()), "mean_energy": float(abs(e.mean() - ref["e_loc"].mean()) * 1e3)},
                      "e_loc_err_rel_largest_addend_max": float(rel.max()),
                      "value_logpsi_abs_err": {"p50": float(np.median(lerr)), "max": float(lerr.max())}}
        print(f"[precision] {prec}: E_L {np.median(ms):.1f} ms, p50 {np.median(err):.3g} mHa, max {err.max():.3g} mHa",
              file=sys.stderr, flush=True)
        del plan, P, R, out, lp
        torch.cuda.empty_cache()
    res = {
        "metric": "walker local energies/sec at stated mHa error vs FP64 oracle; VMC train step ms",
        "value": rows["fp32"]["e_loc_per_s"], "unit": "walkers/s", "n_gpus": 1, "steps": max(2, args.steps),
        "warmup": 1, "ms_per_step": float(np.median(rows["fp32"]["e_loc_ms_events"]["median"])),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64 (bf16 variants below)",
        "data": "synthetic",
        "config": {"workload": f"C4H4-sized: 4 C + 4 H, 14 up + 14 down, {W} walkers, width {a.width}, "
                               f"{a.n_det} dets; step = local energy", "walkers": W},
        "oracle_sample": {"walkers": nw, "seconds": t_or, "cores": torch.get_num_threads(),
                          "params": "float32-rounded"},
        "variants": rows,
    }
    print(json.dumps(res))


def bench_batched(args):
    """The batched workload alone: 16 molecules x 1024 walkers in one graph vs per-molecule launches."""
    import torch
    import qmc_inputs as qi
    wl = qi.workload(4)
    W = args.walkers or wl.walkers
    prec = args.precision
    rec = batched_record(W, prec, args.steps, args.warmup, torch.device("cuda", 0), packing_bound=True)
    Wt = W * len(wl.systems)
    res = {
        "metric": "walker local energies/sec at stated mHa error vs FP64 oracle; VMC train step ms",
        "value": Wt / (rec["batched_graph_ms"] * 1e-3),
        "unit": "walkers/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": rec["batched_graph_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32+f64", "fp64": "f64", "bf16": "bf16+f32+f64", "bf16v": "bf16+f32+f64"}[prec],
        "data": "synthetic",
        "config": {"workload": f"16 molecules ({', '.join(str(n) for n in rec['electrons'])} electrons), "
                               f"{W} walkers each, width {rec['width']}, {rec['dets']} dets; step = local energy + "
                               f"loss gradient of every molecule",
                   "walkers": Wt, "precision": prec},
    }
    res.update(rec)
    print(json.dumps(res))


def bench_scaling(args):
    """Train-step time against system size (Sec. VI, scaling): atoms and hydrogen chains up to 45 electrons,
    2000 walkers each, the N2-sized ansatz at random init; one step = the train step of the headline
    workload (10 Metropolis steps + local energy + clipping + loss gradient + update), captured into
    one HIP graph per system.  A power law t = c N^b is fitted per system class."""
    import torch
    import qmc_inputs as qi
    from paper_2307_14123_amd import qmc

    a = qi.SCALING_ANSATZ
    W = args.walkers or qi.SCALING_WALKERS
    prec = args.precision
    n_mc, tau, lr = 10, 0.2, 1e-8
    dev = torch.device("cuda", 0)
    steps = max(2, args.steps)
    rows = []
    for cls, sizes, make in (("atoms", qi.SCALING_ATOMS, qi.atom), ("chains", qi.SCALING_CHAINS, qi.hydrogen_chain)):
        for n in sizes:
            s = make(n)
            plan = qmc.Plan([s], [W], a, prec, autotune=True)
            P = torch.as_tensor(qi.make_params(s, a, 9000 + n), dtype=plan.param_dtype, device=dev).contiguous()
            R = torch.as_tensor(qi.make_walkers(s, W, 9100 + n), device=dev).contiguous()
            NOISE = torch.as_tensor(qi.make_noise(n_mc, W, s.n_elec, 9200 + n), device=dev).contiguous()
            U = torch.as_tensor(qi.make_uniforms(n_mc, W, 9300 + n), device=dev).contiguous()
            for op in (qmc.OP_LOGPSI, qmc.OP_LOCAL_ENERGY, qmc.OP_METROPOLIS):
                plan.workspace(op)
            lp, _ = plan.logpsi(P, R)
            out = plan.local_energy(P, R)
            G, EM = plan.loss_grad(P, R, out["e_loc"])
            EC = torch.empty_like(out["e_loc"])
            acc = torch.empty(W, dtype=torch.uint8, device=dev)

            def step():
                for t in range(n_mc):
                    plan.metropolis_step(P, R, lp, NOISE[t], U[t], tau, accepted=acc)
                plan.local_energy(P, R, out=out)
                plan.clip_local_energy(out["e_loc"], 5.0, "hard", out=EC)
                plan.loss_grad(P, R, EC, grad=G, e_mean=EM)
                plan.sgd_update(P, G, lr)
                # the next step's Metropolis comparisons need log|psi| under the updated parameters
                plan.logpsi(P, R, out=(lp, None))

            for _ in range(max(1, args.warmup)):
                step()
            torch.cuda.synchronize()
            run, launch = step, "eager"
            try:
                side = torch.cuda.Stream()
                side.wait_stream(torch.cuda.current_stream())
                with torch.cuda.stream(side):
                    step()
                torch.cuda.current_stream().wait_stream(side)
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g):
                    step()
                g.replay()
                torch.cuda.synchronize()
                run, launch = g.replay, "graph"
            except Exception:  # noqa: BLE001 - eager steps then
                g = None
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(steps):
                run()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            e0.record()
            plan.local_energy(P, R, out=out)
            e1.record()
            torch.cuda.synchronize()
            ms_le = e0.elapsed_time(e1)
            finite = float(torch.isfinite(out["e_loc"]).double().mean().item())
            # one eager step with HIP events around every launch: the largest kernel families
            qmc.profile_enable(True)
            qmc.profile_report(reset=True)
            step()
            torch.cuda.synchronize()
            prof = qmc.profile_report(reset=True)
            qmc.profile_enable(False)
            fam = {}
            for kname, (_, kms) in prof.items():
                f = kernel_family(kname)
                fam[f] = fam.get(f, 0.0) + kms
            top = {k: round(v, 2) for k, v in sorted(fam.items(), key=lambda kv: -kv[1])[:6]}
            rows.append({"class": cls, "n": n, "electrons": s.n_elec, "nuclei": s.n_nuc, "step_ms": ms,
                         "e_loc_ms": ms_le, "launch": launch, "finite_e_loc_fraction": finite,
                         "eager_step_kernels_ms": top})
            print(f"[scaling] {cls} n={n}: step {ms:.2f} ms, local energy {ms_le:.2f} ms ({launch})", file=sys.stderr,
                  flush=True)
            del g, plan, P, R, NOISE, U, lp, out, G, EM, EC, acc
            torch.cuda.empty_cache()

    def fit(cls, key, nmin):
        pts = [(r["electrons"], r[key]) for r in rows if r["class"] == cls and r["electrons"] >= nmin]
        b, c = np.polyfit(np.log([x for x, _ in pts]), np.log([y for _, y in pts]), 1)
        return float(b)

    fits = {cls: {"step_exponent_all": fit(cls, "step_ms", 1), "step_exponent_n_ge_10": fit(cls, "step_ms", 10),
                  "e_loc_exponent_all": fit(cls, "e_loc_ms", 1), "e_loc_exponent_n_ge_10": fit(cls, "e_loc_ms", 10)}
            for cls in ("atoms", "chains")}
    largest = max(rows, key=lambda r: r["step_ms"])
    res = {
        "metric": "train step time vs electron count (power-law exponent)",
        "value": fits["chains"]["step_exponent_all"],
        "unit": "exponent",
        "n_gpus": 1, "steps": steps, "warmup": args.warmup, "ms_per_step": largest["step_ms"],
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32+f64", "fp64": "f64", "bf16": "bf16+f32+f64", "bf16v": "bf16+f32+f64"}[prec],
        "data": "synthetic",
        "config": {"workload": f"atoms Z in {list(qi.SCALING_ATOMS)} and hydrogen chains n in "
                               f"{list(qi.SCALING_CHAINS)} (1.8 bohr spacing), {W} walkers, width {a.width}, "
                               f"{a.mp_layers} message-passing layers, {a.n_det} dets; step = {n_mc} Metropolis "
                               f"steps + local energy + clipping + loss gradient + update",
                   "walkers": W, "precision": prec},
        "fits": fits,
        "rows": rows,
    }
    print(json.dumps(res))

if __name__ == "__main__":
    main()
