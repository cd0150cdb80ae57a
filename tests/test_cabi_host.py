"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, computes the parameter count of the pinned blob, and rejects
invalid arguments before launching anything."""
import ctypes
import os
import re

import pytest

import qmc_inputs as qi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qmc.h")


def _lib():
    from paper_2307_14123_amd import qmc
    try:
        return qmc, qmc.lib()
    except RuntimeError as e:  # library not built in this checkout
        pytest.skip(str(e))


def test_header_symbols_exported():
    _, L = _lib()
    text = open(HEADER).read()
    names = set(re.findall(r"^\s*(?:qmc_status|int64_t|const char\*)\s+(qmc_\w+)\s*\(", text, re.M))
    assert len(names) >= 14
    for n in sorted(names):
        assert hasattr(L, n), n


def test_param_count_matches_layout():
    qmc, _ = _lib()
    for k in range(4):
        wl = qi.workload(k)
        assert qmc.param_count(wl.systems[0], wl.ansatz) == qi.param_count(wl.systems[0], wl.ansatz)
    for s in qi.workload(4).systems:
        assert qmc.param_count(s, qi.BATCH_ANSATZ) == qi.param_count(s, qi.BATCH_ANSATZ)


def test_invalid_arguments_rejected():
    qmc, L = _lib()
    a = qmc.make_ansatz(qi.N2_ANSATZ)
    h = qmc._SysHolder(qi.N2)
    vp = ctypes.c_void_p
    # bad system / ansatz
    bad = qmc.QmcSystem(0, h.Z, h.R, 7, 7)
    assert L.qmc_param_count(ctypes.byref(bad), ctypes.byref(a)) < 0
    a2 = qmc.make_ansatz(qi.N2_ANSATZ)
    a2.version = 2
    assert L.qmc_param_count(ctypes.byref(h.s), ctypes.byref(a2)) < 0
    handle = vp(0)
    W = (ctypes.c_int64 * 1)(16)
    arr = (qmc.QmcSystem * 1)(h.s)
    assert L.qmc_plan_create(ctypes.byref(handle), arr, 1, W, ctypes.byref(a), 7, 0) == 1      # precision
    assert L.qmc_plan_create(ctypes.byref(handle), arr, 1, W, ctypes.byref(a), 1, 8) == 1      # unknown flag
    W0 = (ctypes.c_int64 * 1)(0)
    assert L.qmc_plan_create(ctypes.byref(handle), arr, 1, W0, ctypes.byref(a), 1, 0) == 1     # no walkers
    neg = qmc.QmcSystem(2, h.Z, h.R, -1, 7)
    arrn = (qmc.QmcSystem * 1)(neg)
    assert L.qmc_plan_create(ctypes.byref(handle), arrn, 1, W, ctypes.byref(a), 1, 0) == 1
    assert L.qmc_plan_create(ctypes.byref(handle), arr, 1, W, ctypes.byref(a), 1, 0) == 0
    try:
        sz = ctypes.c_size_t()
        assert L.qmc_workspace_size(handle, 1, ctypes.byref(sz)) == 0 and sz.value > 0
        assert L.qmc_workspace_size(handle, 9, ctypes.byref(sz)) == 1
        fake = vp(0x1000)
        # null pointers
        assert L.qmc_local_energy(handle, None, fake, None, None, None, None, fake, fake, sz.value, None) == 1
        # workspace too small
        assert L.qmc_local_energy(handle, fake, fake, None, None, None, None, fake, vp(0x10000), 16, None) == 3
        # misaligned workspace
        assert L.qmc_local_energy(handle, fake, fake, None, None, None, None, fake, vp(0x10001), sz.value, None) == 1
        # Metropolis: negative or non-finite step
        assert L.qmc_workspace_size(handle, 2, ctypes.byref(sz)) == 0
        assert L.qmc_metropolis_step(handle, fake, fake, fake, fake, fake, -0.1, None, vp(0x10000), sz.value,
                                     None) == 1
        assert L.qmc_metropolis_step(handle, fake, fake, fake, fake, fake, float("nan"), None, vp(0x10000),
                                     sz.value, None) == 1
        assert L.qmc_loss_grad(handle, fake, fake, None, fake, None, vp(0x10000), 1 << 40, None) == 1
        # Langevin: step and damping flag, missing gradient, small workspace
        assert L.qmc_workspace_size(handle, 5, ctypes.byref(sz)) == 0
        assert L.qmc_mala_step(handle, fake, fake, fake, fake, fake, fake, -0.1, 1, None, vp(0x10000), sz.value,
                               None) == 1
        assert L.qmc_mala_step(handle, fake, fake, fake, fake, fake, fake, float("inf"), 1, None, vp(0x10000),
                               sz.value, None) == 1
        assert L.qmc_mala_step(handle, fake, fake, fake, fake, fake, fake, 0.1, 2, None, vp(0x10000), sz.value,
                               None) == 1
        assert L.qmc_mala_step(handle, fake, fake, fake, None, fake, fake, 0.1, 1, None, vp(0x10000), sz.value,
                               None) == 1
        assert L.qmc_mala_step(handle, fake, fake, fake, fake, fake, fake, 0.1, 1, None, vp(0x10000), 16,
                               None) == 3
        # clipping: width and mode
        assert L.qmc_clip_local_energy(handle, fake, fake, 0.0, 0, None) == 1
        assert L.qmc_clip_local_energy(handle, fake, fake, float("nan"), 0, None) == 1
        assert L.qmc_clip_local_energy(handle, fake, fake, 5.0, 2, None) == 1
        assert L.qmc_clip_local_energy(handle, None, fake, 5.0, 0, None) == 1
        # determinant entry: bad sizes
        assert L.qmc_det_jets(4, 0, 3, fake, fake, fake, fake, fake, None) == 1
        assert L.qmc_det_jets(4, 33, 3, fake, fake, fake, fake, fake, None) == 1
        assert L.qmc_det_jets(0, 4, 3, None, None, None, None, None, None) == 0
    finally:
        assert L.qmc_plan_destroy(handle) == 0
    assert L.qmc_plan_destroy(None) == 1
    assert L.qmc_status_str(3) == b"QMC_ERR_WORKSPACE_TOO_SMALL"


def test_walker_chunking_bounds_workspace():
    """The plan splits large walker counts into chunks so that the local-energy
    workspace stays under its limit (configs[3]: 8192 walkers of a 28-electron system)."""
    qmc, _ = _lib()
    plan = qmc.Plan([qi.C4H4], [8192], qi.C4H4_ANSATZ, "bf16")
    assert plan.workspace_bytes(qmc.OP_LOCAL_ENERGY) < (25 << 30)
    assert plan.total_params == 2286752


def test_plan_flags_and_tiles():
    """Known flags are accepted (they need a device: without one the plan reports QMC_ERR_HIP);
    a plain plan reports the built-in tile choice (0) for every GEMM class."""
    qmc, L = _lib()
    a = qmc.make_ansatz(qi.BATCH_ANSATZ)
    mols = qi.workload(4).systems[:2]
    hs = [qmc._SysHolder(m) for m in mols]
    arr = (qmc.QmcSystem * 2)(*[h.s for h in hs])
    W = (ctypes.c_int64 * 2)(8, 8)
    for flags in (1, 2, 3):
        handle = ctypes.c_void_p(0)
        st = L.qmc_plan_create(ctypes.byref(handle), arr, 2, W, ctypes.byref(a), 1, flags)
        assert st in (0, 4)
        if st == 0:
            assert L.qmc_plan_destroy(handle) == 0
        else:
            assert not handle.value
    handle = ctypes.c_void_p(0)
    assert L.qmc_plan_create(ctypes.byref(handle), arr, 2, W, ctypes.byref(a), 1, 0) == 0
    try:
        t = (ctypes.c_int32 * 4)()
        assert L.qmc_plan_tiles(handle, 1, t) == 0 and list(t) == [0, 0, 0, 0]
        assert L.qmc_plan_tiles(handle, 2, t) == 1
        assert L.qmc_plan_tiles(handle, -1, t) == 1
    finally:
        L.qmc_plan_destroy(handle)



def test_measure_peaks_rejects_bad_scratch():
    """qmc_measure_peaks validates its scratch buffer on the host before touching the device."""
    qmc, L = _lib()
    out = (ctypes.c_double * 4)()
    bad = [(None, 1 << 30), (ctypes.c_void_p(1 << 20), 1 << 10), (ctypes.c_void_p((1 << 20) + 4), 1 << 30),
           (ctypes.c_void_p(1 << 20), 1 << 40)]
    for ptr, n in bad:
        assert L.qmc_measure_peaks(ptr, n, out, None) == 1  # QMC_ERR_INVALID_ARGUMENT
    assert L.qmc_measure_peaks(ctypes.c_void_p(1 << 20), 1 << 30, None, None) == 1


def test_sgd_update_rejects_bad_arguments():
    """qmc_sgd_update validates on the host before launching."""
    qmc, L = _lib()
    p = ctypes.c_void_p(1 << 20)
    assert L.qmc_sgd_update(1, p, p, -1, 1e-3, None) == 1
    assert L.qmc_sgd_update(1, None, p, 10, 1e-3, None) == 1
    assert L.qmc_sgd_update(1, p, p, 10, float("nan"), None) == 1
    assert L.qmc_sgd_update(7, p, p, 10, 1e-3, None) == 1
    assert L.qmc_sgd_update(1, None, None, 0, 1e-3, None) == 0


def test_ansatz_options_count_and_limits():
    """Parameter counts with the Jastrow, full-determinant and edge-update options match the blob layout; invalid
    option values and a full determinant above 32 electrons are rejected."""
    import dataclasses
    qmc, L = _lib()
    for s in (qi.N2, qi.C4H4, qi.System((3.0, 1.0), ((0.0, 0.0, 0.0), (1.6, 0.2, -0.3)), 3, 1)):
        for opts in ({"jastrow": 1}, {"full_det": 1}, {"jastrow": 1, "full_det": 1, "ee_cusp": 0.5},
                     {"edge_update": 1}, {"edge_update": 1, "mp_layers": 1}, {"edge_update": 1, "jastrow": 1}):
            a = dataclasses.replace(qi.N2_ANSATZ, **opts)
            assert qmc.param_count(s, a) == qi.param_count(s, a)
    h = qmc._SysHolder(qi.N2)
    for opts in ({"jastrow": 2}, {"full_det": -1}, {"ee_cusp": -1.0}, {"ee_cusp": float("inf")}, {"edge_update": 3}):
        a = qmc.make_ansatz(dataclasses.replace(qi.N2_ANSATZ, **opts))
        assert L.qmc_param_count(ctypes.byref(h.s), ctypes.byref(a)) < 0
    big = qi.atom(33)
    hb = qmc._SysHolder(big)
    arr = (qmc.QmcSystem * 1)(hb.s)
    W = (ctypes.c_int64 * 1)(4)
    handle = ctypes.c_void_p()
    a = qmc.make_ansatz(dataclasses.replace(qi.N2_ANSATZ, full_det=1))
    assert L.qmc_plan_create(ctypes.byref(handle), arr, 1, W, ctypes.byref(a), 1, 0) == 2
    a = qmc.make_ansatz(qi.N2_ANSATZ)
    assert L.qmc_plan_create(ctypes.byref(handle), arr, 1, W, ctypes.byref(a), 1, 0) == 0
    try:
        sz = ctypes.c_size_t()
        assert L.qmc_workspace_size(handle, 6, ctypes.byref(sz)) == 0 and sz.value > 0
        fake = ctypes.c_void_p(0x1000)
        assert L.qmc_logpsi_grad(handle, fake, fake, None, fake, ctypes.c_void_p(0x10000), sz.value, None) == 1
        assert L.qmc_logpsi_grad(handle, fake, fake, fake, fake, ctypes.c_void_p(0x10000), 16, None) == 3
    finally:
        assert L.qmc_plan_destroy(handle) == 0


def test_chunk_cap_and_loss_grad_header():
    """qmc_plan_create_ex caps the walkers per chunk (ragged last chunk), rejects a negative cap, and
    the loss-gradient workspace carries its documented header of one int64 count per system."""
    qmc, L = _lib()
    a = qmc.make_ansatz(qi.N2_ANSATZ)
    h = qmc._SysHolder(qi.N2)
    arr = (qmc.QmcSystem * 1)(h.s)
    W = (ctypes.c_int64 * 1)(100)
    handle = ctypes.c_void_p()
    assert L.qmc_plan_create_ex(ctypes.byref(handle), arr, 1, W, ctypes.byref(a), 1, 0, -1) == 1
    sizes = {}
    for cap, expect in ((0, 100), (30, 30), (100, 100), (1000, 100)):
        handle = ctypes.c_void_p()
        assert L.qmc_plan_create_ex(ctypes.byref(handle), arr, 1, W, ctypes.byref(a), 1, 0, cap) == 0
        try:
            wc = ctypes.c_int64()
            assert L.qmc_plan_chunk_walkers(handle, 0, ctypes.byref(wc)) == 0 and wc.value == expect
            assert L.qmc_plan_chunk_walkers(handle, 1, ctypes.byref(wc)) == 1
            sz = {}
            for op in (1, 4):
                b = ctypes.c_size_t()
                assert L.qmc_workspace_size(handle, op, ctypes.byref(b)) == 0
                sz[op] = b.value
            sizes[cap] = sz
        finally:
            assert L.qmc_plan_destroy(handle) == 0
    # a smaller chunk needs a smaller workspace
    assert sizes[30][1] < sizes[0][1] and sizes[30][4] < sizes[0][4]
    assert sizes[1000] == sizes[0]
    # two systems: header of two int64 counts, rounded to 256 bytes, before the regions
    a = qmc.make_ansatz(qi.BATCH_ANSATZ)
    mols = qi.workload(4).systems[:2]
    hs = [qmc._SysHolder(m) for m in mols]
    arr = (qmc.QmcSystem * 2)(*[x.s for x in hs])
    W = (ctypes.c_int64 * 2)(8, 8)
    handle = ctypes.c_void_p()
    assert L.qmc_plan_create_ex(ctypes.byref(handle), arr, 2, W, ctypes.byref(a), 1, 0, 3) == 0
    try:
        wc = ctypes.c_int64()
        for k in range(2):
            assert L.qmc_plan_chunk_walkers(handle, k, ctypes.byref(wc)) == 0 and wc.value == 3
    finally:
        assert L.qmc_plan_destroy(handle) == 0
