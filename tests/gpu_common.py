"""Helpers shared by the GPU tests (no oracle arithmetic here)."""
import numpy as np
import torch


def dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype).cuda().contiguous()


def host(t):
    return t.detach().cpu().numpy()


def rel_err(got, ref, floor=1.0):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return np.abs(got - ref) / np.maximum(np.abs(ref), floor)


def report(name, err_mha):
    e = np.abs(np.asarray(err_mha))
    print(f"[{name}] |dE_L| mHa: p50={np.percentile(e, 50):.4g} p99={np.percentile(e, 99):.4g} max={e.max():.4g}",
          flush=True)
