"""Shared helpers of the GPU tests (no method arithmetic here)."""
from __future__ import annotations

import numpy as np


def rel_fro(x, ref) -> float:
    x = np.asarray(x)
    ref = np.asarray(ref)
    return float(np.linalg.norm((x - ref).ravel()) / np.linalg.norm(ref.ravel()))


def max_row_rel(x, ref) -> float:
    x = np.asarray(x)
    ref = np.asarray(ref)
    num = np.linalg.norm(x - ref, axis=1)
    den = np.linalg.norm(ref, axis=1)
    return float(np.max(num / den))


def dev(t, dtype=None):
    import torch
    a = torch.from_numpy(np.ascontiguousarray(t))
    if dtype is not None:
        a = a.to(dtype)
    return a.cuda()


def host(t) -> np.ndarray:
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def report(name: str, **vals):
    items = " ".join(f"{k}={v:.3e}" if isinstance(v, float) else f"{k}={v}" for k, v in vals.items())
    print(f"[parity] {name}: {items}", flush=True)
