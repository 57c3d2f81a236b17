#!/usr/bin/env python3
"""Band-pair Fock applications per second on one MI355X.

A step is one application of the exchange operator to every target of the
workload: every band pair (i, j) goes through pair density, forward FFT,
Coulomb kernel, backward FFT and multiply-accumulate, plus the per-orbital
transforms and the per-target finish (all inside libfockx.so).  Inputs are
synthetic, seeded, and resident in HBM before the timed region.

Prints one JSON line.  Besides throughput it reports the dominant kernel's
achieved bandwidth against the HBM peak (durations from HIP events recorded
around every launch by the library's tracer, in a second pass over the same
steps) and the CPU FP64 oracle timed on a bounded sample on the host cores.
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

HBM_PEAK_GBS = 8000.0
METRIC = "band-pair Fock applications/sec and HBM GB/s at 1 GPU, FP32-batched vs FP64 plain"

WORKLOADS = {
    # name: (description, builder, complex dtype, bytes per complex)
    "c2_fp64": "64^3 cubic L=20 bohr, 128 orbitals applied to themselves, FP64 (all 16384 pairs)",
    "c3_fp32": "96x96x128 orthorhombic 22x22x30 bohr, 512 orbitals applied to themselves, FP32 (262144 pairs)",
    "c3_fp64": "96x96x128 orthorhombic 22x22x30 bohr, 512 orbitals applied to themselves, FP64 (262144 pairs)",
}


def build_workload(name):
    if name == "c2_fp64":
        s, c = synth.config2()
        return s, c, "c128"
    if name in ("c3_fp32", "c3_fp64"):
        s, c = synth.config3()
        return s, c, "c64" if name.endswith("fp32") else "c128"
    raise SystemExit(f"unknown workload {name}")


# ---------------------------------------------------------------------------
# CPU baseline: the oracle as it stands, one target per worker process
# ---------------------------------------------------------------------------
_CPU = {}


def _cpu_worker(j):
    os.environ["OMP_NUM_THREADS"] = "1"
    from oracle import exx
    s, c, nocc = _CPU["s"], _CPU["c"], _CPU["nocc"]
    t0 = time.perf_counter()
    exx.fock_apply(s.a, s.n, s.miller, np.zeros(3), c[:nocc], np.ones(nocc), c[j:j + 1])
    return time.perf_counter() - t0


def cpu_baseline(s, c, nocc=None):
    cores = len(os.sched_getaffinity(0))
    workers = max(1, min(16, cores))
    if nocc is None:
        nocc = 64 if s.n[0] * s.n[1] * s.n[2] <= 300_000 else 8
    nocc = min(nocc, c.shape[0])
    _CPU.update(s=s, c=c, nocc=nocc)
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        pool.map(abs, range(workers))  # start the workers
        t0 = time.perf_counter()
        pool.map(_cpu_worker, range(workers))
        wall = time.perf_counter() - t0
    pairs = workers * nocc
    return {"value": pairs / wall, "unit": "band-pair applications/s", "cores": workers, "kind": "oracle",
            "sample": f"{workers} targets x first {nocc} occupied orbitals ({pairs} pairs, FP64 scipy FFT, "
                      f"one single-threaded process per target), wall {wall:.2f} s"}


# ---------------------------------------------------------------------------
# algorithmic bytes per launch of the pair kernels (tile ti x tj, N points, b bytes)
# ---------------------------------------------------------------------------
def kernel_bytes(cls, ti, tj, N, b):
    if cls == "p1_pair_plane_fwd":   # read ti + tj orbital boxes, write ti*tj pair boxes
        return (ti * tj + ti + tj) * N * b
    if cls == "p2_pencil_kernel":    # read + write each pair box
        return 2 * ti * tj * N * b
    if cls == "p3_plane_inv_mac":    # read pair boxes and ti orbitals, read-modify-write tj accumulators
        return (ti * tj + ti + 2 * tj) * N * b
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2_fp64", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-trace", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (bandwidth-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    s, c, prec = build_workload(args.workload)
    nb = c.shape[0]
    N = s.n[0] * s.n[1] * s.n[2]
    bpc = 16 if prec == "c128" else 8

    cpu = None if args.no_cpu_baseline else cpu_baseline(s, c)

    import torch
    from paper_1305_7313_amd import fock

    dev = torch.device("cuda:0")
    cdt = torch.complex128 if prec == "c128" else torch.complex64
    cd = torch.from_numpy(c).to(cdt).to(dev)
    f = torch.ones(nb, dtype=torch.float64, device=dev)
    cell = fock.Cell(s.a, s.n, s.miller)
    out = torch.empty((nb, s.npw), dtype=cdt, device=dev)
    ws = fock.workspace(cell, fock.dtype_code(cd), nb, nb, dev)
    q = (0.0, 0.0, 0.0)

    def step():
        fock.fock_apply(cell, q, cd, f, cd, out=out, ws=ws)

    if args.copy_probe:
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = 1e3 * dt / args.steps
    pairs = nb * nb
    value = pairs * args.steps / dt

    roof = None
    kernels = {}
    if not args.no_trace:
        fock.fock_trace_enable(True)
        fock.fock_trace_read(reset=True)
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        tr = fock.fock_trace_read(reset=True)
        fock.fock_trace_enable(False)
        kernels = {k: {"ms_per_step": v[0] / args.steps, "launches_per_step": v[1] / args.steps}
                   for k, v in tr.items() if v[1]}
        pair_cls = [k for k in ("p1_pair_plane_fwd", "p2_pencil_kernel", "p3_plane_inv_mac") if k in tr]
        dom = max(pair_cls, key=lambda k: tr[k][0])
        ti = tj = min(16, nb)
        per_launch = kernel_bytes(dom, ti, tj, N, bpc)
        avg_ms = tr[dom][0] / tr[dom][1]
        achieved = per_launch / (avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": dom,
                "avg_launch_ms": round(avg_ms, 5), "bytes_per_launch": per_launch}

    # whole-path logical bandwidth: 4 N b per pair (read phi_i, psi_j; read+write acc_j)
    logical_gbs = value * 4 * N * bpc / 1e9
    rec = {
        "metric": METRIC, "value": round(value, 1), "unit": "band-pair applications/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == "c128" else "f32", "data": "synthetic",
        "config": {"workload": args.workload, "description": WORKLOADS[args.workload], "grid": list(s.n),
                   "npw": s.npw, "n_occ": nb, "n_tgt": nb, "pairs_per_step": pairs},
        "logical_hbm_gbs": round(logical_gbs, 1),
        "roofline": roof,
        "cpu_baseline": cpu,
        "kernels": kernels,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
