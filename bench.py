#!/usr/bin/env python3
"""Band-pair Fock applications per second on one MI355X.

A step is one application of the exchange operator to every target of the
workload: every band pair (i, j) goes through pair density, forward FFT,
Coulomb kernel, backward FFT and multiply-accumulate, plus the per-orbital
transforms and the per-target finish (all inside libfockx.so).  Inputs are
synthetic, seeded, and resident in HBM before the timed region.

Default workload (the metric's own): the 16-system uneven batch (cubic grids
from {48,64,72,96}^3, 32-242 orbitals each, 451204 pairs), FP32, the whole
batch in one hipGraph replay per step; beside it the FP64 plain form (one
fock_apply per system) and the FP32 plain form on the same systems, the
FP32 error against FP64, and the config-2 FP64 workload (64^3, 128 orbitals)
as a second record.

Also reported: the dominant kernel class against its roofline (algorithmic
bytes, or for a vector-ALU-bound class algorithmic flops, per launch over its
average launch time, measured with HIP events the library records around
every launch on its stream, in a pass over the same kernels); HBM traffic
from rocprofv3 counters when they were taken on the current kernel sources;
and the CPU FP64 oracle timed on a bounded sample on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import shutil
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

HBM_PEAK_GBS = 8000.0
# Vector ALU peak without packed FP32 instructions (the build never emits
# them): 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz, the same for
# FP32 and FP64 on this chip.
VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
METRIC = "band-pair Fock applications/sec and HBM GB/s at 1 GPU, FP32-batched vs FP64 plain"
UNIT = "band-pair applications/s"


def pair_tile(fp64):
    """Largest pair tile edge of the library's single-system schedules: 16 x
    16 pairs in FP64, 32 x 32 in FP32."""
    return 16 if fp64 else 32


def balanced_edge(n, edge):
    """The library's tile edge for a block of n orbitals: the fewest tiles of
    at most `edge`, of near-equal size."""
    if n <= 0:
        return 1
    parts = -(-n // edge)
    return -(-n // parts)

WORKLOADS = {
    "c2_fp64": "64^3 cubic L=20 bohr, 128 orbitals applied to themselves, FP64 (16384 pairs)",
    "c3_fp32": "96x96x128 orthorhombic 22x22x30 bohr, 512 orbitals applied to themselves, FP32 (262144 pairs)",
    "c3_fp64": "96x96x128 orthorhombic 22x22x30 bohr, 512 orbitals applied to themselves, FP64 (262144 pairs)",
    "c2r_fp64": "the c2_fp64 sphere and orbitals with the Fock cutoff at the wave-function cutoff (a quarter of "
                "the density cutoff) on the coarser exchange grid that keeps the result exact, FP64 (16384 pairs)",
    "c3r_fp32": "the c3_fp32 sphere and orbitals with the Fock cutoff at the wave-function cutoff on the coarser "
                "exact exchange grid, FP32 (262144 pairs)",
    "c2g_fp64": "the c2_fp64 cell and sphere with 128 real (Gamma) orbitals applied to themselves, two real "
                "orbitals per complex transform, FP64 (16384 pairs)",
    "c5_fp32_grad": "72^3 cubic L=24, 2x2x2 k-mesh, 256 orbitals per k, GB G=0 term: E_x and its gradient "
                    "(one forward and one backward), FP32 (4194304 pairs in E_x)",
    "c5r_fp32_grad": "the c5_fp32_grad mesh and orbitals with the Fock cutoff at the wave-function cutoff on the "
                     "coarser exact exchange grid for every q = k - k', FP32 (4194304 pairs in E_x)",
    "cp_density_fp64": "band loop: charge density sum_b f_b |psi_b(r)|^2 of the 512 c3 orbitals on 96x96x128, FP64",
    "cp_force_fp64": "band loop: force of H = -1/2 nabla^2 + V(r) on the 512 c3 orbitals on 96x96x128 "
                     "(synthetic normal V), FP64",
    "c4_fp32_batched": "16 systems, cubic grids from {48,64,72,96}^3, L=n/3.2, 32-242 orbitals each, each "
                       "applied to itself, FP32, the whole batch in one hipGraph replay (451204 pairs)",
    "c4_fp64_plain": "the same 16 systems, one FP64 fock_apply per system (451204 pairs)",
}


# ---------------------------------------------------------------------------
# CPU baseline: the oracle as it stands, one target per worker process
# ---------------------------------------------------------------------------
_CPU = {}


def _cpu_init(a, n, miller, ecut, c_occ, c_tgt):
    os.environ["OMP_NUM_THREADS"] = "1"
    _CPU.update(a=a, n=n, miller=miller, ecut=ecut, c_occ=c_occ, c_tgt=c_tgt)


def _cpu_worker(j):
    from oracle import exx
    c_occ = _CPU["c_occ"]
    t0 = time.perf_counter()
    exx.fock_apply(_CPU["a"], _CPU["n"], _CPU["miller"], np.zeros(3), c_occ, np.ones(len(c_occ)),
                   _CPU["c_tgt"][j:j + 1], ecut_fock=_CPU["ecut"])
    return time.perf_counter() - t0


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(s, c, n=None, ecut=0.0, nocc=None):
    n = tuple(s.n if n is None else n)
    workers = cpu_workers(16)
    if nocc is None:
        nocc = 64 if n[0] * n[1] * n[2] <= 300_000 else 8
    nocc = min(nocc, c.shape[0])
    # fresh interpreters: independent of whatever this process has initialised
    ctx = mp.get_context("spawn")
    log(f"CPU oracle baseline: {workers} processes")
    with ctx.Pool(workers, initializer=_cpu_init,
                  initargs=(s.a, n, s.miller, ecut, c[:nocc], c[:workers])) as pool:
        pool.map(abs, range(workers))  # start the workers
        t0 = time.perf_counter()
        pool.map(_cpu_worker, range(workers))
        wall = time.perf_counter() - t0
    pairs = workers * nocc
    return {"value": round(pairs / wall, 2), "unit": UNIT, "cores": workers, "kind": "oracle", "cpu": cpu_model(),
            "sample": f"{workers} targets x first {nocc} occupied orbitals ({pairs} pairs) of the same workload, "
                      f"FP64 scipy FFT, one single-threaded process per target, wall {wall:.2f} s"}


def _band_init(a, n, miller, c, w, v, force):
    os.environ["OMP_NUM_THREADS"] = "1"
    _CPU.update(a=a, n=n, miller=miller, c=c, w=w, v=v, force=force)


def _band_worker(j):
    from oracle import bands
    sl = slice(8 * j, 8 * j + 8)
    t0 = time.perf_counter()
    if _CPU["force"]:
        bands.band_force(_CPU["a"], _CPU["n"], _CPU["miller"], np.zeros(3), _CPU["c"][sl], _CPU["w"][sl], _CPU["v"])
    else:
        bands.band_density(_CPU["a"], _CPU["n"], _CPU["miller"], _CPU["c"][sl], _CPU["w"][sl])
    return time.perf_counter() - t0


def cpu_baseline_bands(s, c, w, v, force):
    workers = cpu_workers(16)
    ctx = mp.get_context("spawn")
    log(f"CPU oracle baseline: {workers} processes")
    with ctx.Pool(workers, initializer=_band_init,
                  initargs=(s.a, tuple(s.n), s.miller, c[:8 * workers], w[:8 * workers], v, force)) as pool:
        pool.map(abs, range(workers))
        t0 = time.perf_counter()
        pool.map(_band_worker, range(workers))
        wall = time.perf_counter() - t0
    nb = 8 * workers
    return {"value": round(nb / wall, 2), "unit": "bands/s", "cores": workers, "kind": "oracle", "cpu": cpu_model(),
            "sample": f"{nb} of the workload's bands, 8 per single-threaded process, FP64 scipy FFT, "
                      f"wall {wall:.2f} s"}


# ---------------------------------------------------------------------------
# Algorithmic bytes of each kernel class over one step (units of N*b).
# Mirrors the library's schedules: tiles of up to 16 x 16 pairs in FP64 and
# 32 x 32 in FP32 (pair_tile); one orbital
# block at q = 0 runs the pair-symmetric schedule (tiles I <= J, diagonal
# tiles holding only the pairs ii <= jj): FP64 planes up to 64 wide use a
# fused inverse + multiply-accumulate for each mirror half (the transform is
# recomputed, nothing written back), FP32 and wider FP64 planes the parallel
# in-place inverse plus one pair multiply-accumulate.
# ---------------------------------------------------------------------------
def sym_schedule(fp64, n3):
    """The library's default for one block applied to itself (FOCK_SYM_SCHEDULE overrides)."""
    env = os.environ.get("FOCK_SYM_SCHEDULE")
    if env in ("0", "1", "2"):
        return int(env)
    return 2 if fp64 and n3 <= 64 else 1


def live_fraction(miller, n):
    """Fraction of the (i2, i3) plane columns a pair density can occupy (its
    support S - S projected on the plane axes): the pair-buffer entries P1
    stores and P2 and the predicated P3 passes read.  1.0 when S - S wraps on
    the grid (reduced-cutoff grids), where every column is kept."""
    n2, n3 = n[1], n[2]
    rows = {}
    for m2, m3 in zip(miller[:, 1].tolist(), miller[:, 2].tolist()):
        lo, hi = rows.get(m3, (m2, m2))
        rows[m3] = (min(lo, m2), max(hi, m2))
    h = {}
    for a, (loa, hia) in rows.items():
        for b, (lob, hib) in rows.items():
            d3 = a - b
            h[d3] = max(h.get(d3, -1), hia - lob, hib - loa)
    col = [-1] * n3
    for d3, v in h.items():
        if 2 * abs(d3) > n3 - 1 or 2 * v > n2 - 1:
            return 1.0
        col[d3 % n3] = v
    live = sum(1 for i3 in range(n3) for i2 in range(n2) if i2 <= col[i3] or i2 >= n2 - col[i3])
    return live / (n2 * n3)


def pair_flops(n):
    """Algorithmic flops per pair and grid point of each kernel class, with the
    usual 5 L log2 L count of a complex transform of length L: a complex
    product is 6 flops, a complex multiply-add 8, a real scale 2."""
    lp = float(np.log2(n[1] * n[2]))
    l1 = float(np.log2(n[0]))
    return {"p1_pair_plane_fwd": 6 + 5 * lp,        # conj(phi) psi, forward plane transform
            "p2_pencil_kernel": 10 * l1 + 2,        # forward pencil transform, x K, backward
            "p3_inplace": 5 * lp,                   # backward plane transform
            "p3_fused": 5 * lp + 8,                 # backward plane transform, f phi v accumulated
            "mac_half": 8}                          # one f phi v (or conj) accumulation


def step_bytes(nb, N, bpc, fp64, sym=True, sched=None, lf=1.0, n=None, flops=None):
    """Algorithmic bytes (and, with n and a dict `flops`, flops) of each kernel
    class over one step: {class: [bytes, launches]}."""
    T = balanced_edge(nb, pair_tile(fp64))
    if sched is None:
        sched = 2 if fp64 else 1
    acc = {}
    pf = pair_flops(n) if n is not None else None

    def add(k, rd, wr, n=1, fl=0.0):
        a = acc.setdefault(k, [0.0, 0])
        a[0] += (rd + wr) * N * bpc
        a[1] += n
        if flops is not None:
            flops[k] = flops.get(k, 0.0) + fl * N

    for j0 in range(0, nb, T):
        tj = min(T, nb - j0)
        for i0 in range(0, (j0 + 1) if sym else nb, T):
            ti = min(T, nb - i0)
            diag = sym and i0 == j0
            # diagonal tiles of schedules 1 and 2 hold only the pairs ii <= jj
            tri = diag and sched != 0
            npr = ti * (ti + 1) // 2 if tri else ti * tj
            # P1 stores and P2 reads only the live columns (fraction lf); P2
            # writes the dead columns' zeros only for the fused P3 passes
            # (schedules 0 and 2), which read every column
            f = pf or {k: 0.0 for k in ("p1_pair_plane_fwd", "p2_pencil_kernel", "p3_inplace", "p3_fused", "mac_half")}
            nmir = (ti * (ti - 1) // 2 if tri else 0) if diag else ti * tj  # pairs of the mirror half
            add("p1_pair_plane_fwd", ti + (0 if diag else tj), npr * lf, fl=npr * f["p1_pair_plane_fwd"])
            add("p2_pencil_kernel", npr * lf, npr * lf if sym and sched == 1 else npr, fl=npr * f["p2_pencil_kernel"])
            if not sym:
                add("p3_plane_inv_mac", ti * tj + ti + tj, tj, fl=npr * f["p3_fused"])
            elif sched in (0, 2):  # fused P3 into acc_J; mirror: recomputed (2) or from v written back (0)
                add("p3_plane_inv_mac", npr + ti + tj, tj + (ti * tj if sched == 0 and not diag else 0),
                    fl=npr * f["p3_fused"])
                mfl = nmir * (f["p3_fused"] if sched == 2 else f["mac_half"])
                if not diag:
                    add("p3_second", ti * tj + tj + ti, ti, fl=mfl)
                elif tri and ti > 1:
                    add("p3_second", ti * (ti - 1) // 2 + tj + ti, ti, fl=mfl)
            else:  # schedule 1: in-place inverse (reads the live columns), one MAC for both halves
                add("p3_plane_inv_mac", npr * lf, npr, fl=npr * f["p3_inplace"])
                add("p3_second", npr + ti + (0 if diag else tj) + tj + ti, tj + (0 if diag and not tri else ti),
                    fl=(npr + nmir) * f["mac_half"])
    return acc


def gamma_step_bytes(n, N, bpc, ti_max=16, tj_max=8, lf=1.0):
    """Algorithmic bytes per step of the Gamma apply (packed tiles of 16 real
    occupied x 8 packed targets, only tiles holding a pair i <= j)."""
    acc = {}

    def add(k, rd, wr):
        a = acc.setdefault(k, [0.0, 0])
        a[0] += (rd + wr) * N * bpc
        a[1] += 1

    m = (n + 1) // 2
    for j0 in range(0, m, tj_max):
        tj = min(tj_max, m - j0)
        for i0 in range(0, n, ti_max):
            if i0 > 2 * (j0 + tj) - 1:
                break
            ti = min(ti_max, n - i0)
            pi = (ti + 1) // 2  # packed planes holding the tile's occupied orbitals
            # diagonal tile: only the pairs i <= 2q + 1 (non-zero weight)
            npr = sum(min(ti, 2 * jj + 2) for jj in range(tj)) if i0 == 2 * j0 else ti * tj
            add("p1_pair_plane_fwd", pi + tj, npr * lf)
            add("p2_pencil_kernel", npr * lf, npr * lf)  # both Gamma schedules mask the dead columns
            add("p3_plane_inv_mac", npr * lf + pi + tj, tj)
            add("p3_second", npr * lf + tj + pi, pi)
    return acc


def band_step_bytes(nb, N, npw, bpc, force, chunk=64, groups=8):
    """Algorithmic bytes per step of the band loops (chunks of 64 bands, 8 band
    groups per plane), per kernel class."""
    acc = {}

    def add(k, nbytes):
        a = acc.setdefault(k, [0.0, 0])
        a[0] += nbytes
        a[1] += 1

    for b0 in range(0, nb, chunk):
        n = min(chunk, nb - b0)
        add("a1_scatter", n * N * bpc + 2 * n * npw * bpc + npw * 4)  # clear, coefficients in and out, slots
        add("a1_pencil_inv", 2 * n * N * bpc)
        if force:
            add("band_plane_vmul", 2 * n * N * bpc + groups * N * bpc // 2)  # V once per band group
            add("a7_pencil_fwd", 2 * n * N * bpc)
            add("band_force_gather", 3 * n * npw * bpc + npw * 4)
        else:
            add("band_plane_density", n * N * bpc + groups * N * 8 * (2 if b0 else 1))
    if not force:
        add("reduce", (groups + 1) * N * 8)
    return acc


def sources_sha():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1305_7313_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".h", ".hip", ".cpp")):
            with open(os.path.join(csrc, name), "rb") as fh:
                h.update(name.encode())
                h.update(fh.read())
    return h.hexdigest()


def pmc_traffic(workload, kernel_class):
    """HBM bytes per launch from the committed counter summary, if it was taken on these sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_sha256") != sources_sha():
        return None
    k = rec.get("kernels", {}).get(kernel_class)
    if not k:
        return None
    return round(1024.0 * (k["fetch_kib"] * rec["fetch_scale"] + k["write_kib"] * rec["write_scale"]))


def log(msg):
    """Progress line on stderr (stdout carries only the JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_steps(step, steps, warmup):
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    log(f"{warmup} warmup step(s) done")
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log(f"{steps} timed step(s): {1e3 * dt / max(steps, 1):.2f} ms per step")
    return dt


def traced(fock, step, steps):
    import torch
    fock.fock_trace_enable(True)
    fock.fock_trace_read(reset=True)
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    tr = fock.fock_trace_read(reset=True)
    fock.fock_trace_enable(False)
    return tr


# A kernel class is set against the vector-ALU roofline when its algorithmic
# intensity (flops per byte moved) lies above the ridge point of the two
# peaks, else against HBM.  In FP32 only the pair pass (P1), which reads its
# two operands from cache and writes one pair buffer, lies above the ridge.
RIDGE_FLOP_PER_BYTE = VALU_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)


_COPY_GBS = None


def copy_gbs():
    """HBM rate of a plain device-to-device copy on this GPU (1 GiB, bytes
    read + written over the time of one copy, best of five), measured once:
    the practical ceiling the streaming passes are compared with."""
    global _COPY_GBS
    if _COPY_GBS is None:
        import torch
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        best = None
        for _ in range(5):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            dst.copy_(src)
            b.record()
            b.synchronize()
            ms = a.elapsed_time(b)
            best = ms if best is None else min(best, ms)
        del src, dst
        torch.cuda.empty_cache()
        _COPY_GBS = 2.0 * (1 << 30) / (best * 1e-3) / 1e9
    return _COPY_GBS


def roofline(tr, acc, steps, workload, fp64=True, flops=None):
    """The dominant kernel class (most time) against its roofline: HBM bytes
    per launch over the launch time, or for an ALU-bound class algorithmic
    flops over the launch time against the vector-ALU peak.  Both rates are
    reported, and the HBM rate also against a plain device copy."""
    pair_cls = [k for k in acc if k in tr and tr[k][1]]
    dom = max(pair_cls, key=lambda k: tr[k][0])
    ms, launches = tr[dom]
    per_launch = acc[dom][0] * steps / launches
    avg_ms = ms / launches
    gbs = per_launch / (avg_ms * 1e-3) / 1e9
    rec = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": pmc_traffic(workload, dom), "kernel": dom,
           "avg_launch_ms": round(avg_ms, 5), "bytes_per_launch": round(per_launch),
           "hbm_gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
    cg = copy_gbs()
    rec.update({"copy_gbs": round(cg, 1), "hbm_vs_copy": round(gbs / cg, 4)})
    # every pair-pass class: algorithmic HBM rate over its summed launch time
    rec["classes"] = {k: {"ms": round(tr[k][0], 3), "gbs": round(acc[k][0] * steps / (tr[k][0] * 1e-3) / 1e9, 1),
                          "vs_copy": round(acc[k][0] * steps / (tr[k][0] * 1e-3) / 1e9 / cg, 3)}
                      for k in pair_cls}
    if flops and dom in flops:
        fl_launch = flops[dom] * steps / launches
        tfs = fl_launch / (avg_ms * 1e-3) / 1e12
        rec.update({"flops_per_launch": round(fl_launch), "valu_tflops": round(tfs, 2),
                    "valu_frac": round(tfs / VALU_PEAK_TFLOPS, 4)})
        rec["flop_per_byte"] = round(fl_launch / per_launch, 2)
        if fl_launch / per_launch > RIDGE_FLOP_PER_BYTE:
            rec.update({"bound": "alu", "achieved": round(tfs, 2), "peak": round(VALU_PEAK_TFLOPS, 1),
                        "unit": "TFLOP/s", "frac": round(tfs / VALU_PEAK_TFLOPS, 4)})
    return rec


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------
def single_block(name, args, cpu):
    import torch
    from paper_1305_7313_amd import fock
    if name.startswith("c2"):
        s, c = synth.config2()
    else:
        s, c = synth.config3()
    fp64 = name.endswith("fp64")
    # reduced Fock cutoff: E_fock = E_wfc on the coarsest grid that keeps the result exact
    ecut = s.ecut if name[2] == "r" else 0.0
    n = tuple(s.n)
    if ecut > 0.0:
        n = fock.fock_exchange_grid(fock.Cell(s.a, s.n, s.miller, ecut_fock=ecut),
                                    dtype=fock.FOCK_C128 if fp64 else fock.FOCK_C64)
    nb, N = c.shape[0], n[0] * n[1] * n[2]
    bpc = 16 if fp64 else 8
    if cpu:
        cpu = cpu_baseline(s, c, n, ecut)
    dev = torch.device("cuda:0")
    cdt = torch.complex128 if fp64 else torch.complex64
    cd = torch.from_numpy(c).to(cdt).to(dev)
    f = torch.ones(nb, dtype=torch.float64, device=dev)
    cell = fock.Cell(s.a, n, s.miller, ecut_fock=ecut)
    out = torch.empty((nb, s.npw), dtype=cdt, device=dev)
    ws = fock.workspace(cell, fock.dtype_code(cd), nb, nb, dev)

    def step():
        fock.fock_apply(cell, (0.0, 0.0, 0.0), cd, f, cd, out=out, ws=ws)

    dt = run_steps(step, args.steps, args.warmup)
    pairs = nb * nb
    rec = {"value": pairs * args.steps / dt, "ms_per_step": 1e3 * dt / args.steps, "dtype": "f64" if fp64 else "f32",
           "config": {"workload": name, "description": WORKLOADS[name], "grid": list(n), "npw": s.npw,
                      "ecut_fock": ecut if ecut > 0.0 else None,
                      "n_occ": nb, "n_tgt": nb, "pairs_per_step": pairs,
                      "pair_symmetry": "rho_ji = conj(rho_ij) reused; pairs counted as n_occ x n_tgt"},
           "cpu_baseline": cpu or None}
    rec["logical_hbm_gbs"] = round(rec["value"] * 4 * N * bpc / 1e9, 1)
    # whole path against the HBM peak at the floor of 4 N b per pair (read both
    # orbitals, read and write the accumulator)
    rec["logical_frac"] = round(rec["logical_hbm_gbs"] / HBM_PEAK_GBS, 4)
    if not args.no_trace:
        tr = traced(fock, step, args.steps)
        fl = {}
        acc = step_bytes(nb, N, bpc, fp64, sched=sym_schedule(fp64, n[2]), lf=live_fraction(s.miller, n), n=n,
                         flops=fl)
        rec["roofline"] = roofline(tr, acc, args.steps, name, fp64=fp64, flops=fl)
        rec["kernels"] = {k: {"ms_per_step": round(v[0] / args.steps, 4), "launches_per_step": v[1] / args.steps}
                          for k, v in tr.items() if v[1]}
    return rec


def gamma_block(name, args, cpu):
    import torch
    from paper_1305_7313_amd import fock
    s, _ = synth.config2(nb=1)
    c = synth.gamma_orbitals(s.a, s.miller, 128, 0)
    nb, N = c.shape[0], s.n[0] * s.n[1] * s.n[2]
    if cpu:
        cpu = cpu_baseline(s, c)
    cd = torch.from_numpy(c).cuda()
    f = torch.ones(nb, dtype=torch.float64, device="cuda")
    cell = fock.Cell(s.a, s.n, s.miller)
    out = torch.empty((nb, s.npw), dtype=torch.complex128, device="cuda")
    ws = torch.empty(int(fock.lib().fock_workspace_size_gamma(fock.ctypes.byref(cell.c), fock.FOCK_C128, nb)),
                     dtype=torch.uint8, device="cuda")

    def step():
        fock.fock_apply_gamma(cell, cd, f, out=out, ws=ws)

    dt = run_steps(step, args.steps, args.warmup)
    # the general path on the same real orbitals, for comparison
    out2 = torch.empty_like(out)
    ws2 = fock.workspace(cell, fock.FOCK_C128, nb, nb, cd.device)
    dt2 = run_steps(lambda: fock.fock_apply(cell, (0.0, 0.0, 0.0), cd, f, cd, out=out2, ws=ws2), args.steps, 1)
    diff = float(torch.linalg.vector_norm(out - out2) / torch.linalg.vector_norm(out2))
    pairs = nb * nb
    rec = {"value": pairs * args.steps / dt, "ms_per_step": 1e3 * dt / args.steps, "dtype": "f64",
           "config": {"workload": name, "description": WORKLOADS[name], "grid": list(s.n), "npw": s.npw,
                      "n_occ": nb, "n_tgt": nb, "pairs_per_step": pairs,
                      "pair_symmetry": "real orbitals packed two per transform and rho_ji = rho_ij reused; pairs "
                                       "counted as n_occ x n_tgt"},
           "general_path_ms_per_step": round(1e3 * dt2 / args.steps, 3), "gamma_vs_general_rel": diff,
           "cpu_baseline": cpu or None}
    if not args.no_trace:
        tr = traced(fock, step, args.steps)
        rec["roofline"] = roofline(tr, gamma_step_bytes(nb, N, 16, lf=live_fraction(s.miller, s.n)), args.steps, name)
        rec["kernels"] = {k: {"ms_per_step": round(v[0] / args.steps, 4), "launches_per_step": v[1] / args.steps}
                          for k, v in tr.items() if v[1]}
    return rec


def tile_bytes(lf, e=32):
    """Algorithmic bytes per launch of each class on full e x e tiles (units
    of N*b), for the k-mesh workload in FP32 (schedule 1): P3 is the in-place
    inverse plane FFT of the tile, the second pass the streaming MAC of both
    halves (pair buffer, both orbital tiles, both accumulator tiles read and
    written).  lf: live fraction of the pair-buffer columns."""
    p = e * e
    return {"p1_pair_plane_fwd": 2 * e + p * lf, "p2_pencil_energy": p * lf, "p2_pencil_kernel": 2 * p * lf,
            "p3_plane_inv_mac": p * lf + p, "p3_second": p + 2 * e + 4 * e}


def tile_flops(n, e=32):
    """Algorithmic flops per launch and grid point of each class on full e x e
    tiles, for the k-mesh workload (pair_flops per pair times e^2 pairs; the
    streaming MAC accumulates both halves)."""
    pf = pair_flops(n)
    l1 = float(np.log2(n[0]))
    p = e * e
    return {"p1_pair_plane_fwd": p * pf["p1_pair_plane_fwd"], "p2_pencil_kernel": p * pf["p2_pencil_kernel"],
            "p2_pencil_energy": p * (5 * l1 + 4), "p3_plane_inv_mac": p * pf["p3_inplace"],
            "p3_second": p * 2 * pf["mac_half"]}


def kmesh_grad(name, args, cpu):
    import torch
    from paper_1305_7313_amd import fock
    s, kpts, orbs = synth.config5()
    nk, nb = len(orbs), orbs[0].shape[0]
    N = s.n[0] * s.n[1] * s.n[2]
    if cpu:
        cpu = cpu_baseline(s, orbs[0])
    n, ecut = tuple(s.n), 0.0
    if name.startswith("c5r"):
        ecut = s.ecut
        qs = [ki - kj for ki in kpts for kj in kpts]
        n = fock.fock_exchange_grid(fock.Cell(s.a, s.n, s.miller, ecut_fock=ecut), qs, dtype=fock.FOCK_C64)
        N = n[0] * n[1] * n[2]
    cell = fock.Cell(s.a, n, s.miller, ecut_fock=ecut, g0=fock.FOCK_G0_GB, gb_alpha=10.0 / s.ecut, nq=(2, 2, 2))
    C = torch.from_numpy(np.stack(orbs)).to(torch.complex64).cuda()
    W = torch.full((nk, nb), 1.0 / nk, dtype=torch.float64, device="cuda")
    ws = fock.workspace_kmesh(cell, fock.FOCK_C64, nk, nb, C.device)
    ex = torch.empty((), dtype=torch.float64, device="cuda")
    G = torch.empty_like(C)

    def step():
        fock.fock_energy_kmesh_grad(cell, kpts, C, W, grad=G, out=ex, ws=ws)

    # one step takes tens of seconds: at most 2 timed steps after 1 warmup
    steps, warmup = min(args.steps, 2), min(args.warmup, 1)
    dt = run_steps(step, steps, warmup)
    pairs = nk * nk * nb * nb
    rec = {"value": pairs * steps / dt, "ms_per_step": 1e3 * dt / steps, "dtype": "f32", "steps": steps,
           "warmup": warmup,
           "config": {"workload": name, "description": WORKLOADS[name], "grid": list(n), "npw": s.npw,
                      "ecut_fock": ecut if ecut > 0.0 else None, "kpoints": nk, "bands_per_k": nb, "pairs_per_step": pairs,
                      "step": "E_x over the mesh and dE/dconj(C) from one pass over the pairs "
                              "(fock_energy_kmesh_grad: each pair of the blocks k < k' transformed once for "
                              "both gradients, E = 1/2 Re <C, dE/dconj(C)>)"},
           "cpu_baseline": cpu or None}
    if not args.no_trace:
        tr = traced(fock, step, 1)
        tb = tile_bytes(live_fraction(s.miller, n))
        acc = {k: [tb[k] * N * 8 * tr[k][1], tr[k][1]] for k in tb if k in tr and tr[k][1]}
        tf = tile_flops(n)
        fl = {k: tf[k] * N * tr[k][1] for k in tf if k in tr and tr[k][1]}
        rec["roofline"] = roofline(tr, acc, 1, name, fp64=False, flops=fl)
        rec["kernels"] = {k: {"ms_per_step": round(v[0], 4), "launches_per_step": v[1]} for k, v in tr.items() if v[1]}
    return rec


def band_loops(name, args, cpu):
    import torch
    from paper_1305_7313_amd import fock
    s, c = synth.config3()
    force = "force" in name
    nb, N = c.shape[0], s.n[0] * s.n[1] * s.n[2]
    w = np.full(nb, 2.0)
    v = np.random.default_rng(20).standard_normal(s.n)
    if cpu:
        cpu = cpu_baseline_bands(s, c, w, v, force)
    cd = torch.from_numpy(c).cuda()
    wd = torch.from_numpy(w).cuda()
    vd = torch.from_numpy(v).cuda()
    cell = fock.Cell(s.a, s.n, s.miller)
    ws = fock.band_workspace(cell, fock.FOCK_C128, nb, cd.device)
    rho = torch.empty(s.n, dtype=torch.float64, device="cuda")
    out = torch.empty_like(cd)

    def step():
        if force:
            fock.fock_band_force(cell, (0.0, 0.0, 0.0), cd, wd, vd, out=out, ws=ws)
        else:
            fock.fock_band_density(cell, cd, wd, out=rho, ws=ws)

    dt = run_steps(step, args.steps, args.warmup)
    rec = {"metric": "CP band-loop bands/sec at 1 GPU", "unit": "bands/s", "value": nb * args.steps / dt,
           "ms_per_step": 1e3 * dt / args.steps, "dtype": "f64",
           "config": {"workload": name, "description": WORKLOADS[name], "grid": list(s.n), "npw": s.npw,
                      "bands": nb}, "cpu_baseline": cpu or None}
    if not args.no_trace:
        tr = traced(fock, step, args.steps)
        acc = band_step_bytes(nb, N, s.npw, 16, force)
        rec["roofline"] = roofline(tr, acc, args.steps, name)
        rec["kernels"] = {k: {"ms_per_step": round(v[0] / args.steps, 4), "launches_per_step": v[1] / args.steps}
                          for k, v in tr.items() if v[1]}
    return rec


def batch_inputs():
    return [synth.config4_system(k) for k in range(16)]


def c4_batched(steps, warmup, systems, tune_cache):
    """FP32-batched: every system of the batch in one hipGraph replay."""
    import torch
    from paper_1305_7313_amd import fock
    cells, C, W = [], [], []
    for s, c in systems:
        cells.append(fock.Cell(s.a, s.n, s.miller))
        C.append(torch.from_numpy(c).to(torch.complex64).cuda())
        W.append(torch.ones(c.shape[0], dtype=torch.float64, device="cuda"))
    t0 = time.perf_counter()
    plan = fock.BatchPlan(cells, C, W, tune_cache=tune_cache)
    create_s = time.perf_counter() - t0
    dt = run_steps(plan.apply, steps, warmup)
    plan.check()
    pairs = sum(c.shape[0] ** 2 for _, c in systems)
    gp = sum(c.shape[0] ** 2 * s.n[0] ** 3 for s, c in systems)
    outs = [o.detach().to(torch.complex128) for o in plan.outs]
    info = plan.info()
    plan.close()
    return {"value": pairs * steps / dt, "ms_per_step": 1e3 * dt / steps,
            "gridpoint_pairs_per_s": gp * steps / dt, "pairs_per_step": pairs,
            "schedule": info, "plan_create_s": round(create_s, 2)}, outs


def c4_plain(steps, warmup, systems, fp32=False, trace=False):
    """One fock_apply per system (FP64, or FP32 with fp32=True); with trace,
    a further pass records every launch with HIP events on its stream."""
    import torch
    from paper_1305_7313_amd import fock
    cdt = torch.complex64 if fp32 else torch.complex128
    items = []
    for s, c in systems:
        cell = fock.Cell(s.a, s.n, s.miller)
        cd = torch.from_numpy(c).to(cdt).cuda()
        f = torch.ones(c.shape[0], dtype=torch.float64, device="cuda")
        out = torch.empty((c.shape[0], s.npw), dtype=cdt, device="cuda")
        ws = fock.workspace(cell, fock.dtype_code(cd), c.shape[0], c.shape[0], cd.device)
        items.append((cell, cd, f, out, ws))

    def step():
        for cell, cd, f, out, ws in items:
            fock.fock_apply(cell, (0.0, 0.0, 0.0), cd, f, cd, out=out, ws=ws)

    dt = run_steps(step, steps, warmup)
    pairs = sum(c.shape[0] ** 2 for _, c in systems)
    gp = sum(c.shape[0] ** 2 * s.n[0] ** 3 for s, c in systems)
    rec = {"value": pairs * steps / dt, "ms_per_step": 1e3 * dt / steps,
           "gridpoint_pairs_per_s": gp * steps / dt, "pairs_per_step": pairs}
    tr = traced(fock, step, 1) if trace else None
    return rec, [it[3] for it in items], [it[1] for it in items], tr


def batch_step_model(systems, fp64):
    """Algorithmic bytes and flops of each kernel class over one apply of
    every system (each system's own schedule, as the per-shape graph runs it)."""
    acc, fl = {}, {}
    bpc = 16 if fp64 else 8
    for s, c in systems:
        n = tuple(s.n)
        N = n[0] * n[1] * n[2]
        a = step_bytes(c.shape[0], N, bpc, fp64, sched=sym_schedule(fp64, n[2]), lf=live_fraction(s.miller, n),
                       n=n, flops=fl)
        for k, (b, l) in a.items():
            e = acc.setdefault(k, [0.0, 0])
            e[0] += b
            e[1] += l
    return acc, fl


# CPU baseline of the batch: per-system sub-blocks timed on the host cores
def _c4_cpu_init():
    os.environ["OMP_NUM_THREADS"] = "1"


def _c4_cpu_task(args):
    from oracle import exx
    k, a, n, miller, c_occ, c_tgt = args
    t0 = time.perf_counter()
    exx.fock_apply(a, n, miller, np.zeros(3), c_occ, np.ones(c_occ.shape[0]), c_tgt)
    return k, c_occ.shape[0] * c_tgt.shape[0], time.perf_counter() - t0


def cpu_workers(ntasks):
    """Worker processes for the oracle baselines: every core of this process's
    affinity mask, at most 16 (one GPU's share of the host) and at most one
    per task."""
    return max(1, min(len(os.sched_getaffinity(0)), 16, ntasks))


def cpu_baseline_batch(systems, nocc=48):
    """The oracle on every system of the batch: target 0 against the first
    `nocc` occupied orbitals, one task per system, on the host cores.  The
    per-pair time of each system, weighted by its n_occ x n_tgt pairs, gives
    the whole-batch rate the host would reach (an extrapolation)."""
    tasks = [(k, s.a, tuple(s.n), s.miller, c[:nocc], c[:1]) for k, (s, c) in enumerate(systems)]
    workers = cpu_workers(len(tasks))
    log(f"CPU oracle baseline: {workers} processes, {len(tasks)} tasks")
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers, initializer=_c4_cpu_init) as pool:
        pool.map(abs, range(workers))
        t0 = time.perf_counter()
        res = pool.map(_c4_cpu_task, tasks)
        wall = time.perf_counter() - t0
    per_pair = {k: t / npairs for k, npairs, t in res}
    total_pairs = sum(c.shape[0] ** 2 for _, c in systems)
    serial_s = sum(c.shape[0] ** 2 * per_pair[k] for k, (_, c) in enumerate(systems))
    sample_pairs = sum(npairs for _, npairs, _ in res)
    cpu_s = sum(t for _, _, t in res)
    return {"value": round(total_pairs * workers / serial_s, 2), "unit": UNIT, "cores": workers,
            "affinity_cores": len(os.sched_getaffinity(0)), "kind": "oracle", "cpu": cpu_model(),
            "sample": f"each of the 16 systems: target 0 against its first {nocc} occupied orbitals "
                      f"({sample_pairs} pairs, {cpu_s:.1f} s of single-threaded FP64 scipy FFT work, one task per "
                      f"system, wall {wall:.2f} s on {workers} processes); whole-batch rate extrapolated from "
                      f"each system's time per pair weighted by its n_occ x n_tgt pairs, over {workers} cores"}


def c4_headline(args):
    """The metric's own workload: the 16-system batch in FP32, one hipGraph
    replay per step, against the FP64 plain form (one fock_apply per system)
    and the FP32 plain form on the same systems."""
    import torch
    systems = batch_inputs()
    log("FP32 batched")
    b32, outs32 = c4_batched(args.steps, args.warmup, systems, args.tune_cache)
    mode = b32["schedule"].get("mode")
    side = max(1, min(args.steps, 3))
    log("FP64 plain")
    p64, outs64, coeffs, _ = c4_plain(side, 1, systems)
    log("FP32 plain")
    p32, _, _, tr = c4_plain(side, 1, systems, fp32=True, trace=not args.no_trace)
    num = sum(float(torch.linalg.vector_norm(a - b) ** 2) for a, b in zip(outs32, outs64))
    den = sum(float(torch.linalg.vector_norm(b) ** 2) for b in outs64)
    # E_x = 1/2 sum_j <psi_j | V_x psi_j> (f = 1, one block per system)
    e32 = sum(0.5 * float(torch.sum(torch.conj(c) * o).real) for c, o in zip(coeffs, outs32))
    e64 = sum(0.5 * float(torch.sum(torch.conj(c) * o).real) for c, o in zip(coeffs, outs64))
    how = ("each system's per-shape kernel schedule, captured one after another in one hipGraph"
           if mode == "kernels" else "one persistent kernel over every stage of every system, in one hipGraph")
    rec = {"value": b32["value"], "ms_per_step": b32["ms_per_step"], "dtype": "f32",
           "config": {"workload": "c4_fp32_batched", "description": WORKLOADS["c4_fp32_batched"],
                      "schedule_run": how, "systems": 16, "pairs_per_step": b32["pairs_per_step"],
                      "pair_symmetry": "rho_ji = conj(rho_ij) reused; pairs counted as n_occ x n_tgt"},
           "schedule": b32["schedule"], "plan_create_s": b32["plan_create_s"],
           "gridpoint_pairs_per_s": round(b32["gridpoint_pairs_per_s"]),
           "fp64_plain": {k: (round(v, 2) if isinstance(v, float) else v) for k, v in p64.items()},
           "fp32_plain": {k: (round(v, 2) if isinstance(v, float) else v) for k, v in p32.items()},
           "speedup_vs_fp64_plain": round(b32["value"] / p64["value"], 3),
           "speedup_vs_fp32_plain": round(b32["value"] / p32["value"], 3),
           "fp32_vs_fp64_vx_rel": float(np.sqrt(num / den)), "fp32_vs_fp64_ex_rel": abs(e32 - e64) / abs(e64),
           "ex_fp64": e64, "ex_fp32": e32}
    if tr is not None:
        acc, fl = batch_step_model(systems, fp64=False)
        rf = roofline(tr, acc, 1, "c4_fp32_batched", fp64=False, flops=fl)
        rf["measured_on"] = ("the per-shape kernels of every system, launched eagerly with HIP events on their "
                             "stream (the kernels the graph replays)")
        rec["roofline"] = rf
        rec["kernels"] = {k: {"ms_per_step": round(v[0], 4), "launches_per_step": v[1]} for k, v in tr.items() if v[1]}
    return rec, systems


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c4_fp32_batched", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-trace", action="store_true")
    ap.add_argument("--no-compare", action="store_true",
                    help="the batched workload without the config-2 FP64 record beside it")
    ap.add_argument("--tune-cache", default=os.path.join(tempfile.gettempdir(), "fock_tune_cache.json"),
                    help="tuned batch schedules (a missing file is seeded from the committed tune seed)")
    ap.add_argument("--no-tune-seed", action="store_true",
                    help="do not seed a missing tune cache from the committed one (forces a fresh tuning)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain device copy of known size (bandwidth-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the exchange path runs on one GPU (no sharded form here); --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    os.makedirs(os.path.dirname(args.tune_cache), exist_ok=True)
    seed_cache = os.path.join(ROOT, "paper_1305_7313_amd", "tune_seed.json")
    if not args.no_tune_seed and not os.path.exists(args.tune_cache) and os.path.exists(seed_cache):
        shutil.copyfile(seed_cache, args.tune_cache)

    wl = args.workload
    log(f"workload {wl}")
    rec = {"metric": METRIC, "unit": UNIT, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "data": "synthetic"}
    if wl in ("c2_fp64", "c3_fp32", "c3_fp64", "c2r_fp64", "c3r_fp32"):
        r = single_block(wl, args, cpu=not args.no_cpu_baseline)
    elif wl in ("c5_fp32_grad", "c5r_fp32_grad"):
        r = kmesh_grad(wl, args, cpu=not args.no_cpu_baseline)
    elif wl == "c2g_fp64":
        r = gamma_block(wl, args, cpu=not args.no_cpu_baseline)
    elif wl.startswith("cp_"):
        r = band_loops(wl, args, cpu=not args.no_cpu_baseline)
    elif wl == "c4_fp32_batched":
        r, systems = c4_headline(args)
        if not args.no_cpu_baseline:
            r["cpu_baseline"] = cpu_baseline_batch(systems)
    else:
        import torch  # noqa: F401
        r, _, _, tr = c4_plain(args.steps, args.warmup, batch_inputs(), trace=not args.no_trace)
        r["dtype"] = "f64"
        r["config"] = {"workload": wl, "description": WORKLOADS[wl], "pairs_per_step": r["pairs_per_step"]}
        if tr is not None:
            acc, fl = batch_step_model(batch_inputs(), fp64=True)
            r["roofline"] = roofline(tr, acc, 1, wl, fp64=True, flops=fl)
    if args.copy_probe:
        import torch
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
    rec.update({k: v for k, v in r.items() if k not in ("pairs_per_step",)})
    rec["value"] = round(rec["value"], 1)
    rec["ms_per_step"] = round(rec["ms_per_step"], 3)
    if not args.no_compare and wl == "c4_fp32_batched":
        # config 2 (64^3 FP64, 128 orbitals) beside the headline, as a second record
        log("config 2 FP64 record")
        c2 = single_block("c2_fp64", args, cpu=False)
        rec["c2_fp64"] = {k: v for k, v in c2.items() if k in ("value", "ms_per_step", "dtype", "roofline",
                                                                 "logical_hbm_gbs")}
        rec["c2_fp64"]["config"] = {k: c2["config"][k] for k in ("workload", "description", "pairs_per_step")}
    order = ["metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
             "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"]
    out = {k: rec[k] for k in order if k in rec}
    out.update({k: v for k, v in rec.items() if k not in out})
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
