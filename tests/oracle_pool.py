"""Runs oracle sub-blocks of the full-size workloads in worker processes.

Workers are spawned (fresh interpreters that never touch the GPU) and rebuild
their inputs from the seeded generator, so nothing large crosses process
boundaries.  The occupied sum is split into chunks whose partial results add
up to the full apply (the band-group split sum pinned in the oracle tests).
"""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np

_CACHE = {}
C3Q_SHIFT = (0.05, -0.03, 0.02)  # bohr^-1


def _workload(name):
    import synth
    if name not in _CACHE:
        if name == "c2":
            s, c = synth.config2()
            _CACHE[name] = (s, {0: c}, {0: np.zeros(3)})
        elif name == "c3":
            s, c = synth.config3()
            _CACHE[name] = (s, {0: c}, {0: np.zeros(3)})
        elif name == "c3q":
            # config 3's orbitals as two sets: targets at k = C3Q_SHIFT, occupied at k = 0
            s, c = synth.config3()
            _CACHE[name] = (s, {0: c, 1: c}, {0: np.array(C3Q_SHIFT), 1: np.zeros(3)})
        elif name == "c5":
            s, kpts, orbs = synth.config5()
            _CACHE[name] = (s, dict(enumerate(orbs)), dict(enumerate(kpts)))
        elif name.startswith("c4:"):
            s, c = synth.config4_system(int(name[3:]))
            _CACHE[name] = (s, {0: c}, {0: np.zeros(3)})
        else:
            raise KeyError(name)
    return _CACHE[name]


def _apply_task(args):
    os.environ["OMP_NUM_THREADS"] = "1"
    from oracle import exx
    name, kt, ko, targets, occ_lo, occ_hi, weight, k0 = args
    s, sets, kp = _workload(name)
    q = kp[kt] - kp[ko]
    occ = sets[ko][occ_lo:occ_hi]
    return exx.fock_apply(s.a, s.n, s.miller, q, occ, np.full(occ.shape[0], weight), sets[kt][targets], k0=k0)


def _energy_task(args):
    os.environ["OMP_NUM_THREADS"] = "1"
    from oracle import exx
    name, kt, ko, tgt_lo, tgt_hi, occ_lo, occ_hi, weight, k0 = args
    s, sets, kp = _workload(name)
    q = kp[kt] - kp[ko]
    occ = sets[ko][occ_lo:occ_hi]
    tgt = sets[kt][tgt_lo:tgt_hi]
    return exx.fock_energy(s.a, s.n, s.miller, q, occ, np.full(occ.shape[0], weight), tgt,
                           np.full(tgt.shape[0], weight), k0=k0)


def workers() -> int:
    return max(1, min(16, len(os.sched_getaffinity(0))))


_SINGLE = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "BLIS_NUM_THREADS")


def _run(fn, tasks, label):
    """Map tasks over spawned single-threaded workers, printing one line per finished task."""
    saved = {k: os.environ.get(k) for k in _SINGLE}
    for k in _SINGLE:
        os.environ[k] = "1"
    try:
        out = [None] * len(tasks)
        with mp.get_context("spawn").Pool(min(workers(), len(tasks))) as pool:
            for done, (i, r) in enumerate(pool.imap_unordered(_indexed, [(fn, i, t) for i, t in enumerate(tasks)])):
                out[i] = r
                print(f"[oracle] {label}: {done + 1}/{len(tasks)} tasks done", flush=True)
        return out
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def _indexed(args):
    fn, i, t = args
    return i, fn(t)


def oracle_apply(name, targets, n_occ, chunk, kt=0, ko=0, weight=1.0, k0=0.0):
    """Oracle (V_x psi_j) for the listed targets, summed over occupied chunks."""
    tasks = [(name, kt, ko, list(targets), lo, min(lo + chunk, n_occ), weight, k0)
             for lo in range(0, n_occ, chunk)]
    return sum(_run(_apply_task, tasks, f"{name} apply"))


def oracle_kmesh_grad_rows(name, kt, targets, n_occ, chunk, nk, weight, k0):
    """Oracle dE/dconj(c_jk) for the listed targets j at k = kt of a k-mesh
    energy with equal weights: weight * sum_k' (V_x psi_jk) with the occupied
    set k' and q = k - k' (both blocks (k, k') and (k', k) contribute half),
    K(0) = k0 only in the block k' = k."""
    tasks = [(name, kt, ko, list(targets), lo, min(lo + chunk, n_occ), weight, k0 if ko == kt else 0.0)
             for ko in range(nk) for lo in range(0, n_occ, chunk)]
    return weight * sum(_run(_apply_task, tasks, f"{name} gradient rows k={kt}"))


def oracle_energy(name, n_tgt, n_occ, chunk, kt=0, ko=0, weight=1.0, k0=0.0):
    """Oracle block energy over targets [0, n_tgt) x occupied [0, n_occ)."""
    tasks = [(name, kt, ko, tl, min(tl + chunk, n_tgt), 0, n_occ, weight, k0) for tl in range(0, n_tgt, chunk)]
    return float(sum(_run(_energy_task, tasks, f"{name} energy")))
