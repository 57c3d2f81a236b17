"""Batched form: several uneven systems in one hipGraph, either one
persistent launch over every stage of every system (mode 0) or each system's
per-shape kernel schedule in turn (mode 1); the tuner keeps the faster."""
import numpy as np
import pytest

import synth
from oracle import exx
from tests.helpers import host, max_row_rel, rel_fro, report

pytestmark = pytest.mark.gpu


def _F():
    from paper_1305_7313_amd import fock
    return fock


def _small_batch():
    specs = [(synth.cubic_cell(7.5), 24, 21, 0), (synth.cubic_cell(15.0), 48, 18, 0),
             (np.array([[10.0, 0.0, 0.0], [0.7, 9.5, 0.0], [0.2, 0.4, 10.5]]), 24, 5, 1)]
    out = []
    for k, (a, n, nb, gb) in enumerate(specs):
        s = synth.make_system(a, (n, n, n))
        c = synth.random_orbitals(s.a, s.miller, nb, 40 + k)
        f = np.random.default_rng(k).uniform(0.3, 1.0, nb)
        out.append((s, c, f, gb))
    return out


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("mode", ["0", "1", "1-branches3", "auto"])
def test_batch_small_vs_single_and_oracle(prec, mode, tmp_path, monkeypatch):
    import torch
    F = _F()
    if mode == "1-branches3":
        # the per-shape schedule on three independent graph branches, untuned
        monkeypatch.setenv("FOCK_BATCH_TUNE", "0")
        monkeypatch.setenv("FOCK_BATCH_BRANCHES", "3")
        mode = "1"
    if mode != "auto":
        monkeypatch.setenv("FOCK_BATCH_MODE", mode)
    cdt = torch.complex128 if prec == "c128" else torch.complex64
    tol = 1e-10 if prec == "c128" else 1e-5
    systems = _small_batch()
    cells, C, W = [], [], []
    for s, c, f, gb in systems:
        cells.append(F.Cell(s.a, s.n, s.miller, g0=gb, gb_alpha=0.6, nq=(2, 2, 2)))
        C.append(torch.from_numpy(c).to(cdt).cuda())
        W.append(torch.from_numpy(f).cuda())
    print(f"[case] batch small {prec} mode={mode}: create (autotune)", flush=True)
    plan = F.BatchPlan(cells, C, W, tune_cache=str(tmp_path / "tune.json"))
    report(f"batch small {prec} schedule", **{k: v for k, v in plan.info().items()})
    if mode != "auto":
        assert plan.info()["mode"] == ("persistent" if mode == "0" else "kernels")
    if plan.info()["mode"] == "kernels":
        assert 1 <= plan.info()["branches"] <= 3
    plan.apply()
    plan.check()
    outs = [host(o).copy() for o in plan.outs]
    ex = host(plan.ex).copy()
    for k, (s, c, f, gb) in enumerate(systems):
        single = host(F.fock_apply(cells[k], (0, 0, 0), C[k], W[k], C[k]))
        k0 = exx.gb_constant(s.a, s.n, (2, 2, 2), 0.6) if gb else 0.0
        ref = exx.fock_apply(s.a, s.n, s.miller, np.zeros(3), c, f, c, k0=k0)
        e1, e2, e3 = rel_fro(outs[k], single), rel_fro(outs[k], ref), max_row_rel(outs[k], ref)
        e_ref = exx.fock_energy(s.a, s.n, s.miller, np.zeros(3), c, f, c, f, k0=k0)
        e4 = abs(ex[k] - e_ref) / abs(e_ref)
        report(f"batch small {prec} system {k}", vs_single=e1, vs_oracle=e2, vs_oracle_maxband=e3, E_rel=e4)
        # the tuned tile may group the accumulation differently from the single-system path
        assert e1 < (1e-12 if prec == "c128" else 1e-6) and e2 < tol and e3 < tol and e4 < tol
    # replays with eager work and synchronisation in between: every replay equals the first
    for rep in range(3):
        junk = torch.randn(1 << 20, device="cuda").cumsum(0)
        torch.cuda.synchronize()
        for o in plan.outs:
            o.zero_()
        plan.apply()
        plan.check()
        for k in range(len(systems)):
            assert np.array_equal(host(plan.outs[k]), outs[k]), (rep, k)
        del junk
    # inputs may change between replays: scale the occupations and replay
    for w in W:
        w.mul_(0.5)
    plan.apply()
    plan.check()
    for k in range(len(systems)):
        assert rel_fro(host(plan.outs[k]), 0.5 * outs[k]) < 1e-6
    if mode == "auto":
        # a second plan on the same batch reads the tune cache instead of re-tuning
        plan2 = F.BatchPlan(cells, C, W, tune_cache=str(tmp_path / "tune.json"))
        keys = [k for k in ("mode", "tile", "units_per_ticket") if k in plan.info()]
        assert {k: plan2.info()[k] for k in keys} == {k: plan.info()[k] for k in keys}
        plan2.close()
    plan.close()


@pytest.mark.parametrize("mode", ["0", "1"])
def test_batch_config4_fp32(mode, monkeypatch):
    """16 systems, grids from {48,64,72,96}^3, 32-242 orbitals, FP32."""
    import torch
    F = _F()
    monkeypatch.setenv("FOCK_BATCH_MODE", mode)
    monkeypatch.setenv("FOCK_BATCH_TUNE", "0")
    grids, nbs = synth.config4_layout()
    cells, C, W, sys_ = [], [], [], []
    for k in range(16):
        s, c = synth.config4_system(k)
        sys_.append((s, c))
        cells.append(F.Cell(s.a, s.n, s.miller))
        C.append(torch.from_numpy(c).to(torch.complex64).cuda())
        W.append(torch.ones(c.shape[0], dtype=torch.float64, device="cuda"))
    print(f"[case] config4 batch create mode={mode}", flush=True)
    plan = F.BatchPlan(cells, C, W)
    report("config4 schedule", **plan.info())
    plan.apply()
    plan.check()
    worst = 0.0
    for k in range(16):
        single = host(F.fock_apply(cells[k], (0, 0, 0), C[k], W[k], C[k]))
        worst = max(worst, rel_fro(host(plan.outs[k]), single))
    # oracle on the smallest system (48^3, 32 orbitals): every target, every occupied orbital
    k = int(np.argmin(nbs))
    s, c = sys_[k]
    ref = exx.fock_apply(s.a, s.n, s.miller, np.zeros(3), c, np.ones(c.shape[0]), c)
    err = rel_fro(host(plan.outs[k]), ref)
    report("config4", batched_vs_single_worst=worst, smallest_system_vs_oracle=err)
    assert worst < 1e-6 and err < 1e-5
    # oracle on one system of each large grid: rows {0, middle, last} against every occupied orbital
    outs = [host(o).astype(np.complex128) for o in plan.outs]
    plan.close()
    for k, (rows, ref) in _config4_oracle_rows().items():
        v = outs[k][rows]
        e1, e2 = rel_fro(v, ref), max_row_rel(v, ref)
        report(f"config4 FP32 batched mode {mode} system {k} ({grids[k]}^3, {nbs[k]} orbitals) rows {rows}",
               vs_oracle=e1, vs_oracle_maxband=e2)
        assert e1 < 1e-5 and e2 < 1e-5


# one system of each large grid of the 16-system workload: 96^3 (system 0),
# 72^3 (system 1), 64^3 (system 3)
_C4_ORACLE_SYSTEMS = (0, 1, 3)
_C4_ORACLE = {}


def _config4_oracle_rows():
    """Oracle (V_x psi_j) for rows {0, middle, last} of systems 0, 1 and 3 of
    the 16-system workload, each against all of its occupied orbitals."""
    from tests import oracle_pool
    if not _C4_ORACLE:
        _, nbs = synth.config4_layout()
        for k in _C4_ORACLE_SYSTEMS:
            nb = int(nbs[k])
            rows = [0, nb // 2, nb - 1]
            _C4_ORACLE[k] = (rows, oracle_pool.oracle_apply(f"c4:{k}", rows, nb, 16))
    return _C4_ORACLE


def test_config4_fp64_single_vs_oracle():
    """The FP64 single-system path on the large grids of the 16-system
    workload, rows against the oracle at the FP64 tolerance."""
    import torch
    F = _F()
    for k, (rows, ref) in _config4_oracle_rows().items():
        s, c = synth.config4_system(k)
        cell = F.Cell(s.a, s.n, s.miller)
        C = torch.from_numpy(c).cuda()
        f = torch.ones(c.shape[0], dtype=torch.float64, device="cuda")
        print(f"[case] config4 FP64 system {k} ({s.n[0]}^3, {c.shape[0]} orbitals)", flush=True)
        v = host(F.fock_apply(cell, (0, 0, 0), C, f, C))[rows]
        e1, e2 = rel_fro(v, ref), max_row_rel(v, ref)
        report(f"config4 FP64 system {k} rows {rows}", vs_oracle=e1, vs_oracle_maxband=e2)
        assert e1 < 1e-10 and e2 < 1e-10


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_batch_general_systems(prec, tmp_path):
    """Occupied and target blocks that differ, q != 0, a non-cubic grid: the
    persistent schedule does not apply and the plan uses per-shape kernels."""
    import torch
    F = _F()
    cdt = torch.complex128 if prec == "c128" else torch.complex64
    tol = 1e-10 if prec == "c128" else 1e-5
    skew = np.array([[10.0, 0.0, 0.0], [1.0, 18.0, 0.0], [0.5, 0.3, 24.0]])
    specs = [  # (cell, grid, n_occ, n_tgt or None (self), q)
        (synth.cubic_cell(10.0), (24, 24, 24), 9, None, (0.0, 0.0, 0.0)),
        (synth.cubic_cell(10.0), (24, 24, 24), 7, 5, (0.1, -0.05, 0.07)),
        (skew, (24, 48, 64), 6, None, (0.03, 0.02, -0.04)),
        (synth.cubic_cell(15.0), (48, 48, 48), 5, 11, (0.0, 0.0, 0.0)),
    ]
    cells, occ, focc, tgt, ftgt, qs, refs = [], [], [], [], [], [], []
    for k, (a, n, no, nt, q) in enumerate(specs):
        s = synth.make_system(a, n)
        co = synth.random_orbitals(s.a, s.miller, no, 60 + k)
        ct = co if nt is None else synth.random_orbitals(s.a, s.miller, nt, 70 + k)
        rng = np.random.default_rng(80 + k)
        fo = rng.uniform(0.3, 1.0, no)
        ft = fo if nt is None else rng.uniform(0.3, 1.0, nt)
        cells.append(F.Cell(s.a, s.n, s.miller))
        occ.append(torch.from_numpy(co).to(cdt).cuda())
        focc.append(torch.from_numpy(fo).cuda())
        tgt.append(occ[-1] if nt is None else torch.from_numpy(ct).to(cdt).cuda())
        ftgt.append(focc[-1] if nt is None else torch.from_numpy(ft).cuda())
        qs.append(q)
        refs.append((exx.fock_apply(s.a, s.n, s.miller, np.array(q), co, fo, ct),
                     exx.fock_energy(s.a, s.n, s.miller, np.array(q), co, fo, ct, ft)))
    print(f"[case] batch general {prec}", flush=True)
    plan = F.BatchPlan(cells, occ, focc, tgt_coeffs=tgt, tgt_weights=ftgt, q=qs, tune_cache=str(tmp_path / "t.json"))
    assert plan.info()["mode"] == "kernels"
    for rep in range(2):
        plan.apply()
        plan.check()
        ex = host(plan.ex)
        for k in range(len(specs)):
            v = host(plan.outs[k])
            single = host(F.fock_apply(cells[k], qs[k], occ[k], focc[k], tgt[k]))
            e1, e2 = rel_fro(v, refs[k][0]), rel_fro(v, single)
            e3 = abs(ex[k] - refs[k][1]) / abs(refs[k][1])
            report(f"batch general {prec} system {k} replay {rep}", vs_oracle=e1, vs_single=e2, E_rel=e3)
            assert e1 < tol and e2 < 1e-12 and e3 < tol
    plan.close()


def test_batch_wait_bound_aborts_and_recovers(monkeypatch):
    """Failure detection of the persistent schedule, forced from the host: with
    a bound of 10 ns on a dependency wait every wait gives up, the launch
    drains (every block stops taking work), fock_batch_check reports
    FOCK_E_HIP, and the next replay with the plan's own bound is correct
    again.  512 units per ticket put dependent units in the first wave of
    tickets, next to the units they depend on, so waits certainly occur."""
    import torch
    F = _F()
    monkeypatch.setenv("FOCK_BATCH_MODE", "0")
    monkeypatch.setenv("FOCK_BATCH_TUNE", "0")
    monkeypatch.setenv("FOCK_BATCH_TICKET", "512")
    systems = _small_batch()
    cells, C, W = [], [], []
    for s, c, f, gb in systems:
        cells.append(F.Cell(s.a, s.n, s.miller, g0=gb, gb_alpha=0.6, nq=(2, 2, 2)))
        C.append(torch.from_numpy(c).to(torch.complex64).cuda())
        W.append(torch.from_numpy(f).cuda())
    print("[case] batch wait bound: create", flush=True)
    plan = F.BatchPlan(cells, C, W)
    info = plan.info()
    assert info["mode"] == "persistent" and info["units_per_ticket"] == 512
    plan.apply()
    plan.check()
    ref = [host(o).copy() for o in plan.outs]
    print("[case] batch wait bound: replay with a 10 ns bound", flush=True)
    plan.set_wait_limit(1e-5)
    plan.apply()
    with pytest.raises(F.FockError) as err:
        plan.check()
    assert err.value.status == F.FOCK_E_HIP and "aborted" in str(err.value)
    print("[case] batch wait bound: replay with the plan's bound", flush=True)
    plan.set_wait_limit(0.0)
    plan.apply()
    plan.check()
    for k in range(len(systems)):
        assert np.array_equal(host(plan.outs[k]), ref[k]), k
    report("batch wait bound", aborted_then_recovered=1)
    plan.close()
