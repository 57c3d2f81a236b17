"""GPU parity for the reduced Fock cutoff on the coarser exchange grid
(section 6: the Fock cutoff may be set below the density cutoff).

The config-2 sphere (L = 20 bohr, |m| <= 15) with E_fock = E_wfc runs on the
48^3 grid that fock_exchange_grid picks instead of the 64^3 density grid.
Checked against the oracle on the coarse grid, and against the GPU path on
the 64^3 grid with the same cutoff: the result must not depend on the grid.
"""
import numpy as np
import pytest

import synth
from oracle import exx
from tests.helpers import dev, host, max_row_rel, rel_fro, report

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-10, "c64": 1e-5}
L2, N2 = 20.0, (64, 64, 64)


def _F():
    from paper_1305_7313_amd import fock
    return fock


def _ctype(name):
    import torch
    return torch.complex128 if name == "c128" else torch.complex64


@pytest.fixture(scope="module")
def sphere():
    a = synth.cubic_cell(L2)
    e = synth.alias_free_ecut(a, N2)
    m = synth.sphere_miller(a, N2, e)
    coarse = _F().fock_exchange_grid(_F().Cell(a, N2, m, ecut_fock=e))
    assert coarse == (48, 48, 48)
    return a, e, m, coarse


@pytest.fixture(scope="module")
def blocks(sphere):
    a, e, m, coarse = sphere
    occ = synth.random_orbitals(a, m, 6, 21)
    tgt = synth.random_orbitals(a, m, 5, 22)
    rng = np.random.default_rng(23)
    f = rng.uniform(0.2, 1.0, 6)
    g = rng.uniform(0.2, 1.0, 5)
    q = np.array([np.pi / L2, 0.0, -0.5 * np.pi / L2])
    ref = {}
    for name, qq in (("q0", np.zeros(3)), ("q", q)):
        ref[name] = (qq, exx.fock_apply(a, coarse, m, qq, occ, f, tgt, ecut_fock=e),
                     exx.fock_energy(a, coarse, m, qq, occ, f, tgt, g, ecut_fock=e))
    return occ, tgt, f, g, ref


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("qname", ["q0", "q"])
def test_coarse_grid_apply_energy(sphere, blocks, prec, qname):
    F = _F()
    a, e, m, coarse = sphere
    occ, tgt, f, g, ref = blocks
    q, v_ref, e_ref = ref[qname]
    assert F.fock_exchange_grid(F.Cell(a, N2, m, ecut_fock=e), [q]) == coarse
    print(f"[case] reduced cutoff {qname} {prec} grid {coarse}", flush=True)
    co, ct = dev(occ, _ctype(prec)), dev(tgt, _ctype(prec))
    fd, gd = dev(f), dev(g)
    out = {}
    for n in (coarse, N2):
        cell = F.Cell(a, n, m, ecut_fock=e)
        out[n] = (host(F.fock_apply(cell, q, co, fd, ct)), float(host(F.fock_energy(cell, q, co, fd, ct, gd))))
    (v_c, e_c), (v_f, e_f) = out[coarse], out[N2]
    errs = dict(apply_rel=rel_fro(v_c, v_ref), apply_maxband=max_row_rel(v_c, v_ref),
                E_rel=abs(e_c - e_ref) / abs(e_ref), coarse_vs_full=rel_fro(v_c, v_f),
                E_coarse_vs_full=abs(e_c - e_f) / abs(e_f))
    report(f"reduced cutoff {qname} {prec}", **errs)
    for k, val in errs.items():
        assert val < TOL[prec], (k, val)


@pytest.mark.parametrize("schedule", ["0", "1", "2"])
def test_coarse_grid_self_schedules(sphere, schedule, monkeypatch):
    """One block applied to itself (pair-symmetric schedules, 2 ragged tiles)."""
    F = _F()
    a, e, m, coarse = sphere
    monkeypatch.setenv("FOCK_SYM_SCHEDULE", schedule)
    occ = synth.random_orbitals(a, m, 20, 24)
    f = np.random.default_rng(25).uniform(0.2, 1.0, 20)
    rows = [0, 7, 19]
    v_ref = exx.fock_apply(a, coarse, m, np.zeros(3), occ, f, occ[rows], ecut_fock=e)
    e_ref = exx.fock_energy(a, coarse, m, np.zeros(3), occ, f, occ, f, ecut_fock=e)
    print(f"[case] reduced cutoff self schedule={schedule}", flush=True)
    co, fd = dev(occ), dev(f)
    cell = F.Cell(a, coarse, m, ecut_fock=e)
    v = host(F.fock_apply(cell, (0, 0, 0), co, fd, co))
    en = float(host(F.fock_energy(cell, (0, 0, 0), co, fd, co, fd)))
    v_full = host(F.fock_apply(F.Cell(a, N2, m, ecut_fock=e), (0, 0, 0), co, fd, co))
    errs = dict(apply_rel=rel_fro(v[rows], v_ref), E_rel=abs(en - e_ref) / abs(e_ref),
                coarse_vs_full=rel_fro(v, v_full))
    report(f"reduced cutoff self schedule={schedule}", **errs)
    for k, val in errs.items():
        assert val < TOL["c128"], (k, val)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_coarse_grid_kmesh_energy_grad(sphere, prec):
    """2x2x2 k-mesh, 2 orbitals per k: the coarse grid must hold every q = k - k'."""
    import torch
    F = _F()
    a, e, m, _ = sphere
    kpts = synth.kmesh_points(a, (2, 2, 2))
    qs = [ki - kj for ki in kpts for kj in kpts]
    grid = F.fock_exchange_grid(F.Cell(a, N2, m, ecut_fock=e), qs)
    assert np.prod(grid) < np.prod(N2)
    sets = [synth.random_orbitals(a, m, 2, 30 + k) for k in range(8)]
    w = [np.full(2, 1.0 / 8) for _ in range(8)]
    e_ref = exx.fock_energy_kmesh(a, grid, m, kpts, sets, w, ecut_fock=e)
    g_ref = np.stack(exx.fock_energy_kmesh_grad(a, grid, m, kpts, sets, w, ecut_fock=e))
    print(f"[case] reduced cutoff kmesh {prec} grid {grid}", flush=True)
    C = torch.from_numpy(np.stack(sets)).to(_ctype(prec)).cuda()
    W = torch.from_numpy(np.stack(w)).cuda()
    one = torch.ones((), dtype=torch.float64, device="cuda")
    res = {}
    for n in (grid, N2):
        cell = F.Cell(a, n, m, ecut_fock=e)
        en = float(host(F.fock_energy_kmesh(cell, kpts, C, W)))
        G = torch.empty_like(C)
        F.fock_energy_kmesh_backward(cell, kpts, C, W, one, [G[k] for k in range(8)])
        res[n] = (en, host(G))
    (e_c, g_c), (e_f, g_f) = res[grid], res[N2]
    errs = dict(E_rel=abs(e_c - e_ref) / abs(e_ref), grad_rel=rel_fro(g_c, g_ref),
                E_coarse_vs_full=abs(e_c - e_f) / abs(e_f), grad_coarse_vs_full=rel_fro(g_c, g_f))
    report(f"reduced cutoff kmesh {prec}", **errs)
    for k, val in errs.items():
        assert val < TOL[prec], (k, val)


def test_coarse_grid_full_size(sphere):
    """The benchmark's reduced-cutoff workload: 128 orbitals applied to
    themselves on 48^3 (FP64), against 64^3 at the same cutoff and, on 4
    sampled targets, against the oracle."""
    F = _F()
    a, e, m, coarse = sphere
    occ = synth.random_orbitals(a, m, 128, 0)
    f = np.ones(128)
    rows = [0, 41, 97, 127]
    print("[case] reduced cutoff full size 128x128 FP64", flush=True)
    v_ref = exx.fock_apply(a, coarse, m, np.zeros(3), occ, f, occ[rows], ecut_fock=e)
    co, fd = dev(occ), dev(f)
    v = host(F.fock_apply(F.Cell(a, coarse, m, ecut_fock=e), (0, 0, 0), co, fd, co))
    v_full = host(F.fock_apply(F.Cell(a, N2, m, ecut_fock=e), (0, 0, 0), co, fd, co))
    errs = dict(sampled_rel=rel_fro(v[rows], v_ref), sampled_maxband=max_row_rel(v[rows], v_ref),
                coarse_vs_full=rel_fro(v, v_full))
    report("reduced cutoff full size", **errs)
    for k, val in errs.items():
        assert val < TOL["c128"], (k, val)
