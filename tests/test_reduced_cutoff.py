"""Reduced Fock cutoff on a coarser exchange grid (section 6: the Fock cutoff
may be set below the density cutoff, four times the wave-function cutoff).

Oracle pins: with K cut at E_fock, the FFT route on any grid that meets the
per-axis rule n_a >= min(F_a, 2 M_a) + 2 M_a + 1 gives the grid-free direct
definition (G-space convolutions, no grid at all), and one point below the
rule it does not.  Library: the grid rule it applies is never below the one
the oracle finds by listing lattice points, and grids below it are refused.
"""
import ctypes

import numpy as np
import pytest

import synth
from oracle import definitions, exx

L_SMALL = 10.0
N_FULL = (24, 24, 24)


def rel(x, y):
    return float(np.linalg.norm(np.ravel(x - y)) / np.linalg.norm(np.ravel(y)))


@pytest.fixture(scope="module")
def small():
    a = synth.cubic_cell(L_SMALL)
    e = synth.alias_free_ecut(a, N_FULL)
    m = synth.sphere_miller(a, N_FULL, e)
    occ = synth.random_orbitals(a, m, 2, 11)
    tgt = synth.random_orbitals(a, m, 2, 12)
    f = np.array([1.0, 0.6])
    return a, m, e, occ, tgt, f


def test_grid_need_by_enumeration(small):
    a, m, e, *_ = small
    # cubic cell, q = 0, E_fock = E_wfc: F = M = 5, so 5 + 10 + 1
    assert exx.exchange_grid_need(a, m, e) == (16, 16, 16)
    # no cutoff: the alias-free rule of the full density cutoff
    assert exx.exchange_grid_need(a, m, 0.0) == (21, 21, 21)
    # a cutoff past 4 E_wfc changes nothing: K only sees |m| <= 2M anyway
    assert exx.exchange_grid_need(a, m, 5.0 * e) == (21, 21, 21)
    # q shifts the ball: half a reciprocal vector along x adds one index there
    q = np.array([np.pi / L_SMALL, 0.0, 0.0])
    assert exx.exchange_grid_need(a, m, e, [q]) == (17, 16, 16)


@pytest.mark.parametrize("q", [(0.0, 0.0, 0.0), (np.pi / L_SMALL, np.pi / (2 * L_SMALL), 0.0)])
def test_coarse_grid_is_exact_and_the_rule_is_tight(small, q):
    a, m, e, occ, tgt, f = small
    q = np.array(q)
    need = exx.exchange_grid_need(a, m, e, [q])
    want = definitions.fock_apply_direct(a, m, q, occ, f, tgt, ecut_fock=e)
    for n in (need, N_FULL):
        got = exx.fock_apply(a, n, m, q, occ, f, tgt, ecut_fock=e, method="fft")
        assert rel(got, want) < 1e-12, n
    # one point short on the axis with the largest need: products alias
    ax = int(np.argmax(need))
    short = tuple(x - 1 if i == ax else x for i, x in enumerate(need))
    got = exx.fock_apply(a, short, m, q, occ, f, tgt, ecut_fock=e, method="fft")
    assert rel(got, want) > 1e-6


def test_coarse_grid_energy(small):
    a, m, e, occ, _, f = small
    q = np.zeros(3)
    need = exx.exchange_grid_need(a, m, e)
    e_coarse = exx.fock_energy(a, need, m, q, occ, f, occ, f, ecut_fock=e, method="fft")
    e_full = exx.fock_energy(a, N_FULL, m, q, occ, f, occ, f, ecut_fock=e, method="fft")
    # E = 1/2 sum_j f_j Re <psi_j | V_x psi_j> with V_x from the direct definition
    v = definitions.fock_apply_direct(a, m, q, occ, f, occ, ecut_fock=e)
    e_direct = 0.5 * float(np.sum(f * np.real(np.sum(np.conj(occ) * v, axis=1))))
    assert abs(e_coarse - e_direct) < 1e-12 * abs(e_direct)
    assert abs(e_full - e_direct) < 1e-12 * abs(e_direct)
    # the cutoff matters: the full-box kernel gives another energy
    e_box = exx.fock_energy(a, N_FULL, m, q, occ, f, occ, f, method="fft")
    assert abs(e_box - e_direct) > 1e-4 * abs(e_direct)


# --- the library's rule (host-only calls: no GPU needed) ------------------

def _F():
    from paper_1305_7313_amd import fock
    return fock


CASES = [
    # (cell, full grid, cutoff factor on E_wfc, q list)
    (synth.cubic_cell(20.0), (64, 64, 64), 1.0, None),
    (synth.cubic_cell(20.0), (64, 64, 64), 0.5, None),
    (synth.cubic_cell(20.0), (64, 64, 64), 2.0, None),
    (synth.cubic_cell(20.0), (64, 64, 64), 0.0, None),
    (synth.ortho_cell(22.0, 22.0, 30.0), (96, 96, 128), 1.0, None),
    (synth.cubic_cell(24.0), (72, 72, 72), 1.0, "mesh"),
    (np.array([[15.0, 0.0, 0.0], [2.0, 15.0, 0.0], [1.0, 1.5, 15.0]]), (48, 48, 48), 1.0, [[0.05, -0.1, 0.08]]),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_library_grid_meets_the_rule(case):
    F = _F()
    a, n, fac, qs = CASES[case]
    e = synth.alias_free_ecut(a, n)
    m = synth.sphere_miller(a, n, e)
    if qs == "mesh":
        k = synth.kmesh_points(a, (2, 2, 2))
        qs = [ki - kj for ki in k for kj in k]
    cell = F.Cell(a, n, m, ecut_fock=fac * e)
    got = F.fock_exchange_grid(cell, qs)
    need = exx.exchange_grid_need(a, m, fac * e, qs)
    assert all(g >= x for g, x in zip(got, need)), (got, need)
    assert np.prod(got) <= np.prod(n)


def test_library_grid_choices():
    F = _F()
    a = synth.cubic_cell(20.0)
    e = synth.alias_free_ecut(a, (64,) * 3)
    m = synth.sphere_miller(a, (64,) * 3, e)
    assert F.fock_exchange_grid(F.Cell(a, (0, 0, 0), m, ecut_fock=e)) == (48, 48, 48)
    assert F.fock_exchange_grid(F.Cell(a, (0, 0, 0), m, ecut_fock=0.0)) == (64, 64, 64)
    a3 = synth.ortho_cell(22.0, 22.0, 30.0)
    e3 = synth.alias_free_ecut(a3, (96, 96, 128))
    m3 = synth.sphere_miller(a3, (96, 96, 128), e3)
    assert F.fock_exchange_grid(F.Cell(a3, (0, 0, 0), m3, ecut_fock=e3)) == (72, 96, 96)
    # a sphere no compiled grid can hold without aliasing
    big = synth.sphere_miller(a, (128,) * 3, synth.alias_free_ecut(a, (128,) * 3)) * 2
    with pytest.raises(F.FockError):
        F.fock_exchange_grid(F.Cell(a, (0, 0, 0), big))


def test_library_refuses_grids_below_the_rule():
    F = _F()
    a = synth.cubic_cell(20.0)
    e = synth.alias_free_ecut(a, (64,) * 3)
    m = synth.sphere_miller(a, (64,) * 3, e)

    def apply(n, ecut):
        cell = F.Cell(a, n, m, ecut_fock=ecut)
        o = F.fock_orbs()
        o.c, o.w, o.nb, o.ld = 0x1000, 0x2000, 4, len(m)
        return F.lib().fock_apply(ctypes.byref(cell.c), F._qarr((0.0, 0.0, 0.0)), 0, ctypes.byref(o),
                                  ctypes.byref(o), 0x3000, 0x4000, 1 << 40, None)

    # 48^3 without a cutoff aliases; with E_fock = E_wfc it passes validation
    # (and then needs a device: FOCK_E_HIP here, FOCK_OK on a GPU)
    assert apply((48, 48, 48), 0.0) == F.FOCK_E_ALIAS
    assert b"smallest without aliasing" in F.lib().fock_last_error()
    assert apply((48, 48, 48), e) != F.FOCK_E_ALIAS
    assert apply((24, 24, 24), e) == F.FOCK_E_ALIAS
