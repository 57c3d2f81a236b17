"""The C ABI: every declared symbol is exported; host-side validation codes.

These run without a GPU: each call below fails validation before any HIP
work is enqueued (the pointers are never dereferenced).
"""
import ctypes
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1305_7313_amd import fock
    return fock


def test_header_symbols_exported():
    F = _lib()
    hdr = open(os.path.join(ROOT, "include", "fock.h")).read()
    names = set(re.findall(r"\b(fock_[a-z0-9_]+)\s*\(", hdr))
    assert {"fock_apply", "fock_energy", "fock_energy_backward", "fock_workspace_size"} <= names
    L = F.lib()
    for n in sorted(names):
        assert hasattr(L, n), n


@pytest.fixture(scope="module")
def c1():
    F = _lib()
    s, o, t = synth.config1()
    return F, s, F.Cell(s.a, s.n, s.miller)


def _orbs(F, nb, ld, c=0x1000, w=0x2000):
    o = F.fock_orbs()
    o.c, o.w, o.nb, o.ld = c, w, nb, ld
    return o


def _apply(F, cell, q=(0.0, 0.0, 0.0), dtype=0, occ=None, tgt=None, out=0x3000, ws=0x4000, ws_bytes=1 << 40):
    occ = occ if occ is not None else _orbs(F, 8, cell.npw)
    tgt = tgt if tgt is not None else _orbs(F, 8, cell.npw)
    return F.lib().fock_apply(ctypes.byref(cell.c), F._qarr(q), dtype, ctypes.byref(occ), ctypes.byref(tgt),
                              out, ws, ws_bytes, None)


def test_workspace_size(c1):
    F, s, cell = c1
    n = 24 ** 3
    got = F.fock_workspace_size(cell, F.FOCK_C128, 8, 8)
    assert got >= (8 + 8 + 8 + 64) * n * 16
    assert F.fock_workspace_size(cell, F.FOCK_C64, 8, 8) < got
    assert F.fock_workspace_size(cell, 7, 8, 8) == 0
    bad = F.Cell(s.a, (24, 24, 25), s.miller)
    assert F.fock_workspace_size(bad, 0, 8, 8) == 0
    # past the pair-tile edge (32 in FP32, 16 in FP64) the pair buffer and the
    # accumulator tile stop growing: more orbitals only add their own planes
    # (occupied and target real-space copies) while the tile count is unchanged
    assert F.fock_workspace_size(cell, F.FOCK_C64, 40, 40) - F.fock_workspace_size(cell, F.FOCK_C64, 33, 33) \
        == 2 * 7 * n * 8
    assert F.fock_workspace_size(cell, F.FOCK_C128, 20, 20) - F.fock_workspace_size(cell, F.FOCK_C128, 17, 17) \
        == 2 * 3 * n * 16
    # below it the pair buffer holds a tile of min(n, edge)^2 pairs
    assert F.fock_workspace_size(cell, F.FOCK_C64, 17, 17) - F.fock_workspace_size(cell, F.FOCK_C64, 16, 16) \
        >= (2 + 1 + 17 * 17 - 16 * 16) * n * 8


def test_error_codes(c1):
    F, s, cell = c1
    assert _apply(F, cell, ws_bytes=10) == F.FOCK_E_WORKSPACE
    assert _apply(F, cell, ws=None) == F.FOCK_E_WORKSPACE
    assert _apply(F, cell, dtype=5) == F.FOCK_E_ARG
    assert _apply(F, cell, occ=_orbs(F, -1, cell.npw)) == F.FOCK_E_ARG
    assert _apply(F, cell, tgt=_orbs(F, 3, cell.npw - 1)) == F.FOCK_E_ARG
    assert _apply(F, cell, occ=_orbs(F, 3, cell.npw, c=None)) == F.FOCK_E_ARG
    assert _apply(F, cell, q=(np.nan, 0, 0)) == F.FOCK_E_ARG
    # q = a reciprocal-lattice vector (2 pi / L along x): singular
    assert _apply(F, cell, q=(2 * np.pi / 10.0, 0.0, 0.0)) == F.FOCK_E_SINGULAR_Q
    assert b"reciprocal-lattice" in F.lib().fock_last_error()
    # unsupported grid
    bad = F.Cell(s.a, (20, 24, 24), s.miller)
    assert _apply(F, bad) == F.FOCK_E_UNSUPPORTED_GRID
    # aliasing sphere: one Miller index beyond (n-1)/4
    m = s.miller.copy()
    m[0] = (6, 0, 0)
    assert _apply(F, F.Cell(s.a, s.n, m)) == F.FOCK_E_ALIAS
    # repeated G
    m = s.miller.copy()
    m[1] = m[0]
    assert _apply(F, F.Cell(s.a, s.n, m)) == F.FOCK_E_ALIAS
    # zero-volume cell
    a = s.a.copy()
    a[2] = a[1]
    assert _apply(F, F.Cell(a, s.n, s.miller)) in (F.FOCK_E_ARG,)
    # GB without a width
    assert _apply(F, F.Cell(s.a, s.n, s.miller, g0=F.FOCK_G0_GB, gb_alpha=0.0)) == F.FOCK_E_ARG
    assert F.lib().fock_status_string(F.FOCK_E_ALIAS).startswith(b"G-sphere")


def test_product_path_fails_loudly_without_library(monkeypatch, tmp_path):
    F = _lib()
    monkeypatch.setattr(F, "_lib", None)
    monkeypatch.setattr(F, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        F.lib()
