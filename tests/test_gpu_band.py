"""GPU parity of the band loops (section 5: charge density and electronic
forces, one 3-D FFT per band) against the CPU FP64 oracle.

Bars as for the exchange path: FP64 within 1e-10 relative, FP32 within 1e-5.
Cases: a cubic 24^3 cell with more bands than one chunk (ragged last chunk),
a skewed cell on a non-cubic grid with k != 0, an empty band list, and the
benchmark's full-size workload on sampled bands.
"""
import numpy as np
import pytest

import synth
from oracle import bands
from tests.helpers import dev, host, max_row_rel, rel_fro, report

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-10, "c64": 1e-5}

CASES = {
    "cubic_ragged": dict(a=synth.cubic_cell(10.0), n=(24, 24, 24), nb=70, k=(0.0, 0.0, 0.0)),
    "skew_k": dict(a=np.array([[10.0, 0.0, 0.0], [1.0, 18.0, 0.0], [0.5, 0.3, 24.0]]), n=(24, 48, 64), nb=9,
                   k=(0.05, -0.03, 0.02)),
}


def _F():
    from paper_1305_7313_amd import fock
    return fock


def _types(prec):
    import torch
    return (torch.complex128, torch.float64) if prec == "c128" else (torch.complex64, torch.float32)


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request):
    c = CASES[request.param]
    s = synth.make_system(c["a"], c["n"])
    coef = synth.random_orbitals(s.a, s.miller, c["nb"], 17)
    rng = np.random.default_rng(18)
    w = rng.uniform(0.1, 2.0, c["nb"])
    v = rng.standard_normal(s.n)
    k = np.array(c["k"])
    rho = bands.band_density(s.a, s.n, s.miller, coef, w)
    force = bands.band_force(s.a, s.n, s.miller, k, coef, w, v)
    return request.param, s, coef, w, v, k, rho, force


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_band_density_and_force(case, prec):
    import torch
    F = _F()
    name, s, coef, w, v, k, rho_ref, f_ref = case
    cdt, rdt = _types(prec)
    print(f"[case] bands {name} {prec}", flush=True)
    cell = F.Cell(s.a, s.n, s.miller)
    cd, wd = dev(coef, cdt), dev(w)
    rho = host(F.fock_band_density(cell, cd, wd))
    force = host(F.fock_band_force(cell, k, cd, wd, dev(v, rdt)))
    errs = dict(rho_rel=rel_fro(rho, rho_ref), force_rel=rel_fro(force, f_ref),
                force_maxband=max_row_rel(force, f_ref))
    report(f"bands {name} {prec}", **errs)
    for key, val in errs.items():
        assert val < TOL[prec], (key, val)


def test_band_density_reproducible_and_empty():
    import torch
    F = _F()
    s = synth.make_system(synth.cubic_cell(10.0), (24, 24, 24))
    coef = synth.random_orbitals(s.a, s.miller, 70, 19)
    cell = F.Cell(s.a, s.n, s.miller)
    cd, wd = dev(coef), dev(np.ones(70))
    r1 = host(F.fock_band_density(cell, cd, wd))
    r2 = host(F.fock_band_density(cell, cd, wd))
    assert np.array_equal(r1, r2)
    empty = torch.empty((0, s.npw), dtype=torch.complex128, device="cuda")
    r0 = host(F.fock_band_density(cell, empty, torch.empty(0, dtype=torch.float64, device="cuda")))
    assert not r0.any()
    f0 = F.fock_band_force(cell, (0, 0, 0), empty, torch.empty(0, dtype=torch.float64, device="cuda"),
                           torch.zeros(s.n, dtype=torch.float64, device="cuda"))
    assert f0.shape == (0, s.npw)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_band_loops_full_size(prec):
    """The benchmark's workload: config 3's cell and 512 orbitals.  Density:
    total charge, the first 32 bands against the oracle, FP32 vs FP64.  Force:
    4 sampled bands against the oracle."""
    import torch
    F = _F()
    s, coef = synth.config3()
    cdt, rdt = _types(prec)
    nb = coef.shape[0]
    w = np.full(nb, 2.0)
    v = np.random.default_rng(20).standard_normal(s.n)
    k = np.zeros(3)
    cell = F.Cell(s.a, s.n, s.miller)
    print(f"[case] bands full size {prec}", flush=True)
    cd, wd, vd = dev(coef, cdt), dev(w), dev(v, rdt)
    rho = host(F.fock_band_density(cell, cd, wd))
    omega = abs(np.linalg.det(s.a))
    charge_err = abs(rho.sum() * omega / np.prod(s.n) - w.sum()) / w.sum()
    rho32 = host(F.fock_band_density(cell, cd[:32].contiguous(), wd[:32].contiguous()))
    rho32_ref = bands.band_density(s.a, s.n, s.miller, coef[:32], w[:32])
    force = host(F.fock_band_force(cell, k, cd, wd, vd))
    rows = [0, 201, 402, 511]
    f_ref = bands.band_force(s.a, s.n, s.miller, k, coef[rows], w[rows], v)
    errs = dict(charge=charge_err, rho32_rel=rel_fro(rho32, rho32_ref), force_rel=rel_fro(force[rows], f_ref),
                force_maxband=max_row_rel(force[rows], f_ref))
    report(f"bands full size {prec}", **errs)
    for key, val in errs.items():
        assert val < TOL[prec], (key, val)
