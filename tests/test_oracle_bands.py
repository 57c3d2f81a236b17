"""Pins of the band-loop oracle (section 5: the charge density and the forces
on the electronic degrees of freedom, one 3-D FFT per band).

Each pin is independent of the FFT route it checks: normalisation, the
Fourier components of the density as diagonal pair densities from the direct
G-space definition, a single plane wave, potentials with closed-form actions
(constant, cosine), and the force as the exact gradient of the band energy.
The mutation tests plant slips in the oracle and check that a pin fails.
"""
import numpy as np
import pytest

import synth
from oracle import bands, definitions, exx

A_SKEW = np.array([[7.0, 0.0, 0.0], [1.0, 8.0, 0.0], [0.5, 0.3, 9.0]])
N_SKEW = (12, 16, 20)
K_SKEW = np.array([0.13, -0.04, 0.09])


@pytest.fixture(scope="module")
def skew():
    s = synth.make_system(A_SKEW, N_SKEW)
    c = synth.random_orbitals(A_SKEW, s.miller, 4, 7)
    w = np.array([1.0, 0.8, 0.5, 0.25])
    v = np.random.default_rng(8).standard_normal(N_SKEW)
    return s, c, w, v


def rel(x, y):
    return float(np.linalg.norm(np.ravel(x - y)) / np.linalg.norm(np.ravel(y)))


def test_density_integrates_to_occupations(skew):
    s, c, w, _ = skew
    rho = bands.band_density(s.a, s.n, s.miller, c, w)
    omega = exx.volume(s.a)
    assert abs(rho.sum() * omega / np.prod(s.n) - w.sum()) < 1e-12 * w.sum()
    assert rho.min() >= 0.0


def test_density_components_are_pair_densities(skew):
    """FFT[rho](G) / N = sum_b w_b rho_bb(G), rho_bb from the direct convolution."""
    s, c, w, _ = skew
    rho = bands.band_density(s.a, s.n, s.miller, c, w)
    rg = exx.fft3(rho.astype(np.complex128), "dft") / np.prod(s.n)
    want = np.zeros(s.n, dtype=np.complex128)
    omega = exx.volume(s.a)
    for b in range(len(c)):
        gm, r = definitions.pair_density(c[b], c[b], s.miller, omega)
        np.add.at(want, (gm[:, 0] % s.n[0], gm[:, 1] % s.n[1], gm[:, 2] % s.n[2]), w[b] * r)
    assert rel(rg, want) < 1e-12


def test_density_single_plane_wave():
    s = synth.make_system(synth.cubic_cell(6.0), (12, 12, 12))
    c = np.zeros((1, s.npw), dtype=np.complex128)
    c[0, s.npw // 3] = 1.0
    rho = bands.band_density(s.a, s.n, s.miller, c, [1.0])
    assert np.abs(rho - 1.0 / exx.volume(s.a)).max() < 1e-14


def test_force_constant_potential(skew):
    s, c, w, _ = skew
    v0 = -0.37
    got = bands.band_force(s.a, s.n, s.miller, K_SKEW, c, w, np.full(s.n, v0))
    g = K_SKEW[None, :] + s.miller @ exx.reciprocal(s.a)
    want = -w[:, None] * (0.5 * np.einsum("ij,ij->i", g, g)[None, :] + v0) * c
    assert rel(got, want) < 1e-13


def test_force_cosine_potential(skew):
    """V(r) = cos(G0.r): (V psi)(G) = (c(G - G0) + c(G + G0)) / 2 on the sphere."""
    s, c, w, _ = skew
    m0 = np.array([1, -2, 1])
    i1, i2, i3 = np.meshgrid(*(np.arange(k) for k in s.n), indexing="ij")
    phase = 2 * np.pi * (m0[0] * i1 / s.n[0] + m0[1] * i2 / s.n[1] + m0[2] * i3 / s.n[2])
    got = bands.band_force(s.a, s.n, s.miller, np.zeros(3), c, np.ones(len(c)), np.cos(phase))
    index = {tuple(m): p for p, m in enumerate(s.miller)}
    vpsi = np.zeros_like(c)
    for p, m in enumerate(s.miller):
        for sh in (m - m0, m + m0):
            q = index.get(tuple(sh))
            if q is not None:
                vpsi[:, p] += 0.5 * c[:, q]
    kin = 0.5 * np.einsum("ij,ij->i", s.miller @ exx.reciprocal(s.a), s.miller @ exx.reciprocal(s.a))
    want = -(kin[None, :] * c + vpsi)
    assert rel(got, want) < 1e-13


def test_force_is_the_energy_gradient(skew):
    """E is quadratic in c, so central differences are exact up to rounding:
    dE/dh along d equals 2 Re sum conj(d) (-F)."""
    s, c, w, v = skew
    f = bands.band_force(s.a, s.n, s.miller, K_SKEW, c, w, v)
    rng = np.random.default_rng(9)
    for _ in range(3):
        d = rng.standard_normal(c.shape) + 1j * rng.standard_normal(c.shape)
        h = 1e-3
        ep = bands.band_energy(s.a, s.n, s.miller, K_SKEW, c + h * d, w, v)
        em = bands.band_energy(s.a, s.n, s.miller, K_SKEW, c - h * d, w, v)
        fd = (ep - em) / (2 * h)
        an = 2.0 * float(np.real(np.sum(np.conj(d) * (-f))))
        assert abs(fd - an) < 1e-10 * max(1.0, abs(an))


# --- planted slips: each must make a pin above fail ----------------------

def test_mutation_missing_volume(skew, monkeypatch):
    monkeypatch.setattr(bands, "volume", lambda a: 1.0)
    with pytest.raises(AssertionError):
        test_density_integrates_to_occupations(skew)


def test_mutation_wrong_transform_sign(skew, monkeypatch):
    monkeypatch.setattr(bands, "fft3", exx.bfft3)
    with pytest.raises(AssertionError):
        test_force_is_the_energy_gradient(skew)


def test_mutation_conjugated_orbital(skew, monkeypatch):
    real_to_grid = exx.to_grid
    monkeypatch.setattr(bands, "to_grid", lambda c, m, n, method="auto": np.conj(real_to_grid(c, m, n, method)))
    with pytest.raises(AssertionError):
        test_force_is_the_energy_gradient(skew)
