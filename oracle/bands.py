"""Band loops of the Car-Parrinello code, in FP64 on the CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 5 of the paper names the two band loops that dominate CP at scale
besides orthogonalisation: the charge density and the forces on the
electronic degrees of freedom, each one 3-D FFT per band.  With the
conventions of ``exx`` (psi_b(r) = Omega^{-1/2} sum_G c_b(G) e^{iG.r}, grid
points r_m = sum_a (m_a / n_a) a_a):

* density  rho(r_m) = sum_b f_b |psi_b(r_m)|^2;
* force    F_b(G) = -f_b ( 1/2 |k+G|^2 c_b(G) + (V psi_b)(G) ) on the sphere,
           (V psi)(G) = N^{-1} sum_m V(r_m) psi~(r_m) e^{-iG.r_m} with
           psi~ = sum_G c(G) e^{iG.r}: the sphere projection of V psi, and
           -F_b = dE/dconj(c_b) for E = sum_b f_b <psi_b| -1/2 nabla^2 + V |psi_b>
           evaluated on the grid.
"""
from __future__ import annotations

import numpy as np

from .exx import box_slots, fft3, reciprocal, to_grid, volume


def band_density(a, n, miller, c, w, method: str = "auto") -> np.ndarray:
    """rho on the grid, [n1, n2, n3] float64."""
    psi = to_grid(c, miller, n, method)  # psi~ = Omega^{1/2} psi
    return np.einsum("b,bxyz->xyz", np.asarray(w, dtype=np.float64), np.abs(psi) ** 2) / volume(a)


def kinetic(a, miller, k) -> np.ndarray:
    """1/2 |k+G|^2 on the sphere."""
    g = np.asarray(k, dtype=np.float64)[None, :] + np.asarray(miller, dtype=np.float64) @ reciprocal(a)
    return 0.5 * np.einsum("ij,ij->i", g, g)


def band_force(a, n, miller, k, c, w, vloc, method: str = "auto") -> np.ndarray:
    """F_b(G) on the sphere, [nb, npw] complex128."""
    psi = to_grid(c, miller, n, method)
    N = int(np.prod(n))
    vpsi = fft3(np.asarray(vloc, dtype=np.float64)[None] * psi, method) / N
    i1, i2, i3 = box_slots(miller, n)
    w = np.asarray(w, dtype=np.float64)
    return -w[:, None] * (kinetic(a, miller, k)[None, :] * c + vpsi[:, i1, i2, i3])


def band_energy(a, n, miller, k, c, w, vloc, method: str = "auto") -> float:
    """E = sum_b f_b ( sum_G 1/2 |k+G|^2 |c_b(G)|^2 + (Omega/N) sum_m V(r_m) |psi_b(r_m)|^2 )."""
    w = np.asarray(w, dtype=np.float64)
    kin = float(np.sum(w[:, None] * kinetic(a, miller, k)[None, :] * np.abs(c) ** 2))
    rho = band_density(a, n, miller, c, w, method)
    return kin + volume(a) / int(np.prod(n)) * float(np.sum(np.asarray(vloc) * rho))
