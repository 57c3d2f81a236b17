"""Seeded synthetic inputs for the exact-exchange (Fock) operator.

This module is shared by the CPU oracle tests, the GPU parity tests and the
benchmark.  It holds no arithmetic of the exchange method itself: it only
builds cells, the plane-wave G-sphere (the list of Miller indices that
represents an orbital) and random, orthonormal orbital coefficients.

Input recipe (the same for every workload):
  * cells are given by their lattice vectors a_1, a_2, a_3 (rows, bohr);
  * per axis the signed index of FFT slot i is i for i < n/2, else i - n;
  * the wavefunction cutoff is the largest sphere whose pair products do not
    alias on the grid: E_cut = min_a [2 pi (n_a - 1) / (4 |a_a|)]^2 (bohr^-2);
  * the sphere S = {G : |G|^2 <= E_cut} is listed in C order of the FFT box;
  * coefficients: complex normal draws (real block first, then imaginary),
    scaled by 1 / (1 + |G|^2)^2, then Loewdin-orthonormalised;
  * occupations are 1 (per spin channel).
The paper's own systems (a-SiO2, cholesterol, carbon nanotubes) need atomic
structures and pseudopotentials; these synthetic orbitals stand in for them
at the paper's large-cell scale.
"""
from __future__ import annotations

import dataclasses
import numpy as np

TWO_PI = 2.0 * np.pi


def cubic_cell(L: float) -> np.ndarray:
    return np.diag([float(L)] * 3)


def ortho_cell(lx: float, ly: float, lz: float) -> np.ndarray:
    return np.diag([float(lx), float(ly), float(lz)])


def reciprocal_rows(a: np.ndarray) -> np.ndarray:
    """Rows b_i with a_i . b_j = 2 pi delta_ij."""
    return TWO_PI * np.linalg.inv(np.asarray(a, dtype=np.float64)).T


def slot_index(n: int) -> np.ndarray:
    """Signed frequency index of each FFT slot (numpy fftfreq order)."""
    i = np.arange(n, dtype=np.int64)
    return np.where(i < (n + 1) // 2 if n % 2 else i < n // 2, i, i - n)


def alias_free_ecut(a: np.ndarray, n) -> float:
    a = np.asarray(a, dtype=np.float64)
    lens = np.linalg.norm(a, axis=1)
    return float(min((TWO_PI * (int(na) - 1) / (4.0 * la)) ** 2 for na, la in zip(n, lens)))


def sphere_miller(a: np.ndarray, n, ecut: float) -> np.ndarray:
    """Miller indices [npw, 3] (int32) of the G-sphere |G|^2 <= ecut, C order of the box."""
    b = reciprocal_rows(a)
    m1, m2, m3 = np.meshgrid(slot_index(n[0]), slot_index(n[1]), slot_index(n[2]), indexing="ij")
    m = np.stack([m1.ravel(), m2.ravel(), m3.ravel()], axis=1)
    g = m.astype(np.float64) @ b
    keep = np.einsum("ij,ij->i", g, g) <= ecut
    return np.ascontiguousarray(m[keep].astype(np.int32))


def sphere_g2(a: np.ndarray, miller: np.ndarray) -> np.ndarray:
    g = np.asarray(miller, dtype=np.float64) @ reciprocal_rows(a)
    return np.einsum("ij,ij->i", g, g)


def loewdin(c: np.ndarray) -> np.ndarray:
    """Symmetric orthonormalisation of the rows of c: returns S^{-1/2}-rotated rows."""
    s = np.conj(c) @ c.T
    w, v = np.linalg.eigh(s)
    s_mhalf = (v * (1.0 / np.sqrt(w))) @ np.conj(v).T
    return s_mhalf.T @ c


def random_orbitals(a: np.ndarray, miller: np.ndarray, nb: int, seed: int) -> np.ndarray:
    """[nb, npw] complex128 orthonormal coefficients, the recipe in the module docstring."""
    npw = miller.shape[0]
    if nb > npw:
        raise ValueError("more orbitals than plane waves")
    rng = np.random.default_rng(seed)
    re = rng.standard_normal((nb, npw))
    im = rng.standard_normal((nb, npw))
    c = re + 1j * im
    c *= 1.0 / (1.0 + sphere_g2(a, miller)) ** 2
    if nb == 0:
        return c
    return np.ascontiguousarray(loewdin(c))


def gamma_orbitals(a: np.ndarray, miller: np.ndarray, nb: int, seed: int) -> np.ndarray:
    """[nb, npw] orthonormal coefficients of real orbitals (Gamma point):
    c(-G) = conj(c(G)).  The draws of random_orbitals are made Hermitian,
    (c(G) + conj(c(-G))) / 2, then Loewdin-orthonormalised with the (real)
    overlap of real functions, which keeps them Hermitian.  The sphere must
    hold -G with every G."""
    m = np.asarray(miller)
    index = {tuple(v): p for p, v in enumerate(m)}
    neg = np.array([index[tuple(-v)] for v in m])
    rng = np.random.default_rng(seed)
    npw = m.shape[0]
    if nb > npw:
        raise ValueError("more orbitals than plane waves")
    c = rng.standard_normal((nb, npw)) + 1j * rng.standard_normal((nb, npw))
    c = 0.5 * (c + np.conj(c[:, neg]))
    c *= 1.0 / (1.0 + sphere_g2(a, miller)) ** 2
    if nb == 0:
        return c
    s = (np.conj(c) @ c.T).real
    w, v = np.linalg.eigh(s)
    s_mhalf = (v * (1.0 / np.sqrt(w))) @ v.T
    return np.ascontiguousarray(s_mhalf.T @ c)


@dataclasses.dataclass
class System:
    """One cell with its grid, sphere and orbital blocks."""
    a: np.ndarray
    n: tuple
    ecut: float
    miller: np.ndarray

    @property
    def npw(self) -> int:
        return int(self.miller.shape[0])

    @property
    def volume(self) -> float:
        return float(abs(np.linalg.det(self.a)))


def make_system(a, n) -> System:
    a = np.asarray(a, dtype=np.float64)
    n = tuple(int(x) for x in n)
    ecut = alias_free_ecut(a, n)
    return System(a=a, n=n, ecut=ecut, miller=sphere_miller(a, n, ecut))


# ----------------------------------------------------------------------------
# The five workloads.  Sizes follow the paper's large-cell scale (a-SiO2 EXX
# benchmark, section 6); the orbitals are synthetic.
# ----------------------------------------------------------------------------

def config1():
    """24^3 cubic L=10: 8 occupied (seed 0) + 8 targets (seed 1)."""
    s = make_system(cubic_cell(10.0), (24, 24, 24))
    occ = random_orbitals(s.a, s.miller, 8, 0)
    tgt = random_orbitals(s.a, s.miller, 8, 1)
    return s, occ, tgt


def config2(nb: int = 128):
    """64^3 cubic L=20: 128 orbitals applied to themselves (seed 0)."""
    s = make_system(cubic_cell(20.0), (64, 64, 64))
    return s, random_orbitals(s.a, s.miller, nb, 0)


def config3(nb: int = 512):
    """96x96x128 orthorhombic 22x22x30 bohr: 512 orbitals (seed 0)."""
    s = make_system(ortho_cell(22.0, 22.0, 30.0), (96, 96, 128))
    return s, random_orbitals(s.a, s.miller, nb, 0)


def config4_layout(seed: int = 0):
    """Grid sizes and band counts of the 16 uneven systems."""
    rng = np.random.default_rng(seed)
    grids = rng.choice([48, 64, 72, 96], 16)
    nbs = rng.integers(32, 257, 16)
    return [int(g) for g in grids], [int(b) for b in nbs]


def config4_system(s_index: int, nb_override: int | None = None):
    grids, nbs = config4_layout()
    g = grids[s_index]
    s = make_system(cubic_cell(g / 3.2), (g, g, g))
    nb = nbs[s_index] if nb_override is None else nb_override
    return s, random_orbitals(s.a, s.miller, nb, s_index)


def kmesh_points(a: np.ndarray, nk) -> np.ndarray:
    """Gamma-centred k-mesh, C order over (k1,k2,k3): k = sum_a (s_a / nk_a) b_a."""
    b = reciprocal_rows(a)
    pts = []
    for s1 in range(nk[0]):
        for s2 in range(nk[1]):
            for s3 in range(nk[2]):
                pts.append((s1 / nk[0]) * b[0] + (s2 / nk[1]) * b[1] + (s3 / nk[2]) * b[2])
    return np.array(pts)


def config5(nb: int = 256, n: int = 72, L: float = 24.0, nk=(2, 2, 2)):
    """72^3 cubic L=24, 2x2x2 Gamma-centred k-mesh, nb orbitals per k (seed = k index)."""
    s = make_system(cubic_cell(L), (n, n, n))
    kpts = kmesh_points(s.a, nk)
    orbs = [random_orbitals(s.a, s.miller, nb, ik) for ik in range(len(kpts))]
    return s, kpts, orbs
