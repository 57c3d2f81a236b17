"""Plain definitions of the exchange quantities, with no FFT anywhere.

TEST INFRASTRUCTURE ONLY (see the package docstring).  These are O(npw^2)
and O(N^2) per pair and serve only to pin the FFT route on tiny inputs.

* ``pair_density``: rho_ij(G) = Omega^{-1} sum_{G1 in S} conj(c_i(G1)) d_j(G1+G),
  the Fourier coefficient of the periodic part of phi_i* psi_j -- the overlap
  charge density M of section 4.
* ``fock_apply_direct``: (V_x psi_j)(G) = -sum_i f_i sum_{G1 in S} c_i(G1) v_ij(G-G1)
  with v_ij = K(q+G) rho_ij(G), projected on S (section 4, V_x on a state,
  read as an operator that multiplies back by the occupied orbital).
* ``energy_realspace``: the exchange-energy double integral of section 4,
  -1/2 sum_ij f_i g_j int int rho_ij*(r) v(r - r') rho_ij(r'), evaluated as a
  double sum over the real-space grid with the periodic Coulomb potential
  written out as a plane-wave sum; exact for band-limited densities.
"""
from __future__ import annotations

import numpy as np

FOUR_PI = 4.0 * np.pi


def _recip(a):
    return 2.0 * np.pi * np.linalg.inv(np.asarray(a, dtype=np.float64)).T


def pair_density(c_i, d_j, miller, omega: float):
    """Return (diff_miller [nd,3], rho [nd]) over all G = G2 - G1, G1, G2 in S."""
    m = np.asarray(miller, dtype=np.int64)
    span = 2 * int(np.abs(m).max()) + 1
    off = span // 2 * 2
    size = 2 * off + 1
    rho = np.zeros((size, size, size), dtype=np.complex128)
    hit = np.zeros((size, size, size), dtype=bool)
    for a in range(m.shape[0]):
        d = m - m[a] + off
        np.add.at(rho, (d[:, 0], d[:, 1], d[:, 2]), np.conj(c_i[a]) * d_j)
        hit[d[:, 0], d[:, 1], d[:, 2]] = True
    idx = np.argwhere(hit)
    return idx - off, rho[idx[:, 0], idx[:, 1], idx[:, 2]] / omega


def kernel_values(a, q, gm, k0: float = 0.0, ecut_fock: float = 0.0):
    """4 pi / |q+G|^2 at Miller indices gm; the point q+G = 0 takes k0."""
    g = np.asarray(q, dtype=np.float64)[None, :] + gm.astype(np.float64) @ _recip(a)
    g2 = np.einsum("ij,ij->i", g, g)
    k = np.empty_like(g2)
    zero = g2 == 0.0
    k[~zero] = FOUR_PI / g2[~zero]
    k[zero] = k0
    if ecut_fock > 0.0:
        k[g2 > ecut_fock] = 0.0
    return k


def fock_apply_direct(a, miller, q, c_occ, f_occ, c_tgt, k0: float = 0.0,
                      ecut_fock: float = 0.0):
    omega = float(abs(np.linalg.det(a)))
    m = np.asarray(miller, dtype=np.int64)
    out = np.zeros((c_tgt.shape[0], m.shape[0]), dtype=np.complex128)
    for j in range(c_tgt.shape[0]):
        for i in range(c_occ.shape[0]):
            gm, rho = pair_density(c_occ[i], c_tgt[j], m, omega)
            v = kernel_values(a, q, gm, k0, ecut_fock) * rho
            vmap = {tuple(x): val for x, val in zip(gm, v)}
            for p in range(m.shape[0]):
                s = 0.0j
                for g1 in range(m.shape[0]):
                    key = tuple(m[p] - m[g1])
                    if key in vmap:
                        s += c_occ[i, g1] * vmap[key]
                out[j, p] -= f_occ[i] * s
    return out


def energy_gspace_direct(a, miller, q, c_occ, f_occ, c_tgt, g_tgt, k0: float = 0.0):
    omega = float(abs(np.linalg.det(a)))
    e = 0.0
    for j in range(c_tgt.shape[0]):
        for i in range(c_occ.shape[0]):
            gm, rho = pair_density(c_occ[i], c_tgt[j], miller, omega)
            e += f_occ[i] * g_tgt[j] * omega * float(np.sum(kernel_values(a, q, gm, k0) * np.abs(rho) ** 2))
    return -0.5 * e


def energy_realspace(a, n, miller, c_occ, f_occ, c_tgt, g_tgt):
    """Real-space double sum at q = 0 with the G = 0 term of v removed.

    E = -1/2 sum_ij f_i g_j (Omega/N)^2 sum_{m,m'} conj(rho_ij(r_m)) W(r_m - r_m') rho_ij(r_m'),
    rho_ij(r) = conj(phi_i(r)) psi_j(r) with the orbitals summed as plane
    waves at the grid points, and W(r) = Omega^-1 sum_{G in box, G != 0}
    4 pi e^{iG.r} / |G|^2 the periodic Coulomb potential.  The grid
    quadrature is exact because every integrand is band-limited below the
    grid's Nyquist limit.  O(N^2) per pair: tiny grids only.
    """
    a = np.asarray(a, dtype=np.float64)
    n = tuple(int(x) for x in n)
    omega = float(abs(np.linalg.det(a)))
    N = n[0] * n[1] * n[2]
    b = _recip(a)
    i1, i2, i3 = np.meshgrid(np.arange(n[0]), np.arange(n[1]), np.arange(n[2]), indexing="ij")
    idx = np.stack([i1.ravel(), i2.ravel(), i3.ravel()], axis=1)       # grid point m
    r = (idx / np.asarray(n, dtype=np.float64)) @ a                     # r_m
    gs = np.asarray(miller, dtype=np.float64) @ b
    phase = np.exp(1j * r @ gs.T)                                        # [N, npw]
    phi = (phase @ np.asarray(c_occ).T).T / np.sqrt(omega)
    psi = (phase @ np.asarray(c_tgt).T).T / np.sqrt(omega)

    def sidx(k):
        t = np.arange(k)
        return np.where(t < k // 2, t, t - k)

    mm = np.stack(np.meshgrid(sidx(n[0]), sidx(n[1]), sidx(n[2]), indexing="ij"), -1).reshape(-1, 3)
    mm = mm[np.any(mm != 0, axis=1)]
    gb = mm.astype(np.float64) @ b
    wg = FOUR_PI / np.einsum("ij,ij->i", gb, gb)
    # W at every grid offset d (r_d is a grid point; W is lattice periodic)
    w_of_d = (np.exp(1j * r @ gb.T) @ wg).real / omega                 # [N]
    # W(r_m - r_m') = W(r_{(m - m') mod n})
    d = (idx[:, None, :] - idx[None, :, :]) % np.asarray(n)
    wmat = w_of_d[(d[..., 0] * n[1] + d[..., 1]) * n[2] + d[..., 2]]    # [N, N]
    e = 0.0
    for j in range(psi.shape[0]):
        for i in range(phi.shape[0]):
            rho = np.conj(phi[i]) * psi[j]
            val = np.conj(rho) @ (wmat @ rho)
            e += f_occ[i] * g_tgt[j] * val.real * (omega / N) ** 2
    return -0.5 * e
