"""FFT route of the plane-wave exact exchange, in FP64 on the CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Conventions (the paper leaves them open; these are the readings used here):

* Hartree atomic units; Coulomb kernel K(q+G) = 4 pi / |q+G|^2.
* An orbital is a list of plane-wave coefficients c(G) on a sphere S, with
  phi(r) = Omega^{-1/2} sum_G c(G) e^{i G.r} (periodic part); sum |c|^2 = 1.
* FFT  = unnormalised sum_r x(r) e^{-i G.r};  BFFT = unnormalised
  sum_G x(G) e^{+i G.r};  r_m = sum_a (m_a / n_a) a_a.
* ``method="dft"`` evaluates every transform as the plain discrete Fourier
  sum, one axis at a time (the 3-D kernel e^{-iG.r} factorises exactly over
  the axes); ``method="fft"`` uses scipy's FFT; ``"auto"`` picks the plain
  sum up to 24^3 points.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

FOUR_PI = 4.0 * np.pi


# --------------------------------------------------------------------------
# Lattice helpers
# --------------------------------------------------------------------------

def volume(a) -> float:
    return float(abs(np.linalg.det(np.asarray(a, dtype=np.float64))))


def reciprocal(a) -> np.ndarray:
    """Rows b_i with a_i . b_j = 2 pi delta_ij."""
    return 2.0 * np.pi * np.linalg.inv(np.asarray(a, dtype=np.float64)).T


def box_index(n: int) -> np.ndarray:
    """Signed index of each FFT slot: i if i < n/2 else i - n."""
    i = np.arange(n)
    return np.where(i < (n + 1) // 2, i, i - n) if n % 2 else np.where(i < n // 2, i, i - n)


def box_qg2(a, n, q) -> np.ndarray:
    """|q + G|^2 at every slot of the FFT box, G = m1 b1 + m2 b2 + m3 b3."""
    b = reciprocal(a)
    m1, m2, m3 = np.meshgrid(box_index(n[0]), box_index(n[1]), box_index(n[2]), indexing="ij")
    gx = q[0] + m1 * b[0, 0] + m2 * b[1, 0] + m3 * b[2, 0]
    gy = q[1] + m1 * b[0, 1] + m2 * b[1, 1] + m3 * b[2, 1]
    gz = q[2] + m1 * b[0, 2] + m2 * b[1, 2] + m3 * b[2, 2]
    return gx * gx + gy * gy + gz * gz


def q_is_lattice_vector(a, q) -> bool:
    frac = np.asarray(a, dtype=np.float64) @ np.asarray(q, dtype=np.float64) / (2.0 * np.pi)
    return bool(np.all(np.abs(frac - np.round(frac)) < 1e-9))


def coulomb_kernel(a, n, q, ecut_fock: float = 0.0, k0: float = 0.0) -> np.ndarray:
    """K(q+G) on the FFT box (section 4, reciprocal-space exchange energy).

    K = 4 pi / |q+G|^2 where |q+G|^2 <= ecut_fock (ecut_fock <= 0: the whole
    box).  The single point q+G = 0 (q = 0, G = 0) takes the value ``k0``:
    0 drops the divergent term, a Gygi-Baldereschi constant corrects it.
    A non-zero q that is itself a reciprocal-lattice vector is rejected.
    """
    q = np.asarray(q, dtype=np.float64)
    q_zero = bool(np.all(q == 0.0))
    if not q_zero and q_is_lattice_vector(a, q):
        raise ValueError("q + G = 0 for a non-zero q: fold q into the Brillouin zone")
    g2 = box_qg2(a, n, q)
    if q_zero:
        g2[0, 0, 0] = 1.0  # placeholder, overwritten below
    k = FOUR_PI / g2
    if ecut_fock > 0.0:
        k[g2 > ecut_fock] = 0.0
    if q_zero:
        k[0, 0, 0] = k0
    return k


def exchange_grid_need(a, miller, ecut_fock: float, qs=None) -> tuple:
    """Smallest grid size per axis on which the FFT route gives the
    grid-independent result of the reduced-cutoff exchange (section 6: the
    Fock cutoff may be set below the density cutoff).

    Pair densities have components at |m_a| <= 2 M_a (M_a: the sphere's
    largest |m_a|).  A grid of n_a points folds the component at m_a + t n_a
    onto m_a, so the components that K keeps (|m_a| <= F_a, the largest |m_a|
    of the points with |q+G|^2 <= ecut_fock) are untouched when
    n_a > F_a + 2 M_a, and phi * v (components up to M_a + min(F_a, 2 M_a))
    lands on the sphere untouched under the same condition.  F_a here is found
    by listing the lattice points of the ball; ecut_fock <= 0 means no cutoff.
    """
    a = np.asarray(a, dtype=np.float64)
    m = np.abs(np.asarray(miller, dtype=np.int64))
    M = m.max(axis=0)
    if ecut_fock <= 0.0:
        return tuple(int(4 * x + 1) for x in M)
    b = reciprocal(a)
    qs = np.zeros((1, 3)) if qs is None else np.asarray(qs, dtype=np.float64).reshape(-1, 3)
    F = np.zeros(3, dtype=np.int64)
    for q in qs:
        # enumerate a box that surely holds the ball, then keep the ball
        r = int(np.ceil(np.sqrt(ecut_fock) * np.linalg.norm(a, axis=1).max() / (2 * np.pi)
                        + np.abs(a @ q).max() / (2 * np.pi))) + 1
        ax = np.arange(-r, r + 1)
        mm = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), axis=-1).reshape(-1, 3)
        g = q[None, :] + mm @ b
        inside = np.einsum("ij,ij->i", g, g) <= ecut_fock
        if inside.any():
            F = np.maximum(F, np.abs(mm[inside]).max(axis=0))
    return tuple(int(min(f, 2 * x) + 2 * x + 1) for f, x in zip(F, M))


def gb_constant(a, n, nq, alpha: float) -> float:
    """Gygi-Baldereschi value of K at q+G = 0 for a Gamma-centred nq mesh.

    With the auxiliary F(k) = 4 pi e^{-alpha k^2} / k^2, whose Brillouin-zone
    integral is known, K0 is chosen so that the mesh-weighted lattice sum of
    F, with K0 in place of the divergent term, equals that integral:
      (1/N_q) [K0 + sum_{q in mesh} sum_{G in box, q+G != 0} F(q+G)]
          = Omega / sqrt(pi alpha).
    """
    omega = volume(a)
    b = reciprocal(a)
    nq = [int(x) for x in nq]
    total = 0.0
    for s1 in range(nq[0]):
        for s2 in range(nq[1]):
            for s3 in range(nq[2]):
                q = (s1 / nq[0]) * b[0] + (s2 / nq[1]) * b[1] + (s3 / nq[2]) * b[2]
                g2 = box_qg2(a, n, q)
                if s1 == 0 and s2 == 0 and s3 == 0:
                    g2 = g2.copy()
                    f = np.zeros_like(g2)
                    mask = np.ones(g2.shape, dtype=bool)
                    mask[0, 0, 0] = False
                    f[mask] = FOUR_PI * np.exp(-alpha * g2[mask]) / g2[mask]
                else:
                    f = FOUR_PI * np.exp(-alpha * g2) / g2
                total += float(np.sum(f))
    nqt = nq[0] * nq[1] * nq[2]
    return nqt * omega / np.sqrt(np.pi * alpha) - total


# --------------------------------------------------------------------------
# Transforms
# --------------------------------------------------------------------------

def _dft_axis(x: np.ndarray, axis: int, sign: int) -> np.ndarray:
    n = x.shape[axis]
    j = np.arange(n)
    w = np.exp(sign * 2j * np.pi * np.outer(j, j) / n)
    return np.moveaxis(np.tensordot(w, np.moveaxis(x, axis, 0), axes=(1, 0)), 0, axis)


def _pick(method: str, shape) -> str:
    if method == "auto":
        return "dft" if int(np.prod(shape[-3:])) <= 24 ** 3 else "fft"
    return method


def fft3(x: np.ndarray, method: str = "auto") -> np.ndarray:
    """Unnormalised forward transform sum_r x(r) e^{-iG.r} over the last 3 axes."""
    if _pick(method, x.shape) == "dft":
        for ax in (-3, -2, -1):
            x = _dft_axis(x, x.ndim + ax, -1)
        return x
    return sfft.fftn(x, axes=(-3, -2, -1), workers=1)


def bfft3(x: np.ndarray, method: str = "auto") -> np.ndarray:
    """Unnormalised backward transform sum_G x(G) e^{+iG.r} over the last 3 axes."""
    if _pick(method, x.shape) == "dft":
        for ax in (-3, -2, -1):
            x = _dft_axis(x, x.ndim + ax, +1)
        return x
    n = int(np.prod(x.shape[-3:]))
    return sfft.ifftn(x, axes=(-3, -2, -1), workers=1) * n


def box_slots(miller, n):
    m = np.asarray(miller, dtype=np.int64)
    return (m[:, 0] % n[0], m[:, 1] % n[1], m[:, 2] % n[2])


def to_grid(c, miller, n, method: str = "auto") -> np.ndarray:
    """Orbitals [nb, npw] on the sphere -> phi~(r) = sum_G c(G) e^{iG.r} on the box.

    Section 4: the orbitals are taken from reciprocal to real space before the
    overlap product is formed.
    """
    c = np.atleast_2d(np.asarray(c, dtype=np.complex128))
    box = np.zeros((c.shape[0],) + tuple(n), dtype=np.complex128)
    s = box_slots(miller, n)
    box[:, s[0], s[1], s[2]] = c
    return bfft3(box, method)


# --------------------------------------------------------------------------
# The exchange operator and energy
# --------------------------------------------------------------------------

def fock_apply(a, n, miller, q, c_occ, f_occ, c_tgt, ecut_fock: float = 0.0,
               k0: float = 0.0, method: str = "auto") -> np.ndarray:
    """(V_x psi_j)(G) on the sphere for every target j (section 4, V_x on a state).

    For each occupied i and target j: pair density conj(phi~_i) psi~_j in real
    space, forward transform, multiply by K(q+G), backward transform, multiply
    by f_i phi~_i, accumulate; then one forward transform per target, the
    sphere components, and the overall factor -1 / (Omega N^2).
    Returns [n_tgt, npw] complex128.
    """
    n = tuple(int(x) for x in n)
    omega = volume(a)
    N = n[0] * n[1] * n[2]
    kern = coulomb_kernel(a, n, q, ecut_fock, k0)
    f_occ = np.asarray(f_occ, dtype=np.float64)
    phi = to_grid(c_occ, miller, n, method)
    psi = to_grid(c_tgt, miller, n, method)
    slots = box_slots(miller, n)
    out = np.empty((psi.shape[0], len(slots[0])), dtype=np.complex128)
    for j in range(psi.shape[0]):
        acc = np.zeros(n, dtype=np.complex128)
        for i in range(phi.shape[0]):
            rho = fft3(np.conj(phi[i]) * psi[j], method)
            v = bfft3(kern * rho, method)
            acc += f_occ[i] * phi[i] * v
        out[j] = -fft3(acc, method)[slots] / (omega * N * N)
    return out


def fock_energy(a, n, miller, q, c_occ, f_occ, c_tgt, g_tgt, ecut_fock: float = 0.0,
                k0: float = 0.0, method: str = "auto") -> float:
    """E = -1/2 sum_ij f_i g_j Omega sum_G K(q+G) |rho_ij(G)|^2 (section 4).

    rho_ij(G) = FFT[conj(phi~_i) psi~_j](G) / (N Omega) is the overlap
    density of the reciprocal-space exchange-energy expression.
    """
    n = tuple(int(x) for x in n)
    omega = volume(a)
    N = n[0] * n[1] * n[2]
    kern = coulomb_kernel(a, n, q, ecut_fock, k0)
    f_occ = np.asarray(f_occ, dtype=np.float64)
    g_tgt = np.asarray(g_tgt, dtype=np.float64)
    phi = to_grid(c_occ, miller, n, method)
    psi = to_grid(c_tgt, miller, n, method)
    e = 0.0
    for j in range(psi.shape[0]):
        for i in range(phi.shape[0]):
            rho = fft3(np.conj(phi[i]) * psi[j], method)
            e += f_occ[i] * g_tgt[j] * float(np.sum(kern * (rho.real ** 2 + rho.imag ** 2)))
    return -0.5 * e / (omega * N * N)


def fock_energy_grad(a, n, miller, q, c_occ, f_occ, c_tgt, g_tgt, ecut_fock: float = 0.0,
                     k0: float = 0.0, method: str = "auto"):
    """Wirtinger derivatives (dE/dc_occ*, dE/dc_tgt*) of ``fock_energy``.

    dE/dd_j* = 1/2 g_j (V_x psi_j) with the operator built on the occupied set;
    dE/dc_i* = 1/2 f_i (V'_x phi_i) with the roles of the two sets swapped
    (occupied <- targets with weights g) and q -> -q.
    """
    q = np.asarray(q, dtype=np.float64)
    g_tgt = np.asarray(g_tgt, dtype=np.float64)
    f_occ = np.asarray(f_occ, dtype=np.float64)
    vt = fock_apply(a, n, miller, q, c_occ, f_occ, c_tgt, ecut_fock, k0, method)
    vo = fock_apply(a, n, miller, -q, c_tgt, g_tgt, c_occ, ecut_fock, k0, method)
    return 0.5 * f_occ[:, None] * vo, 0.5 * g_tgt[:, None] * vt


# --------------------------------------------------------------------------
# k-point mesh (section 4: the sums over k and q)
# --------------------------------------------------------------------------

def fock_energy_kmesh(a, n, miller, kpts, sets, weights, ecut_fock: float = 0.0, k0: float = 0.0,
                      method: str = "auto") -> float:
    """E = sum over all (k, k') blocks of the block energy with targets at k,
    occupied orbitals at k' and q = k - k' (not folded back into the zone).

    ``weights[k]`` already carry the 1/N_k of the mesh average.  The point
    q + G = 0 (k = k', G = 0) takes ``k0``.
    """
    e = 0.0
    for kt in range(len(sets)):
        for ko in range(len(sets)):
            q = np.asarray(kpts[kt], dtype=np.float64) - np.asarray(kpts[ko], dtype=np.float64)
            e += fock_energy(a, n, miller, q, sets[ko], weights[ko], sets[kt], weights[kt], ecut_fock, k0, method)
    return e


def fock_energy_kmesh_grad(a, n, miller, kpts, sets, weights, ecut_fock: float = 0.0, k0: float = 0.0,
                           method: str = "auto"):
    """Wirtinger derivatives dE/dconj(c_k) of ``fock_energy_kmesh``: the sum of
    each block's target and occupied gradients."""
    grads = [np.zeros_like(np.asarray(c, dtype=np.complex128)) for c in sets]
    for kt in range(len(sets)):
        for ko in range(len(sets)):
            q = np.asarray(kpts[kt], dtype=np.float64) - np.asarray(kpts[ko], dtype=np.float64)
            go, gt = fock_energy_grad(a, n, miller, q, sets[ko], weights[ko], sets[kt], weights[kt],
                                      ecut_fock, k0, method)
            grads[ko] += go
            grads[kt] += gt
    return grads
