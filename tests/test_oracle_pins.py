"""Pins of the CPU oracle against what the mathematics of section 4 fixes.

Each pin is chosen so that a plausible slip in the oracle (a dropped 4 pi or
volume, a wrong transform sign, a conjugate on the wrong factor, a transposed
axis, a wrong G = 0 rule) makes at least one of them fail; the mutation tests
at the bottom plant such slips in the oracle and check that.
"""
import os

import numpy as np
import pytest

import synth
from oracle import definitions, ewald, exx

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name, key):
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            if line.startswith(key + " "):
                return float(line.split()[1])
    raise KeyError(key)


# A small non-orthogonal cell with a non-cubic grid and q != 0: every axis,
# index and phase convention is exercised.
A_SKEW = np.array([[7.0, 0.0, 0.0], [1.0, 8.0, 0.0], [0.5, 0.3, 9.0]])
N_SKEW = (12, 16, 20)
Q_SKEW = np.array([0.11, -0.07, 0.05])


@pytest.fixture(scope="module")
def skew():
    s = synth.make_system(A_SKEW, N_SKEW)
    occ = synth.random_orbitals(A_SKEW, s.miller, 3, 5)
    tgt = synth.random_orbitals(A_SKEW, s.miller, 2, 6)
    f = np.array([1.0, 0.7, 0.3])
    return s, occ, tgt, f


def rel(x, y):
    return float(np.linalg.norm(np.ravel(x - y)) / np.linalg.norm(np.ravel(y)))


# P1 -- the plain discrete Fourier sum against the FFT (transform conventions)
def test_p1_dft_matches_fft_and_plane_wave():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 8, 12, 6)) + 1j * rng.standard_normal((2, 8, 12, 6))
    assert rel(exx.fft3(x, "dft"), np.fft.fftn(x, axes=(1, 2, 3))) < 1e-13
    assert rel(exx.bfft3(x, "dft"), exx.bfft3(x, "fft")) < 1e-13
    # a single plane wave: BFFT of a unit coefficient at G is e^{iG.r_m} exactly
    n = (8, 12, 6)
    m = np.array([[2, -3, 1]], dtype=np.int32)
    grid = exx.to_grid(np.array([[1.0 + 0j]]), m, n, "dft")[0]
    i1, i2, i3 = np.meshgrid(*(np.arange(k) for k in n), indexing="ij")
    want = np.exp(2j * np.pi * (2 * i1 / 8 - 3 * i2 / 12 + 1 * i3 / 6))
    assert np.abs(grid - want).max() < 1e-13


# P2 -- direct G-space convolution (no FFT) against the FFT route
def test_p2_direct_convolution(skew):
    s, occ, tgt, f = skew
    v_fft = exx.fock_apply(A_SKEW, N_SKEW, s.miller, Q_SKEW, occ, f, tgt, method="fft")
    v_dft = exx.fock_apply(A_SKEW, N_SKEW, s.miller, Q_SKEW, occ, f, tgt, method="dft")
    v_dir = definitions.fock_apply_direct(A_SKEW, s.miller, Q_SKEW, occ, f, tgt)
    assert rel(v_fft, v_dir) < 1e-13
    assert rel(v_dft, v_dir) < 1e-13
    g = np.array([1.0, 0.5])
    e = exx.fock_energy(A_SKEW, N_SKEW, s.miller, Q_SKEW, occ, f, tgt, g)
    e_dir = definitions.energy_gspace_direct(A_SKEW, s.miller, Q_SKEW, occ, f, tgt, g)
    assert abs(e - e_dir) < 1e-13 * abs(e_dir)


def test_p2_kernel_cutoff_direct(skew):
    # a Fock cutoff placed between |q+G|^2 shells: both routes must drop the same G
    s, occ, tgt, f = skew
    b = exx.reciprocal(A_SKEW)
    g2 = np.sort(np.unique(np.round(exx.box_qg2(A_SKEW, N_SKEW, Q_SKEW).ravel(), 9)))
    cut = 0.5 * (g2[200] + g2[201])
    v_fft = exx.fock_apply(A_SKEW, N_SKEW, s.miller, Q_SKEW, occ, f, tgt, ecut_fock=cut)
    v_dir = definitions.fock_apply_direct(A_SKEW, s.miller, Q_SKEW, occ, f, tgt, ecut_fock=cut)
    v_all = exx.fock_apply(A_SKEW, N_SKEW, s.miller, Q_SKEW, occ, f, tgt)
    assert rel(v_fft, v_dir) < 1e-13
    assert rel(v_fft, v_all) > 1e-6  # the cutoff really removed something
    del b


# P3 -- real-space double sum of section 4's exchange integral
def test_p3_realspace_double_sum():
    a = synth.cubic_cell(6.0)
    n = (12, 12, 12)
    s = synth.make_system(a, n)
    o = synth.random_orbitals(a, s.miller, 3, 0)
    f = np.array([1.0, 0.8, 0.5])
    er = definitions.energy_realspace(a, n, s.miller, o, f, o, f)
    eg = exx.fock_energy(a, n, s.miller, np.zeros(3), o, f, o, f)
    assert abs(er - eg) < 1e-12 * abs(eg)


def _vx_matrix(s, occ, f, chi, q, k0=0.0):
    v = exx.fock_apply(s.a, s.n, s.miller, q, occ, f, chi, k0=k0)
    return np.conj(chi) @ v.T  # M_ab = <chi_a | V_x | chi_b>


# P4, P5 -- Hermiticity and negative semidefiniteness of V_x
@pytest.mark.parametrize("q,k0", [(np.zeros(3), 0.0), (Q_SKEW, 0.0), (np.zeros(3), 37.5)])
def test_p4_p5_hermitian_negative(skew, q, k0):
    s, occ, _, f = skew
    rng = np.random.default_rng(11)
    chi = rng.standard_normal((6, s.npw)) + 1j * rng.standard_normal((6, s.npw))
    m = _vx_matrix(s, occ, f, chi, q, k0)
    assert np.linalg.norm(m - m.conj().T) <= 1e-14 * np.linalg.norm(m)
    ev = np.linalg.eigvalsh(0.5 * (m + m.conj().T))
    assert ev.max() <= 1e-14 * np.linalg.norm(m)
    assert ev.min() < -1e-6 * np.linalg.norm(m)


# P6 -- invariance under a unitary rotation of the occupied orbitals
def test_p6_unitary_invariance(skew):
    s, occ, tgt, _ = skew
    rng = np.random.default_rng(2)
    z = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
    u, _ = np.linalg.qr(z)
    occ_u = u.T @ occ
    ones = np.ones(3)
    e = exx.fock_energy(s.a, s.n, s.miller, np.zeros(3), occ, ones, occ, ones)
    e_u = exx.fock_energy(s.a, s.n, s.miller, np.zeros(3), occ_u, ones, occ_u, ones)
    assert abs(e - e_u) < 1e-13 * abs(e)
    v = exx.fock_apply(s.a, s.n, s.miller, Q_SKEW, occ, ones, tgt)
    v_u = exx.fock_apply(s.a, s.n, s.miller, Q_SKEW, occ_u, ones, tgt)
    assert rel(v_u, v) < 1e-13


def _gaussian(L, n, sigma):
    a = synth.cubic_cell(L)
    mill = synth.sphere_miller(a, n, synth.alias_free_ecut(a, n))
    c = np.exp(-sigma ** 2 * synth.sphere_g2(a, mill))
    c = (c / np.linalg.norm(c))[None, :].astype(np.complex128)
    return a, mill, c


# P7 -- closed-form Coulomb self-energy of a Gaussian pair density
def test_p7_gaussian_self_exchange():
    L, n, sigma = 20.0, (64, 64, 64), 1.2
    a, mill, c = _gaussian(L, n, sigma)
    alpha_m = ewald.madelung_simple_cubic()
    e0 = exx.fock_energy(a, n, mill, np.zeros(3), c, [1.0], c, [1.0])
    ref0 = -(1.0 / (2 * sigma * np.sqrt(np.pi)) - alpha_m / (2 * L) + 2 * np.pi * sigma ** 2 / L ** 3)
    assert abs(e0 - ref0) < 1e-12 * abs(ref0)
    # Gygi-Baldereschi with the auxiliary width equal to sigma^2: exact isolated value
    k0 = exx.gb_constant(a, n, (1, 1, 1), sigma ** 2)
    e1 = exx.fock_energy(a, n, mill, np.zeros(3), c, [1.0], c, [1.0], k0=k0)
    assert abs(e1 + 1.0 / (2 * sigma * np.sqrt(np.pi))) < 1e-12 * abs(e1)


# P8 -- GB constant on simple-cubic cells: closed form through the Madelung constant
@pytest.mark.parametrize("L,n,nq", [(20.0, 64, 1), (24.0, 72, 2), (10.0, 24, 3)])
def test_p8_gb_closed_form(L, n, nq):
    a = synth.cubic_cell(L)
    alpha = 10.0 / synth.alias_free_ecut(a, (n, n, n))
    k0 = exx.gb_constant(a, (n, n, n), (nq, nq, nq), alpha)
    ref = nq ** 3 * L ** 3 * ewald.madelung_simple_cubic() / (nq * L) - 4 * np.pi * alpha
    assert abs(k0 - ref) < 1e-12 * ref
    assert k0 > 0


def test_madelung_converged_and_golden():
    vals = [ewald.madelung_simple_cubic(eta) for eta in (0.9, 1.1, 1.3)]
    assert max(vals) - min(vals) < 1e-12
    assert abs(vals[0] - _golden("madelung_simple_cubic.txt", "alpha_M")) < 1e-12


# P9 -- band-group split sum, energy/apply consistency, gradient by finite differences
def test_p9_band_group_split_sum(skew):
    s, occ, tgt, f = skew
    full = exx.fock_apply(s.a, s.n, s.miller, Q_SKEW, occ, f, tgt)
    parts = sum(exx.fock_apply(s.a, s.n, s.miller, Q_SKEW, occ[sl], f[sl], tgt)
                for sl in (slice(0, 1), slice(1, 3)))
    assert rel(parts, full) < 1e-14


def test_p9_energy_is_half_expectation(skew):
    s, occ, _, f = skew
    q = np.zeros(3)
    e = exx.fock_energy(s.a, s.n, s.miller, q, occ, f, occ, f, k0=12.0)
    v = exx.fock_apply(s.a, s.n, s.miller, q, occ, f, occ, k0=12.0)
    e2 = 0.5 * np.sum(f * np.einsum("ij,ij->i", np.conj(occ), v).real)
    assert abs(e - e2) < 1e-13 * abs(e)


def test_p9_gradient_finite_difference(skew):
    s, occ, tgt, f = skew
    g = np.array([0.9, 0.4])
    q = Q_SKEW
    go, gt = exx.fock_energy_grad(s.a, s.n, s.miller, q, occ, f, tgt, g)
    rng = np.random.default_rng(4)
    do = rng.standard_normal(occ.shape) + 1j * rng.standard_normal(occ.shape)
    dt = rng.standard_normal(tgt.shape) + 1j * rng.standard_normal(tgt.shape)
    h = 1e-5
    ep = exx.fock_energy(s.a, s.n, s.miller, q, occ + h * do, f, tgt + h * dt, g)
    em = exx.fock_energy(s.a, s.n, s.miller, q, occ - h * do, f, tgt - h * dt, g)
    fd = (ep - em) / (2 * h)
    an = 2.0 * (np.sum(np.conj(go) * do).real + np.sum(np.conj(gt) * dt).real)
    assert abs(fd - an) < 1e-8 * abs(an)


# ---------------------------------------------------------------------------
# Mutation checks: plant a slip in the oracle and see a pin catch it.
# ---------------------------------------------------------------------------

def _p2_ok(skew):
    s, occ, tgt, f = skew
    v = exx.fock_apply(A_SKEW, N_SKEW, s.miller, Q_SKEW, occ, f, tgt, method="fft")
    return rel(v, definitions.fock_apply_direct(A_SKEW, s.miller, Q_SKEW, occ, f, tgt)) < 1e-13


def _p7_ok():
    L, n, sigma = 20.0, (48, 48, 48), 1.2
    a, mill, c = _gaussian(L, n, sigma)
    k0 = exx.gb_constant(a, n, (1, 1, 1), sigma ** 2)
    e1 = exx.fock_energy(a, n, mill, np.zeros(3), c, [1.0], c, [1.0], k0=k0)
    return abs(e1 + 1.0 / (2 * sigma * np.sqrt(np.pi))) < 1e-10


def test_mutations_are_caught(skew, monkeypatch):
    assert _p2_ok(skew) and _p7_ok()
    orig_kernel = exx.coulomb_kernel
    orig_fft3 = exx.fft3
    orig_vol = exx.volume
    orig_slots = exx.box_slots

    monkeypatch.setattr(exx, "coulomb_kernel", lambda *a, **k: orig_kernel(*a, **k) / (4 * np.pi))
    assert not _p2_ok(skew) and not _p7_ok()
    monkeypatch.setattr(exx, "coulomb_kernel", orig_kernel)

    monkeypatch.setattr(exx, "fft3", lambda x, method="auto": exx.bfft3(x, method))
    assert not _p2_ok(skew)
    monkeypatch.setattr(exx, "fft3", orig_fft3)

    monkeypatch.setattr(exx, "volume", lambda a: 1.0)
    assert not _p2_ok(skew) and not _p7_ok()
    monkeypatch.setattr(exx, "volume", orig_vol)

    def swapped(miller, n):
        m = np.asarray(miller)[:, [0, 2, 1]]
        return orig_slots(m, n)
    monkeypatch.setattr(exx, "box_slots", swapped)
    assert not _p2_ok(skew)
    monkeypatch.setattr(exx, "box_slots", orig_slots)

    orig_apply = exx.fock_apply

    def conj_target(a, n, miller, q, c_occ, f_occ, c_tgt, *args, **kw):
        # conjugate placed on the target instead of the occupied orbital
        return np.conj(orig_apply(a, n, miller, -np.asarray(q), np.conj(c_occ), f_occ,
                                  np.conj(c_tgt), *args, **kw))
    monkeypatch.setattr(exx, "fock_apply", conj_target)
    s, occ, tgt, f = skew
    v = exx.fock_apply(A_SKEW, N_SKEW, s.miller, Q_SKEW, occ, f, tgt)
    assert rel(v, definitions.fock_apply_direct(A_SKEW, s.miller, Q_SKEW, occ, f, tgt)) > 1e-6


def gaussian_bloch_sets(L, n, sigma, nq):
    """Bloch sums of one Gaussian per cell: c_k(G) ~ exp(-sigma^2 |k+G|^2).

    The pair density of the sets at k' and k then has the coefficient
    Omega^-1 exp(-sigma^2 |q+G|^2 / 2) at G, q = k - k' (a normalised Gaussian
    charge of width sigma, carried by the Bloch phase q)."""
    a = synth.cubic_cell(L)
    mill = synth.sphere_miller(a, n, synth.alias_free_ecut(a, n))
    kpts = synth.kmesh_points(a, nq)
    g = mill.astype(np.float64) @ synth.reciprocal_rows(a)
    sets = []
    for k in kpts:
        kg = g + k[None, :]
        c = np.exp(-sigma ** 2 * np.einsum("ij,ij->i", kg, kg))
        sets.append((c / np.linalg.norm(c))[None, :].astype(np.complex128))
    return a, mill, kpts, sets


# P7 on a k-mesh: a Gaussian Wannier function, weights 1/N_k.  The mesh sum
# with the mesh's Gygi-Baldereschi constant (width sigma^2) is exact for the
# Gaussian charge, so E is again the isolated self-exchange -1/(2 sigma sqrt pi).
def test_p7_gaussian_kmesh_gb():
    L, n, sigma, nq = 20.0, (64, 64, 64), 1.2, (2, 2, 2)
    a, mill, kpts, sets = gaussian_bloch_sets(L, n, sigma, nq)
    nk = len(kpts)
    k0 = exx.gb_constant(a, n, nq, sigma ** 2)
    e = exx.fock_energy_kmesh(a, n, mill, kpts, sets, [np.array([1.0 / nk])] * nk, k0=k0)
    assert abs(e + 1.0 / (2 * sigma * np.sqrt(np.pi))) < 1e-12 * abs(e)


def test_kmesh_gradient_finite_difference():
    a = synth.cubic_cell(8.0)
    n = (12, 12, 12)
    s = synth.make_system(a, n)
    nq = (2, 1, 1)
    kpts = synth.kmesh_points(a, nq)
    sets = [synth.random_orbitals(a, s.miller, 2, 20 + k) for k in range(len(kpts))]
    wts = [np.array([0.5, 0.4]), np.array([0.45, 0.3])]
    k0 = exx.gb_constant(a, n, nq, 0.5)
    grads = exx.fock_energy_kmesh_grad(a, n, s.miller, kpts, sets, wts, k0=k0)
    rng = np.random.default_rng(8)
    d = [rng.standard_normal(c.shape) + 1j * rng.standard_normal(c.shape) for c in sets]
    nrm = np.sqrt(sum(np.sum(np.abs(x) ** 2) for x in d))
    d = [x / nrm for x in d]
    h = 1e-4
    ep = exx.fock_energy_kmesh(a, n, s.miller, kpts, [c + h * x for c, x in zip(sets, d)], wts, k0=k0)
    em = exx.fock_energy_kmesh(a, n, s.miller, kpts, [c - h * x for c, x in zip(sets, d)], wts, k0=k0)
    fd = (ep - em) / (2 * h)
    an = 2.0 * sum(np.sum(np.conj(g) * x).real for g, x in zip(grads, d))
    assert abs(fd - an) < 1e-8 * abs(an)


def test_gamma_real_orbitals_give_a_real_exchange_potential():
    """For real orbitals at q = 0 every pair density and potential is real, so
    V_x psi is a real function: its coefficients are Hermitian."""
    s = synth.make_system(synth.cubic_cell(8.0), (24, 24, 24))
    c = synth.gamma_orbitals(s.a, s.miller, 5, 6)
    f = np.array([1.0, 0.9, 0.6, 0.4, 0.2])
    v = exx.fock_apply(s.a, s.n, s.miller, np.zeros(3), c, f, c)
    index = {tuple(m): p for p, m in enumerate(s.miller)}
    neg = np.array([index[tuple(-m)] for m in s.miller])
    assert np.abs(v - np.conj(v[:, neg])).max() < 1e-14 * np.abs(v).max()
    # and not trivially: a complex block breaks the symmetry
    cz = synth.random_orbitals(s.a, s.miller, 5, 6)
    vz = exx.fock_apply(s.a, s.n, s.miller, np.zeros(3), cz, f, cz)
    assert np.abs(vz - np.conj(vz[:, neg])).max() > 1e-3 * np.abs(vz).max()
