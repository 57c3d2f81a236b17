"""The differentiable form: exchange energy on a k-point mesh behind
torch.autograd.Function, against the oracle, finite differences and fock_apply.

PyTorch's gradient of a real loss with respect to complex z is
2 dL/dconj(z); the exchange operator here is the paper's negative V_x, so
autograd(E) = 2 * (w_k) * sum_k' V_x psi_k (checked element by element).
"""
import numpy as np
import pytest

import synth
from oracle import exx
from tests.helpers import host, rel_fro, report

pytestmark = pytest.mark.gpu


def _mods():
    from paper_1305_7313_amd import autograd, fock
    return fock, autograd


def _gb_cell(F, s, nq, alpha):
    return F.Cell(s.a, s.n, s.miller, g0=F.FOCK_G0_GB, gb_alpha=alpha, nq=nq)


@pytest.fixture(scope="module")
def reduced():
    """Reduced instance of the differentiable workload: 24^3, 2x2x2 mesh, 4 orbitals per k."""
    s = synth.make_system(synth.cubic_cell(8.0), (24, 24, 24))
    nq = (2, 2, 2)
    kpts = synth.kmesh_points(s.a, nq)
    sets = [synth.random_orbitals(s.a, s.miller, 4, k) for k in range(8)]
    w = [np.full(4, 1.0 / 8) for _ in range(8)]
    alpha = 10.0 / s.ecut
    k0 = exx.gb_constant(s.a, s.n, nq, alpha)
    e = exx.fock_energy_kmesh(s.a, s.n, s.miller, kpts, sets, w, k0=k0)
    g = exx.fock_energy_kmesh_grad(s.a, s.n, s.miller, kpts, sets, w, k0=k0)
    return s, nq, kpts, sets, w, alpha, e, g


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_kmesh_energy_grad_vs_oracle(reduced, prec):
    import torch
    F, A = _mods()
    s, nq, kpts, sets, w, alpha, e_ref, g_ref = reduced
    cdt = torch.complex128 if prec == "c128" else torch.complex64
    tol = 1e-10 if prec == "c128" else 1e-5
    cell = _gb_cell(F, s, nq, alpha)
    C = torch.from_numpy(np.stack(sets)).to(cdt).cuda()
    W = torch.from_numpy(np.stack(w)).cuda()
    e = float(host(F.fock_energy_kmesh(cell, kpts, C, W)))
    one = torch.ones((), dtype=torch.float64, device="cuda")
    G = torch.empty_like(C)
    F.fock_energy_kmesh_backward(cell, kpts, C, W, one, [G[k] for k in range(8)])
    err_e = abs(e - e_ref) / abs(e_ref)
    err_g = rel_fro(host(G), np.stack(g_ref))
    report(f"kmesh reduced {prec}", E=e, E_ref=e_ref, E_rel=err_e, grad_rel=err_g)
    assert err_e < tol and err_g < tol


def test_kmesh_autograd_fd_and_apply(reduced):
    """autograd backward == 2 * Wirtinger gradient; per-coefficient central
    differences (h = 1e-4, FP64); and the gradient rebuilt from fock_apply."""
    import torch
    F, A = _mods()
    s, nq, kpts, sets, w, alpha, _, _ = reduced
    cell = _gb_cell(F, s, nq, alpha)
    C = torch.from_numpy(np.stack(sets)).cuda().requires_grad_(True)
    W = torch.from_numpy(np.stack(w)).cuda()
    E = A.exchange_energy_kmesh(C, W, cell, kpts)
    E.backward()
    grad = host(C.grad)
    # finite differences on individual coefficients, real and imaginary parts
    rng = np.random.default_rng(5)
    h = 1e-4
    worst = 0.0
    Cd = C.detach()
    for _ in range(6):
        k, b, p = rng.integers(8), rng.integers(4), rng.integers(s.npw)
        for unit in (1.0, 1j):
            Cp = Cd.clone()
            Cm = Cd.clone()
            Cp[k, b, p] += h * unit
            Cm[k, b, p] -= h * unit
            fd = (float(host(F.fock_energy_kmesh(cell, kpts, Cp, W))) -
                  float(host(F.fock_energy_kmesh(cell, kpts, Cm, W)))) / (2 * h)
            an = (np.conj(grad[k, b, p]) * unit).real  # Re(conj(g) d), g = torch grad
            worst = max(worst, abs(fd - an) / (abs(an) + 1e-12))
    report("kmesh per-coefficient FD", worst_rel=worst)
    assert worst < 1e-5
    # gradient from the exchange operator: 2 w_k sum_k' V_x(occ = k', q = k - k') psi_k
    rebuilt = np.zeros_like(grad)
    for kt in range(8):
        for ko in range(8):
            q = kpts[kt] - kpts[ko]
            cq = cell if np.all(q == 0) else F.Cell(s.a, s.n, s.miller)
            v = F.fock_apply(cq, q, Cd[ko], W[ko], Cd[kt])
            rebuilt[kt] += host(v)
        rebuilt[kt] *= 2.0 * w[kt][:, None]
    err = rel_fro(grad, rebuilt)
    report("kmesh autograd vs 2 w V_x psi", rel=err)
    assert err < 1e-12


def test_autograd_single_block():
    """ExchangeEnergy (one block, q = 0, occupied == target): torch grad == 2 f V_x psi."""
    import torch
    F, A = _mods()
    s = synth.make_system(synth.cubic_cell(10.0), (24, 24, 24))
    occ = synth.random_orbitals(s.a, s.miller, 10, 2)
    f = np.linspace(1.0, 0.5, 10)
    cell = F.Cell(s.a, s.n, s.miller)
    C = torch.from_numpy(occ).cuda().requires_grad_(True)
    fd = torch.from_numpy(f).cuda()
    E = A.exchange_energy(C, C, fd, fd, cell)
    E.backward()
    v = host(F.fock_apply(cell, (0, 0, 0), C.detach(), fd, C.detach()))
    err = rel_fro(host(C.grad), 2.0 * f[:, None] * v)
    report("single-block autograd vs 2 f V_x psi", rel=err)
    assert err < 1e-12


def test_kmesh_gaussian_closed_form():
    """GPU k-mesh sum with the mesh GB constant reproduces -1/(2 sigma sqrt(pi))."""
    import torch
    F, _ = _mods()
    from tests.test_oracle_pins import gaussian_bloch_sets
    L, n, sigma, nq = 20.0, (64, 64, 64), 1.2, (2, 2, 2)
    a, mill, kpts, sets = gaussian_bloch_sets(L, n, sigma, nq)
    cell = F.Cell(a, n, mill, g0=F.FOCK_G0_GB, gb_alpha=sigma ** 2, nq=nq)
    C = torch.from_numpy(np.stack(sets)).cuda()
    W = torch.full((8, 1), 1.0 / 8, dtype=torch.float64, device="cuda")
    e = float(host(F.fock_energy_kmesh(cell, kpts, C, W)))
    ref = -1.0 / (2 * sigma * np.sqrt(np.pi))
    report("kmesh Gaussian closed form", E=e, ref=ref, rel=abs(e - ref) / abs(ref))
    assert abs(e - ref) < 1e-11 * abs(ref)


@pytest.fixture(scope="module")
def kmesh17():
    """2x2x2 mesh, 17 orbitals per k (pair tiles of 16 and 1), random
    weights; the oracle gradient on rows 0 and 16 of every k-point, as
    w_jk sum_k' (V_x with occupied set k', q = k - k') psi_jk."""
    s = synth.make_system(synth.cubic_cell(8.0), (24, 24, 24))
    nq = (2, 2, 2)
    kpts = synth.kmesh_points(s.a, nq)
    sets = [synth.random_orbitals(s.a, s.miller, 17, 50 + k) for k in range(8)]
    w = [np.random.default_rng(60 + k).uniform(0.05, 0.2, 17) for k in range(8)]
    alpha = 10.0 / s.ecut
    k0 = exx.gb_constant(s.a, s.n, nq, alpha)
    rows = [0, 16]
    g = []
    for k in range(8):
        acc = 0.0
        for kp in range(8):
            q = np.asarray(kpts[k]) - np.asarray(kpts[kp])
            acc = acc + exx.fock_apply(s.a, s.n, s.miller, q, sets[kp], w[kp], sets[k][rows], k0=k0)
        g.append(w[k][rows][:, None] * acc)
    return s, nq, kpts, sets, w, alpha, rows, g


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("schedule", ["0", "1", "2"])
def test_kmesh_gradient_cross_blocks(kmesh17, prec, schedule, monkeypatch):
    """Schedules 1 and 2 transform each pair of the blocks k < k' once and
    apply it to both k-points' gradients (the block (k', k) has conj(v) in
    real space); schedule 0 runs every block separately.  Also: gradients
    requested for the even k-points only."""
    import torch
    F, _ = _mods()
    s, nq, kpts, sets, w, alpha, rows, g_ref = kmesh17
    monkeypatch.setenv("FOCK_SYM_SCHEDULE", schedule)
    cdt = torch.complex128 if prec == "c128" else torch.complex64
    tol = 1e-10 if prec == "c128" else 1e-5
    cell = _gb_cell(F, s, nq, alpha)
    C = torch.from_numpy(np.stack(sets)).to(cdt).cuda()
    W = torch.from_numpy(np.stack(w)).cuda()
    one = torch.ones((), dtype=torch.float64, device="cuda")
    print(f"[case] kmesh 17 orbitals {prec} schedule={schedule}", flush=True)
    G = torch.empty_like(C)
    F.fock_energy_kmesh_backward(cell, kpts, C, W, one, [G[k] for k in range(8)])
    Gh = host(G)
    H = torch.full_like(C, float("nan"))
    F.fock_energy_kmesh_backward(cell, kpts, C, W, one, [H[k] if k % 2 == 0 else None for k in range(8)])
    Hh = host(H)
    err = max(rel_fro(Gh[k][rows], g_ref[k]) for k in range(8))
    err_even = max(rel_fro(Hh[k][rows], g_ref[k]) for k in range(0, 8, 2))
    untouched = all(np.isnan(Hh[k]).all() for k in range(1, 8, 2))
    report(f"kmesh 17 {prec} schedule={schedule}", grad_rel=err, even_only_rel=err_even)
    assert err < tol and err_even < tol and untouched


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_kmesh_energy_and_grad_in_one_pass(reduced, kmesh17, prec):
    """fock_energy_kmesh_grad: the gradient sweep alone, E = 1/2 Re <C, dE/dconj C>.
    Against the oracle on the reduced instance; against the separate energy
    and backward calls on the 17-orbital mesh (gradient bit for bit)."""
    import torch
    F, _ = _mods()
    cdt = torch.complex128 if prec == "c128" else torch.complex64
    tol = 1e-10 if prec == "c128" else 1e-5
    one = torch.ones((), dtype=torch.float64, device="cuda")
    s, nq, kpts, sets, w, alpha, e_ref, g_ref = reduced
    cell = _gb_cell(F, s, nq, alpha)
    C = torch.from_numpy(np.stack(sets)).to(cdt).cuda()
    W = torch.from_numpy(np.stack(w)).cuda()
    print(f"[case] kmesh energy+grad one pass {prec}", flush=True)
    e, G = F.fock_energy_kmesh_grad(cell, kpts, C, W)
    err_e = abs(float(host(e)) - e_ref) / abs(e_ref)
    err_g = rel_fro(host(G), np.stack(g_ref))
    s, nq, kpts, sets, w, alpha, rows, _ = kmesh17
    cell = _gb_cell(F, s, nq, alpha)
    C = torch.from_numpy(np.stack(sets)).to(cdt).cuda()
    W = torch.from_numpy(np.stack(w)).cuda()
    e1, G1 = F.fock_energy_kmesh_grad(cell, kpts, C, W)
    e2 = float(host(F.fock_energy_kmesh(cell, kpts, C, W)))
    G2 = torch.empty_like(C)
    F.fock_energy_kmesh_backward(cell, kpts, C, W, one, [G2[k] for k in range(8)])
    err_e17 = abs(float(host(e1)) - e2) / abs(e2)
    same = np.array_equal(host(G1), host(G2))
    report(f"kmesh one pass {prec}", E_rel=err_e, grad_rel=err_g, E_vs_energy_pass=err_e17, grad_bitwise=same)
    assert err_e < tol and err_g < tol and err_e17 < tol and same
