"""Full-size workloads, in the launch configuration the benchmark times.

The oracle is run in parallel worker processes on the host: on every target
of config 2, on sampled targets of the larger workloads (each against every
occupied orbital, on every k-point of a mesh), and on energy sub-blocks; the
FP32 path is also compared with the FP64 path on every element.  Errors are
printed for every result.
"""
import numpy as np
import pytest

import synth
from oracle import exx
from tests import oracle_pool
from tests.helpers import host, max_row_rel, rel_fro, report

pytestmark = pytest.mark.gpu


def _F():
    from paper_1305_7313_amd import fock
    return fock


def test_config2_fp64_all_targets():
    import torch
    F = _F()
    s, c = synth.config2()
    cell = F.Cell(s.a, s.n, s.miller)
    C = torch.from_numpy(c).cuda()
    f = torch.ones(128, dtype=torch.float64, device="cuda")
    print("[case] config2 apply 128x128 FP64", flush=True)
    v = host(F.fock_apply(cell, (0, 0, 0), C, f, C))
    # every target against every occupied orbital (16384 pairs on the host)
    rows = list(range(128))
    ref = oracle_pool.oracle_apply("c2", rows, 128, 8)
    err, errb = rel_fro(v[rows], ref), max_row_rel(v[rows], ref)
    sub = C[:32].contiguous()
    e = float(host(F.fock_energy(cell, (0, 0, 0), sub, f[:32].contiguous(), sub, f[:32].contiguous())))
    e_ref = oracle_pool.oracle_energy("c2", 32, 32, 4)
    report("config2 FP64", apply_rel=err, apply_maxband=errb, E32x32_rel=abs(e - e_ref) / abs(e_ref))
    assert err < 1e-10 and errb < 1e-10 and abs(e - e_ref) < 1e-10 * abs(e_ref)


def test_config3_fp32_vs_fp64_and_oracle():
    import torch
    F = _F()
    s, c = synth.config3()
    cell = F.Cell(s.a, s.n, s.miller)
    f = torch.ones(512, dtype=torch.float64, device="cuda")
    C64 = torch.from_numpy(c).cuda()
    C32 = C64.to(torch.complex64)
    print("[case] config3 apply 512x512 FP32 and FP64", flush=True)
    v32 = host(F.fock_apply(cell, (0, 0, 0), C32, f, C32)).astype(np.complex128)
    print("[case] config3 FP32 apply done", flush=True)
    v64 = host(F.fock_apply(cell, (0, 0, 0), C64, f, C64))
    print("[case] config3 FP64 apply done", flush=True)
    e32 = float(host(F.fock_energy(cell, (0, 0, 0), C32, f, C32, f)))
    e64 = float(host(F.fock_energy(cell, (0, 0, 0), C64, f, C64, f)))
    rows = [0, 311]
    ref = oracle_pool.oracle_apply("c3", rows, 512, 32)
    errs = dict(fp32_vs_fp64_apply=rel_fro(v32, v64), fp32_vs_fp64_maxband=max_row_rel(v32, v64),
                fp32_vs_fp64_E=abs(e32 - e64) / abs(e64),
                fp64_vs_oracle_rows=rel_fro(v64[rows], ref), fp32_vs_oracle_rows=rel_fro(v32[rows], ref))
    sub32 = C32[:32].contiguous()
    sub64 = C64[:32].contiguous()
    f32 = f[:32].contiguous()
    e_ref = oracle_pool.oracle_energy("c3", 32, 32, 2)
    es32 = float(host(F.fock_energy(cell, (0, 0, 0), sub32, f32, sub32, f32)))
    es64 = float(host(F.fock_energy(cell, (0, 0, 0), sub64, f32, sub64, f32)))
    errs.update(E32x32_fp64_rel=abs(es64 - e_ref) / abs(e_ref), E32x32_fp32_rel=abs(es32 - e_ref) / abs(e_ref))
    report("config3", E_fp32=e32, E_fp64=e64, **errs)
    assert errs["fp64_vs_oracle_rows"] < 1e-10 and errs["E32x32_fp64_rel"] < 1e-10
    for k in ("fp32_vs_fp64_apply", "fp32_vs_fp64_maxband", "fp32_vs_fp64_E", "fp32_vs_oracle_rows",
              "E32x32_fp32_rel"):
        assert errs[k] < 1e-5, (k, errs[k])


@pytest.mark.parametrize("sched", ["0", "1"])
def test_config3_two_blocks_q(sched, monkeypatch):
    """96x96x128 planes, occupied orbitals 0-47 applied to targets 100-115 at
    q != 0 (no pair symmetry): every target row against the oracle, FP64 and
    FP32, under both apply schedules (fused, and in-place inverse + streaming
    multiply-accumulate)."""
    import torch
    F = _F()
    monkeypatch.setenv("FOCK_APPLY_SCHEDULE", sched)
    s, c = synth.config3()
    cell = F.Cell(s.a, s.n, s.miller)
    q = oracle_pool.C3Q_SHIFT
    f = torch.ones(48, dtype=torch.float64, device="cuda")
    C64 = torch.from_numpy(c).cuda()
    occ64, tgt64 = C64[:48].contiguous(), C64[100:116].contiguous()
    print(f"[case] config3 two blocks at q != 0, schedule {sched}", flush=True)
    v64 = host(F.fock_apply(cell, q, occ64, f, tgt64))
    v32 = host(F.fock_apply(cell, q, occ64.to(torch.complex64), f, tgt64.to(torch.complex64))).astype(np.complex128)
    ref = oracle_pool.oracle_apply("c3q", list(range(100, 116)), 48, 6, kt=0, ko=1)
    errs = dict(fp64_rel=rel_fro(v64, ref), fp64_maxband=max_row_rel(v64, ref),
                fp32_rel=rel_fro(v32, ref), fp32_maxband=max_row_rel(v32, ref))
    report(f"config3 two blocks q schedule {sched}", **errs)
    assert errs["fp64_rel"] < 1e-10 and errs["fp64_maxband"] < 1e-10
    assert errs["fp32_rel"] < 1e-5 and errs["fp32_maxband"] < 1e-5


@pytest.mark.timeout(900)
def test_config5_full_autograd():
    """72^3, 2x2x2 mesh, 256 orbitals per k: FP32 forward/backward through
    autograd; the gradient element by element against the oracle on rows
    {0, 255} of the k-points 0 and 7, against the FP64 GPU gradient on every
    element, and against central differences of the FP64 energy along three
    random directions."""
    import torch
    F = _F()
    from paper_1305_7313_amd import autograd as A
    s, kpts, orbs = synth.config5()
    nq = (2, 2, 2)
    alpha = 10.0 / s.ecut
    cell = F.Cell(s.a, s.n, s.miller, g0=F.FOCK_G0_GB, gb_alpha=alpha, nq=nq)
    C64 = torch.from_numpy(np.stack(orbs)).cuda()
    W = torch.full((8, 256), 1.0 / 8, dtype=torch.float64, device="cuda")
    C32 = C64.to(torch.complex64).requires_grad_(True)
    print("[case] config5 FP32 forward + backward", flush=True)
    E32 = A.exchange_energy_kmesh(C32, W, cell, kpts)
    E32.backward()
    # PyTorch's gradient of a real loss is 2 dE/dconj(C)
    g32 = C32.grad.detach().to(torch.complex128)
    wg32 = host(g32) / 2.0
    print("[case] config5 FP64 energy and gradient", flush=True)
    ws64 = F.workspace_kmesh(cell, F.FOCK_C128, 8, 256, C64.device)
    e64 = float(host(F.fock_energy_kmesh(cell, kpts, C64, W, ws=ws64)))
    e64g, g64 = F.fock_energy_kmesh_grad(cell, kpts, C64, W, ws=ws64)
    wg64 = host(g64)
    e32 = float(host(E32))
    errs = dict(E_fp32_vs_fp64=abs(e32 - e64) / abs(e64),
                E_from_grad_vs_energy_fp64=abs(float(host(e64g)) - e64) / abs(e64),
                grad_fp32_vs_fp64=rel_fro(wg32.reshape(-1, s.npw), wg64.reshape(-1, s.npw)),
                grad_fp32_vs_fp64_maxband=max_row_rel(wg32.reshape(-1, s.npw), wg64.reshape(-1, s.npw)))
    # oracle: dE/dconj(c_jk) = w sum_k' (V_x psi_jk), occupied set k', q = k - k'
    k0 = exx.gb_constant(s.a, s.n, nq, alpha)
    rows = [0, 255]
    for kt in (0, 7):
        ref = oracle_pool.oracle_kmesh_grad_rows("c5", kt, rows, 256, 64, 8, 1.0 / 8, k0)
        errs[f"grad_k{kt}_fp32_vs_oracle"] = rel_fro(wg32[kt][rows], ref)
        errs[f"grad_k{kt}_fp32_vs_oracle_maxband"] = max_row_rel(wg32[kt][rows], ref)
        errs[f"grad_k{kt}_fp64_vs_oracle"] = rel_fro(wg64[kt][rows], ref)
    # central differences in FP64 along random unit directions
    h = 1e-4
    fd_worst = 0.0
    for seed in (1, 2, 3):
        g = torch.Generator(device="cpu").manual_seed(seed)
        d = torch.complex(torch.randn(C64.shape, generator=g, dtype=torch.float64),
                          torch.randn(C64.shape, generator=g, dtype=torch.float64)).cuda()
        d /= torch.linalg.vector_norm(d)
        print(f"[case] config5 FD direction {seed}", flush=True)
        ep = float(host(F.fock_energy_kmesh(cell, kpts, C64 + h * d, W, ws=ws64)))
        em = float(host(F.fock_energy_kmesh(cell, kpts, C64 - h * d, W, ws=ws64)))
        fd = (ep - em) / (2 * h)
        an = float(torch.sum(torch.conj(g32) * d).real)
        errs[f"fd_dir{seed}_rel"] = abs(fd - an) / abs(an)
        fd_worst = max(fd_worst, errs[f"fd_dir{seed}_rel"])
    # oracle: the (k=1 targets, k=0 occupied) block energy on a 32 x 32 sub-block, FP64 GPU vs oracle
    q = kpts[1] - kpts[0]
    cq = F.Cell(s.a, s.n, s.miller)
    wsub = torch.full((32,), 1.0 / 8, dtype=torch.float64, device="cuda")
    eb = float(host(F.fock_energy(cq, q, C64[0, :32].contiguous(), wsub, C64[1, :32].contiguous(), wsub)))
    eb_ref = oracle_pool.oracle_energy("c5", 32, 32, 2, kt=1, ko=0, weight=1.0 / 8)
    errs["block_E_fp64_vs_oracle"] = abs(eb - eb_ref) / abs(eb_ref)
    report("config5", E_fp32=e32, E_fp64=e64, **errs)
    assert errs["E_fp32_vs_fp64"] < 1e-5 and errs["E_from_grad_vs_energy_fp64"] < 1e-10
    assert errs["grad_fp32_vs_fp64"] < 1e-5 and errs["grad_fp32_vs_fp64_maxband"] < 1e-5
    for kt in (0, 7):
        assert errs[f"grad_k{kt}_fp32_vs_oracle"] < 1e-5 and errs[f"grad_k{kt}_fp32_vs_oracle_maxband"] < 1e-5
        assert errs[f"grad_k{kt}_fp64_vs_oracle"] < 1e-10
    # FP32 gradient against an FP64 difference quotient: the FP32 error bound
    # plus the O(h^2) truncation of the central difference
    assert fd_worst < 1e-4
    assert errs["block_E_fp64_vs_oracle"] < 1e-10
