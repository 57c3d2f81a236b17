"""fock_apply_noalloc, the allocation-free form of fock_apply, through the C
ABI: on consecutive calls (the second and third with smaller inputs, so the
fixed scratch array holds a previous call's contents) it must give
fock_apply's result, within the parity tolerances (FP64 1e-10, FP32 1e-5
relative), and the oracle's on the small cases."""
import numpy as np
import pytest

import synth
from oracle import exx
from tests.helpers import host, max_row_rel, rel_fro, report

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_noalloc_matches_fock_apply(prec):
    import torch
    from paper_1305_7313_amd import fock as F
    cdt = torch.complex128 if prec == "c128" else torch.complex64
    tol = 1e-10 if prec == "c128" else 1e-5
    s, occ, tgt = synth.config1()
    cell = F.Cell(s.a, s.n, s.miller)
    rng = np.random.default_rng(3)
    f8 = rng.uniform(0.4, 1.0, 8)
    cases = [  # (occupied rows, target rows or None (self), q)
        (slice(0, 8), slice(0, 8), (0.0, 0.0, 0.0)),
        (slice(0, 5), slice(2, 5), (0.11, -0.05, 0.07)),
        (slice(1, 7), None, (0.0, 0.0, 0.0)),
    ]
    for k, (so, st, q) in enumerate(cases):
        co = occ[so]
        ct = co if st is None else tgt[st]
        fo = f8[so]
        Co = torch.from_numpy(co).to(cdt).cuda()
        Ct = Co if st is None else torch.from_numpy(ct).to(cdt).cuda()
        fd = torch.from_numpy(fo).cuda()
        out = torch.full((ct.shape[0], s.npw), float("nan"), dtype=cdt, device="cuda")
        print(f"[case] noalloc {prec} call {k}: {co.shape[0]} occupied, {ct.shape[0]} targets, q={q}", flush=True)
        F.fock_apply_noalloc(cell, q, Co, fd, Ct, out)
        v = host(out).astype(np.complex128)
        ref = host(F.fock_apply(cell, q, Co, fd, Ct)).astype(np.complex128)
        e1, e2 = rel_fro(v, ref), max_row_rel(v, ref)
        vals = dict(vs_fock_apply=e1, vs_fock_apply_maxband=e2, identical=int(np.array_equal(v, ref)))
        if k > 0:
            orc = exx.fock_apply(s.a, s.n, s.miller, np.array(q), co, fo, ct)
            vals["vs_oracle"] = rel_fro(v, orc)
            assert vals["vs_oracle"] < tol
        report(f"noalloc {prec} call {k}", **vals)
        assert np.all(np.isfinite(v))
        assert e1 < tol and e2 < tol
