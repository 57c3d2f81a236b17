"""The benchmark's byte model (the roofline denominators), on the CPU.

* The live plane columns of the pair buffer cover the exact support of
  S - S (every difference of two sphere vectors, projected on the plane
  axes), on cubic and skewed cells, and fall back to every column when
  S - S wraps on the grid.
* The per-launch pair counts of the symmetric schedule reproduce the tile
  structure: 36 launches and 8256 transformed pairs for 128 orbitals, the
  figures the PMC traffic of config 2 was checked against.
* The counter summary tells the in-place inverse plane pass after P2 (the
  P3 class) from the same kernel taking orbitals to real space.
"""
import numpy as np

import bench
import synth


def _exact_support(miller):
    p = np.unique(miller[:, 1:3], axis=0)
    d = (p[:, None, :] - p[None, :, :]).reshape(-1, 2)
    return np.unique(d, axis=0)


def _live_table(miller, n):
    # the rule as bench.live_fraction states it, kept per column for the check
    n2, n3 = n[1], n[2]
    rows = {}
    for m2, m3 in zip(miller[:, 1].tolist(), miller[:, 2].tolist()):
        lo, hi = rows.get(m3, (m2, m2))
        rows[m3] = (min(lo, m2), max(hi, m2))
    col = [-1] * n3
    for a, (loa, hia) in rows.items():
        for b, (lob, hib) in rows.items():
            col[(a - b) % n3] = max(col[(a - b) % n3], hia - lob, hib - loa)
    return col


def test_live_columns_cover_the_pair_support():
    skew = np.array([[10.0, 0.0, 0.0], [1.0, 18.0, 0.0], [0.5, 0.3, 24.0]])
    for a, n in ((synth.cubic_cell(10.0), (24, 24, 24)), (skew, (24, 48, 64)), (synth.cubic_cell(20.0), (64, 64, 64))):
        s = synth.make_system(a, n)
        col = _live_table(s.miller, s.n)
        sup = _exact_support(s.miller)
        for d2, d3 in sup:
            i2, h = d2 % n[1], col[d3 % n[2]]
            assert i2 <= h or i2 >= n[1] - h, (n, d2, d3, h)
        lf = bench.live_fraction(s.miller, s.n)
        assert len(sup) <= lf * n[1] * n[2] + 1e-9
        assert 0.5 < lf < 0.8


def test_live_fraction_is_one_when_the_support_wraps():
    s = synth.make_system(synth.cubic_cell(20.0), (64, 64, 64))
    assert bench.live_fraction(s.miller, (48, 48, 48)) == 1.0


def test_step_bytes_tile_structure():
    acc = bench.step_bytes(128, 1, 1, True, sched=2)
    b, launches = acc["p2_pencil_kernel"]
    assert launches == 36
    assert b == 2 * (28 * 256 + 8 * 136)  # pairs read and written, N*b units
    lf = 0.75
    b2, _ = bench.step_bytes(128, 1, 1, True, sched=2, lf=lf)["p2_pencil_kernel"]
    assert abs(b2 - (1 + lf) * (28 * 256 + 8 * 136)) < 1e-9
    # schedule 1: the in-place inverse masks the dead columns, so P2 writes
    # only the live ones
    b3, _ = bench.step_bytes(128, 1, 1, True, sched=1, lf=lf)["p2_pencil_kernel"]
    assert abs(b3 - 2 * lf * (28 * 256 + 8 * 136)) < 1e-9


def test_roofline_picks_the_dominant_class_and_its_bound(monkeypatch):
    """The roofline record: the class with the most time is reported; it is
    measured against the vector-ALU peak when its algorithmic intensity is
    above the ridge point (78.6 TFLOP/s / 8 TB/s), else against HBM; every
    pair-pass class is listed against the plain-copy rate."""
    monkeypatch.setattr(bench, "copy_gbs", lambda: 5000.0)
    monkeypatch.setattr(bench, "pmc_traffic", lambda workload, kernel_class: None)
    # ms over the run and launches per class; bytes and flops per step
    tr = {"p1_pair_plane_fwd": [300.0, 1000], "p2_pencil_kernel": [290.0, 1000], "p3_second": [230.0, 1000]}
    acc = {"p1_pair_plane_fwd": [7.0e11, 1000], "p2_pencil_kernel": [1.4e12, 1000], "p3_second": [1.1e12, 1000]}
    flops = {"p1_pair_plane_fwd": 7.0e12, "p2_pencil_kernel": 6.5e12, "p3_second": 1.6e12}
    rec = bench.roofline(tr, acc, 1, "c4_fp32_batched", fp64=False, flops=flops)
    assert rec["kernel"] == "p1_pair_plane_fwd" and rec["bound"] == "alu" and rec["unit"] == "TFLOP/s"
    assert abs(rec["achieved"] - 7.0e12 / 0.3 / 1e12) < 0.01
    assert abs(rec["frac"] - rec["achieved"] / bench.VALU_PEAK_TFLOPS) < 1e-3
    assert abs(rec["hbm_gbs"] - 7.0e11 / 0.3 / 1e9) < 0.1
    assert set(rec["classes"]) == set(tr) and abs(rec["classes"]["p2_pencil_kernel"]["vs_copy"] - 1.4e12 / 0.29 / 1e9 / 5000.0) < 1e-3
    # P1 faster than P2: P2 dominates, and its intensity (4.6 flop/B) lies below the ridge
    tr["p1_pair_plane_fwd"] = [280.0, 1000]
    rec = bench.roofline(tr, acc, 1, "c4_fp32_batched", fp64=False, flops=flops)
    assert rec["kernel"] == "p2_pencil_kernel" and rec["bound"] == "hbm" and rec["unit"] == "GB/s"
    assert abs(rec["frac"] - 1.4e12 / 0.29 / 1e9 / bench.HBM_PEAK_GBS) < 1e-3


def test_traffic_summary_splits_the_inverse_plane_pass_by_role(tmp_path):
    """The in-place inverse plane pass after P2 on a queue is the P3 class;
    after the inverse pencil pass it is the orbital transform.  Two queues
    interleave as graph branches do; the copy probe sets the scales."""
    from paper_1305_7313_amd import profsum
    pl = "void fockx::plane_kernel<float, 96, 96, 768, true, {m}, 1>(fockx::PlaneArgs)"
    pe = "void fockx::pencil_kernel<float, 96, 64, 512, false, {m}, 1>(fockx::PencilArgs)"
    seq = [(1, pe.format(m=3), 10), (1, pl.format(m=3), 20),          # orbitals, queue 1
           (2, pe.format(m=3), 10), (1, pl.format(m=0), 30),
           (2, pl.format(m=3), 20), (1, pe.format(m=0), 40),          # orbitals, queue 2
           (2, pl.format(m=0), 30), (1, pl.format(m=3), 50),          # P3 on queue 1
           (2, pe.format(m=0), 40), (2, pl.format(m=3), 70),          # P3 on queue 2
           (1, "__amd_rocclr_copyBuffer", 100)]
    cols = ["Dispatch_Id", "Queue_Id", "Kernel_Name", "Counter_Value"]
    path = tmp_path / "c.csv"
    with open(path, "w") as fh:
        fh.write(",".join(cols) + "\n")
        for d, (q, name, v) in enumerate(seq):
            fh.write(f'{d + 1},{q},"{name}",{v}\n')
    out = tmp_path / "t.json"
    profsum.traffic(str(path), str(path), "w", str(out), "cmd", "sha")
    import json
    rec = json.load(open(out))
    k = rec["kernels"]
    assert k["plane_inv"]["dispatches"] == 2 and k["plane_inv"]["fetch_kib"] == 20
    assert k["p3_plane_inv_mac"]["dispatches"] == 2 and k["p3_plane_inv_mac"]["fetch_kib"] == 60
    assert k["p2_pencil_kernel"]["dispatches"] == 2 and k["a1_pencil_inv"]["dispatches"] == 2
    assert rec["fetch_scale"] == 1.0 and rec["copy_probe"]["fetch_kib"] == 100
