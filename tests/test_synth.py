"""The seeded generator: determinism, orthonormality, sphere sizes."""
import numpy as np

import synth


def test_config_sizes():
    assert synth.config1()[0].npw == 799
    assert synth.make_system(synth.cubic_cell(20.0), (64,) * 3).npw == 16375
    assert synth.make_system(synth.ortho_cell(22.0, 22.0, 30.0), (96, 96, 128)).npw == 72115
    assert synth.make_system(synth.cubic_cell(24.0), (72,) * 3).npw == 23583
    grids, nbs = synth.config4_layout()
    assert len(grids) == 16 and set(grids) <= {48, 64, 72, 96}
    assert all(32 <= b <= 256 for b in nbs)


def test_orthonormal_and_deterministic():
    s, occ, tgt = synth.config1()
    assert np.abs(np.conj(occ) @ occ.T - np.eye(8)).max() < 1e-13
    assert np.abs(np.conj(tgt) @ tgt.T - np.eye(8)).max() < 1e-13
    s2, occ2, _ = synth.config1()
    assert np.array_equal(occ, occ2)


def test_sphere_is_alias_free():
    for n in [(12, 12, 12), (24, 24, 24), (16, 24, 32), (96, 96, 128)]:
        s = synth.make_system(np.diag([n[0] / 3.2, n[1] / 3.0, n[2] / 2.9]), n)
        for ax in range(3):
            assert np.abs(s.miller[:, ax]).max() <= (n[ax] - 1) / 4


def test_gamma_orbitals_are_real_and_orthonormal():
    from oracle import exx
    s = synth.make_system(synth.cubic_cell(8.0), (24, 24, 24))
    c = synth.gamma_orbitals(s.a, s.miller, 6, 4)
    assert np.abs(np.conj(c) @ c.T - np.eye(6)).max() < 1e-13
    psi = exx.to_grid(c, s.miller, s.n)
    assert np.abs(psi.imag).max() < 1e-13 * np.abs(psi.real).max()
