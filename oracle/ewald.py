"""Ewald lattice sums used by the closed-form pins.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import numpy as np
from scipy.special import erfc


def madelung_simple_cubic(eta: float = 0.9, nmax: int = 6) -> float:
    """Madelung constant alpha_M of a simple-cubic lattice of unit spacing.

    alpha_M is defined by the energy per point charge of the lattice with a
    neutralising background, E = -alpha_M / (2 L).  Ewald split with width
    eta: E = 1/2 [ sum_{R!=0} erfc(eta R)/R + (4 pi / Omega) sum_{G!=0}
    e^{-G^2/(4 eta^2)} / G^2 - 2 eta / sqrt(pi) - pi / (Omega eta^2) ].
    The result must not depend on eta (checked by the pins).
    """
    r = np.arange(-nmax, nmax + 1)
    x, y, z = np.meshgrid(r, r, r, indexing="ij")
    v = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1).astype(np.float64)
    v = v[np.any(v != 0, axis=1)]
    rl = np.linalg.norm(v, axis=1)
    real = np.sum(erfc(eta * rl) / rl)
    g = 2.0 * np.pi * v
    g2 = np.einsum("ij,ij->i", g, g)
    recip = 4.0 * np.pi * np.sum(np.exp(-g2 / (4.0 * eta * eta)) / g2)
    e = 0.5 * (real + recip - 2.0 * eta / np.sqrt(np.pi) - np.pi / (eta * eta))
    return -2.0 * e
