"""CPU FP64 oracle of the exact-exchange (Fock) operator.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import or run anything in this package; the
product path (the HIP library and its Python binding) never does, and this
package imports nothing from it.

It is a plain, slow, obviously correct statement of what the GPU path
computes (Varini et al., "Enhancement of DFT-calculations at Petascale",
section 4):

* ``exx``          -- the FFT route the method itself describes: orbitals to
                      real space, pair (overlap) density, forward transform,
                      Coulomb kernel, inverse transform, multiply back and
                      accumulate; the exchange energy; its gradient; the
                      Gygi-Baldereschi G=0 constant.
* ``definitions``  -- the same quantities from their plain definitions with no
                      FFT at all (direct G-space convolution, real-space
                      double sum), used only to pin ``exx`` on tiny inputs.
* ``ewald``        -- Ewald lattice sums (simple-cubic Madelung constant) used
                      by the closed-form pins.
* ``bands``        -- the band loops of the Car-Parrinello code (section 5):
                      charge density and the force of the local Hamiltonian.

Every function is FP64 NumPy/SciPy.  Pins live in ``tests/test_oracle_*.py``.
"""
from . import bands, exx, definitions, ewald  # noqa: F401
