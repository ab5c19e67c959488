"""FP64 CPU oracle for one real-time TDDFT time step on a real-space grid.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import or run anything in this package; the
product path (the HIP library and its Python binding) never does, and this
package imports nothing from the product.

The oracle is deliberately plain: NumPy/SciPy in float64, no blocking or
fusion beyond what the definitions state.  Each function names the passage of
arXiv:2410.09189 (Jakowski et al., "Real-time TDDFT ... RMG") it follows.
Where the paper is silent, the reading taken is stated in the docstring.

Modules
  grid         finite-difference Laplacian, grid coordinates, quadrature
  system       Gaussian local wells and separable projectors
  hamiltonian  density, Hartree, LDA exchange, H applied to orbitals, H[P]
  propagate    Magnus midpoint step (exact exponential and commutator series),
               delta kick, self-consistent time loop
  ground_state Kohn-Sham ground state used as the input active space
  spectrum     photoabsorption spectrum from the dipole history
  predictor    learned first guess: features, network forward/backward, Adam
               (imported by its tests as oracle.predictor)

Functions whose result has no independent pin say "parity unpinned" here and
in their docstring.  Currently: none.
"""

from . import grid, system, hamiltonian, propagate, ground_state, spectrum  # noqa: F401
from .hamiltonian import Model  # noqa: F401
from .propagate import run, kick, NoConvergence  # noqa: F401
