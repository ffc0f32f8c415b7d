"""Plain FP64 CPU oracle for the Leja exponential integrator.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check of the entry
module and the benchmark's CPU-baseline leg may import this package.  The
product path (the HIP library and its Python binding) never imports, links or
calls anything here, and this package imports nothing from the product.

Everything is plain NumPy in float64, single-threaded, written for a reader
to check against the paper (Deka, Kissmann, Einkemmer, "Efficient numerical
methods for anisotropic diffusion of Galactic cosmic rays", ICRC 2023):

  operator.py     A = div(D grad .) + div(a .)              (Sec. 1 eq. 2, Sec. 2)
  phi.py          scalar phi_l functions                    (Sec. 2, phi recursion)
  leja.py         Leja points, divided differences, Newton  (Sec. 2, Leja method)
                  interpolation sweep, substepping
  integrators.py  exponential midpoint / two-stage rules    (Sec. 2 eq. 3-5)
  bounds.py       Gershgorin bound, power iteration         (Sec. 2)
  rng.py          counter-based splitmix64 generator
  features.py     coefficient-field statistics (learned bound inputs)
  mlp.py          the bound-predictor network, its gradient and Adam

Each function's docstring names the passage it follows; readings of silent
or ambiguous passages are marked "Reading:".
"""
from . import operator, phi, leja, integrators, bounds, rng, features, mlp  # noqa: F401
