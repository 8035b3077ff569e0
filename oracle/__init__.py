"""FP64 CPU oracle for the phase-field lattice Boltzmann method with wetting
folded into the chemical potential (arXiv:2312.00369).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, whole-array NumPy
restatement of the paper's equations, written to check the GPU library.  Only
the test-suite, the smoke check and the CPU-baseline leg of the benchmark may
import it.  The product path (the HIP library and its Python binding) never
imports, links or calls anything here, and nothing here imports the product.

Modules
  lattice      velocity sets, weights, sound speed, opposite table, source
               coefficients (Sec. 2.1.2 Eq. ci / 3ci and the weights that follow;
               Sec. 2.1.3 Eq. F_i)
  model        node classes, effective area, ghost fill, stencils, equilibria,
               forcing, chemical potential, one time step (Sec. 2.1, 2.2)
  diagnostics  mass, mass budget, steady residual, contact-angle estimator
"""
from . import lattice, model, diagnostics  # noqa: F401
from .model import Params, Oracle  # noqa: F401
