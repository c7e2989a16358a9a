"""FP64 CPU oracle for Parareal on the 2.5D kinematic dynamo.

TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously correct NumPy (float64 /
complex128) code that states what the GPU path computes, following
Clarke, Davies, Ruprecht & Tobias, "Parallel-in-time integration of kinematic
dynamos" (arXiv:1902.00387).  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import it; the product library never does,
and the two share no code.

Modules
  spectral  grid, wavenumbers, 2/3 box, flows, explicit operator curl(u x b)
  stepper   IMEX SBDF1/SBDF2 slice propagators, Fourier restriction/prolongation
  parareal  Parareal iteration, defect, growth rate, speed-up model
  network   FP64 reference of the learned coarse-propagator correction

Parity status of each function is stated in its docstring; every function is
pinned by a CPU test in ``tests/test_oracle_*.py`` except where the docstring
says "parity unpinned".
"""
from . import spectral, stepper, parareal, network  # noqa: F401
