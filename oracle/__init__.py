"""FP64 CPU oracle for the regularized spectral-Ewald polarization solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the test suite, the smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code with the HIP
library; the only common dependency is the seeded input generator, which
holds none of the method's arithmetic.

Modules
-------
ewald     the potential tensor M and its gradient by the plain Fourier-sum
          definition and by an Ewald split (two independent evaluations)
se        "mode B": the discretized spectral-Ewald operator written out by
          brute force (explicit window sums and explicit DFT matrices)
saddle    the conductor saddle-point system, its dense solve, dipoles,
          energies, bead forces, body forces and torques
freespace the same quantities without periodicity (closed-form pins)
"""
from . import ewald, se, saddle, freespace  # noqa: F401
