"""FP64 CPU oracle for the Gaussian-Polynomial Approximation (GPA) of the
bilateral filter (Chaudhury & Dabhade, "Fast and Provably Accurate
Bilateral Filtering", arXiv 1603.08109).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package's smoke check
and the benchmark's CPU-baseline leg may import this package.  The HIP
library never calls it, and it shares no code, table or constant with the
HIP path: both sides draw their inputs from ``synthimg`` and nothing else.

Contents (plain numpy / scipy / torch-CPU, float64 throughout):

* ``kernels``   - spatial kernels of eqs. (spatial_kernel1/2): box and
                  Gaussian taps, the support W = ceil(3 sigma_s) and the
                  normalised centre weight w(0).
* ``bf``        - eq. (BF) evaluated directly, O(W^2) per pixel.
* ``gpa``       - eq. (GPA) evaluated pair by pair with the
                  Gaussian-polynomial phi_N of eq. (GaussPolynomial), and
                  Algorithm 2 of Sec. 3 step by step.
* ``order``     - the kernel-error bound of Prop. (upperBound), the
                  Chernoff order of Prop. (LambW), Algorithm 1, Cor. (eps),
                  and eq. (Nvsdelta).
* ``grad``      - reference gradients of the GPA output (FP64 autograd
                  through a plain GPA, and central finite differences).

Pins (tests under ``tests/`` marked "not gpu") tie every function to values
the paper prints or to mathematics that fixes the result independently.
"""
from . import kernels, bf, gpa, order  # noqa: F401
