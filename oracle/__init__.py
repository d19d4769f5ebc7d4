"""CPU FP64 oracle for the AZ RBF least-squares solver (Zhou & Huybrechs,
"Efficient least squares approximation and collocation methods using radial
basis functions").

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, dense reference that
follows the paper's definitions: it builds the collocation matrix entry by
entry, solves least-squares problems by a truncated SVD, and builds the
paper's periodic solver Z* = F B^+ P E from explicit DFT matrices.  Only the
test suite, the smoke check and the CPU-baseline leg of the benchmark may
import it.  The GPU library never calls it, and it shares no code with the GPU
library; the only shared module is ``workloads`` (problem data, no solver
arithmetic).

Modules
  rbf       Gaussian RBF, its second derivative and their periodizations
  grids     centre grid, oversampled grid, collocation subsets
  dense     dense system matrices for approximation and collocation
  lstsq     truncated-SVD least squares (the oracle's solver)
  periodic  the block-column circulant solver and Z* (section 3.1/3.2)
  az        the AZ algorithm (Algorithm 1) with dense matrices
  spectra   closed forms of the spectra by Poisson summation (Lemma 4.3)
  philox    Philox4x32-10 counter-based generator and Gaussian sketch
  evaluate  residuals and approximant evaluation on test sets
"""
