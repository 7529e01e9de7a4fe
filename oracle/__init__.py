"""CPU oracle for the parallel inverse fast multipole method (IFMM).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link anything under this directory: only the tests, the package's smoke entry
and the CPU-baseline leg of the benchmark use it.  It shares no code with the
HIP implementation; the only common dependency is the seeded geometry module
``synth``, which holds no IFMM arithmetic.

The oracle is plain FP64 numpy/scipy, written for a reader holding the paper
(Takahashi, Chen, Darve, "Parallelization of the inverse fast multipole method
with an application to boundary element method"):

* ``tree``  -- uniform octree, neighbour / interaction lists (Sec. 2.1 and the
  normalised distance equation of Sec. 3) and the greedy colouring (Alg. 3).
* ``cheb``  -- black-box (Chebyshev) FMM operators for the 3-D Laplace kernel,
  the "different FMM" the paper allows in Sec. 4.2.
* ``ifmm``  -- the extended sparse system (eq. ext), the colour-by-colour
  factorisation (Alg. 1 with the colour loops of Sec. 3.2/3.3) and the solve
  (Alg. 2), plus the dense matrix that the extended system represents.

Readings of the paper that it had to make are listed in each module header.
"""
