"""FP64 CPU oracle for QTT contraction, orthogonalisation, rounding and inner products.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check of the package
entry file and the CPU-baseline leg of the benchmark may import this package.
The product path (the HIP library and its Python binding) never calls it and
shares no code with it.

Everything here is plain NumPy in float64 with LAPACK QR/SVD through
numpy.linalg, written from the paper's definitions:

  * contraction: Sec. 3.1, eqs. quant_sum and einsum -- local core
    contractions with the bond indices flattened as xi = (mu, nu), mu major;
  * exact addition: Sec. 3.1, the block-diagonal core structure;
  * orthogonalisation: the QR-based normalisation step of Sec. 3.2 (and the
    canonical form of Sec. 1), swept left to right;
  * rounding: a left-to-right QR sweep followed by a right-to-left truncated
    SVD sweep -- the TT-rounding algorithm of Oseledets (2011), which the
    paper cites for tensor trains; the paper's "decomposition(max_rank,
    cutoff)" options are read as a relative Frobenius tolerance and a rank cap;
  * inner product: the <C|C>-type contractions of Sec. 3.3;
  * decomposition ("zip-up") algorithm of Sec. 3.2: operands normalised to
    the left end, then a super-core of N exact product cores split off one
    truncated-SVD core at a time while the next product core is added;
  * variational fitting of Sec. 3.3 (eq. variational): one core at a time,
    the derivative of <C|Y> with every other core orthonormal, and the
    multi-core strategy with super-cores of two cores, decomposed again by a
    truncated SVD so that the ranks adapt;
  * the DMRG-like linear solver of Sec. 5 for symmetric positive definite
    operators: the energy <x, W x> - 2 <x, b> minimised over one core or a
    super-core of two cores at a time (local dense solves);
  * the AMEn linear solver of Sec. 5: one-core energy minimisation, a
    truncation of each solved core and its basis enriched by the projection
    of the residual b - W x onto the frames of a second train z that tracks
    the residual (Dolgov and Savostyanov's alternating minimal energy method);
  * sums of many trains (the block structure of Sec. 3.1, operators
    included) and the operator product 'ij,jk->ik';
  * general digit bases (factorised dimensions, Sec. 2): every function takes
    per-core physical sizes.

Pins (tests/test_oracle_*.py) tie each function to something other than
itself: dense reconstruction + numpy.einsum on tiny grids, the closed forms of
Sec. 4 (exp rank 1, cos/sin rank 2, degree-p polynomial rank p+1, the shift
matrices of Sec. 4.2), the discrete Poisson solution j (N + 1 - j) / 2,
Laplacian eigenvectors, dense solves, and invariants.
"""
from .tt import *  # noqa: F401,F403
from .tt import __all__  # noqa: F401
