"""FP64 reference oracle for the truncated-decomposition approximate product.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import anything here.  The product library
never calls into this package, and this package imports nothing from the
product library: the two share no code.  The only common inputs are the seeded
matrices, which callers draw first and hand to both sides.

Every function is a plain, slow, float64 restatement of the paper:

* ``circulant``  -- cycle decomposition (appendix example, Alg. A.2), the
  circulant decomposition (Thm. 1.1) computed with Alg. 2.2, the magnitude
  ranking and eigenvalue lists of Alg. 2.3 (steps 2-4), the zeroth-order
  product (step 5) and the first-order term (step 6); plus the dense
  entrywise truncated matrix for the independent "definition" path.
* ``tsvd``       -- truncated SVD products of Sec. 2.2 (SVD based).
* ``sparse``     -- dominant-entry sparsification with a truncated residue,
  first-order form of eq. (2.4).
* ``product``    -- the combination rules of eq. (2.1)-(2.3).
* ``sfft``       -- Fourier-domain sparsification (Sec. 2.4, Alg. 2.4/2.5).
* ``estimators`` -- relative-error estimates of the first-order product
  (Sec. 2.5, Thm. 3.6, Cor. 3.7, Thm. 3.8, the circulant residual theorem) and
  the smallest truncation meeting a tolerance.

numpy's FFT, matmul, SVD and sort act as single library steps, never with any
blocking, fusion or reordering beyond the paper's own statement.

Parity status per function is recorded in each module header; every function
here is pinned by a ``-m "not gpu"`` test against a value that does not come
from the oracle itself (closed forms, worked examples, brute force).
"""
from . import circulant, tsvd, sparse, product, estimators, sfft  # noqa: F401
