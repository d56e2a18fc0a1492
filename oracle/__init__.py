"""FP64 CPU oracle for the T-product Sylvester solvers.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the C-ABI library
and its Python binding) may import, call or link anything in this package;
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It shares no code, table or helper with the HIP path.

Contents (each function cites the passage of the paper it follows):

* ``tproduct``  -- section 2: bcirc/unfold/fold, the T-product by explicit
  circulant sums (no FFT anywhere), transpose, inner product, tubes.
* ``krylov``    -- section 3 (tArnoldi, tFOM, tGMRES, Algorithm 3) and
  section 5 (Normalization, Tubal-QR, TBA, TBAS(m)).
* ``tbs``       -- section 4: t-Schur and t-Bartels-Stewart with
  t-back-substitution on tubes.
* ``kron``      -- brute-force Kronecker solve of the equivalent linear
  system on tiny inputs.

Every routine works in float64 (complex128 where the paper's objects are
complex) with numpy's own summation order.  Where a passage of the paper is
ambiguous or garbled, the docstring of the routine that depends on it states
the reading taken.
"""

from . import tproduct, krylov, tbs, kron  # noqa: F401
