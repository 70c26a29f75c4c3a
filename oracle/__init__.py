"""FP64 CPU oracle for the coupled-macromodel solve  (I - S T) x = b.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import anything from this package; the GPU
library never does, and this package never touches the GPU library.

What it computes, each function citing the passage it follows:

* ``coupling``  -- the synthetic free-space coupling blocks T(d) between two
  boxes of the lattice (point-sampled Green's function between patch centres,
  source-area weighted), the dense block-Toeplitz matrix T of Sec. III-B /
  Sec. IV-A, and its product with a vector in two plain forms: dense, and a
  direct sum over lattice offsets.  No FFT anywhere.
* ``macromodel`` -- the block-diagonal macromodel apply of Sec. III-A
  (one dense block per element, shared by elements of a cell type) and the
  operator A = I - S T.
* ``krylov`` -- restarted GMRES with classical Gram-Schmidt applied twice and
  complex Givens rotations, plus a dense LU reference solve.
* ``split_bf16`` -- the split-bfloat16 definition of the reduced-precision
  block products (a = a_hi + a_lo, three or one real products per entry),
  combined exactly in FP64.

Every function is plain numpy in complex128.  The parity status of each is
listed in its docstring: the pins live in ``tests/test_oracle_*.py``.
"""
from . import coupling, macromodel, krylov  # noqa: F401
