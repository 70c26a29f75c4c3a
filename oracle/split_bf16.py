"""Oracle: the split-bfloat16 block product (reduced-precision definition).

TEST INFRASTRUCTURE ONLY, like the rest of this package.

The paper computes its Fourier-domain block products (Sec. IV-B) in full
precision.  The reduced-precision applies EMSURF_BF16X3 and EMSURF_BF16 keep
the FFTs in FP32 and form each product from bfloat16 halves.  The definition
follows the split-precision GEMM of Henry, Tang and Heinecke (ARITH 2019):

* an FP32 value a is split as a_hi = bf16(a), a_lo = bf16(a - a_hi), where
  bf16(.) keeps 8 significant bits and rounds to nearest, ties to even
  (a - a_hi is exact in FP32);
* the three-product form takes a b ~ a_hi b_hi + a_hi b_lo + a_lo b_hi
  (the dropped a_lo b_lo is below 2^-16 |a b|); the one-product form takes
  a_hi b_hi;
* a complex product runs on its real embedding, Re(a x) = ar xr - ai xi and
  Im(a x) = ar xi + ai xr, with every real product split as above.

Here the split parts are combined in FP64, where every product of two
8-bit significands is exact; the GPU accumulates in FP32, so the two differ
by FP32 summation rounding only.

Parity: pinned in tests/test_oracle_split_bf16.py by a library bfloat16
conversion, explicit ties, exact reconstruction of 16-bit significands,
exactness on bfloat16-representable inputs, and the error bound of the
definition on random data.
"""
from __future__ import annotations

import numpy as np


def round_bf16(a: np.ndarray) -> np.ndarray:
    """Round real values to 8 significant bits, ties to even (bfloat16 in its
    normal range), returned as float64.  Zero stays zero."""
    a = np.asarray(a, dtype=np.float64)
    m, e = np.frexp(a)                  # a = m 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.rint(m * 256.0) / 256.0, e)   # np.rint: nearest, ties to even


def split(a: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """(a_hi, a_lo) of the FP32 rounding of a real array."""
    a32 = np.asarray(a, dtype=np.float32).astype(np.float64)
    hi = round_bf16(a32)
    lo = round_bf16(a32 - hi)
    return hi, lo


def split_product(A: np.ndarray, X: np.ndarray, terms: int = 3) -> np.ndarray:
    """A X for complex A [n][m] and X [m][r] with split-bfloat16 real products.

    terms = 3: a_hi b_hi + a_hi b_lo + a_lo b_hi; terms = 1: a_hi b_hi."""
    if terms not in (1, 3):
        raise ValueError("terms must be 1 or 3")
    arh, arl = split(A.real)
    aih, ail = split(A.imag)
    xrh, xrl = split(X.real)
    xih, xil = split(X.imag)

    def prod(ah, al, bh, bl):
        out = ah @ bh
        if terms == 3:
            out = out + ah @ bl + al @ bh
        return out

    re = prod(arh, arl, xrh, xrl) - prod(aih, ail, xih, xil)
    im = prod(arh, arl, xih, xil) + prod(aih, ail, xrh, xrl)
    return re + 1j * im
