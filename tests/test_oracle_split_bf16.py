"""Pins of the split-bfloat16 product model (oracle/split_bf16.py) against a
library bfloat16 conversion, explicit ties, exactness cases and the error
bound of the definition -- none of them a retyping of its code."""
import numpy as np
import pytest

from oracle import split_bf16 as SB

torch = pytest.importorskip("torch")


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def test_rounding_matches_library_bfloat16():
    # torch's CPU float32 -> bfloat16 conversion rounds to nearest, ties to even
    rng = _rng(1)
    a = (rng.standard_normal(20000) * 10.0 ** rng.uniform(-20, 20, 20000)).astype(np.float32)
    lib = torch.from_numpy(a).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(SB.round_bf16(a.astype(np.float64)), lib)


def test_rounding_ties_go_to_even():
    u = 2.0 ** -8                       # half an ulp of bfloat16 at 1
    cases = {1 + u: 1.0, 1 + 3 * u: 1 + 4 * u, -(1 + u): -1.0, 1 + 5 * u: 1 + 4 * u,
             255.0 + 0.5: 256.0, 254.0 + 0.5: 254.0 + 0.0, 0.0: 0.0}
    # 255.5 lies between 255 and 256: with 8 significant bits 255 and 256 are
    # neighbours (ulp 1 in [128, 256)), the tie goes to the even 256; 254.5 to 254
    for a, want in cases.items():
        assert SB.round_bf16(np.array([a]))[0] == want, a


def test_split_reconstructs_sixteen_bit_significands_exactly():
    rng = _rng(2)
    sig = rng.integers(2 ** 15, 2 ** 16, 5000)          # exactly 16 significant bits
    a = np.ldexp(sig.astype(np.float64) * np.where(rng.random(5000) < 0.5, -1, 1),
                 rng.integers(-40, 40, 5000) - 16)
    hi, lo = SB.split(a)
    assert np.array_equal(hi + lo, a)
    assert np.array_equal(SB.round_bf16(hi), hi) and np.array_equal(SB.round_bf16(lo), lo)


def test_split_error_bound():
    # |a - a_hi| <= 2^-8 |a| and |a - a_hi - a_lo| <= 2^-16 |a| for FP32 a
    rng = _rng(3)
    a = rng.standard_normal(50000).astype(np.float32).astype(np.float64)
    hi, lo = SB.split(a)
    assert np.all(np.abs(a - hi) <= 2.0 ** -8 * np.abs(a))
    assert np.all(np.abs(a - hi - lo) <= 2.0 ** -16 * np.abs(a))
    assert np.max(np.abs(a - hi - lo) / np.abs(a)) > 2.0 ** -18   # the bound is nearly reached


def test_product_exact_on_representable_inputs():
    # small integers have lo = 0: both forms equal the exact complex product,
    # which fixes the signs of the real embedding and the operand orientation
    rng = _rng(4)
    A = rng.integers(-50, 50, (7, 5)) + 1j * rng.integers(-50, 50, (7, 5))
    X = rng.integers(-50, 50, (5, 3)) + 1j * rng.integers(-50, 50, (5, 3))
    for terms in (1, 3):
        assert np.array_equal(SB.split_product(A, X, terms), A @ X)


def test_product_error_bounds_on_random_data():
    # per real product: three terms within 3 * 2^-16 |a||b| (+ FP32 rounding of
    # the inputs), one term within (2^-7 + 2^-16) |a||b|; summed, componentwise
    # against |Re A||Re X| + |Im A||Im X| (real part) and the cross terms (imaginary)
    rng = _rng(5)
    n = 96
    A = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))).astype(np.complex64).astype(np.complex128)
    X = (rng.standard_normal((n, 4)) + 1j * rng.standard_normal((n, 4))).astype(np.complex64).astype(np.complex128)
    exact = A @ X
    mre = np.abs(A.real) @ np.abs(X.real) + np.abs(A.imag) @ np.abs(X.imag)
    mim = np.abs(A.real) @ np.abs(X.imag) + np.abs(A.imag) @ np.abs(X.real)
    for terms, bound in ((3, 3 * 2.0 ** -16 + 2.0 ** -30), (1, 2.0 ** -7 + 2.0 ** -16)):
        y = SB.split_product(A, X, terms)
        assert np.all(np.abs(y.real - exact.real) <= bound * mre)
        assert np.all(np.abs(y.imag - exact.imag) <= bound * mim)
    # the three-term form is far closer than the one-term form
    e3 = np.linalg.norm(SB.split_product(A, X, 3) - exact) / np.linalg.norm(exact)
    e1 = np.linalg.norm(SB.split_product(A, X, 1) - exact) / np.linalg.norm(exact)
    assert e3 < 2e-5 and e1 > 100 * e3


def test_dropping_a_term_breaks_the_bound():
    # the three-term bound is tight enough to see a missing a_lo b_hi term
    rng = _rng(6)
    a = rng.standard_normal(20000).astype(np.float32).astype(np.float64)
    b = rng.standard_normal(20000).astype(np.float32).astype(np.float64)
    ah, al = SB.split(a)
    bh, bl = SB.split(b)
    partial = ah * bh + ah * bl
    assert np.any(np.abs(partial - a * b) > 3 * 2.0 ** -16 * np.abs(a * b))
    full = partial + al * bh
    assert np.all(np.abs(full - a * b) <= (3 * 2.0 ** -16 + 2.0 ** -30) * np.abs(a * b))
