"""The C-ABI library loads and exports every function include/emsurf.h declares
(no compute calls: runs without a GPU)."""
import ctypes
import os

import numpy as np
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "emsurf.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"\b(emsurf_[A-Za-z_0-9]+)\s*\(", txt)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("emsurf_plan_create", "emsurf_apply_S", "emsurf_apply_T", "emsurf_apply_A", "emsurf_solve",
              "emsurf_plan_destroy", "emsurf_plan_bytes"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1911_04576_amd as E
    if not os.path.exists(E.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(E.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding wraps every declared function under the same name
    assert not [n for n in declared_functions() if not hasattr(E, n)]


def test_host_only_calls():
    import paper_1911_04576_amd as E
    if not os.path.exists(E.LIB_PATH):
        pytest.skip("library not built")
    assert E.emsurf_status_str(E.EMSURF_ERR_NOT_CONVERGED) == "not converged"
    # admission estimate: FP32 store of the 128 x 128, n_eq 192 plan is 256*256*192*192*8 bytes
    b32 = E.emsurf_plan_bytes(128, 128, 192, 16, 4, store=E.EMSURF_STORE_FP32)
    assert b32 > 256 * 256 * 192 * 192 * 8
    assert E.emsurf_plan_bytes(0, 4, 96, 4, 1) == 0
    assert E.emsurf_plan_bytes(4, 4, 96, 4, 65) == 0


def test_plan_bytes_refuses_fft_spans_beyond_32_bits():
    # a full-width apply's pass along y spans Lx Ly max_rhs n_eq values (32-bit
    # offsets in the FFT kernels): such plans are refused at creation
    import paper_1911_04576_amd as E
    if not os.path.exists(E.LIB_PATH):
        pytest.skip("library not built")
    assert E.emsurf_plan_bytes(128, 128, 512, 16, 64) == 0            # 256^2 x 64 x 512 = 2^31
    assert E.emsurf_plan_bytes(128, 128, 512, 16, 63) > 0
    assert E.emsurf_plan_bytes(512, 512, 96, 4, 32) == 0              # 1024^2 x 32 x 96 > 2^31
    assert E.emsurf_plan_bytes(512, 512, 96, 4, 21) > 0
    assert E.emsurf_plan_bytes(128, 128, 192, 16, 32) > 0             # the 128 x 128 serving shape


@pytest.mark.parametrize("Lx,Ly", [(1, 1), (2, 1), (3, 1), (1, 4), (3, 3), (4, 6), (12, 8), (6, 3), (256, 256)])
def test_spectrum_pairs_cover_every_frequency_once(Lx, Ly):
    import paper_1911_04576_amd as E
    if not os.path.exists(E.LIB_PATH):
        pytest.skip("library not built")
    pr = E.emsurf_spectrum_pairs(Lx, Ly)
    P = Lx * Ly
    self_paired = (2 if Lx % 2 == 0 else 1) * (2 if Ly % 2 == 0 else 1)
    assert pr.shape == ((P + self_paired) // 2, 2)
    k, kb = pr[:, 0].astype(np.int64), pr[:, 1].astype(np.int64)
    ky, kx = k // Lx, k % Lx
    assert np.array_equal(kb, ((Ly - ky) % Ly) * Lx + (Lx - kx) % Lx)
    assert np.all(k <= kb) and np.all(np.diff(k) > 0)
    seen = np.zeros(P, np.int64)
    np.add.at(seen, k, 1)
    np.add.at(seen, kb[kb != k], 1)
    assert np.all(seen == 1)
    assert int(np.sum(k == kb)) == self_paired


def test_reciprocal_plan_bytes_and_desc_checks():
    import paper_1911_04576_amd as E
    if not os.path.exists(E.LIB_PATH):
        pytest.skip("library not built")
    full = E.emsurf_plan_bytes(128, 128, 192, 16, 4, store=E.EMSURF_STORE_FP32)
    half = E.emsurf_plan_bytes(128, 128, 192, 16, 4, store=E.EMSURF_STORE_FP32, recip=1)
    store = 256 * 256 * 192 * 192 * 8
    assert abs((full - half) - (store // 2 - 2 * 192 * 192 * 8 - (256 * 256 // 2 + 2) * 8 - 192 * 24)) <= 0
    # recip must be 0 or 1
    assert E.emsurf_plan_bytes(8, 8, 96, 4, 1, recip=2) == 0
    # structured form: one [L | K] record (96 x 192) per pair instead of L and K per frequency
    lk_full = E.emsurf_plan_bytes(128, 128, 192, 16, 4, store=E.EMSURF_STORE_FP32, form=E.EMSURF_T_LK)
    lk_half = E.emsurf_plan_bytes(128, 128, 192, 16, 4, store=E.EMSURF_STORE_FP32, form=E.EMSURF_T_LK, recip=1)
    lk_store = 256 * 256 * 2 * 96 * 96 * 8
    assert lk_full - lk_half == lk_store - 32770 * 96 * 192 * 8 - 32770 * 8 - 192 * 24
    assert E.emsurf_plan_bytes(8, 8, 416, 4, 1, form=E.EMSURF_T_LK, recip=1) > 0
    assert E.emsurf_plan_bytes(8, 8, 418, 4, 1, form=E.EMSURF_T_LK, recip=1) == 0


def test_split_bf16_store_bytes_and_desc_checks():
    import paper_1911_04576_amd as E
    if not os.path.exists(E.LIB_PATH):
        pytest.skip("library not built")
    # hi and lo bfloat16 planes: 8 bytes per complex entry, as much as the FP32 store
    b32 = E.emsurf_plan_bytes(64, 64, 288, 32, 16, store=E.EMSURF_STORE_FP32)
    b16 = E.emsurf_plan_bytes(64, 64, 288, 32, 16, store=E.EMSURF_STORE_BF16)
    both = E.emsurf_plan_bytes(64, 64, 288, 32, 16, store=E.EMSURF_STORE_FP32 | E.EMSURF_STORE_BF16)
    store = 128 * 128 * 288 * 288 * 8
    assert b16 == b32 and both - b32 == store
    # dense, full (non-reciprocal) plans with n_eq a multiple of 32 in [32, 480] only
    assert E.emsurf_plan_bytes(8, 8, 96, 4, 1, store=E.EMSURF_STORE_BF16, recip=1) == 0
    assert E.emsurf_plan_bytes(8, 8, 96, 4, 1, store=E.EMSURF_STORE_BF16, form=E.EMSURF_T_LK) == 0
    assert E.emsurf_plan_bytes(8, 8, 48, 4, 1, store=E.EMSURF_STORE_BF16) == 0
    assert E.emsurf_plan_bytes(8, 8, 512, 4, 1, store=E.EMSURF_STORE_BF16) == 0
    assert E.emsurf_plan_bytes(8, 8, 480, 4, 1, store=E.EMSURF_STORE_BF16) > 0
    assert E.emsurf_plan_bytes(8, 8, 96, 4, 1, store=8) == 0
