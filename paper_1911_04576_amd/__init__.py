"""Python binding of the emsurf C ABI (include/emsurf.h): argument marshalling
only.  Every step of the coupled-macromodel path runs in the HIP kernels of
libemsurf.so; there is no Python or CPU fallback, and importing the binding
fails loudly when the library has not been built.

Device buffers are passed as torch tensors (their data_ptr()) or raw integer
addresses; host arrays as numpy arrays.  Streams are torch.cuda.Stream objects,
raw hipStream_t integers, or None for the null stream.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libemsurf.so")

EMSURF_OK = 0
EMSURF_ERR_ARG = 1
EMSURF_ERR_OOM = 2
EMSURF_ERR_DEVICE = 3
EMSURF_ERR_NOT_CONVERGED = 4
EMSURF_ERR_BUSY = 5
EMSURF_ERR_UNSUPPORTED = 6

EMSURF_FP64 = 0
EMSURF_FP32 = 1
EMSURF_FP32_IR = 2
EMSURF_BF16X3 = 3
EMSURF_BF16 = 4

EMSURF_STORE_FP64 = 1
EMSURF_STORE_FP32 = 2
EMSURF_STORE_BF16 = 4

EMSURF_T_DENSE = 0
EMSURF_T_LK = 1

EMSURF_BP_AUTO = -1
EMSURF_BP_GEMV = 0
EMSURF_BP_MFMA_T1 = 1
EMSURF_BP_MFMA_T2 = 2
EMSURF_BP_MFMA_T3 = 3
EMSURF_BP_MFMA_T4 = 4
EMSURF_BP_MFMA_T1_DEEP = 5
EMSURF_BP_MFMA_T2_DEEP = 6
EMSURF_BP_MFMA_T3_DEEP = 7
EMSURF_BP_MFMA_T4_DEEP = 8
EMSURF_BP_NVARIANTS = 9
BP_NAMES = ("gemv", "mfma_t1", "mfma_t2", "mfma_t3", "mfma_t4", "mfma_t1_deep", "mfma_t2_deep", "mfma_t3_deep",
            "mfma_t4_deep")

EMSURF_OP_T = 0
EMSURF_OP_S = 1
EMSURF_OP_A = 2

PHASES = ("fft_x_fwd", "fft_y_fwd", "block_product", "fft_y_inv", "fft_x_inv")


class EmsurfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"emsurf status {status}: {msg}")
        self.status = status


class emsurf_plan_desc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("n_eq", ctypes.c_int32),
                ("n_types", ctypes.c_int32), ("max_rhs", ctypes.c_int32), ("store", ctypes.c_uint32),
                ("form", ctypes.c_int32), ("recip", ctypes.c_int32), ("coef", ctypes.c_double * 8)]


class emsurf_geom(ctypes.Structure):
    _fields_ = [("n_patch", ctypes.c_int32), ("rho", ctypes.c_void_p), ("area", ctypes.c_void_p),
                ("tan", ctypes.c_void_p), ("pitch", ctypes.c_double), ("k", ctypes.c_double)]


class emsurf_solve_opts(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int), ("tol", ctypes.c_double), ("restart", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("use_x0", ctypes.c_int32), ("inner_tol", ctypes.c_double),
                ("max_outer", ctypes.c_int32)]


class emsurf_solve_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("outer_iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("rel_res_true", ctypes.c_double), ("ms", ctypes.c_double)]


class emsurf_server_desc(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_size_t), ("max_slots", ctypes.c_int32), ("store", ctypes.c_uint32),
                ("opts", emsurf_solve_opts)]


class emsurf_server_stats(ctypes.Structure):
    _fields_ = [("queued", ctypes.c_int32), ("active", ctypes.c_int32), ("resident_plans", ctypes.c_int32),
                ("bytes_used", ctypes.c_size_t), ("plans_built", ctypes.c_int64), ("evictions", ctypes.c_int64),
                ("admit_ms", ctypes.c_double), ("step_ms", ctypes.c_double)]


class emsurf_precond_stats(ctypes.Structure):
    _fields_ = [("n_tiles", ctypes.c_int32), ("nq_max", ctypes.c_int32), ("near_entries", ctypes.c_int64),
                ("bytes", ctypes.c_size_t), ("build_ms", ctypes.c_double)]


class emsurf_plan_stats(ctypes.Structure):
    _fields_ = [("Lx", ctypes.c_int32), ("Ly", ctypes.c_int32), ("n_freq", ctypes.c_int64),
                ("bytes_that64", ctypes.c_size_t), ("bytes_that32", ctypes.c_size_t),
                ("bytes_total", ctypes.c_size_t), ("n_stored", ctypes.c_int64),
                ("bytes_that16", ctypes.c_size_t)]


_P = ctypes.c_void_p
_SIGS = {
    "emsurf_plan_bytes": (ctypes.c_size_t, [ctypes.POINTER(emsurf_plan_desc)]),
    "emsurf_plan_create": (ctypes.c_int, [ctypes.POINTER(emsurf_plan_desc), _P, ctypes.c_int32, _P, _P, _P,
                                          ctypes.POINTER(_P)]),
    "emsurf_plan_create_green": (ctypes.c_int, [ctypes.POINTER(emsurf_plan_desc), ctypes.POINTER(emsurf_geom), _P,
                                                _P, _P, ctypes.POINTER(_P)]),
    "emsurf_plan_create_reciprocal": (ctypes.c_int, [ctypes.POINTER(emsurf_plan_desc), _P, ctypes.c_int32, _P, _P,
                                                     _P, _P, ctypes.POINTER(_P)]),
    "emsurf_spectrum_pairs": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, _P, ctypes.POINTER(ctypes.c_int64)]),
    "emsurf_fill_T_point_green": (ctypes.c_int, [ctypes.POINTER(emsurf_geom), ctypes.c_int32, ctypes.c_int32, _P, _P]),
    "emsurf_fill_LK_point_green": (ctypes.c_int, [ctypes.POINTER(emsurf_geom), ctypes.c_int32, ctypes.c_int32, _P, _P]),
    "emsurf_macromodels": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, _P, _P, _P, _P]),
    "emsurf_far_field": (ctypes.c_int, [ctypes.POINTER(emsurf_geom), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_int32, _P, _P, _P]),
    "emsurf_directivity": (ctypes.c_int, [ctypes.POINTER(emsurf_geom), ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, _P,
                                          ctypes.POINTER(ctypes.c_double), _P]),
    "emsurf_apply_T": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int32, _P, _P, _P]),
    "emsurf_apply_S": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int32, _P, _P, _P]),
    "emsurf_apply_A": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int32, _P, _P, _P]),
    "emsurf_apply_T_noalloc": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int32, _P, _P, _P]),
    "emsurf_apply_T_noalloc_limit": (ctypes.c_size_t, []),
    "emsurf_solve": (ctypes.c_int, [_P, ctypes.POINTER(emsurf_solve_opts), ctypes.c_int32, _P, _P,
                                    ctypes.POINTER(emsurf_solve_info), _P]),
    "emsurf_plan_query": (ctypes.c_int, [_P, ctypes.POINTER(emsurf_plan_stats)]),
    "emsurf_overlap_create": (ctypes.c_int, [_P, ctypes.POINTER(emsurf_geom), ctypes.c_int32, _P,
                                             ctypes.POINTER(_P)]),
    "emsurf_overlap_query": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                            ctypes.POINTER(ctypes.c_size_t)]),
    "emsurf_overlap_expand": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P]),
    "emsurf_overlap_reduce": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P]),
    "emsurf_apply_reduced": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P]),
    "emsurf_overlap_destroy": (None, [_P]),
    "emsurf_precond_create": (ctypes.c_int, [_P, ctypes.POINTER(emsurf_geom), ctypes.c_double, ctypes.c_int32,
                                             ctypes.c_int32, _P, _P, ctypes.POINTER(_P)]),
    "emsurf_precond_apply": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P]),
    "emsurf_precond_query": (ctypes.c_int, [_P, ctypes.POINTER(emsurf_precond_stats)]),
    "emsurf_precond_destroy": (None, [_P]),
    "emsurf_solve_precond": (ctypes.c_int, [_P, _P, ctypes.POINTER(emsurf_solve_opts), ctypes.c_int32, _P, _P,
                                            ctypes.POINTER(emsurf_solve_info), _P]),
    "emsurf_kernel_timing": (ctypes.c_int, [_P, ctypes.c_int32]),
    "emsurf_kernel_times": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]),
    "emsurf_plan_destroy": (None, [_P]),
    "emsurf_plan_autotune": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                            ctypes.POINTER(ctypes.c_int32), _P]),
    "emsurf_plan_set_variant": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32]),
    "emsurf_graph_create": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int, ctypes.c_int32, _P, _P, _P,
                                           ctypes.POINTER(_P)]),
    "emsurf_graph_launch": (ctypes.c_int, [_P, _P]),
    "emsurf_graph_destroy": (None, [_P]),
    "emsurf_session_bytes": (ctypes.c_size_t, [_P, ctypes.c_int32, ctypes.POINTER(emsurf_solve_opts)]),
    "emsurf_session_create": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(emsurf_solve_opts), _P,
                                             ctypes.POINTER(_P)]),
    "emsurf_session_submit": (ctypes.c_int, [_P, _P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32)]),
    "emsurf_session_step": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32)]),
    "emsurf_session_finished": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64),
                                               ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "emsurf_session_active": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32)]),
    "emsurf_session_collect": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.POINTER(emsurf_solve_info)]),
    "emsurf_session_destroy": (None, [_P]),
    "emsurf_server_create": (ctypes.c_int, [ctypes.POINTER(emsurf_server_desc), ctypes.POINTER(_P)]),
    "emsurf_server_submit": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.POINTER(emsurf_plan_desc),
                                            ctypes.POINTER(emsurf_geom), _P, _P, ctypes.c_int32, _P,
                                            ctypes.POINTER(ctypes.c_int64)]),
    "emsurf_server_step": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32)]),
    "emsurf_server_next_completed": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64),
                                                    ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)]),
    "emsurf_server_fetch": (ctypes.c_int, [_P, ctypes.c_int64, _P, ctypes.POINTER(emsurf_solve_info),
                                           ctypes.POINTER(ctypes.c_double)]),
    "emsurf_server_query": (ctypes.c_int, [_P, ctypes.POINTER(emsurf_server_stats)]),
    "emsurf_server_destroy": (None, [_P]),
    "emsurf_server_entry_bytes": (ctypes.c_size_t, [_P, ctypes.POINTER(emsurf_plan_desc)]),
    "emsurf_server_slot_bytes": (ctypes.c_size_t, [_P, ctypes.POINTER(emsurf_plan_desc)]),
    "emsurf_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "emsurf_last_error": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """Load libemsurf.so (raises if it has not been built: no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(python -m paper_1911_04576_amd._build)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(st: int):
    if st != EMSURF_OK:
        msg = lib().emsurf_last_error().decode()
        raise EmsurfError(st, msg)


def _dptr(t) -> int:
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return int(t.data_ptr())


def _stream(s) -> int:
    if s is None:
        return None
    if isinstance(s, int):
        return s
    return int(s.cuda_stream)


def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(ctypes.c_void_p)


class Geometry:
    """Host-side emsurf_geom that keeps its arrays alive."""

    def __init__(self, rho, area, tan, pitch: float, k: float):
        self._rho, prho = _host(rho, np.float64)
        self._area, parea = _host(area, np.float64)
        self._tan, ptan = _host(tan, np.float64)
        assert self._rho.shape[1:] == (3,) and self._tan.shape[1:] == (2, 3)
        self.c = emsurf_geom(self._rho.shape[0], prho, parea, ptan, float(pitch), float(k))

    @property
    def n_patch(self):
        return self._rho.shape[0]


class Plan:
    """An emsurf_plan handle (destroyed with the object or by .destroy())."""

    def __init__(self, handle: int, desc: emsurf_plan_desc):
        self.h = handle
        self.desc = desc

    def destroy(self):
        if self.h:
            lib().emsurf_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def stats(self) -> emsurf_plan_stats:
        return emsurf_plan_query(self)


def _desc(nx, ny, n_eq, n_types, max_rhs, store, form=EMSURF_T_DENSE, coef=None, recip=0):
    """coef: the four complex constants (a, b, c, e) of EMSURF_T_LK; recip: 1 for
    a reciprocal plan (one stored block per frequency pair)."""
    c8 = (ctypes.c_double * 8)()
    if coef is not None:
        for i, z in enumerate(coef):
            c8[2 * i], c8[2 * i + 1] = complex(z).real, complex(z).imag
    return emsurf_plan_desc(int(nx), int(ny), int(n_eq), int(n_types), int(max_rhs), int(store), int(form),
                            int(recip), c8)


def emsurf_plan_bytes(nx, ny, n_eq, n_types, max_rhs, store=EMSURF_STORE_FP64 | EMSURF_STORE_FP32,
                      form=EMSURF_T_DENSE, recip=0) -> int:
    d = _desc(nx, ny, n_eq, n_types, max_rhs, store, form, (0, 0, 0, 0) if form == EMSURF_T_LK else None, recip)
    return int(lib().emsurf_plan_bytes(ctypes.byref(d)))


def _blocks_arg(T_blocks):
    if isinstance(T_blocks, np.ndarray):
        tb, ptb = _host(T_blocks, np.complex128)
        return tb, ptb, 0
    return T_blocks, _dptr(T_blocks), 1


def emsurf_plan_create(nx, ny, n_eq, n_types, max_rhs, T_blocks, S_types, elem_type,
                       store=EMSURF_STORE_FP64 | EMSURF_STORE_FP32, stream=None, form=EMSURF_T_DENSE,
                       coef=None, recip=0) -> Plan:
    """T_blocks: numpy complex128 [2ny-1][2nx-1][n][n] (dense) or [2ny-1][2nx-1][2][n/2][n/2]
    (EMSURF_T_LK: L then K), host array or device tensor."""
    d = _desc(nx, ny, n_eq, n_types, max_rhs, store, form, coef, recip)
    tb, ptb, is_dev = _blocks_arg(T_blocks)
    S, pS = _host(S_types, np.complex128)
    et, pet = _host(elem_type, np.int32)
    out = ctypes.c_void_p()
    _check(lib().emsurf_plan_create(ctypes.byref(d), ptb, is_dev, pS, pet, _stream(stream), ctypes.byref(out)))
    return Plan(out.value, d)


def emsurf_plan_create_reciprocal(nx, ny, n_eq, n_types, max_rhs, T_blocks, weights, S_types, elem_type,
                                  store=EMSURF_STORE_FP64 | EMSURF_STORE_FP32, stream=None, recip=1,
                                  form=EMSURF_T_DENSE, coef=None) -> Plan:
    """Dense blocks with T(-d) = W^-1 T(d)^T W (weights: n_eq reals), or with
    form=EMSURF_T_LK structured blocks [..][2][n_eq/2][n_eq/2] whose L and K are
    each reciprocal under n_eq/2 weights; None means all ones."""
    d = _desc(nx, ny, n_eq, n_types, max_rhs, store, form, coef, recip)
    tb, ptb, is_dev = _blocks_arg(T_blocks)
    if weights is None:
        wt, pw = None, None
    else:
        wt, pw = _host(weights, np.float64)
    S, pS = _host(S_types, np.complex128)
    et, pet = _host(elem_type, np.int32)
    out = ctypes.c_void_p()
    _check(lib().emsurf_plan_create_reciprocal(ctypes.byref(d), ptb, is_dev, pw, pS, pet, _stream(stream),
                                               ctypes.byref(out)))
    return Plan(out.value, d)


def emsurf_spectrum_pairs(Lx, Ly) -> np.ndarray:
    """Stored frequency pairs (k, -k) of a reciprocal plan: int32 [count][2]."""
    cnt = ctypes.c_int64(0)
    _check(lib().emsurf_spectrum_pairs(int(Lx), int(Ly), None, ctypes.byref(cnt)))
    out = np.zeros((cnt.value, 2), dtype=np.int32)
    if cnt.value:
        _check(lib().emsurf_spectrum_pairs(int(Lx), int(Ly), out.ctypes.data_as(ctypes.c_void_p), ctypes.byref(cnt)))
    return out


def emsurf_plan_create_green(nx, ny, n_types, max_rhs, geom: Geometry, S_types, elem_type,
                             store=EMSURF_STORE_FP64 | EMSURF_STORE_FP32, stream=None, form=EMSURF_T_DENSE,
                             coef=None, recip=0) -> Plan:
    d = _desc(nx, ny, 4 * geom.n_patch, n_types, max_rhs, store, form, coef, recip)
    S, pS = _host(S_types, np.complex128)
    et, pet = _host(elem_type, np.int32)
    out = ctypes.c_void_p()
    _check(lib().emsurf_plan_create_green(ctypes.byref(d), ctypes.byref(geom.c), pS, pet, _stream(stream),
                                          ctypes.byref(out)))
    return Plan(out.value, d)


def emsurf_fill_T_point_green(geom: Geometry, nx, ny, T_blocks_dev, stream=None):
    _check(lib().emsurf_fill_T_point_green(ctypes.byref(geom.c), int(nx), int(ny), _dptr(T_blocks_dev),
                                           _stream(stream)))


def emsurf_fill_LK_point_green(geom: Geometry, nx, ny, LK_blocks_dev, stream=None):
    _check(lib().emsurf_fill_LK_point_green(ctypes.byref(geom.c), int(nx), int(ny), _dptr(LK_blocks_dev),
                                            _stream(stream)))


def emsurf_macromodels(n_types, n_eq, n_int, Z_dev, Zself_dev, S_dev, Zt_dev=None, stream=None):
    """Device tensors: Z [T][N][N], Zself [n][n] or None, S out [T][n][n], Zt out or None."""
    _check(lib().emsurf_macromodels(int(n_types), int(n_eq), int(n_int), _dptr(Z_dev),
                                    None if Zself_dev is None else _dptr(Zself_dev), _dptr(S_dev),
                                    None if Zt_dev is None else _dptr(Zt_dev), _stream(stream)))


def emsurf_far_field(geom: Geometry, nx, ny, nrhs, Lu, Lv, x_dev, E_dev, stream=None):
    """x_dev c128 [nrhs][ny][nx][n_eq]; E_dev c128 [nrhs][Lv][Lu][2] (E_theta, E_phi)."""
    _check(lib().emsurf_far_field(ctypes.byref(geom.c), int(nx), int(ny), int(nrhs), int(Lu), int(Lv),
                                  _dptr(x_dev), _dptr(E_dev), _stream(stream)))


def emsurf_directivity(geom: Geometry, nx, ny, nrhs, Lu, Lv, x_dev, D_dev, stream=None):
    """Returns P_rad per right-hand side (numpy float64 [nrhs]); D_dev receives
    the directivity, float64 [nrhs][2][Lv][Lu]."""
    pr = (ctypes.c_double * int(nrhs))()
    _check(lib().emsurf_directivity(ctypes.byref(geom.c), int(nx), int(ny), int(nrhs), int(Lu), int(Lv),
                                    _dptr(x_dev), _dptr(D_dev), pr, _stream(stream)))
    return np.array(pr[:], dtype=np.float64)


def emsurf_apply_T(plan: Plan, prec, nrhs, x_dev, y_dev, stream=None):
    _check(lib().emsurf_apply_T(plan.h, int(prec), int(nrhs), _dptr(x_dev), _dptr(y_dev), _stream(stream)))


def emsurf_apply_T_noalloc(plan: Plan, prec, nrhs, x_dev, y_dev, stream=None):
    _check(lib().emsurf_apply_T_noalloc(plan.h, int(prec), int(nrhs), _dptr(x_dev), _dptr(y_dev), _stream(stream)))


def emsurf_apply_T_noalloc_limit() -> int:
    return int(lib().emsurf_apply_T_noalloc_limit())


def emsurf_apply_S(plan: Plan, prec, nrhs, x_dev, y_dev, stream=None):
    _check(lib().emsurf_apply_S(plan.h, int(prec), int(nrhs), _dptr(x_dev), _dptr(y_dev), _stream(stream)))


def emsurf_apply_A(plan: Plan, prec, nrhs, x_dev, y_dev, stream=None):
    _check(lib().emsurf_apply_A(plan.h, int(prec), int(nrhs), _dptr(x_dev), _dptr(y_dev), _stream(stream)))


def solve_opts(prec=EMSURF_FP64, tol=1e-10, restart=30, max_iter=500, use_x0=0, inner_tol=1e-6, max_outer=10):
    return emsurf_solve_opts(int(prec), float(tol), int(restart), int(max_iter), int(use_x0), float(inner_tol),
                             int(max_outer))


def emsurf_solve(plan: Plan, opts: emsurf_solve_opts, nrhs, b_dev, x_dev, stream=None, raise_not_converged=False):
    """Returns (status, [info per RHS as dicts])."""
    infos = (emsurf_solve_info * int(nrhs))()
    st = lib().emsurf_solve(plan.h, ctypes.byref(opts), int(nrhs), _dptr(b_dev), _dptr(x_dev), infos,
                            _stream(stream))
    if st != EMSURF_OK and (st != EMSURF_ERR_NOT_CONVERGED or raise_not_converged):
        _check(st)
    out = [dict(iters=i.iters, outer_iters=i.outer_iters, converged=bool(i.converged),
                rel_res_true=i.rel_res_true, ms=i.ms) for i in infos]
    return st, out


class Overlap:
    """Handle of a touching-box incidence U_o (destroyed before its plan)."""

    def __init__(self, handle, plan: Plan):
        self.h = handle
        self.plan = plan

    def destroy(self):
        if self.h:
            lib().emsurf_overlap_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def sizes(self):
        return emsurf_overlap_query(self)


def emsurf_overlap_create(plan: Plan, geom: Geometry, ground_plane=0, stream=None) -> Overlap:
    out = ctypes.c_void_p()
    _check(lib().emsurf_overlap_create(plan.h, ctypes.byref(geom.c), int(ground_plane), _stream(stream),
                                       ctypes.byref(out)))
    return Overlap(out.value, plan)


def emsurf_overlap_query(ov: Overlap):
    nf, nu, nb = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_size_t()
    _check(lib().emsurf_overlap_query(ov.h, ctypes.byref(nf), ctypes.byref(nu), ctypes.byref(nb)))
    return dict(n_full=nf.value, n_unique=nu.value, bytes=nb.value)


def emsurf_overlap_expand(ov: Overlap, nrhs, xt_dev, x_dev, stream=None):
    _check(lib().emsurf_overlap_expand(ov.h, int(nrhs), _dptr(xt_dev), _dptr(x_dev), _stream(stream)))


def emsurf_overlap_reduce(ov: Overlap, nrhs, y_dev, yt_dev, stream=None):
    _check(lib().emsurf_overlap_reduce(ov.h, int(nrhs), _dptr(y_dev), _dptr(yt_dev), _stream(stream)))


def emsurf_apply_reduced(ov: Overlap, nrhs, xt_dev, yt_dev, stream=None):
    _check(lib().emsurf_apply_reduced(ov.h, int(nrhs), _dptr(xt_dev), _dptr(yt_dev), _stream(stream)))


def emsurf_overlap_destroy(ov: Overlap):
    ov.destroy()


class Precond:
    """Handle of a near-field right preconditioner (destroyed with destroy()
    or when garbage collected, before its plan)."""

    def __init__(self, handle, plan: Plan):
        self.h = handle
        self.plan = plan

    def destroy(self):
        if self.h:
            lib().emsurf_precond_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def stats(self):
        return emsurf_precond_query(self)


def emsurf_precond_create(plan: Plan, geom: Geometry, delta_nf, tile_x, tile_y, T_near=None, stream=None) -> Precond:
    """T_near: numpy complex128 [3][3][n_eq][n_eq] (host) or None for the point-sampled fill of geom."""
    if T_near is not None:
        tn, ptn = _host(T_near, np.complex128)
    else:
        tn, ptn = None, None
    out = ctypes.c_void_p()
    _check(lib().emsurf_precond_create(plan.h, ctypes.byref(geom.c), float(delta_nf), int(tile_x), int(tile_y), ptn,
                                       _stream(stream), ctypes.byref(out)))
    return Precond(out.value, plan)


def emsurf_precond_apply(pc: Precond, nrhs, y_dev, x_dev, stream=None):
    _check(lib().emsurf_precond_apply(pc.h, int(nrhs), _dptr(y_dev), _dptr(x_dev), _stream(stream)))


def emsurf_precond_query(pc: Precond):
    s = emsurf_precond_stats()
    _check(lib().emsurf_precond_query(pc.h, ctypes.byref(s)))
    return dict(n_tiles=s.n_tiles, nq_max=s.nq_max, near_entries=s.near_entries, bytes=s.bytes, build_ms=s.build_ms)


def emsurf_precond_destroy(pc: Precond):
    pc.destroy()


def emsurf_solve_precond(plan: Plan, pc: Precond, opts: emsurf_solve_opts, nrhs, b_dev, x_dev, stream=None,
                         raise_not_converged=False):
    """emsurf_solve on the right-preconditioned system; returns (status, [info per RHS])."""
    infos = (emsurf_solve_info * int(nrhs))()
    st = lib().emsurf_solve_precond(plan.h, pc.h, ctypes.byref(opts), int(nrhs), _dptr(b_dev), _dptr(x_dev), infos,
                                    _stream(stream))
    if st != EMSURF_OK and (st != EMSURF_ERR_NOT_CONVERGED or raise_not_converged):
        _check(st)
    out = [dict(iters=i.iters, outer_iters=i.outer_iters, converged=bool(i.converged),
                rel_res_true=i.rel_res_true, ms=i.ms) for i in infos]
    return st, out


def emsurf_plan_query(plan: Plan) -> emsurf_plan_stats:
    s = emsurf_plan_stats()
    _check(lib().emsurf_plan_query(plan.h, ctypes.byref(s)))
    return s


def emsurf_kernel_timing(plan: Plan, enable: bool):
    _check(lib().emsurf_kernel_timing(plan.h, 1 if enable else 0))


def emsurf_kernel_times(plan: Plan):
    """Summed ms and launch counts per apply_T phase since the last call."""
    ms = (ctypes.c_double * 5)()
    cnt = (ctypes.c_int64 * 5)()
    _check(lib().emsurf_kernel_times(plan.h, ms, cnt))
    return {p: (ms[i], cnt[i]) for i, p in enumerate(PHASES)}


def emsurf_status_str(st: int) -> str:
    return lib().emsurf_status_str(int(st)).decode()


def emsurf_last_error() -> str:
    return lib().emsurf_last_error().decode()


def emsurf_plan_destroy(plan: Plan):
    plan.destroy()


def emsurf_plan_autotune(plan: Plan, nrhs, stream=None):
    """Returns (best variant, {variant name: ms or None})."""
    ms = (ctypes.c_double * EMSURF_BP_NVARIANTS)()
    best = ctypes.c_int32()
    _check(lib().emsurf_plan_autotune(plan.h, int(nrhs), ms, ctypes.byref(best), _stream(stream)))
    return best.value, {BP_NAMES[i]: (ms[i] if ms[i] >= 0 else None) for i in range(EMSURF_BP_NVARIANTS)}


def emsurf_plan_set_variant(plan: Plan, nrhs, variant):
    _check(lib().emsurf_plan_set_variant(plan.h, int(nrhs), int(variant)))


class Graph:
    def __init__(self, handle):
        self.h = handle

    def launch(self, stream=None):
        emsurf_graph_launch(self, stream)

    def destroy(self):
        if self.h:
            lib().emsurf_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def emsurf_graph_create(plan: Plan, op, prec, nrhs, x_dev, y_dev, stream) -> Graph:
    out = ctypes.c_void_p()
    _check(lib().emsurf_graph_create(plan.h, int(op), int(prec), int(nrhs), _dptr(x_dev), _dptr(y_dev),
                                     _stream(stream), ctypes.byref(out)))
    return Graph(out.value)


def emsurf_graph_launch(graph: Graph, stream=None):
    _check(lib().emsurf_graph_launch(graph.h, _stream(stream)))


def emsurf_graph_destroy(graph: Graph):
    graph.destroy()


def _info_dict(i):
    return dict(iters=i.iters, outer_iters=i.outer_iters, converged=bool(i.converged),
                rel_res_true=i.rel_res_true, ms=i.ms)


class Session:
    def __init__(self, handle):
        self.h = handle

    def destroy(self):
        if self.h:
            lib().emsurf_session_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def emsurf_session_bytes(plan: Plan, max_slots, opts) -> int:
    return int(lib().emsurf_session_bytes(plan.h, int(max_slots), ctypes.byref(opts)))


def emsurf_session_create(plan: Plan, max_slots, opts, stream=None) -> Session:
    out = ctypes.c_void_p()
    _check(lib().emsurf_session_create(plan.h, int(max_slots), ctypes.byref(opts), _stream(stream), ctypes.byref(out)))
    return Session(out.value)


def emsurf_session_submit(sess: Session, b_dev, tag=0) -> int:
    slot = ctypes.c_int32()
    _check(lib().emsurf_session_submit(sess.h, _dptr(b_dev), int(tag), ctypes.byref(slot)))
    return slot.value


def emsurf_session_step(sess: Session) -> int:
    n = ctypes.c_int32()
    _check(lib().emsurf_session_step(sess.h, ctypes.byref(n)))
    return n.value


def emsurf_session_finished(sess: Session, cap=64):
    slots = (ctypes.c_int32 * cap)()
    tags = (ctypes.c_int64 * cap)()
    cnt = ctypes.c_int32()
    _check(lib().emsurf_session_finished(sess.h, slots, tags, int(cap), ctypes.byref(cnt)))
    return [(slots[i], tags[i]) for i in range(min(cnt.value, cap))]


def emsurf_session_active(sess: Session) -> int:
    n = ctypes.c_int32()
    _check(lib().emsurf_session_active(sess.h, ctypes.byref(n)))
    return n.value


def emsurf_session_collect(sess: Session, slot, x_dev=None):
    info = emsurf_solve_info()
    _check(lib().emsurf_session_collect(sess.h, int(slot), _dptr(x_dev), ctypes.byref(info)))
    return _info_dict(info)


def emsurf_session_destroy(sess: Session):
    sess.destroy()


class Server:
    def __init__(self, handle):
        self.h = handle

    def destroy(self):
        if self.h:
            lib().emsurf_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def emsurf_server_create(budget_bytes, max_slots, opts, store=EMSURF_STORE_FP64 | EMSURF_STORE_FP32) -> Server:
    d = emsurf_server_desc(int(budget_bytes), int(max_slots), int(store), opts)
    out = ctypes.c_void_p()
    _check(lib().emsurf_server_create(ctypes.byref(d), ctypes.byref(out)))
    return Server(out.value)


def emsurf_server_submit(srv: Server, key, nx, ny, n_types, geom: Geometry, S_types, elem_type, b,
                         form=EMSURF_T_DENSE, coef=None, recip=0) -> int:
    """b: numpy complex128 [nrhs][ny][nx][n_eq] (host)."""
    d = _desc(nx, ny, 4 * geom.n_patch, n_types, 1, EMSURF_STORE_FP64, form, coef, recip)
    S, pS = _host(S_types, np.complex128)
    et, pet = _host(elem_type, np.int32)
    bb, pb = _host(b, np.complex128)
    rid = ctypes.c_int64()
    _check(lib().emsurf_server_submit(srv.h, int(key), ctypes.byref(d), ctypes.byref(geom.c), pS, pet,
                                      int(bb.shape[0]), pb, ctypes.byref(rid)))
    return rid.value


def emsurf_server_step(srv: Server) -> int:
    n = ctypes.c_int32()
    _check(lib().emsurf_server_step(srv.h, ctypes.byref(n)))
    return n.value


def emsurf_server_next_completed(srv: Server):
    rid = ctypes.c_int64()
    nrhs = ctypes.c_int32()
    nu = ctypes.c_int64()
    _check(lib().emsurf_server_next_completed(srv.h, ctypes.byref(rid), ctypes.byref(nrhs), ctypes.byref(nu)))
    return (rid.value, nrhs.value, nu.value) if rid.value >= 0 else None


def emsurf_server_fetch(srv: Server, req_id, nrhs, n_unknowns, want_x=True):
    x = np.empty((nrhs, n_unknowns), dtype=np.complex128) if want_x else None
    infos = (emsurf_solve_info * int(nrhs))()
    times = (ctypes.c_double * 2)()
    _check(lib().emsurf_server_fetch(srv.h, int(req_id), x.ctypes.data_as(ctypes.c_void_p) if want_x else None,
                                     infos, times))
    return x, [_info_dict(i) for i in infos], (times[0], times[1])


def emsurf_server_query(srv: Server):
    s = emsurf_server_stats()
    _check(lib().emsurf_server_query(srv.h, ctypes.byref(s)))
    return dict(queued=s.queued, active=s.active, resident_plans=s.resident_plans, bytes_used=s.bytes_used,
                plans_built=s.plans_built, evictions=s.evictions, admit_ms=round(s.admit_ms, 1),
                step_ms=round(s.step_ms, 1))


def emsurf_server_destroy(srv: Server):
    srv.destroy()


def emsurf_server_entry_bytes(srv: Server, nx, ny, n_eq, n_types) -> int:
    d = _desc(nx, ny, n_eq, n_types, 1, EMSURF_STORE_FP64)
    return int(lib().emsurf_server_entry_bytes(srv.h, ctypes.byref(d)))


def emsurf_server_slot_bytes(srv: Server, nx, ny, n_eq, n_types) -> int:
    d = _desc(nx, ny, n_eq, n_types, 1, EMSURF_STORE_FP64)
    return int(lib().emsurf_server_slot_bytes(srv.h, ctypes.byref(d)))
