"""Oracle: Krylov solve of A x = b, and a dense LU reference.

The paper solves its final system iteratively with GMRES (Sec. IV-A) and does
not state its variant.  The reading used here (and by the GPU solver):

* restarted GMRES(m) of Saad and Schultz (1986): Arnoldi basis, Hessenberg
  least squares by Givens rotations, x = x0 + V y at the end of a cycle;
* classical Gram-Schmidt applied twice per Arnoldi step ("twice is enough"),
  Hermitian inner product u^H v;
* complex Givens rotation [c s; -conj(s) c] with real c;
* stop a cycle when the estimated relative residual |g_{j+1}|/||b|| <= tol,
  then confirm with the true residual ||b - A x|| / ||b||; if it is not yet
  below tol, restart from that x;
* lucky breakdown when h_{j+1,j} <= 1e-14 * ||A v_j||;
* x0 = 0 unless given; each right-hand side is an independent solve;
* optional right preconditioning (Sec. IV-A, eq. (final_precond)): the
  Arnoldi process runs on A M^-1, the cycle ends with x += M^-1 (V y), and
  every residual is the unpreconditioned b - A x.

Parity: pinned by dense LU (library zgesv), by scipy's GMRES iteration counts,
by finite termination on tiny systems and by the closed-form solves in
tests/test_oracle_krylov.py.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class GmresInfo:
    iters: int
    converged: bool
    rel_res_true: float
    history: list          # estimated relative residual after every Arnoldi step
    restarts: int


def givens(a: complex, b: complex):
    """Rotation (c, s) with c real such that [c s; -conj(s) c] [a; b] = [rho; 0]."""
    if b == 0:
        return 1.0, 0.0 + 0.0j
    if a == 0:
        return 0.0, np.conj(b) / abs(b)
    r = np.hypot(abs(a), abs(b))
    return abs(a) / r, (a / abs(a)) * np.conj(b) / r


def gmres(apply_A, b: np.ndarray, tol: float, restart: int = 30, max_iter: int = 500,
          x0: np.ndarray | None = None, breakdown: float = 1e-14, M_inv=None):
    """Solve A x = b for one right-hand side (flat complex vector); M_inv, if
    given, is the right preconditioner's solve v -> M^-1 v."""
    b = np.asarray(b, dtype=np.complex128).ravel()
    bnorm = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128).ravel()
    hist = []
    if bnorm == 0.0:
        return np.zeros_like(b), GmresInfo(0, True, 0.0, hist, 0)
    total = 0
    restarts = 0
    while True:
        r = b - apply_A(x)
        beta = np.linalg.norm(r)
        if beta / bnorm <= tol:
            return x, GmresInfo(total, True, beta / bnorm, hist, restarts)
        if total >= max_iter:
            return x, GmresInfo(total, False, beta / bnorm, hist, restarts)
        m = restart
        V = np.zeros((m + 1, b.size), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        V[0] = r / beta
        j_end = None
        for j in range(m):
            w = apply_A(V[j] if M_inv is None else M_inv(V[j]))
            total += 1
            wnorm0 = np.linalg.norm(w)
            h = np.zeros(j + 1, dtype=np.complex128)
            for _ in range(2):                       # classical Gram-Schmidt, twice
                c = V[: j + 1].conj() @ w
                w = w - c @ V[: j + 1]
                h += c
            hn = np.linalg.norm(w)
            H[: j + 1, j] = h
            H[j + 1, j] = hn
            for i in range(j):                       # previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            cs[j], sn[j] = givens(H[j, j], H[j + 1, j])
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            est = abs(g[j + 1]) / bnorm
            hist.append(est)
            lucky = hn <= breakdown * wnorm0
            if est <= tol or lucky or total >= max_iter or j == m - 1:
                j_end = j
                break
            V[j + 1] = w / hn
        k = j_end + 1
        y = _back_substitute(H[:k, :k], g[:k])
        x = x + (y @ V[:k] if M_inv is None else M_inv(y @ V[:k]))
        restarts += 1


def _back_substitute(R: np.ndarray, g: np.ndarray) -> np.ndarray:
    k = R.shape[0]
    y = np.zeros(k, dtype=np.complex128)
    for i in range(k - 1, -1, -1):
        y[i] = (g[i] - R[i, i + 1:] @ y[i + 1:]) / R[i, i]
    return y


def gmres_multi(apply_A_multi, b: np.ndarray, tol: float, **kw):
    """Independent GMRES per right-hand side; b is [nrhs][...]."""
    shape = b.shape
    nrhs = shape[0]
    xs, infos = [], []
    for r in range(nrhs):
        def A1(v, _r=r):
            return apply_A_multi(v.reshape((1,) + shape[1:])).ravel()
        x, info = gmres(A1, b[r].ravel(), tol, **kw)
        xs.append(x.reshape(shape[1:]))
        infos.append(info)
    return np.stack(xs), infos


def solve_dense(A: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Direct solve by LU with partial pivoting (LAPACK zgesv)."""
    return np.linalg.solve(A, b)
