"""Oracle (test infrastructure only): boundary conditions on touching
fictitious surfaces (Sec. III-D, eqs. (connections_IUI), (final)).

When adjacent boxes touch (lattice pitch equal to the box edge), a face of one
box coincides with a face of its neighbour and the currents of that face are
expanded twice.  The paper keeps one set of unknowns through the sparse
incidence U_o, Y = U_o Y~, and solves U_o^T [Z_eq + Z_o] U_o Y~ = U_o^T V.

Readings for the point-sampled patches used here:
* duplicates: patch p' of element m' = m + d (d = (0, 1) or (1, 0), the
  neighbour in +x or +y) whose centre coincides with patch p of element m;
  the tangential fields are continuous across the shared face and the two
  boxes' outward normals are opposite, so the equivalent currents
  (J = n x H, M = -n x E) reverse: x[m', tau, p', b] = -sum_a (t_p'b . t_pa)
  x[m, tau, p, a] for both currents tau; the unknowns of m keep the face;
* ground plane (optional): the bottom face of every box lies on a PEC ground
  plane, where the tangential electric field vanishes, so its M unknowns are
  zero and leave the system; its J unknowns stay.  The paper's rules at the
  edges of ground planes act on RWG edge functions, which the point-sampled
  patches do not have;
* U_o columns: the unknowns that are neither duplicates nor eliminated, in
  increasing order of their full index m n_eq + u;
* the paper's Z_eq + Z_o is D + T here, D = -S^-1 per element (S the
  macromodel of the block-Jacobi form, so that (I - S T) = -S (D + T)).

Pins (tests/test_oracle_overlap.py): the counts of shared-face and
ground-plane unknowns in closed form; U_o = I for boxes that do not touch;
U_o^T U_o = diag(multiplicities); the expanded currents cancel on every
shared face; the reduced system's solution expands to a solution of the
full system restricted to range(U_o); the coincident-patch Green's term
against a numerical integral over the square.
"""
from __future__ import annotations

import numpy as np


def _patch_of(u: int, P: int):
    tau, r = divmod(u, 2 * P)
    return tau, r // 2, r % 2


def incidence(rho: np.ndarray, tan: np.ndarray, nx: int, ny: int, pitch: float, ground_plane: bool = False,
              tol: float = 1e-9) -> np.ndarray:
    """Dense U_o, [M n_eq][N~] (small lattices)."""
    P = rho.shape[0]
    n = 4 * P
    N = nx * ny * n
    # for each full unknown: its source (m, u) and the coefficient matrix entry, or None
    src = {}
    zmin = rho[:, 2].min()
    bottom = [np.isclose(rho[p, 2], zmin, atol=tol) and abs(tan[p, 0, 2]) < tol and abs(tan[p, 1, 2]) < tol
              for p in range(P)]
    for iy in range(ny):
        for ix in range(nx):
            m = iy * nx + ix
            for d in ((0, 1), (1, 0)):                     # (dy, dx) to the neighbour m - d that keeps the face
                jy, jx = iy - d[0], ix - d[1]
                if jy < 0 or jx < 0:
                    continue
                mo = jy * nx + jx
                for pp in range(P):                          # patch of m coinciding with patch p of mo
                    for p in range(P):
                        if np.linalg.norm(rho[pp] + pitch * np.array([d[1], d[0], 0.0]) - rho[p]) <= tol:
                            for tau in (0, 1):
                                for b in (0, 1):
                                    u = tau * 2 * P + 2 * pp + b
                                    src[m * n + u] = [(mo * n + tau * 2 * P + 2 * p + a, -float(tan[pp, b] @ tan[p, a]))
                                                      for a in (0, 1)]
    elim = set()
    if ground_plane:
        for m in range(nx * ny):
            for p in range(P):
                if bottom[p]:
                    for a in (0, 1):
                        elim.add(m * n + 2 * P + 2 * p + a)
    keep = [i for i in range(N) if i not in src and i not in elim]
    col = {i: c for c, i in enumerate(keep)}
    U = np.zeros((N, len(keep)))
    for i in keep:
        U[i, col[i]] = 1.0
    for i, terms in src.items():
        if i in elim:
            continue
        for j, c in terms:
            assert j not in src, "a shared face's kept unknown is itself a duplicate"
            if j in col and c != 0.0:
                U[i, col[j]] += c
    return U


def dense_D(S: np.ndarray, tm: np.ndarray) -> np.ndarray:
    """Block diagonal D = -S^-1 per element (LAPACK inverse of each type)."""
    n = S.shape[-1]
    Dt = np.stack([-np.linalg.inv(S[t]) for t in range(S.shape[0])])
    M = tm.size
    D = np.zeros((M * n, M * n), dtype=np.complex128)
    for m, t in enumerate(tm.ravel()):
        D[m * n:(m + 1) * n, m * n:(m + 1) * n] = Dt[t]
    return D


def reduced_operator(U: np.ndarray, D: np.ndarray, T: np.ndarray) -> np.ndarray:
    """A~ = U_o^T (D + T) U_o (eq. (final), the D and T defined here)."""
    return U.T @ (D + T) @ U
