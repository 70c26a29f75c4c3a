"""Seeded synthetic inputs for the coupled-macromodel solve of a lattice of
fictitious boxes (Patel, Triverio, Hum, "A Fast Macromodeling Approach to
Efficiently Simulate Inhomogeneous Electromagnetic Surfaces").

This module only *draws and lays out inputs*: the patch geometry of one box,
random per-cell-type macromodels, the cell-type map of the lattice, incidence
angles, the sampled plane-wave excitation, random dense coupling blocks and
random vectors.  None of the method's arithmetic lives here: no coupling
operator, no FFT, no macromodel apply, no Krylov solve.  Both the CPU oracle
and the GPU library consume what this module produces; neither is imported.

Conventions (one wavelength = 1, so k = 2*pi; e^{+j w t} time convention,
free-space impedance eta = 1 so that M is scaled by 1/eta):

* Box of one lattice element: 0.45 x 0.45 x 0.10, centred on its lattice
  point; lattice pitch 0.5 so facing faces of neighbours leave a 0.05 gap.
* Patches: the +z and -z faces carry an n_t x n_t grid; each of the four side
  faces an s_a (along its 0.45 edge) x s_h (along z) grid.  Face order
  [+z, -z, +x, -x, +y, -y]; row-major inside a face with the index along the
  first tangent fastest.  Tangents: +-z faces (x, y); +-x faces (y, z);
  +-y faces (x, z).  Normals point out of the box.
* Local unknown order on one box (J block first, then M, Sec. II-A):
  u = tau*(2*n_patch) + 2*p + alpha, tau = 0 for J, 1 for M, alpha the
  tangent index.  Element m = iy*nx + ix; vectors are [rhs][iy][ix][u]
  (the element-major stacking of Sec. III-A).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_ROOT = 191104576          # arXiv id 1911.04576
WAVELENGTH = 1.0
K0 = 2.0 * math.pi / WAVELENGTH
PITCH = 0.5
BOX_A = 0.45                    # box edge along x and y
BOX_H = 0.10                    # box height along z

# Constants (a, b, c, e) of the structured outer operator
# T = [[a L, b K], [c K, e L]]: the outer EFIE and MFIE scale L by -j omega mu0
# and +j omega eps0 and K by +1 and -1; with eta = 1 both products are k.
OUTER_COEF = (-1j * K0, 1.0 + 0j, -1.0 + 0j, 1j * K0)

# (n_t, s_a, s_h) patch grids -> 24, 48, 72 patches per box
PATCH_GRIDS = {24: (2, 2, 2), 48: (4, 4, 1), 72: (4, 5, 2)}

# stream order of SeedSequence.spawn for every config
_STREAMS = ("s_types", "type_map", "rhs_angles", "arrivals", "serving", "test_blocks")


@dataclasses.dataclass(frozen=True)
class BoxGeometry:
    """Patch layout of one fictitious box (identical for every element)."""
    rho: np.ndarray      # [n_patch, 3] patch centres relative to the box centre
    area: np.ndarray     # [n_patch]
    tan: np.ndarray      # [n_patch, 2, 3] unit tangents
    normal: np.ndarray   # [n_patch, 3] outward unit normal
    grid: tuple

    @property
    def n_patch(self) -> int:
        return int(self.rho.shape[0])

    @property
    def n_eq(self) -> int:
        return 4 * self.n_patch


def box_geometry(n_patch: int) -> BoxGeometry:
    n_t, s_a, s_h = PATCH_GRIDS[n_patch]
    a, h = BOX_A, BOX_H
    ex, ey, ez = np.eye(3)
    rho, area, tan, nrm = [], [], [], []

    def face(origin, t1, t2, n1, n2, len1, len2, normal):
        d1, d2 = len1 / n1, len2 / n2
        for i2 in range(n2):
            for i1 in range(n1):
                c = origin + t1 * (-len1 / 2 + (i1 + 0.5) * d1) + t2 * (-len2 / 2 + (i2 + 0.5) * d2)
                rho.append(c)
                area.append(d1 * d2)
                tan.append(np.stack([t1, t2]))
                nrm.append(normal)

    face(+ez * h / 2, ex, ey, n_t, n_t, a, a, +ez)
    face(-ez * h / 2, ex, ey, n_t, n_t, a, a, -ez)
    face(+ex * a / 2, ey, ez, s_a, s_h, a, h, +ex)
    face(-ex * a / 2, ey, ez, s_a, s_h, a, h, -ex)
    face(+ey * a / 2, ex, ez, s_a, s_h, a, h, +ey)
    face(-ey * a / 2, ex, ez, s_a, s_h, a, h, -ey)
    g = BoxGeometry(np.array(rho, dtype=np.float64), np.array(area, dtype=np.float64),
                    np.array(tan, dtype=np.float64), np.array(nrm, dtype=np.float64),
                    (n_t, s_a, s_h))
    assert g.n_patch == n_patch
    return g


@dataclasses.dataclass(frozen=True)
class Config:
    cfg: int
    nx: int
    ny: int
    n_patch: int
    n_types: int
    angles: tuple          # ((theta_rad, pol), ...) pol in {"TE", "TM"}
    tol: float

    @property
    def n_eq(self) -> int:
        return 4 * self.n_patch

    @property
    def M(self) -> int:
        return self.nx * self.ny

    @property
    def nrhs(self) -> int:
        return len(self.angles)

    @property
    def n_unknowns(self) -> int:
        return self.M * self.n_eq


def streams(cfg: int):
    ss = np.random.SeedSequence([SEED_ROOT, cfg])
    kids = ss.spawn(len(_STREAMS))
    return {name: np.random.Generator(np.random.PCG64(k)) for name, k in zip(_STREAMS, kids)}


def config(cfg: int) -> Config:
    """The four fixed lattice workloads (the fifth, serving, is drawn per request)."""
    d = math.radians
    if cfg == 1:
        return Config(1, 4, 4, 24, 4, ((0.0, "TE"),), 1e-10)
    if cfg == 2:
        return Config(2, 32, 32, 48, 16, ((d(30.0), "TE"),), 1e-8)
    if cfg == 3:
        th = np.sort(streams(3)["rhs_angles"].uniform(0.0, d(60.0), size=8))
        ang = tuple((float(t), p) for t in th for p in ("TE", "TM"))
        return Config(3, 64, 64, 72, 32, ang, 1e-6)
    if cfg == 4:
        ang = tuple((d(t), p) for t in (0.0, 30.0) for p in ("TE", "TM"))
        return Config(4, 128, 128, 48, 16, ang, 1e-6)
    raise ValueError(f"no fixed config {cfg}")


def small_config(nx: int, ny: int, n_patch: int = 24, n_types: int = 4, nrhs: int = 1, seed: int = 0) -> Config:
    """Reduced lattices for tests (same recipe, seeded by `seed` instead of a config id)."""
    angles = tuple((math.radians(10.0 * i), "TE" if i % 2 == 0 else "TM") for i in range(nrhs))
    return Config(1000 + seed, nx, ny, n_patch, n_types, angles, 1e-10)


def s_types(cfg: Config, rng=None) -> np.ndarray:
    """Per-cell-type macromodels: iid complex Gaussian, scaled to spectral norm 0.5.

    Returns complex128 [n_types][n_eq][n_eq]; the apply is y_u = sum_v S[u][v] x_v.
    """
    rng = rng if rng is not None else streams(cfg.cfg)["s_types"]
    n = cfg.n_eq
    out = np.empty((cfg.n_types, n, n), dtype=np.complex128)
    for t in range(cfg.n_types):
        z = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / math.sqrt(2.0)
        smax = np.linalg.svd(z, compute_uv=False)[0]
        out[t] = 0.5 * z / smax
    return out


def type_map(cfg: Config, rng=None) -> np.ndarray:
    """Cell type of every element, int32 [ny][nx], uniform over the types."""
    rng = rng if rng is not None else streams(cfg.cfg)["type_map"]
    return rng.integers(0, cfg.n_types, size=(cfg.ny, cfg.nx)).astype(np.int32)


def element_positions(nx: int, ny: int, pitch: float = PITCH) -> np.ndarray:
    """Lattice point of every element, [ny][nx][3]; element (0, 0) at the origin."""
    iy, ix = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    pos = np.zeros((ny, nx, 3))
    pos[..., 0] = ix * pitch
    pos[..., 1] = iy * pitch
    return pos


def incident_fields(theta: float, pol: str, pts: np.ndarray, k: float = K0):
    """Plane wave travelling along k_hat = (sin t, 0, -cos t) (phi = 0).

    TE: E along y; TM: E along y x k_hat.  eta = 1, so H = k_hat x E.
    Returns (E, H), each complex [..., 3] at the points `pts` [..., 3].
    """
    khat = np.array([math.sin(theta), 0.0, -math.cos(theta)])
    yhat = np.array([0.0, 1.0, 0.0])
    ehat = yhat if pol == "TE" else np.cross(yhat, khat)
    phase = np.exp(-1j * k * (pts @ khat))
    E = phase[..., None] * ehat
    H = phase[..., None] * np.cross(khat, ehat)
    return E, H


def box_excitation(theta: float, pol: str, geom: BoxGeometry, k: float = K0) -> np.ndarray:
    """Excitation of the box at the origin: the equivalent incident currents
    J = n x H_inc and M = -n x E_inc (Love's equivalence, Sec. II-A) at the
    patch centres, projected on each patch tangent.  complex128 [n_eq]."""
    E, H = incident_fields(theta, pol, geom.rho, k)
    nxH = np.cross(geom.normal, H)
    nxE = np.cross(geom.normal, E)
    npch = geom.n_patch
    c = np.zeros(4 * npch, dtype=np.complex128)
    for a in range(2):
        t = geom.tan[:, a, :]
        c[2 * np.arange(npch) + a] = np.sum(t * nxH, axis=-1)
        c[2 * npch + 2 * np.arange(npch) + a] = np.sum(t * (-nxE), axis=-1)
    return c


def plane_wave_rhs(cfg: Config, geom: BoxGeometry | None = None, pitch: float = PITCH, k: float = K0) -> np.ndarray:
    """Excitation b sampled at the patch centres of every element,
    complex128 [nrhs][ny][nx][n_eq].  A plane wave seen from element m differs
    from the box at the origin only by the phase exp(-j k k_hat . R_m), so each
    right-hand side is that phase times the box excitation."""
    geom = geom if geom is not None else box_geometry(cfg.n_patch)
    pos = element_positions(cfg.nx, cfg.ny, pitch)                    # [ny][nx][3]
    b = np.empty((cfg.nrhs, cfg.ny, cfg.nx, geom.n_eq), dtype=np.complex128)
    for r, (theta, pol) in enumerate(cfg.angles):
        khat = np.array([math.sin(theta), 0.0, -math.cos(theta)])
        phase = np.exp(-1j * k * (pos @ khat))                         # [ny][nx]
        np.multiply(phase[:, :, None], box_excitation(theta, pol, geom, k)[None, None, :], out=b[r])
    return b


def random_blocks(nx: int, ny: int, n_eq: int, seed: int, zero_self: bool = True) -> np.ndarray:
    """Dense, non-symmetric random coupling blocks T(d), complex128
    [2ny-1][2nx-1][n_eq][n_eq] indexed [dy+ny-1][dx+nx-1].  T(0) = 0 unless
    `zero_self` is False.  Scaled so the summed operator has modest norm."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, 77, seed])))
    shape = (2 * ny - 1, 2 * nx - 1, n_eq, n_eq)
    scale = 0.5 / math.sqrt(n_eq * max(1, nx * ny))
    t = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * scale
    if zero_self:
        t[ny - 1, nx - 1] = 0.0
    return t


def random_weights(n_eq: int, seed: int, signed: bool = True) -> np.ndarray:
    """Per-unknown reciprocity weights in [0.5, 2) with random signs (or all
    positive)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, 81, seed])))
    w = 0.5 * 4.0 ** rng.random(n_eq)
    if signed:
        w *= np.where(rng.random(n_eq) < 0.5, -1.0, 1.0)
    return w


def random_reciprocal_blocks(nx: int, ny: int, n_eq: int, w: np.ndarray, seed: int,
                             zero_self: bool = True) -> np.ndarray:
    """Random blocks with T(-d) = W^-1 T(d)^T W, W = diag(w): T(d) is drawn for
    the offsets after (0, 0) in [dy][dx] order and mirrored onto -d; T(0) =
    W^-1 Q with Q complex symmetric (zero if `zero_self`).  Same layout and
    scale as random_blocks."""
    t = random_blocks(nx, ny, n_eq, seed, zero_self=True)
    w = np.asarray(w, dtype=np.float64)
    cy, cx = ny - 1, nx - 1
    for dy in range(-(ny - 1), ny):
        for dx in range(-(nx - 1), nx):
            if (dy, dx) <= (0, 0):
                continue
            t[cy - dy, cx - dx] = (t[cy + dy, cx + dx].T * w[None, :]) / w[:, None]
    if not zero_self:
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, 82, seed])))
        q = rng.standard_normal((n_eq, n_eq)) + 1j * rng.standard_normal((n_eq, n_eq))
        q = (q + q.T) * (0.25 / math.sqrt(n_eq * max(1, nx * ny)))
        t[cy, cx] = q / w[:, None]
    return t


def random_reciprocal_lk_blocks(nx: int, ny: int, n_h: int, w: np.ndarray, seed: int) -> np.ndarray:
    """Random structured blocks [2ny-1][2nx-1][2][n_h][n_h] (L then K), each
    reciprocal under the n_h weights w: X(-d) = W^-1 X(d)^T W, X(0) = 0."""
    L = random_reciprocal_blocks(nx, ny, n_h, w, seed)
    K = random_reciprocal_blocks(nx, ny, n_h, w, seed + 1000)
    return np.stack([L, K], axis=2)


def random_vectors(nrhs: int, nx: int, ny: int, n_eq: int, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, 78, seed])))
    shape = (nrhs, ny, nx, n_eq)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def random_types(n_types: int, n_eq: int, seed: int, norm: float = 0.5) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, 79, seed])))
    out = np.empty((n_types, n_eq, n_eq), dtype=np.complex128)
    for t in range(n_types):
        z = (rng.standard_normal((n_eq, n_eq)) + 1j * rng.standard_normal((n_eq, n_eq))) / math.sqrt(2.0)
        out[t] = norm * z / np.linalg.svd(z, compute_uv=False)[0]
    return out


def random_type_map(nx: int, ny: int, n_types: int, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, 80, seed])))
    return rng.integers(0, n_types, size=(ny, nx)).astype(np.int32)


# ----------------------------------------------------------------------------- serving
@dataclasses.dataclass(frozen=True)
class Surface:
    """One surface of the serving catalogue: an n x n lattice of boxes with
    n_patch patches each and its own seeded macromodels and type map."""
    key: int
    n: int
    n_patch: int
    n_types: int
    seed: int

    @property
    def n_eq(self) -> int:
        return 4 * self.n_patch

    def config(self, angles=((0.0, "TE"),)) -> Config:
        return Config(5000 + self.key, self.n, self.n, self.n_patch, self.n_types, tuple(angles), 1e-6)

    def s_types(self) -> np.ndarray:
        return random_types(self.n_types, self.n_eq, seed=self.seed)

    def type_map(self) -> np.ndarray:
        return random_type_map(self.n, self.n, self.n_types, seed=self.seed)


@dataclasses.dataclass(frozen=True)
class Request:
    rid: int
    arrival_s: float
    surface: int      # index into the catalogue
    nrhs: int
    angles: tuple


def serving_catalogue(n_surfaces: int = 12, n_min: int = 8, n_max: int = 96, patches=(24, 48, 72),
                      n_types: int = 16, cfg: int = 5):
    """Surfaces with lattices n ~ U{n_min..n_max} (n x n), n_eq ~ U{96, 192, 288}."""
    par = streams(cfg)["serving"]
    out = []
    for k in range(n_surfaces):
        n = int(par.integers(n_min, n_max + 1))
        npch = int(par.choice(patches))
        out.append(Surface(k, n, npch, n_types, int(par.integers(0, 2**31 - 1))))
    return out


def serving_stream(n_requests: int, rate_hz: float, n_surfaces: int, max_rhs: int = 32, cfg: int = 5):
    """Poisson arrivals of solve requests on a catalogue of surfaces: surface
    uniform, nrhs ~ U{1..max_rhs}, seeded incidence angles theta ~ U[0, 60 deg]
    and polarisations.  Arrival times scale with 1 / rate_hz (the same draws
    for every rate)."""
    st = streams(cfg)
    gaps = st["arrivals"].exponential(1.0, size=n_requests)
    arr = np.cumsum(gaps) / rate_hz
    par = st["test_blocks"]
    out = []
    for i in range(n_requests):
        k = int(par.integers(0, n_surfaces))
        nrhs = int(par.integers(1, max_rhs + 1))
        th = par.uniform(0.0, math.radians(60.0), size=nrhs)
        pol = par.integers(0, 2, size=nrhs)
        ang = tuple((float(t), "TE" if q == 0 else "TM") for t, q in zip(th, pol))
        out.append(Request(i, float(arr[i]), k, nrhs, ang))
    return out

def cell_interiors(n_types: int, n_eq: int, n_int: int, seed: int):
    """Synthetic discretised cells for macromodel generation: per cell type the
    reduced system [[Z_eq,eq, Z_eq,int], [Z_int,eq, Z_int,int]] (complex128
    [n_types][N][N], N = n_eq + n_int, equivalent-surface unknowns first) and
    the box self block Z_o^self ([n_eq][n_eq], shared by every type).  Diagonally
    dominant interior and surface blocks with weak coupling, so that the
    resulting S = -(Z~ + Z_self)^-1 has norm about 0.5 like the direct S draws."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, 80, seed])))
    N = n_eq + n_int

    def cn(*shape):
        return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)

    Z = np.zeros((n_types, N, N), dtype=np.complex128)
    for t in range(n_types):
        Z[t, :n_eq, :n_eq] = 2.0 * np.eye(n_eq) + 0.25 * cn(n_eq, n_eq) / math.sqrt(n_eq)
        if n_int:
            c = 0.3 / math.sqrt(math.sqrt(n_eq * n_int))
            Z[t, :n_eq, n_eq:] = c * cn(n_eq, n_int)
            Z[t, n_eq:, :n_eq] = c * cn(n_int, n_eq)
            Z[t, n_eq:, n_eq:] = (1.0 + 0.5j) * np.eye(n_int) + 0.3 * cn(n_int, n_int) / math.sqrt(n_int)
    Zself = 0.2 * cn(n_eq, n_eq) / math.sqrt(n_eq)
    return Z, Zself
