"""Seeded synthetic inputs shared by the FP64 oracle tests, the GPU tests and the
benchmark.

This module builds inputs only: voxel grids, an ellipsoid-thorax phantom, an
analytic breathing deformation, the PCA motion model trained on it, measured
projection geometry and seeded random arrays.  It holds none of the
reconstruction arithmetic (deformation composition, warping, projection, cost,
gradient, solver, localisation); those live separately in the oracle and in the
HIP library, and both receive what this module makes as plain arrays.

Paper basis (Li et al., "Real-time volumetric image reconstruction and 3D tumor
localization based on a single x-ray projection image"):
  * PCA motion model, eq. (1) in section 2.1: x(t) ~ mean + sum_k u_k w_k(t),
    trained on the N-1 DVFs between a reference phase and the other phases.
  * Section 3: 10 breathing phases, end-of-exhale reference, 9 DVFs, K = 3,
    4 s period, test motion at 1.5x the training amplitude, 360 projections
    over one gantry rotation, a 40x30 cm imager.
The paper's NCAT phantom and demons-registered DVFs are not available; the
ellipsoid thorax and the analytic DVF below stand in for them (shapes and
motion statistics as in section 3, all constants are this project's choices).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Grid", "Geom", "phantom", "ellipsoid_volume", "dvf_patterns",
    "phase_coeffs", "analytic_dvf", "PCAModel", "pca_model", "truth_w",
    "tumor_center", "CONFIGS", "config", "seeded", "geom_for",
]


# ---------------------------------------------------------------- grids ----
@dataclass
class Grid:
    """Voxel grid: n = (nx, ny, nz), spacing in mm, origin = centre of voxel
    (0,0,0) in mm.  Arrays are stored [nz][ny][nx] (x fastest).  The default
    origin puts the volume centre at (0,0,0)."""
    n: tuple
    spacing: tuple
    origin: tuple = None

    def __post_init__(self):
        self.n = tuple(int(v) for v in self.n)
        self.spacing = tuple(float(v) for v in self.spacing)
        if self.origin is None:
            self.origin = tuple(-0.5 * (n - 1) * s for n, s in zip(self.n, self.spacing))
        self.origin = tuple(float(v) for v in self.origin)

    @property
    def N(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]

    @property
    def shape(self):  # numpy shape, z slowest
        return (self.n[2], self.n[1], self.n[0])

    @property
    def fov(self):
        return tuple(n * s for n, s in zip(self.n, self.spacing))

    def axes(self):
        """World coordinates (mm) of voxel centres along x, y, z."""
        return [self.origin[a] + self.spacing[a] * np.arange(self.n[a]) for a in range(3)]

    def mesh(self):
        """Broadcastable (z,y,x)-shaped world coordinate arrays px, py, pz."""
        x, y, z = self.axes()
        return x[None, None, :], y[None, :, None], z[:, None, None]


@dataclass
class Geom:
    """Cone-beam geometry of one projection (mm, radians).

    Source s = iso + (SAD sin t, -SAD cos t, 0); detector centre
    c = iso + (-(SDD-SAD) sin t, (SDD-SAD) cos t, 0); detector axes
    e_u = (cos t, sin t, 0), e_v = (0, 0, 1); pixel (iu, iv) centre
    c + ((iu-(nu-1)/2) du + off_u) e_u + ((iv-(nv-1)/2) dv + off_v) e_v.
    Pixel pitch is measured at the detector plane.  Ray samples sit at
    t = n*step from the source."""
    angle: float
    nu: int
    nv: int
    du: float
    dv: float
    step: float
    sad: float = 1000.0
    sdd: float = 1500.0
    off_u: float = 0.0
    off_v: float = 0.0
    iso: tuple = (0.0, 0.0, 0.0)

    def with_angle(self, angle):
        return Geom(angle, self.nu, self.nv, self.du, self.dv, self.step, self.sad,
                    self.sdd, self.off_u, self.off_v, tuple(self.iso))


# -------------------------------------------------------------- phantom ----
def ellipsoid_volume(grid: Grid, centre, semi, mu, rot=None, supersample=1):
    """Attenuation volume of one uniform ellipsoid (p-c)^T M (p-c) <= 1,
    M = R diag(semi^-2) R^T, voxelised at voxel centres, or as the mean over
    supersample^3 sub-points per voxel."""
    centre = np.asarray(centre, float)
    semi = np.asarray(semi, float)
    R = np.eye(3) if rot is None else np.asarray(rot, float)
    M = R @ np.diag(semi ** -2) @ R.T
    out = np.zeros(grid.shape)
    ss = int(supersample)
    offs = (np.arange(ss) + 0.5) / ss - 0.5
    x, y, z = grid.axes()
    for oz in offs:
        for oy in offs:
            for ox in offs:
                dx = (x + ox * grid.spacing[0] - centre[0])[None, None, :]
                dy = (y + oy * grid.spacing[1] - centre[1])[None, :, None]
                dz = (z + oz * grid.spacing[2] - centre[2])[:, None, None]
                q = (M[0, 0] * dx * dx + M[1, 1] * dy * dy + M[2, 2] * dz * dz
                     + 2 * M[0, 1] * dx * dy + 2 * M[0, 2] * dx * dz + 2 * M[1, 2] * dy * dz)
                out += (q <= 1.0)
    return out * (mu / ss ** 3)


def tumor_center(grid: Grid):
    """Tumour centre (mm): centre of the right lung (-x side) shifted
    inferiorly by 0.10 of the SI field of view."""
    L = grid.fov
    return np.array([-0.17 * L[0], 0.02 * L[1], 0.05 * L[2] - 0.10 * L[2]])


def phantom(grid: Grid, seed: int = 0, texture: float = 0.05, dtype=np.float64):
    """Ellipsoid thorax (attenuation in 1/mm), painter's order body -> lungs ->
    tumour: body 0.02/mm with semi-axes (0.40, 0.30, 0.60) x FOV; two lungs
    0.004/mm centred at (+-0.17, 0.02, 0.05) x FOV with semi-axes
    (0.13, 0.20, 0.30) x FOV; a 10 mm radius tumour 0.02/mm.  Texture: i.i.d.
    N(0,1) per voxel (numpy PCG64 seeded by `seed`), Gaussian-smoothed with
    sigma = 1 voxel, rescaled to unit variance, applied as mu (1 + texture z)
    wherever mu > 0."""
    L = np.asarray(grid.fov)
    px, py, pz = grid.mesh()
    mu = np.zeros(grid.shape)

    def inside(c, s):
        return (((px - c[0]) / s[0]) ** 2 + ((py - c[1]) / s[1]) ** 2
                + ((pz - c[2]) / s[2]) ** 2) <= 1.0

    mu[inside((0, 0, 0), np.array([0.40, 0.30, 0.60]) * L)] = 0.02
    for sx in (+1, -1):
        c = np.array([sx * 0.17, 0.02, 0.05]) * L
        mu[inside(c, np.array([0.13, 0.20, 0.30]) * L)] = 0.004
    tc = tumor_center(grid)
    mu[inside(tc, (10.0, 10.0, 10.0))] = 0.02
    if texture:
        from scipy.ndimage import gaussian_filter
        rng = np.random.default_rng(seed)
        z = rng.standard_normal(grid.shape, dtype=np.float32)
        z = gaussian_filter(z, sigma=1.0, mode="constant")
        z = z / z.std()
        mu = mu * (1.0 + texture * z)
    return mu.astype(dtype)


# ------------------------------------------------------------ motion -------
# Analytic pull-back DVF (mm) at breathing phase phi (eq. (1)'s x(t) stand-in):
#   x(p, phi) = A g(p) sum_i amp_i c_i(phi) e_i(p)
# g(p) = exp(-(p_x / (0.35 L_x))^2) decays laterally; pattern i is one fixed
# spatial field times one scalar function of phase, so the field has rank R and
# PCA with K = R recovers its span exactly.
_AMP = 10.0
_PATTERN_AMPS = (1.0, 0.3, 0.15, 0.1, 0.08)


def phase_coeffs(phi, R: int):
    """c_i(phi), i < R: SI breathing (1-cos)/2, hysteresis sin, then the next
    harmonics (1-cos 2phi)/2, sin 2phi, (1-cos 3phi)/2."""
    phi = np.asarray(phi, float)
    c = [(1 - np.cos(phi)) / 2, np.sin(phi), (1 - np.cos(2 * phi)) / 2,
         np.sin(2 * phi), (1 - np.cos(3 * phi)) / 2]
    if not 1 <= R <= 5:
        raise ValueError("rank must be in 1..5")
    return np.array(c[:R])


def dvf_patterns(grid: Grid, R: int, dtype=np.float64):
    """Spatial patterns [R][3][nz][ny][nx] in mm (amplitudes folded in)."""
    L = grid.fov
    px, py, pz = grid.mesh()
    g = np.exp(-(px / (0.35 * L[0])) ** 2) * np.ones(grid.shape)
    hz = pz / L[2] * np.ones(grid.shape)          # SI gradient, zero-mean
    sx = px / L[0] * np.ones(grid.shape)          # LR gradient
    out = np.zeros((R, 3) + grid.shape, dtype=dtype)
    comps = [(2, g), (1, g), (2, g * hz), (1, g * hz), (0, g * sx)]
    for i in range(R):
        ax, field_ = comps[i]
        out[i, ax] = _AMP * _PATTERN_AMPS[i] * field_
    return out


def analytic_dvf(grid: Grid, phi: float, R: int = 3, scale: float = 1.0):
    """x(p, phi) [3][nz][ny][nx] (mm); `scale` multiplies the amplitude (1.5 for
    the test motion of section 3)."""
    P = dvf_patterns(grid, R)
    c = phase_coeffs(phi, R) * scale
    return np.tensordot(c, P, axes=(0, 0))


# --------------------------------------------------------------- PCA -------
def training_dvfs(grid: Grid, R: int, n_phases: int = 10, dtype=np.float32, patterns=None):
    """The training DVFs of the PCA model below: x(p, phi_j) at the phases
    phi_j = 2 pi j / n_phases, j = 1..n_phases-1, as [n_phases-1][3][nz][ny][nx]."""
    P = dvf_patterns(grid, R) if patterns is None else patterns
    phis = 2 * np.pi * np.arange(1, n_phases) / n_phases
    return np.tensordot(phase_coeffs(phis, R).T, P, axes=(1, 0)).astype(dtype)


@dataclass
class PCAModel:
    grid: Grid
    K: int
    R: int
    mean: np.ndarray            # [3][nz][ny][nx] float64
    U: np.ndarray               # [K][3][nz][ny][nx] float64, unit norm columns
    sing: np.ndarray            # singular values of the centred training matrix
    w_train: np.ndarray         # [9][K] training coefficients
    Z: np.ndarray = field(repr=False, default=None)   # U = sum_i Z[i,k] P_i
    Q: np.ndarray = field(repr=False, default=None)   # pattern Gram matrix
    cbar: np.ndarray = field(repr=False, default=None)

    @property
    def step0(self) -> float:
        """Half the RMS norm of the training coefficient vectors: the size of
        the first trial step of the line search."""
        return 0.5 * float(np.sqrt(np.mean(np.sum(self.w_train ** 2, axis=1))))


def _sign_index(u):
    """Index of the first entry (storage order) whose magnitude is within 1e-5
    (relative) of the largest; symmetric motion patterns have several such
    entries, and the tolerance sits well above FP32 rounding."""
    a = np.abs(u)
    return int(np.flatnonzero(a >= (1 - 1e-5) * a.max())[0])


def pca_model(grid: Grid, K: int, R: int | None = None, n_phases: int = 10,
              patterns=None) -> PCAModel:
    """PCA motion model (eq. (1), section 2.1; section 3): training DVFs at
    phases 2 pi j / n_phases, j = 1..n_phases-1 (j = 0 is the end-of-exhale
    reference with x = 0), mean = their average, U = the K leading left
    singular vectors of the centred 3N x (n_phases-1) matrix, each flipped so
    that its largest-magnitude entry (the first, within 1e-5) is positive.

    Because every training DVF is X = P C (patterns P, coefficients C), the
    SVD is taken exactly through the R x R pattern Gram matrix Q = P^T P:
    with Q = L L^T, X = (P L^-T)(L^T C) and P L^-T has orthonormal columns."""
    R = K if R is None else R
    if K > R:
        raise ValueError("K must not exceed the motion rank")
    P = dvf_patterns(grid, R) if patterns is None else patterns
    Pf = P.reshape(R, -1)
    phis = 2 * np.pi * np.arange(1, n_phases) / n_phases
    C = phase_coeffs(phis, R)                       # [R][9]
    cbar = C.mean(axis=1)
    Cc = C - cbar[:, None]
    Q = Pf @ Pf.T
    Lc = np.linalg.cholesky(Q)
    A, sing, _ = np.linalg.svd(Lc.T @ Cc, full_matrices=False)
    Z = np.linalg.solve(Lc.T, A)[:, :K]             # U = P Z
    U = (Z.T @ Pf)                                  # [K][3N]
    for k in range(K):
        j = _sign_index(U[k])
        if U[k, j] < 0:
            U[k] *= -1.0
            Z[:, k] *= -1.0
    mean = (cbar @ Pf).reshape((3,) + grid.shape)
    w_train = (Cc.T @ Q @ Z)                        # [9][K] = (X^T U)
    return PCAModel(grid, K, R, mean, U.reshape((K, 3) + grid.shape), sing, w_train, Z, Q, cbar)


def truth_w(model: PCAModel, phi: float, scale: float = 1.5):
    """w* = U^T (scale * x(phi) - mean): exact when K equals the motion rank,
    because the test DVF then lies in the span of U."""
    c = phase_coeffs(phi, model.R) * scale - model.cbar
    return model.Z.T @ model.Q @ c


# ------------------------------------------------------------- configs ----
CONFIGS = {
    # tiny FP64 case: 64^3 at 4 mm, 128x96 detector at 1.6 mm, 30 deg
    "tiny": dict(n=(64, 64, 64), spacing=(4.0, 4.0, 4.0), K=3, nu=128, nv=96,
               du=1.6, dv=1.6, step=2.0, angles=[math.radians(30.0)], max_iter=30),
    # paper-scale FP32: 256x256x100 at 1.875x1.875x2.5 mm, 512x384 at 0.776 mm
    "paper": dict(n=(256, 256, 100), spacing=(1.875, 1.875, 2.5), K=3, nu=512, nv=384,
               du=0.776, dv=0.776, step=0.9375,
               angles=[math.radians(i) for i in range(360)], rate_hz=11.0, max_iter=50),
    # differentiation: 128^3 at 3 mm, 256x192 at 1.552 mm, K in {3, 5}
    "diff": dict(n=(128, 128, 128), spacing=(3.0, 3.0, 3.0), K=3, nu=256, nv=192,
               du=1.552, dv=1.552, step=1.5, n_angles=8, angle_seed=2),
    # precision: 256x256x128, K = 4, 16-bit storage
    "precision": dict(n=(256, 256, 128), spacing=(1.875, 1.875, 2.5), K=4, nu=512, nv=384,
               du=0.776, dv=0.776, step=0.9375,
               angles=[math.radians(i) for i in range(360)], rate_hz=11.0, max_iter=50),
}


def config(name: str) -> dict:
    cfg = dict(CONFIGS[name])
    if name == "diff":
        rng = np.random.default_rng(cfg["angle_seed"])
        cfg["angles"] = list(rng.uniform(0, 2 * np.pi, cfg["n_angles"]))
    return cfg


def grid_for(name: str) -> Grid:
    c = CONFIGS[name]
    return Grid(c["n"], c["spacing"])


def geom_for(name: str, angle: float | None = None) -> Geom:
    c = config(name)
    a = c["angles"][0] if angle is None else angle
    return Geom(a, c["nu"], c["nv"], c["du"], c["dv"], c["step"])


def seeded(seed: int, shape, kind="normal", dtype=np.float64):
    """Seeded random array (numpy PCG64)."""
    rng = np.random.default_rng(seed)
    if kind == "normal":
        return rng.standard_normal(shape).astype(dtype)
    if kind == "uniform":
        return rng.uniform(0.0, 1.0, shape).astype(dtype)
    raise ValueError(kind)


def breathing_phase(t_s: float, period_s: float = 4.0) -> float:
    """Breathing phase (rad) at time t for a 4 s period (section 3)."""
    return 2 * np.pi * (t_s / period_s)
