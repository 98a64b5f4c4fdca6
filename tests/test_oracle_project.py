"""Pins for the oracle's projector P and backprojector P^T (eq. (2)'s
projection matrix; the P^T of the gradient in section 2.2).

  * a dense matrix built in numpy by an unclipped march of the whole
    source-to-pixel segment on the same sample grid must reproduce P x, and
    its transpose must reproduce P^T y (8^3 brute force);
  * line integrals through off-centre rotated uniform ellipsoids must match
    the analytic chord length times mu, at four gantry angles, with the
    discretisation error shrinking as voxels are halved;
  * an axis-aligned ray through a uniform box returns mu * n * h exactly;
  * translating the image by whole voxels equals translating source and
    detector by the same amount;
  * <P x, y> = <x, P^T y>.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1004_0014_amd import synth as S


# ---------------------------------------------------------------- helpers --
def _np_source_pixel(geom, iu, iv):
    """Independent restatement of the cone-beam geometry for the tests."""
    t = geom.angle
    R = np.array([[math.cos(t), -math.sin(t), 0.0], [math.sin(t), math.cos(t), 0.0], [0, 0, 1.0]])
    # at angle 0: source on -y, detector on +y, u along +x, v along +z
    s0 = np.array([0.0, -geom.sad, 0.0])
    u = (iu - (geom.nu - 1) / 2) * geom.du + geom.off_u
    v = (iv - (geom.nv - 1) / 2) * geom.dv + geom.off_v
    pix0 = np.array([u, geom.sdd - geom.sad, v])
    iso = np.asarray(geom.iso, float)
    return iso + R @ s0, iso + R @ pix0


def _dense_P(grid, geom):
    """Dense (M x N) system matrix: march every ray over the full segment
    [0, |pix - s|] at t = n * step with numpy trilinear weights, in-grid
    corners only (no clipping to the volume)."""
    N, M = grid.N, geom.nu * geom.nv
    A = np.zeros((M, N))
    nx, ny, nz = grid.n
    sp, org = np.array(grid.spacing), np.array(grid.origin)
    for iv in range(geom.nv):
        for iu in range(geom.nu):
            s, pix = _np_source_pixel(geom, iu, iv)
            L = np.linalg.norm(pix - s)
            d = (pix - s) / L
            n = np.arange(0, int(np.floor(L / geom.step)) + 1)
            pts = s[None, :] + (n * geom.step)[:, None] * d[None, :]
            q = (pts - org) / sp
            i0 = np.floor(q).astype(int)
            ph = q - i0
            row = iu + geom.nu * iv
            for c in range(2):
                for b in range(2):
                    for a in range(2):
                        ii, jj, kk = i0[:, 0] + a, i0[:, 1] + b, i0[:, 2] + c
                        wgt = ((ph[:, 0] if a else 1 - ph[:, 0]) * (ph[:, 1] if b else 1 - ph[:, 1])
                               * (ph[:, 2] if c else 1 - ph[:, 2]))
                        ok = (ii >= 0) & (jj >= 0) & (kk >= 0) & (ii < nx) & (jj < ny) & (kk < nz)
                        np.add.at(A[row], (ii[ok] + nx * (jj[ok] + ny * kk[ok])), wgt[ok] * geom.step)
    return A


def _chord(s, d, c, M):
    """Length of the line s + t d inside the ellipsoid (p-c)^T M (p-c) <= 1."""
    e = s - c
    A = d @ M @ d
    B = 2 * d @ M @ e
    Cc = e @ M @ e - 1
    disc = B * B - 4 * A * Cc
    return math.sqrt(disc) / A if disc > 0 else 0.0


def _rot(ax, ay, az):
    cx, sx, cy, sy, cz, sz = (math.cos(ax), math.sin(ax), math.cos(ay), math.sin(ay),
                              math.cos(az), math.sin(az))
    Rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
    Ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
    Rz = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]])
    return Rz @ Ry @ Rx


# ------------------------------------------------------------------ tests --
def test_geometry_matches_independent_restatement():
    geom = S.Geom(math.radians(37.0), nu=9, nv=7, du=1.3, dv=0.9, step=1.0,
                  off_u=0.4, off_v=-0.3, iso=(3.0, -2.0, 1.5))
    for iu, iv in [(0, 0), (8, 6), (4, 3), (2, 5)]:
        s, pix = oracle.source_pixel(geom, iu, iv)
        s2, pix2 = _np_source_pixel(geom, iu, iv)
        np.testing.assert_allclose(s, s2, atol=1e-12)
        np.testing.assert_allclose(pix, pix2, atol=1e-12)
    s, pix = oracle.source_pixel(geom, 4, 3)
    iso = np.array(geom.iso)
    assert abs(np.linalg.norm(s - iso) - geom.sad) < 1e-9


@pytest.mark.parametrize("angle_deg", [0.0, 33.0, 90.0, 211.0])
def test_bruteforce_8cube(angle_deg):
    g = S.Grid((8, 8, 8), (4.0, 4.0, 4.0))
    geom = S.Geom(math.radians(angle_deg), nu=12, nv=10, du=5.0, dv=5.0, step=1.7,
                  sad=100.0, sdd=150.0, off_u=0.9, off_v=-1.3, iso=(1.0, -2.0, 0.5))
    A = _dense_P(g, geom)
    x = S.seeded(10, g.shape)
    p = oracle.project(g, geom, x)
    np.testing.assert_allclose(p.ravel(), A @ x.ravel(), rtol=1e-13, atol=1e-13 * np.abs(A @ x.ravel()).max())
    y = S.seeded(11, (geom.nv, geom.nu))
    bp = oracle.backproject(g, geom, y)
    ref = A.T @ y.ravel()
    np.testing.assert_allclose(bp.ravel(), ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
    assert np.count_nonzero(A) > 1000    # the rays really cross the volume


def test_uniform_box_axis_aligned_ray_exact():
    g = S.Grid((64, 64, 64), (4.0, 4.0, 4.0))
    f = np.zeros(g.shape)
    f[8:56, 8:56, 8:56] = 0.02
    # central ray along +y through x = z = 0 (pixel centred on the axis)
    geom = S.Geom(0.0, nu=4, nv=4, du=1.0, dv=1.0, step=2.0, off_u=0.5, off_v=0.5)
    p = oracle.project(g, geom, f)
    assert abs(p[1, 1] - 0.02 * 48 * 4.0) < 1e-12
    # same at 90 degrees (ray along -x)
    geom90 = S.Geom(math.pi / 2, nu=4, nv=4, du=1.0, dv=1.0, step=2.0, off_u=0.5, off_v=0.5)
    p = oracle.project(g, geom90, f)
    assert abs(p[1, 1] - 0.02 * 48 * 4.0) < 1e-12


def _ellipsoid_case(n, h, angle):
    g = S.Grid((n, n, n), (h, h, h))
    centre = np.array([22.0, -15.0, 12.0])
    semi = np.array([70.0, 45.0, 55.0])
    R = _rot(0.3, -0.2, 0.5)
    M = R @ np.diag(semi ** -2) @ R.T
    mu = 0.02
    f = S.ellipsoid_volume(g, centre, semi, mu, rot=R, supersample=4)
    geom = S.Geom(angle, nu=64, nv=48, du=4.0, dv=4.0, step=h / 2)
    p = oracle.project(g, geom, f)
    exact = np.zeros_like(p)
    for iv in range(geom.nv):
        for iu in range(geom.nu):
            s, pix = _np_source_pixel(geom, iu, iv)
            d = (pix - s) / np.linalg.norm(pix - s)
            exact[iv, iu] = mu * _chord(s, d, centre, M)
    return p, exact


@pytest.mark.parametrize("angle_deg", [0.0, 30.0, 90.0, 200.0])
def test_ellipsoid_closed_form_chords(angle_deg):
    p, exact = _ellipsoid_case(64, 4.0, math.radians(angle_deg))
    err = np.linalg.norm(p - exact) / np.linalg.norm(exact)
    assert err < 4e-2, err      # measured 2.7-3.1e-2; halves with h (next test)
    # a mirrored or rotated geometry would fail badly: compare against flips
    for wrong in (exact[:, ::-1], exact[::-1, :]):
        assert np.linalg.norm(p - wrong) / np.linalg.norm(exact) > 0.2


def test_ellipsoid_error_shrinks_with_voxel_size():
    errs = []
    for n, h in [(32, 8.0), (64, 4.0), (128, 2.0)]:
        p, exact = _ellipsoid_case(n, h, math.radians(30.0))
        errs.append(np.linalg.norm(p - exact) / np.linalg.norm(exact))
    assert errs[1] < 0.6 * errs[0] and errs[2] < 0.6 * errs[1], errs


@pytest.mark.parametrize("c", [(2, -1, 3), (-3, 2, 0)])
def test_translation_equals_geometry_shift(c):
    g = S.Grid((40, 40, 32), (3.0, 3.0, 4.0))
    f0 = S.phantom(S.Grid((40, 40, 32), (3.0, 3.0, 4.0)), texture=0.05)
    # shrink the object away from the borders: keep a 4-voxel air margin
    f0[:4], f0[-4:], f0[:, :4], f0[:, -4:], f0[:, :, :4], f0[:, :, -4:] = 0, 0, 0, 0, 0, 0
    x = np.empty((3,) + g.shape)
    for a in range(3):
        x[a] = c[a] * g.spacing[a]
    f = oracle.warp(g, f0, x)
    for ang in (0.4, 2.2):
        geom = S.Geom(ang, nu=48, nv=40, du=3.0, dv=3.0, step=1.5)
        shift = tuple(c[a] * g.spacing[a] for a in range(3))
        geom_c = S.Geom(ang, nu=48, nv=40, du=3.0, dv=3.0, step=1.5, iso=shift)
        p1 = oracle.project(g, geom, f)
        p2 = oracle.project(g, geom_c, f0)
        np.testing.assert_allclose(p1, p2, rtol=0, atol=1e-11 * np.abs(p2).max())


def test_adjoint_identity():
    g = S.Grid((24, 22, 20), (2.0, 2.0, 2.5))
    geom = S.Geom(0.7, nu=40, nv=30, du=2.2, dv=2.2, step=1.0)
    x = S.seeded(3, g.shape)
    y = S.seeded(4, (geom.nv, geom.nu))
    lhs = np.vdot(oracle.project(g, geom, x), y)
    rhs = np.vdot(x, oracle.backproject(g, geom, y))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_ray_missing_volume_is_zero():
    g = S.Grid((8, 8, 8), (1.0, 1.0, 1.0))
    f = np.ones(g.shape)
    geom = S.Geom(0.0, nu=4, nv=4, du=1.0, dv=1.0, step=0.5, off_u=500.0)
    assert np.all(oracle.project(g, geom, f) == 0.0)
