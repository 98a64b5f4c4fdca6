"""Pins for the oracle's interpolation, warp, warp Jacobian and warp adjoint
(section 2.2: trilinear interpolation and a gradient consistent with it;
sections 2.2-2.3: the pull-back warp f(p) = f0(p + x(p))).

Each check is fixed by mathematics, not by re-running the oracle's formulas:
trilinear interpolation reproduces affine functions exactly, an integer
translation is an exact shift, the Jacobian matches finite differences away
from cell faces, and the adjoint satisfies <W a, b> = <a, W^T b>."""
import numpy as np
import pytest

import oracle
from paper_1004_0014_amd import synth as S

pytestmark = pytest.mark.filterwarnings("ignore")


def _affine_volume(grid, c0, gx, gy, gz):
    k, j, i = np.meshgrid(np.arange(grid.n[2]), np.arange(grid.n[1]), np.arange(grid.n[0]),
                          indexing="ij")
    return c0 + gx * i + gy * j + gz * k


def test_interp_reproduces_affine_inside():
    g = S.Grid((7, 6, 5), (1.0, 1.0, 1.0))
    F = _affine_volume(g, 0.3, 1.25, -0.5, 2.0)
    rng = np.random.default_rng(0)
    for _ in range(200):
        q = rng.uniform([0, 0, 0], [6, 5, 4])        # interior: all 8 corners in grid
        expect = 0.3 + 1.25 * q[0] - 0.5 * q[1] + 2.0 * q[2]
        assert abs(oracle.interp(F, g, q) - expect) < 1e-12
        np.testing.assert_allclose(oracle.interp_grad(F, g, q), [1.25, -0.5, 2.0], atol=1e-12)


def test_interp_grid_points_and_support():
    g = S.Grid((5, 4, 3), (1.0, 1.0, 1.0))
    F = S.seeded(11, g.shape) + 3.0
    for (i, j, k) in [(0, 0, 0), (4, 3, 2), (2, 1, 1)]:
        assert oracle.interp(F, g, [i, j, k]) == F[k, j, i]
    # zero (air) outside the grid; continuous at the support edge (-1 and n)
    assert oracle.interp(F, g, [-1.0, 1.0, 1.0]) == 0.0
    assert oracle.interp(F, g, [5.0, 1.0, 1.0]) == 0.0
    assert oracle.interp(F, g, [-1.5, 1.0, 1.0]) == 0.0
    assert abs(oracle.interp(F, g, [-1.0 + 1e-9, 1.0, 1.0])) < 1e-8
    # halfway to air: half the edge voxel value
    assert abs(oracle.interp(F, g, [-0.5, 1.0, 1.0]) - 0.5 * F[1, 1, 0]) < 1e-14
    # the single-voxel "hat" along x: T = 1 - |q - i| for a delta volume
    D = np.zeros(g.shape)
    D[1, 2, 2] = 1.0
    for qx in np.linspace(0.6, 3.4, 15):
        assert abs(oracle.interp(D, g, [qx, 2.0, 1.0]) - max(0.0, 1 - abs(qx - 2.0))) < 1e-14


def test_interp_grad_matches_fd_off_faces():
    g = S.Grid((6, 6, 6), (1.0, 1.0, 1.0))
    F = S.seeded(3, g.shape)
    rng = np.random.default_rng(1)
    h = 1e-6
    for _ in range(50):
        q = np.floor(rng.uniform(-1, 5, 3)) + rng.uniform(0.1, 0.9, 3)   # off cell faces
        d = oracle.interp_grad(F, g, q)
        for a in range(3):
            e = np.zeros(3); e[a] = h
            fd = (oracle.interp(F, g, q + e) - oracle.interp(F, g, q - e)) / (2 * h)
            assert abs(fd - d[a]) < 1e-7


def test_compose_is_mean_plus_Uw():
    g = S.Grid((4, 3, 2), (1.0, 2.0, 3.0))
    mean = S.seeded(1, (3,) + g.shape)
    U = S.seeded(2, (3, 3) + g.shape)
    w = np.array([0.5, -2.0, 3.0])
    x = oracle.compose(g, mean, U, w)
    # element-wise definition written as a tensor contraction
    assert np.allclose(x, mean + np.einsum("k,kazyx->azyx", w, U), atol=1e-14)


def test_identity_warp_is_bitwise():
    g = S.grid_for("tiny")
    f0 = S.phantom(g)
    f = oracle.warp(g, f0, np.zeros((3,) + g.shape))
    assert np.array_equal(f, f0)


@pytest.mark.parametrize("c", [(2, -1, 3), (-3, 0, 1), (0, 2, -2)])
def test_integer_translation_is_exact_shift(c):
    g = S.Grid((20, 18, 16), (1.875, 1.875, 2.5))
    f0 = S.seeded(5, g.shape)
    x = np.empty((3,) + g.shape)
    for a in range(3):
        x[a] = c[a] * g.spacing[a]
    f = oracle.warp(g, f0, x)
    nz, ny, nx = g.shape
    expect = np.zeros(g.shape)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                ii, jj, kk = i + c[0], j + c[1], k + c[2]
                if 0 <= ii < nx and 0 <= jj < ny and 0 <= kk < nz:
                    expect[k, j, i] = f0[kk, jj, ii]
    assert np.array_equal(f, expect)


def test_subvoxel_translation_of_affine_image():
    g = S.Grid((10, 9, 8), (2.0, 1.5, 2.5))
    f0 = _affine_volume(g, 1.0, 0.2, -0.1, 0.3)
    c_mm = np.array([0.7, -0.4, 1.1])
    x = np.empty((3,) + g.shape)
    for a in range(3):
        x[a] = c_mm[a]
    f = oracle.warp(g, f0, x)
    shift = c_mm / np.array(g.spacing)
    expect = f0 + 0.2 * shift[0] - 0.1 * shift[1] + 0.3 * shift[2]
    # interior voxels whose displaced point keeps all 8 corners in the grid
    inner = (slice(0, 7), slice(1, 8), slice(0, 9))
    np.testing.assert_allclose(f[inner], expect[inner], atol=1e-12)


def test_warp_jacobian_matches_fd():
    g = S.Grid((16, 14, 12), (3.0, 2.0, 2.5))
    f0 = S.phantom(g, texture=0.05)
    rng = np.random.default_rng(7)
    x = rng.uniform(-4, 4, (3,) + g.shape)
    G = oracle.warp_jacobian(g, f0, x)
    h = 1e-7
    for a in range(3):
        e = np.zeros((3,) + g.shape)
        e[a] = h
        fd = (oracle.warp(g, f0, x + e) - oracle.warp(g, f0, x - e)) / (2 * h)
        # skip voxels whose displaced point lies within 1e-5 of a cell face
        q = x[a] / g.spacing[a]
        frac = np.abs(q - np.round(q))
        ok = frac > 1e-5
        assert np.abs(fd[ok] - G[a][ok]).max() < 1e-6


def test_warp_adjoint_identity():
    g = S.Grid((11, 10, 9), (2.0, 2.0, 2.0))
    rng = np.random.default_rng(3)
    x = rng.uniform(-3, 3, (3,) + g.shape)
    a = S.seeded(4, g.shape)
    b = S.seeded(5, g.shape)
    lhs = np.vdot(oracle.warp(g, a, x), b)
    rhs = np.vdot(a, oracle.warp_adjoint(g, x, b))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + np.abs(a).sum())
