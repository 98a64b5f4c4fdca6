"""Pins for the oracle's cost, gradient, step 2, solver and localisation
(section 2.2, eqs. (2)-(4) and the gradient formula; section 2.3).

  * dJ/dw matches central finite differences of the cost (h = 1e-3 |w| + 1e-6),
  * the adjoint gradient equals the tangent form 2 <r, P (G . u_k)>,
  * dJ/df0 = W^T P^T 2r matches finite differences on seeded voxels,
  * step 2 equals a least-squares fit and zeroes dJ/da and dJ/db,
  * J never increases over the iterations (section 2.2),
  * an inverse-crime projection is fitted back to the closed-form w*,
    and an affine intensity map y = alpha P f + beta gives a = 1/alpha,
  * the fixed point inverts constant and affine DVFs exactly.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1004_0014_amd import synth as S


@pytest.fixture(scope="module")
def small():
    g = S.Grid((32, 32, 32), (6.0, 6.0, 6.0))
    f0 = S.phantom(g)
    m = S.pca_model(g, 3)
    geom = S.Geom(0.9, nu=64, nv=48, du=3.1, dv=3.1, step=3.0)
    return g, f0, m, geom


def _measure(g, f0, m, geom, w):
    x = oracle.compose(g, m.mean, m.U, w)
    return oracle.project(g, geom, oracle.warp(g, f0, x))


def test_gradient_matches_central_fd(small):
    g, f0, m, geom = small
    w_true = S.truth_w(m, 2.1)
    y = _measure(g, f0, m, geom, w_true)
    w = w_true * np.array([0.8, 1.1, 0.7]) + np.array([35.0, -20.0, 10.0])
    a, b = 1.02, -0.03
    J, grad = oracle.cost_grad(g, geom, f0, m.mean, m.U, w, y, a, b)
    for k in range(3):
        # the prescribed step may carry a sample point across a cell face (a
        # kink of the trilinear interpolant): loose bound; a 10x smaller step
        # stays off the kinks here and must agree to rounding
        for rel, tol in ((1e-3, 2e-3), (1e-4, 1e-8)):
            h = rel * abs(w[k]) + 1e-6
            e = np.zeros(3); e[k] = h
            Jp, _ = oracle.cost_grad(g, geom, f0, m.mean, m.U, w + e, y, a, b)
            Jm, _ = oracle.cost_grad(g, geom, f0, m.mean, m.U, w - e, y, a, b)
            fd = (Jp - Jm) / (2 * h)
            assert abs(fd - grad[k]) <= tol * abs(grad[k]), (k, rel, fd, grad[k])


def test_gradient_tangent_equals_adjoint(small):
    g, f0, m, geom = small
    w = S.truth_w(m, 1.0) * 0.6
    y = _measure(g, f0, m, geom, S.truth_w(m, 1.0))
    a, b = 0.97, 0.01
    J, grad, p = oracle.cost_grad(g, geom, f0, m.mean, m.U, w, y, a, b, want_p=True)
    x = oracle.compose(g, m.mean, m.U, w)
    Gj = oracle.warp_jacobian(g, f0, x)
    r = p - a * y - b
    assert abs(J - np.sum(r * r)) <= 1e-12 * J
    for k in range(3):
        h_k = np.sum(Gj * m.U[k], axis=0)              # G . u_k per voxel
        tang = 2 * np.vdot(r, oracle.project(g, geom, h_k))
        assert abs(tang - grad[k]) <= 1e-10 * np.abs(grad).max()


def test_gradient_wrt_reference_image_fd(small):
    g, f0, m, geom = small
    w = S.truth_w(m, 0.5)
    y = _measure(g, f0, m, geom, S.truth_w(m, 2.5))
    a, b = 1.0, 0.0
    x = oracle.compose(g, m.mean, m.U, w)
    p = oracle.project(g, geom, oracle.warp(g, f0, x))
    r = p - a * y - b
    df0 = oracle.warp_adjoint(g, x, oracle.backproject(g, geom, 2 * r))
    rng = np.random.default_rng(3)
    flat = np.flatnonzero(np.abs(df0.ravel()) > 1e-3 * np.abs(df0).max())
    for idx in rng.choice(flat, 6, replace=False):
        h = 1e-4
        fp = f0.copy().ravel(); fp[idx] += h
        fm = f0.copy().ravel(); fm[idx] -= h
        Jp = oracle.cost(oracle.project(g, geom, oracle.warp(g, fp.reshape(g.shape), x)), y, a, b)
        Jm = oracle.cost(oracle.project(g, geom, oracle.warp(g, fm.reshape(g.shape), x)), y, a, b)
        fd = (Jp - Jm) / (2 * h)
        # J is quadratic in f0, so central differences are exact up to rounding
        assert abs(fd - df0.ravel()[idx]) <= 1e-6 * abs(df0.ravel()[idx]) + 1e-9


def test_step2_is_least_squares_and_stationary():
    rng = np.random.default_rng(0)
    y = rng.uniform(0.5, 2.0, 300)
    p = 1.7 * y + 0.3 + 0.05 * rng.standard_normal(300)
    a, b = oracle.step2(oracle.regression_sums(y, p))
    Y = np.stack([y, np.ones_like(y)], 1)
    ref = np.linalg.lstsq(Y, p, rcond=None)[0]
    assert abs(a - ref[0]) < 1e-12 and abs(b - ref[1]) < 1e-12
    r = p - a * y - b
    assert abs(np.sum(r * y)) < 1e-10 and abs(np.sum(r)) < 1e-10    # dJ/da = dJ/db = 0


def test_step2_degenerate_constant_y():
    y = np.full(50, 3.0)
    p = np.linspace(0, 1, 50)
    a, b = oracle.step2(oracle.regression_sums(y, p))
    assert a == 0.0 and abs(b - p.mean()) < 1e-14


def test_inverse_crime_recovery_and_monotone(small):
    g, f0, m, geom = small
    w_true = S.truth_w(m, 2.6)
    y = _measure(g, f0, m, geom, w_true)
    opts = oracle.SolveOpts(max_iter=150, step0=m.step0, eps_g=1e-7)
    w, (a, b), st, Jh = oracle.solve(g, geom, f0, m.mean, m.U, y, np.zeros(3), opts)
    assert np.all(np.diff(Jh) <= 0.0), Jh          # J never increases
    assert st["J"] < 1e-6 * st["J0"]
    assert np.linalg.norm(w - w_true) < 1e-3 * np.linalg.norm(w_true), (w, w_true)
    assert abs(a - 1) < 1e-4 and abs(b) < 1e-3


def test_affine_intensity_map_recovered(small):
    g, f0, m, geom = small
    w_true = S.truth_w(m, 1.7)
    alpha, beta = 2.5, 0.4
    y = (_measure(g, f0, m, geom, w_true) - beta) / alpha    # so that P f = alpha y + beta
    opts = oracle.SolveOpts(max_iter=150, step0=m.step0, eps_g=1e-7)
    w, (a, b), st, Jh = oracle.solve(g, geom, f0, m.mean, m.U, y, np.zeros(3), opts)
    assert abs(a - alpha) < 1e-3 * alpha and abs(b - beta) < 1e-2
    assert np.linalg.norm(w - w_true) < 2e-3 * np.linalg.norm(w_true)


def test_fixed_step_mode_is_plain_gradient_descent(small):
    g, f0, m, geom = small
    y = _measure(g, f0, m, geom, S.truth_w(m, 2.0))
    mu = 2e4
    opts = oracle.SolveOpts(max_iter=2, fixed_mu=mu, eps_g=0.0)
    w, ab, st, Jh = oracle.solve(g, geom, f0, m.mean, m.U, y, np.zeros(3), opts)
    # replay by hand: step 2, gradient, step, step 2, gradient, step
    wr = np.zeros(3)
    for _ in range(2):
        p = _measure(g, f0, m, geom, wr)
        a_, b_ = oracle.step2(oracle.regression_sums(y, p))
        _, gr = oracle.cost_grad(g, geom, f0, m.mean, m.U, wr, y, a_, b_)
        wr = wr - mu * gr
    np.testing.assert_allclose(w, wr, rtol=1e-12)
    assert st["iterations"] == 2 and st["trials"] == 2


def test_line_search_on_exact_quadratic_is_block_coordinate_descent():
    """A reference image linear in z, warped by one mode that vanishes near the
    grid faces, is reproduced exactly by trilinear interpolation, so P f is
    affine in w and J(w, a, b) is an exact quadratic.  Along a line it is then
    exactly phi(mu) = J - |g|^2 mu + c mu^2, so from the second iteration on
    the first Armijo trial is the exact line minimiser 1 / (2 |P h|^2): no
    trial is rejected and the iterates are those of block-coordinate descent
    (exact minimisation in w, then in (a, b)), computed here from p(0) and
    q = p(1) - p(0) alone."""
    g = S.Grid((20, 18, 22), (5.0, 5.0, 5.0))
    nz, ny, nx = g.shape
    k = np.arange(nz)[:, None, None] * np.ones((nz, ny, nx))
    f0 = 0.01 + 0.002 * k
    bump = lambda n: np.where((np.arange(n) >= 3) & (np.arange(n) <= n - 4),
                              np.sin(np.pi * (np.arange(n) - 3) / (n - 7)) ** 2, 0.0)
    U = np.zeros((1, 3) + g.shape)
    U[0, 2] = 4.0 * bump(nz)[:, None, None] * bump(ny)[None, :, None] * bump(nx)[None, None, :]
    mean = np.zeros((3,) + g.shape)
    geom = S.Geom(0.4, nu=40, nv=36, du=4.0, dv=4.0, step=2.5)
    proj = lambda w: oracle.project(g, geom, oracle.warp(g, f0, oracle.compose(g, mean, U, [w])))
    p0 = proj(0.0)
    q = proj(1.0) - p0
    y = (proj(0.37) - 0.002) / 1.7
    Y = np.stack([y.ravel(), np.ones(y.size)], axis=1)
    ab_of = lambda w: np.linalg.lstsq(Y, (p0 + w * q).ravel(), rcond=None)[0]
    qq = float(np.sum(q * q))
    mu_star = 1.0 / (2.0 * qq)
    a, b = ab_of(0.0)
    g0 = 2.0 * float(np.sum(q * (p0 - a * y - b)))
    # model iterates: a 0.7 mu* first step, then exact line minimisation
    ws, w = [], 0.0
    for n in range(5):
        grad = 2.0 * float(np.sum(q * (p0 + w * q - a * y - b)))
        w = w - (0.7 if n == 0 else 1.0) * mu_star * grad
        a, b = ab_of(w)
        ws.append((w, a, b))
    for N in (1, 2, 3, 5):
        opts = oracle.SolveOpts(max_iter=N, step0=0.7 * mu_star * abs(g0), eps_g=0.0, step_rule=1)
        w, (a, b), st, _ = oracle.solve(g, geom, f0, mean, U, y, [0.0], opts)
        assert st["iterations"] == N and st["trials"] == N
        np.testing.assert_allclose([w[0], a, b], ws[N - 1], rtol=1e-7, atol=1e-12)
    assert abs(ws[-1][0] - 0.37) < 1e-3
    # a given first step size: mu0 = mu* makes every step the exact line
    # minimiser, and the solver reports mu* as its next step size
    for N in (1, 3):
        opts = oracle.SolveOpts(max_iter=N, step0=1.0, eps_g=0.0, mu0=mu_star, step_rule=1)
        wo, (ao, bo), st, _ = oracle.solve(g, geom, f0, mean, U, y, [0.0], opts)
        wm, am, bm = 0.0, *ab_of(0.0)
        for n in range(N):
            grad = 2.0 * float(np.sum(q * (p0 + wm * q - am * y - bm)))
            wm = wm - mu_star * grad
            am, bm = ab_of(wm)
        assert st["trials"] == N
        np.testing.assert_allclose([wo[0], ao, bo], [wm, am, bm], rtol=1e-7, atol=1e-12)
        assert abs(st["mu"] - mu_star) <= 1e-6 * mu_star


@pytest.mark.parametrize("rule", [0, 1])
def test_solver_steps_on_exact_quadratic_two_modes(rule):
    """The same exact quadratic with two modes (both z displacements that
    vanish near the faces, of a z-linear image): P f = p0 + w_0 q_0 + w_1 q_1
    exactly.  A loop written here from the algorithm's statement (Armijo's
    sufficient decrease with backtracking by beta, step 2 by least squares,
    the first trial of a later line from the secant s.y / y.y or, for rule 1
    or s.y <= 0, from the quadratic through the last line) on that affine map
    alone reproduces the oracle's iterates, trial counts and next step."""
    g = S.Grid((20, 18, 22), (5.0, 5.0, 5.0))
    nz, ny, nx = g.shape
    k = np.arange(nz)[:, None, None] * np.ones((nz, ny, nx))
    f0 = 0.01 + 0.002 * k
    bump = lambda n, e: np.where((np.arange(n) >= 3) & (np.arange(n) <= n - 4),
                                 np.sin(np.pi * (np.arange(n) - 3) / (n - 7)) ** e, 0.0)
    U = np.zeros((2, 3) + g.shape)
    U[0, 2] = 4.0 * bump(nz, 2)[:, None, None] * bump(ny, 2)[None, :, None] * bump(nx, 2)[None, None, :]
    U[1, 2] = 3.0 * bump(nz, 4)[:, None, None] * bump(ny, 2)[None, :, None] * bump(nx, 6)[None, None, :]
    mean = np.zeros((3,) + g.shape)
    geom = S.Geom(0.4, nu=40, nv=36, du=4.0, dv=4.0, step=2.5)
    proj = lambda w: oracle.project(g, geom, oracle.warp(g, f0, oracle.compose(g, mean, U, w)))
    p0 = proj([0.0, 0.0])
    q = [proj([1.0, 0.0]) - p0, proj([0.0, 1.0]) - p0]
    y = (proj([0.37, -0.21]) - 0.002) / 1.7
    Y = np.stack([y.ravel(), np.ones(y.size)], axis=1)
    pw = lambda w: p0 + w[0] * q[0] + w[1] * q[1]
    ab_of = lambda w: np.linalg.lstsq(Y, pw(w).ravel(), rcond=None)[0]
    Jf = lambda w, a, b: float(np.sum((pw(w) - a * y - b) ** 2))
    gf = lambda w, a, b: np.array([2.0 * float(np.sum(qk * (pw(w) - a * y - b))) for qk in q])
    sigma, beta, step0 = 1e-4, 0.5, 0.05

    def model(N):
        w = np.zeros(2)
        a, b = ab_of(w)
        J, gr = Jf(w, a, b), gf(w, a, b)
        mu = step0 / np.linalg.norm(gr)
        trials = 0
        for _ in range(N):
            while True:
                wt = w - mu * gr
                Jt = Jf(wt, a, b)
                trials += 1
                if Jt <= J - sigma * mu * float(gr @ gr):
                    break
                mu *= beta
            J_line, g2 = J, float(gr @ gr)
            s, g_old = wt - w, gr
            w = wt
            a, b = ab_of(w)
            J, gr = Jf(w, a, b), gf(w, a, b)
            yv = gr - g_old
            if rule == 0 and s @ yv > 0 and yv @ yv > 0:
                mu = float(s @ yv) / float(yv @ yv)
            else:
                c = (Jt - J_line + mu * g2) / mu ** 2
                m = g2 / (2 * c) if c > 0 else mu / beta
                mu = min(max(m, beta * mu), mu / beta)
        return w, a, b, trials, mu

    for N in (1, 2, 3, 5, 8):
        wm, am, bm, tm, mum = model(N)
        opts = oracle.SolveOpts(max_iter=N, step0=step0, eps_g=0.0, step_rule=rule)
        wo, (ao, bo), st, _ = oracle.solve(g, geom, f0, mean, U, y, [0.0, 0.0], opts)
        assert st["iterations"] == N and st["trials"] == tm, (N, st, tm)
        np.testing.assert_allclose([*wo, ao, bo], [*wm, am, bm], rtol=1e-7, atol=1e-12)
        # the next step from a secant divides by a change of the gradient:
        # compared while the gradient is well above its rounding floor
        if np.linalg.norm(gf(wm, am, bm)) > 1e-4 * np.linalg.norm(gf(np.zeros(2), *ab_of(np.zeros(2)))):
            assert abs(st["mu"] - mum) <= 1e-6 * abs(mum)


def test_localize_constant_dvf():
    g = S.Grid((10, 10, 10), (2.0, 2.0, 2.0))
    c = np.array([1.5, -2.0, 3.25])
    mean = np.empty((3,) + g.shape)
    for a in range(3):
        mean[a] = c[a]
    U = np.zeros((1, 3) + g.shape)
    p_ref = np.array([0.3, -1.1, 2.0])
    p, st, it = oracle.localize(g, mean, U, [0.0], p_ref)
    assert st == 0 and it <= 2
    np.testing.assert_allclose(p, p_ref - c, atol=1e-12)


def test_localize_affine_dvf():
    g = S.Grid((30, 30, 30), (2.0, 2.0, 2.0))
    A = np.array([[0.05, 0.02, -0.01], [0.0, -0.04, 0.03], [0.02, 0.01, 0.06]])
    c = np.array([2.0, -1.0, 4.0])
    px, py, pz = g.mesh()
    P = np.stack(np.broadcast_arrays(px, py, pz))
    mean = np.einsum("ab,bzyx->azyx", A, P) + c[:, None, None, None]
    U = np.stack([np.ones((3,) + g.shape) * 0.0, np.ones((3,) + g.shape)])   # K = 2
    w = np.array([7.0, 0.5])                                                 # adds 0.5 mm
    p_ref = np.array([3.0, -4.0, 5.0])
    p, st, it = oracle.localize(g, mean, U, w, p_ref, tol=1e-12)
    expect = np.linalg.solve(np.eye(3) + A, p_ref - c - 0.5)
    assert st == 0
    np.testing.assert_allclose(p, expect, atol=1e-9)
    # the defining property of the pull-back inverse: p + x(p) = p_ref
    np.testing.assert_allclose(p + A @ p + c + 0.5, p_ref, atol=1e-9)


def test_localize_reports_nonconvergence():
    g = S.Grid((10, 10, 10), (1.0, 1.0, 1.0))
    px, py, pz = g.mesh()
    mean = np.stack(np.broadcast_arrays(3.0 * px, 0 * py, 0 * pz))  # |dx/dp| = 3: not contractive
    U = np.zeros((1, 3) + g.shape)
    p, st, it = oracle.localize(g, mean, U, [0.0], [0.7, 0.0, 0.0], max_iter=50)
    assert st == oracle.EDIVERGE and it == 50


def test_localize_analytic_motion_tumour():
    """Truth: the analytic DVF moves the reference tumour centre to the point p
    with p + x(p) = p_ref; K = motion rank, so U w* reproduces x exactly."""
    g = S.Grid((48, 48, 40), (5.0, 5.0, 6.0))
    m = S.pca_model(g, 3)
    phi = 2.4
    w = S.truth_w(m, phi)
    p_ref = S.tumor_center(g)
    p, st, it = oracle.localize(g, m.mean, m.U, w, p_ref, tol=1e-10)
    assert st == 0
    # evaluate the analytic field at p in closed form
    L = g.fov
    gx = math.exp(-(p[0] / (0.35 * L[0])) ** 2)
    c = S.phase_coeffs(phi, 3) * 1.5
    x = np.array([0.0, 10 * 0.3 * gx * c[1], 10 * gx * c[0] + 10 * 0.15 * gx * (p[2] / L[2]) * c[2]])
    # trilinear interpolation of the smooth field: agreement to its discretisation error
    np.testing.assert_allclose(p + x, p_ref, atol=2e-2)
    assert np.linalg.norm(p - p_ref) > 5.0          # the tumour really moved
