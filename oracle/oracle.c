/*
 * FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Each function restates one step of the method of Li et al. (section 2) in
 * plain double precision: no blocking, fusion or reordering beyond what the
 * definition states.  Where the paper is silent, the reading taken is stated
 * at the function and collected in the design notes.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_ENOCONV (-4)
#define ORC_EDIVERGE (-5)

/* Threads the OpenMP regions of the oracle use. */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the thread count of the later OpenMP regions (n >= 1). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

static long vol_size(const orc_grid* g) { return (long)g->n[0] * g->n[1] * g->n[2]; }

static double fetch(const double* F, const int n[3], long i, long j, long k)
{
    if (i < 0 || j < 0 || k < 0 || i >= n[0] || j >= n[1] || k >= n[2]) return 0.0;
    return F[i + (long)n[0] * (j + (long)n[1] * k)];
}

/* Trilinear interpolation (section 2.2: the reconstructed image is found
 * through trilinear interpolation).  i0 = floor(q), phi = q - i0, weights
 * (1 - phi) and phi per axis over the 8 corners.  Reading: the reference
 * image is zero (air) outside its grid, so T has support [-1, n) per axis. */
double orc_interp(const double* F, const int n[3], const double q[3])
{
    long i0[3];
    double ph[3];
    for (int a = 0; a < 3; ++a) {
        if (!(q[a] >= -1.0 && q[a] < (double)n[a])) return 0.0;
        double fl = floor(q[a]);
        i0[a] = (long)fl;
        ph[a] = q[a] - fl;
    }
    double s = 0.0;
    for (int c = 0; c < 2; ++c)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
                double w = (a ? ph[0] : 1.0 - ph[0]) * (b ? ph[1] : 1.0 - ph[1]) *
                           (c ? ph[2] : 1.0 - ph[2]);
                s += w * fetch(F, n, i0[0] + a, i0[1] + b, i0[2] + c);
            }
    return s;
}

/* Exact derivative of the trilinear interpolant (section 2.2: df/dx must be
 * consistent with the interpolation; it is a combination of the reference
 * image's differences at the eight neighbouring grid points weighted by the
 * fractional parts).  Same floor cell as the value, so at an integer
 * coordinate this is the right derivative. */
void orc_interp_grad(const double* F, const int n[3], const double q[3], double out[3])
{
    long i0[3];
    double ph[3];
    out[0] = out[1] = out[2] = 0.0;
    for (int a = 0; a < 3; ++a) {
        if (!(q[a] >= -1.0 && q[a] < (double)n[a])) return;
        double fl = floor(q[a]);
        i0[a] = (long)fl;
        ph[a] = q[a] - fl;
    }
    double c[2][2][2];
    for (int z = 0; z < 2; ++z)
        for (int y = 0; y < 2; ++y)
            for (int x = 0; x < 2; ++x) c[z][y][x] = fetch(F, n, i0[0] + x, i0[1] + y, i0[2] + z);
    double wx[2] = {1.0 - ph[0], ph[0]}, wy[2] = {1.0 - ph[1], ph[1]}, wz[2] = {1.0 - ph[2], ph[2]};
    for (int z = 0; z < 2; ++z)
        for (int y = 0; y < 2; ++y) out[0] += wy[y] * wz[z] * (c[z][y][1] - c[z][y][0]);
    for (int z = 0; z < 2; ++z)
        for (int x = 0; x < 2; ++x) out[1] += wx[x] * wz[z] * (c[z][1][x] - c[z][0][x]);
    for (int y = 0; y < 2; ++y)
        for (int x = 0; x < 2; ++x) out[2] += wx[x] * wy[y] * (c[1][y][x] - c[0][y][x]);
}

/* DVF composition, eq. (2) constraint and eq. (1): x = mean + U w (mm). */
void orc_compose(const orc_grid* g, int K, const double* mean, const double* U,
                 const double* w, double* x)
{
    long N = vol_size(g);
#pragma omp parallel for schedule(static)
    for (long v = 0; v < N; ++v)
        for (int a = 0; a < 3; ++a) {
            double s = mean[a * N + v];
            for (int k = 0; k < K; ++k) s += w[k] * U[((long)k * 3 + a) * N + v];
            x[a * N + v] = s;
        }
}

/* Index-space sample point of voxel v displaced by x[v]: the world point
 * p_v + x[v] = org + (v + x/s) s, i.e. q = v + x / s. */
static void warp_point(const orc_grid* g, const double* x, long N, long i, long j, long k,
                       long v, double q[3])
{
    q[0] = (double)i + x[v] / g->sp[0];
    q[1] = (double)j + x[N + v] / g->sp[1];
    q[2] = (double)k + x[2 * N + v] / g->sp[2];
}

/* Pull-back warp (sections 2.2 and 2.3): f(p) = f0(p + x(p)) evaluated at
 * every voxel centre by trilinear interpolation of f0. */
void orc_warp(const orc_grid* g, const double* f0, const double* x, double* f)
{
    long N = vol_size(g);
    int nx = g->n[0], ny = g->n[1], nz = g->n[2];
#pragma omp parallel for schedule(static)
    for (long k = 0; k < nz; ++k)
        for (long j = 0; j < ny; ++j)
            for (long i = 0; i < nx; ++i) {
                long v = i + nx * (j + ny * k);
                double q[3];
                warp_point(g, x, N, i, j, k, v, q);
                f[v] = orc_interp(f0, g->n, q);
            }
}

/* Transpose of the warp as a linear map of f0 (the gradient with respect to
 * the reference image): every voxel v spreads gv[v] onto the eight corners of
 * its sample point with the trilinear weights.  Serial, so the summation
 * order is fixed. */
void orc_warp_adjoint(const orc_grid* g, const double* x, const double* gv, double* out)
{
    long N = vol_size(g);
    int nx = g->n[0], ny = g->n[1], nz = g->n[2];
    memset(out, 0, sizeof(double) * N);
    for (long k = 0; k < nz; ++k)
        for (long j = 0; j < ny; ++j)
            for (long i = 0; i < nx; ++i) {
                long v = i + nx * (j + ny * k);
                double q[3];
                warp_point(g, x, N, i, j, k, v, q);
                int ok = 1;
                long i0[3];
                double ph[3];
                for (int a = 0; a < 3; ++a) {
                    if (!(q[a] >= -1.0 && q[a] < (double)g->n[a])) ok = 0;
                    else {
                        double fl = floor(q[a]);
                        i0[a] = (long)fl;
                        ph[a] = q[a] - fl;
                    }
                }
                if (!ok) continue;
                for (int c = 0; c < 2; ++c)
                    for (int b = 0; b < 2; ++b)
                        for (int a = 0; a < 2; ++a) {
                            long ii = i0[0] + a, jj = i0[1] + b, kk = i0[2] + c;
                            if (ii < 0 || jj < 0 || kk < 0 || ii >= nx || jj >= ny || kk >= nz) continue;
                            double w = (a ? ph[0] : 1.0 - ph[0]) * (b ? ph[1] : 1.0 - ph[1]) *
                                       (c ? ph[2] : 1.0 - ph[2]);
                            out[ii + nx * (jj + ny * kk)] += w * gv[v];
                        }
            }
}

/* Warp Jacobian df/dx (section 2.2): G[a][v] = (1/s_a) dT[f0]/dq_a at the
 * displaced point of voxel v (mm^-1 units, since x is in mm). */
void orc_warp_jacobian(const orc_grid* g, const double* f0, const double* x, double* G)
{
    long N = vol_size(g);
    int nx = g->n[0], ny = g->n[1], nz = g->n[2];
#pragma omp parallel for schedule(static)
    for (long k = 0; k < nz; ++k)
        for (long j = 0; j < ny; ++j)
            for (long i = 0; i < nx; ++i) {
                long v = i + nx * (j + ny * k);
                double q[3], d[3];
                warp_point(g, x, N, i, j, k, v, q);
                orc_interp_grad(f0, g->n, q, d);
                for (int a = 0; a < 3; ++a) G[a * N + v] = d[a] / g->sp[a];
            }
}

/* Cone-beam geometry (reading; the paper only states a cone beam, gantry
 * rotation and the imager size in section 3): rotation about z through the
 * isocentre, source s = iso + (SAD sin t, -SAD cos t, 0), detector centre
 * iso + (-(SDD-SAD) sin t, (SDD-SAD) cos t, 0), detector axes
 * e_u = (cos t, sin t, 0) and e_v = (0, 0, 1). */
void orc_source_pixel(const orc_geom* G, int iu, int iv, double s[3], double pix[3])
{
    double st = sin(G->angle), ct = cos(G->angle);
    double u = ((double)iu - 0.5 * (G->nu - 1)) * G->du + G->off_u;
    double vv = ((double)iv - 0.5 * (G->nv - 1)) * G->dv + G->off_v;
    double dd = G->sdd - G->sad;
    s[0] = G->iso[0] + G->sad * st;
    s[1] = G->iso[1] - G->sad * ct;
    s[2] = G->iso[2];
    pix[0] = G->iso[0] - dd * st + u * ct;
    pix[1] = G->iso[1] + dd * ct + u * st;
    pix[2] = G->iso[2] + vv;
}

/* Parameter interval [t0, t1] of the segment source -> pixel inside the
 * support box of the interpolant, (org - s, org + n s) per axis. */
static int ray_clip(const orc_grid* g, const double s[3], const double d[3], double L,
                    double* t0, double* t1)
{
    double tmin = 0.0, tmax = L;
    for (int a = 0; a < 3; ++a) {
        double lo = g->org[a] - g->sp[a], hi = g->org[a] + g->n[a] * g->sp[a];
        if (d[a] == 0.0) {
            if (s[a] <= lo || s[a] >= hi) return 0;
        } else {
            double ta = (lo - s[a]) / d[a], tb = (hi - s[a]) / d[a];
            if (ta > tb) { double t = ta; ta = tb; tb = t; }
            if (ta > tmin) tmin = ta;
            if (tb < tmax) tmax = tb;
        }
    }
    if (tmax < tmin) return 0;
    *t0 = tmin;
    *t1 = tmax;
    return 1;
}

/* One detector pixel of the projection P f (eq. (2); the discretisation of P
 * is a reading): p = dt * sum_n T[f](q(s + n dt d)), over the integers n whose
 * sample lies on the clipped segment; samples outside contribute zero. */
double orc_project_ray(const orc_grid* g, const orc_geom* G, const double* f, int iu, int iv)
{
    double s[3], pix[3], d[3];
    orc_source_pixel(G, iu, iv, s, pix);
    double L = 0.0;
    for (int a = 0; a < 3; ++a) { d[a] = pix[a] - s[a]; L += d[a] * d[a]; }
    L = sqrt(L);
    for (int a = 0; a < 3; ++a) d[a] /= L;
    double t0, t1;
    if (!ray_clip(g, s, d, L, &t0, &t1)) return 0.0;
    double dt = G->step;
    long n0 = (long)ceil(t0 / dt), n1 = (long)floor(t1 / dt);
    double acc = 0.0;
    for (long n = n0; n <= n1; ++n) {
        double t = (double)n * dt, q[3];
        for (int a = 0; a < 3; ++a) q[a] = (s[a] + t * d[a] - g->org[a]) / g->sp[a];
        acc += orc_interp(f, g->n, q);
    }
    return dt * acc;
}

void orc_project(const orc_grid* g, const orc_geom* G, const double* f, double* p)
{
    long M = (long)G->nu * G->nv;
#pragma omp parallel for schedule(dynamic, 64)
    for (long m = 0; m < M; ++m) p[m] = orc_project_ray(g, G, f, (int)(m % G->nu), (int)(m / G->nu));
}

/* Backprojection P^T r (the P^T in the gradient of section 2.2): the exact
 * transpose of orc_project, spreading r * dt * (trilinear weight) of every
 * sample onto its in-grid corners.  Each thread accumulates into a private
 * volume; the volumes are summed in thread order. */
void orc_backproject(const orc_grid* g, const orc_geom* G, const double* r, double* out)
{
    long N = vol_size(g), M = (long)G->nu * G->nv;
    int nx = g->n[0], ny = g->n[1], nz = g->n[2];
    int nth = 1;
#ifdef _OPENMP
    nth = omp_get_max_threads();
#endif
    double* priv = (double*)calloc((size_t)nth * N, sizeof(double));
#pragma omp parallel num_threads(nth)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* acc = priv + (size_t)tid * N;
#pragma omp for schedule(static)
        for (long m = 0; m < M; ++m) {
            if (r[m] == 0.0) continue;
            double s[3], pix[3], d[3];
            orc_source_pixel(G, (int)(m % G->nu), (int)(m / G->nu), s, pix);
            double L = 0.0;
            for (int a = 0; a < 3; ++a) { d[a] = pix[a] - s[a]; L += d[a] * d[a]; }
            L = sqrt(L);
            for (int a = 0; a < 3; ++a) d[a] /= L;
            double t0, t1;
            if (!ray_clip(g, s, d, L, &t0, &t1)) continue;
            double dt = G->step, rw = r[m] * dt;
            long n0 = (long)ceil(t0 / dt), n1 = (long)floor(t1 / dt);
            for (long n = n0; n <= n1; ++n) {
                double t = (double)n * dt, q[3], ph[3];
                long i0[3];
                int ok = 1;
                for (int a = 0; a < 3; ++a) {
                    q[a] = (s[a] + t * d[a] - g->org[a]) / g->sp[a];
                    if (!(q[a] >= -1.0 && q[a] < (double)g->n[a])) ok = 0;
                    else {
                        double fl = floor(q[a]);
                        i0[a] = (long)fl;
                        ph[a] = q[a] - fl;
                    }
                }
                if (!ok) continue;
                for (int c = 0; c < 2; ++c)
                    for (int b = 0; b < 2; ++b)
                        for (int a = 0; a < 2; ++a) {
                            long ii = i0[0] + a, jj = i0[1] + b, kk = i0[2] + c;
                            if (ii < 0 || jj < 0 || kk < 0 || ii >= nx || jj >= ny || kk >= nz) continue;
                            double w = (a ? ph[0] : 1.0 - ph[0]) * (b ? ph[1] : 1.0 - ph[1]) *
                                       (c ? ph[2] : 1.0 - ph[2]);
                            acc[ii + nx * (jj + ny * kk)] += w * rw;
                        }
            }
        }
    }
    memset(out, 0, sizeof(double) * N);
    for (int t = 0; t < nth; ++t) {
        const double* acc = priv + (size_t)t * N;
        for (long v = 0; v < N; ++v) out[v] += acc[v];
    }
    free(priv);
}

/* Sums for the closed-form intensity fit, eq. (4) with Y = [y, 1]:
 * S = (sum y, sum y^2, sum p, sum y p, M). */
void orc_regression_sums(int M, const double* y, const double* p, double S[5])
{
    double sy = 0, syy = 0, sp = 0, syp = 0;
    for (int m = 0; m < M; ++m) {
        sy += y[m];
        syy += y[m] * y[m];
        sp += p[m];
        syp += y[m] * p[m];
    }
    S[0] = sy; S[1] = syy; S[2] = sp; S[3] = syp; S[4] = (double)M;
}

/* Step 2, eq. (4): (a, b)^T = (Y^T Y)^-1 Y^T P f, the unique minimiser of J
 * for fixed w.  Reading for a singular Y^T Y (constant y): a = 0 and b = the
 * mean of P f. */
void orc_step2(const double S[5], double ab[2])
{
    double sy = S[0], syy = S[1], sp = S[2], syp = S[3], M = S[4];
    double D = syy * M - sy * sy;
    if (!(D > 1e-12 * syy * M)) {
        ab[0] = 0.0;
        ab[1] = M > 0 ? sp / M : 0.0;
        return;
    }
    ab[0] = (M * syp - sy * sp) / D;
    ab[1] = (syy * sp - sy * syp) / D;
}

/* Cost, eq. (2): J = || P f - a y - b 1 ||^2 (no factor 1/2); optionally
 * returns the residual r. */
double orc_cost(int M, const double* p, const double* y, double a, double b, double* r)
{
    double J = 0.0;
    for (int m = 0; m < M; ++m) {
        double rm = p[m] - a * y[m] - b;
        if (r) r[m] = rm;
        J += rm * rm;
    }
    return J;
}

/* Cost and gradient (section 2.2): dJ/dw = 2 U^T (df/dx)^T P^T (P f - a y - b),
 * evaluated in the paper's order: backproject 2r, multiply by the warp
 * Jacobian, contract with each eigenvector field. */
double orc_cost_grad(const orc_grid* g, const orc_geom* G, const double* f0,
                     int K, const double* mean, const double* U, const double* w,
                     const double* y, double a, double b, double* grad, double* p_out)
{
    long N = vol_size(g);
    int M = G->nu * G->nv;
    double* x = (double*)malloc(sizeof(double) * 3 * N);
    double* f = (double*)malloc(sizeof(double) * N);
    double* p = (double*)malloc(sizeof(double) * M);
    double* r = (double*)malloc(sizeof(double) * M);
    double* gv = (double*)malloc(sizeof(double) * N);
    double* Gj = (double*)malloc(sizeof(double) * 3 * N);
    orc_compose(g, K, mean, U, w, x);
    orc_warp(g, f0, x, f);
    orc_project(g, G, f, p);
    double J = orc_cost(M, p, y, a, b, r);
    for (int m = 0; m < M; ++m) r[m] *= 2.0;
    orc_backproject(g, G, r, gv);
    orc_warp_jacobian(g, f0, x, Gj);
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
        for (long v = 0; v < N; ++v) {
            double d = 0.0;
            for (int c = 0; c < 3; ++c) d += Gj[c * N + v] * U[((long)k * 3 + c) * N + v];
            s += gv[v] * d;
        }
        grad[k] = s;
    }
    if (p_out) memcpy(p_out, p, sizeof(double) * M);
    free(x); free(f); free(p); free(r); free(gv); free(Gj);
    return J;
}

static void forward_at(const orc_grid* g, const orc_geom* G, const double* f0, int K,
                       const double* mean, const double* U, const double* w, double* p)
{
    long N = vol_size(g);
    double* x = (double*)malloc(sizeof(double) * 3 * N);
    double* f = (double*)malloc(sizeof(double) * N);
    orc_compose(g, K, mean, U, w, x);
    orc_warp(g, f0, x, f);
    orc_project(g, G, f, p);
    free(x);
    free(f);
}

static double norm(int K, const double* v)
{
    double s = 0.0;
    for (int k = 0; k < K; ++k) s += v[k] * v[k];
    return sqrt(s);
}

/* First trial step of the next iteration from the line just searched:
 * phi(mu) = J - g2 mu + c mu^2 through phi(mu_acc) = Jt has its minimum at
 * g2 / (2 c); the result is kept within one backtracking factor of mu_acc. */
static double next_initial_step(double J, double g2, double Jt, double mu_acc, double beta)
{
    double c = (Jt - J + mu_acc * g2) / (mu_acc * mu_acc);
    double m = c > 0.0 ? g2 / (2.0 * c) : mu_acc / beta;
    if (m < beta * mu_acc) m = beta * mu_acc;
    if (m > mu_acc / beta) m = mu_acc / beta;
    return m;
}

/* The alternating algorithm of section 2.2.  Readings where the paper is
 * silent: (a, b) start with step 2 at w_0; step 1 is gradient descent on w
 * with a, b fixed and the step from Armijo's rule: trial w - mu g accepted
 * when J' <= J - sigma mu |g|^2 (ties accept), otherwise mu <- beta mu for at
 * most max_backtracks trials; the first trial of a solve moves w by step0
 * (or uses the given step size mu0, e.g. carried over from the previous
 * frame's solve); step 2 then refits (a, b) at the accepted w.
 * Each later iteration's first trial (step_rule 0, the default) is the
 * secant step s.y / y.y, with s the last accepted step in w and y the
 * change of the gradient over it (each gradient taken with its own a, b);
 * where s.y <= 0, or with step_rule 1, it is the minimiser of the quadratic
 * in mu that matches the previous iteration's line (its J, its slope -|g|^2
 * and the accepted trial's J'), kept within [beta mu', mu'/beta] of the
 * accepted mu' (mu'/beta where that quadratic has no minimum).  Stop when |g_n| <= eps_g |g_0|, or
 * at the iteration cap, or when the line search is exhausted (the last
 * accepted w is kept).  J_hist, if given, receives J after each step 2. */
int orc_solve(const orc_grid* g, const orc_geom* G, const double* f0, int K,
              const double* mean, const double* U, const double* y,
              const orc_opts* o, double* w, double ab[2], orc_stats* st, double* J_hist)
{
    int M = G->nu * G->nv;
    double* p = (double*)malloc(sizeof(double) * M);
    double* grad = (double*)malloc(sizeof(double) * K);
    double* wt = (double*)malloc(sizeof(double) * K);
    double* w_prev = (double*)malloc(sizeof(double) * K);
    double* g_prev = (double*)malloc(sizeof(double) * K);
    double S[5];
    int status = ORC_OK, iters = 0, trials = 0;

    forward_at(g, G, f0, K, mean, U, w, p);
    orc_regression_sums(M, y, p, S);
    orc_step2(S, ab);
    double J = orc_cost_grad(g, G, f0, K, mean, U, w, y, ab[0], ab[1], grad, NULL);
    double gn = norm(K, grad), g0 = gn, J0 = J;
    if (J_hist) J_hist[0] = J;
    double mu = o->fixed_mu > 0 ? o->fixed_mu : (o->mu0 > 0 ? o->mu0 : (g0 > 0 ? o->step0 / g0 : 0.0));

    for (int n = 0;; ++n) {
        if (gn <= o->eps_g * g0) break;
        if (n == o->max_iter) { status = ORC_ENOCONV; break; }
        int accepted = 0;
        double Jt = 0.0;
        if (o->fixed_mu > 0) {
            for (int k = 0; k < K; ++k) wt[k] = w[k] - mu * grad[k];
            forward_at(g, G, f0, K, mean, U, wt, p);
            ++trials;
            accepted = 1;
        } else {
            for (int l = 0; l < o->max_backtracks; ++l) {
                for (int k = 0; k < K; ++k) wt[k] = w[k] - mu * grad[k];
                forward_at(g, G, f0, K, mean, U, wt, p);
                ++trials;
                Jt = orc_cost(M, p, y, ab[0], ab[1], NULL);
                if (Jt <= J - o->sigma * mu * gn * gn) { accepted = 1; break; }
                mu *= o->beta;
            }
        }
        if (!accepted) { status = ORC_ENOCONV; break; }
        double J_line = J, g2_line = gn * gn;
        for (int k = 0; k < K; ++k) {
            w_prev[k] = w[k];
            g_prev[k] = grad[k];
            w[k] = wt[k];
        }
        orc_regression_sums(M, y, p, S);
        orc_step2(S, ab);
        J = orc_cost_grad(g, G, f0, K, mean, U, w, y, ab[0], ab[1], grad, NULL);
        gn = norm(K, grad);
        iters = n + 1;
        if (J_hist) J_hist[iters] = J;
        if (!(o->fixed_mu > 0)) {
            double sy = 0.0, yy = 0.0;
            for (int k = 0; k < K; ++k) {
                double sk = w[k] - w_prev[k], yk = grad[k] - g_prev[k];
                sy += sk * yk;
                yy += yk * yk;
            }
            if (o->step_rule == 0 && sy > 0.0 && yy > 0.0)
                mu = sy / yy;
            else
                mu = next_initial_step(J_line, g2_line, Jt, mu, o->beta);
        }
    }
    if (st) {
        st->iterations = iters; st->trials = trials; st->status = status;
        st->J0 = J0; st->J = J; st->gnorm0 = g0; st->gnorm = gn;
        st->a = ab[0]; st->b = ab[1];
        st->mu = mu;
    }
    free(p); free(grad); free(wt); free(w_prev); free(g_prev);
    return status;
}

/* Displacement at an arbitrary point (mm) by trilinear interpolation of the
 * composed DVF with clamp-to-edge (reading: the tumour is interior). */
static void dvf_at(const orc_grid* g, const double* x, const double p[3], double out[3])
{
    long N = vol_size(g);
    long i0[3];
    double ph[3];
    for (int a = 0; a < 3; ++a) {
        double q = (p[a] - g->org[a]) / g->sp[a];
        double hi = (double)(g->n[a] - 1);
        if (q < 0.0) q = 0.0;
        if (q > hi) q = hi;
        double fl = floor(q);
        if (g->n[a] >= 2 && fl > hi - 1.0) fl = hi - 1.0;
        i0[a] = (long)fl;
        ph[a] = q - fl;
    }
    for (int c3 = 0; c3 < 3; ++c3) {
        double s = 0.0;
        for (int c = 0; c < 2; ++c)
            for (int b = 0; b < 2; ++b)
                for (int a = 0; a < 2; ++a) {
                    double w = (a ? ph[0] : 1.0 - ph[0]) * (b ? ph[1] : 1.0 - ph[1]) *
                               (c ? ph[2] : 1.0 - ph[2]);
                    if (w == 0.0) continue;
                    long ii = i0[0] + a, jj = i0[1] + b, kk = i0[2] + c;
                    s += w * x[c3 * N + ii + g->n[0] * (jj + (long)g->n[1] * kk)];
                }
        out[c3] = s;
    }
}

/* Tumour localisation (section 2.3): the reconstructed DVF is pull-back, so
 * the tumour at p_ref in the reference image sits at the point p with
 * p + x(p) = p_ref.  Solved by the fixed-point iteration p <- p_ref - x(p)
 * of Chen et al. (the paper's ref. 13), evaluated at the tumour point only;
 * stops when the update is shorter than tol (mm). */
int orc_localize(const orc_grid* g, int K, const double* mean, const double* U,
                 const double* w, const double p_ref[3], double tol, int max_iter,
                 double p_out[3], int* iters)
{
    long N = vol_size(g);
    double* x = (double*)malloc(sizeof(double) * 3 * N);
    orc_compose(g, K, mean, U, w, x);
    double p[3] = {p_ref[0], p_ref[1], p_ref[2]};
    int status = ORC_EDIVERGE, it;
    for (it = 1; it <= max_iter; ++it) {
        double X[3], pn[3], d = 0.0;
        dvf_at(g, x, p, X);
        for (int a = 0; a < 3; ++a) {
            pn[a] = p_ref[a] - X[a];
            d += (pn[a] - p[a]) * (pn[a] - p[a]);
            p[a] = pn[a];
        }
        if (sqrt(d) < tol) { status = ORC_OK; break; }
    }
    if (iters) *iters = it > max_iter ? max_iter : it;
    p_out[0] = p[0]; p_out[1] = p[1]; p_out[2] = p[2];
    free(x);
    return status;
}
