/*
 * FP64 CPU oracle for single-projection reconstruction under a PCA lung-motion
 * model (Li et al., "Real-time volumetric image reconstruction and 3D tumor
 * localization based on a single x-ray projection image for lung cancer
 * radiotherapy").
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, obviously-correct
 * definition that the HIP library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it; the
 * product path never does.  It shares no code, header or helper with the HIP
 * library.
 *
 * Conventions (all in double precision):
 *   volumes   [nz][ny][nx], flat index i + nx*(j + ny*k); origin = centre of
 *             voxel (0,0,0) in mm; spacing in mm.
 *   DVF       pull-back, mm, structure of arrays [3][N] (x, y, z components).
 *   model     mean [3][N], U [K][3][N].
 *   detector  [nv][nu], flat iu + nu*iv.
 */
#ifndef PCR_ORACLE_H
#define PCR_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int n[3];          /* nx, ny, nz */
    double sp[3];      /* voxel spacing (mm) */
    double org[3];     /* centre of voxel (0,0,0) (mm) */
} orc_grid;

typedef struct {
    double angle;      /* gantry angle (rad) */
    double sad, sdd;   /* source-isocentre and source-detector distances (mm) */
    int nu, nv;        /* detector columns, rows */
    double du, dv;     /* pixel pitch at the detector plane (mm) */
    double off_u, off_v;
    double step;       /* ray sample spacing (mm), samples at t = n*step */
    double iso[3];     /* isocentre (mm) */
} orc_geom;

typedef struct {
    int max_iter;         /* iteration cap */
    int max_backtracks;   /* Armijo trials per iteration */
    double sigma, beta;   /* Armijo sufficient-decrease constant and shrink */
    double eps_g;         /* stop when |g_n| <= eps_g |g_0| */
    double step0;         /* first trial moves w by this distance */
    double fixed_mu;      /* > 0: constant step, no line search */
    double mu0;           /* > 0: step size of the first trial (else step0 / |g_0|) */
    int step_rule;        /* first trial of each later iteration: 0 = secant
                             s.y / y.y of the last step, 1 = quadratic model */
} orc_opts;

typedef struct {
    int iterations, trials, status;
    double J0, J, gnorm0, gnorm, a, b;
    double mu;            /* step size the next iteration would try first */
} orc_stats;

int orc_num_threads(void);
void orc_set_num_threads(int n);

/* Trilinear interpolant T[F](q) at index-space point q; F = 0 outside. */
double orc_interp(const double* F, const int n[3], const double q[3]);
/* Exact partial derivatives dT/dq_a of the same interpolant (floor cell). */
void orc_interp_grad(const double* F, const int n[3], const double q[3], double out[3]);

void orc_compose(const orc_grid* g, int K, const double* mean, const double* U,
                 const double* w, double* x);
void orc_warp(const orc_grid* g, const double* f0, const double* x, double* f);
void orc_warp_adjoint(const orc_grid* g, const double* x, const double* gv, double* out);
void orc_warp_jacobian(const orc_grid* g, const double* f0, const double* x, double* G);

void orc_source_pixel(const orc_geom* G, int iu, int iv, double s[3], double pix[3]);
double orc_project_ray(const orc_grid* g, const orc_geom* G, const double* f, int iu, int iv);
void orc_project(const orc_grid* g, const orc_geom* G, const double* f, double* p);
void orc_backproject(const orc_grid* g, const orc_geom* G, const double* r, double* out);

void orc_regression_sums(int M, const double* y, const double* p, double S[5]);
void orc_step2(const double S[5], double ab[2]);
double orc_cost(int M, const double* p, const double* y, double a, double b, double* r);
double orc_cost_grad(const orc_grid* g, const orc_geom* G, const double* f0,
                     int K, const double* mean, const double* U, const double* w,
                     const double* y, double a, double b, double* grad,
                     double* p_out);
int orc_solve(const orc_grid* g, const orc_geom* G, const double* f0, int K,
              const double* mean, const double* U, const double* y,
              const orc_opts* o, double* w, double ab[2], orc_stats* st,
              double* J_hist);
int orc_localize(const orc_grid* g, int K, const double* mean, const double* U,
                 const double* w, const double p_ref[3], double tol, int max_iter,
                 double p_out[3], int* iters);

#ifdef __cplusplus
}
#endif
#endif
