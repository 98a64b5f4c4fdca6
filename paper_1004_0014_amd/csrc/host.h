// Host-side building blocks shared by the C ABI (api.hip) and the serving
// engine (serve.hip): error reporting, validation, device scratch, the
// per-projection evaluator and the resumable solver state machine.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstring>

#include "pcr.h"
#include "pcr_internal.h"

namespace pcr {

// ------------------------------------------------------------- errors ----
// Records a thread-local description (pcr_last_error) and returns `code`.
pcr_status fail(pcr_status code, const char* fmt, ...);

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return ::pcr::fail(e_ == hipErrorOutOfMemory ? PCR_ENOMEM : PCR_EDEVICE,         \
                               "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__,    \
                               __LINE__);                                                    \
    } while (0)

#define PCR_TRY(expr)                                                                        \
    do {                                                                                     \
        pcr_status s_ = (expr);                                                              \
        if (s_ != PCR_OK) return s_;                                                         \
    } while (0)

// ----------------------------------------------------------- profiler ----
namespace prof {
enum Id { WARP, MARCH, REDUCE, BACKPROJ, CONTRACT, LOCALIZE, ZERO, PAD, UNPAD, COMPOSE, WARP_PLAIN,
          WARP_ADJ, PCA_GRAM, PCA_FIELDS, NKERN };
// Brackets one launch with HIP events on `s` while profiling is enabled.
struct Scope {
    hipStream_t s;
    int id;
    hipEvent_t a = nullptr;
    Scope(int id_, hipStream_t s_);
    ~Scope();
};
}  // namespace prof
#define PCR_PROF_CAT2(a, b) a##b
#define PCR_PROF_CAT(a, b) PCR_PROF_CAT2(a, b)
#define PROF(id, s) ::pcr::prof::Scope PCR_PROF_CAT(prof_scope_, __LINE__)(::pcr::prof::id, s)

// --------------------------------------------------------- validation ----
size_t dtype_size(pcr_dtype d);
pcr_status check_grid(const pcr_grid* g);
pcr_status check_geom(const pcr_geom* G);
// PCR_EINVAL unless the FP32 march can address an image of C channels per
// cell on this grid in both in-plane axis orders (see march_f32_fits).
pcr_status check_march_image(const pcr_grid& g, int C, pcr_dtype compute);
pcr_status check_march_steps(const pcr_grid& g, const pcr_geom& G, pcr_dtype compute);
pcr_status check_compute(pcr_dtype d);
pcr_status check_storage(pcr_dtype d);
pcr_status check_model(const pcr_model* m);
pcr_status check_finite(const double* v, int n, const char* what);
pcr_status check_opts(const pcr_solve_opts* o);

inline void effective_w(const pcr_model& m, const double* w, double* w_eff)
{
    for (int k = 0; k < m.K; ++k) w_eff[k] = w[k] * (m.scale ? m.scale[k] : 1.0);
}

// Channels per cell of an image with kc channels in use: 1, 2, 4, 6 or 8
// (6: 24-byte FP32 cells for K = 4 and 5).  FP16 cells take 4 or 8 channels
// (their loads read 8 halves at a time), so 5 or 6 in use take 8 there.
inline int channels_for(int kc) { return kc <= 1 ? 1 : kc <= 2 ? 2 : kc <= 4 ? 4 : kc <= 6 ? 6 : 8; }
inline int channels_for_half(int kc) { return kc <= 2 ? 2 : kc <= 4 ? 4 : 8; }

// Device bytes of a model and reference image stored as given.
inline size_t model_bytes(const pcr_grid& g, int K, pcr_dtype storage, pcr_dtype f0_dtype)
{
    size_t N = (size_t)g.n[0] * g.n[1] * g.n[2];
    return N * (3 * (size_t)(K + 1) * dtype_size(storage) + dtype_size(f0_dtype));
}

// ------------------------------------------------------- device scratch --
// Grow-only device buffer owned by the library.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    int device = -1;
    pcr_status ensure(size_t need, int dev, hipStream_t s);
    void release();
};

// Pinned, coherent host memory that kernels can write directly (d: its
// device address).
struct HostBuf {
    double* p = nullptr;
    double* d = nullptr;
    size_t n = 0;
    pcr_status ensure(size_t need);
    void release();
};

// Host staging of an evaluation's results: the moments and the samples
// count, then (at kDoneSlot, as an unsigned 64-bit word) the sequence number
// the final-sum kernel stores once they are written.
constexpr int kDoneSlot = kMaxMoments + 2;
constexpr int kHostSlots = kMaxMoments + 4;

// Moments of one projection (see n_moments) and the quantities of section
// 2.2 formed from them.
struct Moments {
    double m[kMaxMoments];
    double M;
    double samples = 0;   // ray samples marched
    int K;
    // J(a, b) = sum (p - a y - b)^2 expanded in the moments (eq. (2))
    double J(double a, double b) const
    {
        return m[4] - 2 * a * m[3] - 2 * b * m[2] + a * a * m[1] + 2 * a * b * m[0] + b * b * M;
    }
    // dJ/dw_eff_k = 2 sum (p - a y - b) t_k
    double grad(int k, double a, double b) const
    {
        return 2.0 * (m[5 + 3 * k] - a * m[6 + 3 * k] - b * m[7 + 3 * k]);
    }
    // step 2, eq. (4): least-squares (a, b) for Y = [y, 1]; a singular
    // Y^T Y (constant y) gives a = 0 and b = mean(p)
    void step2(double* a, double* b) const
    {
        double sy = m[0], syy = m[1], sp = m[2], syp = m[3];
        double D = syy * M - sy * sy;
        if (!(D > 1e-12 * syy * M)) {
            *a = 0.0;
            *b = M > 0 ? sp / M : 0.0;
            return;
        }
        *a = (M * syp - sy * sp) / D;
        *b = (syy * sp - sy * syp) / D;
    }
};

// Device scratch of one solve in flight: the zero-padded fused image, the
// single-channel image, backprojection and projection buffers of the
// adjoint mode, reduction partials, moments and pinned host staging.
struct Scratch {
    int device = -1;
    PadLayout Lc{}, L1{};
    PadLayout volc_layout{};   // layout whose zero borders volc holds
    bool volc_zeroed = false;
    size_t volc_floor = 0;     // allocate volc at least this large (a serving slot
                               // sized once for every admitted stream)
    DevBuf volc, vol1, acc1, p, partials, moments;
    HostBuf host;
    unsigned long long seq = 0;   // sequence number of the last evaluation
    void release();
    size_t device_bytes() const
    {
        return volc.bytes + vol1.bytes + acc1.bytes + p.bytes + partials.bytes + moments.bytes;
    }
};

// Where the warped image can be nonzero.  f0 is zero outside the index box
// [lo, hi] of its nonzero voxels, and a displacement moves values by at most
// max|mean_a| + sum_k |w_k| max|U_k,a| along axis a, so the warped channels
// (f and the tangents, which use the same eight taps) vanish outside that
// box dilated by the displacement and one cell, and a ray sample contributes
// nothing outside it dilated by one more cell.  The march clips rays to this
// box: the samples it skips are exactly zero, the sample grid is unchanged.
//
// Within the box, rays are clipped further to slabs of slab_t slices: per
// slab an octagon in (i, j) (bounds on i, j, i + j, i - j) and a range in k
// holding its nonzero voxels, dilated the same way (slab_buf: the FP32
// tables of RayGeom::slabs, x-fastest axis order then y-fastest).
struct Support {
    bool valid = false;
    int lo[3], hi[3];        // nonzero f0 voxels (lo > hi: none)
    double mmax[3];          // max |mean_a| (mm)
    double umax[8][3];       // max |U_k,a| of the stored fields
    double f0max;            // max |f0|
    int nslab = 0, slab_t = 1;
    DevBuf slab_buf;         // owned; release() frees it
    void release() { slab_buf.release(); }
};
// FP16 channel scales (powers of two): f is bounded by max|f0| and h_k by
// 2 max|f0| sum_a max|U_k,a| / s_a (each partial derivative of the
// interpolant is a weighted difference of neighbouring values).
void half_scales(const Support& sp, const pcr_grid& g, int K, float hs[8]);
pcr_status compute_support(const pcr_grid& g, const pcr_model& m, pcr_dtype f0_dtype,
                           const void* f0, int device, hipStream_t s, Support* out);
// Ray clip box (index space; x and y swapped for the y-fastest layout).
void clip_box(const Support& sp, const pcr_grid& g, int K, const double* w_eff, bool swap_xy,
              double clo[3], double chi[3]);
// Clips a ray geometry (built with the same swap_xy) to the box and slabs
// for the displacements of w_eff.
void clip_geom(const Support& sp, const pcr_grid& g, int K, const double* w_eff, bool swap_xy,
               RayGeom& rg);
// Voxels {lo x, lo y, lo z, hi x, hi y, hi z} (hi exclusive) whose cells the
// samples of rays clipped to g's box can read (grid axis order): the warp
// computes only these, since no other cell is sampled.
void warp_box(const RayGeom& g, const pcr_grid& grid, int box[6]);

// Evaluates projections of trial w for one (grid, model, f0, y, geometry)
// into one Scratch on one stream.
struct Evaluator {
    const pcr_grid* grid;
    const pcr_model* model;   // scale already applied through effective_w
    pcr_dtype f0_dtype, compute;
    const void* f0;
    Scratch* sc;
    hipStream_t s;
    const Support* sup = nullptr;   // null: rays span the whole support box
    bool image_f16 = false;         // FP16 fused image (FP32 compute, support known)
    // per projection
    const void* y = nullptr;
    RayGeom rg{}, rgc{};
    MarchShape ms{}, msc{};
    int M = 0, blocks = 0, blocksc = 0, mode = PCR_GRAD_FUSED;

    pcr_status prepare(const void* y_, const pcr_geom& G, int mode_);
    // Enqueues warp + march + final sum; the sum writes the moments into the
    // host staging and then publishes the evaluation's sequence number.
    pcr_status enqueue_eval(const double* w);
    // Spins until the last evaluation's moments are published (checking the
    // stream for errors now and then).
    pcr_status wait_published();
    // After the stream finished the last eval (or it was published): its
    // moments.
    void collect(Moments& out) const;
    pcr_status eval_sync(const double* w, Moments& out);
    // Adjoint mode: dJ/dw_eff at the w of the last eval (its p is kept).
    pcr_status grad_adjoint(const double* w, double a, double b, double* grad);
};

// The alternating algorithm of section 2.2 as a resumable state machine:
// the caller evaluates the projection at eval_w() and feeds its moments
// until done().  The blocking solve and the serving engine drive the same
// machine, so a solve takes identical steps alone and in a batch.
// Armijo's rule (section 2.2) leaves each line's first trial open.  Secant
// rule (the default): s.y / y.y, with s the last accepted step in w and y the
// change of the gradient over it.  Quadratic rule (and the fallback where
// s.y <= 0): the minimiser of the quadratic phi(mu) = J - g2 mu + c mu^2 that
// passes through the accepted trial phi(mu_acc) = Jt of the line just
// searched, kept within [beta mu_acc, mu_acc / beta] (mu_acc / beta when
// c <= 0).
inline double next_initial_step(double J, double g2, double Jt, double mu_acc, double beta)
{
    const double c = (Jt - J + mu_acc * g2) / (mu_acc * mu_acc);
    double m = c > 0.0 ? g2 / (2.0 * c) : mu_acc / beta;
    if (m < beta * mu_acc) m = beta * mu_acc;
    if (m > mu_acc / beta) m = mu_acc / beta;
    return m;
}

struct SolveSM {
    int K = 0;
    pcr_solve_opts o{};
    double scale[8];
    double w[8], wt[8], g[8];
    double a = 0, b = 0, J = 0, gn = 0, g0 = 0, J0 = 0, mu = 0, samples = 0;
    int iters = 0, trials = 0, n = 0, l = 0;
    enum State { NEED_INIT, NEED_TRIAL, DONE } state = NEED_INIT;
    pcr_status status = PCR_OK;

    void begin(int K_, const pcr_solve_opts& opts, const double* scale_or_null, const double* w0);
    const double* eval_w() const { return state == NEED_INIT ? w : wt; }
    bool done() const { return state == DONE; }
    // grad_fn (adjoint mode) computes dJ/dw_eff at (w, a, b) from the last
    // evaluation; null in fused mode (gradient from the moments).
    template <typename GradFn>
    pcr_status feed(const Moments& mo, GradFn&& grad_fn);
    void fill_stats(pcr_solve_stats* st) const;

  private:
    void advance();
};

inline void SolveSM::begin(int K_, const pcr_solve_opts& opts, const double* sc, const double* w0)
{
    K = K_;
    o = opts;
    for (int k = 0; k < 8; ++k) scale[k] = (sc && k < K) ? sc[k] : 1.0;
    for (int k = 0; k < K; ++k) w[k] = w0[k];
    iters = trials = n = l = 0;
    samples = 0;
    state = NEED_INIT;
    status = PCR_OK;
}

template <typename GradFn>
inline pcr_status SolveSM::feed(const Moments& mo, GradFn&& grad_fn)
{
    const bool fixed = o.fixed_mu > 0;
    samples += mo.samples;
    auto gradient = [&](const double* wv) -> pcr_status {
        if (o.grad_mode == PCR_GRAD_FUSED) {
            for (int k = 0; k < K; ++k) g[k] = mo.grad(k, a, b);
        } else {
            pcr_status st = grad_fn(wv, a, b, g);
            if (st != PCR_OK) return st;
        }
        double s2 = 0.0;
        for (int k = 0; k < K; ++k) {
            g[k] *= scale[k];
            s2 += g[k] * g[k];
        }
        gn = std::sqrt(s2);
        return PCR_OK;
    };
    if (state == NEED_INIT) {
        mo.step2(&a, &b);
        J = mo.J(a, b);
        PCR_TRY(gradient(w));
        g0 = gn;
        J0 = J;
        mu = fixed ? o.fixed_mu : (o.mu0 > 0 ? o.mu0 : (g0 > 0 ? o.step0 / g0 : 0.0));
        advance();
        return PCR_OK;
    }
    if (state != NEED_TRIAL) return PCR_OK;
    ++trials;
    const double Jt = mo.J(a, b);
    if (fixed || Jt <= J - o.sigma * mu * gn * gn) {
        const double J_line = J, g2_line = gn * gn;
        double w_prev[8], g_prev[8];
        for (int k = 0; k < K; ++k) {
            w_prev[k] = w[k];
            g_prev[k] = g[k];
            w[k] = wt[k];
        }
        mo.step2(&a, &b);
        J = mo.J(a, b);
        PCR_TRY(gradient(w));
        iters = ++n;
        if (!fixed) {
            double sy = 0.0, yy = 0.0;
            for (int k = 0; k < K; ++k) {
                const double sk = w[k] - w_prev[k], yk = g[k] - g_prev[k];
                sy += sk * yk;
                yy += yk * yk;
            }
            if (o.step_rule == PCR_STEP_SECANT && sy > 0.0 && yy > 0.0)
                mu = sy / yy;
            else
                mu = next_initial_step(J_line, g2_line, Jt, mu, o.beta);
        }
        advance();
        return PCR_OK;
    }
    mu *= o.beta;
    if (++l == o.max_backtracks) {
        status = PCR_ENOCONV;
        state = DONE;
        return PCR_OK;
    }
    for (int k = 0; k < K; ++k) wt[k] = w[k] - mu * g[k];
    return PCR_OK;
}

inline void SolveSM::advance()
{
    if (!std::isfinite(J) || !std::isfinite(gn)) {
        status = PCR_EDEVICE;
        state = DONE;
        return;
    }
    if (gn <= o.eps_g * g0) {
        state = DONE;
        return;
    }
    if (n == o.max_iter) {
        status = PCR_ENOCONV;
        state = DONE;
        return;
    }
    l = 0;
    for (int k = 0; k < K; ++k) wt[k] = w[k] - mu * g[k];
    state = NEED_TRIAL;
}

inline void SolveSM::fill_stats(pcr_solve_stats* st) const
{
    std::memset(st, 0, sizeof *st);
    st->status = status;
    st->iterations = iters;
    st->trials = trials;
    st->J0 = J0;
    st->J = J;
    st->gnorm0 = g0;
    st->gnorm = gn;
    st->a = a;
    st->b = b;
    st->samples = samples;
    st->mu = mu;
    st->fp_status = PCR_OK;
}

}  // namespace pcr
