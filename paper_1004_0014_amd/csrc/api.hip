// C ABI of the reconstruction library: validation, device scratch, the
// kernel profiler, the stateless entry points, the solver context and the
// per-projection solve (section 2.2 of Li et al.).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "host.h"
#include "scheduler.h"

using namespace pcr;

#define PCR_VERSION_STRING "pcr 0.2.0 (gfx950)"

namespace pcr {

// ------------------------------------------------------------- errors ----
static thread_local std::string g_err;

pcr_status fail(pcr_status code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

// --------------------------------------------------------- validation ----
size_t dtype_size(pcr_dtype d)
{
    switch (d) {
    case PCR_F32: return 4;
    case PCR_F64: return 8;
    case PCR_BF16: return 2;
    case PCR_F16: return 2;
    }
    return 0;
}

pcr_status check_grid(const pcr_grid* g)
{
    if (!g) return fail(PCR_EINVAL, "grid is NULL");
    for (int a = 0; a < 3; ++a) {
        if (g->n[a] <= 0) return fail(PCR_EINVAL, "grid n[%d] = %d must be > 0", a, g->n[a]);
        if (!(g->spacing_mm[a] > 0) || !std::isfinite(g->spacing_mm[a]))
            return fail(PCR_EINVAL, "grid spacing[%d] must be finite and > 0", a);
        if (!std::isfinite(g->origin_mm[a])) return fail(PCR_EINVAL, "grid origin must be finite");
    }
    if (g->n[2] > 65535 || g->n[1] > 65535)
        return fail(PCR_EINVAL, "grid n = (%d, %d, %d) exceeds the launch limits", g->n[0], g->n[1], g->n[2]);
    double cells = (double)(g->n[0] + 3) * (g->n[1] + 3) * (g->n[2] + 3);
    if (cells > 2.0e9) return fail(PCR_EINVAL, "grid too large (%.3g padded cells)", cells);
    return PCR_OK;
}

pcr_status check_march_image(const pcr_grid& g, int C, pcr_dtype compute)
{
    if (compute != PCR_F32) return PCR_OK;   // the FP64 march uses 64-bit offsets
    for (int yf = 0; yf < 2; ++yf)
        if (!march_f32_fits(make_pad(g, C, yf != 0)))
            return fail(PCR_EINVAL,
                        "grid (%d, %d, %d) with %d FP32 channels per cell exceeds the march's "
                        "32-bit addressing (padded image < 2 GiB, padded rows < 16 MiB, padded "
                        "y x z < 2^24 cells)",
                        g.n[0], g.n[1], g.n[2], C);
    return PCR_OK;
}

// The FP32 march indexes a ray's samples from its segment start with an FP32
// counter, exact below 2^24: the longest possible path through the padded
// grid must hold fewer samples than that.
pcr_status check_march_steps(const pcr_grid& g, const pcr_geom& G, pcr_dtype compute)
{
    if (compute != PCR_F32) return PCR_OK;
    double d2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double e = (g.n[a] + 3.0) * g.spacing_mm[a];
        d2 += e * e;
    }
    if (std::sqrt(d2) / G.step_mm >= 16777216.0)
        return fail(PCR_EINVAL, "step_mm %.3g too small for the FP32 march: a ray through the grid would "
                                "take 2^24 samples or more", G.step_mm);
    return PCR_OK;
}

pcr_status check_geom(const pcr_geom* G)
{
    if (!G) return fail(PCR_EINVAL, "geometry is NULL");
    const double v[] = {G->angle_rad, G->sad_mm, G->sdd_mm, G->du_mm, G->dv_mm, G->off_u_mm,
                        G->off_v_mm, G->step_mm, G->iso_mm[0], G->iso_mm[1], G->iso_mm[2]};
    for (double x : v)
        if (!std::isfinite(x)) return fail(PCR_EINVAL, "geometry has a non-finite value");
    if (!(G->sad_mm > 0)) return fail(PCR_EINVAL, "sad_mm must be > 0");
    if (!(G->sdd_mm > G->sad_mm)) return fail(PCR_EINVAL, "sdd_mm must exceed sad_mm");
    if (G->nu <= 0 || G->nv <= 0) return fail(PCR_EINVAL, "detector size must be > 0");
    if ((double)G->nu * G->nv > 1.0e8) return fail(PCR_EINVAL, "detector too large");
    if (!(G->du_mm > 0) || !(G->dv_mm > 0)) return fail(PCR_EINVAL, "pixel pitch must be > 0");
    if (!(G->step_mm > 0)) return fail(PCR_EINVAL, "step_mm must be > 0");
    double L = std::sqrt(G->sdd_mm * G->sdd_mm + 0.25 * (G->nu * G->du_mm) * (G->nu * G->du_mm) +
                         0.25 * (G->nv * G->dv_mm) * (G->nv * G->dv_mm)) +
               std::fabs(G->off_u_mm) + std::fabs(G->off_v_mm);
    if (L / G->step_mm > 2.0e9) return fail(PCR_EINVAL, "too many samples per ray");
    return PCR_OK;
}

pcr_status check_compute(pcr_dtype d)
{
    if (d != PCR_F32 && d != PCR_F64) return fail(PCR_EINVAL, "compute dtype must be F32 or F64");
    return PCR_OK;
}

pcr_status check_storage(pcr_dtype d)
{
    if (dtype_size(d) == 0) return fail(PCR_EINVAL, "unknown dtype %d", (int)d);
    return PCR_OK;
}

pcr_status check_model(const pcr_model* m)
{
    if (!m) return fail(PCR_EINVAL, "model is NULL");
    if (m->K < 1 || m->K > 8) return fail(PCR_EINVAL, "model K = %d must be in 1..8", m->K);
    PCR_TRY(check_storage(m->storage));
    if (!m->mean || !m->U) return fail(PCR_EINVAL, "model fields are NULL");
    if (m->scale)
        for (int k = 0; k < m->K; ++k)
            if (!std::isfinite(m->scale[k])) return fail(PCR_EINVAL, "model scale must be finite");
    return PCR_OK;
}

pcr_status check_finite(const double* v, int n, const char* what)
{
    if (!v) return fail(PCR_EINVAL, "%s is NULL", what);
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) return fail(PCR_EINVAL, "%s[%d] is not finite", what, i);
    return PCR_OK;
}

pcr_status check_opts(const pcr_solve_opts* o)
{
    if (!o) return fail(PCR_EINVAL, "opts is NULL");
    if (o->max_iter < 0 || o->max_backtracks < 1) return fail(PCR_EINVAL, "bad iteration limits");
    if (!(o->sigma > 0 && o->sigma < 1)) return fail(PCR_EINVAL, "sigma must be in (0, 1)");
    if (!(o->beta > 0 && o->beta < 1)) return fail(PCR_EINVAL, "beta must be in (0, 1)");
    if (!(o->eps_g >= 0) || !std::isfinite(o->eps_g)) return fail(PCR_EINVAL, "bad eps_g");
    if (!(o->fixed_mu >= 0) || !std::isfinite(o->fixed_mu)) return fail(PCR_EINVAL, "bad fixed_mu");
    if (!(o->mu0 >= 0) || !std::isfinite(o->mu0)) return fail(PCR_EINVAL, "bad mu0");
    if (o->fixed_mu == 0 && !(o->step0 > 0 && std::isfinite(o->step0)))
        return fail(PCR_EINVAL, "step0 must be > 0");
    if (o->grad_mode != PCR_GRAD_FUSED && o->grad_mode != PCR_GRAD_ADJOINT)
        return fail(PCR_EINVAL, "unknown grad_mode %d", o->grad_mode);
    if (o->step_rule != PCR_STEP_SECANT && o->step_rule != PCR_STEP_QUADRATIC)
        return fail(PCR_EINVAL, "unknown step_rule %d", o->step_rule);
    if (o->localize) {
        PCR_TRY(check_finite(o->p_ref_mm, 3, "p_ref_mm"));
        if (!(o->fp_tol_mm > 0) || o->fp_max_iter < 1) return fail(PCR_EINVAL, "bad fixed-point options");
    }
    return PCR_OK;
}

// ------------------------------------------------------- device scratch --
pcr_status DevBuf::ensure(size_t need, int dev, hipStream_t s)
{
    need = (need + 255) & ~(size_t)255;
    if (p && bytes >= need && device == dev) return PCR_OK;
    if (p) {
        HIP_TRY(hipStreamSynchronize(s));
        HIP_TRY(hipFree(p));
        p = nullptr;
        bytes = 0;
    }
    HIP_TRY(hipMalloc(&p, need));
    bytes = need;
    device = dev;
    return PCR_OK;
}

void DevBuf::release()
{
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
}

pcr_status HostBuf::ensure(size_t need)
{
    if (p && n >= need) return PCR_OK;
    if (p) HIP_TRY(hipHostFree(p));
    p = d = nullptr;
    n = 0;
    HIP_TRY(hipHostMalloc((void**)&p, need * sizeof(double), hipHostMallocCoherent | hipHostMallocMapped));
    std::memset(p, 0, need * sizeof(double));
    hipError_t e = hipHostGetDevicePointer((void**)&d, p, 0);
    if (e != hipSuccess) {
        (void)hipHostFree(p);
        p = d = nullptr;
        return fail(PCR_EDEVICE, "host staging: %s", hipGetErrorString(e));
    }
    n = need;
    return PCR_OK;
}

void HostBuf::release()
{
    if (p) (void)hipHostFree(p);
    p = d = nullptr;
    n = 0;
}

void Scratch::release()
{
    volc.release();
    vol1.release();
    acc1.release();
    p.release();
    partials.release();
    moments.release();
    host.release();
}

// ----------------------------------------------------------- profiler ----
// Opt-in per-kernel timing: every launch of the library is bracketed by two
// HIP events on the stream it runs on; durations are resolved when read.
namespace prof {
static const char* kNames[NKERN] = {"warp_fused", "march", "reduce", "backproject", "contract",
                                    "localize", "zero", "pad", "unpad", "compose", "warp",
                                    "warp_adjoint", "pca_gram", "pca_fields"};
struct Rec {
    hipEvent_t a, b;
    int id;
};
static std::mutex mu;
static bool enabled = false;
static uint32_t mask = 0xffffffffu;
static std::vector<Rec> pending;
static std::vector<hipEvent_t> pool;
static double total_ms[NKERN];
static long long counts[NKERN];
static long long dropped = 0;

static hipEvent_t get_event()
{
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

Scope::Scope(int id_, hipStream_t s_) : s(s_), id(id_)
{
    std::lock_guard<std::mutex> lk(mu);
    if (!enabled || !((mask >> id) & 1u)) return;
    a = get_event();
    if (a && hipEventRecord(a, s) != hipSuccess) {
        pool.push_back(a);
        a = nullptr;
    }
}

Scope::~Scope()
{
    if (!a) return;
    std::lock_guard<std::mutex> lk(mu);
    hipEvent_t b = get_event();
    if (!b || hipEventRecord(b, s) != hipSuccess) {
        pool.push_back(a);
        if (b) pool.push_back(b);
        ++dropped;
        return;
    }
    pending.push_back({a, b, id});
}

static void flush_locked()
{
    for (auto& r : pending) {
        float ms = 0.f;
        if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            total_ms[r.id] += ms;
            counts[r.id] += 1;
        } else {
            ++dropped;
        }
        pool.push_back(r.a);
        pool.push_back(r.b);
    }
    pending.clear();
}
}  // namespace prof

// ------------------------------------------------------------ evaluator --
pcr_status Evaluator::prepare(const void* y_, const pcr_geom& G, int mode_)
{
    PCR_TRY(check_march_image(*grid, mode_ == PCR_GRAD_FUSED ? channels_for(model->K + 1) : 1, compute));
    PCR_TRY(check_march_steps(*grid, G, compute));
    y = y_;
    mode = mode_;
    rg = make_ray_geom(*grid, G);
    ms = choose_march_shape(rg);
    M = G.nu * G.nv;
    blocks = march_blocks(rg, ms);
    const bool yfast = prefer_yfast(G);
    const int Cc = channels_for(model->K + 1);
    const size_t esz = dtype_size(compute);
    sc->Lc = make_pad(*grid, Cc, yfast);
    // FP16 fused image on request: half the bytes per tap for the march,
    // FP32 arithmetic and FP64 moments; the channel scales need the bounds
    // the support pass records
    if (image_f16 && compute == PCR_F32 && sup && sup->valid) {
        sc->Lc = make_pad(*grid, channels_for_half(model->K + 1), yfast);
        sc->Lc.half = true;
        half_scales(*sup, *grid, model->K, sc->Lc.hs);
    }
    sc->L1 = make_pad(*grid, 1);
    rgc = make_ray_geom(*grid, G, yfast);
    msc = choose_march_shape(rgc);
    blocksc = march_blocks(rgc, msc);
    const int dev = sc->device;
    if (mode == PCR_GRAD_FUSED) {
        const size_t need = sc->Lc.cells() * sc->Lc.cell_bytes(esz);
        bool fresh = sc->volc.p == nullptr || sc->volc.bytes < need;
        PCR_TRY(sc->volc.ensure(std::max(need, sc->volc_floor), dev, s));
        if (fresh || !sc->volc_zeroed || !sc->volc_layout.same_storage(sc->Lc)) {
            // border cells of one layout (grid, channel count, element
            // type, axis order) are interior cells of another; only this
            // layout's cells are read (a serving slot's buffer is sized for
            // its largest stream)
            PROF(ZERO, s);
            HIP_TRY(launch_zero(sc->volc.p, need, s));
            sc->volc_layout = sc->Lc;
            sc->volc_zeroed = true;
        }
    } else {
        size_t b1 = sc->L1.cells() * esz;
        bool fresh = sc->vol1.p == nullptr || sc->vol1.bytes < b1;
        PCR_TRY(sc->vol1.ensure(b1, dev, s));
        if (fresh) {
            PROF(ZERO, s);
            HIP_TRY(launch_zero(sc->vol1.p, sc->vol1.bytes, s));
        }
        PCR_TRY(sc->acc1.ensure((size_t)grid->n[0] * grid->n[1] * grid->n[2] * esz, dev, s));
        PCR_TRY(sc->p.ensure((size_t)M * esz, dev, s));
    }
    int cblocks = contract_blocks(*grid);
    PCR_TRY(sc->partials.ensure((size_t)std::max(std::max(blocks, blocksc), cblocks) * kMaxMoments *
                                    sizeof(double),
                                dev, s));
    PCR_TRY(sc->moments.ensure(kMaxMoments * sizeof(double), dev, s));
    PCR_TRY(sc->host.ensure(kHostSlots));
    return PCR_OK;
}

pcr_status compute_support(const pcr_grid& g, const pcr_model& m, pcr_dtype f0_dtype,
                           const void* f0, int device, hipStream_t s, Support* out)
{
    const int rows = 3 + 3 * m.K;   // then one more: max |f0|
    const int nz = g.n[2];
    const size_t sl_bytes = ((size_t)8 * nz * sizeof(int) + 255) / 256 * 256;
    DevBuf d;
    PCR_TRY(d.ensure(sl_bytes + (rows + 1) * sizeof(float), device, s));
    std::vector<int> sl((size_t)8 * nz);
    for (size_t e = 0; e < sl.size(); ++e) sl[e] = (e & 1) ? INT_MIN : INT_MAX;
    float mx[28] = {0};
    float* dmx = (float*)((char*)d.p + sl_bytes);
    auto fin = [&](pcr_status e) {
        d.release();
        return e;
    };
    const size_t N = (size_t)g.n[0] * g.n[1] * nz;
    hipError_t he = hipMemcpyAsync(d.p, sl.data(), sl.size() * sizeof(int), hipMemcpyHostToDevice, s);
    if (he == hipSuccess) he = hipMemcpyAsync(dmx, mx, (rows + 1) * sizeof(float), hipMemcpyHostToDevice, s);
    if (he == hipSuccess) he = launch_support(f0_dtype, g, f0, (int*)d.p, s);
    if (he == hipSuccess) he = launch_absmax_rows(m.storage, m.mean, N, 3, dmx, s);
    if (he == hipSuccess) he = launch_absmax_rows(m.storage, m.U, N, 3 * m.K, dmx + 3, s);
    if (he == hipSuccess) he = launch_absmax_rows(f0_dtype, f0, N, 1, dmx + rows, s);
    if (he == hipSuccess) he = hipMemcpyAsync(sl.data(), d.p, sl.size() * sizeof(int), hipMemcpyDeviceToHost, s);
    if (he == hipSuccess) he = hipMemcpyAsync(mx, dmx, (rows + 1) * sizeof(float), hipMemcpyDeviceToHost, s);
    if (he == hipSuccess) he = hipStreamSynchronize(s);
    if (he != hipSuccess) return fin(fail(PCR_EDEVICE, "support pass: %s", hipGetErrorString(he)));
    // the box: the union of the slices
    for (int a = 0; a < 3; ++a) {
        out->lo[a] = INT_MAX;
        out->hi[a] = INT_MIN;
    }
    for (int z = 0; z < nz; ++z) {
        const int* q = &sl[(size_t)8 * z];
        if (q[0] > q[1]) continue;
        out->lo[0] = std::min(out->lo[0], q[0]);
        out->hi[0] = std::max(out->hi[0], q[1]);
        out->lo[1] = std::min(out->lo[1], q[2]);
        out->hi[1] = std::max(out->hi[1], q[3]);
        out->lo[2] = std::min(out->lo[2], z);
        out->hi[2] = std::max(out->hi[2], z);
    }
    for (int a = 0; a < 3; ++a) {
        out->mmax[a] = mx[a];
        for (int k = 0; k < 8; ++k) out->umax[k][a] = k < m.K ? mx[3 + 3 * k + a] : 0.0;
    }
    out->f0max = mx[rows];
    // slabs of at most 16 per volume, at least 4 slices thick; a ray meets
    // those within its z range plus the dilation
    const int T = std::max(4, (nz + 15) / 16);
    const int ns = (nz + T - 1) / T;
    std::vector<float> tab((size_t)20 * ns);
    for (int sb = 0; sb < ns; ++sb) {
        int b[8] = {INT_MAX, INT_MIN, INT_MAX, INT_MIN, INT_MAX, INT_MIN, INT_MAX, INT_MIN};
        int klo = INT_MAX, khi = INT_MIN;
        for (int z = sb * T; z < std::min(nz, (sb + 1) * T); ++z) {
            const int* q = &sl[(size_t)8 * z];
            if (q[0] > q[1]) continue;
            for (int c = 0; c < 4; ++c) {
                b[2 * c] = std::min(b[2 * c], q[2 * c]);
                b[2 * c + 1] = std::max(b[2 * c + 1], q[2 * c + 1]);
            }
            klo = std::min(klo, z);
            khi = std::max(khi, z);
        }
        float* t = &tab[(size_t)10 * sb];            // x-fastest order (i = x)
        float* u = &tab[(size_t)10 * (ns + sb)];     // y-fastest order (i = y)
        if (klo > khi) {
            for (int c = 0; c < 10; ++c) t[c] = u[c] = 0.0f;
            t[8] = u[8] = 1.0f;   // empty: k lo > k hi
            continue;
        }
        const float v[10] = {(float)b[0], (float)b[1], (float)b[2], (float)b[3], (float)b[4],
                             (float)b[5], (float)b[6], (float)b[7], (float)klo, (float)khi};
        for (int c = 0; c < 10; ++c) t[c] = v[c];
        const float w[10] = {v[2], v[3], v[0], v[1], v[4], v[5], -v[7], -v[6], v[8], v[9]};
        for (int c = 0; c < 10; ++c) u[c] = w[c];
    }
    d.release();
    PCR_TRY(out->slab_buf.ensure(tab.size() * sizeof(float), device, s));
    HIP_TRY(hipMemcpyAsync(out->slab_buf.p, tab.data(), tab.size() * sizeof(float),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    out->nslab = ns;
    out->slab_t = T;
    out->valid = true;
    return PCR_OK;
}

void half_scales(const Support& sp, const pcr_grid& g, int K, float hs[8])
{
    auto pow2_for = [](double bound) {
        // largest power of two with bound * scale <= 2^14 (FP16 max 65504)
        if (!(bound > 0.0) || !std::isfinite(bound)) return 1.0f;
        int e = (int)std::floor(std::log2(16384.0 / bound));
        e = std::max(-100, std::min(100, e));
        return (float)std::ldexp(1.0, e);
    };
    for (int c = 0; c < 8; ++c) hs[c] = 1.0f;
    hs[0] = pow2_for(sp.f0max);
    for (int k = 0; k < K && k < 7; ++k) {
        double b = 0.0;
        for (int a = 0; a < 3; ++a) b += sp.umax[k][a] / g.spacing_mm[a];
        hs[k + 1] = pow2_for(2.0 * sp.f0max * b);
    }
}

// Half-widths (voxels) of the dilation: the displacement bound along each
// axis, with room for the FP32 rounding of the displacements, plus 2.5 cells
// (one for the trilinear taps of f0, one for those of the sample, a half
// for rounding).
static void dilation(const Support& sp, const pcr_grid& g, int K, const double* w_eff, double h[3])
{
    for (int a = 0; a < 3; ++a) {
        double d = sp.mmax[a];
        for (int k = 0; k < K; ++k) d += std::fabs(w_eff[k]) * sp.umax[k][a];
        h[a] = d * 1.0001 / g.spacing_mm[a] + 2.5;
    }
}

void clip_box(const Support& sp, const pcr_grid& g, int K, const double* w_eff, bool swap_xy,
              double clo[3], double chi[3])
{
    for (int a = 0; a < 3; ++a) {
        if (sp.lo[a] > sp.hi[a]) {   // f0 is zero: so is every projection
            clo[0] = clo[1] = clo[2] = chi[0] = chi[1] = chi[2] = -1.0;
            return;
        }
    }
    double h[3];
    dilation(sp, g, K, w_eff, h);
    for (int a = 0; a < 3; ++a) {
        clo[a] = std::max(-1.0, (double)sp.lo[a] - h[a]);
        chi[a] = std::min((double)g.n[a], (double)sp.hi[a] + h[a]);
    }
    if (swap_xy) {
        std::swap(clo[0], clo[1]);
        std::swap(chi[0], chi[1]);
    }
}

void clip_geom(const Support& sp, const pcr_grid& g, int K, const double* w_eff, bool swap_xy,
               RayGeom& rg)
{
    clip_box(sp, g, K, w_eff, swap_xy, rg.clo, rg.chi);
    if (sp.lo[0] > sp.hi[0] || sp.nslab == 0 || !sp.slab_buf.p) return;
    double h[3];
    dilation(sp, g, K, w_eff, h);
    if (swap_xy) std::swap(h[0], h[1]);
    rg.slabs = (const float*)sp.slab_buf.p + (swap_xy ? 10 * sp.nslab : 0);
    rg.nslab = sp.nslab;
    rg.slab_t = sp.slab_t;
    for (int a = 0; a < 3; ++a) rg.h[a] = (float)h[a];
}

void warp_box(const RayGeom& g, const pcr_grid& grid, int box[6])
{
    for (int a = 0; a < 3; ++a) {
        // a ray's samples lie within one step (dt / s_a voxels) of the clip
        // box; each reads the cells floor(q) and floor(q) + 1; one more cell
        // on each side covers the FP32 rounding of the sample positions
        const double e = g.dt / g.sp[a];
        box[a] = std::max(0, (int)std::floor(g.clo[a] - e) - 1);
        box[3 + a] = std::min(grid.n[a], (int)std::floor(g.chi[a] + e) + 3);
    }
}

pcr_status Evaluator::enqueue_eval(const double* w)
{
    double w_eff[8];
    effective_w(*model, w, w_eff);
    const int K = model->K;
    const int kc = mode == PCR_GRAD_FUSED ? K + 1 : 1;
    // the final sum writes the moments straight into the host staging and
    // then publishes this evaluation's sequence number there
    double* mom = sc->host.d;
    unsigned long long* done = (unsigned long long*)(sc->host.d + kDoneSlot);
    const unsigned long long seq = ++sc->seq;
    RayGeom gc = rgc, g1 = rg;
    int vbox[6];
    const int* box = nullptr;
    if (sup && sup->valid) {
        clip_geom(*sup, *grid, K, w_eff, sc->Lc.yfast, gc);
        clip_geom(*sup, *grid, K, w_eff, false, g1);
        warp_box(g1, *grid, vbox);
        box = vbox;
    }
    if (mode == PCR_GRAD_FUSED) {
        {
            PROF(WARP, s);
            HIP_TRY(launch_warp_fused(compute, model->storage, f0_dtype, *grid, sc->Lc, K, true, f0,
                                      model->mean, model->U, w_eff, box, sc->volc.p, s));
        }
        {
            PROF(MARCH, s);
            HIP_TRY(launch_march(compute, sc->Lc, kc, gc, msc, sc->volc.p, y, nullptr,
                                 (double*)sc->partials.p, mom, done, seq, s));
        }
    } else {
        {
            PROF(WARP, s);
            HIP_TRY(launch_warp_fused(compute, model->storage, f0_dtype, *grid, sc->L1, K, false, f0,
                                      model->mean, model->U, w_eff, box, sc->vol1.p, s));
        }
        {
            PROF(MARCH, s);
            HIP_TRY(launch_march(compute, sc->L1, 1, g1, ms, sc->vol1.p, y, sc->p.p,
                                 (double*)sc->partials.p, mom, done, seq, s));
        }
    }
    return PCR_OK;
}

pcr_status Evaluator::wait_published()
{
    const unsigned long long* done = (const unsigned long long*)(sc->host.p + kDoneSlot);
    const unsigned long long want = sc->seq;
    for (unsigned long n = 1;; ++n) {
        if (__atomic_load_n(done, __ATOMIC_ACQUIRE) == want) return PCR_OK;
        if ((n & 4095) == 0) {
            // now and then: has the stream failed, or finished without
            // publishing (which would be a bug)?
            const hipError_t q = hipStreamQuery(s);
            if (q == hipSuccess) {
                if (__atomic_load_n(done, __ATOMIC_ACQUIRE) == want) return PCR_OK;
                return fail(PCR_EDEVICE, "evaluation finished without publishing its moments");
            }
            if (q != hipErrorNotReady) return fail(PCR_EDEVICE, "evaluation: %s", hipGetErrorString(q));
        }
        __builtin_ia32_pause();
    }
}

void Evaluator::collect(Moments& out) const
{
    const int kc = mode == PCR_GRAD_FUSED ? model->K + 1 : 1;
    std::memset(out.m, 0, sizeof out.m);
    std::memcpy(out.m, sc->host.p, n_moments(kc) * sizeof(double));
    out.samples = sc->host.p[n_moments(kc)];
    out.M = (double)M;
    out.K = model->K;
}

pcr_status Evaluator::eval_sync(const double* w, Moments& out)
{
    PCR_TRY(enqueue_eval(w));
    PCR_TRY(wait_published());
    collect(out);
    return PCR_OK;
}

pcr_status Evaluator::grad_adjoint(const double* w, double a, double b, double* grad)
{
    double w_eff[8];
    effective_w(*model, w, w_eff);
    const int K = model->K;
    {
        PROF(BACKPROJ, s);
        HIP_TRY(launch_backproject(compute, *grid, rg, nullptr, sc->p.p, y, a, b, 2.0, sc->acc1.p, s));
    }
    {
        PROF(CONTRACT, s);
        HIP_TRY(launch_contract(compute, model->storage, f0_dtype, *grid, K, f0, model->mean, model->U,
                                w_eff, sc->acc1.p, (double*)sc->partials.p, s));
    }
    {
        PROF(REDUCE, s);
        HIP_TRY(launch_reduce((const double*)sc->partials.p, contract_blocks(*grid), K,
                              (double*)sc->moments.p, s));
    }
    HIP_TRY(hipMemcpyAsync(sc->host.p, sc->moments.p, K * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int k = 0; k < K; ++k) grad[k] = sc->host.p[k];
    return PCR_OK;
}

}  // namespace pcr

// Per-thread scratch of the stateless entry points.
namespace {
struct TlsScratch {
    DevBuf pad, small;
    HostBuf host;
    ~TlsScratch()
    {
        pad.release();
        small.release();
        host.release();
    }
};
thread_local TlsScratch tls;

pcr_status current_device(int* dev)
{
    HIP_TRY(hipGetDevice(dev));
    return PCR_OK;
}

// Device array of the allocation-free projection (pcr_forward_project_noalloc).
// Its name is a host-side stand-in: host code uses only the device address
// looked up per device, never the name itself.
static __device__ __align__(256) unsigned char scratch[PCR_NOALLOC_SCRATCH_BYTES];
constexpr int kMaxScratchDevices = 64;
std::mutex scratch_mu;
void* scratch_dev_ptr[kMaxScratchDevices];

// The address of `scratch` on the current device `dev`, looked up on the
// first call there.
pcr_status scratch_on_device(int dev, void** out)
{
    if (dev < 0 || dev >= kMaxScratchDevices)
        return fail(PCR_EDEVICE, "device %d beyond the %d devices the fixed scratch table covers", dev,
                    kMaxScratchDevices);
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_dev_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return fail(PCR_EDEVICE, "scratch address on device %d: %s", dev, hipGetErrorString(e));
        if (!p) return fail(PCR_EDEVICE, "scratch address on device %d is null", dev);
        scratch_dev_ptr[dev] = p;
    }
    *out = scratch_dev_ptr[dev];
    return PCR_OK;
}

struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) == hipSuccess && (prev == dev || hipSetDevice(dev) == hipSuccess)) ok = true;
    }
    ~DeviceGuard()
    {
        if (ok && prev >= 0) (void)hipSetDevice(prev);
    }
};
}  // namespace

// ============================================================ C ABI =======
extern "C" {

const char* pcr_version(void) { return PCR_VERSION_STRING; }
const char* pcr_last_error(void) { return pcr::g_err.c_str(); }

void pcr_profile_enable(int32_t on)
{
    std::lock_guard<std::mutex> lk(prof::mu);
    prof::flush_locked();
    if (on) {
        for (int i = 0; i < prof::NKERN; ++i) {
            prof::total_ms[i] = 0.0;
            prof::counts[i] = 0;
        }
        prof::dropped = 0;
    }
    prof::enabled = on != 0;
}

void pcr_profile_select(uint32_t mask)
{
    std::lock_guard<std::mutex> lk(prof::mu);
    prof::mask = mask;
}

int32_t pcr_profile_read(int32_t max, const char** names, double* total_ms, int64_t* counts)
{
    std::lock_guard<std::mutex> lk(prof::mu);
    prof::flush_locked();
    int n = std::min<int>(max, prof::NKERN);
    for (int i = 0; i < n; ++i) {
        if (names) names[i] = prof::kNames[i];
        if (total_ms) total_ms[i] = prof::total_ms[i];
        if (counts) counts[i] = prof::counts[i];
    }
    return prof::NKERN;
}

void pcr_solve_opts_default(pcr_solve_opts* o)
{
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->max_iter = 50;
    o->max_backtracks = 30;
    o->sigma = 1e-4;
    o->beta = 0.5;
    o->eps_g = 1e-4;
    o->step0 = 1.0;
    o->fixed_mu = 0.0;
    o->grad_mode = PCR_GRAD_FUSED;
    o->localize = 0;
    o->fp_tol_mm = 1e-6;
    o->fp_max_iter = 200;
    o->step_rule = PCR_STEP_SECANT;
}

pcr_status pcr_dvf_compose(const pcr_grid* grid, const pcr_model* model, const double* w_host,
                           pcr_dtype compute, void* dvf_dev, void* stream)
{
    PCR_TRY(check_grid(grid));
    PCR_TRY(check_model(model));
    PCR_TRY(check_compute(compute));
    PCR_TRY(check_finite(w_host, model->K, "w"));
    if (!dvf_dev) return fail(PCR_EINVAL, "dvf_dev is NULL");
    double w_eff[8];
    effective_w(*model, w_host, w_eff);
    hipStream_t s = (hipStream_t)stream;
    PROF(COMPOSE, s);
    HIP_TRY(launch_compose(compute, model->storage, *grid, model->K, model->mean, model->U, w_eff,
                           dvf_dev, s));
    return PCR_OK;
}

pcr_status pcr_warp_volume(const pcr_grid* grid, pcr_dtype f0_dtype, const void* f0_dev,
                           pcr_dtype compute, const void* dvf_dev, void* f_dev, void* stream)
{
    PCR_TRY(check_grid(grid));
    PCR_TRY(check_storage(f0_dtype));
    PCR_TRY(check_compute(compute));
    if (!f0_dev || !dvf_dev || !f_dev) return fail(PCR_EINVAL, "NULL device pointer");
    if (f_dev == f0_dev) return fail(PCR_EINVAL, "f_dev must not alias f0_dev");
    hipStream_t s = (hipStream_t)stream;
    PROF(WARP_PLAIN, s);
    HIP_TRY(launch_warp_plain(compute, f0_dtype, *grid, f0_dev, dvf_dev, f_dev, s));
    return PCR_OK;
}

pcr_status pcr_warp_adjoint(const pcr_grid* grid, pcr_dtype compute, const void* dvf_dev,
                            const void* g_dev, void* out_dev, void* stream)
{
    PCR_TRY(check_grid(grid));
    PCR_TRY(check_compute(compute));
    if (!dvf_dev || !g_dev || !out_dev) return fail(PCR_EINVAL, "NULL device pointer");
    size_t N = (size_t)grid->n[0] * grid->n[1] * grid->n[2];
    hipStream_t s = (hipStream_t)stream;
    {
        PROF(ZERO, s);
        HIP_TRY(launch_zero(out_dev, N * dtype_size(compute), s));
    }
    PROF(WARP_ADJ, s);
    HIP_TRY(launch_warp_adjoint(compute, *grid, dvf_dev, g_dev, out_dev, s));
    return PCR_OK;
}

pcr_status pcr_forward_project(const pcr_grid* grid, const pcr_geom* geom, pcr_dtype compute,
                               const void* vol_dev, void* proj_dev, void* stream)
{
    PCR_TRY(check_grid(grid));
    PCR_TRY(check_geom(geom));
    PCR_TRY(check_compute(compute));
    if (!vol_dev || !proj_dev) return fail(PCR_EINVAL, "NULL device pointer");
    PCR_TRY(check_march_image(*grid, 1, compute));
    PCR_TRY(check_march_steps(*grid, *geom, compute));
    hipStream_t s = (hipStream_t)stream;
    int dev;
    PCR_TRY(current_device(&dev));
    PadLayout L = make_pad(*grid, 1);
    size_t bytes = L.cells() * dtype_size(compute);
    PCR_TRY(tls.pad.ensure(bytes, dev, s));
    {
        PROF(ZERO, s);
        HIP_TRY(launch_zero(tls.pad.p, bytes, s));
    }
    {
        PROF(PAD, s);
        HIP_TRY(launch_pad(compute, L, vol_dev, tls.pad.p, s));
    }
    RayGeom rg = make_ray_geom(*grid, *geom);
    MarchShape ms = choose_march_shape(rg);
    PROF(MARCH, s);
    HIP_TRY(launch_march(compute, L, 1, rg, ms, tls.pad.p, nullptr, proj_dev, nullptr, nullptr, nullptr, 0,
                         s));
    return PCR_OK;
}

pcr_status pcr_forward_project_noalloc(const pcr_grid* grid, const pcr_geom* geom, pcr_dtype compute,
                                       const void* vol_dev, void* proj_dev, void* stream)
{
    PCR_TRY(check_grid(grid));
    PCR_TRY(check_geom(geom));
    PCR_TRY(check_compute(compute));
    if (!vol_dev || !proj_dev) return fail(PCR_EINVAL, "NULL device pointer");
    PCR_TRY(check_march_image(*grid, 1, compute));
    PCR_TRY(check_march_steps(*grid, *geom, compute));
    PadLayout L = make_pad(*grid, 1);
    const size_t bytes = L.cells() * dtype_size(compute);
    if (bytes > PCR_NOALLOC_SCRATCH_BYTES)
        return fail(PCR_EINVAL,
                    "grid (%d, %d, %d): the padded copy needs %zu bytes, more than the %zu bytes of "
                    "the fixed scratch array",
                    grid->n[0], grid->n[1], grid->n[2], bytes, (size_t)PCR_NOALLOC_SCRATCH_BYTES);
    hipStream_t s = (hipStream_t)stream;
    int dev;
    PCR_TRY(current_device(&dev));
    void* pad = nullptr;
    PCR_TRY(scratch_on_device(dev, &pad));
    // the array keeps the previous call's contents: clear the border cells
    HIP_TRY(launch_zero(pad, bytes, s));
    HIP_TRY(launch_pad(compute, L, vol_dev, pad, s));
    RayGeom rg = make_ray_geom(*grid, *geom);
    MarchShape ms = choose_march_shape(rg);
    HIP_TRY(launch_march(compute, L, 1, rg, ms, pad, nullptr, proj_dev, nullptr, nullptr, nullptr, 0, s));
    return PCR_OK;
}

pcr_status pcr_backproject_residual(const pcr_grid* grid, const pcr_geom* geom, pcr_dtype compute,
                                    const void* resid_dev, void* vol_dev, void* stream)
{
    PCR_TRY(check_grid(grid));
    PCR_TRY(check_geom(geom));
    PCR_TRY(check_compute(compute));
    if (!resid_dev || !vol_dev) return fail(PCR_EINVAL, "NULL device pointer");
    hipStream_t s = (hipStream_t)stream;
    RayGeom rg = make_ray_geom(*grid, *geom);
    PROF(BACKPROJ, s);
    HIP_TRY(launch_backproject(compute, *grid, rg, resid_dev, nullptr, nullptr, 0.0, 0.0, 1.0, vol_dev, s));
    return PCR_OK;
}

pcr_status pcr_warp_contract(const pcr_grid* grid, const pcr_model* model, pcr_dtype f0_dtype,
                             const void* f0_dev, const double* w_host, pcr_dtype compute,
                             const void* g_dev, double* grad_host, void* stream)
{
    PCR_TRY(check_grid(grid));
    PCR_TRY(check_model(model));
    PCR_TRY(check_storage(f0_dtype));
    PCR_TRY(check_compute(compute));
    PCR_TRY(check_finite(w_host, model->K, "w"));
    if (!f0_dev || !g_dev || !grad_host) return fail(PCR_EINVAL, "NULL pointer");
    hipStream_t s = (hipStream_t)stream;
    int dev;
    PCR_TRY(current_device(&dev));
    const int nb = contract_blocks(*grid);
    PCR_TRY(tls.pad.ensure((size_t)nb * 8 * sizeof(double) + 8 * sizeof(double), dev, s));
    PCR_TRY(tls.host.ensure(8));
    double w_eff[8];
    effective_w(*model, w_host, w_eff);
    double* part = (double*)tls.pad.p;
    double* out = part + (size_t)nb * 8;
    {
        PROF(CONTRACT, s);
        HIP_TRY(launch_contract(compute, model->storage, f0_dtype, *grid, model->K, f0_dev, model->mean,
                                model->U, w_eff, g_dev, part, s));
    }
    {
        PROF(REDUCE, s);
        HIP_TRY(launch_reduce(part, nb, model->K, out, s));
    }
    HIP_TRY(hipMemcpyAsync(tls.host.p, out, model->K * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int k = 0; k < model->K; ++k) grad_host[k] = tls.host.p[k] * (model->scale ? model->scale[k] : 1.0);
    return PCR_OK;
}

pcr_status pcr_predict_w(const double* w_hist, const double* t_hist, int32_t n, int32_t K,
                         double t_next, int32_t order, double* w_out)
{
    if (!w_hist || !t_hist || !w_out) return fail(PCR_EINVAL, "NULL argument");
    if (n < 1 || K < 1 || K > 8 || order < 0 || order > 2) return fail(PCR_EINVAL, "bad n, K or order");
    PCR_TRY(check_finite(w_hist, n * K, "w_hist"));
    PCR_TRY(check_finite(t_hist, n, "t_hist"));
    if (!std::isfinite(t_next)) return fail(PCR_EINVAL, "t_next must be finite");
    const int d = std::min(order, n - 1);
    const int first = n - 1 - d;
    for (int i = first + 1; i < n; ++i)
        if (!(t_hist[i] > t_hist[i - 1])) return fail(PCR_EINVAL, "t_hist must increase");
    sched::extrapolate_w(w_hist, t_hist, n, K, t_next, order, w_out);
    return PCR_OK;
}

pcr_status pcr_localize_tumor(const pcr_grid* grid, const pcr_model* model, const double* w_host,
                              const double p_ref_mm[3], double tol_mm, int32_t max_iter,
                              double p_out_mm[3], int32_t* iters, void* stream)
{
    PCR_TRY(check_grid(grid));
    PCR_TRY(check_model(model));
    PCR_TRY(check_finite(w_host, model->K, "w"));
    PCR_TRY(check_finite(p_ref_mm, 3, "p_ref_mm"));
    if (!p_out_mm) return fail(PCR_EINVAL, "p_out_mm is NULL");
    if (!(tol_mm > 0) || max_iter < 1) return fail(PCR_EINVAL, "need tol_mm > 0 and max_iter >= 1");
    hipStream_t s = (hipStream_t)stream;
    int dev;
    PCR_TRY(current_device(&dev));
    PCR_TRY(tls.small.ensure(8 * sizeof(double), dev, s));
    PCR_TRY(tls.host.ensure(8));
    double w_eff[8];
    effective_w(*model, w_host, w_eff);
    {
        PROF(LOCALIZE, s);
        HIP_TRY(launch_localize(model->storage, *grid, model->K, model->mean, model->U, w_eff, p_ref_mm,
                                tol_mm, max_iter, (double*)tls.small.p, s));
    }
    HIP_TRY(hipMemcpyAsync(tls.host.p, tls.small.p, 5 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int a = 0; a < 3; ++a) p_out_mm[a] = tls.host.p[a];
    if (iters) *iters = (int32_t)tls.host.p[3];
    if (tls.host.p[4] != 1.0) return fail(PCR_EDIVERGE, "fixed point did not converge in %d iterations", max_iter);
    return PCR_OK;
}

}  // extern "C"

// ============================================================ context =====
struct pcr_ctx {
    pcr_grid grid;
    pcr_model model;
    double scale[8];
    pcr_dtype f0_dtype, compute;
    const void* f0;
    Scratch sc;
    Support sup;   // computed on the first evaluation
    bool image_f16 = false;
    ~pcr_ctx()
    {
        sc.release();
        sup.release();
    }
};

extern "C" {

pcr_status pcr_ctx_create(const pcr_grid* grid, const pcr_model* model, pcr_dtype f0_dtype,
                          const void* f0_dev, pcr_dtype compute, pcr_ctx** out)
{
    if (!out) return fail(PCR_EINVAL, "out is NULL");
    *out = nullptr;
    PCR_TRY(check_grid(grid));
    PCR_TRY(check_model(model));
    PCR_TRY(check_storage(f0_dtype));
    PCR_TRY(check_compute(compute));
    if (!f0_dev) return fail(PCR_EINVAL, "f0_dev is NULL");
    PCR_TRY(check_march_image(*grid, channels_for(model->K + 1), compute));
    pcr_ctx* c = new (std::nothrow) pcr_ctx();
    if (!c) return fail(PCR_ENOMEM, "host allocation failed");
    c->grid = *grid;
    c->model = *model;
    for (int k = 0; k < 8; ++k) c->scale[k] = (model->scale && k < model->K) ? model->scale[k] : 1.0;
    c->model.scale = model->scale ? c->scale : nullptr;
    c->f0_dtype = f0_dtype;
    c->compute = compute;
    c->f0 = f0_dev;
    pcr_status st = current_device(&c->sc.device);
    if (st != PCR_OK) {
        delete c;
        return st;
    }
    *out = c;
    return PCR_OK;
}

void pcr_ctx_destroy(pcr_ctx* ctx)
{
    if (!ctx) return;
    DeviceGuard dg(ctx->sc.device);
    (void)hipDeviceSynchronize();
    delete ctx;
}

size_t pcr_ctx_device_bytes(const pcr_ctx* c) { return c ? c->sc.device_bytes() : 0; }

pcr_status pcr_ctx_set_image_dtype(pcr_ctx* ctx, pcr_dtype dtype)
{
    if (!ctx) return fail(PCR_EINVAL, "ctx is NULL");
    if (dtype != PCR_F32 && dtype != PCR_F16) return fail(PCR_EINVAL, "image dtype must be F32 or F16");
    if (dtype == PCR_F16 && ctx->compute != PCR_F32)
        return fail(PCR_EINVAL, "an FP16 image needs FP32 compute");
    ctx->image_f16 = dtype == PCR_F16;
    return PCR_OK;
}

pcr_status pcr_cost_grad(pcr_ctx* ctx, const void* y_dev, const pcr_geom* geom,
                         const double* w_host, double a, double b, int32_t grad_mode,
                         double* cost_host, double* grad_host, void* stream)
{
    if (!ctx) return fail(PCR_EINVAL, "ctx is NULL");
    PCR_TRY(check_geom(geom));
    PCR_TRY(check_finite(w_host, ctx->model.K, "w"));
    if (!std::isfinite(a) || !std::isfinite(b)) return fail(PCR_EINVAL, "a, b must be finite");
    if (!y_dev || !cost_host || !grad_host) return fail(PCR_EINVAL, "NULL pointer");
    if (grad_mode != PCR_GRAD_FUSED && grad_mode != PCR_GRAD_ADJOINT)
        return fail(PCR_EINVAL, "unknown grad_mode %d", grad_mode);
    DeviceGuard dg(ctx->sc.device);
    if (!dg.ok) return fail(PCR_EDEVICE, "cannot select device %d", ctx->sc.device);
    if (!ctx->sup.valid)
        PCR_TRY(compute_support(ctx->grid, ctx->model, ctx->f0_dtype, ctx->f0, ctx->sc.device,
                                (hipStream_t)stream, &ctx->sup));
    Evaluator E{&ctx->grid, &ctx->model, ctx->f0_dtype, ctx->compute, ctx->f0, &ctx->sc,
                (hipStream_t)stream};
    E.sup = &ctx->sup;
    E.image_f16 = ctx->image_f16;
    PCR_TRY(E.prepare(y_dev, *geom, grad_mode));
    Moments mo;
    PCR_TRY(E.eval_sync(w_host, mo));
    *cost_host = mo.J(a, b);
    const int K = ctx->model.K;
    if (grad_mode == PCR_GRAD_FUSED) {
        for (int k = 0; k < K; ++k) grad_host[k] = mo.grad(k, a, b);
    } else {
        PCR_TRY(E.grad_adjoint(w_host, a, b, grad_host));
    }
    for (int k = 0; k < K; ++k) grad_host[k] *= ctx->scale[k];
    return PCR_OK;
}

pcr_status pcr_reconstruct_from_projection(pcr_ctx* ctx, const void* y_dev, const pcr_geom* geom,
                                           const pcr_solve_opts* opts, double* w_inout,
                                           double* ab_out, pcr_solve_stats* stats, void* stream)
{
    if (!ctx) return fail(PCR_EINVAL, "ctx is NULL");
    PCR_TRY(check_geom(geom));
    const int K = ctx->model.K;
    PCR_TRY(check_opts(opts));
    PCR_TRY(check_finite(w_inout, K, "w_inout"));
    if (!y_dev) return fail(PCR_EINVAL, "y_dev is NULL");
    DeviceGuard dg(ctx->sc.device);
    if (!dg.ok) return fail(PCR_EDEVICE, "cannot select device %d", ctx->sc.device);
    if (!ctx->sup.valid)
        PCR_TRY(compute_support(ctx->grid, ctx->model, ctx->f0_dtype, ctx->f0, ctx->sc.device,
                                (hipStream_t)stream, &ctx->sup));
    Evaluator E{&ctx->grid, &ctx->model, ctx->f0_dtype, ctx->compute, ctx->f0, &ctx->sc,
                (hipStream_t)stream};
    E.sup = &ctx->sup;
    E.image_f16 = ctx->image_f16;
    PCR_TRY(E.prepare(y_dev, *geom, opts->grad_mode));
    SolveSM sm;
    sm.begin(K, *opts, ctx->model.scale ? ctx->scale : nullptr, w_inout);
    auto gfn = [&E](const double* w, double a, double b, double* g) { return E.grad_adjoint(w, a, b, g); };
    while (!sm.done()) {
        Moments mo;
        PCR_TRY(E.eval_sync(sm.eval_w(), mo));
        PCR_TRY(sm.feed(mo, gfn));
    }
    pcr_status status = sm.status;
    if (status == PCR_EDEVICE) return fail(PCR_EDEVICE, "non-finite cost or gradient (input contains NaN/Inf?)");
    if (status == PCR_ENOCONV)
        fail(PCR_ENOCONV, "no convergence: %d iterations, %d trials", sm.iters, sm.trials);
    for (int k = 0; k < K; ++k) w_inout[k] = sm.w[k];
    if (ab_out) {
        ab_out[0] = sm.a;
        ab_out[1] = sm.b;
    }
    pcr_solve_stats st;
    sm.fill_stats(&st);
    if (opts->localize) {
        pcr_status ls = pcr_localize_tumor(&ctx->grid, &ctx->model, sm.w, opts->p_ref_mm, opts->fp_tol_mm,
                                           opts->fp_max_iter, st.tumor_mm, &st.fp_iterations, stream);
        st.fp_status = ls;
        if (ls != PCR_OK && ls != PCR_EDIVERGE) return ls;
    }
    if (stats) *stats = st;
    return status;
}

}  // extern "C"
