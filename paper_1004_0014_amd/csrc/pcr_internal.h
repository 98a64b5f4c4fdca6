// Internal interfaces between the C ABI (api.hip) and the kernels
// (kernels.hip).  Not installed; the public surface is include/pcr.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "pcr.h"

namespace pcr {

// Zero-padded multi-channel image layout used by the ray march: voxel (i,j,k)
// of an nx x ny x nz grid lives at padded cell (i+1, j+1, k+1) of a
// (nx+3) x (ny+3) x (nz+3) array whose border cells stay zero, channels
// interleaved per cell.  Sample points are clamped to the support [-1, n] of
// the interpolant per axis, so every tap of every sample is in bounds and
// samples outside the support read only zero cells.
//
// The two in-plane axes may be stored in either order: x fastest
// ([z][y][x], yfast = false) or y fastest ([z][x][y], yfast = true).  The
// march then reads a geometry with x and y swapped, so that detector rows
// (which run along e_u = (cos t, sin t, 0)) walk the fastest memory axis at
// every gantry angle.  px, py are the padded dims in memory order.
//
// Channels are stored in the compute type, or (FP32 compute, `half`) as FP16
// holding value * hs[c], with hs[c] a power of two chosen from a bound on the
// channel's magnitude so that no value overflows; the march multiplies its
// sums by 1 / hs[c] (exact).
struct PadLayout {
    int nx, ny, nz;
    int px, py, pz;      // padded dims in memory order (fast, mid, slow)
    int C;               // channel stride (1, 2, 4, 6 or 8)
    bool yfast;
    bool half = false;   // FP16 channels (FP32 compute only)
    float hs[8] = {1, 1, 1, 1, 1, 1, 1, 1};
    size_t cells() const { return (size_t)px * py * pz; }
    size_t cell_bytes(size_t compute_size) const { return (size_t)C * (half ? 2 : compute_size); }
    // same memory image: a buffer laid out for one is laid out for the other
    bool same_storage(const PadLayout& o) const
    {
        return nx == o.nx && ny == o.ny && nz == o.nz && C == o.C && yfast == o.yfast &&
               half == o.half;
    }
};
PadLayout make_pad(const pcr_grid& g, int C, bool yfast = false);
// y-fastest storage for rays close to the x axis (the detector's u axis
// close to y)
bool prefer_yfast(const pcr_geom& G);

// Per-projection ray geometry in index space, computed on the host in FP64.
// A ray from the source q_s towards pixel (iu, iv) has the index-space point
// q(t) = q_s + t * dq at distance t (mm) from the source.
struct RayGeom {
    double qs[3];        // source (index coordinates)
    double qc[3];        // detector centre (index coordinates)
    double eu[3], ev[3]; // detector axes (index units per mm)
    double sp[3];        // voxel spacing (mm)
    double lim[3];       // upper support bound n_a (the lower one is -1)
    double clo[3], chi[3]; // box the rays are clipped to: the support (-1, n_a) by
                           // default, or a tighter box outside which the
                           // image is known to be zero (no sample there
                           // contributes)
    double u0, v0;       // detector coordinate (mm) of pixel 0 along e_u, e_v
    double du, dv;       // pixel pitch (mm)
    double dt;           // sample spacing (mm)
    int nu, nv;
    // Tighter clipping within the box (null: none): per slab of slab_t
    // slices, 10 floats {i lo, hi; j lo, hi; i+j lo, hi; i-j lo, hi; k lo, hi}
    // bound the nonzero voxels of the reference image (index space, this
    // geometry's axis order; lo > hi: empty slab).  Dilated by h (i, j, k),
    // and by h_i + h_j along the diagonals, they bound where a sample can be
    // nonzero; a ray is clipped to the hull of the slabs it meets.
    const float* slabs = nullptr;
    int nslab = 0, slab_t = 1;
    float h[3] = {0.0f, 0.0f, 0.0f};
};
// swap_xy: express the geometry in (y, x, z) index order (y-fastest layout).
RayGeom make_ray_geom(const pcr_grid& g, const pcr_geom& G, bool swap_xy = false);

// Launch shape of the ray-march kernels.
struct MarchShape {
    int tile_u;          // pixels along u covered by one wave (64 / tile_u rows)
    int seg;             // ray segments (threads) per ray: 1, 2 or 4
};
MarchShape choose_march_shape(const RayGeom& rg);

// Moments returned by a ray march over channels (f, h_1..h_K):
//   0 sum y, 1 sum y^2, 2 sum p, 3 sum y p, 4 sum p^2,
//   5+3k sum p t_k, 6+3k sum y t_k, 7+3k sum t_k,
// with p = P f and t_k = P h_k per ray.  FP64.
inline int n_moments(int kc) { return 5 + 3 * (kc - 1); }
// with moments != null the march also returns, after the n_moments(kc)
// moments, the number of ray samples it marched
constexpr int kMaxMoments = 5 + 3 * 8;

int march_blocks(const RayGeom& rg, const MarchShape& ms);
// The FP32 march addresses its image with 32-bit byte offsets formed from
// 24-bit products: it needs the image below 2^31 bytes, (padded y) x (padded
// z) below 2^24 and the padded row below 2^24 bytes.  launch_march returns
// hipErrorInvalidValue for an FP32 layout that does not fit.
bool march_f32_fits(const PadLayout& L);

// All launchers enqueue on `s` and return hipGetLastError().
// `compute` is PCR_F32 or PCR_F64 throughout.
hipError_t launch_compose(pcr_dtype compute, pcr_dtype storage, const pcr_grid& g, int K,
                          const void* mean, const void* U, const double* w_eff, void* dvf,
                          hipStream_t s);
hipError_t launch_warp_plain(pcr_dtype compute, pcr_dtype f0_dtype, const pcr_grid& g,
                             const void* f0, const void* dvf, void* f, hipStream_t s);
// Fused compose + warp (+ tangents): writes channel 0 = f and, when
// tangent, channels 1..K = h_k = (df/dx) . u_k into the padded layout, for
// the voxels of box {lo x, lo y, lo z, hi x, hi y, hi z} (hi exclusive,
// clamped to the grid; null = every voxel).  Cells outside it keep what they
// held.
hipError_t launch_warp_fused(pcr_dtype compute, pcr_dtype storage, pcr_dtype f0_dtype,
                             const pcr_grid& g, const PadLayout& L, int K, bool tangent,
                             const void* f0, const void* mean, const void* U,
                             const double* w_eff, const int* box, void* padded, hipStream_t s);
hipError_t launch_pad(pcr_dtype compute, const PadLayout& L, const void* vol, void* padded,
                      hipStream_t s);
hipError_t launch_unpad(pcr_dtype compute, const PadLayout& L, const void* padded, void* vol,
                        hipStream_t s);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
// Ray march over kc used channels of a padded image; writes p (may be null)
// and, when moments != null, the detector moments (y required then; uses
// `partials`, room for march_blocks x kMaxMoments doubles).  With done !=
// null the final sum then stores `seq` into *done (system scope, after the
// moments are visible there): moments and done may point into mapped host
// memory.
hipError_t launch_march(pcr_dtype compute, const PadLayout& L, int kc, const RayGeom& rg,
                        const MarchShape& ms, const void* padded, const void* y, void* p_out,
                        double* partials, double* moments, unsigned long long* done,
                        unsigned long long seq, hipStream_t s);
// Fixed-order final sum of per-block partials: out[m] for m < nm.
// Per slice z of f0, bounds of its nonzero voxels (i, j): sl[8 z ..] =
// {min i, max i, min j, max j, min i+j, max i+j, min i-j, max i-j}; the
// caller initialises every (min, max) pair to (INT_MAX, INT_MIN).
hipError_t launch_support(pcr_dtype f0_dtype, const pcr_grid& g, const void* f0, int* sl,
                          hipStream_t s);
// out[r] = max_i |a[r][i]| for `rows` rows of n values (out zeroed by the caller).
hipError_t launch_absmax_rows(pcr_dtype dt, const void* a, size_t n, int rows, float* out,
                              hipStream_t s);
// out[m] = sum over blocks b of partials[m * nblocks + b] (slot-major), m < nm;
// fixed order.
hipError_t launch_reduce(const double* partials, int nblocks, int nm, double* out, hipStream_t s);
// Backprojection out = P^T r (unpadded [N], fully overwritten) with r = resid
// (when resid != null) else scale * (p - a y - b); x-fastest geometry.
hipError_t launch_backproject(pcr_dtype compute, const pcr_grid& g, const RayGeom& rg,
                              const void* resid, const void* p, const void* y, double a, double b,
                              double scale, void* out, hipStream_t s);
// Gradient contraction: partials[k * blocks + block] = sum_v g[v] (df/dx)[v] . u_k[v].
int contract_blocks(const pcr_grid& g);
hipError_t launch_contract(pcr_dtype compute, pcr_dtype storage, pcr_dtype f0_dtype,
                           const pcr_grid& g, int K, const void* f0, const void* mean,
                           const void* U, const double* w_eff, const void* gv, double* partials,
                           hipStream_t s);
hipError_t launch_warp_adjoint(pcr_dtype compute, const pcr_grid& g, const void* dvf,
                               const void* gv, void* out, hipStream_t s);
// Fixed-point localisation; writes out[0..2] = p, out[3] = iterations,
// out[4] = converged (1) or not (0).
hipError_t launch_localize(pcr_dtype storage, const pcr_grid& g, int K, const void* mean,
                           const void* U, const double* w_eff, const double* p_ref, double tol,
                           int max_iter, double* out, hipStream_t s);

}  // namespace pcr
