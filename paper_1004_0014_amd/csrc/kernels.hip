// HIP kernels for gfx950 (MI355X, CDNA4, wave64).
//
// Hot path of single-projection reconstruction under a PCA motion model
// (Li et al., section 2.2): per iteration compose the DVF, warp the
// reference image, ray-march the cone-beam projection, form the residual and
// return the cost and its gradient in w.
//
//  * Voxel passes (compose, warp, contraction) stream HBM: one thread per
//    voxel, x-contiguous lanes, structure-of-arrays fields.
//  * The ray march gathers from a zero-padded, channel-interleaved copy of
//    the warped image that stays resident in L2/MALL; each lane marches one
//    ray (or one segment of one) so a wave's taps fall in a compact 3-D
//    region; samples are clamped to the interpolant's support so no tap
//    needs a bounds check.
//  * Detector-wide and volume-wide sums accumulate in FP64: wave shuffles,
//    then LDS, then per-block partials, then one fixed-order final pass, so
//    every result is bitwise reproducible (no floating-point atomics in any
//    reduction).
#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <climits>
#include <cstdint>
#include <cstdlib>
#include <type_traits>
#include <utility>

#include "pcr_internal.h"

namespace pcr {

// ------------------------------------------------------------ storage ----
struct bf16 {
    uint16_t bits;
};

template <typename R, typename S>
__device__ __forceinline__ R widen(S v);
template <> __device__ __forceinline__ float widen<float, float>(float v) { return v; }
template <> __device__ __forceinline__ double widen<double, float>(float v) { return v; }
template <> __device__ __forceinline__ float widen<float, double>(double v) { return (float)v; }
template <> __device__ __forceinline__ double widen<double, double>(double v) { return v; }
template <> __device__ __forceinline__ float widen<float, bf16>(bf16 v)
{
    return __uint_as_float((uint32_t)v.bits << 16);
}
template <> __device__ __forceinline__ double widen<double, bf16>(bf16 v)
{
    return (double)__uint_as_float((uint32_t)v.bits << 16);
}
template <> __device__ __forceinline__ float widen<float, _Float16>(_Float16 v) { return (float)v; }
template <> __device__ __forceinline__ double widen<double, _Float16>(_Float16 v) { return (double)(float)v; }

// C channels of type R, aligned to the largest power of two (at most 16
// bytes) that divides their size, so that arrays of cells have no padding
// (6 FP32 channels: 24-byte cells at 8-byte alignment).
template <typename R, int C>
struct alignas(((sizeof(R) * C) & (0 - sizeof(R) * C)) >= 16 ? 16 : ((sizeof(R) * C) & (0 - sizeof(R) * C))) Chan {
    R v[C];
};

template <typename T>
__device__ __forceinline__ T clampv(T x, T lo, T hi)
{
    return fmin(fmax(x, lo), hi);
}
__device__ __forceinline__ float clampv(float x, float lo, float hi) { return fminf(fmaxf(x, lo), hi); }

// ----------------------------------------------------------- reductions --
// Sum over the 64 lanes of a wave with the device library's wave reduction
// (a fixed DPP tree: the same order on every call, deterministic).
extern "C" __device__ __attribute__((const)) double __ockl_wfred_add_f64(double);
__device__ __forceinline__ double wave_sum(double v) { return __ockl_wfred_add_f64(v); }

// Block (256 threads = 4 waves) sum of NM doubles per thread; thread t < nm
// writes dst[t * stride].  Only waves 0 .. nw-1 hold data (the others add
// nothing and skip their sums).  Fixed order: wave tree, then waves 0..nw-1.
template <int NM>
__device__ __forceinline__ void block_sum_store(double (&m)[NM], int nm, double* dst, int stride,
                                                int nw = 4)
{
    __shared__ double red[4][NM];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (wv < nw) {
#pragma unroll
        for (int i = 0; i < NM; ++i) {
            double s = wave_sum(m[i]);
            if (lane == 0) red[wv][i] = s;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < nm) {
        double s = red[0][threadIdx.x];
        for (int w2 = 1; w2 < nw; ++w2) s += red[w2][threadIdx.x];
        dst[(size_t)threadIdx.x * stride] = s;
    }
}

// The ray segments' sums (and sample counts) into segment 0's thread of
// each ray (threads [0, rpb)); smem holds 256 (C + 1) words.  Afterwards
// only segment 0 holds data: the block's moments need only its waves.
template <int C>
__device__ __forceinline__ void gather_segments(char* smem, int seg, int rpb, int sid, float (&acc)[C],
                                                int& nsamp)
{
    float* segbuf = (float*)smem;
    int* segn = (int*)(segbuf + 256 * C);
#pragma unroll
    for (int c = 0; c < C; ++c) segbuf[threadIdx.x * C + c] = acc[c];
    segn[threadIdx.x] = nsamp;
    __syncthreads();
    if (sid == 0)
        for (int s2 = 1; s2 < seg; ++s2) {
#pragma unroll
            for (int c = 0; c < C; ++c) acc[c] += segbuf[(threadIdx.x + s2 * rpb) * C + c];
            nsamp += segn[threadIdx.x + s2 * rpb];
        }
}

// Sum over the blocks of their partial sums, stored slot-major: part[m *
// nblocks + b] is slot m of block b.  out[0..nm) = sums of slots 0..nm-1;
// with extra >= 0 also out[nm] = the sum of slot `extra`.  One wave per
// output: lane l adds blocks l, l + 64, ... in order (coalesced loads), then
// a fixed shuffle tree: deterministic.
// With done != null the sums are stored at system scope (through to memory),
// every wave waits for its stores to complete, and after the block barrier
// `seq` is stored into *done with a system-scope release: a host polling
// *done in mapped memory sees the sums once it sees seq.  One release fence
// per launch, not one per wave.
__global__ void __launch_bounds__(1024) k_reduce(const double* __restrict__ part, int nblocks, int nm,
                                                 int extra, double* __restrict__ out,
                                                 unsigned long long* done, unsigned long long seq)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int nout = nm + (extra >= 0 ? 1 : 0);
    for (int o = wv; o < nout; o += 16) {
        const double* r = part + (size_t)(o < nm ? o : extra) * nblocks;
        double s = 0.0;
#pragma unroll 8
        for (int b = lane; b < nblocks; b += 64) s += r[b];
        s = wave_sum(s);
        if (lane == 0) {
            if (done) __hip_atomic_store(&out[o], s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            else out[o] = s;
        }
    }
    if (done) {
        // every wave waits for its own stores to complete (the barrier alone
        // does not), then one system-scope release publishes seq
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x == 0) __hip_atomic_store(done, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

static hipError_t run_reduce(const double* part, int nblocks, int nm, int extra, double* out,
                             hipStream_t s, unsigned long long* done = nullptr, unsigned long long seq = 0)
{
    k_reduce<<<1, 1024, 0, s>>>(part, nblocks, nm, extra, out, done, seq);
    return hipGetLastError();
}

// ------------------------------------------------------------ compose ----
template <typename R, typename S>
__global__ void __launch_bounds__(256) k_compose(const S* __restrict__ mean,
                                                 const S* __restrict__ U, int K, size_t N,
                                                 Chan<double, 8> w, R* __restrict__ dvf)
{
    size_t v = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= N) return;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        R x = widen<R>(mean[a * N + v]);
        for (int k = 0; k < K; ++k) x += (R)w.v[k] * widen<R>(U[(size_t)(k * 3 + a) * N + v]);
        dvf[a * N + v] = x;
    }
}

// --------------------------------------------------------------- warp ----
// Trilinear sample of an unpadded image at index-space point q, zero outside;
// optionally also the exact partial derivatives dT/dq (floor cell).
template <typename R, typename S, bool GRAD>
__device__ __forceinline__ R sample_f0(const S* __restrict__ f0, int nx, int ny, int nz,
                                       R qx, R qy, R qz, R* dT)
{
    qx = clampv(qx, (R)-2, (R)(nx + 1));
    qy = clampv(qy, (R)-2, (R)(ny + 1));
    qz = clampv(qz, (R)-2, (R)(nz + 1));
    R fx = floor(qx), fy = floor(qy), fz = floor(qz);
    int i0 = (int)fx, j0 = (int)fy, k0 = (int)fz;
    R ax = qx - fx, ay = qy - fy, az = qz - fz;
    R bx = (R)1 - ax, by = (R)1 - ay, bz = (R)1 - az;
    R c[2][2][2];
#pragma unroll
    for (int dz = 0; dz < 2; ++dz)
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) {
                int i = i0 + dx, j = j0 + dy, k = k0 + dz;
                bool in = (unsigned)i < (unsigned)nx && (unsigned)j < (unsigned)ny &&
                          (unsigned)k < (unsigned)nz;
                c[dz][dy][dx] = in ? widen<R>(f0[(size_t)i + (size_t)nx * ((size_t)j + (size_t)ny * k)])
                                   : (R)0;
            }
    R w00 = by * bz, w10 = ay * bz, w01 = by * az, w11 = ay * az;
    R val = w00 * (bx * c[0][0][0] + ax * c[0][0][1]) + w10 * (bx * c[0][1][0] + ax * c[0][1][1]) +
            w01 * (bx * c[1][0][0] + ax * c[1][0][1]) + w11 * (bx * c[1][1][0] + ax * c[1][1][1]);
    if (GRAD) {
        dT[0] = w00 * (c[0][0][1] - c[0][0][0]) + w10 * (c[0][1][1] - c[0][1][0]) +
                w01 * (c[1][0][1] - c[1][0][0]) + w11 * (c[1][1][1] - c[1][1][0]);
        dT[1] = bx * bz * (c[0][1][0] - c[0][0][0]) + ax * bz * (c[0][1][1] - c[0][0][1]) +
                bx * az * (c[1][1][0] - c[1][0][0]) + ax * az * (c[1][1][1] - c[1][0][1]);
        dT[2] = bx * by * (c[1][0][0] - c[0][0][0]) + ax * by * (c[1][0][1] - c[0][0][1]) +
                bx * ay * (c[1][1][0] - c[0][1][0]) + ax * ay * (c[1][1][1] - c[0][1][1]);
    }
    return val;
}

struct VoxGrid {
    int nx, ny, nz;
    double sp[3];
};

// Standalone warp: f[v] = T[f0](v + dvf[v] / s).
template <typename R, typename S>
__global__ void __launch_bounds__(256) k_warp_plain(const S* __restrict__ f0,
                                                    const R* __restrict__ dvf, VoxGrid g,
                                                    R* __restrict__ f)
{
    int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y * 4 + threadIdx.y, k = blockIdx.z;
    if (i >= g.nx || j >= g.ny) return;
    size_t N = (size_t)g.nx * g.ny * g.nz;
    size_t v = (size_t)i + (size_t)g.nx * ((size_t)j + (size_t)g.ny * k);
    R qx = (R)i + dvf[v] / (R)g.sp[0];
    R qy = (R)j + dvf[N + v] / (R)g.sp[1];
    R qz = (R)k + dvf[2 * N + v] / (R)g.sp[2];
    f[v] = sample_f0<R, S, false>(f0, g.nx, g.ny, g.nz, qx, qy, qz, nullptr);
}

// Fused compose + warp (+ tangents) of one voxel: channel 0 = f, channels
// 1..K = h_k = sum_a (1/s_a) dT[f0]/dq_a u_k[a] (tangent), rest zero.
template <typename R, typename S, typename F, int C, bool TAN>
__device__ __forceinline__ Chan<R, C> warp_cell(const F* __restrict__ f0, const S* __restrict__ mean,
                                                const S* __restrict__ U, int K,
                                                const Chan<double, 8>& w, const VoxGrid& g, int i,
                                                int j, int k)
{
    size_t N = (size_t)g.nx * g.ny * g.nz;
    size_t v = (size_t)i + (size_t)g.nx * ((size_t)j + (size_t)g.ny * k);
    R x[3];
    R u[TAN ? 8 : 1][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) x[a] = widen<R>(mean[a * N + v]);
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
        if (kk < K) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                R uv = widen<R>(U[(size_t)(kk * 3 + a) * N + v]);
                x[a] += (R)w.v[kk] * uv;
                if (TAN) u[TAN ? kk : 0][a] = uv;
            }
        }
    }
    R qx = (R)i + x[0] / (R)g.sp[0];
    R qy = (R)j + x[1] / (R)g.sp[1];
    R qz = (R)k + x[2] / (R)g.sp[2];
    R dT[3];
    Chan<R, C> o;
#pragma unroll
    for (int c = 0; c < C; ++c) o.v[c] = (R)0;
    o.v[0] = sample_f0<R, F, TAN>(f0, g.nx, g.ny, g.nz, qx, qy, qz, dT);
    if (TAN) {
        R G0 = dT[0] / (R)g.sp[0], G1 = dT[1] / (R)g.sp[1], G2 = dT[2] / (R)g.sp[2];
#pragma unroll
        for (int kk = 0; kk < C - 1; ++kk)
            if (kk < K) o.v[kk + 1] = G0 * u[TAN ? kk : 0][0] + G1 * u[TAN ? kk : 0][1] + G2 * u[TAN ? kk : 0][2];
    }
    return o;
}

// Cell as stored: the compute type, or (H) FP16 of value * hs[c].
template <typename R, int C, bool H>
using CellOf = Chan<typename std::conditional<H, _Float16, R>::type, C>;
template <typename R, int C, bool H>
__device__ __forceinline__ CellOf<R, C, H> store_cell(const Chan<R, C>& o, const Chan<float, 8>& hs)
{
    if constexpr (!H) {
        return o;
    } else {
        CellOf<R, C, H> h;
#pragma unroll
        for (int c = 0; c < C; ++c) h.v[c] = (_Float16)((float)o.v[c] * hs.v[c]);
        return h;
    }
}

// Voxels [lo, hi) per axis that a launch computes.
struct VoxBox {
    int lo[3], hi[3];
};

// Blocks are dispatched round-robin over the 8 XCDs, each with its own L2.
// xcd_tile maps dispatch index b of nb to a logical index such that each XCD
// takes one contiguous run of logical indices (in order).
__device__ __forceinline__ int xcd_tile(int b, int nb)
{
    const int q = nb >> 3, rem = nb & 7, x = b & 7;
    return x * q + min(x, rem) + (b >> 3);
}

// x-fastest padded layout: a block per 256-voxel run along x, coalesced in x
// both ways (longer runs than 64 x 4 blocks: 49.5 against 57.7 us at paper
// scale).  (Ordering the runs by XCD, as the y-fastest tiles are, was 2-4 %
// slower here: in dispatch order the XCDs work on neighbouring rows at the
// same time and share their f0 taps through the Infinity Cache.)
template <typename R, typename S, typename F, int C, bool TAN, bool H>
__global__ void __launch_bounds__(256) k_warp_fused(const F* __restrict__ f0,
                                                    const S* __restrict__ mean,
                                                    const S* __restrict__ U, int K,
                                                    Chan<double, 8> w, VoxGrid g, int px, int py,
                                                    Chan<float, 8> hs, VoxBox b,
                                                    CellOf<R, C, H>* __restrict__ out)
{
    const int i = b.lo[0] + blockIdx.x * 256 + threadIdx.x, j = b.lo[1] + blockIdx.y;
    const int k = b.lo[2] + blockIdx.z;
    if (i >= b.hi[0] || j >= b.hi[1]) return;
    Chan<R, C> o = warp_cell<R, S, F, C, TAN>(f0, mean, U, K, w, g, i, j, k);
    out[(size_t)(i + 1) + (size_t)px * ((size_t)(j + 1) + (size_t)py * (k + 1))] =
        store_cell<R, C, H>(o, hs);
}

// Width (x) of the y-fastest warp's tiles: the widest of 128, 64 or 32
// voxels whose 8-row tile of cells stays within about 8 KB of LDS, so that a
// block still finds room on a CU whose LDS the march's staging mostly holds
// (a serving engine runs both at once).
template <typename R, int C, bool H>
constexpr int yf_tile_x()
{
    constexpr int cb = (int)sizeof(CellOf<R, C, H>);
    return 8 * 128 * cb <= 8448 ? 128 : (8 * 64 * cb <= 8448 ? 64 : 32);
}

// y-fastest padded layout: a TX x 8 (x, y) tile per block, computed with
// x-contiguous reads (runs of 4 TX bytes of each field), staged in LDS and
// written as 8-cell runs along y.
template <typename R, typename S, typename F, int C, bool TAN, bool H>
__global__ void __launch_bounds__(256) k_warp_fused_yf(const F* __restrict__ f0,
                                                       const S* __restrict__ mean,
                                                       const S* __restrict__ U, int K,
                                                       Chan<double, 8> w, VoxGrid g, int px,
                                                       int py, Chan<float, 8> hs, VoxBox b,
                                                       int gx, int gy,
                                                       CellOf<R, C, H>* __restrict__ out)
{
    constexpr int TX = yf_tile_x<R, C, H>();
    __shared__ CellOf<R, C, H> tile[8][TX + 1];
    // tiles in XCD order: each XCD's L2 sees a contiguous band of tile rows,
    // so the f0 taps that neighbouring tiles share (displacements reach
    // several voxels) are fetched into one L2 (-7 % at 80-90 deg)
    const int lb = xcd_tile(blockIdx.x, gridDim.x);
    const int bx = lb % gx, rb = lb / gx;
    const int i0 = b.lo[0] + bx * TX, j0 = b.lo[1] + (rb % gy) * 8, k = b.lo[2] + rb / gy;
    const int t = threadIdx.x;
#pragma unroll
    for (int r = 0; r < TX / 32; ++r) {
        const int il = t % TX, jl = t / TX + (256 / TX) * r;
        const int i = i0 + il, j = j0 + jl;
        if (i < b.hi[0] && j < b.hi[1])
            tile[jl][il] = store_cell<R, C, H>(warp_cell<R, S, F, C, TAN>(f0, mean, U, K, w, g, i, j, k), hs);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < TX / 32; ++r) {
        const int jl = t & 7, il = (t >> 3) + 32 * r;
        const int i = i0 + il, j = j0 + jl;
        if (i < b.hi[0] && j < b.hi[1])
            out[(size_t)(j + 1) + (size_t)px * ((size_t)(i + 1) + (size_t)py * (k + 1))] = tile[jl][il];
    }
}

template <typename R>
__global__ void __launch_bounds__(256) k_pad(const R* __restrict__ vol, VoxGrid g, int px, int py,
                                             R* __restrict__ pad)
{
    int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y * 4 + threadIdx.y, k = blockIdx.z;
    if (i >= g.nx || j >= g.ny) return;
    size_t v = (size_t)i + (size_t)g.nx * ((size_t)j + (size_t)g.ny * k);
    pad[(size_t)(i + 1) + (size_t)px * ((size_t)(j + 1) + (size_t)py * (k + 1))] = vol[v];
}

template <typename R>
__global__ void __launch_bounds__(256) k_unpad(const R* __restrict__ pad, VoxGrid g, int px,
                                               int py, R* __restrict__ vol)
{
    int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y * 4 + threadIdx.y, k = blockIdx.z;
    if (i >= g.nx || j >= g.ny) return;
    size_t v = (size_t)i + (size_t)g.nx * ((size_t)j + (size_t)g.ny * k);
    vol[v] = pad[(size_t)(i + 1) + (size_t)px * ((size_t)(j + 1) + (size_t)py * (k + 1))];
}

__global__ void __launch_bounds__(256) k_zero16(uint4* __restrict__ p, size_t n16)
{
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    for (; i < n16; i += (size_t)gridDim.x * 256) p[i] = make_uint4(0, 0, 0, 0);
}

__global__ void __launch_bounds__(256) k_zero4(uint32_t* __restrict__ p, size_t n4)
{
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    for (; i < n4; i += (size_t)gridDim.x * 256) p[i] = 0u;
}

// ---------------------------------------------------------- ray march ----
template <typename R>
struct RaySeg {
    R q0[3];         // index-space point of the segment's first sample
    R dq[3];         // index-space step per sample
    int count;       // samples in the segment
};

// One direction of the slab tests along a ray: the coordinate o + t d,
// with 1 / d and the offsets that fold the dilation into one FMA per bound:
// t = lo * inv + nlo is where the coordinate reaches lo - h, t = hi * inv + nhi
// where it reaches hi + h.  |d| < 1e-20: the coordinate is taken as
// constant (it moves by < 1e-16 index units over any ray; 1 / d would
// overflow the offsets).
struct SlabAxis {
    float o, inv, nlo, nhi;
    bool flat;
    __device__ __forceinline__ void init(float o_, float d, float h)
    {
        o = o_;
        flat = fabsf(d) < 1e-20f;
        inv = flat ? 0.0f : 1.0f / d;
        nlo = -(o + h) * inv;
        nhi = (h - o) * inv;
    }
    __device__ __forceinline__ void clip(float lo, float hi, float h, float& ta, float& tb) const
    {
        if (!flat) {
            const float t1 = fmaf(lo, inv, nlo), t2 = fmaf(hi, inv, nhi);
            ta = fmaxf(ta, fminf(t1, t2));
            tb = fminf(tb, fmaxf(t1, t2));
        } else if (!(o >= lo - h && o <= hi + h)) {
            ta = INFINITY;
        }
    }
};

// Narrows the box segment [tmin, tmax] of a ray (direction dq, index units
// per mm) to the hull of its intersections with the dilated slab regions:
// outside every one of them all of the ray's samples are exactly zero.  The
// bounds are evaluated in FP32: where a constraint binds, the rounding moves
// the cut point by ~1e-4 index units along that constraint's own axis,
// against the half-cell slack of the dilation.
__device__ __forceinline__ void refine_by_slabs(const RayGeom& g, const double dq[3], double& tmin,
                                                double& tmax)
{
    const double za = g.qs[2] + tmin * dq[2], zb = g.qs[2] + tmax * dq[2];
    // slab s (slices sT .. sT + T - 1) reaches k in [sT - h, sT + T - 1 + h]
    const float zlo = (float)fmin(za, zb) - g.h[2], zhi = (float)fmax(za, zb) + g.h[2];
    const float T = (float)g.slab_t, lim = (float)g.nslab + 2.0f;
    const int s0 = max(0, (int)floorf(fminf(fmaxf((zlo + 1.0f) / T - 1.0f, -2.0f), lim)) - 1);
    const int s1 = min(g.nslab - 1, (int)floorf(fminf(fmaxf(zhi / T, -2.0f), lim)));
    const float o0 = (float)g.qs[0], o1 = (float)g.qs[1], d0 = (float)dq[0], d1 = (float)dq[1];
    const float hd = g.h[0] + g.h[1];
    SlabAxis ax, ay, ap, am, az;
    ax.init(o0, d0, g.h[0]);
    ay.init(o1, d1, g.h[1]);
    ap.init(o0 + o1, d0 + d1, hd);
    am.init(o0 - o1, d0 - d1, hd);
    az.init((float)g.qs[2], (float)dq[2], g.h[2]);
    float tin = INFINITY, tout = -INFINITY;
    for (int s = s0; s <= s1; ++s) {
        const float* b = g.slabs + 10 * s;
        if (b[8] > b[9]) continue;   // no nonzero voxel in this slab
        float ta = -INFINITY, tb = INFINITY;
        az.clip(b[8], b[9], g.h[2], ta, tb);
        ax.clip(b[0], b[1], g.h[0], ta, tb);
        ay.clip(b[2], b[3], g.h[1], ta, tb);
        ap.clip(b[4], b[5], hd, ta, tb);
        am.clip(b[6], b[7], hd, ta, tb);
        if (ta <= tb) {
            tin = fminf(tin, ta);
            tout = fmaxf(tout, tb);
        }
    }
    tmin = fmax(tmin, (double)tin);
    tmax = fmin(tmax, (double)tout);
}

// Global sample range [n0, n1] of ray (iu, iv) (n1 < n0: none) on the grid
// t = n dt, clipped to the box (at most the support [-1, n_a] of the
// interpolant) and the slabs, widened by one sample at each end (samples
// outside the support are clamped onto zero cells), and the ray's direction
// (index units per mm).  FP64, once per ray.
struct RayRange {
    int n0, n1;
    double dq[3];
};

__device__ __forceinline__ RayRange ray_range(const RayGeom& g, int iu, int iv)
{
    RayRange r;
    double u = g.u0 + iu * g.du, v = g.v0 + iv * g.dv;
    double D[3], L2 = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        D[a] = g.qc[a] + u * g.eu[a] + v * g.ev[a] - g.qs[a];
        double w = D[a] * g.sp[a];
        L2 += w * w;
    }
    double L = sqrt(L2);
    double tmin = 0.0, tmax = L;
    bool hit = L > 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        r.dq[a] = hit ? D[a] / L : 0.0;
        if (r.dq[a] != 0.0) {
            double t1 = (g.clo[a] - g.qs[a]) / r.dq[a], t2 = (g.chi[a] - g.qs[a]) / r.dq[a];
            tmin = fmax(tmin, fmin(t1, t2));
            tmax = fmin(tmax, fmax(t1, t2));
        } else if (!(g.qs[a] > g.clo[a] && g.qs[a] < g.chi[a])) {
            hit = false;
        }
    }
    if (g.slabs && hit && tmin <= tmax) refine_by_slabs(g, r.dq, tmin, tmax);
    r.n0 = 0;
    r.n1 = -1;
    if (!hit || !(tmin <= tmax)) return r;
    long nlast = (long)floor(L / g.dt);
    long n0 = (long)ceil(tmin / g.dt) - 1, n1 = (long)floor(tmax / g.dt) + 1;
    if (n0 < 0) n0 = 0;
    if (n1 > nlast) n1 = nlast;
    if (n1 >= n0) {
        r.n0 = (int)n0;
        r.n1 = (int)n1;
    }
    return r;
}

// The ray's range split into `seg` equal segments: segment `sid`.
template <typename R>
__device__ __forceinline__ RaySeg<R> ray_segment(const RayGeom& g, int iu, int iv, int seg, int sid)
{
    RaySeg<R> r;
    const RayRange rr = ray_range(g, iu, iv);
    const long cnt = rr.n1 >= rr.n0 ? (long)rr.n1 - rr.n0 + 1 : 0;
    long m0 = cnt * sid / seg, m1 = cnt * (sid + 1) / seg;
    r.count = (int)(m1 - m0);
    double t0 = (double)(rr.n0 + m0) * g.dt;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        r.q0[a] = (R)(g.qs[a] + t0 * rr.dq[a]);
        r.dq[a] = (R)(g.dt * rr.dq[a]);
    }
    return r;
}

__device__ __forceinline__ void ray_of_thread(const MarchShape& ms, int tiles_u, int& iu, int& iv,
                                              int& sid, int& rloc)
{
    const int rpb = 256 / ms.seg;
    rloc = threadIdx.x % rpb;
    sid = threadIdx.x / rpb;
    const int tv_rows = rpb / ms.tile_u;
    int tu = blockIdx.x % tiles_u, tv = blockIdx.x / tiles_u;
    iu = tu * ms.tile_u + rloc % ms.tile_u;
    iv = tv * tv_rows + rloc / ms.tile_u;
}

// Ray march over the padded image; p and moments per ray.
template <typename R, int C>
__global__ void __launch_bounds__(256) k_march(RayGeom g, MarchShape ms, int tiles_u,
                                               const Chan<R, C>* __restrict__ vol, int px,
                                               int py, float fnx, float fny, float fnz, int kc,
                                               const R* __restrict__ y, R* __restrict__ p_out,
                                               double* __restrict__ partials)
{
    int iu, iv, sid, rloc;
    ray_of_thread(ms, tiles_u, iu, iv, sid, rloc);
    const bool valid = iu < g.nu && iv < g.nv;
    R acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = (R)0;
    int nsamp = 0;
    if (valid) {
        RaySeg<R> rs = ray_segment<R>(g, iu, iv, ms.seg, sid);
        nsamp = rs.count;
        const long pxy = (long)px * py;
        const Chan<R, C>* base = vol + (1 + px + pxy);   // cell of voxel (0,0,0)
        for (int m = 0; m < rs.count; ++m) {
            R fm = (R)m;
            R qx = clampv(fma(fm, rs.dq[0], rs.q0[0]), (R)-1, (R)fnx);
            R qy = clampv(fma(fm, rs.dq[1], rs.q0[1]), (R)-1, (R)fny);
            R qz = clampv(fma(fm, rs.dq[2], rs.q0[2]), (R)-1, (R)fnz);
            R flx = floor(qx), fly = floor(qy), flz = floor(qz);
            int ix = (int)flx, iy = (int)fly, iz = (int)flz;
            R ax = qx - flx, ay = qy - fly, az = qz - flz;
            R bx = (R)1 - ax, by = (R)1 - ay, bz = (R)1 - az;
            R w00 = by * bz, w10 = ay * bz, w01 = by * az, w11 = ay * az;
            const Chan<R, C>* c0 = base + ((long)ix + (long)px * iy + pxy * iz);
            Chan<R, C> t000 = c0[0], t100 = c0[1], t010 = c0[px], t110 = c0[px + 1];
            Chan<R, C> t001 = c0[pxy], t101 = c0[pxy + 1], t011 = c0[pxy + px],
                       t111 = c0[pxy + px + 1];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                R x00 = bx * t000.v[c] + ax * t100.v[c];
                R x10 = bx * t010.v[c] + ax * t110.v[c];
                R x01 = bx * t001.v[c] + ax * t101.v[c];
                R x11 = bx * t011.v[c] + ax * t111.v[c];
                acc[c] += w00 * x00 + w10 * x10 + w01 * x01 + w11 * x11;
            }
        }
    }
    if (ms.seg > 1) {
        __shared__ R segbuf[256 * C];
#pragma unroll
        for (int c = 0; c < C; ++c) segbuf[threadIdx.x * C + c] = acc[c];
        __syncthreads();
        if (sid == 0) {
            const int rpb = 256 / ms.seg;
            for (int s = 1; s < ms.seg; ++s)
#pragma unroll
                for (int c = 0; c < C; ++c) acc[c] += segbuf[(threadIdx.x + s * rpb) * C + c];
        }
    }
    const bool owner = valid && sid == 0;
    const R dt = (R)g.dt;
    if (owner && p_out) p_out[iu + (size_t)g.nu * iv] = dt * acc[0];
    if (partials) {
        // record per block: the moments, then the number of samples marched
        constexpr int NM = 5 + 3 * (C - 1);
        double m[NM + 1];
#pragma unroll
        for (int i = 0; i < NM; ++i) m[i] = 0.0;
        m[NM] = (double)nsamp;
        if (owner) {
            double yd = (double)y[iu + (size_t)g.nu * iv];
            double pd = (double)(dt * acc[0]);
            m[0] = yd;
            m[1] = yd * yd;
            m[2] = pd;
            m[3] = yd * pd;
            m[4] = pd * pd;
#pragma unroll
            for (int k = 0; k < C - 1; ++k) {
                if (k + 1 < kc) {
                    double tk = (double)(dt * acc[k + 1]);
                    m[5 + 3 * k] = pd * tk;
                    m[6 + 3 * k] = yd * tk;
                    m[7 + 3 * k] = tk;
                }
            }
        }
        block_sum_store<NM + 1>(m, NM + 1, partials + blockIdx.x, (int)gridDim.x);
    }
}

// ---------------------------------------------------- FP32 ray march ----
// (Blocks go to the XCDs round-robin: xcd_tile, defined with the warps,
// gives each XCD one contiguous band of detector rows, so that the rays
// sharing an XCD's L2 cross the same part of the volume.)

// One padded cell pair (x and x+1) of C float channels.
template <int C>
struct CellPair {
    float a[C], b[C];
};
// The pair at byte offset `off` from `base` (plain global loads).
template <int C>
__device__ __forceinline__ CellPair<C> load_pair_g(const char* base, int off)
{
    CellPair<C> p;
    const float* a = (const float*)(base + off);
#pragma unroll
    for (int c = 0; c < C; ++c) {
        p.a[c] = a[c];
        p.b[c] = a[C + c];
    }
    return p;
}

// Same pair from FP16 cells (values as stored: times the channel scale).
typedef _Float16 h4v __attribute__((ext_vector_type(4)));
typedef _Float16 h8v __attribute__((ext_vector_type(8)));
template <int C>
__device__ __forceinline__ CellPair<C> load_pair_h(const char* base, int off)
{
    CellPair<C> p;
    if constexpr (C == 2) {
        h4v v;
        __builtin_memcpy(&v, base + off, sizeof v);
        p.a[0] = (float)v[0];
        p.a[1] = (float)v[1];
        p.b[0] = (float)v[2];
        p.b[1] = (float)v[3];
    } else {
#pragma unroll
        for (int h = 0; h < C / 4; ++h) {
            // cells x and x+1 are adjacent: 2 C halves, read 8 at a time
            h8v v;
            __builtin_memcpy(&v, base + off + 16 * h, sizeof v);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int idx = 8 * h + e;       // half index within the pair
                if (idx < C) p.a[idx] = (float)v[e];
                else p.b[idx - C] = (float)v[e];
            }
        }
    }
    return p;
}

struct MarchArgs {
    RayGeom g;
    MarchShape ms;
    int tiles_u;
    const void* vol;       // padded image, C float channels per cell
    int px, py, pz;        // padded dims in memory order (cells)
    int ys, zs;            // byte strides of the padded y and z axes (offsets are
                           // 32-bit: march_f32_fits bounds the image)
    float fn1[3];          // clamp bound n_a + 1 (padded index space)
    int kc;                // channels used
    const float* y;        // measured projection (moments) or null
    float* p_out;          // projection out or null
    double* partials;      // [NM][blocks] (slot-major) or null
    double* moments;       // final moments (last block) or null
    float ihs[8];          // FP16 cells: 1 / channel scale
};

// The march gathering its taps through the vector L1.  The library launches
// it for FP16 cells (H), where the VALU binds; FP32 cells go to the
// LDS-staged k_march_lds below, which takes the same samples in the same
// order and gives bitwise the same sums as this kernel's FP32 form.
template <int C, bool H>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(C <= 4 ? 8 : 1))) k_march_f32(MarchArgs A)
{
    constexpr int CB = (H ? 2 : 4) * C;   // bytes per cell
    const RayGeom& g = A.g;
    const int rpb = 256 / A.ms.seg;
    const int rloc = threadIdx.x % rpb, sid = threadIdx.x / rpb;
    const int rows = rpb / A.ms.tile_u;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int tu = tile % A.tiles_u, tv = tile / A.tiles_u;
    const int iu = tu * A.ms.tile_u + rloc % A.ms.tile_u;
    const int iv = tv * rows + rloc / A.ms.tile_u;
    const bool valid = iu < g.nu && iv < g.nv;
    float acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = 0.f;
    int nsamp = 0;
    // The wave marches the union of its rays' sample ranges in step: at each
    // iteration all its lanes sit at the same global sample index n (t = n
    // dt), so neighbouring rays read neighbouring cells and share cache
    // lines; a lane skips the indices outside its own ray's range.  The waves
    // holding the same 64 rays (one per segment) split the union into equal
    // parts, so each sample of a ray is taken exactly once.
    RayRange rr;
    rr.n0 = 0;
    rr.n1 = -1;
    rr.dq[0] = rr.dq[1] = rr.dq[2] = 0.0;
    // LDS: first the block's ray set-ups, then the segments' partial sums
    constexpr int kSeg = 256 * (C + 1) * 4;   // gather_segments
    constexpr int kSmem = kSeg > 128 * (int)sizeof(RayRange) ? kSeg : 128 * (int)sizeof(RayRange);
    __shared__ __align__(16) char smem[kSmem];
    if (A.ms.seg > 1) {
        // the segment-0 waves set up the block's rays, the others read them
        RayRange* rbuf = (RayRange*)smem;
        if (sid == 0) {
            if (valid) rr = ray_range(g, iu, iv);
            rbuf[rloc] = rr;
        }
        __syncthreads();
        rr = rbuf[rloc];
        __syncthreads();   // before the buffer is reused for the partial sums
    } else if (valid) {
        rr = ray_range(g, iu, iv);
    }
    int N0 = rr.n1 >= rr.n0 ? rr.n0 : INT_MAX, N1 = rr.n1 >= rr.n0 ? rr.n1 : INT_MIN;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        N0 = min(N0, __shfl_xor(N0, o));
        N1 = max(N1, __shfl_xor(N1, o));
    }
    N0 = __builtin_amdgcn_readfirstlane(N0);
    N1 = __builtin_amdgcn_readfirstlane(N1);
    if (N0 <= N1) {
        const long span = (long)N1 - N0 + 1;
        const int na = __builtin_amdgcn_readfirstlane(N0 + (int)(span * sid / A.ms.seg));
        const int nb = __builtin_amdgcn_readfirstlane(N0 + (int)(span * (sid + 1) / A.ms.seg));
        // padded index space: cell i+1 holds voxel i, so q + 1 >= 0 after the
        // clamp and truncation is the floor
        const double ta = (double)na * g.dt;
        const float q0x = (float)(g.qs[0] + ta * rr.dq[0]) + 1.f;
        const float q0y = (float)(g.qs[1] + ta * rr.dq[1]) + 1.f;
        const float q0z = (float)(g.qs[2] + ta * rr.dq[2]) + 1.f;
        const float dqx = (float)(g.dt * rr.dq[0]), dqy = (float)(g.dt * rr.dq[1]),
                    dqz = (float)(g.dt * rr.dq[2]);
        const int YS = A.ys, ZS = A.zs, YZ = A.ys + A.zs, PY = A.py;
        // A step is half a voxel or less, so consecutive samples of a lane
        // often fall in the same cell: with FP32 cells (bound by the L1) the
        // lane keeps its last 8 cells and loads only when the cell changes
        // (lanes that reuse are masked out of the load and cost no L1
        // bandwidth).  FP16 cells (bound by the VALU) always load: there the
        // branch costs more than the bandwidth it saves (measured).
        CellPair<C> p00, p10, p01, p11;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            p00.a[c] = p00.b[c] = p10.a[c] = p10.b[c] = 0.f;
            p01.a[c] = p01.b[c] = p11.a[c] = p11.b[c] = 0.f;
        }
        int last = -1;
        for (int n = na; n < nb; ++n) {
            if (n < rr.n0 || n > rr.n1) continue;
            ++nsamp;
            const float fm = (float)(n - na);
            float qx = __builtin_amdgcn_fmed3f(fmaf(fm, dqx, q0x), 0.f, A.fn1[0]);
            float qy = __builtin_amdgcn_fmed3f(fmaf(fm, dqy, q0y), 0.f, A.fn1[1]);
            float qz = __builtin_amdgcn_fmed3f(fmaf(fm, dqz, q0z), 0.f, A.fn1[2]);
            const int ix = (int)qx, iy = (int)qy, iz = (int)qz;
            const float ax = __builtin_amdgcn_fractf(qx), ay = __builtin_amdgcn_fractf(qy),
                        az = __builtin_amdgcn_fractf(qz);
            // (iz py + iy) < 2^24 and YS < 2^24, and every offset is below
            // the image size < 2^31 (checked at launch), so the 24-bit
            // products are exact
            const int voff = ix * CB + (int)__umul24(__umul24(iz, PY) + iy, YS);
            if (H || voff != last) {
                last = voff;
                if constexpr (H) {
                    const char* vb = (const char*)A.vol;
                    p00 = load_pair_h<C>(vb, voff);
                    p10 = load_pair_h<C>(vb, voff + YS);
                    p01 = load_pair_h<C>(vb, voff + ZS);
                    p11 = load_pair_h<C>(vb, voff + YZ);
                } else {
                    const char* vb = (const char*)A.vol;
                    p00 = load_pair_g<C>(vb, voff);
                    p10 = load_pair_g<C>(vb, voff + YS);
                    p01 = load_pair_g<C>(vb, voff + ZS);
                    p11 = load_pair_g<C>(vb, voff + YZ);
                }
            }
            const float bx = 1.f - ax, by = 1.f - ay, bz = 1.f - az;
            const float w00 = by * bz, w10 = ay * bz, w01 = by * az, w11 = ay * az;
            const float w000 = bx * w00, w100 = ax * w00, w010 = bx * w10, w110 = ax * w10;
            const float w001 = bx * w01, w101 = ax * w01, w011 = bx * w11, w111 = ax * w11;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                float t = acc[c];
                t = fmaf(w000, p00.a[c], t);
                t = fmaf(w100, p00.b[c], t);
                t = fmaf(w010, p10.a[c], t);
                t = fmaf(w110, p10.b[c], t);
                t = fmaf(w001, p01.a[c], t);
                t = fmaf(w101, p01.b[c], t);
                t = fmaf(w011, p11.a[c], t);
                t = fmaf(w111, p11.b[c], t);
                acc[c] = t;
            }
        }
    }
    if (A.ms.seg > 1) gather_segments<C>(smem, A.ms.seg, rpb, sid, acc, nsamp);
    if constexpr (H) {
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] *= A.ihs[c];   // exact: powers of two
    }
    const bool owner = valid && sid == 0;
    const float dt = (float)g.dt;
    if (owner && A.p_out) A.p_out[iu + (size_t)g.nu * iv] = dt * acc[0];
    if (A.partials) {
        // record per block: the moments, then the number of samples marched
        constexpr int NM = 5 + 3 * (C - 1);
        double mo[NM + 1];
#pragma unroll
        for (int i = 0; i < NM; ++i) mo[i] = 0.0;
        mo[NM] = sid == 0 ? (double)nsamp : 0.0;   // segments were gathered
        if (owner) {
            double yd = (double)A.y[iu + (size_t)g.nu * iv];
            double pd = (double)(dt * acc[0]);
            mo[0] = yd;
            mo[1] = yd * yd;
            mo[2] = pd;
            mo[3] = yd * pd;
            mo[4] = pd * pd;
#pragma unroll
            for (int k = 0; k < C - 1; ++k) {
                if (k + 1 < A.kc) {
                    double tk = (double)(dt * acc[k + 1]);
                    mo[5 + 3 * k] = pd * tk;
                    mo[6 + 3 * k] = yd * tk;
                    mo[7 + 3 * k] = tk;
                }
            }
        }
        block_sum_store<NM + 1>(mo, NM + 1, A.partials + blockIdx.x, (int)gridDim.x, rpb / 64);
    }
}

// ------------------------------------------ FP32 ray march, LDS-staged ----
// The same march as k_march_f32 (same rays per wave, same segments, same
// sample positions, weights and summation order: bitwise the same sums), but
// each wave gathers its taps from a private LDS copy of the cells it is about
// to sample instead of through the vector L1.  The wave's sample range is cut
// into chunks of S sample indices; for each chunk the wave finds the index
// box of the cells its active lanes will read (the floor cells of the first
// and last sample of each lane's share of the chunk, plus one: positions are
// monotone in n, so the extremes bound every sample between), copies that
// box from the image into LDS with coalesced row loads (one 16-byte lane
// load per cell at C = 4), and marches the chunk out of LDS.  A chunk whose
// box exceeds the wave's buffer is retried at half the length; at the
// shortest length it falls back to gathering through the L1.  A short box
// grows the next chunk.  Each staged cell serves ~40 sample taps at paper
// scale, so the L1 sees a few coalesced row loads per chunk instead of 8
// scattered cells per sample.
// LDS per wave: six 256-thread blocks per CU at C <= 4 (74 VGPRs), five at
// C = 6 (85-94 VGPRs), four at C = 8 (114 VGPRs), the most that the
// registers allow in each case (at C = 6, 6 KB and five blocks beat 9 KB
// and four by 5-9 % at paper scale)
template <int C>
constexpr int stage_bytes() { return C <= 6 ? 6144 : 9216; }
template <int C>
constexpr int march_waves_per_eu() { return C <= 4 ? 6 : (C <= 6 ? 5 : 4); }

// a * b + c with a, b < 2^24 in one v_mad_u32_u24 (b wave-uniform; left to
// itself the compiler spreads a two-term cell offset over more instructions)
__device__ __forceinline__ unsigned mad_u24(int a, unsigned b, unsigned c)
{
    unsigned d;
    asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(d) : "v"(a), "s"(b), "v"(c));
    return d;
}

// floor(x / d) for 0 <= x < 2^21 and d >= 1, given rd = rcp(d) from the
// hardware reciprocal (within 1 ulp): (x + 0.5) rd is within 2^-22 relative
// of (x + 0.5) / d, less than 0.5 / d absolute, and (x + 0.5) / d lies at
// least 0.5 / d from every integer, so truncation gives the exact quotient.
__device__ __forceinline__ int small_quot(int x, float rd)
{
    return (int)(((float)x + 0.5f) * rd);
}

// The cells at byte offset `off` of a staging buffer of C-float cells and
// the cell after it.
template <int C>
__device__ __forceinline__ void lds_pair(const char* st, unsigned off, float (&a)[C], float (&b)[C])
{
    if constexpr (C % 4 == 0) {
        const float4* q = (const float4*)(st + off);
#pragma unroll
        for (int h = 0; h < C / 4; ++h) {
            const float4 u = q[h], v = q[C / 4 + h];
            a[4 * h] = u.x; a[4 * h + 1] = u.y; a[4 * h + 2] = u.z; a[4 * h + 3] = u.w;
            b[4 * h] = v.x; b[4 * h + 1] = v.y; b[4 * h + 2] = v.z; b[4 * h + 3] = v.w;
        }
    } else if constexpr (C % 2 == 0) {
        // 8-byte aligned cells (C = 2, 6): pairs of channels
#pragma unroll
        for (int h = 0; h < C / 2; ++h) {
            const float2 u = *(const float2*)(st + off + 8 * h), v = *(const float2*)(st + off + 4 * C + 8 * h);
            a[2 * h] = u.x; a[2 * h + 1] = u.y; b[2 * h] = v.x; b[2 * h + 1] = v.y;
        }
    } else {
        const float* q = (const float*)(st + off);
        a[0] = q[0];
        b[0] = q[1];
    }
}

// Copies one C-float cell (global, 4C-byte aligned) into a staging buffer.
template <int C>
__device__ __forceinline__ void stage_cell(const char* src, float* dst)
{
    if constexpr (C % 4 == 0) {
#pragma unroll
        for (int h = 0; h < C / 4; ++h) ((float4*)dst)[h] = ((const float4*)src)[h];
    } else if constexpr (C % 2 == 0) {
#pragma unroll
        for (int h = 0; h < C / 2; ++h) ((float2*)dst)[h] = ((const float2*)src)[h];
    } else {
        static_assert(C == 1, "cells of 1, 2, 4, 6 or 8 channels");
        *dst = *(const float*)src;
    }
}

// KC: the channels whose sums are used (A.kc: the moments and the projection
// read only those; the others stay zero); the sample loop accumulates only
// these, so a 5-channel image stored in 6-channel cells (K = 4) does not pay
// for the channel it does not use.
template <int C, int KC = C>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(march_waves_per_eu<C>()))) k_march_lds(MarchArgs A)
{
    static_assert(KC >= 1 && KC <= C, "used channels");
    constexpr int CB = 4 * C;                    // bytes per cell
    constexpr int kStageBytes = stage_bytes<C>();
    constexpr int BUF = kStageBytes / CB;        // cells per wave
    const RayGeom& g = A.g;
    const int rpb = 256 / A.ms.seg;
    const int rloc = threadIdx.x % rpb, sid = threadIdx.x / rpb;
    const int rows = rpb / A.ms.tile_u;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int tu = tile % A.tiles_u, tv = tile / A.tiles_u;
    const int iu = tu * A.ms.tile_u + rloc % A.ms.tile_u;
    const int iv = tv * rows + rloc / A.ms.tile_u;
    const bool valid = iu < g.nu && iv < g.nv;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = 0.f;
    int nsamp = 0;
    RayRange rr;
    rr.n0 = 0;
    rr.n1 = -1;
    rr.dq[0] = rr.dq[1] = rr.dq[2] = 0.0;
    // LDS: the block's ray set-ups, then the waves' staging buffers, then
    // the segments' partial sums (one after the other, so they share it)
    constexpr int kStage = 4 * kStageBytes;
    constexpr int kSeg = 256 * (C + 1) * 4;   // gather_segments
    constexpr int kRest = kSeg > 128 * (int)sizeof(RayRange) ? kSeg : 128 * (int)sizeof(RayRange);
    constexpr int kSmem = kStage > kRest ? kStage : kRest;
    __shared__ __align__(16) char smem[kSmem];
    if (A.ms.seg > 1) {
        RayRange* rbuf = (RayRange*)smem;
        if (sid == 0) {
            if (valid) rr = ray_range(g, iu, iv);
            rbuf[rloc] = rr;
        }
        __syncthreads();
        rr = rbuf[rloc];
        __syncthreads();   // before the buffer is reused for staging
    } else if (valid) {
        rr = ray_range(g, iu, iv);
    }
    int N0 = rr.n1 >= rr.n0 ? rr.n0 : INT_MAX, N1 = rr.n1 >= rr.n0 ? rr.n1 : INT_MIN;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        N0 = min(N0, __shfl_xor(N0, o));
        N1 = max(N1, __shfl_xor(N1, o));
    }
    N0 = __builtin_amdgcn_readfirstlane(N0);
    N1 = __builtin_amdgcn_readfirstlane(N1);
    float* st = (float*)(smem + wave * kStageBytes);
    if (N0 <= N1) {
        const long span = (long)N1 - N0 + 1;
        const int na = __builtin_amdgcn_readfirstlane(N0 + (int)(span * sid / A.ms.seg));
        const int nb = __builtin_amdgcn_readfirstlane(N0 + (int)(span * (sid + 1) / A.ms.seg));
        const double ta = (double)na * g.dt;
        const float q0x = (float)(g.qs[0] + ta * rr.dq[0]) + 1.f;
        const float q0y = (float)(g.qs[1] + ta * rr.dq[1]) + 1.f;
        const float q0z = (float)(g.qs[2] + ta * rr.dq[2]) + 1.f;
        const float dqx = (float)(g.dt * rr.dq[0]), dqy = (float)(g.dt * rr.dq[1]),
                    dqz = (float)(g.dt * rr.dq[2]);
        const int YS = A.ys, ZS = A.zs, YZ = A.ys + A.zs, PY = A.py;
        const char* vb = (const char*)A.vol;
        // the chunk's samples: the same positions, weights and order as
        // in k_march_f32; a lane reloads its cells P (the pairs at +0, +y,
        // +z, +y+z) only when they change
        // (fm: the sample's index relative to na, as a float)
        auto step = [&](float fm, CellPair<C> (&P)[4], auto&& load) {
            float qx = __builtin_amdgcn_fmed3f(fmaf(fm, dqx, q0x), 0.f, A.fn1[0]);
            float qy = __builtin_amdgcn_fmed3f(fmaf(fm, dqy, q0y), 0.f, A.fn1[1]);
            float qz = __builtin_amdgcn_fmed3f(fmaf(fm, dqz, q0z), 0.f, A.fn1[2]);
            const int ix = (int)qx, iy = (int)qy, iz = (int)qz;
            const float ax = __builtin_amdgcn_fractf(qx), ay = __builtin_amdgcn_fractf(qy),
                        az = __builtin_amdgcn_fractf(qz);
            load(ix, iy, iz);
            const float bx = 1.f - ax, by = 1.f - ay, bz = 1.f - az;
            const float w00 = by * bz, w10 = ay * bz, w01 = by * az, w11 = ay * az;
            const float w000 = bx * w00, w100 = ax * w00, w010 = bx * w10, w110 = ax * w10;
            const float w001 = bx * w01, w101 = ax * w01, w011 = bx * w11, w111 = ax * w11;
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                float t = acc[c];
                t = fmaf(w000, P[0].a[c], t);
                t = fmaf(w100, P[0].b[c], t);
                t = fmaf(w010, P[1].a[c], t);
                t = fmaf(w110, P[1].b[c], t);
                t = fmaf(w001, P[2].a[c], t);
                t = fmaf(w101, P[2].b[c], t);
                t = fmaf(w011, P[3].a[c], t);
                t = fmaf(w111, P[3].b[c], t);
                acc[c] = t;
            }
        };
        int S = 16;
        bool gather = false;   // the rest of the range through the L1
        int c0 = na;
        while (c0 < nb) {
            // the chunk [c0, c1) and the box of the cells its samples read;
            // a box beyond the buffer is retried at half the length (in a
            // loop of its own, so the chunk loop has a single way round)
            int c1, lo0, lo1, lo2, hi0, hi1, hi2, dx, dy, dz, dxy, cells;
            for (;;) {
                c1 = min(nb, c0 + S);
                // this lane's samples in the chunk, and the cells they read
                const int s0 = max(c0, rr.n0), s1 = min(c1 - 1, rr.n1);
                lo0 = lo1 = lo2 = INT_MAX;
                hi0 = hi1 = hi2 = INT_MIN;
                if (s0 <= s1) {
                    const float fa = (float)(s0 - na), fb = (float)(s1 - na);
                    const float xa = __builtin_amdgcn_fmed3f(fmaf(fa, dqx, q0x), 0.f, A.fn1[0]);
                    const float ya = __builtin_amdgcn_fmed3f(fmaf(fa, dqy, q0y), 0.f, A.fn1[1]);
                    const float za = __builtin_amdgcn_fmed3f(fmaf(fa, dqz, q0z), 0.f, A.fn1[2]);
                    const float xb = __builtin_amdgcn_fmed3f(fmaf(fb, dqx, q0x), 0.f, A.fn1[0]);
                    const float yb = __builtin_amdgcn_fmed3f(fmaf(fb, dqy, q0y), 0.f, A.fn1[1]);
                    const float zb = __builtin_amdgcn_fmed3f(fmaf(fb, dqz, q0z), 0.f, A.fn1[2]);
                    lo0 = (int)fminf(xa, xb);
                    lo1 = (int)fminf(ya, yb);
                    lo2 = (int)fminf(za, zb);
                    hi0 = (int)fmaxf(xa, xb) + 1;
                    hi1 = (int)fmaxf(ya, yb) + 1;
                    hi2 = (int)fmaxf(za, zb) + 1;
                }
                lo0 = __ockl_wfred_min_i32(lo0);
                lo1 = __ockl_wfred_min_i32(lo1);
                lo2 = __ockl_wfred_min_i32(lo2);
                hi0 = __ockl_wfred_max_i32(hi0);
                hi1 = __ockl_wfred_max_i32(hi1);
                hi2 = __ockl_wfred_max_i32(hi2);
                if (lo0 > hi0) break;   // no lane samples this chunk
                dx = hi0 - lo0 + 1;
                dy = hi1 - lo1 + 1;
                dz = hi2 - lo2 + 1;
                dxy = dx * dy;
                cells = dxy * dz;
                if (cells <= BUF || S <= 4) break;
                S >>= 1;
            }
            if (lo0 > hi0) {
                c0 = c1;
                continue;
            }
            if (cells > BUF) {
                // the rays spread too far for the buffer even over 4 samples
                // (coarse detectors): gather the rest through the L1
                gather = true;
                break;
            }
            {
                // every lane is past the previous chunk's reads (the wave runs
                // in order); copy the box, rows along the fastest axis
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                __builtin_amdgcn_wave_barrier();
                // cell e = row dx + lx, row = lz dy + ly: each lane starts at
                // e = lane and advances by 64 cells, i.e. by sz slices, sy
                // rows and sx cells with at most one carry into the row and
                // one into the slice; its image offset follows the same
                // carries (unsigned: the offset one step past the box may
                // wrap, but every offset loaded is that of a box cell)
                const float rdx = __builtin_amdgcn_rcpf((float)dx), rdy = __builtin_amdgcn_rcpf((float)dy);
                const int row = small_quot(lane, rdx);
                int lx = lane - row * dx;
                const int lz = small_quot(row, rdy);
                int ly = row - lz * dy;
                const int srow = __builtin_amdgcn_readfirstlane(small_quot(64, rdx));
                const int sz = __builtin_amdgcn_readfirstlane(small_quot(srow, rdy));
                const int sx = 64 - srow * dx, sy = srow - sz * dy;
                const unsigned uYS = (unsigned)YS, uZS = (unsigned)ZS;
                const unsigned a0 = (unsigned)(sx * CB) + (unsigned)sy * uYS + (unsigned)sz * uZS;
                const unsigned a1 = uYS - (unsigned)(dx * CB), a2 = uZS - (unsigned)dy * uYS;
                unsigned goff = (unsigned)((lo0 + lx) * CB) + __umul24(__umul24(lo2 + lz, PY) + lo1 + ly, YS);
                for (int e = lane; e < cells; e += 64) {
                    stage_cell<C>(vb + goff, st + e * C);
                    lx += sx;
                    const bool carry_x = lx >= dx;
                    lx -= carry_x ? dx : 0;
                    ly += sy + (carry_x ? 1 : 0);
                    const bool carry_y = ly >= dy;
                    ly -= carry_y ? dy : 0;
                    goff += a0 + (carry_x ? a1 : 0u) + (carry_y ? a2 : 0u);
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            }
            // the cells live only within the chunk (no copies of them carried
            // around the chunk loop) and need no initial value: every cell
            // offset in the box is >= 0, so a lane's first sample loads
            // (the box cell of padded cell (ix, iy, iz) at byte offset
            // iz cz + iy cy + ix CB - (lo2 cz + lo1 cy + lo0 CB), in unsigned
            // arithmetic: the wrap of the products cancels in the difference)
            CellPair<C> P[4];
            unsigned last = ~0u;
            const int s_lo = max(c0, rr.n0), s_hi = min(c1 - 1, rr.n1);
            const unsigned cy = (unsigned)(dx * CB), cz = (unsigned)(dxy * CB);
            // (offsets from the start of the block's LDS: the wave's buffer
            // starts kStageBytes x wave into it)
            const unsigned base = (unsigned)lo2 * cz + (unsigned)lo1 * cy + (unsigned)(lo0 * CB) -
                                  (unsigned)__builtin_amdgcn_readfirstlane(wave * kStageBytes);
            const char* stb = smem;
            // the samples, counted once per chunk; the loop runs on the
            // index as a float (0 <= n - na < 2^24: exact)
            const int cnt = s_hi - s_lo + 1;
            if (cnt > 0) nsamp += cnt;
            const float fe = (float)(s_hi - na);
            for (float fm = (float)(s_lo - na); fm <= fe; fm += 1.0f)
                step(fm, P, [&](int ix, int iy, int iz) {
                    const unsigned loc = mad_u24(iz, cz, mad_u24(iy, cy, (unsigned)(ix * CB) - base));
                    if (loc != last) {
                        last = loc;
                        lds_pair<C>(stb, loc, P[0].a, P[0].b);
                        lds_pair<C>(stb, loc + cy, P[1].a, P[1].b);
                        lds_pair<C>(stb, loc + cz, P[2].a, P[2].b);
                        lds_pair<C>(stb, loc + cz + cy, P[3].a, P[3].b);
                    }
                });
            if (cells * 3 < BUF && S < 64) S <<= 1;
            c0 = c1;
        }
        if (gather) {
            CellPair<C> P[4];   // offsets are >= 0: the first sample loads
            int last = -1;
            const int g0 = max(c0, rr.n0), g1 = min(nb - 1, rr.n1);
            if (g1 >= g0) nsamp += g1 - g0 + 1;
            const float fe = (float)(g1 - na);
            for (float fm = (float)(g0 - na); fm <= fe; fm += 1.0f)
                step(fm, P, [&](int ix, int iy, int iz) {
                    const int voff = ix * CB + (int)__umul24(__umul24(iz, PY) + iy, YS);
                    if (voff != last) {
                        last = voff;
                        P[0] = load_pair_g<C>(vb, voff);
                        P[1] = load_pair_g<C>(vb, voff + YS);
                        P[2] = load_pair_g<C>(vb, voff + ZS);
                        P[3] = load_pair_g<C>(vb, voff + YZ);
                    }
                });
        }
    }
    if (A.ms.seg > 1) {
        __syncthreads();   // every wave is done with its staging buffer
        gather_segments<C>(smem, A.ms.seg, rpb, sid, acc, nsamp);
    }
    const bool owner = valid && sid == 0;
    const float dt = (float)g.dt;
    if (owner && A.p_out) A.p_out[iu + (size_t)g.nu * iv] = dt * acc[0];
    if (A.partials) {
        constexpr int NM = 5 + 3 * (C - 1);
        double mo[NM + 1];
#pragma unroll
        for (int i = 0; i < NM; ++i) mo[i] = 0.0;
        mo[NM] = sid == 0 ? (double)nsamp : 0.0;   // segments were gathered
        if (owner) {
            double yd = (double)A.y[iu + (size_t)g.nu * iv];
            double pd = (double)(dt * acc[0]);
            mo[0] = yd;
            mo[1] = yd * yd;
            mo[2] = pd;
            mo[3] = yd * pd;
            mo[4] = pd * pd;
#pragma unroll
            for (int k = 0; k < C - 1; ++k) {
                if (k + 1 < A.kc) {
                    double tk = (double)(dt * acc[k + 1]);
                    mo[5 + 3 * k] = pd * tk;
                    mo[6 + 3 * k] = yd * tk;
                    mo[7 + 3 * k] = tk;
                }
            }
        }
        block_sum_store<NM + 1>(mo, NM + 1, A.partials + blockIdx.x, (int)gridDim.x, rpb / 64);
    }
}

// ------------------------------------------------------------ support --
// Bounds of the nonzero voxels of each slice of an image (see
// launch_support), combined with atomics.  NaN counts as nonzero.
template <typename F>
__global__ void __launch_bounds__(256) k_support(const F* __restrict__ f0, int nx, int ny, int nz,
                                                 int* __restrict__ sl)
{
    __shared__ int sb[8];
    const int nxy = nx * ny;
    for (int z = blockIdx.y; z < nz; z += gridDim.y) {
        if (threadIdx.x < 8) sb[threadIdx.x] = (threadIdx.x & 1) ? INT_MIN : INT_MAX;
        __syncthreads();
        int b[8] = {INT_MAX, INT_MIN, INT_MAX, INT_MIN, INT_MAX, INT_MIN, INT_MAX, INT_MIN};
        for (int e = blockIdx.x * 256 + threadIdx.x; e < nxy; e += gridDim.x * 256) {
            const float v = widen<float>(f0[(size_t)z * nxy + e]);
            if (!(v == 0.0f)) {
                const int x = e % nx, y = e / nx;
                const int q[4] = {x, y, x + y, x - y};
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    b[2 * c] = min(b[2 * c], q[c]);
                    b[2 * c + 1] = max(b[2 * c + 1], q[c]);
                }
            }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                b[2 * c] = min(b[2 * c], __shfl_xor(b[2 * c], o));
                b[2 * c + 1] = max(b[2 * c + 1], __shfl_xor(b[2 * c + 1], o));
            }
        }
        if ((threadIdx.x & 63) == 0) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                atomicMin(&sb[2 * c], b[2 * c]);
                atomicMax(&sb[2 * c + 1], b[2 * c + 1]);
            }
        }
        __syncthreads();
        if (threadIdx.x < 8) {
            int* t = sl + (size_t)8 * z + threadIdx.x;
            if (threadIdx.x & 1) atomicMax(t, sb[threadIdx.x]);
            else atomicMin(t, sb[threadIdx.x]);
        }
        __syncthreads();
    }
}

// out[row] = max |a[row][i]| over i < n, combined with atomics on the bit
// patterns of the (non-negative) floats; the caller zeroes `out` first.
template <typename S>
__global__ void __launch_bounds__(256) k_absmax_rows(const S* __restrict__ a, size_t n,
                                                     float* __restrict__ out)
{
    __shared__ float wm[4];
    const S* row = a + (size_t)blockIdx.y * n;
    float m = 0.0f;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
        m = fmaxf(m, fabsf(widen<float>(row[i])));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
    __syncthreads();
    // one atomic per block (few blocks per row: little contention)
    if (threadIdx.x == 0)
        atomicMax((int*)&out[blockIdx.y], __float_as_int(fmaxf(fmaxf(wm[0], wm[1]), fmaxf(wm[2], wm[3]))));
}

// ------------------------------------------------- gather backprojection --
// P^T r as a gather: every output voxel sums, over the rays whose samples can
// touch it, r * dt * (its trilinear weight) at each sample -- the weight the
// forward march gives that voxel as a corner of the sample's cell, i.e.
// prod_a max(0, 1 - |q_a - v_a|).  No global atomics, and every voxel's sum
// is formed in a fixed order, so the result is deterministic.
//
// A workgroup owns a brick of 16 x 4 x 4 voxels whose long side runs along
// the rays' dominant in-plane axis A: 16 columns of 16 voxels along A.  It
// walks the brick's detector footprint in tiles of 8 (u) x 32 (v) pixels; per
// tile every thread stages one ray in LDS (the sample nearest the brick centre relative
// to the brick origin, the step per sample, slab bounds, r dt and the valid
// sample range [0, floor(L / dt)]).  Then the 16 threads of a column split
// the rays of the column's own footprint between them; for each ray a slab
// test gives the samples that pass within one voxel of the column's line,
// and each such sample adds its weight to the two voxels of the column that
// straddle it along A (a per-thread run of 16 accumulators in LDS).  Per ray
// the set-up is paid once per column instead of once per voxel, and each
// sample is visited once.  A fixed-order sum over the 16 threads of each
// column gives the voxel values.
struct BPFoot {
    // for an index-space point X: a = a0 + an.X (depth along the central
    // ray, mm), b = b0 + bn.X and c = c0 + cn.X (offsets along e_u, e_v);
    // it projects to u = sdd b / a + su, v = sdd c / a + sv (mm)
    float a0, an[3], b0, bn[3], c0, cn[3];
    float sdd, su, sv, u0, inv_du, v0, inv_dv;
    int nu, nv;
};

// Pixel box (inclusive, clipped to the detector) that holds every ray
// meeting the index-space box [lo, hi]: the pixels whose centres lie in the
// bounding box of the projected corners (the box projects inside their
// convex hull), widened by `eps` pixels for the FP32 rounding of the
// projection; empty (i0 > i1) if none can.
__device__ __forceinline__ void footprint(const BPFoot& F, const float lo[3], const float hi[3],
                                          float eps, int& iu0, int& iu1, int& iv0, int& iv1)
{
    float umin = 3.0e38f, umax = -3.0e38f, vmin = 3.0e38f, vmax = -3.0e38f;
    bool front = true;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const float X = (c & 1) ? hi[0] : lo[0], Y = (c & 2) ? hi[1] : lo[1], Z = (c & 4) ? hi[2] : lo[2];
        const float a = F.a0 + F.an[0] * X + F.an[1] * Y + F.an[2] * Z;
        const float b = F.b0 + F.bn[0] * X + F.bn[1] * Y + F.bn[2] * Z;
        const float cc = F.c0 + F.cn[0] * X + F.cn[1] * Y + F.cn[2] * Z;
        front = front && a > 1e-3f;
        // the boxes are widened by at least 0.02 pixels, far beyond the
        // error of the hardware reciprocal
        const float t = F.sdd * __builtin_amdgcn_rcpf(a);
        const float u = fmaf(t, b, F.su), v = fmaf(t, cc, F.sv);
        umin = fminf(umin, u);
        umax = fmaxf(umax, u);
        vmin = fminf(vmin, v);
        vmax = fmaxf(vmax, v);
    }
    if (!front) {  // the box reaches behind the source: every pixel
        iu0 = 0; iu1 = F.nu - 1; iv0 = 0; iv1 = F.nv - 1;
        return;
    }
    iu0 = max(0, (int)ceilf(fmaxf((umin - F.u0) * F.inv_du - eps, -2.0f)));
    iu1 = min(F.nu - 1, (int)floorf(fminf((umax - F.u0) * F.inv_du + eps, (float)F.nu + 2.0f)));
    iv0 = max(0, (int)ceilf(fmaxf((vmin - F.v0) * F.inv_dv - eps, -2.0f)));
    iv1 = min(F.nv - 1, (int)floorf(fminf((vmax - F.v0) * F.inv_dv + eps, (float)F.nv + 2.0f)));
}

struct BPArgs {
    RayGeom g;            // unswapped (x-fastest) geometry
    BPFoot F;
    int ax;               // column axis A: 0 (x) or 1 (y)
    int bx, by, bz;       // brick: 16 along A, 4 along the other two axes
    int nbx, nby;         // bricks per axis
    int nx, ny, nz;
    double a, b, scale;   // r = scale (p - a y - b) when no residual is given
    double inv_dt;        // 1 / sample spacing
};

template <typename R>
struct alignas(4 * sizeof(R)) BPVec4 {
    R x, y, z, w;
};

template <typename R>
__global__ void __launch_bounds__(256) k_backproject_columns(BPArgs A, const R* __restrict__ resid,
                                                             const R* __restrict__ p,
                                                             const R* __restrict__ y,
                                                             R* __restrict__ out)
{
    // One staged ray in four 16-byte records (two 32-byte ones in FP64), read
    // with one wide load each; consecutive rays sit in consecutive records,
    // so the lanes of a column, which take consecutive rays, read without
    // bank conflicts.  Axes in column order (A, B, z):
    //   s_r0: the sample nearest the brick centre minus the brick origin, r dt
    //   s_r1: the index-space step per sample, slab lower bound along A
    //   s_r2: slab upper bound along A; lo, hi, 1/step across the column in B
    //   s_r3: lo, hi, 1/step across the column in z
    // Slab bounds are in samples: |q_a + m d_a - l| < 1 for m in
    // (lo_a + l inv_a, hi_a + l inv_a); along A the whole column (-1, 16),
    // narrowed to the ray's valid samples.
    __shared__ BPVec4<R> s_r0[256], s_r1[256];
    __shared__ float4 s_r2[256], s_r3[256];
    // thread t's run of 21 accumulators: 16 voxels along A at slots [2, 18)
    // (two pad slots each side take the clipped weights of samples just
    // outside the column, so the accumulation needs no branch); slot-major,
    // slot s of thread t at s * 256 + t, so each slot of the 64 lanes of a
    // wave spans all banks and a lane's bank does not depend on the slot:
    // the read-modify-writes never conflict
    __shared__ R s_acc[21 * 256];
    __shared__ int s_box[4];
    const RayGeom& g = A.g;
    const int t = threadIdx.x;
    const int bid = blockIdx.x;
    const int b0[3] = {(bid % A.nbx) * A.bx, ((bid / A.nbx) % A.nby) * A.by, (bid / (A.nbx * A.nby)) * A.bz};
    const int AX = A.ax, BX = 1 - A.ax;           // column axis and the other in-plane axis
    // a wave holds 4 columns x 16 lanes: consecutive lanes take consecutive
    // rays of one column, so their record loads hit distinct banks
    const int col = t >> 4, lane = t & 15;        // column (lb, lz) and ray lane
    const int lb = col & 3, lz = col >> 2;
    for (int e = t; e < 256 * 21; e += 256) s_acc[e] = (R)0;
    R* acc = s_acc + 2 * 256 + t;
    if (t == 0) {
        const float lo[3] = {(float)(b0[0] - 1), (float)(b0[1] - 1), (float)(b0[2] - 1)};
        const float hi[3] = {(float)(b0[0] + A.bx), (float)(b0[1] + A.by), (float)(b0[2] + A.bz)};
        footprint(A.F, lo, hi, 1.0f, s_box[0], s_box[1], s_box[2], s_box[3]);
    }
    // the column's footprint: its line (-1, 16) along A, one voxel around it
    int ru0, ru1, rv0, rv1;
    {
        float lo[3], hi[3];
        lo[AX] = (float)(b0[AX] - 1);
        hi[AX] = (float)(b0[AX] + 16);
        lo[BX] = (float)(b0[BX] + lb - 1);
        hi[BX] = (float)(b0[BX] + lb + 1);
        lo[2] = (float)(b0[2] + lz - 1);
        hi[2] = (float)(b0[2] + lz + 1);
        footprint(A.F, lo, hi, 0.02f, ru0, ru1, rv0, rv1);
    }
    __syncthreads();
    const int bu0 = s_box[0], bu1 = s_box[1], bv0 = s_box[2], bv1 = s_box[3];
    const double cb[3] = {b0[0] + 0.5 * (A.bx - 1), b0[1] + 0.5 * (A.by - 1), b0[2] + 0.5 * (A.bz - 1)};
    const float flb = (float)lb, flz = (float)lz;
    const R rlb = (R)lb, rlz = (R)lz;
    // Tiles of 8 (u) x 32 (v) rays: a column's footprint is wide along u (the
    // column runs along A) and short along v, so a tall, narrow tile holds
    // the footprints of all 16 columns at once and gives the 16 lanes of a
    // column rays that cross it alike (the lanes of a wave then run their
    // sample loops for similar lengths: ~0.55 of the lanes busy in the loop
    // against ~0.3 with 16 x 16 tiles, and ~40 % fewer rounds of rays)
    for (int tv0 = bv0; tv0 <= bv1; tv0 += 32) {
        for (int tu0 = bu0; tu0 <= bu1; tu0 += 8) {
            {   // stage one ray per thread (FP64 set-up, once per ray and brick)
                const int iu = tu0 + (t & 7), iv = tv0 + (t >> 3);
                int m0 = 1, m1 = 0;
                R rw = (R)0;
                double qr[3] = {0.0, 0.0, 0.0}, dq[3] = {0.0, 0.0, 0.0};
                if (iu <= bu1 && iv <= bv1) {
                    const size_t pix = iu + (size_t)g.nu * iv;
                    const double r = resid ? (double)resid[pix]
                                           : A.scale * ((double)p[pix] - A.a * (double)y[pix] - A.b);
                    const double uu = g.u0 + iu * g.du, vv = g.v0 + iv * g.dv;
                    double D[3], L2 = 0.0;
#pragma unroll
                    for (int ax = 0; ax < 3; ++ax) {
                        D[ax] = g.qc[ax] + uu * g.eu[ax] + vv * g.ev[ax] - g.qs[ax];
                        const double w = D[ax] * g.sp[ax];
                        L2 += w * w;
                    }
                    if (L2 > 0.0 && r != 0.0) {
                        // 1/L from the hardware reciprocal square root and two
                        // Newton steps (each doubles the correct bits)
                        double invL = __builtin_amdgcn_rsq(L2);
                        invL = fma(0.5 * invL, fma(-L2 * invL, invL, 1.0), invL);
                        invL = fma(0.5 * invL, fma(-L2 * invL, invL, 1.0), invL);
                        const double L = L2 * invL;
                        double tc = 0.0;
#pragma unroll
                        for (int ax = 0; ax < 3; ++ax) {
                            D[ax] *= invL;   // index units per mm
                            tc += (cb[ax] - g.qs[ax]) * g.sp[ax] * g.sp[ax] * D[ax];
                        }
                        // the last sample lies at the detector, far outside the
                        // volume, and the centre sample only anchors m: neither
                        // needs a correctly rounded quotient
                        const double nlast = floor(L * A.inv_dt);
                        const double nc = fmin(fmax(rint(tc * A.inv_dt), 0.0), nlast);
                        const double tn = nc * g.dt;
#pragma unroll
                        for (int ax = 0; ax < 3; ++ax) {
                            qr[ax] = g.qs[ax] + tn * D[ax] - (double)b0[ax];
                            dq[ax] = g.dt * D[ax];
                        }
                        m0 = -(int)nc;
                        m1 = (int)(nlast - nc);
                        rw = (R)(r * g.dt);
                    }
                }
                float lo[3], hi[3], inv[3];
#pragma unroll
                for (int ax = 0; ax < 3; ++ax) {
                    const float df = (float)dq[ax];
                    // the slab bounds carry a 1e-3 sample slack, so the
                    // hardware reciprocal (1 ulp) is exact enough
                    inv[ax] = fabsf(df) > 1e-30f ? __builtin_amdgcn_rcpf(df) : 1.0e30f;
                    const float e1 = (-1.0f - (float)qr[ax]) * inv[ax];
                    const float e2 = ((ax == AX ? 16.0f : 1.0f) - (float)qr[ax]) * inv[ax];
                    lo[ax] = fminf(e1, e2);
                    hi[ax] = fmaxf(e1, e2);
                }
                // the valid samples [m0, m1] narrow the bounds along A: with
                // the half-sample margin the rounding below yields exactly
                // max(m0, .) and min(m1, .) (|m| < 2^22 where they bind)
                const float la = fmaxf(lo[AX], (float)m0 - 0.5f), ha = fminf(hi[AX], (float)m1 + 0.5f);
                s_r0[t] = {(R)qr[AX], (R)qr[BX], (R)qr[2], rw};
                s_r1[t] = {(R)dq[AX], (R)dq[BX], (R)dq[2], (R)la};
                s_r2[t] = make_float4(ha, lo[BX], hi[BX], inv[BX]);
                s_r3[t] = make_float4(lo[2], hi[2], inv[2], 0.0f);
            }
            __syncthreads();
            // rays of this tile inside the column's footprint, split over the
            // column's 16 lanes
            const int ua = max(ru0, tu0), ub = min(ru1, tu0 + 7);
            const int va = max(rv0, tv0), vb = min(rv1, tv0 + 31);
            const int wu = ub - ua + 1, nr = (ub >= ua && vb >= va) ? wu * (vb - va + 1) : 0;
            // ray i of the clipped box (row-major) is (i % wu, i / wu); the
            // lane steps i by 16, i.e. (16 % wu, 16 / wu) with one carry
            const int kb = ((va - tv0) << 3) + (ua - tu0);
            int ou = 0, ov = 0, su = 0, sv = 0;
            if (nr > 0) {
                ou = lane % wu;
                ov = lane / wu;
                su = 16 % wu;
                sv = 16 / wu;
            }
            for (int i = lane; i < nr; i += 16) {
                const int k = kb + (ov << 3) + ou;
                ou += su;
                ov += sv;
                if (ou >= wu) {
                    ou -= wu;
                    ++ov;
                }
                // samples within one voxel of the column line (slab test; the
                // 1e-3 sample slack covers the FP32 rounding of the bounds and
                // the weights clip any sample it admits)
                const BPVec4<R> r0 = s_r0[k], r1 = s_r1[k];
                const float4 r2 = s_r2[k], r3 = s_r3[k];
                float lo = fmaxf(fmaxf((float)r1.w, fmaf(flb, r2.w, r2.y)), fmaf(flz, r3.z, r3.x));
                float hi = fminf(fminf(r2.x, fmaf(flb, r2.w, r2.z)), fmaf(flz, r3.z, r3.y));
                lo = fminf(fmaxf(lo, -1.0e6f), 1.0e6f);   // |m| stays far inside int range
                hi = fminf(fmaxf(hi, -1.0e6f), 1.0e6f);
                const int m0 = (int)ceilf(lo - 1.0e-3f);
                const int m1 = (int)floorf(hi + 1.0e-3f);
                if (m0 > m1) continue;
                const R qa = r0.x, qb = r0.y - rlb, qz = r0.z - rlz;
                const R da = r1.x, db = r1.y, dz = r1.z;
                const R rw = r0.w;
                // the sample index runs as a float (|m| < 1e6: exact)
                const R fm1 = (R)m1;
                // the ray's values are in registers before the loop starts,
                // so no wait inside it holds back for the previous sample's
                // LDS write
                __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0)
                for (R fm = (R)m0; fm <= fm1; fm += (R)1) {
                    const R wbz = fmax((R)0, (R)1 - fabs(fma(fm, db, qb))) *
                                  fmax((R)0, (R)1 - fabs(fma(fm, dz, qz))) * rw;
                    const R xa = fma(fm, da, qa);
                    const R fl = floor(xa);
                    // the slab range keeps xa within (-1.01, 16.01); the clamp
                    // only guards the LDS run
                    const int j = min(max((int)fl, -2), 16);
                    const R fa = xa - fl;
                    // the thread's own LDS run: a plain read-modify-write
                    acc[j * 256] += ((R)1 - fa) * wbz;
                    acc[(j + 1) * 256] += fa * wbz;
                }
            }
            __syncthreads();
        }
    }
    // voxel (column c, position j along A): the sum over the column's 16
    // lanes, in an order rotated by j so that the lanes of a wave read
    // different banks
    {
        const int c = t >> 4, j = t & 15;
        R v = (R)0;
        for (int l = 0; l < 16; ++l) v += s_acc[(2 + j) * 256 + c * 16 + ((l + j) & 15)];
        int vx[3];
        vx[AX] = b0[AX] + j;
        vx[BX] = b0[BX] + (c & 3);
        vx[2] = b0[2] + (c >> 2);
        if (vx[0] < A.nx && vx[1] < A.ny && vx[2] < A.nz)
            out[(size_t)vx[0] + (size_t)A.nx * ((size_t)vx[1] + (size_t)A.ny * vx[2])] = v;
    }
}

// ---------------------------------------------------------- contraction --
// partials[k * blocks + block] = sum_v g[v] * sum_a (1/s_a) dT[f0]/dq_a(q_v) u_k[a][v]
template <typename R, typename S, typename F>
__global__ void __launch_bounds__(256) k_contract(const F* __restrict__ f0,
                                                  const S* __restrict__ mean,
                                                  const S* __restrict__ U, int K,
                                                  Chan<double, 8> w, VoxGrid g,
                                                  const R* __restrict__ gpad,
                                                  double* __restrict__ partials)
{
    const int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y * 4 + threadIdx.y;
    double m[8];
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) m[kk] = 0.0;
    for (int k = blockIdx.z; k < g.nz; k += gridDim.z) {
    if (i < g.nx && j < g.ny) {
        size_t N = (size_t)g.nx * g.ny * g.nz;
        size_t v = (size_t)i + (size_t)g.nx * ((size_t)j + (size_t)g.ny * k);
        R gv = gpad[v];
        if (gv != (R)0) {
            R x[3], u[8][3];
#pragma unroll
            for (int a = 0; a < 3; ++a) x[a] = widen<R>(mean[a * N + v]);
#pragma unroll
            for (int kk = 0; kk < 8; ++kk)
                if (kk < K)
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        u[kk][a] = widen<R>(U[(size_t)(kk * 3 + a) * N + v]);
                        x[a] += (R)w.v[kk] * u[kk][a];
                    }
            R qx = (R)i + x[0] / (R)g.sp[0];
            R qy = (R)j + x[1] / (R)g.sp[1];
            R qz = (R)k + x[2] / (R)g.sp[2];
            R dT[3];
            sample_f0<R, F, true>(f0, g.nx, g.ny, g.nz, qx, qy, qz, dT);
            double G0 = (double)dT[0] / g.sp[0], G1 = (double)dT[1] / g.sp[1],
                   G2 = (double)dT[2] / g.sp[2];
            double gd = (double)gv;
#pragma unroll
            for (int kk = 0; kk < 8; ++kk)
                if (kk < K)
                    m[kk] += gd * (G0 * (double)u[kk][0] + G1 * (double)u[kk][1] + G2 * (double)u[kk][2]);
        }
    }
    }
    // threadIdx is 2-D (64 x 4): flatten for the block reduction
    __shared__ double red[4][8];
    const int lane = threadIdx.x, wv = threadIdx.y;
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
        double s = wave_sum(m[kk]);
        if (lane == 0) red[wv][kk] = s;
    }
    __syncthreads();
    int t = threadIdx.x + 64 * threadIdx.y;
    if (t < K) {
        size_t blk = blockIdx.x + (size_t)gridDim.x * (blockIdx.y + (size_t)gridDim.y * blockIdx.z);
        size_t nblk = (size_t)gridDim.x * gridDim.y * gridDim.z;
        partials[t * nblk + blk] = red[0][t] + red[1][t] + red[2][t] + red[3][t];
    }
}

// -------------------------------------------------------- warp adjoint ---
template <typename R>
__global__ void __launch_bounds__(256) k_warp_adjoint(const R* __restrict__ dvf,
                                                      const R* __restrict__ gv, VoxGrid g,
                                                      R* __restrict__ out)
{
    int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y * 4 + threadIdx.y, k = blockIdx.z;
    if (i >= g.nx || j >= g.ny) return;
    size_t N = (size_t)g.nx * g.ny * g.nz;
    size_t v = (size_t)i + (size_t)g.nx * ((size_t)j + (size_t)g.ny * k);
    R val = gv[v];
    if (val == (R)0) return;
    R qx = (R)i + dvf[v] / (R)g.sp[0];
    R qy = (R)j + dvf[N + v] / (R)g.sp[1];
    R qz = (R)k + dvf[2 * N + v] / (R)g.sp[2];
    qx = clampv(qx, (R)-2, (R)(g.nx + 1));
    qy = clampv(qy, (R)-2, (R)(g.ny + 1));
    qz = clampv(qz, (R)-2, (R)(g.nz + 1));
    R fx = floor(qx), fy = floor(qy), fz = floor(qz);
    int i0 = (int)fx, j0 = (int)fy, k0 = (int)fz;
    R ax = qx - fx, ay = qy - fy, az = qz - fz;
    R wx[2] = {(R)1 - ax, ax}, wy[2] = {(R)1 - ay, ay}, wz[2] = {(R)1 - az, az};
#pragma unroll
    for (int dz = 0; dz < 2; ++dz)
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) {
                int ii = i0 + dx, jj = j0 + dy, kk = k0 + dz;
                if ((unsigned)ii < (unsigned)g.nx && (unsigned)jj < (unsigned)g.ny &&
                    (unsigned)kk < (unsigned)g.nz)
                    unsafeAtomicAdd(out + ((size_t)ii + (size_t)g.nx * ((size_t)jj + (size_t)g.ny * kk)),
                                    wx[dx] * wy[dy] * wz[dz] * val);
            }
}

// ------------------------------------------------------------ localise ---
// One wave: lane t < 8 owns trilinear corner t; FP64 throughout.
template <typename S>
__global__ void __launch_bounds__(64) k_localize(const S* __restrict__ mean,
                                                 const S* __restrict__ U, int K,
                                                 Chan<double, 8> w, VoxGrid g, double pr0,
                                                 double pr1, double pr2, double org0, double org1,
                                                 double org2, double tol, int max_iter,
                                                 double* __restrict__ out)
{
    const int t = threadIdx.x;
    const size_t N = (size_t)g.nx * g.ny * g.nz;
    const int n[3] = {g.nx, g.ny, g.nz};
    const double org[3] = {org0, org1, org2};
    const double pref[3] = {pr0, pr1, pr2};
    double p[3] = {pr0, pr1, pr2};
    int it = 0, conv = 0;
    for (it = 1; it <= max_iter; ++it) {
        int i0[3];
        double ph[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double q = (p[a] - org[a]) / g.sp[a];
            double hi = (double)(n[a] - 1);
            q = fmin(fmax(q, 0.0), hi);
            double fl = floor(q);
            if (n[a] >= 2 && fl > hi - 1.0) fl = hi - 1.0;
            i0[a] = (int)fl;
            ph[a] = q - fl;
        }
        double X[3] = {0.0, 0.0, 0.0};
        if (t < 8) {
            int dx = t & 1, dy = (t >> 1) & 1, dz = t >> 2;
            double wt = (dx ? ph[0] : 1.0 - ph[0]) * (dy ? ph[1] : 1.0 - ph[1]) *
                        (dz ? ph[2] : 1.0 - ph[2]);
            if (wt != 0.0) {
                size_t v = (size_t)(i0[0] + dx) + (size_t)g.nx * ((size_t)(i0[1] + dy) + (size_t)g.ny * (i0[2] + dz));
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    double x = widen<double>(mean[a * N + v]);
                    for (int k = 0; k < K; ++k) x += w.v[k] * widen<double>(U[(size_t)(k * 3 + a) * N + v]);
                    X[a] = wt * x;
                }
            }
        }
        // fixed-order sum over the 8 corners
#pragma unroll
        for (int a = 0; a < 3; ++a) {
#pragma unroll
            for (int off = 4; off > 0; off >>= 1) X[a] += __shfl_down(X[a], off, 8);
            X[a] = __shfl(X[a], 0, 64);
        }
        double d2 = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double pn = pref[a] - X[a];
            d2 += (pn - p[a]) * (pn - p[a]);
            p[a] = pn;
        }
        if (sqrt(d2) < tol) {
            conv = 1;
            break;
        }
    }
    if (t == 0) {
        out[0] = p[0];
        out[1] = p[1];
        out[2] = p[2];
        out[3] = (double)(it > max_iter ? max_iter : it);
        out[4] = (double)conv;
    }
}

// ============================================================ launchers ===
static VoxGrid vox(const pcr_grid& g)
{
    VoxGrid v;
    v.nx = g.n[0];
    v.ny = g.n[1];
    v.nz = g.n[2];
    for (int a = 0; a < 3; ++a) v.sp[a] = g.spacing_mm[a];
    return v;
}
static dim3 vox_grid(const pcr_grid& g)
{
    return dim3((g.n[0] + 63) / 64, (g.n[1] + 3) / 4, g.n[2]);
}
static Chan<double, 8> wvec(const double* w, int K)
{
    Chan<double, 8> c;
    for (int k = 0; k < 8; ++k) c.v[k] = k < K ? w[k] : 0.0;
    return c;
}

PadLayout make_pad(const pcr_grid& g, int C, bool yfast)
{
    PadLayout L;
    L.nx = g.n[0];
    L.ny = g.n[1];
    L.nz = g.n[2];
    L.px = (yfast ? L.ny : L.nx) + 3;
    L.py = (yfast ? L.nx : L.ny) + 3;
    L.pz = L.nz + 3;
    L.C = C;
    L.yfast = yfast;
    return L;
}

bool prefer_yfast(const pcr_geom& G)
{
    // Measured on the paper-scale volume: the x-fastest layout with compact
    // ray tiles is fastest at every angle except within ~15 degrees of the y
    // axis (rays along x), where the y-fastest layout with one thread per ray
    // gains ~10 %.
    return std::fabs(std::sin(G.angle_rad)) > 0.97;
}

RayGeom make_ray_geom(const pcr_grid& g, const pcr_geom& G, bool swap_xy)
{
    RayGeom r;
    double st = std::sin(G.angle_rad), ct = std::cos(G.angle_rad);
    double s[3] = {G.iso_mm[0] + G.sad_mm * st, G.iso_mm[1] - G.sad_mm * ct, G.iso_mm[2]};
    double dd = G.sdd_mm - G.sad_mm;
    double c[3] = {G.iso_mm[0] - dd * st, G.iso_mm[1] + dd * ct, G.iso_mm[2]};
    double eu[3] = {ct, st, 0.0}, ev[3] = {0.0, 0.0, 1.0};
    for (int a = 0; a < 3; ++a) {
        r.sp[a] = g.spacing_mm[a];
        r.qs[a] = (s[a] - g.origin_mm[a]) / g.spacing_mm[a];
        r.qc[a] = (c[a] - g.origin_mm[a]) / g.spacing_mm[a];
        r.eu[a] = eu[a] / g.spacing_mm[a];
        r.ev[a] = ev[a] / g.spacing_mm[a];
        r.lim[a] = (double)g.n[a];
        r.clo[a] = -1.0;
        r.chi[a] = r.lim[a];
    }
    if (swap_xy) {
        std::swap(r.sp[0], r.sp[1]);
        std::swap(r.qs[0], r.qs[1]);
        std::swap(r.qc[0], r.qc[1]);
        std::swap(r.eu[0], r.eu[1]);
        std::swap(r.ev[0], r.ev[1]);
        std::swap(r.lim[0], r.lim[1]);
        std::swap(r.chi[0], r.chi[1]);
    }
    r.u0 = -0.5 * (G.nu - 1) * G.du_mm + G.off_u_mm;
    r.v0 = -0.5 * (G.nv - 1) * G.dv_mm + G.off_v_mm;
    r.du = G.du_mm;
    r.dv = G.dv_mm;
    r.dt = G.step_mm;
    r.nu = G.nu;
    r.nv = G.nv;
    return r;
}

MarchShape choose_march_shape(const RayGeom& rg)
{
    MarchShape ms;
    long rays = (long)rg.nu * rg.nv;
    // aim for >= ~8 waves per SIMD on 1024 SIMDs: split rays into segments
    // when they are few; each wave takes 4 (u) x 16 (v) rays, stepping
    // through the union of their sample ranges together (measured best on
    // both layouts)
    ms.seg = rays >= 8L * 1024 * 64 ? 1 : (rays >= 4L * 1024 * 64 ? 2 : 4);
    ms.tile_u = 4;
    return ms;
}

static int tiles_u_of(const RayGeom& rg, const MarchShape& ms)
{
    return (rg.nu + ms.tile_u - 1) / ms.tile_u;
}

int march_blocks(const RayGeom& rg, const MarchShape& ms)
{
    int rpb = 256 / ms.seg, rows = rpb / ms.tile_u;
    return tiles_u_of(rg, ms) * ((rg.nv + rows - 1) / rows);
}

// Contraction grid: x-y tiles of 64 x 4 voxels, z split over enough blocks to
// fill the chip (each block then loops over its z slices).
static dim3 contract_grid(const pcr_grid& g)
{
    dim3 d = vox_grid(g);
    unsigned xy = d.x * d.y;
    unsigned zb = std::max(1u, std::min((unsigned)g.n[2], (2048u + xy - 1) / xy));
    return dim3(d.x, d.y, zb);
}

int contract_blocks(const pcr_grid& g)
{
    dim3 d = contract_grid(g);
    return (int)(d.x * d.y * d.z);
}

#define PCR_DISPATCH_S(dt, S, ...)                                   \
    switch (dt) {                                                    \
    case PCR_F32: { using S = float; __VA_ARGS__; } break;           \
    case PCR_F64: { using S = double; __VA_ARGS__; } break;          \
    case PCR_BF16: { using S = bf16; __VA_ARGS__; } break;           \
    case PCR_F16: { using S = _Float16; __VA_ARGS__; } break;        \
    default: return hipErrorInvalidValue;                            \
    }
#define PCR_DISPATCH_R(dt, R, ...)                                   \
    switch (dt) {                                                    \
    case PCR_F32: { using R = float; __VA_ARGS__; } break;           \
    case PCR_F64: { using R = double; __VA_ARGS__; } break;          \
    default: return hipErrorInvalidValue;                            \
    }

hipError_t launch_compose(pcr_dtype compute, pcr_dtype storage, const pcr_grid& g, int K,
                          const void* mean, const void* U, const double* w_eff, void* dvf,
                          hipStream_t s)
{
    size_t N = (size_t)g.n[0] * g.n[1] * g.n[2];
    unsigned blocks = (unsigned)((N + 255) / 256);
    PCR_DISPATCH_R(compute, R, PCR_DISPATCH_S(storage, S,
        k_compose<R, S><<<blocks, 256, 0, s>>>((const S*)mean, (const S*)U, K, N, wvec(w_eff, K),
                                               (R*)dvf)));
    return hipGetLastError();
}

hipError_t launch_warp_plain(pcr_dtype compute, pcr_dtype f0_dtype, const pcr_grid& g,
                             const void* f0, const void* dvf, void* f, hipStream_t s)
{
    PCR_DISPATCH_R(compute, R, PCR_DISPATCH_S(f0_dtype, S,
        k_warp_plain<R, S><<<vox_grid(g), dim3(64, 4), 0, s>>>((const S*)f0, (const R*)dvf, vox(g),
                                                               (R*)f)));
    return hipGetLastError();
}

template <typename R, typename S, typename F>
static hipError_t warp_fused_c(const pcr_grid& g, const PadLayout& L, int K, bool tangent,
                               const void* f0, const void* mean, const void* U,
                               const double* w_eff, const int* box, void* padded, hipStream_t s)
{
    VoxBox b;
    for (int a = 0; a < 3; ++a) {
        b.lo[a] = box ? std::max(0, box[a]) : 0;
        b.hi[a] = box ? std::min(g.n[a], box[3 + a]) : g.n[a];
        if (b.hi[a] <= b.lo[a]) return hipSuccess;   // nothing to compute
    }
    const int ex = b.hi[0] - b.lo[0], ey = b.hi[1] - b.lo[1], ez = b.hi[2] - b.lo[2];
    dim3 grid((ex + 255) / 256, ey, ez), blk(256, 1);
    auto w = wvec(w_eff, K);
    // one-dimensional grid (the kernel orders its tiles by XCD), tiles of
    // yf_tile_x x 8 voxels
    const int gyy = (ey + 7) / 8;
    auto grid_yf = [&](int tx) { return dim3((unsigned)((long)((ex + tx - 1) / tx) * gyy * ez)); };
    if ((long)((ex + 31) / 32) * gyy * ez > 0x7fffffffL) return hipErrorInvalidValue;
    Chan<float, 8> hs;
    for (int c = 0; c < 8; ++c) hs.v[c] = L.hs[c];
#define PCR_WF2(C, T, H)                                                                          \
    (L.yfast ? k_warp_fused_yf<R, S, F, C, T, H><<<grid_yf(yf_tile_x<R, C, H>()), 256, 0, s>>>(  \
                   (const F*)f0, (const S*)mean, (const S*)U, K, w, vox(g), L.px, L.py, hs, b,    \
                   (ex + yf_tile_x<R, C, H>() - 1) / yf_tile_x<R, C, H>(), gyy,                   \
                   (CellOf<R, C, H>*)padded)                                                      \
             : k_warp_fused<R, S, F, C, T, H><<<grid, blk, 0, s>>>(                               \
                   (const F*)f0, (const S*)mean, (const S*)U, K, w, vox(g), L.px, L.py, hs, b,    \
                   (CellOf<R, C, H>*)padded))
#define PCR_WF(C, T) (L.half ? PCR_WF2(C, T, true) : PCR_WF2(C, T, false))
    if (L.half && !std::is_same<R, float>::value) return hipErrorInvalidValue;
    if (K < 1 || K > 8 || (tangent && K > L.C - 1)) return hipErrorInvalidValue;
    if (!tangent) {
        switch (L.C) {
        case 1: PCR_WF(1, false); break;
        case 2: PCR_WF(2, false); break;
        case 4: PCR_WF(4, false); break;
        case 6: PCR_WF(6, false); break;
        case 8: PCR_WF(8, false); break;
        default: return hipErrorInvalidValue;
        }
    } else {
        switch (L.C) {
        case 2: PCR_WF(2, true); break;
        case 4: PCR_WF(4, true); break;
        case 6: PCR_WF(6, true); break;
        case 8: PCR_WF(8, true); break;
        default: return hipErrorInvalidValue;
        }
    }
#undef PCR_WF
#undef PCR_WF2
    return hipGetLastError();
}

hipError_t launch_warp_fused(pcr_dtype compute, pcr_dtype storage, pcr_dtype f0_dtype,
                             const pcr_grid& g, const PadLayout& L, int K, bool tangent,
                             const void* f0, const void* mean, const void* U,
                             const double* w_eff, const int* box, void* padded, hipStream_t s)
{
    PCR_DISPATCH_R(compute, R, PCR_DISPATCH_S(storage, S, PCR_DISPATCH_S(f0_dtype, F,
        return warp_fused_c<R, S, F>(g, L, K, tangent, f0, mean, U, w_eff, box, padded, s))));
    return hipSuccess;
}

hipError_t launch_pad(pcr_dtype compute, const PadLayout& L, const void* vol, void* padded,
                      hipStream_t s)
{
    pcr_grid g{};
    g.n[0] = L.nx; g.n[1] = L.ny; g.n[2] = L.nz;
    g.spacing_mm[0] = g.spacing_mm[1] = g.spacing_mm[2] = 1.0;
    PCR_DISPATCH_R(compute, R,
        k_pad<R><<<vox_grid(g), dim3(64, 4), 0, s>>>((const R*)vol, vox(g), L.px, L.py, (R*)padded));
    return hipGetLastError();
}

hipError_t launch_unpad(pcr_dtype compute, const PadLayout& L, const void* padded, void* vol,
                        hipStream_t s)
{
    pcr_grid g{};
    g.n[0] = L.nx; g.n[1] = L.ny; g.n[2] = L.nz;
    g.spacing_mm[0] = g.spacing_mm[1] = g.spacing_mm[2] = 1.0;
    PCR_DISPATCH_R(compute, R,
        k_unpad<R><<<vox_grid(g), dim3(64, 4), 0, s>>>((const R*)padded, vox(g), L.px, L.py, (R*)vol));
    return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s)
{
    // A fill kernel rather than a memset node, so that the call is safe to
    // capture into a graph.  Buffers are whole 4-byte words.
    if (bytes == 0) return hipSuccess;
    if (bytes % 4 != 0 || (uintptr_t)p % 4 != 0) return hipErrorInvalidValue;
    if ((uintptr_t)p % 16 == 0 && bytes % 16 == 0) {
        size_t n16 = bytes / 16;
        unsigned blocks = (unsigned)std::min<size_t>((n16 + 255) / 256, 8192);
        k_zero16<<<blocks, 256, 0, s>>>((uint4*)p, n16);
    } else {
        size_t n4 = bytes / 4;
        unsigned blocks = (unsigned)std::min<size_t>((n4 + 255) / 256, 8192);
        k_zero4<<<blocks, 256, 0, s>>>((uint32_t*)p, n4);
    }
    return hipGetLastError();
}

template <typename R>
static hipError_t march_r(const PadLayout& L, int kc, const RayGeom& rg, const MarchShape& ms,
                          const void* padded, const void* y, void* p_out, double* partials,
                          double* moments, unsigned long long* done, unsigned long long seq,
                          hipStream_t s)
{
    int tiles_u = tiles_u_of(rg, ms);
    int blocks = march_blocks(rg, ms);
#define PCR_MARCH(C)                                                                     \
    k_march<R, C><<<blocks, 256, 0, s>>>(rg, ms, tiles_u, (const Chan<R, C>*)padded, L.px, \
                                         L.py, (float)rg.lim[0], (float)rg.lim[1],         \
                                         (float)rg.lim[2], kc, (const R*)y, (R*)p_out,     \
                                         moments ? partials : nullptr)
    switch (L.C) {
    case 1: PCR_MARCH(1); break;
    case 2: PCR_MARCH(2); break;
    case 4: PCR_MARCH(4); break;
    case 6: PCR_MARCH(6); break;
    case 8: PCR_MARCH(8); break;
    default: return hipErrorInvalidValue;
    }
#undef PCR_MARCH
    if (moments) {
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        return run_reduce(partials, blocks, n_moments(kc), n_moments(L.C), moments, s, done, seq);
    }
    return hipGetLastError();
}

bool march_f32_fits(const PadLayout& L)
{
    const double cb = (double)L.cell_bytes(4);
    return (double)L.px * L.py * L.pz * cb < 2147483648.0 && (double)L.py * L.pz < 16777216.0 &&
           (double)L.px * cb < 16777216.0;
}

static hipError_t march_f32(const PadLayout& L, int kc, const RayGeom& rg, const MarchShape& ms,
                            const void* padded, const void* y, void* p_out, double* partials,
                            double* moments, unsigned long long* done, unsigned long long seq,
                            hipStream_t s)
{
    if (!march_f32_fits(L)) return hipErrorInvalidValue;
    MarchArgs A;
    A.g = rg;
    A.ms = ms;
    A.tiles_u = tiles_u_of(rg, ms);
    A.vol = padded;
    const int cb = (int)L.cell_bytes(4);
    A.px = L.px;
    A.py = L.py;
    A.pz = L.pz;
    A.ys = L.px * cb;
    A.zs = L.px * L.py * cb;
    for (int c = 0; c < 8; ++c) A.ihs[c] = 1.0f / L.hs[c];
    for (int a = 0; a < 3; ++a) A.fn1[a] = (float)(rg.lim[a] + 1.0);
    A.kc = kc;
    A.y = (const float*)y;
    A.p_out = (float*)p_out;
    A.partials = moments ? partials : nullptr;
    A.moments = moments;
    int blocks = march_blocks(rg, ms);
    if (L.half && L.C == 1) return hipErrorInvalidValue;
    if (L.half) {
        switch (L.C) {
        case 2: k_march_f32<2, true><<<blocks, 256, 0, s>>>(A); break;
        case 4: k_march_f32<4, true><<<blocks, 256, 0, s>>>(A); break;
        case 8: k_march_f32<8, true><<<blocks, 256, 0, s>>>(A); break;
        default: return hipErrorInvalidValue;
        }
    } else {
        // every FP32 cell size stages through LDS (8-byte cells too: 11-18 %
        // faster than the gather through the L1 at paper scale, K = 1)
        switch (L.C) {
        case 1: k_march_lds<1><<<blocks, 256, 0, s>>>(A); break;
        case 2: k_march_lds<2><<<blocks, 256, 0, s>>>(A); break;
        case 4: k_march_lds<4><<<blocks, 256, 0, s>>>(A); break;
        case 6:
            // K = 4 sums 5 of the 6 channels.  (Summing only the channels in
            // use pays where the unused ones drop whole loads; 12-byte LDS
            // reads, as for K = 2 in 4-channel cells, were slower than
            // summing the zero channel: 183.6 against 145.6 us at K = 2.)
            if (kc == 5) k_march_lds<6, 5><<<blocks, 256, 0, s>>>(A);
            else k_march_lds<6><<<blocks, 256, 0, s>>>(A);
            break;
        case 8: k_march_lds<8><<<blocks, 256, 0, s>>>(A); break;
        default: return hipErrorInvalidValue;
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !moments) return e;
    return run_reduce(partials, blocks, n_moments(kc), n_moments(L.C), moments, s, done, seq);
}

hipError_t launch_march(pcr_dtype compute, const PadLayout& L, int kc, const RayGeom& rg,
                        const MarchShape& ms, const void* padded, const void* y, void* p_out,
                        double* partials, double* moments, unsigned long long* done,
                        unsigned long long seq, hipStream_t s)
{
    if (compute == PCR_F32)
        return march_f32(L, kc, rg, ms, padded, y, p_out, partials, moments, done, seq, s);
    if (compute == PCR_F64)
        return march_r<double>(L, kc, rg, ms, padded, y, p_out, partials, moments, done, seq, s);
    return hipErrorInvalidValue;
}

hipError_t launch_reduce(const double* partials, int nblocks, int nm, double* out, hipStream_t s)
{
    return run_reduce(partials, nblocks, nm, -1, out, s);
}

hipError_t launch_backproject(pcr_dtype compute, const pcr_grid& g, const RayGeom& rg,
                              const void* resid, const void* p, const void* y, double a, double b,
                              double scale, void* out, hipStream_t s)
{
    BPArgs A;
    A.g = rg;
    // footprint geometry (physical, mm): n = unit vector source -> detector
    // centre, e_u / e_v the detector axes; for X in index space the offset
    // from the source is (X - qs) * sp
    double n[3], eu[3], ev[3], nn = 0.0, sdd;
    for (int ax = 0; ax < 3; ++ax) {
        n[ax] = (rg.qc[ax] - rg.qs[ax]) * rg.sp[ax];
        nn += n[ax] * n[ax];
        eu[ax] = rg.eu[ax] * rg.sp[ax];
        ev[ax] = rg.ev[ax] * rg.sp[ax];
    }
    sdd = std::sqrt(nn);
    if (!(sdd > 0.0)) return hipErrorInvalidValue;
    double a0 = 0.0, b0 = 0.0, c0 = 0.0, su = 0.0, sv = 0.0;
    for (int ax = 0; ax < 3; ++ax) {
        n[ax] /= sdd;
        A.F.an[ax] = (float)(rg.sp[ax] * n[ax]);
        A.F.bn[ax] = (float)(rg.sp[ax] * eu[ax]);
        A.F.cn[ax] = (float)(rg.sp[ax] * ev[ax]);
        a0 -= rg.qs[ax] * rg.sp[ax] * n[ax];
        b0 -= rg.qs[ax] * rg.sp[ax] * eu[ax];
        c0 -= rg.qs[ax] * rg.sp[ax] * ev[ax];
        su += (rg.qs[ax] - rg.qc[ax]) * rg.sp[ax] * eu[ax];
        sv += (rg.qs[ax] - rg.qc[ax]) * rg.sp[ax] * ev[ax];
    }
    A.F.a0 = (float)a0;
    A.F.b0 = (float)b0;
    A.F.c0 = (float)c0;
    A.F.sdd = (float)sdd;
    A.F.su = (float)su;
    A.F.sv = (float)sv;
    A.F.u0 = (float)rg.u0;
    A.F.inv_du = (float)(1.0 / rg.du);
    A.F.v0 = (float)rg.v0;
    A.F.inv_dv = (float)(1.0 / rg.dv);
    A.F.nu = rg.nu;
    A.F.nv = rg.nv;
    // bricks elongated along the rays' dominant in-plane axis
    const double rx = std::fabs(rg.qc[0] - rg.qs[0]) * rg.sp[0], ry = std::fabs(rg.qc[1] - rg.qs[1]) * rg.sp[1];
    if (ry >= rx) { A.ax = 1; A.bx = 4; A.by = 16; } else { A.ax = 0; A.bx = 16; A.by = 4; }
    A.bz = 4;
    A.nx = g.n[0];
    A.ny = g.n[1];
    A.nz = g.n[2];
    A.nbx = (A.nx + A.bx - 1) / A.bx;
    A.nby = (A.ny + A.by - 1) / A.by;
    const int nbz = (A.nz + A.bz - 1) / A.bz;
    A.a = a;
    A.b = b;
    A.scale = scale;
    A.inv_dt = 1.0 / rg.dt;
    const long blocks = (long)A.nbx * A.nby * nbz;
    if (blocks <= 0 || blocks > 0x7fffffffL) return hipErrorInvalidValue;
    PCR_DISPATCH_R(compute, R,
        k_backproject_columns<R><<<(unsigned)blocks, 256, 0, s>>>(A, (const R*)resid, (const R*)p,
                                                                (const R*)y, (R*)out));
    return hipGetLastError();
}

hipError_t launch_contract(pcr_dtype compute, pcr_dtype storage, pcr_dtype f0_dtype,
                           const pcr_grid& g, int K, const void* f0, const void* mean,
                           const void* U, const double* w_eff, const void* gv, double* partials,
                           hipStream_t s)
{
    auto w = wvec(w_eff, K);
    PCR_DISPATCH_R(compute, R, PCR_DISPATCH_S(storage, S, PCR_DISPATCH_S(f0_dtype, F,
        k_contract<R, S, F><<<contract_grid(g), dim3(64, 4), 0, s>>>((const F*)f0, (const S*)mean,
                                                                (const S*)U, K, w, vox(g),
                                                                (const R*)gv, partials))));
    return hipGetLastError();
}

hipError_t launch_warp_adjoint(pcr_dtype compute, const pcr_grid& g, const void* dvf,
                               const void* gv, void* out, hipStream_t s)
{
    PCR_DISPATCH_R(compute, R,
        k_warp_adjoint<R><<<vox_grid(g), dim3(64, 4), 0, s>>>((const R*)dvf, (const R*)gv, vox(g),
                                                              (R*)out));
    return hipGetLastError();
}

hipError_t launch_support(pcr_dtype f0_dtype, const pcr_grid& g, const void* f0, int* sl,
                          hipStream_t s)
{
    const long nxy = (long)g.n[0] * g.n[1];
    const unsigned bx = (unsigned)std::min<long>((nxy + 2047) / 2048, 32);
    const unsigned bz = (unsigned)std::min(g.n[2], 65535);
    PCR_DISPATCH_S(f0_dtype, F,
        k_support<F><<<dim3(bx, bz), 256, 0, s>>>((const F*)f0, g.n[0], g.n[1], g.n[2], sl));
    return hipGetLastError();
}

hipError_t launch_absmax_rows(pcr_dtype dt, const void* a, size_t n, int rows, float* out,
                              hipStream_t s)
{
    const unsigned bx = (unsigned)std::min<size_t>((n + 1023) / 1024, 256);
    PCR_DISPATCH_S(dt, S,
        k_absmax_rows<S><<<dim3(bx, (unsigned)rows), 256, 0, s>>>((const S*)a, n, out));
    return hipGetLastError();
}

hipError_t launch_localize(pcr_dtype storage, const pcr_grid& g, int K, const void* mean,
                           const void* U, const double* w_eff, const double* p_ref, double tol,
                           int max_iter, double* out, hipStream_t s)
{
    auto w = wvec(w_eff, K);
    PCR_DISPATCH_S(storage, S,
        k_localize<S><<<1, 64, 0, s>>>((const S*)mean, (const S*)U, K, w, vox(g), p_ref[0],
                                       p_ref[1], p_ref[2], g.origin_mm[0], g.origin_mm[1],
                                       g.origin_mm[2], tol, max_iter, out));
    return hipGetLastError();
}

}  // namespace pcr
