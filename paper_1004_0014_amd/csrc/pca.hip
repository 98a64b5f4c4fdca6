// PCA training of the motion model on the GPU (section 2.1, eq. (1); section
// 3: PCA over the N-1 DVFs between the reference phase and the other
// phases).  For J training DVFs d_j [3][N]:
//   mean  = (1/J) sum_j d_j
//   U     = the K leading left singular vectors of the centred 3N x J matrix
//           [d_1 - mean, ..., d_J - mean], unit norm, each flipped so that its
//           largest-magnitude entry (the first within 1e-5 of it) is positive
//   w_train[j][k] = <U_k, d_j - mean>.
// One streaming pass forms the raw Gram matrix G_ij = <d_i, d_j> in FP64; the
// centred Gram follows exactly in J x J algebra; a cyclic Jacobi eigen-solve
// on the host gives V and the singular values; a second streaming pass writes
// the mean and U_k = sum_j V_jk (d_j - mean) / sigma_k.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "host.h"

using namespace pcr;

namespace {

constexpr int kMaxJ = 16;
constexpr int kMaxPairs = kMaxJ * (kMaxJ + 1) / 2;

// Raw Gram matrix of the J fields (upper triangle, FP64 per-block partials).
template <int J>
__global__ void __launch_bounds__(256) k_gram(const float* __restrict__ d, size_t E,
                                              double* __restrict__ partials)
{
    constexpr int P = J * (J + 1) / 2;
    double acc[P];
#pragma unroll
    for (int p = 0; p < P; ++p) acc[p] = 0.0;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < E; e += (size_t)gridDim.x * 256) {
        double v[J];
#pragma unroll
        for (int j = 0; j < J; ++j) v[j] = (double)d[(size_t)j * E + e];
        int p = 0;
#pragma unroll
        for (int i = 0; i < J; ++i)
#pragma unroll
            for (int j = i; j < J; ++j) acc[p++] += v[i] * v[j];
    }
    __shared__ double red[4][P];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        double s = acc[p];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
        if (lane == 0) red[wv][p] = s;
    }
    __syncthreads();
    for (int p = threadIdx.x; p < P; p += 256)
        partials[(size_t)blockIdx.x * P + p] = red[0][p] + red[1][p] + red[2][p] + red[3][p];
}

// G[p] = sum over blocks of partials[b][p]: one wave per entry, each lane
// summing every 64th block in order, then a fixed-shape wave sum
// (deterministic).
__global__ void __launch_bounds__(1024) k_sum_partials(const double* __restrict__ part, int nb,
                                                       int P, double* __restrict__ out)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int p = wv; p < P; p += 16) {
        double s = 0.0;
        for (int b = lane; b < nb; b += 64) s += part[(size_t)b * P + p];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
        if (lane == 0) out[p] = s;
    }
}

struct Coef {
    float v[kMaxJ * 8];   // V_jk / sigma_k
    float sign[8];
};

// mean and U_k = sign_k sum_j (V_jk / sigma_k) (d_j - mean).  J is a
// template parameter so that the J loads of an element are in flight together
// and stay in registers.
template <int J>
__global__ void __launch_bounds__(256) k_pca_fields(const float* __restrict__ d, size_t E, int K,
                                                    Coef c, float* __restrict__ mean,
                                                    float* __restrict__ U)
{
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < E; e += (size_t)gridDim.x * 256) {
        float v[J];
#pragma unroll
        for (int j = 0; j < J; ++j) v[j] = d[(size_t)j * E + e];
        float s = 0.f;
#pragma unroll
        for (int j = 0; j < J; ++j) s += v[j];
        const float m = s / (float)J;
        mean[e] = m;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (k < K) {
                float u = 0.f;
#pragma unroll
                for (int j = 0; j < J; ++j) u = fmaf(c.v[j * 8 + k], v[j] - m, u);
                U[(size_t)k * E + e] = c.sign[k] * u;
            }
        }
    }
}

// max |U_k| per field (bits of non-negative floats order like the floats):
// one pass over the K fields, block maximum in LDS, then one atomic per block
// and field
template <int K>
__global__ void __launch_bounds__(256) k_absmax(const float* __restrict__ U, size_t E,
                                                unsigned* __restrict__ out)
{
    __shared__ float red[4][K];
    float mx[K];
#pragma unroll
    for (int k = 0; k < K; ++k) mx[k] = 0.f;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < E; e += (size_t)gridDim.x * 256) {
        float v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = U[(size_t)k * E + e];
#pragma unroll
        for (int k = 0; k < K; ++k) mx[k] = fmaxf(mx[k], fabsf(v[k]));
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        float m = mx[k];
        for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_down(m, off, 64));
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][k] = m;
    }
    __syncthreads();
    if (threadIdx.x < K) {
        const int k = threadIdx.x;
        atomicMax(out + k, __float_as_uint(fmaxf(fmaxf(red[0][k], red[1][k]), fmaxf(red[2][k], red[3][k]))));
    }
}

template <int K>
hipError_t launch_absmax(const float* U, size_t E, unsigned* out, unsigned nb, hipStream_t s)
{
    k_absmax<K><<<nb, 256, 0, s>>>(U, E, out);
    return hipGetLastError();
}

// first index whose |U_k| reaches (1 - 1e-5) of the maximum (a tolerance
// well above FP32 rounding, so near-ties of symmetric fields resolve alike
// in FP32 and FP64): one pass over the K fields, each thread stopping once it
// has a hit in every field; block minimum in LDS, one atomic per block and
// field
template <int K>
__global__ void __launch_bounds__(256) k_first_max(const float* __restrict__ U, size_t E,
                                                   const unsigned* __restrict__ mx,
                                                   unsigned long long* __restrict__ first)
{
    __shared__ unsigned long long red[4][K];
    float thr[K];
    unsigned long long best[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        thr[k] = __uint_as_float(mx[k]) * (1.0f - 1e-5f);
        best[k] = ~0ull;
    }
    constexpr unsigned all = (1u << K) - 1u;
    unsigned found = 0u;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < E && found != all;
         e += (size_t)gridDim.x * 256) {
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (!(found & (1u << k)) && fabsf(U[(size_t)k * E + e]) >= thr[k]) {
                best[k] = e;
                found |= 1u << k;
            }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        unsigned long long b = best[k];
        for (int off = 32; off > 0; off >>= 1) {
            unsigned long long o = __shfl_down(b, off, 64);
            b = o < b ? o : b;
        }
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][k] = b;
    }
    __syncthreads();
    if (threadIdx.x < K) {
        const int k = threadIdx.x;
        unsigned long long b = red[0][k];
        for (int i = 1; i < 4; ++i) b = red[i][k] < b ? red[i][k] : b;
        if (b != ~0ull) atomicMin(first + k, b);
    }
}

template <int K>
hipError_t launch_first_max(const float* U, size_t E, const unsigned* mx, unsigned long long* first,
                            unsigned nb, hipStream_t s)
{
    k_first_max<K><<<nb, 256, 0, s>>>(U, E, mx, first);
    return hipGetLastError();
}

// clears the reduction targets of the sign rule
__global__ void k_sign_init(unsigned* __restrict__ mx, unsigned long long* __restrict__ first)
{
    if (threadIdx.x < 8) {
        mx[threadIdx.x] = 0u;
        first[threadIdx.x] = ~0ull;
    }
}

// val[k] = U_k at its sign-deciding index
__global__ void k_sign_pick(const float* __restrict__ U, size_t E, int K,
                            const unsigned long long* __restrict__ first, float* __restrict__ val)
{
    const int k = threadIdx.x;
    if (k < K) {
        const unsigned long long i = first[k];
        val[k] = i < E ? U[(size_t)k * E + i] : 0.f;
    }
}

__global__ void k_flip(float* __restrict__ U, size_t E, int k)
{
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < E; e += (size_t)gridDim.x * 256)
        U[(size_t)k * E + e] = -U[(size_t)k * E + e];
}

// Cyclic Jacobi eigen-decomposition of a symmetric n x n matrix (row-major):
// A is overwritten; on exit lam[i] = eigenvalues, V (row-major) the
// eigenvectors in columns.
void jacobi_eigen(std::vector<double>& A, int n, std::vector<double>& lam, std::vector<double>& V)
{
    V.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                tot += A[(size_t)i * n + j] * A[(size_t)i * n + j];
                if (i != j) off += A[(size_t)i * n + j] * A[(size_t)i * n + j];
            }
        if (off <= 1e-30 * tot) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                double apq = A[(size_t)p * n + q];
                if (apq == 0.0) continue;
                double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
                double theta = (aqq - app) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {   // A <- J^T A J, rows/cols p, q
                    double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
                    A[(size_t)k * n + p] = c * akp - s * akq;
                    A[(size_t)k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
                    A[(size_t)p * n + k] = c * apk - s * aqk;
                    A[(size_t)q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
                    V[(size_t)k * n + p] = c * vkp - s * vkq;
                    V[(size_t)k * n + q] = s * vkp + c * vkq;
                }
            }
    }
    lam.resize(n);
    for (int i = 0; i < n; ++i) lam[i] = A[(size_t)i * n + i];
}

template <int J>
hipError_t launch_gram(const float* d, size_t E, double* part, int nb, hipStream_t s)
{
    k_gram<J><<<nb, 256, 0, s>>>(d, E, part);
    return hipGetLastError();
}

template <int J>
hipError_t launch_fields(const float* d, size_t E, int K, const Coef& c, float* mean, float* U,
                         unsigned nb, hipStream_t s)
{
    k_pca_fields<J><<<nb, 256, 0, s>>>(d, E, K, c, mean, U);
    return hipGetLastError();
}

}  // namespace

extern "C" {

pcr_status pcr_pca_train(const pcr_grid* grid, int32_t J, const float* dvfs_dev, int32_t K,
                         float* mean_dev, float* U_dev, double* sing_host, double* w_train_host,
                         void* stream)
{
    PCR_TRY(check_grid(grid));
    if (J < 2 || J > kMaxJ) return fail(PCR_EINVAL, "J = %d must be in 2..%d", J, kMaxJ);
    if (K < 1 || K > 8 || K > J - 1) return fail(PCR_EINVAL, "K = %d must be in 1..min(8, J-1)", K);
    if (!dvfs_dev || !mean_dev || !U_dev) return fail(PCR_EINVAL, "NULL device pointer");
    hipStream_t s = (hipStream_t)stream;
    const size_t E = 3 * (size_t)grid->n[0] * grid->n[1] * grid->n[2];
    const int P = J * (J + 1) / 2;
    const int nb = 1024;
    DevBuf part, small;
    int dev;
    HIP_TRY(hipGetDevice(&dev));
    PCR_TRY(part.ensure((size_t)nb * kMaxPairs * sizeof(double), dev, s));
    PCR_TRY(small.ensure(4096, dev, s));
    double* Gd = (double*)small.p;
    unsigned* mx = (unsigned*)((char*)small.p + 2048);
    unsigned long long* first = (unsigned long long*)((char*)small.p + 3072);
    hipError_t e;
    {
        PROF(PCA_GRAM, s);
        switch (J) {
#define PCR_G(n) case n: e = launch_gram<n>(dvfs_dev, E, (double*)part.p, nb, s); break;
            PCR_G(2) PCR_G(3) PCR_G(4) PCR_G(5) PCR_G(6) PCR_G(7) PCR_G(8) PCR_G(9)
            PCR_G(10) PCR_G(11) PCR_G(12) PCR_G(13) PCR_G(14) PCR_G(15) PCR_G(16)
#undef PCR_G
        default: e = hipErrorInvalidValue;
        }
    }
    if (e != hipSuccess) { part.release(); small.release(); HIP_TRY(e); }
    k_sum_partials<<<1, 1024, 0, s>>>((const double*)part.p, nb, P, Gd);
    std::vector<double> Gu(P);
    e = hipMemcpyAsync(Gu.data(), Gd, P * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { part.release(); small.release(); HIP_TRY(e); }
    // centred Gram: Gc_ij = G_ij - (r_i + r_j)/J + T/J^2
    std::vector<double> G((size_t)J * J), r(J, 0.0);
    for (int i = 0, p = 0; i < J; ++i)
        for (int j = i; j < J; ++j, ++p) G[(size_t)i * J + j] = G[(size_t)j * J + i] = Gu[p];
    double T = 0.0;
    for (int i = 0; i < J; ++i) {
        for (int j = 0; j < J; ++j) r[i] += G[(size_t)i * J + j];
        T += r[i];
    }
    std::vector<double> Gc((size_t)J * J);
    for (int i = 0; i < J; ++i)
        for (int j = 0; j < J; ++j) Gc[(size_t)i * J + j] = G[(size_t)i * J + j] - (r[i] + r[j]) / J + T / ((double)J * J);
    std::vector<double> lam, V;
    jacobi_eigen(Gc, J, lam, V);
    std::vector<int> order(J);
    for (int i = 0; i < J; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int a, int b) { return lam[a] > lam[b]; });
    Coef c{};
    double sig[8];
    for (int k = 0; k < K; ++k) {
        sig[k] = std::sqrt(std::max(lam[order[k]], 0.0));
        if (!(sig[k] > 0.0)) { part.release(); small.release(); return fail(PCR_EINVAL, "training DVFs have rank < K"); }
        for (int j = 0; j < J; ++j) c.v[j * 8 + k] = (float)(V[(size_t)j * J + order[k]] / sig[k]);
        c.sign[k] = 1.f;
    }
    const unsigned gb = (unsigned)std::min<size_t>((E + 255) / 256, 4096);
    {
        PROF(PCA_FIELDS, s);
        switch (J) {
#define PCR_F(n) case n: e = launch_fields<n>(dvfs_dev, E, K, c, mean_dev, U_dev, gb, s); break;
            PCR_F(2) PCR_F(3) PCR_F(4) PCR_F(5) PCR_F(6) PCR_F(7) PCR_F(8) PCR_F(9)
            PCR_F(10) PCR_F(11) PCR_F(12) PCR_F(13) PCR_F(14) PCR_F(15) PCR_F(16)
#undef PCR_F
        default: e = hipErrorInvalidValue;
        }
    }
    if (e != hipSuccess) { part.release(); small.release(); HIP_TRY(e); }
    // sign rule: the first entry within 1e-5 of the largest magnitude is positive
    float* pick = (float*)((char*)small.p + 3584);
    const unsigned gr = std::min(gb, 1024u);
    k_sign_init<<<1, 64, 0, s>>>(mx, first);
    e = hipGetLastError();
    if (e == hipSuccess) {
        switch (K) {
#define PCR_A(n) case n: e = launch_absmax<n>(U_dev, E, mx, gr, s); break;
            PCR_A(1) PCR_A(2) PCR_A(3) PCR_A(4) PCR_A(5) PCR_A(6) PCR_A(7) PCR_A(8)
#undef PCR_A
        default: e = hipErrorInvalidValue;
        }
    }
    if (e == hipSuccess) {
        switch (K) {
#define PCR_M(n) case n: e = launch_first_max<n>(U_dev, E, mx, first, gr, s); break;
            PCR_M(1) PCR_M(2) PCR_M(3) PCR_M(4) PCR_M(5) PCR_M(6) PCR_M(7) PCR_M(8)
#undef PCR_M
        default: e = hipErrorInvalidValue;
        }
    }
    if (e == hipSuccess) { k_sign_pick<<<1, 64, 0, s>>>(U_dev, E, K, first, pick); e = hipGetLastError(); }
    float val[8] = {0.f};
    if (e == hipSuccess) e = hipMemcpyAsync(val, pick, K * sizeof(float), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    double sgn[8];
    for (int k = 0; k < K && e == hipSuccess; ++k) {
        sgn[k] = val[k] < 0.f ? -1.0 : 1.0;
        if (val[k] < 0.f) {
            k_flip<<<gb, 256, 0, s>>>(U_dev, E, k);
            e = hipGetLastError();
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    part.release();
    small.release();
    HIP_TRY(e);
    // w_train[j][k] = <U_k, d_j - mean> = sign_k sigma_k V_jk
    for (int k = 0; k < K; ++k) {
        if (sing_host) sing_host[k] = sig[k];
        if (w_train_host)
            for (int j = 0; j < J; ++j) w_train_host[j * K + k] = sgn[k] * sig[k] * V[(size_t)j * J + order[k]];
    }
    return PCR_OK;
}

}  // extern "C"
