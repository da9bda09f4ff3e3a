// Kernels of the iterative inverse DRT (Sec. 5.2): the 3x3x3 high-pass
// filter, the Radon-domain restriction S, the image-domain prolongation P,
// and the small vector operations of iterative improvement. All float32; all
// bound by HBM bandwidth (a few bytes moved per flop).

#include <hip/hip_runtime.h>

#include <algorithm>

#include "drt3d_internal.h"

namespace drt3d {

namespace {

constexpr int kBlock = 256;

inline unsigned grid_for_elems(long long n)
{
    return (unsigned)std::max(1LL, std::min((n + kBlock - 1) / kBlock, 1LL << 20));
}

// half-sample symmetric reflection of an index into [0, N)
__device__ __forceinline__ int reflect(int i, int N)
{
    return i < 0 ? -1 - i : (i >= N ? 2 * N - 1 - i : i);
}

// out[v] = (accumulate ? out[v] : 0) + c * sum_o h[o] y[v + o]: the filter of
// Sec. 5.2, centre 7/8, faces -1/16, edges -1/32, corners -1/64, i.e.
// delta - g x g x g with g = (1/4, 1/2, 1/4), applied as y - (g x g x g) y.
// Borders reflect (x[-1] = x[0]), so constants filter to zero everywhere.
__global__ void __launch_bounds__(kBlock)
hp_filter_kernel(const float* __restrict__ y, float* __restrict__ out, int N, float c, int accumulate)
{
    const long long n = (long long)N * N * N;
    for (long long v = (long long)blockIdx.x * kBlock + threadIdx.x; v < n; v += (long long)gridDim.x * kBlock) {
        const int z = (int)(v % N);
        const int yy = (int)((v / N) % N);
        const int x = (int)(v / ((long long)N * N));
        const float g[3] = {0.25f, 0.5f, 0.25f};
        float blur = 0.f;
        for (int i = 0; i < 3; ++i) {
            const long long xi = (long long)reflect(x + i - 1, N) * N * N;
            float row = 0.f;
            for (int j = 0; j < 3; ++j) {
                const float* p = y + xi + (long long)reflect(yy + j - 1, N) * N;
                const float t = 0.25f * p[reflect(z - 1, N)] + 0.5f * p[z] + 0.25f * p[reflect(z + 1, N)];
                row += g[j] * t;
            }
            blur += g[i] * row;
        }
        const float hv = y[v] - blur;
        out[v] = (accumulate ? out[v] : 0.f) + c * hv;
    }
}

// r[i] = b[i] - ax[i]
__global__ void __launch_bounds__(kBlock)
residual_kernel(const float* __restrict__ b, const float* ax, float* r, long long n)
{
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock)
        r[i] = b[i] - ax[i];
}

// S of Sec. 5.2 per dodecant, in the stored displacement dd = N-1-d:
// Rc[k][s1][s2][dd] = (R[k][2 s1][2 s2][2 dd] + R[k][2 s1][2 s2][2 dd + 1]) / 8
__global__ void __launch_bounds__(kBlock)
restrict_kernel(const float* __restrict__ R, float* __restrict__ Rc, int N)
{
    const int Nc = N / 2;
    const int E = 3 * N - 2, Ec = 3 * Nc - 2;
    const long long n = 12LL * Nc * Nc * Ec;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock) {
        const int dd = (int)(i % Ec);
        long long q = i / Ec;
        const int s2 = (int)(q % Nc);
        q /= Nc;
        const int s1 = (int)(q % Nc);
        const int k = (int)(q / Nc);
        const float* col = R + (((long long)k * N + 2 * s1) * N + 2 * s2) * E;
        Rc[i] = (col[2 * dd] + col[2 * dd + 1]) * 0.125f;
    }
}

// P of Sec. 5.2 added in: x[v] += e[v / 2] (nearest neighbour, 2x per axis)
__global__ void __launch_bounds__(kBlock)
prolong_add_kernel(const float* __restrict__ e, float* __restrict__ x, int N)
{
    const int Nc = N / 2;
    const long long n = (long long)N * N * N;
    for (long long v = (long long)blockIdx.x * kBlock + threadIdx.x; v < n; v += (long long)gridDim.x * kBlock) {
        const int z = (int)(v % N);
        const int y = (int)((v / N) % N);
        const int xx = (int)(v / ((long long)N * N));
        x[v] += e[((long long)(xx >> 1) * Nc + (y >> 1)) * Nc + (z >> 1)];
    }
}

// size 1: the least-squares solution of twelve copies of one unknown
__global__ void base_mean_kernel(const float* __restrict__ b12, float* __restrict__ x1)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        float s = 0.f;
        for (int k = 0; k < 12; ++k) s += b12[k];
        x1[0] = s / 12.f;
    }
}

__global__ void __launch_bounds__(kBlock) fill_kernel(float* __restrict__ p, float v, long long n)
{
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock)
        p[i] = v;
}

// v[x][y][z] = ((73 x + 151 y + 277 z) mod 29) - 14: the power iteration's start
__global__ void __launch_bounds__(kBlock) power_start_kernel(float* __restrict__ v, int N)
{
    const long long n = (long long)N * N * N;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock) {
        const long long z = i % N, y = (i / N) % N, x = i / ((long long)N * N);
        v[i] = (float)((73 * x + 151 * y + 277 * z) % 29 - 14);
    }
}

// partial[b] = sum of squares over block b's grid-stride share, in double
__global__ void __launch_bounds__(kBlock)
sumsq_partial_kernel(const float* __restrict__ w, long long n, double* __restrict__ partial)
{
    __shared__ double red[kBlock];
    double s = 0.0;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock)
        s += (double)w[i] * (double)w[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = kBlock / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// norm[0] = sqrt(sum of the partials)
__global__ void __launch_bounds__(kBlock)
norm_finish_kernel(const double* __restrict__ partial, int np, double* __restrict__ norm)
{
    __shared__ double red[kBlock];
    double s = 0.0;
    for (int i = threadIdx.x; i < np; i += kBlock) s += partial[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = kBlock / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) norm[0] = sqrt(red[0]);
}

// v[i] = w[i] / norm[0]
__global__ void __launch_bounds__(kBlock)
scale_by_inverse_norm_kernel(const float* __restrict__ w, const double* __restrict__ norm, float* __restrict__ v,
                             long long n)
{
    const float s = (float)(1.0 / norm[0]);
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock)
        v[i] = w[i] * s;
}

}  // namespace

constexpr int kNormParts = 1024;

hipError_t launch_hp_filter(const float* y, float* out, int N, float c, int accumulate, hipStream_t s)
{
    const long long n = (long long)N * N * N;
    hipLaunchKernelGGL(hp_filter_kernel, dim3(grid_for_elems(n)), dim3(kBlock), 0, s, y, out, N, c, accumulate);
    return hipGetLastError();
}

hipError_t launch_residual(const float* b, const float* ax, float* r, long long n, hipStream_t s)
{
    hipLaunchKernelGGL(residual_kernel, dim3(grid_for_elems(n)), dim3(kBlock), 0, s, b, ax, r, n);
    return hipGetLastError();
}

hipError_t launch_restrict(const float* R, float* Rc, int N, hipStream_t s)
{
    const long long n = 12LL * (N / 2) * (N / 2) * (3 * (N / 2) - 2);
    hipLaunchKernelGGL(restrict_kernel, dim3(grid_for_elems(n)), dim3(kBlock), 0, s, R, Rc, N);
    return hipGetLastError();
}

hipError_t launch_prolong_add(const float* e, float* x, int N, hipStream_t s)
{
    const long long n = (long long)N * N * N;
    hipLaunchKernelGGL(prolong_add_kernel, dim3(grid_for_elems(n)), dim3(kBlock), 0, s, e, x, N);
    return hipGetLastError();
}

hipError_t launch_base_mean(const float* b12, float* x1, hipStream_t s)
{
    hipLaunchKernelGGL(base_mean_kernel, dim3(1), dim3(64), 0, s, b12, x1);
    return hipGetLastError();
}

hipError_t launch_fill(float* p, float v, long long n, hipStream_t s)
{
    hipLaunchKernelGGL(fill_kernel, dim3(grid_for_elems(n)), dim3(kBlock), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_power_start(float* v, int N, hipStream_t s)
{
    const long long n = (long long)N * N * N;
    hipLaunchKernelGGL(power_start_kernel, dim3(grid_for_elems(n)), dim3(kBlock), 0, s, v, N);
    return hipGetLastError();
}

size_t norm_scratch_bytes() { return (kNormParts + 1) * sizeof(double); }

// norm[kNormParts] (inside `scratch`) = |w|, then v = w / |w|
hipError_t launch_normalize(const float* w, float* v, long long n, double* scratch, hipStream_t s)
{
    const int np = (int)std::min<long long>(kNormParts, (n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(sumsq_partial_kernel, dim3(np), dim3(kBlock), 0, s, w, n, scratch);
    hipLaunchKernelGGL(norm_finish_kernel, dim3(1), dim3(kBlock), 0, s, scratch, np, scratch + kNormParts);
    hipLaunchKernelGGL(scale_by_inverse_norm_kernel, dim3(grid_for_elems(n)), dim3(kBlock), 0, s, w,
                       scratch + kNormParts, v, n);
    return hipGetLastError();
}

}  // namespace drt3d
