// Algorithm 2's merged output: the 12 dodecants' N x N x (3N-2) outputs
// rotated by the OutOrder rows and placed at the DodecantCoords blocks of a
// 4N x 4N x (3N-2) net, the 4 unused corner blocks zero. A gather by whole
// displacement columns, so reads and writes are unit-stride runs; HBM-bound.

#include <hip/hip_runtime.h>

#include <algorithm>

#include "drt3d_internal.h"

namespace drt3d {

namespace {

// Algorithm 2's OutOrder (1-based axes (s1, s2, d); a negative entry flips
// that axis of the permuted block) and DodecantCoords, as printed
__constant__ int kOutOrder[12][2] = {
    {-2, -1}, {-1, 2}, {2, 1}, {1, -2}, {2, 1}, {1, -2},
    {-1, 2}, {-2, -1}, {2, 1}, {-1, 2}, {1, -2}, {-2, -1},
};
// block (row, column) of the net -> dodecant, -1 for the empty corners
__constant__ int kBlockDodecant[4][4] = {
    {-1, 5, 4, -1},
    {9, 0, 1, 11},
    {8, 3, 2, 10},
    {-1, 7, 6, -1},
};

// One wavefront per net column (row, col): the column's source is one
// contiguous (s1, s2) column of a dodecant (or zeros), so each wavefront
// streams 3N-2 elements in 64-lane runs; the index arithmetic is per column.
template <typename T>
__global__ void __launch_bounds__(256)
merge_net_kernel(const T* __restrict__ R, T* __restrict__ net, int N)
{
    const int P = 3 * N - 2;
    const long long ncols = 16LL * N * N;
    const int lane = threadIdx.x & 63;
    const long long waves = (long long)gridDim.x * 4;
    for (long long q = (long long)blockIdx.x * 4 + (threadIdx.x >> 6); q < ncols; q += waves) {
        const int col = (int)(q % (4 * N));
        const int row = (int)(q / (4 * N));
        const int k = kBlockDodecant[row / N][col / N];
        T* dst = net + q * P;
        if (k < 0) {
            for (int dd = lane; dd < P; dd += 64) dst[dd] = T(0);
            continue;
        }
        const int o0 = kOutOrder[k][0], o1 = kOutOrder[k][1];
        // cell (b0, b1) of the permuted block before its flips
        const int b0 = o0 < 0 ? N - 1 - row % N : row % N;
        const int b1 = o1 < 0 ? N - 1 - col % N : col % N;
        const bool swap = (o0 < 0 ? -o0 : o0) == 2;
        const int s1 = swap ? b1 : b0, s2 = swap ? b0 : b1;
        const T* src = R + (((long long)k * N + s1) * N + s2) * P;
        for (int dd = lane; dd < P; dd += 64) dst[dd] = src[dd];
    }
}

}  // namespace

hipError_t launch_merge_net(int is_float, const void* R, void* net, int N, hipStream_t s)
{
    const long long ncols = 16LL * N * N;  // four columns per 256-thread block
    const unsigned grid = (unsigned)std::max(1LL, std::min((ncols + 3) / 4, 1LL << 20));
    if (is_float)
        hipLaunchKernelGGL(merge_net_kernel<float>, dim3(grid), dim3(256), 0, s, (const float*)R, (float*)net, N);
    else
        hipLaunchKernelGGL(merge_net_kernel<uint32_t>, dim3(grid), dim3(256), 0, s, (const uint32_t*)R,
                           (uint32_t*)net, N);
    return hipGetLastError();
}

}  // namespace drt3d
