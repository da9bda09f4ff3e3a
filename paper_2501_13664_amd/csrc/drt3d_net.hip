// Algorithm 2's merged output: the 12 dodecants' N x N x (3N-2) outputs
// rotated by the OutOrder rows and placed at the DodecantCoords blocks of a
// 4N x 4N x (3N-2) net, the 4 unused corner blocks zero. A gather, one thread
// per net element with the displacement fastest, so reads and writes are both
// unit-stride runs; HBM-bound.

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

template <typename T>
__global__ void __launch_bounds__(256)
merge_net_kernel(const T* __restrict__ R, T* __restrict__ net, int N)
{
    const long long P = 3LL * N - 2;
    const long long total = 16LL * N * N * P;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < total; i += (long long)gridDim.x * 256) {
        const long long dd = i % P;
        const long long q = i / P;
        const int col = (int)(q % (4 * N));
        const int row = (int)(q / (4 * N));
        const int k = kBlockDodecant[row / N][col / N];
        T v = T(0);
        if (k >= 0) {
            const int o0 = kOutOrder[k][0], o1 = kOutOrder[k][1];
            // cell (b0, b1) of the permuted block before its flips
            const int b0 = o0 < 0 ? N - 1 - row % N : row % N;
            const int b1 = o1 < 0 ? N - 1 - col % N : col % N;
            const bool swap = (o0 < 0 ? -o0 : o0) == 2;
            const int s1 = swap ? b1 : b0, s2 = swap ? b0 : b1;
            v = R[(((long long)k * N + s1) * N + s2) * P + dd];
        }
        net[i] = v;
    }
}

}  // namespace

hipError_t launch_merge_net(int is_float, const void* R, void* net, int N, hipStream_t s)
{
    const long long total = 16LL * N * N * (3LL * N - 2);
    const unsigned grid = (unsigned)std::max(1LL, std::min((total + 255) / 256, 1LL << 20));
    if (is_float)
        hipLaunchKernelGGL(merge_net_kernel<float>, dim3(grid), dim3(256), 0, s, (const float*)R, (float*)net, N);
    else
        hipLaunchKernelGGL(merge_net_kernel<uint32_t>, dim3(grid), dim3(256), 0, s, (const uint32_t*)R,
                           (uint32_t*)net, N);
    return hipGetLastError();
}

}  // namespace drt3d
