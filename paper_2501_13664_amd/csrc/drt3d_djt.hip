// DJT pass kernels: one per (dtype, stages fused K, LDS row chunks).

#include <algorithm>

#include "drt3d_kernels.h"

namespace drt3d {

template <typename T, int K, int NCC>
static const void* djt_kernel_c(int nco)
{
    if (nco == NCC) return reinterpret_cast<const void*>(&djt_pass_kernel<T, K, NCC, NCC>);
    if (NCC > 1 && nco == NCC - 1) return reinterpret_cast<const void*>(&djt_pass_kernel<T, K, NCC, (NCC > 1 ? NCC - 1 : 1)>);
    return nullptr;
}

template <typename T, int K>
static const void* djt_kernel_k(int ncc, int nco)
{
    switch (ncc) {
    case 1: return djt_kernel_c<T, K, 1>(nco);
    case 2: return djt_kernel_c<T, K, 2>(nco);
    case 3: return djt_kernel_c<T, K, 3>(nco);
    case 5: return djt_kernel_c<T, K, 5>(nco);
    case 9: return djt_kernel_c<T, K, 9>(nco);
    default: return nullptr;
    }
}

template <typename T>
static const void* djt_kernel(int K, int ncc, int nco)
{
    switch (K) {
    case 1: return djt_kernel_k<T, 1>(ncc, nco);
    case 2: return djt_kernel_k<T, 2>(ncc, nco);
    case 3: return djt_kernel_k<T, 3>(ncc, nco);
    default: return nullptr;
    }
}

const void* djt_pass_kernel_ptr(int is_float, int K, int ncc, int nco)
{
    return is_float ? djt_kernel<float>(K, ncc, nco) : djt_kernel<uint32_t>(K, ncc, nco);
}

template <typename T, int K>
static const void* djt_adj_kernel_k(int ncc)
{
    switch (ncc) {
    case 1: return reinterpret_cast<const void*>(&djt_adj_kernel<T, K, 1>);
    case 2: return reinterpret_cast<const void*>(&djt_adj_kernel<T, K, 2>);
    case 3: return reinterpret_cast<const void*>(&djt_adj_kernel<T, K, 3>);
    case 4: return reinterpret_cast<const void*>(&djt_adj_kernel<T, K, 4>);
    case 5: return reinterpret_cast<const void*>(&djt_adj_kernel<T, K, 5>);
    case 8: return reinterpret_cast<const void*>(&djt_adj_kernel<T, K, 8>);
    default: return nullptr;
    }
}

template <typename T>
static const void* djt_adj_kernel_t(int K, int ncc)
{
    switch (K) {
    case 1: return djt_adj_kernel_k<T, 1>(ncc);
    case 2: return djt_adj_kernel_k<T, 2>(ncc);
    case 3: return djt_adj_kernel_k<T, 3>(ncc);
    default: return nullptr;
    }
}

const void* djt_adj_kernel_ptr(int is_float, int K, int ncc)
{
    return is_float ? djt_adj_kernel_t<float>(K, ncc) : djt_adj_kernel_t<uint32_t>(K, ncc);
}

hipError_t launch_djt_adj(int is_float, int K, int ncc, const DjtDesc* d_descs, int ndesc, long long total_wg,
                          int grid, size_t lds_bytes, hipStream_t s)
{
    const void* k = djt_adj_kernel_ptr(is_float, K, ncc);
    if (!k) return hipErrorInvalidValue;
    (void)lds_bytes;  // the ring is static LDS
    void* args[] = {&d_descs, &ndesc, &total_wg};
    return hipLaunchKernel(k, dim3(grid), dim3(512), args, 0, s);
}

hipError_t launch_sum_parts(int is_float, const void* parts, int nparts, void* out, long long n, int accum,
                            hipStream_t s)
{
    const long long blocks = std::min<long long>((n + 255) / 256, 65536);
    if (is_float)
        hipLaunchKernelGGL(sum_parts_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                           reinterpret_cast<const float*>(parts), nparts, reinterpret_cast<float*>(out), n, accum);
    else
        hipLaunchKernelGGL(sum_parts_kernel<uint32_t>, dim3((unsigned)blocks), dim3(256), 0, s,
                           reinterpret_cast<const uint32_t*>(parts), nparts, reinterpret_cast<uint32_t*>(out), n,
                           accum);
    return hipGetLastError();
}

int djt_tile_rows(int K) { return djt_rows_per_tile(K); }
int djt_adj_tile_rows() { return kDjtAdjRows; }
// static LDS of the adjoint kernel for (K, ncc): its three-window ring
template <int K>
static int djt_adj_ring_elems(int ncc)
{
    switch (ncc) {
    case 1: return 3 * djt_adj_window<K, 1>();
    case 2: return 3 * djt_adj_window<K, 2>();
    case 3: return 3 * djt_adj_window<K, 3>();
    case 4: return 3 * djt_adj_window<K, 4>();
    case 5: return 3 * djt_adj_window<K, 5>();
    case 8: return 3 * djt_adj_window<K, 8>();
    default: return 0;
    }
}

size_t djt_adj_lds_bytes(int K, int ncc)
{
    const int e = K == 1 ? djt_adj_ring_elems<1>(ncc) : K == 2 ? djt_adj_ring_elems<2>(ncc)
                : K == 3 ? djt_adj_ring_elems<3>(ncc) : 0;
    return (size_t)e * 4;
}

int djt_chunks_for(int cols)
{
    for (int ncc : kDjtChunkCounts)
        if (64 * ncc >= cols) return ncc;
    return 0;
}

int djt_adj_chunks_for(int cols)
{
    for (int ncc : kDjtAdjChunkCounts)
        if (64 * ncc >= cols) return ncc;
    return 0;
}

}  // namespace drt3d
