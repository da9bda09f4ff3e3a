// DJT pass kernels: one per (dtype, stages fused K, LDS row chunks).

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

int djt_tile_rows(int K) { return djt_rows_per_tile(K); }

int djt_chunks_for(int cols)
{
    for (int ncc : kDjtChunkCounts)
        if (64 * ncc >= cols) return ncc;
    return 0;
}

}  // namespace drt3d
