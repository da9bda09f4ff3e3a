// Host-side launchers of the drt3d kernels, and the kernels that need no
// shape specialisation (the generic DRT pass, the transposes).

#include "drt3d_kernels.h"

namespace drt3d {

// ---------------------------------------------------------------------------
// Shape-specialised kernels live in their own translation units.
static const void* fast_kernel(int is_float, int kx, int ky, int nch, int mode, int waves, int sb = 4, int db = 4)
{
    if (nch < 1 || nch > 6) return nullptr;
    if (sb != 4 || db != 4) {
        if (is_float || waves != 8) return nullptr;
        if (kx == 3 && ky == 3) return drt_fast_kernel_narrow_3_3(nch, mode, sb, db);
        if (kx == 2 && ky == 2) return drt_fast_kernel_narrow_2_2(nch, mode, sb, db);
        if (kx == 3 && ky == 2) return drt_fast_kernel_narrow_3_2(nch, mode, sb, db);
        if (kx == 2 && ky == 3) return drt_fast_kernel_narrow_2_3(nch, mode, sb, db);
        return nullptr;
    }
    if (kx == 3 && ky == 3) return drt_fast_kernel_3_3(is_float, nch, mode, waves);
    if (kx == 2 && ky == 2) return drt_fast_kernel_2_2(is_float, nch, mode, waves);
    if (kx == 3 && ky == 2) return drt_fast_kernel_3_2(is_float, nch, mode, waves);
    if (kx == 2 && ky == 3) return drt_fast_kernel_2_3(is_float, nch, mode, waves);
    return nullptr;
}

hipError_t set_drt_lds_limit(int is_float, size_t bytes)
{
    for (int K = 1; K <= 3; ++K)
        for (int ncc : kDjtChunkCounts)
            for (int nco = ncc > 1 ? ncc - 1 : 1; nco <= ncc; ++nco) {
                hipError_t e = hipFuncSetAttribute(djt_pass_kernel_ptr(is_float, K, ncc, nco),
                                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
                if (e != hipSuccess) return e;
            }
    const int shapes[4][2] = {{3, 3}, {2, 2}, {3, 2}, {2, 3}};
    for (auto& sh : shapes)
        for (int nc = 1; nc <= 6; ++nc)
            for (int mode = 0; mode < 3; ++mode)
                for (int waves : {8, 16}) {
                    const void* k = fast_kernel(is_float, sh[0], sh[1], nc, mode, waves);
                    if (!k) continue;
                    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
                    if (e != hipSuccess) return e;
                }
    for (int K = 2; K <= 3; ++K)
        for (int nc = 1; nc <= 6; ++nc)
            for (int waves : {8, 16}) {
                const void* k = drt_adj_group_kernel(is_float, K, nc, waves);
                if (!k) continue;
                hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
                if (e != hipSuccess) return e;
            }
    const int narrow[4][3] = {{0, 1, 2}, {0, 2, 4}, {1, 2, 4}, {1, 1, 4}};  // (mode, sb, db)
    if (!is_float)
        for (auto& sh : shapes)
            for (int nc = 1; nc <= 6; ++nc)
                for (auto& m : narrow) {
                    const void* k = fast_kernel(0, sh[0], sh[1], nc, m[0], 8, m[1], m[2]);
                    if (!k) continue;
                    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
                    if (e != hipSuccess) return e;
                }
    if (is_float)
        return hipFuncSetAttribute(reinterpret_cast<const void*>(&drt_pass_kernel<float>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&drt_pass_kernel<uint32_t>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

int drt_fast_available(int kx, int ky, int nch, int waves, int mode, int sb, int db)
{
    return fast_kernel(0, kx, ky, nch, mode, waves, sb, db) != nullptr;
}

hipError_t launch_drt_fast(int is_float, int kx, int ky, int nch, int mode, int waves, const DrtDesc* d_descs,
                           int ndesc, long long total_wg, int grid, size_t lds_bytes, hipStream_t s, int sb, int db)
{
    const void* k = fast_kernel(is_float, kx, ky, nch, mode, waves, sb, db);
    if (!k) return hipErrorInvalidValue;
    void* args[] = {&d_descs, &ndesc, &total_wg};
    return hipLaunchKernel(k, dim3(grid), dim3(64 * waves), args, lds_bytes, s);
}

hipError_t launch_drt_pass(int is_float, const DrtDesc* d_descs, int ndesc, long long total_wg,
                           int block, int grid, size_t lds_bytes, hipStream_t s)
{
    if (is_float)
        hipLaunchKernelGGL(drt_pass_kernel<float>, dim3(grid), dim3(block), lds_bytes, s, d_descs, ndesc,
                           total_wg);
    else
        hipLaunchKernelGGL(drt_pass_kernel<uint32_t>, dim3(grid), dim3(block), lds_bytes, s, d_descs, ndesc,
                           total_wg);
    return hipGetLastError();
}

hipError_t launch_djt_pass(int is_float, int K, int ncc, int nco, const DjtDesc* d_descs, int ndesc,
                           long long total_wg, int grid, size_t lds_bytes, hipStream_t s)
{
    const void* k = djt_pass_kernel_ptr(is_float, K, ncc, nco);
    if (!k) return hipErrorInvalidValue;
    void* args[] = {&d_descs, &ndesc, &total_wg};
    return hipLaunchKernel(k, dim3(grid), dim3(512), args, lds_bytes, s);
}

const void* drt_adj_group_kernel(int is_float, int K, int nch, int waves)
{
    if (K == 3) return drt_adj_group_kernel_3_3(is_float, nch, waves);
    if (K == 2) return drt_adj_group_kernel_2_2(is_float, nch, waves);
    return nullptr;
}

hipError_t launch_drt_adj_group(int is_float, int K, int nch, int waves, const DrtDesc* d_descs, int ndesc,
                                long long total_wg, int grid, size_t lds_bytes, hipStream_t s)
{
    const void* k = drt_adj_group_kernel(is_float, K, nch, waves);
    if (!k) return hipErrorInvalidValue;
    void* args[] = {&d_descs, &ndesc, &total_wg};
    return hipLaunchKernel(k, dim3(grid), dim3(64 * waves), args, lds_bytes, s);
}

hipError_t launch_transpose_u8(const TransDesc* d_descs, int ndesc, long long total_wg, hipStream_t s)
{
    if (total_wg <= 0) return hipSuccess;
    if (total_wg > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(transpose_kernel<uint8_t>, dim3((unsigned)total_wg), dim3(256), 0, s, d_descs, ndesc);
    return hipGetLastError();
}

hipError_t launch_transpose(int is_float, const TransDesc* d_descs, int ndesc, long long total_wg,
                            hipStream_t s)
{
    if (total_wg <= 0) return hipSuccess;
    if (total_wg > 0x7fffffffLL) return hipErrorInvalidValue;
    if (is_float)
        hipLaunchKernelGGL(transpose_kernel<float>, dim3((unsigned)total_wg), dim3(256), 0, s, d_descs, ndesc);
    else
        hipLaunchKernelGGL(transpose_kernel<uint32_t>, dim3((unsigned)total_wg), dim3(256), 0, s, d_descs, ndesc);
    return hipGetLastError();
}

}  // namespace drt3d
