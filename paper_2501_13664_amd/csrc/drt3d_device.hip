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

// out[b][c][r] = in[b][r][c] for bytes, 128 x 128 tiles moved as 4-byte
// words: R, C and both bases are multiples of 4 (checked by the planner), so a
// word of 4 bytes of one row is in range whole or not at all. Each thread
// loads a 4 x 4 block (one word from each of four rows), transposes it in
// registers, and puts the four words into LDS under an XOR swizzle that keeps
// both the scattered writes and the row-wise reads free of bank conflicts.
static __global__ void __launch_bounds__(256)
transpose_u8_wide_kernel(const TransDesc* __restrict__ descs, int ndesc)
{
    // word w of tile row q (input column c0 + q, input rows r0 + 4w ... 4w + 3)
    // sits at q * 32 + (w ^ (q >> 2))
    __shared__ uint32_t tile[128 * 32];
    const long long wg = blockIdx.x;
    int lo = 0, hi = ndesc - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (descs[mid].wg_begin <= wg) lo = mid; else hi = mid - 1;
    }
    const TransDesc& d = descs[lo];
    long long local = wg - d.wg_begin;
    const int tc = (int)(local % d.tiles_c);
    local /= d.tiles_c;
    const int tr = (int)(local % d.tiles_r);
    const long long b = local / d.tiles_r;
    const int R = d.R, C = d.C;
    const long long plane = (long long)R * C;
    const uint8_t* src = reinterpret_cast<const uint8_t*>(d.in) + b * plane;
    uint8_t* dst = reinterpret_cast<uint8_t*>(d.out) + b * plane;
    const int c0 = tc * 128, r0 = tr * 128;
    const int lw = threadIdx.x & 31, grp = threadIdx.x >> 5;  // word in a row, row group
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int br = grp + 8 * i;  // rows r0 + 4 br ... + 3
        const int c = c0 + 4 * lw;
        uint32_t w[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = r0 + 4 * br + j;
            w[j] = (r < R && c < C) ? *reinterpret_cast<const uint32_t*>(src + (long long)r * C + c) : 0u;
        }
        // byte k of the four row words -> word k, rows in byte order
        const uint32_t lo01 = __builtin_amdgcn_perm(w[1], w[0], 0x05010400u);  // w0b0 w1b0 w0b1 w1b1
        const uint32_t hi01 = __builtin_amdgcn_perm(w[1], w[0], 0x07030602u);  // w0b2 w1b2 w0b3 w1b3
        const uint32_t lo23 = __builtin_amdgcn_perm(w[3], w[2], 0x05010400u);
        const uint32_t hi23 = __builtin_amdgcn_perm(w[3], w[2], 0x07030602u);
        const uint32_t o[4] = {
            __builtin_amdgcn_perm(lo23, lo01, 0x05040100u),  // byte 0 of rows 0..3
            __builtin_amdgcn_perm(lo23, lo01, 0x07060302u),  // byte 1
            __builtin_amdgcn_perm(hi23, hi01, 0x05040100u),  // byte 2
            __builtin_amdgcn_perm(hi23, hi01, 0x07060302u),  // byte 3
        };
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int q = 4 * lw + k;  // q >> 2 == lw
            tile[q * 32 + (br ^ lw)] = o[k];
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int q = grp + 8 * i;
        const int c = c0 + q, r = r0 + 4 * lw;
        if (c < C && r < R)
            *reinterpret_cast<uint32_t*>(dst + (long long)c * R + r) = tile[q * 32 + (lw ^ (q >> 2))];
    }
}

hipError_t launch_transpose_u8(const TransDesc* d_descs, int ndesc, long long total_wg, int wide, hipStream_t s)
{
    if (total_wg <= 0) return hipSuccess;
    if (total_wg > 0x7fffffffLL) return hipErrorInvalidValue;
    if (wide)
        hipLaunchKernelGGL(transpose_u8_wide_kernel, dim3((unsigned)total_wg), dim3(256), 0, s, d_descs, ndesc);
    else
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
