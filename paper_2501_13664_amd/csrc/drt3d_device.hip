// Device code of the drt3d library for gfx950 (CDNA4, wave64).
//
// DRT passes (forward eq. (11), adjoint eq. (17)). The stage map of eq. (11)
// shifts along the displacement axis only, and its x-part (slope s1, block
// bit v1) and y-part (s2, v2) add independent shifts, so a dodecant's n
// stages factor into n x-stages followed by n y-stages (the 2D transform
// applied twice, Sec. 6.3). A pass runs K consecutive stages of one axis on a
// group of 2^K columns that only exchange data among themselves: the columns
// sharing the low m0 slope bits and the block bits above m0+K. The group's
// columns (a displacement tile of them plus the halo the K shifts reach) sit
// in LDS; every stage is an in-place butterfly over column pairs, one
// wavefront per pair, lanes along the displacement, so every LDS access of a
// wave is 64 consecutive words and every shift is wave-uniform.
//
// In-place slot order: before local stage j, LDS slot p holds, in bits
// [0, j), the slope bits already produced (newest in bit j-1) and, in bits
// [j, K), the remaining block index. The pair (p, p | 2^j) are the two block
// halves of one slope; their two results (new slope bit 0 and 1) overwrite the
// same two slots. After K stages slot p holds the slope bitreverse_K(p).
//
// DJT stages (eq. (15)): each work item merges the block pair (2v, 2v+1) of
// one slope pair and writes the four children (new slope bits a, b) of a band
// of rows; lanes run along the contiguous displacement e2.

#include "drt3d_internal.h"

namespace drt3d {

__device__ __forceinline__ int bitrev(int x, int bits)
{
    return bits ? (int)(__brev((unsigned)x) >> (32 - bits)) : 0;
}

template <typename T>
__device__ __forceinline__ T zero_of() { return T(0); }

// Offset of column c (along the pass axis) crossed with column c_other.
__device__ __forceinline__ long long col_offset(int axis, int c, int c_other, int n, int P)
{
    long long idx = axis == 0 ? (((long long)c << n) + c_other) : (((long long)c_other << n) + c);
    return idx * P;
}

__device__ __forceinline__ int find_desc_drt(const DrtDesc* __restrict__ descs, int ndesc, long long wg)
{
    int lo = 0, hi = ndesc - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (descs[mid].wg_begin <= wg) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <typename T>
__global__ void __launch_bounds__(512)
drt_pass_kernel(const DrtDesc* __restrict__ descs, int ndesc, long long total_wg)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* lds = reinterpret_cast<T*>(smem_raw);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;

    for (long long wg = blockIdx.x; wg < total_wg; wg += gridDim.x) {
        const DrtDesc* d = descs + find_desc_drt(descs, ndesc, wg);
        const int ntiles = d->ntiles, groups = d->groups;
        long long local = wg - d->wg_begin;
        const int tile = (int)(local % ntiles);
        local /= ntiles;
        const int g = (int)(local % groups);
        const int slot = (int)(local / groups);

        const int n = d->n, N = d->N, K = d->K, m0 = d->m0, axis = d->axis;
        const int L = d->L, Lp = d->Lp, TT = d->T, H = d->H;
        const int c_other = g & (N - 1);
        const int gg = g >> n;
        const int sigma0 = gg & ((1 << m0) - 1);
        const int vhi_off = (gg >> m0) << (m0 + K);
        const int nslot = 1 << K;
        const int adjoint = d->adjoint;
        const int d0 = tile * TT;
        // displacement index of LDS position 0
        const int dd0 = adjoint ? d0 : d0 - H;

        // ---------------- load ----------------
        for (int p = wave; p < nslot; p += nwaves) {
            T* s = lds + (long long)p * Lp;
            int col;
            if (!adjoint) col = sigma0 + (p << m0) + vhi_off;           // slot p = block w
            else col = bitrev(p, K) + (sigma0 << K) + vhi_off;          // slot p = slope bitrev(p)
            if (d->src_mode == 0) {
                const T* src = reinterpret_cast<const T*>(d->src) + d->phys[slot] * d->src_slot_stride +
                               col_offset(axis, col, c_other, n, d->P_in);
                const int E = d->E_in;
#pragma unroll 4
                for (int l = lane; l < L; l += 64) {
                    const int dd = dd0 + l;
                    s[l] = (dd >= 0 && dd < E) ? src[dd] : zero_of<T>();
                }
            } else {
                // first forward pass (x axis, m0 = 0): x' = col, y' = c_other
                const FrameMap f = d->fm[slot];
                const T* v = reinterpret_cast<const T*>(d->vsrc[f.group]);
                const long long base = (long long)f.base + (long long)f.sx * col + (long long)f.sy * c_other;
#pragma unroll 4
                for (int l = lane; l < L; l += 64) {
                    const int dd = dd0 + l;
                    s[l] = (dd >= 0 && dd < N) ? v[base + (long long)f.sd * dd] : zero_of<T>();
                }
            }
        }
        __syncthreads();

        // ---------------- stages ----------------
        const int npairs = nslot >> 1;
        if (!adjoint) {
            for (int j = 0; j < K; ++j) {
                const int h = 1 << j;
                const int sig_hi = sigma0 << j;
                for (int q = wave; q < npairs; q += nwaves) {
                    const int p0 = ((q >> j) << (j + 1)) | (q & (h - 1));
                    const int sig = bitrev(p0 & (h - 1), j) + sig_hi;
                    T* s0 = lds + (long long)p0 * Lp;
                    T* s1 = s0 + (long long)h * Lp;
                    // descending chunks: reads at l - sig - 1 .. l never meet
                    // positions this wave has already overwritten
                    for (int base = ((L - 1) >> 6) << 6; base >= 0; base -= 64) {
                        const int l = base + lane;
                        if (l < L) {
                            const T a = s0[l];
                            const int i0 = l - sig;
                            const T b0 = i0 >= 0 ? s1[i0] : zero_of<T>();
                            const T b1 = i0 >= 1 ? s1[i0 - 1] : zero_of<T>();
                            s0[l] = a + b0;
                            s1[l] = a + b1;
                        }
                    }
                }
                __syncthreads();
            }
        } else {
            for (int j = K - 1; j >= 0; --j) {
                const int h = 1 << j;
                const int sig_hi = sigma0 << j;
                for (int q = wave; q < npairs; q += nwaves) {
                    const int p0 = ((q >> j) << (j + 1)) | (q & (h - 1));
                    const int sig = bitrev(p0 & (h - 1), j) + sig_hi;
                    T* s0 = lds + (long long)p0 * Lp;
                    T* s1 = s0 + (long long)h * Lp;
                    // ascending chunks: reads at l .. l + sig + 1 never meet
                    // positions this wave has already overwritten
                    for (int base = 0; base < L; base += 64) {
                        const int l = base + lane;
                        if (l < L) {
                            const T a0 = s0[l];
                            const T a1 = s1[l];
                            const int i0 = l + sig;
                            const T c0 = i0 < L ? s0[i0] : zero_of<T>();
                            const T c1 = i0 + 1 < L ? s1[i0 + 1] : zero_of<T>();
                            s0[l] = a0 + a1;
                            s1[l] = c0 + c1;
                        }
                    }
                }
                __syncthreads();
            }
        }

        // ---------------- store ----------------
        const int qmax = min(TT, d->E_out - d0);
        const int lofs = adjoint ? 0 : H;
        for (int p = wave; p < nslot; p += nwaves) {
            const T* s = lds + (long long)p * Lp + lofs;
            int col;
            if (!adjoint) col = bitrev(p, K) + (sigma0 << K) + vhi_off;
            else col = sigma0 + (p << m0) + vhi_off;
            if (d->dst_mode == 0) {
                T* dst = reinterpret_cast<T*>(d->dst) + d->phys[slot] * d->dst_slot_stride +
                         col_offset(axis, col, c_other, n, d->P_out) + d0;
#pragma unroll 4
                for (int q = lane; q < qmax; q += 64) dst[q] = s[q];
            } else {
                // last adjoint pass (x axis, m0 = 0): x' = col, y' = c_other
                const FrameMap f = d->fm[slot];
                T* v = reinterpret_cast<T*>(d->vdst[f.group]);
                const long long base = (long long)f.base + (long long)f.sx * col + (long long)f.sy * c_other;
                if (d->accum[slot]) {
#pragma unroll 4
                    for (int q = lane; q < qmax; q += 64) {
                        const long long o = base + (long long)f.sd * (d0 + q);
                        v[o] = v[o] + s[q];
                    }
                } else {
#pragma unroll 4
                    for (int q = lane; q < qmax; q += 64) v[base + (long long)f.sd * (d0 + q)] = s[q];
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// out[b][c][r] (+)= in[b][r][c]; 64 x 64 tiles through LDS, 256 threads.
template <typename T>
__global__ void __launch_bounds__(256)
transpose_kernel(const T* __restrict__ in, T* __restrict__ out, int R, int C, int add)
{
    __shared__ T tile[64][65];
    const long long b = blockIdx.z;
    const long long plane = (long long)R * C;
    const T* src = in + b * plane;
    T* dst = out + b * plane;
    const int c0 = blockIdx.x * 64, r0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int r = r0 + ty + 4 * i, c = c0 + tx;
        if (r < R && c < C) tile[ty + 4 * i][tx] = src[(long long)r * C + c];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int c = c0 + ty + 4 * i, r = r0 + tx;
        if (r < R && c < C) {
            const long long o = (long long)c * R + r;
            const T v = tile[tx][ty + 4 * i];
            dst[o] = add ? dst[o] + v : v;
        }
    }
}

// ---------------------------------------------------------------------------
__device__ __forceinline__ int find_desc_djt(const DjtDesc* __restrict__ descs, int ndesc, long long wg)
{
    int lo = 0, hi = ndesc - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (descs[mid].wg_begin <= wg) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <typename T>
__global__ void __launch_bounds__(256)
djt_stage_kernel(const DjtDesc* __restrict__ descs, int ndesc, long long total_wg)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
    for (long long wg = blockIdx.x; wg < total_wg; wg += gridDim.x) {
        const DjtDesc* d = descs + find_desc_djt(descs, ndesc, wg);
        long long local = wg - d->wg_begin;
        const int band = (int)(local % d->nbands);
        local /= d->nbands;
        const int grp = (int)(local % d->groups);
        const int slot = (int)(local / d->groups);

        const int n = d->n, N = d->N, m = d->m;
        const int Vn = N >> (m + 1);            // blocks after the stage
        const int vp = grp % Vn;                // merged block index v'
        const int sl = grp / Vn;                // sigma1 * 2^m + sigma2
        const int sig1 = sl >> m, sig2 = sl & ((1 << m) - 1);
        const int Ein = d->E_in, Eout = d->E_out;
        const long long pin = (long long)Ein * Ein, pout = (long long)Eout * Eout;
        const int Vm = N >> m;
        const long long in0 = ((long long)sl * Vm + 2 * vp) * pin;
        const long long in1 = in0 + pin;
        const T* src = reinterpret_cast<const T*>(d->src) + (d->src_mode ? 0 : slot * d->src_slot_stride);
        T* dst = reinterpret_cast<T*>(d->dst) + slot * d->dst_slot_stride;
        // children (a, b): slope pair (a + 2 sigma1, b + 2 sigma2) at stage m+1
        const int h2 = 2 << m;
        long long outp[4];
#pragma unroll
        for (int ab = 0; ab < 4; ++ab) {
            const int a = ab >> 1, b = ab & 1;
            outp[ab] = ((long long)((a + 2 * sig1) * h2 + (b + 2 * sig2)) * Vn + vp) * pout;
        }
        const FrameMap f = d->fm[slot];
        const int r_begin = band * d->rows_per_band;
        const int r_end = min(Eout, r_begin + d->rows_per_band);
        for (int e1 = r_begin + wave; e1 < r_end; e1 += nwaves) {
            for (int e2 = lane; e2 < Eout; e2 += 64) {
                T x0, y[4];
                const int r0 = e1 - sig1, c0 = e2 - sig2;
                if (d->src_mode == 0) {
                    x0 = (e1 < Ein && e2 < Ein) ? src[in0 + (long long)e1 * Ein + e2] : zero_of<T>();
#pragma unroll
                    for (int ab = 0; ab < 4; ++ab) {
                        const int r = r0 - (ab >> 1), c = c0 - (ab & 1);
                        y[ab] = (r >= 0 && c >= 0 && r < Ein && c < Ein) ? src[in1 + (long long)r * Ein + c]
                                                                       : zero_of<T>();
                    }
                } else {
                    // stage 0 from the volume: block v = z'; plane position (e1, e2)
                    const long long zb = (long long)f.sd * (2 * vp);
                    x0 = (e1 < N && e2 < N) ? src[f.base + (long long)f.sx * e1 + (long long)f.sy * e2 + zb]
                                            : zero_of<T>();
#pragma unroll
                    for (int ab = 0; ab < 4; ++ab) {
                        const int r = r0 - (ab >> 1), c = c0 - (ab & 1);
                        y[ab] = (r >= 0 && c >= 0 && r < N && c < N)
                                    ? src[f.base + (long long)f.sx * r + (long long)f.sy * c + zb + f.sd]
                                    : zero_of<T>();
                    }
                }
                const long long o = (long long)e1 * Eout + e2;
                if (d->final_stage) {
#pragma unroll
                    for (int ab = 0; ab < 4; ++ab) __builtin_nontemporal_store(x0 + y[ab], dst + outp[ab] + o);
                } else {
#pragma unroll
                    for (int ab = 0; ab < 4; ++ab) dst[outp[ab] + o] = x0 + y[ab];
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
hipError_t set_drt_lds_limit(int is_float, size_t bytes)
{
    if (is_float)
        return hipFuncSetAttribute(reinterpret_cast<const void*>(&drt_pass_kernel<float>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&drt_pass_kernel<uint32_t>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
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

hipError_t launch_djt_stage(int is_float, const DjtDesc* d_descs, int ndesc, long long total_wg,
                            int block, int grid, hipStream_t s)
{
    if (is_float)
        hipLaunchKernelGGL(djt_stage_kernel<float>, dim3(grid), dim3(block), 0, s, d_descs, ndesc, total_wg);
    else
        hipLaunchKernelGGL(djt_stage_kernel<uint32_t>, dim3(grid), dim3(block), 0, s, d_descs, ndesc, total_wg);
    return hipGetLastError();
}

hipError_t launch_transpose(int is_float, const void* in, void* out, int R, int C, int batches, int add,
                            hipStream_t s)
{
    dim3 grid((C + 63) / 64, (R + 63) / 64, batches);
    if (is_float)
        hipLaunchKernelGGL(transpose_kernel<float>, grid, dim3(256), 0, s, reinterpret_cast<const float*>(in),
                           reinterpret_cast<float*>(out), R, C, add);
    else
        hipLaunchKernelGGL(transpose_kernel<uint32_t>, grid, dim3(256), 0, s,
                           reinterpret_cast<const uint32_t*>(in), reinterpret_cast<uint32_t*>(out), R, C, add);
    return hipGetLastError();
}

}  // namespace drt3d
