// Device code of the drt3d library for gfx950 (CDNA4, wave64).
//
// DRT passes (forward eq. (11), adjoint eq. (17)). The stage map of eq. (11)
// shifts along the displacement axis only, and its x-part (slope s1, block
// bit v1) and y-part (s2, v2) add independent shifts, so the x- and y-stages
// of a dodecant commute and can be grouped freely (the 2D transform applied
// twice, Sec. 6.3). A pass runs the x-stages mx0..mx0+Kx-1 and the y-stages
// my0..my0+Ky-1 on a group of 2^Kx x 2^Ky columns that exchange data only
// among themselves (those sharing the low slope bits sx0, sy0 and the block
// bits above each range). The group's columns, over one displacement tile plus
// a halo, sit in LDS; every stage is an in-place butterfly over a column pair,
// one wavefront per pair, lanes along the displacement: every LDS access of a
// wave is 64 consecutive words and every shift is wave-uniform.
//
// Slot order: LDS slot p = px + (py << Kx). Before an x-stage j, bits [0, j)
// of px hold the slope bits already produced (newest in bit j-1) and bits
// [j, Kx) the remaining block index; the pair (p, p + 2^j) are the two block
// halves of one slope and their two results (new slope bit 0, 1) overwrite the
// same two slots. After the pass slot p holds slope (bitrev(px), bitrev(py)).
//
// Skewed origins. At x-stage j the shift of a pair is its slope
// t + sx0 * 2^j plus the new bit; sx0 is common to the group. Column w of the
// group is loaded with its displacement origin lowered by sx0*w + sy0*w_y, so
// the common part of every shift is absorbed by the origins (the pair's
// origins differ by exactly sx0 * 2^j) and LDS only sees the local shift
// t + bit <= 2^j; after the last stage all slots share one origin. The halo of
// a tile is therefore (2^Kx - 1) + (2^Ky - 1) whatever stages the pass covers.
// The adjoint runs the same butterflies transposed and in reverse order; its
// outputs inherit the skew instead of its inputs.
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

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
template <typename T> struct Vec4;
template <> struct Vec4<uint32_t> { using type = u32x4; };
template <> struct Vec4<float> { using type = f32x4; };

__device__ __forceinline__ int find_desc_drt(const DrtDesc* __restrict__ descs, int ndesc, long long wg)
{
    int lo = 0, hi = ndesc - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (descs[mid].wg_begin <= wg) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// LDS layout of a work item: [pad zeros][slot 0: L][pad zeros][slot 1: L] ...
// [slot n-1: L][pad zeros], L a multiple of 64, slot pitch Lp = L + pad. Reads
// that leave a slot by up to `pad` positions (below in the forward, above in
// the adjoint) hit zeros, so the stage loops carry no bounds checks; the pad
// covers the largest shift of the pass.
__device__ __forceinline__ int slot_offset(int p, int Lp, int pad) { return pad + p * Lp; }

// Forward radix-2 step (one stage of one axis) on the pair (s0, s1) with
// local shift t: s0[l] += s1[l-t], s1[l] = s0_old[l] + s1[l-t-1]. In place,
// 64-position chunks from the top down: a chunk reads only at or below its
// own positions, and writes after all of its reads.
template <typename T>
__device__ __forceinline__ void step2_fwd(T* s0, T* s1, int nch, int t, int lane)
{
    for (int c = nch - 1; c >= 0; --c) {
        const int l = 64 * c + lane;
        const T a = s0[l], b0 = s1[l - t], b1 = s1[l - t - 1];
        s0[l] = a + b0;
        s1[l] = a + b1;
    }
}

// Forward radix-4 step: x-stage and y-stage of the same index fused, which is
// the four-term stage map of eq. (11) itself. Slot s_ab receives the slope
// whose new x bit is a and new y bit is b.
template <typename T>
__device__ __forceinline__ void step4_fwd(T* s00, T* s10, T* s01, T* s11, int nch, int tx, int ty, int lane)
{
    const int txy = tx + ty;
    for (int c = nch - 1; c >= 0; --c) {
        const int l = 64 * c + lane;
        const T f00 = s00[l];
        const T f10a = s10[l - tx], f10b = s10[l - tx - 1];
        const T f01a = s01[l - ty], f01b = s01[l - ty - 1];
        const T f11a = s11[l - txy], f11b = s11[l - txy - 1], f11c = s11[l - txy - 2];
        const T x0 = f00 + f10a, x1 = f00 + f10b;
        s00[l] = x0 + (f01a + f11a);
        s10[l] = x1 + (f01a + f11b);
        s01[l] = x0 + (f01b + f11b);
        s11[l] = x1 + (f01b + f11c);
    }
}

// Adjoint radix-2 step (transpose of step2_fwd), chunks from the bottom up.
template <typename T>
__device__ __forceinline__ void step2_adj(T* s0, T* s1, int nch, int t, int lane)
{
    for (int c = 0; c < nch; ++c) {
        const int l = 64 * c + lane;
        const T a0 = s0[l], a1 = s1[l], c0 = s0[l + t], c1 = s1[l + t + 1];
        s0[l] = a0 + a1;
        s1[l] = c0 + c1;
    }
}

// Adjoint radix-4 step (transpose of step4_fwd).
template <typename T>
__device__ __forceinline__ void step4_adj(T* s00, T* s10, T* s01, T* s11, int nch, int tx, int ty, int lane)
{
    const int txy = tx + ty;
    for (int c = 0; c < nch; ++c) {
        const int l = 64 * c + lane;
        const T c00 = (s00[l] + s10[l]) + (s01[l] + s11[l]);
        const T c10 = (s00[l + tx] + s10[l + tx + 1]) + (s01[l + tx] + s11[l + tx + 1]);
        const T c01 = (s00[l + ty] + s10[l + ty]) + (s01[l + ty + 1] + s11[l + ty + 1]);
        const T c11 = (s00[l + txy] + s10[l + txy + 1]) + (s01[l + txy + 1] + s11[l + txy + 2]);
        s00[l] = c00;
        s10[l] = c10;
        s01[l] = c01;
        s11[l] = c11;
    }
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
        const int ntiles = d->ntiles;
        const int groups = d->groups_x * d->groups_y;
        long long local = wg - d->wg_begin;
        const int tile = (int)(local % ntiles);
        local /= ntiles;
        const int g = (int)(local % groups);
        const int slot = (int)(local / groups);

        const int N = d->N, n = d->n;
        const int Kx = d->Kx, Ky = d->Ky, mx0 = d->mx0, my0 = d->my0;
        const int L = d->L, Lp = d->Lp, TT = d->T, H = d->H;
        const int pad = Lp - L;
        const int nch = L >> 6;
        const int adjoint = d->adjoint;
        const int gy = g & (d->groups_y - 1), gx = g >> (n - Ky);
        const int sx0 = gx & ((1 << mx0) - 1);
        const int vhx = (gx >> mx0) << (mx0 + Kx);
        const int sy0 = gy & ((1 << my0) - 1);
        const int vhy = (gy >> my0) << (my0 + Ky);
        const int nslot = 1 << (Kx + Ky);
        const int xmask = (1 << Kx) - 1;
        const int d0 = tile * TT;
        // adjoint outputs are skewed by up to smax: tiles past it hold nothing
        if (adjoint && d0 >= d->E_out + sx0 * xmask + sy0 * ((1 << Ky) - 1)) continue;

        // zero pads (their positions depend on L, which varies across descriptors)
        for (int i = threadIdx.x; i < (nslot + 1) * pad; i += blockDim.x) {
            const int p = i / pad, o = i - p * pad;
            lds[p * Lp + o] = zero_of<T>();
        }

        // ---------------- load ----------------
        // slot p holds the column of block (px, py) (forward, skewed origin)
        // or of slope (bitrev px, bitrev py) (adjoint, common origin).
        const T* srcbase = d->src_mode == 0 ? reinterpret_cast<const T*>(d->src) + d->phys[slot] * d->src_slot_stride
                                            : reinterpret_cast<const T*>(d->vsrc[d->fm[slot].group]);
        const int Ein = d->src_mode == 0 ? d->E_in : N;
        {
            constexpr int G = 2, CB = 8;
            for (int p0 = wave; p0 < nslot; p0 += G * nwaves) {
                const T* col[G];
                int sdv[G], dd0v[G];
                bool live[G];
#pragma unroll
                for (int gq = 0; gq < G; ++gq) {
                    const int p = p0 + gq * nwaves;
                    live[gq] = p < nslot;
                    const int px = p & xmask, py = p >> Kx;
                    int c1, c2;
                    if (!adjoint) {
                        c1 = sx0 + (px << mx0) + vhx;
                        c2 = sy0 + (py << my0) + vhy;
                        dd0v[gq] = d0 - H - sx0 * px - sy0 * py;
                    } else {
                        c1 = bitrev(px, Kx) + (sx0 << Kx) + vhx;
                        c2 = bitrev(py, Ky) + (sy0 << Ky) + vhy;
                        dd0v[gq] = d0;
                    }
                    if (d->src_mode == 0) {
                        col[gq] = srcbase + (((long long)c1 << n) + c2) * d->P_in;
                        sdv[gq] = 1;
                    } else {
                        const FrameMap f = d->fm[slot];
                        col[gq] = srcbase + ((long long)f.base + (long long)f.sx * c1 + (long long)f.sy * c2);
                        sdv[gq] = f.sd;
                    }
                }
                for (int cb = 0; cb < nch; cb += CB) {
                    T v[G][CB];
#pragma unroll
                    for (int gq = 0; gq < G; ++gq)
#pragma unroll
                        for (int c = 0; c < CB; ++c) {
                            const int l = 64 * (cb + c) + lane;
                            const int dd = dd0v[gq] + l;
                            v[gq][c] = (live[gq] && cb + c < nch && dd >= 0 && dd < Ein) ? col[gq][sdv[gq] * dd]
                                                                                       : zero_of<T>();
                        }
#pragma unroll
                    for (int gq = 0; gq < G; ++gq) {
                        T* s = lds + slot_offset(p0 + gq * nwaves, Lp, pad);
#pragma unroll
                        for (int c = 0; c < CB; ++c)
                            if (live[gq] && cb + c < nch) s[64 * (cb + c) + lane] = v[gq][c];
                    }
                }
            }
        }
        __syncthreads();

        // ---------------- stages ----------------
        // x-stage j and y-stage j run together as one radix-4 step while both
        // axes have them; the rest run as radix-2 steps. Each axis keeps its
        // stage order, which is all the in-place slot convention needs.
        const int kmax = Kx > Ky ? Kx : Ky;
        for (int jj = 0; jj < kmax; ++jj) {
            const int j = adjoint ? kmax - 1 - jj : jj;
            const bool hx = j < Kx, hy = j < Ky;
            const int bx = 1 << j, by = 1 << (Kx + j);
            if (hx && hy) {
                const int nq = nslot >> 2;
                for (int q = wave; q < nq; q += nwaves) {
                    // insert zero bits at positions j (x) and Kx + j (y)
                    int p = q;
                    p = ((p >> j) << (j + 1)) | (p & (bx - 1));
                    p = ((p >> (Kx + j)) << (Kx + j + 1)) | (p & (by - 1));
                    const int tx = bitrev(p & (bx - 1), j);
                    const int ty = bitrev((p >> Kx) & (bx - 1), j);
                    T* s00 = lds + slot_offset(p, Lp, pad);
                    T* s10 = lds + slot_offset(p + bx, Lp, pad);
                    T* s01 = lds + slot_offset(p + by, Lp, pad);
                    T* s11 = lds + slot_offset(p + bx + by, Lp, pad);
                    if (!adjoint) step4_fwd(s00, s10, s01, s11, nch, tx, ty, lane);
                    else step4_adj(s00, s10, s01, s11, nch, tx, ty, lane);
                }
            } else {
                const int bit = hx ? j : Kx + j;
                const int h = 1 << bit;
                const int np = nslot >> 1;
                for (int q = wave; q < np; q += nwaves) {
                    const int p = ((q >> bit) << (bit + 1)) | (q & (h - 1));
                    const int axis_bits = hx ? (p & xmask) : (p >> Kx);
                    const int t = bitrev(axis_bits & ((1 << j) - 1), j);
                    T* s0 = lds + slot_offset(p, Lp, pad);
                    if (!adjoint) step2_fwd(s0, s0 + h * Lp, nch, t, lane);
                    else step2_adj(s0, s0 + h * Lp, nch, t, lane);
                }
            }
            __syncthreads();
        }

        // ---------------- store ----------------
        {
            const int q0 = adjoint ? 0 : H;
            const int Eout = d->dst_mode == 0 ? d->E_out : N;
            T* dstbase = d->dst_mode == 0 ? reinterpret_cast<T*>(d->dst) + d->phys[slot] * d->dst_slot_stride
                                          : reinterpret_cast<T*>(d->vdst[d->fm[slot].group]);
            const int accum = d->dst_mode == 1 && d->accum[slot];
            const int nt = d->nt_store;
            for (int p = wave; p < nslot; p += nwaves) {
                const int px = p & xmask, py = p >> Kx;
                int c1, c2, dd0;
                if (!adjoint) {  // common origin: positions H.. hold dd = d0..
                    c1 = bitrev(px, Kx) + (sx0 << Kx) + vhx;
                    c2 = bitrev(py, Ky) + (sy0 << Ky) + vhy;
                    dd0 = d0;
                } else {         // child column (px, py) at its skewed origin
                    c1 = sx0 + (px << mx0) + vhx;
                    c2 = sy0 + (py << my0) + vhy;
                    dd0 = d0 - sx0 * px - sy0 * py;
                }
                T* col;
                int sd;
                if (d->dst_mode == 0) {
                    col = dstbase + (((long long)c1 << n) + c2) * d->P_out;
                    sd = 1;
                } else {
                    const FrameMap f = d->fm[slot];
                    col = dstbase + ((long long)f.base + (long long)f.sx * c1 + (long long)f.sy * c2);
                    sd = f.sd;
                }
                const T* s = lds + slot_offset(p, Lp, pad) + q0;
                const int qlo = max(0, -dd0), qhi = min(TT, Eout - dd0);
                for (int q = qlo + lane; q < qhi; q += 64) {
                    T* dst = col + sd * (dd0 + q);
                    T v = s[q];
                    if (accum) v += *dst;
                    if (nt) __builtin_nontemporal_store(v, dst);
                    else *dst = v;
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
