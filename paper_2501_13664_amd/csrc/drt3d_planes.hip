// Plane detection in the DRT (the application of Sec. 6.1): the largest bin of
// the output is the dominant plane; the bins whose planes are orthogonal to it,
// that are relative maxima of their dodecant's output and that reach a
// threshold relative to the dominant bin are the other planes. Backprojecting
// the listed bins (the adjoint of a 0/1 projection) marks their voxels.
//
// Everything here is bound by HBM bandwidth or latency: the maximum reads the
// whole output once; the peak search reads only the columns whose planes are
// orthogonal to the dominant one (plus their neighbours, from cache).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "drt3d_internal.h"

namespace drt3d {

namespace {

constexpr int kBlock = 256;

template <typename T>
__device__ __forceinline__ T lowest_of();
template <>
__device__ __forceinline__ int lowest_of<int>() { return INT_MIN; }
template <>
__device__ __forceinline__ float lowest_of<float>() { return -INFINITY; }

// (v1, i1) ranks above (v2, i2): larger value, ties to the smaller index
template <typename T>
__device__ __forceinline__ bool better(T v1, long long i1, T v2, long long i2)
{
    return v1 > v2 || (v1 == v2 && i1 < i2);
}

template <typename T>
__device__ __forceinline__ void wave_best(T& v, long long& i)
{
    for (int off = 32; off > 0; off >>= 1) {
        const T ov = __shfl_xor(v, off);
        const long long oi = __shfl_xor(i, off);
        if (better(ov, oi, v, i)) { v = ov; i = oi; }
    }
}

// block-wide best of (v, i); the result is valid in thread 0
template <typename T>
__device__ __forceinline__ void block_best(T& v, long long& i)
{
    __shared__ T sv[kBlock / 64];
    __shared__ long long si[kBlock / 64];
    wave_best(v, i);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { sv[w] = v; si[w] = i; }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int q = 1; q < kBlock / 64; ++q)
            if (better(sv[q], si[q], v, i)) { v = sv[q]; i = si[q]; }
}

template <typename T>
__device__ __forceinline__ T from_bits32(uint32_t u);
template <>
__device__ __forceinline__ int from_bits32<int>(uint32_t u) { return (int)u; }
template <>
__device__ __forceinline__ float from_bits32<float>(uint32_t u) { return __uint_as_float(u); }

// per block: the best (value, index) of its grid-stride share of the n = 4 nq
// elements, read as 16-byte quads, four quads in flight per lane
template <typename T>
__global__ void __launch_bounds__(kBlock)
argmax_partial_kernel(const uint4* __restrict__ p4, long long nq, T* __restrict__ pv, long long* __restrict__ pi)
{
    const long long n = 4 * nq;
    T bv = lowest_of<T>();
    long long bi = n;  // "none": any element ranks above it
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long q0 = (long long)blockIdx.x * kBlock + threadIdx.x; q0 < nq; q0 += 4 * stride) {
        uint4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const long long q = q0 + u * stride;
            v[u] = q < nq ? p4[q] : make_uint4(0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const long long q = q0 + u * stride;
            if (q >= nq) continue;
            const uint32_t e[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const T x = from_bits32<T>(e[c]);
                if (better(x, 4 * q + c, bv, bi)) { bv = x; bi = 4 * q + c; }
            }
        }
    }
    block_best(bv, bi);
    if (threadIdx.x == 0) { pv[blockIdx.x] = bv; pi[blockIdx.x] = bi; }
}

// the best of the partials: top[0] = its index, thr[0] = rel * its value,
// bins[0] = its index
template <typename T>
__global__ void __launch_bounds__(kBlock)
argmax_final_kernel(const T* __restrict__ p, long long n, const T* __restrict__ pv, const long long* __restrict__ pi,
                    int nparts, double rel, long long* __restrict__ top, double* __restrict__ thr,
                    long long* __restrict__ bins)
{
    T bv = lowest_of<T>();
    long long bi = n;
    for (int q = threadIdx.x; q < nparts; q += kBlock)
        if (better(pv[q], pi[q], bv, bi)) { bv = pv[q]; bi = pi[q]; }
    block_best(bv, bi);
    if (threadIdx.x == 0) {
        const long long idx = bi < n ? bi : 0;  // no element ranked (all NaN): index 0
        top[0] = idx;
        thr[0] = rel * (double)p[idx];
        bins[0] = idx;
    }
}

// Integer normal (x, y, z) of dodecant k's planes at slopes (s1, s2), scaled by
// N-1: (-s1, -s2, N-1) in the primed frame, each original axis taking the
// primed component that runs along it, negated where that axis is mirrored.
__device__ __forceinline__ void plane_normal(const PlaneFrames& F, int k, int s1, int s2, int N, long long n[3])
{
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int a = F.axis[k][i];
        n[i] = F.sign[k][i] * (long long)(a == 0 ? -s1 : a == 1 ? -s2 : N - 1);
    }
}

// |cos| <= cos_tol between the two normals, as (a.b)^2 <= tol2 |a|^2 |b|^2
// with both integer products exact in float64
__device__ __forceinline__ bool orthogonal(const long long a[3], const long long b[3], double tol2)
{
    const long long dot = a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
    const long long na = a[0] * a[0] + a[1] * a[1] + a[2] * a[2];
    const long long nb = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
    return (double)(dot * dot) <= tol2 * (double)(na * nb);
}

// Relative maximum inside the dodecant: every existing neighbour (s1+a, s2+b,
// dd+c) that comes earlier in the layout is strictly below v, every later one
// is not above it.
template <typename T>
__device__ __forceinline__ bool local_max(const T* __restrict__ Rj, int N, int E, int s1, int s2, int dd, T v)
{
#pragma unroll
    for (int a = -1; a <= 1; ++a)
#pragma unroll
        for (int b = -1; b <= 1; ++b)
#pragma unroll
            for (int c = -1; c <= 1; ++c) {
                if (a == 0 && b == 0 && c == 0) continue;
                const int t1 = s1 + a, t2 = s2 + b, t3 = dd + c;
                if ((unsigned)t1 >= (unsigned)N || (unsigned)t2 >= (unsigned)N || (unsigned)t3 >= (unsigned)E) continue;
                const T w = Rj[((long long)t1 * N + t2) * E + t3];
                const bool later = a > 0 || (a == 0 && (b > 0 || (b == 0 && c > 0)));
                if (later ? w > v : w >= v) return false;
            }
    return true;
}

// Wavefronts stride over the output columns (j, s1, s2), lanes along dd.
// WRITE = 0: counts[column] = number of qualifying bins. WRITE = 1: their
// flat indices go to bins[1 + offsets[column] + rank] while that is below cap.
template <typename T, int WRITE>
__global__ void __launch_bounds__(kBlock)
plane_peaks_kernel(const T* __restrict__ p, int N, int nk, PlaneFrames F, const long long* __restrict__ top,
                   const double* __restrict__ thr, double tol2, int* __restrict__ counts,
                   const long long* __restrict__ offsets, long long* __restrict__ bins, long long cap)
{
    const int E = 3 * N - 2;
    const long long ncol = (long long)nk * N * N;
    const long long nwaves = (long long)gridDim.x * (kBlock / 64);
    const int lane = threadIdx.x & 63;
    long long nt[3] = {0, 0, 0};
    if (!WRITE) {
        const long long t = top[0];
        const long long per = (long long)N * N * E;
        const int tj = (int)(t / per);
        const long long tr = t - tj * per;
        plane_normal(F, F.ks[tj], (int)(tr / ((long long)N * E)), (int)((tr / E) % N), N, nt);
    }
    const double th = thr[0];
    for (long long col = (long long)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); col < ncol; col += nwaves) {
        if (WRITE && counts[col] == 0) continue;
        // N is a power of two: the column's (j, s1, s2) by shifts
        const int lg = 31 - __clz(N);
        const int j = (int)(col >> (2 * lg));
        const int s1 = (int)(col >> lg) & (N - 1), s2 = (int)col & (N - 1);
        if (!WRITE) {
            long long nc[3];
            plane_normal(F, F.ks[j], s1, s2, N, nc);
            if (!orthogonal(nt, nc, tol2)) {
                if (lane == 0) counts[col] = 0;
                continue;
            }
        }
        const T* Rj = p + (long long)j * N * N * E;
        const long long cbase = col * E;
        const long long off = WRITE ? offsets[col] : 0;
        int cnt = 0;
        // four 64-displacement chunks per round, their loads in flight together
        for (int d0 = 0; d0 < E; d0 += 256) {
            T v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int dd = d0 + 64 * u + lane;
                v[u] = dd < E ? p[cbase + dd] : lowest_of<T>();
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int dd = d0 + 64 * u + lane;
                const bool q = dd < E && (double)v[u] >= th && local_max(Rj, N, E, s1, s2, dd, v[u]);
                const unsigned long long m = __ballot(q);
                if (WRITE && q) {
                    const long long pos = 1 + off + cnt + __popcll(m & ((1ULL << lane) - 1));
                    if (pos < cap) bins[pos] = cbase + dd;
                }
                cnt += __popcll(m);
            }
        }
        if (!WRITE && lane == 0) counts[col] = cnt;
    }
}

// Exclusive prefix sums of counts[0, m) into offsets, in three phases over
// chunks of kScanChunk counts: the chunk sums, their scan (one work group,
// which also writes count[0] = 1 + the total: the dominant bin plus the
// qualifying ones), then each chunk's scan plus its offset.
constexpr int kScanPer = 16;
constexpr int kScanChunk = kBlock * kScanPer;

__device__ __forceinline__ long long block_inclusive_scan(long long x)
{
    __shared__ long long sh[kBlock];
    sh[threadIdx.x] = x;
    __syncthreads();
    for (int h = 1; h < kBlock; h <<= 1) {
        const long long add = (int)threadIdx.x >= h ? sh[threadIdx.x - h] : 0;
        __syncthreads();
        sh[threadIdx.x] += add;
        __syncthreads();
    }
    return sh[threadIdx.x];
}

__global__ void __launch_bounds__(kBlock)
scan_chunk_sums_kernel(const int* __restrict__ counts, long long m, long long* __restrict__ csum)
{
    const long long b = (long long)blockIdx.x * kScanChunk + (long long)threadIdx.x * kScanPer;
    long long s = 0;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i)
        if (b + i < m) s += counts[b + i];
    s = block_inclusive_scan(s);
    if (threadIdx.x == kBlock - 1) csum[blockIdx.x] = s;
}

// in place: csum[c] becomes the exclusive prefix of the chunk sums
__global__ void __launch_bounds__(kBlock)
scan_chunk_offsets_kernel(long long* __restrict__ csum, long long nc, long long* __restrict__ count)
{
    const long long per = (nc + kBlock - 1) / kBlock;
    const long long b0 = per * threadIdx.x;
    const long long b = b0 < nc ? b0 : nc, e = b + per < nc ? b + per : nc;
    long long s = 0;
    for (long long i = b; i < e; ++i) s += csum[i];
    const long long incl = block_inclusive_scan(s);
    long long run = incl - s;
    for (long long i = b; i < e; ++i) {
        const long long c = csum[i];
        csum[i] = run;
        run += c;
    }
    if (threadIdx.x == kBlock - 1) count[0] = 1 + incl;
}

__global__ void __launch_bounds__(kBlock)
scan_chunk_write_kernel(const int* __restrict__ counts, long long m, const long long* __restrict__ coff,
                        long long* __restrict__ offsets)
{
    const long long b = (long long)blockIdx.x * kScanChunk + (long long)threadIdx.x * kScanPer;
    int c[kScanPer];
    long long s = 0;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        c[i] = b + i < m ? counts[b + i] : 0;
        s += c[i];
    }
    long long run = coff[blockIdx.x] + block_inclusive_scan(s) - s;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        if (b + i < m) offsets[b + i] = run;
        run += c[i];
    }
}

// marker[bins[i]] = one for i < min(count[0], cap); indices outside [0, n)
// are skipped
__global__ void __launch_bounds__(kBlock)
scatter_ones_kernel(const long long* __restrict__ bins, const long long* __restrict__ count, long long cap,
                    uint32_t* __restrict__ marker, long long n, uint32_t one)
{
    const long long m = count[0] < cap ? count[0] : cap;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < m; i += (long long)gridDim.x * kBlock) {
        const long long b = bins[i];
        if (b >= 0 && b < n) marker[b] = one;
    }
}

}  // namespace

int argmax_parts(long long n)
{
    const long long nq = n / 4;
    return (int)std::max(1LL, std::min(2048LL, (nq + 4LL * kBlock - 1) / (4LL * kBlock)));
}

long long scan_chunks(long long m) { return std::max(1LL, (m + kScanChunk - 1) / kScanChunk); }

hipError_t launch_argmax(int is_float, const void* p, long long n, void* pv, long long* pi, int nparts, double rel,
                         long long* top, double* thr, long long* bins, hipStream_t s)
{
    if (n % 4) return hipErrorInvalidValue;  // DRT outputs hold a multiple of 4 elements
    const uint4* p4 = (const uint4*)p;
    if (is_float) {
        hipLaunchKernelGGL(argmax_partial_kernel<float>, dim3(nparts), dim3(kBlock), 0, s, p4, n / 4, (float*)pv, pi);
        hipLaunchKernelGGL(argmax_final_kernel<float>, dim3(1), dim3(kBlock), 0, s, (const float*)p, n,
                           (const float*)pv, (const long long*)pi, nparts, rel, top, thr, bins);
    } else {
        hipLaunchKernelGGL(argmax_partial_kernel<int>, dim3(nparts), dim3(kBlock), 0, s, p4, n / 4, (int*)pv, pi);
        hipLaunchKernelGGL(argmax_final_kernel<int>, dim3(1), dim3(kBlock), 0, s, (const int*)p, n, (const int*)pv,
                           (const long long*)pi, nparts, rel, top, thr, bins);
    }
    return hipGetLastError();
}

hipError_t launch_plane_peaks(int is_float, int write, const void* p, int N, int nk, const PlaneFrames& F,
                              const long long* top, const double* thr, double tol2, int* counts,
                              const long long* offsets, long long* bins, long long cap, hipStream_t s)
{
    const long long ncol = (long long)nk * N * N;
    const dim3 grid((unsigned)std::min(4096LL, (ncol + kBlock / 64 - 1) / (kBlock / 64)));
#define DRT3D_PEAKS(T, W)                                                                                      \
    hipLaunchKernelGGL((plane_peaks_kernel<T, W>), grid, dim3(kBlock), 0, s, (const T*)p, N, nk, F, top, thr, \
                       tol2, counts, offsets, bins, cap)
    if (is_float) {
        if (write) DRT3D_PEAKS(float, 1);
        else DRT3D_PEAKS(float, 0);
    } else {
        if (write) DRT3D_PEAKS(int, 1);
        else DRT3D_PEAKS(int, 0);
    }
#undef DRT3D_PEAKS
    return hipGetLastError();
}

hipError_t launch_peak_scan(const int* counts, long long m, long long* offsets, long long* csum, long long* count,
                            hipStream_t s)
{
    const long long nc = scan_chunks(m);
    hipLaunchKernelGGL(scan_chunk_sums_kernel, dim3((unsigned)nc), dim3(kBlock), 0, s, counts, m, csum);
    hipLaunchKernelGGL(scan_chunk_offsets_kernel, dim3(1), dim3(kBlock), 0, s, csum, nc, count);
    hipLaunchKernelGGL(scan_chunk_write_kernel, dim3((unsigned)nc), dim3(kBlock), 0, s, counts, m,
                       (const long long*)csum, offsets);
    return hipGetLastError();
}

hipError_t launch_scatter_ones(const long long* bins, const long long* count, long long cap, uint32_t* marker,
                               long long n, uint32_t one, hipStream_t s)
{
    const unsigned grid = (unsigned)std::max(1LL, std::min((cap + kBlock - 1) / kBlock, 4096LL));
    hipLaunchKernelGGL(scatter_ones_kernel, dim3(grid), dim3(kBlock), 0, s, bins, count, cap, marker, n, one);
    return hipGetLastError();
}

}  // namespace drt3d
