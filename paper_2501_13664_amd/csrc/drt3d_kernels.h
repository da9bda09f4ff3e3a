// Device code of the drt3d library for gfx950 (CDNA4, wave64).
//
// DRT passes (forward eq. (11), adjoint eq. (17)). The stage map of eq. (11)
// shifts along the displacement axis only, and its x-part (slope s1, block
// bit v1) and y-part (s2, v2) add independent shifts, so the x- and y-stages
// of a dodecant commute and can be grouped freely (the 2D transform applied
// twice, Sec. 6.2). A pass runs the x-stages mx0..mx0+Kx-1 and the y-stages
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
// DJT passes (eq. (15)): K stages fused per launch; see djt_pass_kernel.
//
// This header holds the kernels as templates. The translation units that
// instantiate them (drt3d_device.hip, drt3d_fast.hip once per pass shape,
// drt3d_djt.hip) compile in parallel.

#pragma once

#include <type_traits>

#include "drt3d_internal.h"

namespace drt3d {

__device__ __forceinline__ int bitrev(int x, int bits)
{
    return bits ? (int)(__brev((unsigned)x) >> (32 - bits)) : 0;
}

template <typename T>
__device__ __forceinline__ T zero_of() { return T(0); }

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
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

// Raw buffer access with the hardware range check: a buffer resource covers
// one column (or one volume line) exactly, so reads outside it return 0 and
// writes outside it are dropped, with no compare in the code. Offsets are in
// bytes; a negative offset wraps to a huge one and is out of range too.
constexpr int kBufferConfig = 0x00020000;  // gfx9 raw-buffer dword 3
// The DRT passes' stores carry the non-temporal hint: every pass writes a
// buffer that no work group of the same launch reads, in whole 128-byte lines
// (the line-aligned store windows), and the next pass streams it back from
// HBM (it is far larger than the caches), so keeping it in L2 only evicts the
// lines the loads reuse. Measured at N = 512: forward 13.0 -> 12.3 ms. The DJT
// passes write rows of 2N-1 elements that end mid-line; they keep the default
// policy, under which L2 merges the partial lines (with the hint the N = 128
// DJT took 21.6 ms instead of 14.3).
constexpr int kStorePolicy = 2;  // cache policy bits of the store: nt

template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const T* base, int elems)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(base), (short)0, elems * (int)sizeof(T), kBufferConfig);
}

__device__ __forceinline__ uint32_t bload(__amdgpu_buffer_rsrc_t r, int off)
{
    return __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
}

__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, int off, uint32_t v)
{
    __builtin_amdgcn_raw_buffer_store_b32(v, r, off, 0, kStorePolicy);
}

// a store under the default cache policy
__device__ __forceinline__ void bstore_cached(__amdgpu_buffer_rsrc_t r, int off, uint32_t v)
{
    __builtin_amdgcn_raw_buffer_store_b32(v, r, off, 0, 0);
}

// Narrow storage (1- or 2-byte elements in HBM, 32-bit arithmetic in
// registers and LDS): loads zero-extend, stores keep the low bytes.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc_bytes(const void* base, int bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, bytes, kBufferConfig);
}

template <int B>
__device__ __forceinline__ uint32_t bload_n(__amdgpu_buffer_rsrc_t r, int off)
{
    static_assert(B == 1 || B == 2 || B == 4, "element bytes");
    if constexpr (B == 4) return __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
    else if constexpr (B == 2) return (uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0);
    else return (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(r, off, 0, 0);
}

template <int B>
__device__ __forceinline__ void bstore_n(__amdgpu_buffer_rsrc_t r, int off, uint32_t v)
{
    static_assert(B == 2 || B == 4, "element bytes");
    if constexpr (B == 4) __builtin_amdgcn_raw_buffer_store_b32(v, r, off, 0, kStorePolicy);
    else __builtin_amdgcn_raw_buffer_store_b16((unsigned short)v, r, off, 0, kStorePolicy);
}

template <typename T> __device__ __forceinline__ uint32_t to_bits(T v) { return __builtin_bit_cast(uint32_t, v); }
template <typename T> __device__ __forceinline__ T from_bits(uint32_t v) { return __builtin_bit_cast(T, v); }

// Forward radix-2 step (one stage of one axis) on the pair (s0, s1) with
// local shift t: s0[l] += s1[l-t], s1[l] = s0_old[l] + s1[l-t-1]. In place,
// 64-position chunks from the top down: a chunk reads only at or below its
// own positions, and writes after all of its reads.
template <typename T, int NCH>
__device__ __forceinline__ void step2_fwd(T* s0, T* s1, int nch, int t, int lane)
{
    T* w0 = s0 + lane;
    T* w1 = s1 + lane;
    const T* r1 = s1 + lane - t - 1;
    const int n = NCH ? NCH : nch;
#pragma unroll
    for (int c = n - 1; c >= 0; --c) {
        const T a = w0[64 * c], b1 = r1[64 * c], b0 = r1[64 * c + 1];
        w0[64 * c] = a + b0;
        w1[64 * c] = a + b1;
    }
}

// Forward radix-4 step: x-stage and y-stage of the same index fused, which is
// the four-term stage map of eq. (11) itself. Slot s_ab receives the slope
// whose new x bit is a and new y bit is b.
template <typename T, int NCH>
__device__ __forceinline__ void step4_fwd(T* s00, T* s10, T* s01, T* s11, int nch, int tx, int ty, int lane)
{
    T* w00 = s00 + lane;
    T* w10 = s10 + lane;
    T* w01 = s01 + lane;
    T* w11 = s11 + lane;
    const T* r10 = s10 + lane - tx - 1;
    const T* r01 = s01 + lane - ty - 1;
    const T* r11 = s11 + lane - tx - ty - 2;
    const int n = NCH ? NCH : nch;
#pragma unroll
    for (int c = n - 1; c >= 0; --c) {
        const int o = 64 * c;
        const T f00 = w00[o];
        const T f10b = r10[o], f10a = r10[o + 1];
        const T f01b = r01[o], f01a = r01[o + 1];
        const T f11c = r11[o], f11b = r11[o + 1], f11a = r11[o + 2];
        const T x0 = f00 + f10a, x1 = f00 + f10b;
        w00[o] = x0 + (f01a + f11a);
        w10[o] = x1 + (f01a + f11b);
        w01[o] = x0 + (f01b + f11b);
        w11[o] = x1 + (f01b + f11c);
    }
}

// Adjoint radix-2 step (transpose of step2_fwd), chunks from the bottom up.
template <typename T, int NCH>
__device__ __forceinline__ void step2_adj(T* s0, T* s1, int nch, int t, int lane)
{
    T* w0 = s0 + lane;
    T* w1 = s1 + lane;
    const T* r0 = s0 + lane + t;
    const T* r1 = s1 + lane + t + 1;
    const int n = NCH ? NCH : nch;
#pragma unroll
    for (int c = 0; c < n; ++c) {
        const int o = 64 * c;
        const T a0 = w0[o], a1 = w1[o], c0 = r0[o], c1 = r1[o];
        w0[o] = a0 + a1;
        w1[o] = c0 + c1;
    }
}

// Adjoint radix-4 step (transpose of step4_fwd).
template <typename T, int NCH>
__device__ __forceinline__ void step4_adj(T* s00, T* s10, T* s01, T* s11, int nch, int tx, int ty, int lane)
{
    T* w00 = s00 + lane;
    T* w10 = s10 + lane;
    T* w01 = s01 + lane;
    T* w11 = s11 + lane;
    const int txy = tx + ty;
    const int n = NCH ? NCH : nch;
#pragma unroll
    for (int c = 0; c < n; ++c) {
        const int o = 64 * c;
        const T c00 = (w00[o] + w10[o]) + (w01[o] + w11[o]);
        const T c10 = (w00[o + tx] + w10[o + tx + 1]) + (w01[o + tx] + w11[o + tx + 1]);
        const T c01 = (w00[o + ty] + w10[o + ty]) + (w01[o + ty + 1] + w11[o + ty + 1]);
        const T c11 = (w00[o + txy] + w10[o + txy + 1]) + (w01[o + txy + 1] + w11[o + txy + 2]);
        w00[o] = c00;
        w10[o] = c10;
        w01[o] = c01;
        w11[o] = c11;
    }
}

// All stages of one pass on the LDS slots (forward or adjoint). x-stage j and
// y-stage j run together as one radix-4 step while both axes have them; the
// rest run as radix-2 steps. Each axis keeps its stage order, which is all the
// in-place slot convention needs.
template <typename T, int NCH>
__device__ __forceinline__ void run_stages(T* lds, int Lp, int pad, int nch, int Kx, int Ky, int adjoint, int wave,
                                           int nwaves, int lane)
{
    const int nslot = 1 << (Kx + Ky);
    const int xmask = (1 << Kx) - 1;
    const int kmax = Kx > Ky ? Kx : Ky;
    for (int jj = 0; jj < kmax; ++jj) {
        const int j = adjoint ? kmax - 1 - jj : jj;
        const bool hx = j < Kx, hy = j < Ky;
        const int bx = 1 << j, by = 1 << (Kx + j);
        if (hx && hy) {
            const int nq = nslot >> 2;
            for (int q = wave; q < nq; q += nwaves) {
                // insert zero bits at positions j (x) and Kx + j (y)
                int p = ((q >> j) << (j + 1)) | (q & (bx - 1));
                p = ((p >> (Kx + j)) << (Kx + j + 1)) | (p & (by - 1));
                const int tx = bitrev(p & (bx - 1), j);
                const int ty = bitrev((p >> Kx) & (bx - 1), j);
                T* s00 = lds + slot_offset(p, Lp, pad);
                if (!adjoint) step4_fwd<T, NCH>(s00, s00 + bx * Lp, s00 + by * Lp, s00 + (bx + by) * Lp, nch, tx, ty, lane);
                else step4_adj<T, NCH>(s00, s00 + bx * Lp, s00 + by * Lp, s00 + (bx + by) * Lp, nch, tx, ty, lane);
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
                if (!adjoint) step2_fwd<T, NCH>(s0, s0 + h * Lp, nch, t, lane);
                else step2_adj<T, NCH>(s0, s0 + h * Lp, nch, t, lane);
            }
        }
        __syncthreads();
    }
}

// Geometry of one work item (one column group, one displacement tile, one
// dodecant slot), shared by its load, stage and store phases.
struct ItemGeom {
    int N, n, Kx, Ky, mx0, my0;
    int sx0, sy0, vhx, vhy;
    int L, Lp, pad, T, H, d0;
    int adjoint;
};

// Column of slot p in its stage buffer (or frame view): block (px, py) for
// the forward input / adjoint output, slope (bitrev px, bitrev py) for the
// forward output / adjoint input.
__device__ __forceinline__ void block_col(const ItemGeom& g, int p, int& c1, int& c2)
{
    const int px = p & ((1 << g.Kx) - 1), py = p >> g.Kx;
    c1 = g.sx0 + (px << g.mx0) + g.vhx;
    c2 = g.sy0 + (py << g.my0) + g.vhy;
}

__device__ __forceinline__ void slope_col(const ItemGeom& g, int p, int& c1, int& c2)
{
    const int px = p & ((1 << g.Kx) - 1), py = p >> g.Kx;
    c1 = bitrev(px, g.Kx) + (g.sx0 << g.Kx) + g.vhx;
    c2 = bitrev(py, g.Ky) + (g.sy0 << g.Ky) + g.vhy;
}

__device__ __forceinline__ int skew_of(const ItemGeom& g, int p)
{
    return g.sx0 * (p & ((1 << g.Kx) - 1)) + g.sy0 * (p >> g.Kx);
}

// Buffer resource and byte offset of lane 0 for a column whose element dd is
// at col[sd * dd], valid for dd in [0, E), addressed from displacement dd0.
template <typename T>
__device__ __forceinline__ void column_rsrc(const T* col, int sd, int E, int dd0, int lane,
                                            __amdgpu_buffer_rsrc_t& rs, int& voff)
{
    if (sd > 0) {
        rs = make_rsrc(col, E);
        voff = 4 * (dd0 + lane);
    } else {  // element dd at col - dd: the resource starts at dd = E - 1
        rs = make_rsrc(col - (E - 1), E);
        voff = 4 * (E - 1 - dd0 - lane);
    }
}

// Buffer resource and lane-0 byte offset of the column that LDS slot p loads
// for the tile at g.d0: block (px, py) at a skewed origin (forward) or slope
// (bitrev px, bitrev py) at the common origin (adjoint).
template <typename T>
__device__ __forceinline__ void src_column(const DrtDesc* __restrict__ d, const ItemGeom& g, int slot, int p, int lane,
                                           __amdgpu_buffer_rsrc_t& rs, int& voff, int& step)
{
    int c1, c2, dd0;
    if (!g.adjoint) {
        block_col(g, p, c1, c2);
        dd0 = g.d0 - g.H - skew_of(g, p);
    } else {
        slope_col(g, p, c1, c2);
        dd0 = g.d0;
    }
    if (d->src_mode == 0) {
        const T* base = reinterpret_cast<const T*>(d->src) + d->phys[slot] * d->src_slot_stride;
        column_rsrc(base + (((long long)c1 << g.n) + c2) * d->P_in, 1, d->E_in, dd0, lane, rs, voff);
        step = 256;
    } else {
        const FrameMap f = d->fm[slot];
        const T* base = reinterpret_cast<const T*>(d->vsrc[f.group]);
        column_rsrc(base + ((long long)f.base + (long long)f.sx * c1 + (long long)f.sy * c2), f.sd, g.N, dd0, lane,
                    rs, voff);
        step = 256 * f.sd;
    }
}

// Issues every global load of the wave's slots (p = wave + i * nwaves) for the
// tile at g.d0: SPW * NCH loads in flight at once.
template <typename T, int NCH, int SPW>
__device__ __forceinline__ void load_regs(const DrtDesc* __restrict__ d, const ItemGeom& g, int slot, int wave,
                                          int nwaves, int lane, uint32_t (&v)[SPW][NCH])
{
#pragma unroll
    for (int i = 0; i < SPW; ++i) {
        __amdgpu_buffer_rsrc_t rs;
        int voff, step;
        src_column<T>(d, g, slot, wave + i * nwaves, lane, rs, voff, step);
#pragma unroll
        for (int c = 0; c < NCH; ++c) v[i][c] = bload(rs, voff + step * c);
    }
}

template <typename T, int NCH, int SPW>
__device__ __forceinline__ void regs_to_lds(const ItemGeom& g, T* lds, int wave, int nwaves, int lane,
                                            const uint32_t (&v)[SPW][NCH])
{
#pragma unroll
    for (int i = 0; i < SPW; ++i) {
        T* s = lds + slot_offset(wave + i * nwaves, g.Lp, g.pad) + lane;
#pragma unroll
        for (int c = 0; c < NCH; ++c) s[64 * c] = from_bits<T>(v[i][c]);
    }
}

// Unpipelined load for shapes without a register buffer (NCH = 0 or many
// slots per wave): per slot, all chunks in flight, then written to LDS.
template <typename T, int NCH>
__device__ __forceinline__ void load_direct(const DrtDesc* __restrict__ d, const ItemGeom& g, int slot, T* lds,
                                            int wave, int nwaves, int lane)
{
    const int nch = NCH ? NCH : (g.L >> 6);
    const int nslot = 1 << (g.Kx + g.Ky);
    for (int p = wave; p < nslot; p += nwaves) {
        __amdgpu_buffer_rsrc_t rs;
        int voff, step;
        src_column<T>(d, g, slot, p, lane, rs, voff, step);
        T* s = lds + slot_offset(p, g.Lp, g.pad) + lane;
        if (NCH) {
            uint32_t v[NCH ? NCH : 1];
#pragma unroll
            for (int c = 0; c < NCH; ++c) v[c] = bload(rs, voff + step * c);
#pragma unroll
            for (int c = 0; c < NCH; ++c) s[64 * c] = from_bits<T>(v[c]);
        } else {
            for (int c = 0; c < nch; ++c) s[64 * c] = from_bits<T>(bload(rs, voff + step * c));
        }
    }
}

// Stores the tile at g.d0 of every slot. The destination column is one buffer
// resource: writes outside [0, E) are dropped; positions past the tile width
// (last chunk) are masked.
template <typename T>
__device__ __forceinline__ void store_tile(const DrtDesc* __restrict__ d, const ItemGeom& g, int slot, const T* lds,
                                           int wave, int nwaves, int lane)
{
    const int nslot = 1 << (g.Kx + g.Ky);
    const int q0 = g.adjoint ? 0 : g.H;
    const int Eout = d->dst_mode == 0 ? d->E_out : g.N;
    T* dstbase = d->dst_mode == 0 ? reinterpret_cast<T*>(d->dst) + d->dphys[slot] * d->dst_slot_stride
                                  : reinterpret_cast<T*>(d->vdst[d->fm[slot].group]);
    const int accum = d->dst_mode == 1 && d->accum[slot];
    const FrameMap f = d->fm[slot];
    const int sdv = d->dst_mode == 0 ? 1 : f.sd;
    const int step = 256 * sdv;
    const int last = (g.T - 1) >> 6;  // chunk holding the tile's end
    const bool last_live = 64 * last + lane < g.T;
    for (int p = wave; p < nslot; p += nwaves) {
        int c1, c2, dd0;
        if (!g.adjoint) {  // common origin: positions H.. hold dd = d0..
            slope_col(g, p, c1, c2);
            dd0 = g.d0;
        } else {           // child column (px, py) at its skewed origin
            block_col(g, p, c1, c2);
            dd0 = g.d0 - skew_of(g, p);
        }
        T* col = d->dst_mode == 0 ? dstbase + (((long long)c1 << g.n) + c2) * d->P_out
                                  : dstbase + ((long long)f.base + (long long)f.sx * c1 + (long long)f.sy * c2);
        __amdgpu_buffer_rsrc_t rs;
        int voff;
        column_rsrc(col, sdv, Eout, dd0, lane, rs, voff);
        const T* s = lds + slot_offset(p, g.Lp, g.pad) + q0 + lane;
        for (int c = 0; c <= last; ++c) {
            if (c < last || last_live) {
                T v = s[64 * c];
                const int off = voff + step * c;
                if (accum) v += from_bits<T>(bload(rs, off));
                bstore_cached(rs, off, to_bits(v));  // tiles end mid-line
            }
        }
    }
}

// Line-aligned store of the tile at g.d0 for the wave's slots. HBM writes are
// cheapest as whole 128-byte lines, and a column's tile rarely starts or ends
// on one, so each tile writes only the lines it completes: elements from the
// last line boundary the previous tile reached (kept in `carry`, at most 31
// of them) up to the last line boundary inside this tile, or to the column
// end on the last tile. The tail goes into `carry` for the next tile. Lines
// split between two columns at a column start stay partial. Needs T >= 32.
template <typename T, int SPW>
__device__ __forceinline__ void store_tile_aligned(const DrtDesc* __restrict__ d, const ItemGeom& g, int slot,
                                                   const T* lds, int wave, int nwaves, int lane, bool last_tile,
                                                   uint32_t (&carry)[SPW])
{
    const int q0 = g.adjoint ? 0 : g.H;
    const int Eout = d->dst_mode == 0 ? d->E_out : g.N;
    T* dstbase = d->dst_mode == 0 ? reinterpret_cast<T*>(d->dst) + d->dphys[slot] * d->dst_slot_stride
                                  : reinterpret_cast<T*>(d->vdst[d->fm[slot].group]);
    const int accum = d->dst_mode == 1 && d->accum[slot];
    const FrameMap f = d->fm[slot];
    const int sdv = d->dst_mode == 0 ? 1 : f.sd;
#pragma unroll
    for (int i = 0; i < SPW; ++i) {
        const int p = wave + i * nwaves;
        int c1, c2, dd0;
        if (!g.adjoint) {  // common origin: positions H.. hold dd = d0..
            slope_col(g, p, c1, c2);
            dd0 = g.d0;
        } else {           // child column (px, py) at its skewed origin
            block_col(g, p, c1, c2);
            dd0 = g.d0 - skew_of(g, p);
        }
        const long long cofs = d->dst_mode == 0 ? (((long long)c1 << g.n) + c2) * d->P_out
                                                : (long long)f.base + (long long)f.sx * c1 + (long long)f.sy * c2;
        // element index of displacement dd is cofs + sdv * dd; a line boundary
        // at dd means that index (for sdv = -1: index + 1) is a multiple of 32.
        const int mis = sdv > 0 ? (int)(cofs & 31) : (int)((cofs + 1) & 31);
        auto line_floor = [&](int x) { return sdv > 0 ? x - ((mis + x) & 31) : x - ((x - mis) & 31); };
        const int fbeg = dd0 <= 0 ? dd0 : line_floor(dd0);   // first dd written now
        const int fend = last_tile ? dd0 + g.T : line_floor(dd0 + g.T);
        __amdgpu_buffer_rsrc_t rs;
        int voff;
        column_rsrc(dstbase + cofs, sdv, Eout, fbeg, lane, rs, voff);
        const T* s = lds + slot_offset(p, g.Lp, g.pad) + q0 - dd0;  // s[dd] holds displacement dd
        const int cnt = fend - fbeg;
        for (int c = 0; 64 * c < cnt; ++c) {
            const int k = 64 * c + lane;
            if (k < cnt) {
                const int dd = fbeg + k;
                T v = dd < dd0 ? from_bits<T>(carry[i]) : s[dd];
                const int off = voff + 256 * sdv * c;
                if (accum) v += from_bits<T>(bload(rs, off));
                bstore(rs, off, to_bits(v));
            }
        }
        // tail [fend, dd0 + T) for the next tile: lane k holds dd = fend + k
        if (!last_tile) {
            const int tail = dd0 + g.T - fend;
            carry[i] = lane < tail ? to_bits(s[fend + lane]) : 0u;
        }
    }
}

__device__ __forceinline__ void zero_pads_fn(void* lds_raw, int elem_bytes, const ItemGeom& g, int wave, int nwaves,
                                             int lane)
{
    uint32_t* lds = reinterpret_cast<uint32_t*>(lds_raw);
    const int nslot = 1 << (g.Kx + g.Ky);
    for (int p = wave; p <= nslot; p += nwaves)
        if (lane < g.pad) lds[p * g.Lp + lane] = 0u;
    (void)elem_bytes;
}

// All tiles of one work item (one column group of one slot). With a register
// buffer (SPW > 0) the next tile's loads are issued before the current tile's
// stages run, so global latency overlaps LDS work.
template <typename T, int NCH, int SPW>
__device__ __forceinline__ void process_group(const DrtDesc* __restrict__ d, ItemGeom& g, int slot, int ntiles,
                                              T* lds, int wave, int nwaves, int lane)
{
    const int nch = NCH ? NCH : (g.L >> 6);
    zero_pads_fn(lds, sizeof(T), g, wave, nwaves, lane);
    if constexpr (SPW > 0) {
        uint32_t v[SPW][NCH];
        uint32_t carry[SPW];
#pragma unroll
        for (int i = 0; i < SPW; ++i) carry[i] = 0u;
        g.d0 = 0;
        load_regs<T, NCH, SPW>(d, g, slot, wave, nwaves, lane, v);
        for (int tile = 0; tile < ntiles; ++tile) {
            g.d0 = tile * g.T;
            regs_to_lds<T, NCH, SPW>(g, lds, wave, nwaves, lane, v);
            __syncthreads();
            if (tile + 1 < ntiles) {
                ItemGeom gn = g;
                gn.d0 = (tile + 1) * g.T;
                load_regs<T, NCH, SPW>(d, gn, slot, wave, nwaves, lane, v);
            }
            run_stages<T, NCH>(lds, g.Lp, g.pad, nch, g.Kx, g.Ky, g.adjoint, wave, nwaves, lane);
            store_tile_aligned<T, SPW>(d, g, slot, lds, wave, nwaves, lane, tile + 1 == ntiles, carry);
            __syncthreads();
        }
    } else {
        for (int tile = 0; tile < ntiles; ++tile) {
            g.d0 = tile * g.T;
            load_direct<T, NCH>(d, g, slot, lds, wave, nwaves, lane);
            __syncthreads();
            run_stages<T, NCH>(lds, g.Lp, g.pad, nch, g.Kx, g.Ky, g.adjoint, wave, nwaves, lane);
            store_tile<T>(d, g, slot, lds, wave, nwaves, lane);
            __syncthreads();
        }
    }
}

// Register-buffer shape: SPW slots per wave, NCH chunks, at most 48 values.
template <typename T, int NCH>
__device__ __forceinline__ void dispatch_spw(const DrtDesc* __restrict__ d, ItemGeom& g, int slot, int ntiles, T* lds,
                                             int wave, int nwaves, int lane)
{
    const int nslot = 1 << (g.Kx + g.Ky);
    const int spw = (nslot % nwaves == 0) ? nslot / nwaves : 0;
    if (NCH && spw == 8 && 8 * NCH <= 48) process_group<T, NCH, (NCH && 8 * NCH <= 48) ? 8 : 0>(d, g, slot, ntiles, lds, wave, nwaves, lane);
    else if (NCH && spw == 4 && 4 * NCH <= 48) process_group<T, NCH, (NCH && 4 * NCH <= 48) ? 4 : 0>(d, g, slot, ntiles, lds, wave, nwaves, lane);
    else if (NCH && spw == 2 && 2 * NCH <= 48) process_group<T, NCH, (NCH && 2 * NCH <= 48) ? 2 : 0>(d, g, slot, ntiles, lds, wave, nwaves, lane);
    else if (NCH && spw == 1) process_group<T, NCH, NCH ? 1 : 0>(d, g, slot, ntiles, lds, wave, nwaves, lane);
    else process_group<T, NCH, 0>(d, g, slot, ntiles, lds, wave, nwaves, lane);
}

template <typename T>
__global__ void __launch_bounds__(512)
drt_pass_kernel(const DrtDesc* __restrict__ descs, int ndesc, long long total_wg)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* lds = reinterpret_cast<T*>(smem_raw);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nwaves = blockDim.x >> 6;

    // A work item is one column group of one dodecant slot; its work group
    // walks the group's displacement tiles in order, so the cache lines that a
    // tile boundary splits are completed in the same L2 and the halo a tile
    // shares with the previous one is read from it.
    for (long long wg = blockIdx.x; wg < total_wg; wg += gridDim.x) {
        const DrtDesc* d = descs + find_desc_drt(descs, ndesc, wg);
        const int local = (int)(wg - d->wg_begin);
        const int lg_groups = (d->n - d->Kx) + (d->n - d->Ky);
        const int gidx = local & ((1 << lg_groups) - 1);
        const int slot = local >> lg_groups;

        ItemGeom g;
        g.N = d->N; g.n = d->n;
        g.Kx = d->Kx; g.Ky = d->Ky; g.mx0 = d->mx0; g.my0 = d->my0;
        g.L = d->L; g.Lp = d->Lp; g.pad = g.Lp - g.L; g.T = d->T; g.H = d->H;
        g.adjoint = d->adjoint;
        g.d0 = 0;
        const int gy = gidx & (d->groups_y - 1), gx = gidx >> (g.n - g.Ky);
        g.sx0 = gx & ((1 << g.mx0) - 1);
        g.vhx = (gx >> g.mx0) << (g.mx0 + g.Kx);
        g.sy0 = gy & ((1 << g.my0) - 1);
        g.vhy = (gy >> g.my0) << (g.my0 + g.Ky);
        // adjoint outputs are skewed by up to smax: the group needs fewer tiles
        const int span = g.adjoint ? d->E_out + g.sx0 * ((1 << g.Kx) - 1) + g.sy0 * ((1 << g.Ky) - 1) : d->E_out;
        const int ntiles = min(d->ntiles, (span + g.T - 1) / g.T);

        switch (g.L >> 6) {
            case 1: dispatch_spw<T, 1>(d, g, slot, ntiles, lds, wave, nwaves, lane); break;
            case 2: dispatch_spw<T, 2>(d, g, slot, ntiles, lds, wave, nwaves, lane); break;
            case 3: dispatch_spw<T, 3>(d, g, slot, ntiles, lds, wave, nwaves, lane); break;
            case 4: dispatch_spw<T, 4>(d, g, slot, ntiles, lds, wave, nwaves, lane); break;
            case 5: dispatch_spw<T, 5>(d, g, slot, ntiles, lds, wave, nwaves, lane); break;
            case 6: dispatch_spw<T, 6>(d, g, slot, ntiles, lds, wave, nwaves, lane); break;
            default: dispatch_spw<T, 0>(d, g, slot, ntiles, lds, wave, nwaves, lane); break;
        }
    }
}

// ---------------------------------------------------------------------------
// Shape-specialised pass kernel: KX x-stages, KY y-stages (KX, KY <= 3,
// 2^(KX+KY) >= 8 columns), L = 64 * NCH, eight wavefronts. Wave w owns the
// slots p = w + 8 i, which share the x index px = w mod 2^KX, so a slot's
// column offset is a per-wave base plus a per-slot stride. Each side of the
// pass (source, destination) is one buffer resource over its whole region (a
// stage buffer slot, one dodecant of the output, or the volume; regions below
// 2^31 bytes); column offsets travel in VGPRs, so the hardware range check
// covers the full offset, and each column's own range [0, E) is enforced in
// the lanes: out-of-range loads are replaced by zero, out-of-range stores are
// masked.
namespace fast {

template <int KX, int NW>
__device__ __forceinline__ int py_of(int wave, int i) { return (wave >> KX) + i * (NW >> KX); }

// FINAL: the forward's last pass, whose output columns are the caller's
// projections. A column (s1, s2) is zero past dd = N-1+s1+s2 (the support of
// eq. (9)), so a tile past the support of every column of the group is written
// as zeros straight from registers, with no loads and no LDS stages.
// MODE: 0 a forward pass into a stage buffer, 1 the forward's last pass
// (FINAL), 2 an adjoint pass; fixing it at compile time drops the other
// modes' bookkeeping from the kernel.
// NW: wavefronts per work group (8, or 16 for the 64-column 3.3 passes).
// SB, DB: bytes per element of the source and destination in HBM (4, or the
// narrow storage of 8-bit volumes: 1 for the volume, 2 for the first stage
// buffer, whose partial sums of at most 2^(KX+KY) <= 256 voxels of 0..255 fit
// 16 bits). Arithmetic stays 32-bit.
// The first pass of an 8-bit volume (SB = 1) packs two column groups into
// the 16-bit halves of each LDS word: every partial sum stays below 2^16, so
// one 32-bit add adds both halves with no carry between them, and one pass of
// stages serves two groups. The groups share every shift (the first pass has
// no skew), and the second group is the first one's neighbour.
template <typename T, int KX, int KY, int NCH, int MODE, int NW, int SB = 4, int DB = 4>
__global__ void __launch_bounds__(64 * NW, NW == 16 ? 8 : SB == 1 && DB == 2 ? 4 : 6)
drt_pass_fast(const DrtDesc* __restrict__ descs, int ndesc, long long total_wg)
{
    static_assert((SB == 4 && DB == 4) || (MODE != 2 && sizeof(T) == 4), "narrow storage: forward passes only");
    constexpr int PK = SB == 1 && DB == 2 ? 1 : 0;  // column groups packed per work item: 2^PK
    static_assert(!PK || (MODE == 0 && NW == 8), "packed groups: the 8-bit first pass");
    constexpr int LINE = 128 / DB;  // destination elements per 128-byte line
    constexpr bool FINAL = MODE == 1;
    constexpr int adjoint = MODE == 2 ? 1 : 0;
    constexpr int NS = 1 << (KX + KY), SPW = NS / NW, L = 64 * NCH;
    static_assert(NS >= 8 && KX <= 3 && KY <= 3, "shape");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* lds = reinterpret_cast<T*>(smem_raw);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int px = wave & ((1 << KX) - 1);
    const int rpx = bitrev(px, KX);

    for (long long wg = blockIdx.x; wg < total_wg; wg += gridDim.x) {
        const DrtDesc* d = descs + find_desc_drt(descs, ndesc, wg);
        const int local = (int)(wg - d->wg_begin);
        const int n = d->n, N = d->N, mx0 = d->mx0, my0 = d->my0;
        const int lg_groups = (n - KX) + (n - KY);
        int gidx = local & ((1 << (lg_groups - PK)) - 1);
        int slot = local >> (lg_groups - PK);
        int gidx2 = 2 * gidx + 1;  // packed: the second group, the next along y
        if (PK) gidx = 2 * gidx;
        if (KX == KY && d->xcd_run > 0) {
            // runs of xcd_run slots; inside a run, work group w takes block
            // (w / (8 run)) * 8 + w % 8 of slot (w / 8) % run, in the layout's
            // own block coordinates, then maps it into the slot's frame
            // (packed: block pairs along the layout's second index)
            const int rl = d->xcd_run, ng = (1 << lg_groups) >> PK;
            const int run = local / (rl * ng), rem = local - run * rl * ng;
            const int hi = rem / (8 * rl), lo = rem - hi * 8 * rl;
            slot = run * rl + lo / 8;
            const int b = hi * 8 + (lo & 7);
            const int G = N >> KX, GP = G >> PK;
            const int b1 = b / GP, b2 = (b - b1 * GP) << PK;
            const FrameMap f = d->fm[slot];
            // x' runs along the layout's first index (stride N^2) or its second
            const bool along_first = f.sx == N * N || f.sx == -N * N;
            auto frame_gidx = [&](int c1, int c2) {
                const int bx = along_first ? (f.sx > 0 ? c1 : G - 1 - c1) : (f.sx > 0 ? c2 : G - 1 - c2);
                const int by = along_first ? (f.sy > 0 ? c2 : G - 1 - c2) : (f.sy > 0 ? c1 : G - 1 - c1);
                return (bx << (n - KY)) | by;
            };
            gidx = frame_gidx(b1, b2);
            if (PK) gidx2 = frame_gidx(b1, b2 + 1);
        }
        const int T_ = d->T, H = d->H, Lp = d->Lp, pad = Lp - L;
        const int gy = gidx & ((1 << (n - KY)) - 1), gx = gidx >> (n - KY);
        const int sx0 = gx & ((1 << mx0) - 1);
        const int vhx = (gx >> mx0) << (mx0 + KX);
        const int sy0 = gy & ((1 << my0) - 1);
        const int vhy = (gy >> my0) << (my0 + KY);
        const int span = adjoint ? d->E_out + sx0 * ((1 << KX) - 1) + sy0 * ((1 << KY) - 1) : d->E_out;
        const int ntiles = min(d->ntiles, (span + T_ - 1) / T_);
        // tiles [0, nlive) hold the group's support, the rest are zero (FINAL)
        int nlive = ntiles;
        if (FINAL) {
            const int supp = N - 1 + (sx0 << KX) + (1 << KX) - 1 + (sy0 << KY) + (1 << KY) - 1;
            nlive = min(ntiles, supp / T_ + 1);
        }
        const FrameMap fm = d->fm[slot];

        // block column (px, py): c1 = sx0 + (px << mx0) + vhx, c2 = sy0 + (py << my0) + vhy
        // slope column:          c1 = bitrev(px) + (sx0 << KX) + vhx, c2 = bitrev(py) + (sy0 << KY) + vhy
        const int c1b = sx0 + (px << mx0) + vhx, c2b = sy0 + vhy;
        const int c1s = rpx + (sx0 << KX) + vhx, c2s = (sy0 << KY) + vhy;
        // source: element of slot i at displacement dd is region[o + y(i)*ys + sd*dd]
        __amdgpu_buffer_rsrc_t rs_src, rs_dst;
        int so, sys, ssd, sE, do_, dys, dsd, dE;
        if (d->src_mode == 0) {
            const char* base = reinterpret_cast<const char*>(d->src) + (long long)SB * d->phys[slot] * d->src_slot_stride;
            rs_src = make_rsrc_bytes(base, SB * (int)d->src_slot_stride);
            const int c1 = adjoint ? c1s : c1b, c2 = adjoint ? c2s : c2b;
            so = ((c1 << n) + c2) * d->P_in;
            sys = adjoint ? d->P_in : (d->P_in << my0);
            ssd = 1;
            sE = d->E_in;
        } else {
            rs_src = make_rsrc_bytes(d->vsrc[fm.group], SB * N * N * N);
            so = fm.base + fm.sx * c1b + fm.sy * c2b;
            sys = fm.sy * (1 << my0);
            ssd = fm.sd;
            sE = N;
        }
        // float last pass with `sub`: the stores write sub - result
        constexpr bool SUBT = FINAL && std::is_same<T, float>::value && DB == 4 && NW == 8;
        const bool has_sub = SUBT && d->sub != nullptr;
        __amdgpu_buffer_rsrc_t rs_sub = rs_src;
        if (d->dst_mode == 0) {
            char* base = reinterpret_cast<char*>(d->dst) + (long long)DB * d->dphys[slot] * d->dst_slot_stride;
            rs_dst = make_rsrc_bytes(base, DB * (int)d->dst_slot_stride);
            if (has_sub)
                rs_sub = make_rsrc_bytes(reinterpret_cast<const char*>(d->sub) +
                                             (long long)DB * d->dphys[slot] * d->dst_slot_stride,
                                         DB * (int)d->dst_slot_stride);
            const int c1 = adjoint ? c1b : c1s, c2 = adjoint ? c2b : c2s;
            do_ = ((c1 << n) + c2) * d->P_out;
            dys = adjoint ? (d->P_out << my0) : d->P_out;
            dsd = 1;
            dE = d->E_out;
        } else {
            rs_dst = make_rsrc(reinterpret_cast<T*>(d->vdst[fm.group]), N * N * N);
            do_ = fm.base + fm.sx * c1b + fm.sy * c2b;
            dys = fm.sy * (1 << my0);
            dsd = fm.sd;
            dE = N;
        }
        // packed: the second group's source and destination columns sit a
        // fixed offset from the first's (a first pass: block columns are
        // c1 = px + (gx << KX), c2 = py + (gy << KY))
        int so2 = 0, do2 = 0;
        if constexpr (PK) {
            const int gy2 = gidx2 & ((1 << (n - KY)) - 1), gx2 = gidx2 >> (n - KY);
            const int dc1 = (gx2 - gx) << KX, dc2 = (gy2 - gy) << KY;
            so2 = fm.sx * dc1 + fm.sy * dc2;        // volume (src_mode 1), bytes
            do2 = (dc1 * N + dc2) * d->P_out;       // stage buffer (dst_mode 0), elements
        }
        // only the adjoint's last pass adds into the volume accumulators
        const bool accum = MODE == 2 && d->dst_mode == 1 && d->accum[slot];
        const int q0 = adjoint ? 0 : H;

        // zero pads
        for (int p = wave; p <= NS; p += NW)
            if (lane < pad) lds[p * Lp + lane] = zero_of<T>();

        uint32_t v[SPW][NCH];
        uint32_t v2[PK ? SPW : 1][PK ? NCH : 1];  // packed: the second group's elements
        uint32_t carry[SPW];
        uint32_t carry2[SPW];  // the last pass's pair stores carry pairs: the second element
#pragma unroll
        for (int i = 0; i < SPW; ++i) carry[i] = carry2[i] = 0u;
        // x * sd for sd = +-1, without a branch: (x ^ neg) - neg, neg = 0 or -1
        const int sneg = ssd > 0 ? 0 : -1, dneg = dsd > 0 ? 0 : -1;

        // columns run with unit stride, up or down (ssd, dsd = +-1): byte
        // offsets advance by +-64 SB per 64-element chunk, no multiplies
        // packed 8-bit first pass: lanes load 4-byte words (elements dd0 + 4w ...
        // 4w + 3 of a column; dd0 = d0 - H is a multiple of 4, since the
        // first pass has no skew and its halo H is rounded up to a multiple
        // of 4). An ascending column starts on a word (its base has no N - 1
        // term) and a descending one ends on one (base = 3 mod 4); N is a
        // multiple of 4, so a word is inside the column whole or not at all.
        // A descending column's word holds its elements in reverse byte order.
        constexpr int NWD = (16 * NCH + 63) / 64;  // word loads per slot, group and tile
        auto issue_loads = [&](int d0) {
            if constexpr (PK) {
#pragma unroll
                for (int i = 0; i < SPW; ++i) {
                    const int colo = so + py_of<KX, NW>(wave, i) * sys;
#pragma unroll
                    for (int c = 0; c < NWD; ++c) {
                        const int w = lane + 64 * c;
                        const int e = d0 - H + 4 * w;
                        const bool in = (16 * NCH % 64 == 0 || w < 16 * NCH) && (unsigned)e < (unsigned)sE;
                        const int off = colo + (e ^ sneg) - sneg + (sneg & -3);
                        v[i][c] = __builtin_amdgcn_raw_buffer_load_b32(rs_src, in ? off : -1, 0, 0);
                        v2[i][c] = __builtin_amdgcn_raw_buffer_load_b32(rs_src, in ? so2 + off : -1, 0, 0);
                    }
                }
                return;
            }
#pragma unroll
            for (int i = 0; i < SPW; ++i) {
                const int py = py_of<KX, NW>(wave, i);
                const int y = adjoint ? bitrev(py, KY) : py;
                const int dd0 = adjoint ? d0 : d0 - H - sx0 * px - sy0 * py;
                const int colo = so + y * sys;
                const int dl = dd0 + lane;
                const int ob = SB * colo + ((SB * dl) ^ sneg) - sneg;
#pragma unroll
                for (int c = 0; c < NCH; ++c) {
                    // lanes outside the column get an offset past the resource:
                    // the hardware returns 0 for them without touching memory
                    const bool in = (unsigned)(dl + 64 * c) < (unsigned)sE;
                    v[i][c] = bload_n<SB>(rs_src, in ? ob + ((64 * SB * c) ^ sneg) - sneg : -1);
                }
            }
        };

        issue_loads(0);
        for (int tile = 0; tile < ntiles; ++tile) {
            const int d0 = tile * T_;
            const bool live = !FINAL || tile < nlive;
            if (live) {
                if constexpr (PK) {
                    // the two groups' bytes into the 16-bit halves of 4 LDS words
#pragma unroll
                    for (int i = 0; i < SPW; ++i) {
                        T* sl = lds + slot_offset(wave + i * NW, Lp, pad);
#pragma unroll
                        for (int c = 0; c < NWD; ++c) {
                            const int w = lane + 64 * c;
                            const uint32_t xa = sneg ? __builtin_bswap32(v[i][c]) : v[i][c];
                            const uint32_t xb = sneg ? __builtin_bswap32(v2[i][c]) : v2[i][c];
                            // bytes k of xa and xb -> (a_k, b_k) 16-bit halves
                            const u32x4 q = {__builtin_amdgcn_perm(xb, xa, 0x0c040c00u), __builtin_amdgcn_perm(xb, xa, 0x0c050c01u),
                                             __builtin_amdgcn_perm(xb, xa, 0x0c060c02u), __builtin_amdgcn_perm(xb, xa, 0x0c070c03u)};
                            if (16 * NCH % 64 == 0 || w < 16 * NCH) *reinterpret_cast<u32x4*>(sl + 4 * w) = q;
                        }
                    }
                } else {
#pragma unroll
                    for (int i = 0; i < SPW; ++i) {
                        T* sl = lds + slot_offset(wave + i * NW, Lp, pad) + lane;
#pragma unroll
                        for (int c = 0; c < NCH; ++c) sl[64 * c] = from_bits<T>(v[i][c]);
                    }
                }
                __syncthreads();
                if (tile + 1 < nlive) issue_loads(d0 + T_);
                run_stages<T, NCH>(lds, Lp, pad, NCH, KX, KY, adjoint, wave, NW, lane);
            }

            // line-aligned store with carry (see store_tile_aligned)
            const bool last_tile = tile + 1 == ntiles;
            if constexpr (MODE != 2 && (DB == 4 || DB == 2) && NW == 8) {
                // Forward passes: lanes store pairs of elements (8 bytes, or two
                // 16-bit halves of one word in narrow storage). Every
                // window edge (line boundaries, column ends, d0 and T) is even,
                // since 3N - 2, the stage extents and pitches, the tile widths
                // L - H and the halos 2^KX + 2^KY - 2 all are, so a pair is
                // stored whole or not at all. The slot's window is read from
                // LDS in one batch (indices clamped, so lanes that store nothing
                // still read inside the work group's LDS), then the pairs inside
                // the window store. (With sixteen wavefronts the pairs would not
                // fit 64 registers.)
                constexpr int NP = (NCH + 2) / 2;  // 128-element store chunks
#pragma unroll
                for (int i = 0; i < SPW; ++i) {
                    const int py = py_of<KX, NW>(wave, i);
                    const int colo = do_ + bitrev(py, KY) * dys;  // even; forward outputs run upwards
                    const int fbeg = d0 <= 0 ? d0 : d0 - ((colo + d0) & (LINE - 1));
                    const int fend = last_tile ? d0 + T_ : d0 + T_ - ((colo + d0 + T_) & (LINE - 1));
                    const T* slot_base = lds + slot_offset(wave + i * NW, Lp, pad);
                    const int rel = q0 - d0;  // in-slot index of displacement dd: rel + dd (even)
                    const int fl = fbeg + 2 * lane;
                    u32x2 val[NP];
#pragma unroll
                    for (int c = 0; c < NP; ++c) {
                        const int q = min(max(rel + fl + 128 * c, -pad), L + pad - 2);
                        val[c] = live ? *reinterpret_cast<const u32x2*>(slot_base + q) : u32x2{0u, 0u};
                    }
                    // only the first chunk reaches below d0: those lanes hold the carry
                    if (fl < d0) val[0] = u32x2{carry[i], carry2[i]};
                    if constexpr (SUBT) {
                        if (has_sub) {
                            // the window's pairs of sub, then sub - result (lanes
                            // outside the window read past the resource: 0)
                            u32x2 sv[NP];
#pragma unroll
                            for (int c = 0; c < NP; ++c) {
                                const int dd = fl + 128 * c;
                                sv[c] = __builtin_amdgcn_raw_buffer_load_b64(
                                    rs_sub, dd < fend && (unsigned)dd < (unsigned)dE ? 4 * (colo + dd) : -1, 0, 0);
                            }
#pragma unroll
                            for (int c = 0; c < NP; ++c)
                                val[c] = u32x2{to_bits(from_bits<float>(sv[c].x) - from_bits<float>(val[c].x)),
                                               to_bits(from_bits<float>(sv[c].y) - from_bits<float>(val[c].y))};
                        }
                    }
                    u32x2 next_carry = {0u, 0u};
                    if (!last_tile && live)
                        next_carry = *reinterpret_cast<const u32x2*>(
                            slot_base + min(max(rel + fend + 2 * lane, -pad), L + pad - 2));
#pragma unroll
                    for (int c = 0; c < NP; ++c) {
                        const int dd = fl + 128 * c;
                        if (dd < fend && (unsigned)dd < (unsigned)dE) {
                            if constexpr (DB == 4)
                                __builtin_amdgcn_raw_buffer_store_b64(val[c], rs_dst, 4 * (colo + dd), 0, kStorePolicy);
                            else
                                __builtin_amdgcn_raw_buffer_store_b32((val[c].x & 0xffffu) | (val[c].y << 16), rs_dst,
                                                                      2 * (colo + dd), 0, kStorePolicy);
                            if constexpr (PK)  // the second group: the high halves
                                __builtin_amdgcn_raw_buffer_store_b32((val[c].x >> 16) | (val[c].y & 0xffff0000u), rs_dst,
                                                                      2 * (colo + do2 + dd), 0, kStorePolicy);
                        }
                    }
                    const bool keep = !last_tile && 2 * lane < d0 + T_ - fend;
                    carry[i] = keep ? next_carry.x : 0u;
                    carry2[i] = keep ? next_carry.y : 0u;
                }
            } else if constexpr (FINAL) {
                // The slot's window is read from LDS in one batch (in-slot
                // indices clamped, so that lanes which store nothing still read
                // inside the work group's LDS), then the lanes inside the
                // window and the column store: no store waits on its own read.
#pragma unroll
                for (int i = 0; i < SPW; ++i) {
                    const int py = py_of<KX, NW>(wave, i);
                    const int colo = do_ + bitrev(py, KY) * dys;
                    const int mis = dsd > 0 ? (colo & (LINE - 1)) : ((colo + 1) & (LINE - 1));
                    auto line_floor = [&](int x) {
                        return dsd > 0 ? x - ((mis + x) & (LINE - 1)) : x - ((x - mis) & (LINE - 1));
                    };
                    const int fbeg = d0 <= 0 ? d0 : line_floor(d0);
                    const int fend = last_tile ? d0 + T_ : line_floor(d0 + T_);
                    const T* slot_base = lds + slot_offset(wave + i * NW, Lp, pad);
                    const int rel = q0 - d0;  // in-slot index of displacement dd: rel + dd
                    const int cnt = fend - fbeg;
                    const int fl = fbeg + lane;
                    const int ob = DB * colo + ((DB * fl) ^ dneg) - dneg;
                    uint32_t val[NCH + 1];
#pragma unroll
                    for (int c = 0; c < NCH + 1; ++c)
                        val[c] = live ? to_bits(slot_base[min(max(rel + fl + 64 * c, -pad), L + pad - 1)]) : 0u;
                    // only the first chunk reaches below d0: those lanes hold the carry
                    if (fl < d0) val[0] = carry[i];
                    const uint32_t next_carry =
                        !last_tile && live ? to_bits(slot_base[min(max(rel + fend + lane, -pad), L + pad - 1)]) : 0u;
#pragma unroll
                    for (int c = 0; c < NCH + 1; ++c) {
                        const int dd = fl + 64 * c;
                        if (64 * c + lane < cnt && (unsigned)dd < (unsigned)dE)
                            bstore_n<DB>(rs_dst, ob + ((64 * DB * c) ^ dneg) - dneg, val[c]);
                    }
                    if (!last_tile) carry[i] = lane < d0 + T_ - fend ? next_carry : 0u;
                }
            } else {
#pragma unroll
                for (int i = 0; i < SPW; ++i) {
                    const int py = py_of<KX, NW>(wave, i);
                    const int y = adjoint ? py : bitrev(py, KY);
                    const int dd0 = adjoint ? d0 - sx0 * px - sy0 * py : d0;
                    const int colo = do_ + y * dys;
                    const int mis = dsd > 0 ? (colo & (LINE - 1)) : ((colo + 1) & (LINE - 1));
                    auto line_floor = [&](int x) {
                        return dsd > 0 ? x - ((mis + x) & (LINE - 1)) : x - ((x - mis) & (LINE - 1));
                    };
                    const int fbeg = dd0 <= 0 ? dd0 : line_floor(dd0);
                    const int fend = last_tile ? dd0 + T_ : line_floor(dd0 + T_);
                    const T* sl = lds + slot_offset(wave + i * NW, Lp, pad) + q0 - dd0;
                    const int cnt = fend - fbeg;
                    const int fl = fbeg + lane;
                    const int ob = DB * colo + (dsd > 0 ? DB * fl : -DB * fl);
#pragma unroll
                    for (int c = 0; c < NCH + 1; ++c) {
                        const int k = 64 * c + lane;
                        const int dd = fbeg + k;
                        if (k < cnt && (unsigned)dd < (unsigned)dE) {
                            T val = dd < dd0 ? from_bits<T>(carry[i]) : live ? sl[dd] : zero_of<T>();
                            const int off = ob + (dsd > 0 ? 64 * DB * c : -64 * DB * c);
                            if (accum) val += from_bits<T>(bload(rs_dst, off));
                            bstore_n<DB>(rs_dst, off, to_bits(val));
                        }
                    }
                    if (!last_tile) {
                        const int tail = dd0 + T_ - fend;
                        carry[i] = lane < tail && live ? to_bits(sl[fend + lane]) : 0u;
                    }
                }
            }
            if (live) __syncthreads();
        }
    }
}

// The adjoint's last pass (the transpose of the forward's first pass: stages
// 0..2 of both axes) fused over a volume layout group. The four dodecants of
// a group write the same layout, their frames differ by a rotation or
// reflection of the slope plane, and they share the displacement axis (same
// sign and origin), so their 8 x 8 column blocks and displacement tiles map
// onto the same physical block and z range. A work item owns one physical
// block: for each tile it runs the four dodecants' transposed stages in turn
// (each loaded into LDS ahead of time, the next while the current one runs),
// adds each result into registers in physical column order, and writes the
// block once. The volume is written once instead of once per dodecant with
// three read-backs. Slots 4g..4g+3 of the descriptor are group g's dodecants.
// Each step's columns load straight into LDS (buffer loads to LDS, no
// register staging), so the sums and tails fit in 80 registers: three work
// groups of eight wavefronts per CU, whose load phases overlap each other's
// stages (two groups of sixteen).
// K: stages per axis of the pass (blocks of B x B columns, B = 2^K); NW:
// wavefronts, a multiple of B (wave w owns slots p = w + NW i, whose x index
// w mod B is fixed per wave, as in drt_pass_fast).
template <typename T, int K, int NCH, int NW>
__global__ void __launch_bounds__(64 * NW, NW == 16 ? 8 : 6)
drt_adj_last_group(const DrtDesc* __restrict__ descs, int ndesc, long long total_wg)
{
    constexpr int B = 1 << K, NS = B * B, SPW = NS / NW, L = 64 * NCH, NDOD = 4;
    static_assert(NW % B == 0 && NS % NW == 0, "slots per wave");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* lds = reinterpret_cast<T*>(smem_raw);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int px = wave & (B - 1);  // x index of the wave's slots (frame side) and columns (physical side)
    const int rpx = bitrev(px, K);
    auto y_of = [&](int i) { return (wave >> K) + i * (NW >> K); };

    for (long long wg = blockIdx.x; wg < total_wg; wg += gridDim.x) {
        const DrtDesc* d = descs + find_desc_drt(descs, ndesc, wg);
        const int local = (int)(wg - d->wg_begin);
        const int n = d->n, N = d->N;
        const int G = N >> K;
        const int lg = 2 * (n - K);
        const int blk = local & ((1 << lg) - 1);
        const int grp = local >> lg;
        const int b1 = blk / G, b2 = blk - b1 * G;  // physical block along the layout's first and second index
        const int T_ = d->T, Lp = d->Lp, pad = Lp - L;
        const int ntiles = min(d->ntiles, (d->E_out + T_ - 1) / T_);
        const FrameMap f0 = d->fm[NDOD * grp];
        const int dsd = f0.sd;                        // shared by the group
        const int zb = dsd > 0 ? 0 : N - 1;           // column origin along the displacement axis
        const __amdgpu_buffer_rsrc_t rs_dst = make_rsrc(reinterpret_cast<T*>(d->vdst[f0.group]), N * N * N);

        // frame view of dodecant r: its block of the physical block, and the
        // LDS slot of physical position (pa, pb) in the block
        auto frame_block = [&](const FrameMap& f, int& bx, int& by) {
            const bool first = f.sx == N * N || f.sx == -N * N;
            bx = first ? (f.sx > 0 ? b1 : G - 1 - b1) : (f.sx > 0 ? b2 : G - 1 - b2);
            by = first ? (f.sy > 0 ? b2 : G - 1 - b2) : (f.sy > 0 ? b1 : G - 1 - b1);
        };
        auto frame_slot = [&](const FrameMap& f, int pa, int pb) {
            const bool first = f.sx == N * N || f.sx == -N * N;
            const int qx = first ? (f.sx > 0 ? pa : B - 1 - pa) : (f.sx > 0 ? pb : B - 1 - pb);
            const int qy = first ? (f.sy > 0 ? pb : B - 1 - pb) : (f.sy > 0 ? pa : B - 1 - pa);
            return qx + B * qy;
        };

        for (int p = wave; p <= NS; p += NW)
            if (lane < pad) lds[p * Lp + lane] = zero_of<T>();

        T acc[SPW][NCH + 1];  // this tile's sums over the dodecants, per physical column and store chunk
        uint32_t carry[SPW];  // the previous tile's tail sums (lane k: displacement fbeg + k)
        T ncarry[SPW];        // this tile's tail sums
#pragma unroll
        for (int i = 0; i < SPW; ++i) carry[i] = 0u;

        // step j = tile * 4 + r loads dodecant r's slope columns for the tile
        // into their LDS slots; lanes past the input extent load zeros
        typedef __attribute__((address_space(3))) void lds_void;
        auto issue_loads = [&](int j) {
            const int tile = j >> 2, r = j & 3;
            const int s = NDOD * grp + r;
            const FrameMap f = d->fm[s];
            int bx, by;
            frame_block(f, bx, by);
            const char* base = reinterpret_cast<const char*>(d->src) + 4LL * d->phys[s] * d->src_slot_stride;
            const __amdgpu_buffer_rsrc_t rs = make_rsrc_bytes(base, 4 * (int)d->src_slot_stride);
            const int so = (((rpx + B * bx) << n) + B * by) * d->P_in;
            const int d0 = tile * T_;
#pragma unroll
            for (int i = 0; i < SPW; ++i) {
                const int colo = so + bitrev(y_of(i), K) * d->P_in;
                const int dl = d0 + lane;
                const int ob = 4 * (colo + dl);
                T* dst = lds + slot_offset(wave + i * NW, Lp, pad);
#pragma unroll
                for (int c = 0; c < NCH; ++c) {
                    const bool in = (unsigned)(dl + 64 * c) < (unsigned)d->E_in;
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void*)(dst + 64 * c), 4, in ? ob + 256 * c : -1,
                                                            0, 0, 0);
                }
            }
        };

        const int nsteps = ntiles * NDOD;
        __syncthreads();  // the slot pads are written
        for (int j = 0; j < nsteps; ++j) {
            const int tile = j >> 2, r = j & 3;
            const int d0 = tile * T_;
            const bool last_tile = tile + 1 == ntiles;
            issue_loads(j);
            // this wave's loads have landed in LDS; then every wave's have
            asm volatile("" ::: "memory");
            __builtin_amdgcn_s_waitcnt(0 | (7 << 4) | (0 << 8) | (0 << 14));
            __builtin_amdgcn_s_barrier();
            asm volatile("" ::: "memory");
            run_stages<T, NCH>(lds, Lp, pad, NCH, K, K, 1, wave, NW, lane);
            __syncthreads();
            // the wave's physical columns (pa, pb) = (px, y_of(i)); a column's
            // line-aligned window [fbeg, fend) is the same for every dodecant
            const FrameMap f = d->fm[NDOD * grp + r];
#pragma unroll
            for (int i = 0; i < SPW; ++i) {
                const int pb = y_of(i);
                const int colo = (B * b1 + px) * N * N + (B * b2 + pb) * N + zb;
                const int mis = dsd > 0 ? (colo & 31) : ((colo + 1) & 31);
                auto line_floor = [&](int x) { return dsd > 0 ? x - ((mis + x) & 31) : x - ((x - mis) & 31); };
                const int fbeg = d0 <= 0 ? d0 : line_floor(d0);
                const int fend = last_tile ? d0 + T_ : line_floor(d0 + T_);
                const int cnt = fend - fbeg;
                const T* sl = lds + slot_offset(frame_slot(f, px, pb), Lp, pad) - d0;  // sl[dd]: displacement dd
#pragma unroll
                for (int c = 0; c < NCH + 1; ++c) {
                    const int k = 64 * c + lane;
                    const int dd = fbeg + k;
                    const T x = k < cnt && dd >= d0 ? sl[dd] : zero_of<T>();
                    acc[i][c] = r == 0 ? x : acc[i][c] + x;
                }
                const int tail = d0 + T_ - fend;
                const T t = !last_tile && lane < tail ? sl[fend + lane] : zero_of<T>();
                ncarry[i] = r == 0 ? t : ncarry[i] + t;
                if (r == NDOD - 1) {
                    // every dodecant is in: one line-aligned store of the sums
                    const int fl = fbeg + lane;
                    const int ob = 4 * colo + (dsd > 0 ? 4 * fl : -4 * fl);
#pragma unroll
                    for (int c = 0; c < NCH + 1; ++c) {
                        const int k = 64 * c + lane;
                        const int dd = fbeg + k;
                        if (k < cnt && (unsigned)dd < (unsigned)N) {
                            const T val = dd < d0 ? from_bits<T>(carry[i]) : acc[i][c];
                            bstore(rs_dst, ob + (dsd > 0 ? 256 * c : -256 * c), to_bits(val));
                        }
                    }
                    carry[i] = to_bits(ncarry[i]);
                }
            }
            __syncthreads();  // the LDS is free for the next dodecant
        }
    }
}

}  // namespace fast

// ---------------------------------------------------------------------------
// out[b][c][r] (+)= in[b][r][c]; 64 x 64 tiles through LDS, 256 threads.
template <typename T>
__global__ void __launch_bounds__(256)
transpose_kernel(const TransDesc* __restrict__ descs, int ndesc)
{
    __shared__ T tile[64][65];
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
    const T* src = reinterpret_cast<const T*>(d.in) + b * plane;
    T* dst = reinterpret_cast<T*>(d.out) + b * plane;
    const int c0 = tc * 64, r0 = tr * 64;
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
            dst[o] = d.add ? dst[o] + v : v;
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

// DJT pass: stages m0 .. m0+K-1 of eq. (15) fused. After them the plane of
// output slopes (s1 * 2^K + A, s2 * 2^K + B) and block V is
//   out[e1][e2] = sum_j c_j[e1 - s1*j - loc(j, A)][e2 - s2*j - loc(j, B)],
// c_j the input plane of block V*2^K + j. Stage t of the pass shifts the second
// half of each merged pair by its slope (the stage-t slope plus the new bit),
// so block j collects s*j from the slope bits the pass inherits and loc(j, A)
// from the bits it appends: every stage t with bit t of j set adds
// ceil((A >> (K-1-t)) / 2), at most 2^K - 1 in all. The inherited part is
// taken out by loading block j's tile at an origin lowered by s1*j rows and
// s2*j columns; inside the LDS tile only the local shifts remain.
template <int K>
__device__ __forceinline__ int djt_loc(int j, int A)
{
    int s = 0;
#pragma unroll
    for (int t = 0; t < K; ++t)
        if ((j >> t) & 1) s += ((A >> (K - 1 - t)) + 1) >> 1;
    return s;
}

// Rows of output per tile of a K-stage DJT pass: eight wavefronts each load
// four new input rows per tile (2^K planes x T1 rows in all).
constexpr int djt_rows_per_tile(int K) { return 32 >> K; }
// 64-column chunks of an LDS row (E_out + 2^K - 1 columns), one kernel per
// count; the largest takes N = 256.
constexpr int kDjtChunkCounts[] = {1, 2, 3, 5, 9};
// The adjoint's window rows hold E_out columns (its reads that matter stay
// below column E_out - 1), one kernel per count; the largest takes N = 256.
constexpr int kDjtAdjChunkCounts[] = {1, 2, 3, 4, 5, 8};

// NCC: 64-column chunks of an LDS row (E_out + 2^K - 1 columns); NCO: of an
// output row (E_out columns), NCC or NCC - 1.
template <typename T, int K, int NCC, int NCO>
__global__ void __launch_bounds__(512)
djt_pass_kernel(const DjtDesc* __restrict__ descs, int ndesc, long long total_wg)
{
    constexpr int NB = 1 << K, H = NB - 1, NO = NB * NB, NWV = 8;
    constexpr int T1 = djt_rows_per_tile(K), RPW = NB * T1 / NWV;
    constexpr int HPW = (NB * H + NWV - 1) / NWV;    // halo rows per wave
    constexpr int OPW = NO >= NWV ? NO / NWV : 1;    // output planes per wave
    constexpr int RSTEP = NO >= NWV ? 1 : NWV / NO;  // stride of its output rows
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* lds = reinterpret_cast<T*>(smem_raw);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (long long wg = blockIdx.x; wg < total_wg; wg += gridDim.x) {
        const DjtDesc* d = descs + find_desc_djt(descs, ndesc, wg);
        const long long local = wg - d->wg_begin;
        const int grp = (int)(local % d->groups);
        const int slot = (int)(local / d->groups);
        const int N = d->N, m0 = d->m0, P = d->P;
        const int Ein = d->E_in, Eout = d->E_out;
        const int Vout = N >> (m0 + K);
        const int V = grp % Vout;
        const int sl = grp / Vout;
        const int s1 = sl >> m0, s2 = sl & ((1 << m0) - 1);
        const int R = T1 + H;                 // LDS rows per plane
        const int cols_in = Eout + H;
        const bool fin = d->final_stage != 0;
        const int ntiles = d->ntiles;
        // final tiles past the support e1 <= N-1+s1 of every output slope of
        // the group are all zeros: no loads, no LDS
        const int nlive = fin ? min(ntiles, (N - 1 + s1 * NB + H) / T1 + 1) : ntiles;

        // input: the group's 2^K planes are consecutive in the stage buffer;
        // stage 0 reads the volume through the frame map. Out-of-range lanes
        // get an offset past the resource: the hardware returns 0.
        __amdgpu_buffer_rsrc_t rs_in;
        int ib, isx, isy, isd, Elim;
        if (d->src_mode == 0) {
            const long long pin = (long long)Ein * Ein;
            const T* base = reinterpret_cast<const T*>(d->src) + slot * d->src_slot_stride +
                            ((long long)sl * (N >> m0) + (long long)V * NB) * pin;
            rs_in = make_rsrc(base, (int)(NB * pin));
            ib = 0; isx = Ein; isy = 1; isd = (int)pin; Elim = Ein;
        } else {
            const FrameMap f = d->fm[slot];
            rs_in = make_rsrc(reinterpret_cast<const T*>(d->src), N * N * N);
            ib = f.base + f.sd * V * NB; isx = f.sx; isy = f.sy; isd = f.sd; Elim = N;
        }
        // output: the group's planes (t1, t2) = (s1*2^K + A, s2*2^K + B) lie
        // inside 2^K runs of 2^K planes, Sout planes apart
        const int Sout = 1 << (m0 + K);
        const int pout = Eout * Eout;
        const __amdgpu_buffer_rsrc_t rs_out = make_rsrc(
            reinterpret_cast<T*>(d->dst) + slot * d->dst_slot_stride +
                ((long long)(s1 * NB * Sout + s2 * NB) * Vout + V) * pout,
            ((H * Sout + NB - 1) * Vout + 1) * pout);
        const int o0 = wave % (NO >= NWV ? NWV : NO);
        const int r0w = NO >= NWV ? 0 : wave / NO;

        uint32_t v[RPW][NCC];
        // the T1 new rows of tile `tile`: LDS rows H..H+T1-1 of every plane
        auto issue = [&](int tile) {
#pragma unroll
            for (int i = 0; i < RPW; ++i) {
                const int q = wave + NWV * i;  // (plane j, new row r) = (q / T1, q % T1)
                const int j = q / T1, r = q % T1;
                const int e1 = tile * T1 - s1 * j + r;
                const bool rin = (unsigned)e1 < (unsigned)Elim;
                const int rowb = ib + isd * j + isx * e1;
#pragma unroll
                for (int t = 0; t < NCC; ++t) {
                    const int e2 = 64 * t + lane - s2 * j - H;
                    const bool in = rin && (unsigned)e2 < (unsigned)Elim;
                    v[i][t] = bload(rs_in, in ? 4 * (rowb + isy * e2) : -1);
                }
            }
        };
        if (nlive > 0) issue(0);
        for (int tile = 0; tile < ntiles; ++tile) {
            const int e1_0 = tile * T1;
            const int rows = min(T1, Eout - e1_0);
            const bool live = tile < nlive;
            if (live) {
                // halo: the previous tile's top H rows (zeros for the first)
                uint32_t h[HPW][NCC];
#pragma unroll
                for (int i = 0; i < HPW; ++i) {
                    const int q = wave + NWV * i;  // (plane, halo row) = (q / H, q % H)
#pragma unroll
                    for (int t = 0; t < NCC; ++t) {
                        const int c = 64 * t + lane;
                        h[i][t] = tile > 0 && q < NB * H && c < cols_in
                                      ? to_bits(lds[((q / H) * R + T1 + q % H) * P + c])
                                      : 0u;
                    }
                }
                __syncthreads();  // previous output phase and halo reads done
#pragma unroll
                for (int i = 0; i < HPW; ++i) {
                    const int q = wave + NWV * i;
#pragma unroll
                    for (int t = 0; t < NCC; ++t) {
                        const int c = 64 * t + lane;
                        if (q < NB * H && c < cols_in) lds[((q / H) * R + q % H) * P + c] = from_bits<T>(h[i][t]);
                    }
                }
#pragma unroll
                for (int i = 0; i < RPW; ++i) {
                    const int q = wave + NWV * i;
#pragma unroll
                    for (int t = 0; t < NCC; ++t) {
                        const int c = 64 * t + lane;
                        if (c < cols_in) lds[((q / T1) * R + H + q % T1) * P + c] = from_bits<T>(v[i][t]);
                    }
                }
                __syncthreads();
            }
            // outputs: each wave owns planes o = o0 + NWV * p and rows
            // r = r0 + RSTEP * i of the tile. The loop is unrolled with every
            // store unconditional (lanes past a row or past the last row get
            // an offset outside the resource), so the next tile's loads can be
            // issued half way through and waited for with the later half of
            // the stores still in flight.
            constexpr int RPWO = T1 / RSTEP;  // output rows per wave per plane
#pragma unroll
            for (int p = 0; p < OPW; ++p) {
                const int o = o0 + NWV * p;
                const int A = o >> K, B = o & H;
                const int t1 = s1 * NB + A;
                const int pb = (A * Sout + B) * Vout * pout;  // plane offset inside rs_out
                const int ccap = fin ? min(Eout, N + s2 * NB + B) : Eout;
                int lb[NB];
#pragma unroll
                for (int j = 0; j < NB; ++j) lb[j] = (j * R + H - djt_loc<K>(j, A)) * P + H - djt_loc<K>(j, B);
#pragma unroll
                for (int i = 0; i < RPWO; ++i) {
                    if (p * RPWO + i == (OPW * RPWO) / 2 && live && tile + 1 < nlive) issue(tile + 1);
                    const int r = r0w + RSTEP * i;
                    const int e1 = e1_0 + r;
                    // final output: rows past N-1+t1 and columns past N-1+t2 are zero
                    const int cmax = !live || r >= rows || (fin && e1 > N - 1 + t1) ? 0 : ccap;
                    const int ob = r < rows ? pb + e1 * Eout : -(1 << 30);
#pragma unroll
                    for (int t = 0; t < NCO; ++t) {
                        const int c = 64 * t + lane;
                        T x = zero_of<T>();
                        if (c < cmax) {
#pragma unroll
                            for (int j = 0; j < NB; ++j) x += lds[lb[j] + r * P + c];
                        }
                        bstore_cached(rs_out, c < Eout && ob >= 0 ? 4 * (ob + c) : -1, to_bits(x));
                    }
                }
            }
        }
        __syncthreads();  // the next work item reuses the LDS
    }
}

// ---------------------------------------------------------------------------
// DJT adjoint pass (Sec. 5.1, eq. (18) over K stages): the transpose of
// djt_pass_kernel for the same (m0, K). The forward writes out_{A,B}[e] = sum_j in_j[e - s*j - loc(j, .)]; its
// transpose gathers, for e on the forward's output grid,
//   in_j[e - s*j] = sum_{A,B} out_{A,B}[e + loc(j, A), e2 + loc(j, B)],
// so the 4^K output planes are read on one aligned window per tile (no skew)
// and every input row x = e - s1*j is produced whole by the one tile holding
// e. Reading those planes is the pass's whole cost (the last pass reads the
// full projection set), so they stream through a ring of three LDS windows
// filled by direct-to-LDS buffer loads two planes ahead of the one being
// summed: the loads in flight hold no registers, and each plane costs one
// barrier. Each thread accumulates its 2^K x (rows) x (chunks) sums.
constexpr int kDjtAdjRows = 16;  // forward-output rows e per adjoint tile
// LDS ring of one adjoint work group: three windows of (T1 + H) rows at a
// pitch of whole 64-column chunks covering E_out (every lane of a direct load
// lands inside its row; the sums that are written read below column E_out,
// the others may read into the next row), plus room past each for the
// discarded reads of shifted chunks and for the loads of rows a wave does
// not own
template <int K, int NCC>
constexpr int djt_adj_window() { return (kDjtAdjRows + (1 << K) - 1) * 64 * NCC + 128; }

template <int VMCNT>
__device__ __forceinline__ void wait_vm_lds_then_barrier()
{
    // this wave's loads older than the newest VMCNT have landed, its LDS reads
    // are done; then every wave of the group has reached the same point
    static_assert(VMCNT >= 0 && VMCNT < 64, "vmcnt field");
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt((VMCNT & 15) | (7 << 4) | (0 << 8) | ((VMCNT >> 4) << 14));
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

template <typename T, int K, int NCC>
__global__ void __launch_bounds__(512)
djt_adj_kernel(const DjtDesc* __restrict__ descs, int ndesc, long long total_wg)
{
    constexpr int NB = 1 << K, H = NB - 1, NO = NB * NB, NWV = 8;
    constexpr int T1 = kDjtAdjRows, RW = T1 / NWV;  // output-grid rows per wave
    constexpr int WROWS = T1 + H;                   // window rows
    constexpr int WR = (WROWS + NWV - 1) / NWV;     // window rows loaded per wave
    constexpr int WP = 64 * NCC;                    // LDS row pitch
    constexpr int WSZ = djt_adj_window<K, NCC>();
    constexpr int LPP = WR * NCC;                   // direct loads per wave per plane
    static_assert(2 * LPP < 64, "two planes in flight fit the vmcnt field");
    typedef __attribute__((address_space(3))) void lds_void;
    __shared__ __align__(16) uint32_t win0[WSZ];
    __shared__ __align__(16) uint32_t win1[WSZ];
    __shared__ __align__(16) uint32_t win2[WSZ];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (long long wg = blockIdx.x; wg < total_wg; wg += gridDim.x) {
        const DjtDesc* d = descs + find_desc_djt(descs, ndesc, wg);
        long long local = wg - d->wg_begin;
        // work groups go to the XCDs round robin: eight (slot, group) pairs
        // share each run of 8 x ntiles work groups, so the tiles of one pair
        // (which overlap by H rows) are read through the same L2
        const long long pairs = (long long)d->nslots * d->groups;
        int tile;
        if ((pairs & 7) == 0) {
            const long long run = local / (8LL * d->ntiles);
            const long long in_run = local - run * 8LL * d->ntiles;
            tile = (int)(in_run >> 3);
            local = run * 8 + (in_run & 7);
        } else {
            tile = (int)(local % d->ntiles);
            local /= d->ntiles;
        }
        const int grp = (int)(local % d->groups);
        const int slot = (int)(local / d->groups);
        const int N = d->N, m0 = d->m0;
        const int Ein = d->E_in, Eout = d->E_out;
        const int Vout = N >> (m0 + K);
        const int V = grp % Vout;
        const int sl = grp / Vout;
        const int s1 = sl >> m0, s2 = sl & ((1 << m0) - 1);
        const int e0 = tile * T1;
        const int Sout = 1 << (m0 + K);
        const int pout = Eout * Eout;
        const bool fin = d->final_stage != 0;
        // the group's output planes (t1, t2) = (s1*2^K + A, s2*2^K + B)
        const __amdgpu_buffer_rsrc_t rs_in = make_rsrc(
            reinterpret_cast<const T*>(d->src) + slot * d->src_slot_stride +
                ((long long)(s1 * NB * Sout + s2 * NB) * Vout + V) * pout,
            ((H * Sout + NB - 1) * Vout + 1) * pout);
        // final: forward-output rows past N-1+t1 and columns past N-1+t2 are
        // outside every line's support (no voxel reaches them): they are not
        // read. A window past the support of every plane of the group
        // contributes nothing.
        const bool zero_tile = fin && e0 > N - 1 + s1 * NB + H;

        T acc[NB][RW][NCC];
#pragma unroll
        for (int j = 0; j < NB; ++j)
#pragma unroll
            for (int i = 0; i < RW; ++i)
#pragma unroll
                for (int t = 0; t < NCC; ++t) acc[j][i][t] = zero_of<T>();

        if (!zero_tile) {
            // window rows [e0, e0 + T1 + H) of plane o into W; loads outside
            // the plane (or its support) get an offset past the resource and
            // land as zeros. A wave's rows past the window load into the spare
            // room after it, so every wave issues LPP loads per plane.
            auto issue = [&](uint32_t* W, int o) __attribute__((always_inline)) {
                const int A = o >> K, B = o & H;
                const int pb = (A * Sout + B) * Vout * pout;
                const int ccap = fin ? min(Eout, N + s2 * NB + B) : Eout;
#pragma unroll
                for (int i = 0; i < WR; ++i) {
                    const int r = wave + NWV * i;
                    const int e1 = e0 + r;
                    const bool real = r < WROWS;
                    const bool rin = real && e1 < Eout && !(fin && e1 > N - 1 + s1 * NB + A);
#pragma unroll
                    for (int t = 0; t < NCC; ++t) {
                        const int c = 64 * t + lane;
                        const int off = rin && c < ccap ? 4 * (pb + e1 * Eout + c) : -1;
                        uint32_t* dst = real ? W + r * WP + 64 * t : W + WROWS * WP;
                        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs_in, (lds_void*)dst, 4, off, 0, 0, 0);
                    }
                }
            };
            auto sum_plane = [&](const uint32_t* W, int o) __attribute__((always_inline)) {
                const int A = o >> K, B = o & H;
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    const int lj = djt_loc<K>(j, A) * WP + djt_loc<K>(j, B);
#pragma unroll
                    for (int i = 0; i < RW; ++i) {
                        const int r = wave + NWV * i;
#pragma unroll
                        for (int t = 0; t < NCC; ++t)
                            acc[j][i][t] += from_bits<T>(W[lj + r * WP + 64 * t + lane]);
                    }
                }
            };
            // plane o lives in window o % 3; plane o + 2 is issued into the
            // window that plane o - 1 used, once every wave is past it
            auto step = [&](int o, uint32_t* cur, uint32_t* nxt) __attribute__((always_inline)) {
                if (o + 1 < NO) wait_vm_lds_then_barrier<LPP>();  // plane o + 1 may stay in flight
                else wait_vm_lds_then_barrier<0>();
                if (o + 2 < NO) issue(nxt, o + 2);
                sum_plane(cur, o);
            };
            issue(win0, 0);
            issue(win1, 1);
            for (int o = 0; o < NO; o += 3) {
                step(o, win0, win2);
                if (o + 1 < NO) step(o + 1, win1, win0);
                if (o + 2 < NO) step(o + 2, win2, win1);
            }
            wait_vm_lds_then_barrier<0>();  // the next work item refills the ring
        }
        // write in_j row x1 = e - s1*j, columns x2 = e2 - s2*j, inside E_in
        T* dst = reinterpret_cast<T*>(d->dst);
        const FrameMap f = d->fm[slot];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int u = V * NB + j;  // block index of plane j at stage m0
#pragma unroll
            for (int i = 0; i < RW; ++i) {
                const int x1 = e0 + wave + NWV * i - s1 * j;
                if ((unsigned)x1 >= (unsigned)Ein) continue;
#pragma unroll
                for (int t = 0; t < NCC; ++t) {
                    const int x2 = 64 * t + lane - s2 * j;
                    if ((unsigned)x2 >= (unsigned)Ein) continue;
                    if (d->dst_mode == 0) {
                        const long long pin = (long long)Ein * Ein;
                        dst[slot * d->dst_slot_stride + ((long long)sl * (N >> m0) + u) * pin +
                            (long long)x1 * Ein + x2] = acc[j][i][t];
                    } else {
                        // stage 0: block u is the volume slice at driving
                        // coordinate u; this dodecant's own volume
                        dst[slot * d->dst_slot_stride + f.base + (long long)f.sd * u + (long long)f.sx * x1 +
                            (long long)f.sy * x2] = acc[j][i][t];
                    }
                }
            }
        }
    }
}

// out[i] = (accum ? out[i] : 0) + sum of the parts at i
template <typename T>
__global__ void __launch_bounds__(256)
sum_parts_kernel(const T* __restrict__ parts, int nparts, T* __restrict__ out, long long n, int accum)
{
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        T s = accum ? out[i] : zero_of<T>();
        for (int p = 0; p < nparts; ++p) s += parts[p * n + i];
        out[i] = s;
    }
}

}  // namespace drt3d
