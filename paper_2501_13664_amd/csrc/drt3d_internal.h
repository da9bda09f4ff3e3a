// Internal declarations shared by the device code and the host runtime of the
// drt3d library. Not part of the public interface (include/drt3d.h).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace drt3d {

// Affine element offset of a frame view of an N^3 volume:
//   offset = base + sx * a + sy * b + sd * c.
// DRT: (a, b, c) = (x', y', N-1-z'), the stage-0 column in displacement
// orientation; DJT: (a, b, c) = (N-1-x', N-1-y', z'), the plane in intercept
// orientation and the driving coordinate.
// N <= 1024 keeps every term inside int32.
struct FrameMap {
    int base, sx, sy, sd;
    int group;  // volume layout the map addresses (DRT: 0 z-, 1 y-, 2 x-normal)
};

constexpr int kMaxSlots = 12;

// One DRT pass: the x-stages mx0..mx0+Kx-1 (slope s1) and the y-stages
// my0..my0+Ky-1 (slope s2) of eq. (11), forward or adjoint (eq. (17)), for
// every column group of every dodecant slot. A group is the 2^Kx x 2^Ky
// columns that exchange data in these stages. Work items are
// (slot, group, displacement tile) flattened; `wg_begin` is the first
// flattened index of this descriptor inside its launch.
struct DrtDesc {
    long long wg_begin;
    long long src_slot_stride, dst_slot_stride;  // elements between slots
    const void* src;                             // stage buffer (src_mode 0)
    void* dst;                                   // stage buffer (dst_mode 0)
    const void* vsrc[3];                         // volume layouts (src_mode 1)
    void* vdst[3];                               // volume accumulators (dst_mode 1)
    int groups_x, groups_y, ntiles, nslots;
    int N, n;
    int mx0, Kx, my0, Ky;
    int E_in, P_in, E_out, P_out;
    int T, H, L, Lp;       // tile width, local halo, LDS column length and pitch
    int src_mode, dst_mode, adjoint, nt_store;
    // > 0: the slots form runs of xcd_run dodecants that read the same volume
    // layout; work items are ordered so that the run's dodecants take the
    // same original column block in work groups 8 apart (same XCD, close in
    // time), sharing its loads through that XCD's L2
    int xcd_run;
    int sb, db;            // bytes per element of the source and destination in HBM (4, or narrow storage)
    // adjoint's last pass, one work item per volume layout group and block:
    // slots 4g .. 4g+3 are group g's four dodecants (drt_adj_last_group)
    int fused_group;
    // float forward's last pass only: when set, it writes sub - result (the
    // same layout as the output, e.g. the inverse's residual b - A x)
    const void* sub;
    int phys[kMaxSlots];   // slot -> slot index inside the source (stage buffer or projections)
    int dphys[kMaxSlots];  // slot -> slot index inside the destination (dst_mode 0)
    int accum[kMaxSlots];  // dst_mode 1: add into the volume (1) or overwrite (0)
    FrameMap fm[kMaxSlots];
};

// One DJT pass: stages m0 .. m0+K-1 of eq. (15) fused, for every group of
// every dodecant slot. A group is a slope pair (s1, s2) of stage m0 and the
// 2^K blocks it merges into one block V of stage m0+K; it reads 2^K planes and
// writes 4^K. Planes are E x E, row-major in (e1, e2); buffers are
// [s1 * 2^m + s2][block][e1][e2] (the final output: [s1][s2][e1][e2]). Work
// items are (slot, group) flattened; each runs over its tiles of T1 output
// rows in order.
struct DjtDesc {
    long long wg_begin;
    long long src_slot_stride, dst_slot_stride;  // elements between slots
    const void* src;  // stage buffer, or the volume when src_mode == 1
    void* dst;
    int groups, ntiles, T1, nslots;
    int N, n, m0, K;
    int E_in, E_out;  // plane extents before and after the pass
    int P;            // LDS row pitch (>= E_out + 2^K - 1)
    int src_mode;
    int final_stage;  // output is the caller's buffer: zero tails skipped, streamed past the caches
    // adjoint passes (djt_adj_kernel) run a forward pass's transpose: they read
    // `src` = that pass's outputs (the caller's projections when final_stage)
    // and write `dst` = its inputs (per-dodecant volumes when dst_mode == 1)
    int dst_mode;
    FrameMap fm[kMaxSlots];
};

// out[i] = (accum ? out[i] : 0) + sum over s < nparts of parts[s * n + i]
// (the per-dodecant volumes of the DJT adjoint)
hipError_t launch_sum_parts(int is_float, const void* parts, int nparts, void* out, long long n, int accum,
                            hipStream_t s);

// One transpose out[b][c][r] (+)= in[b][r][c], b < batches, r < R, c < C, in
// 64 x 64 tiles; work items are (b, tile row, tile column) flattened, from
// `wg_begin` inside the launch.
struct TransDesc {
    long long wg_begin;
    const void* in;
    void* out;
    int R, C, batches, add;
    int tiles_r, tiles_c;
};

// Launchers (device code translation unit).
hipError_t launch_drt_pass(int is_float, const DrtDesc* d_descs, int ndesc, long long total_wg,
                           int block, int grid, size_t lds_bytes, hipStream_t s);
// Output rows per tile of a K-stage DJT pass, and the 64-column chunk count
// of the kernel that takes LDS rows of `cols` columns (0: none does).
int djt_tile_rows(int K);
int djt_adj_tile_rows();  // forward-output rows per DJT adjoint tile
size_t djt_adj_lds_bytes(int K, int ncc);  // static LDS of one DJT adjoint work group
int djt_chunks_for(int cols);
int djt_adj_chunks_for(int cols);  // the adjoint's: rows of cols = E_out columns
hipError_t launch_djt_pass(int is_float, int K, int ncc, int nco, const DjtDesc* d_descs, int ndesc,
                           long long total_wg, int grid, size_t lds_bytes, hipStream_t s);
hipError_t launch_transpose(int is_float, const TransDesc* d_descs, int ndesc, long long total_wg,
                            hipStream_t s);
hipError_t set_drt_lds_limit(int is_float, size_t bytes);
// Kernel handles of the shape-specialised DRT passes (one translation unit
// per shape) and of the DJT passes.
const void* drt_fast_kernel_3_3(int is_float, int nch, int mode, int waves);
const void* drt_fast_kernel_2_2(int is_float, int nch, int mode, int waves);
const void* drt_fast_kernel_3_2(int is_float, int nch, int mode, int waves);
const void* drt_fast_kernel_2_3(int is_float, int nch, int mode, int waves);
// the same passes over narrow storage (see drt_pass_fast's SB, DB)
const void* drt_fast_kernel_narrow_3_3(int nch, int mode, int sb, int db);
const void* drt_fast_kernel_narrow_2_2(int nch, int mode, int sb, int db);
const void* drt_fast_kernel_narrow_3_2(int nch, int mode, int sb, int db);
const void* drt_fast_kernel_narrow_2_3(int nch, int mode, int sb, int db);
const void* djt_pass_kernel_ptr(int is_float, int K, int ncc, int nco);
const void* djt_adj_kernel_ptr(int is_float, int K, int ncc);
hipError_t launch_djt_adj(int is_float, int K, int ncc, const DjtDesc* d_descs, int ndesc, long long total_wg,
                          int grid, size_t lds_bytes, hipStream_t s);
// Shape-specialised DRT pass kernels (eight wavefronts per work group).
// mode: 0 forward into a stage buffer, 1 the forward's last pass (every
// descriptor writes the caller's output), 2 adjoint.
// sb, db: bytes per element of the pass's source and destination (4 unless
// the call is over narrow storage).
int drt_fast_available(int kx, int ky, int nch, int waves, int mode = 0, int sb = 4, int db = 4);
hipError_t launch_drt_fast(int is_float, int kx, int ky, int nch, int mode, int waves, const DrtDesc* d_descs,
                           int ndesc, long long total_wg, int grid, size_t lds_bytes, hipStream_t s, int sb = 4,
                           int db = 4);
// wide: 128 x 128 tiles moved as 4-byte words (every R, C and base a multiple
// of 4, no accumulation); else the element-wise 64 x 64 kernel
hipError_t launch_transpose_u8(const TransDesc* d_descs, int ndesc, long long total_wg, int wide, hipStream_t s);
// The adjoint's last pass fused over layout groups (square K.K passes, K = 2
// or 3; eight wavefronts, or sixteen for 3.3).
const void* drt_adj_group_kernel_3_3(int is_float, int nch, int waves);
const void* drt_adj_group_kernel_2_2(int is_float, int nch, int waves);
const void* drt_adj_group_kernel(int is_float, int K, int nch, int waves);
// reference stream: read read_bytes of src, write write_bytes of dst (16-byte multiples)
hipError_t launch_stream_probe(const void* src, size_t read_bytes, void* dst, size_t write_bytes, int cus,
                               hipStream_t s);
hipError_t launch_drt_adj_group(int is_float, int K, int nch, int waves, const DrtDesc* d_descs, int ndesc,
                                long long total_wg, int grid, size_t lds_bytes, hipStream_t s);

// Iterative inverse (float32): filter, residual, restriction, prolongation,
// and the vector steps of the power iteration.
hipError_t launch_hp_filter(const float* y, float* out, int N, float c, int accumulate, hipStream_t s);
hipError_t launch_residual(const float* b, const float* ax, float* r, long long n, hipStream_t s);
hipError_t launch_restrict(const float* R, float* Rc, int N, hipStream_t s);
hipError_t launch_prolong_add(const float* e, float* x, int N, hipStream_t s);
hipError_t launch_base_mean(const float* b12, float* x1, hipStream_t s);
hipError_t launch_fill(float* p, float v, long long n, hipStream_t s);
hipError_t launch_power_start(float* v, int N, hipStream_t s);
size_t norm_scratch_bytes();
// scratch[norm_scratch_bytes()]: ends holding |w| (a double) at its last slot
hipError_t launch_normalize(const float* w, float* v, long long n, double* scratch, hipStream_t s);
// Algorithm 2's merged 4N x 4N x (3N-2) net from the 12-dodecant output.
hipError_t launch_merge_net(int is_float, const void* R, void* net, int N, hipStream_t s);

// Plane detection (Sec. 6.1). For the output's dodecant rank j, ks[j] is the
// dodecant; for dodecant k and original axis i (x, y, z), axis[k][i] is the
// primed axis that runs along it and sign[k][i] is -1 where it is mirrored.
struct PlaneFrames {
    int ks[12];
    signed char axis[12][3];
    signed char sign[12][3];
};
int argmax_parts(long long n);
// pv[nparts] (4-byte values), pi[nparts]: partials; top[0] = the largest
// element's index (ties: the smallest), thr[0] = rel * its value, bins[0] = top
hipError_t launch_argmax(int is_float, const void* p, long long n, void* pv, long long* pi, int nparts, double rel,
                         long long* top, double* thr, long long* bins, hipStream_t s);
hipError_t launch_plane_peaks(int is_float, int write, const void* p, int N, int nk, const PlaneFrames& F,
                              const long long* top, const double* thr, double tol2, int* counts,
                              const long long* offsets, long long* bins, long long cap, hipStream_t s);
long long scan_chunks(long long m);
// offsets[i] = counts[0] + ... + counts[i-1]; count[0] = 1 + the total;
// csum: scan_chunks(m) int64 of scratch
hipError_t launch_peak_scan(const int* counts, long long m, long long* offsets, long long* csum, long long* count,
                            hipStream_t s);
hipError_t launch_scatter_ones(const long long* bins, const long long* count, long long cap, uint32_t* marker,
                               long long n, uint32_t one, hipStream_t s);

}  // namespace drt3d
