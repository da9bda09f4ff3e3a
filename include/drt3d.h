/*
 * drt3d.h — C ABI of the MI355X (gfx950) library for the 3D multiscale discrete
 * Radon transform of planes (DRT), the 3D discrete John transform of lines (DJT)
 * and their adjoints, after Marichal-Hernandez et al., "Three-dimensional
 * multiscale discrete Radon and John transforms" (arXiv 2501.13664).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Volume: N x N x N, N = 2^n with 2 <= N <= DRT3D_MAX_N, C order [x][y][z]
 *   (z fastest), device memory owned by the caller. Inputs are never modified.
 * Dodecants: bit k of `mask` (k = 0..11) selects dodecant k, the input seen
 *   through row k of the InOrder table of Algorithm 2 (Sec. 3.2), read as:
 *   mirror every original axis |o_j| with o_j < 0, then send original axis i to
 *   primed axis |o_i|. Under this reading the 12 frames tile the hemisphere of
 *   plane normals (Sec. 3.2) and of line directions (Sec. 4.1). Outputs hold the
 *   selected dodecants in increasing k. DRT3D_ALL selects all twelve.
 * DRT output (Sec. 3.1, eq. (9)): [popcount(mask)][N][N][3N-2], element
 *   [j][s1][s2][dd] = sum over x',y' of g_k(x', y', l_{s1}(x') + l_{s2}(y') + N-1-dd),
 *   with l the discrete line of eq. (4) and g_k the frame-k view of the volume;
 *   dd = N-1-d mirrors the displacement d of eq. (9), so the non-null values of
 *   slope pair (s1,s2) occupy dd = 0..N-1+s1+s2 (Sec. 3.2). Zero tails are written.
 * DJT output (Sec. 4.1, eq. (13)): [popcount(mask)][N][N][2N-1][2N-1], element
 *   [j][s1][s2][e1][e2] = sum over u of g_k(l_{s1}(u)+N-1-e1, l_{s2}(u)+N-1-e2, u):
 *   lines driven along z' with slopes (s1,s2) over (x',y'); e = N-1-d.
 * Adjoints (Sec. 5.1, eqs. (16)-(18)): vol_out[x][y][z] = sum over the
 *   selected dodecants and all slope pairs of the DRT (DJT) value of the one
 *   plane (line) through the voxel; the exact transpose of drt3d_forward
 *   (djt3d_forward), no normalisation.
 * Arithmetic: DRT3D_I32 is int32 with two's-complement wrap (results are exact
 *   modulo 2^32, bit-identical to any exact summation order); DRT3D_F32 is
 *   float32 accumulation in the paper's recursion order.
 * Workspace: device memory of at least the size returned by the matching
 *   *_workspace_bytes query, owned by the caller, 256-byte aligned; its contents
 *   need not be initialised and are clobbered. Calls that share a workspace must
 *   not overlap in time.
 * Streams: every call is stream-ordered and asynchronous on `stream` (a
 *   hipStream_t; NULL = the default stream). Errors in argument validation are
 *   reported before any GPU work is queued.
 * Errors: functions return DRT3D_OK (0) or a negative status; the message of the
 *   last failure on the calling thread is available from drt3d_last_error().
 *   No C++ exception crosses this interface.
 * Alignment: vol/out/proj/workspace pointers must be 16-byte aligned.
 */
#ifndef DRT3D_H
#define DRT3D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DRT3D_ABI_VERSION 1
/* Largest N any entry point accepts. Every kernel addresses a dodecant's output
 * region, a stage buffer slot and the volume with 32-bit byte offsets, which
 * hold up to N = 512 (a 512^3 int32 volume is 2^29 bytes, a dodecant of the
 * DRT output 1.6 GB); larger N is rejected with DRT3D_EINVAL. */
#define DRT3D_MAX_N 512
#define DRT3D_ALL 0xFFFu

typedef enum {
    DRT3D_I32 = 0, /* int32 in, int32 out, wrap-around arithmetic */
    DRT3D_F32 = 1, /* float32 in, float32 out */
    DRT3D_U8 = 2   /* uint8 volume in, int32 out (drt3d_forward only, N >= 32): the
                      int32 transform of the same values, bit for bit */
} drt3d_dtype;

typedef enum {
    DRT3D_OK = 0,
    DRT3D_EINVAL = -1,      /* bad argument: N, mask, null or misaligned pointer, dtype, count */
    DRT3D_ENOMEM = -2,      /* workspace smaller than the query, or a host allocation failed */
    DRT3D_EHIP = -3,        /* a HIP runtime call failed (message names it) */
    DRT3D_EUNSUPPORTED = -4 /* no gfx950 device, or a feature not built */
} drt3d_status;

/* Message of the last failure on the calling thread ("" if none). */
const char* drt3d_last_error(void);
int drt3d_abi_version(void);

/* ---- size queries (host only, pure) ------------------------------------ */
/* Elements of the DRT output: popcount(mask) * N * N * (3N-2); 0 if invalid. */
size_t drt3d_out_elems(int N, uint32_t mask);
/* Elements of the DJT output: popcount(mask) * N * N * (2N-1)^2; 0 if invalid. */
size_t djt3d_out_elems(int N, uint32_t mask);
/* Workspace bytes for drt3d_forward / djt3d_forward / drt3d_adjoint /
 * djt3d_adjoint (any tuning choice fits). 0 if the arguments are invalid. */
size_t drt3d_workspace_bytes(int N, uint32_t mask, int dtype);
size_t djt3d_workspace_bytes(int N, uint32_t mask, int dtype);
size_t drt3d_adjoint_workspace_bytes(int N, uint32_t mask, int dtype);
size_t djt3d_adjoint_workspace_bytes(int N, uint32_t mask, int dtype);
/* Workspace bytes for the batched variants over `count` volumes of sizes Ns[]. */
size_t drt3d_forward_batched_workspace_bytes(int count, const int* Ns, uint32_t mask, int dtype);
size_t djt3d_forward_batched_workspace_bytes(int count, const int* Ns, uint32_t mask, int dtype);
size_t drt3d_adjoint_batched_workspace_bytes(int count, const int* Ns, uint32_t mask, int dtype);
size_t djt3d_adjoint_batched_workspace_bytes(int count, const int* Ns, uint32_t mask, int dtype);

/* ---- transforms ----------------------------------------------------------- */
/* 3D DRT of planes, Algorithm 1 (stage map eq. (11)) over the dodecants of
 * `mask` (Algorithm 2's input frames). vol: [N][N][N] of dtype; out:
 * drt3d_out_elems(N, mask) elements of dtype (int32 for DRT3D_U8), fully
 * overwritten. DRT3D_U8 keeps the data narrow in HBM where it fits (Sec. 6
 * points at 8-bit data): the volume and its frame copies at 1 byte, the first
 * pass's partial sums (at most 2^6 voxels of 0..255) at 2 bytes, the rest at 4,
 * with 32-bit adds throughout (the first pass adds two column groups at once,
 * packed in the 16-bit halves of each word); it needs a tuning whose passes all have
 * shape-specialised kernels (the built-in ones for N = 32..512), else
 * DRT3D_EUNSUPPORTED. */
int drt3d_forward(const void* vol, void* out, int N, uint32_t mask, int dtype,
                  void* workspace, size_t workspace_bytes, void* stream);

/* drt3d_forward for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc. The
 * call allocates nothing (no hipMalloc or hipFree, no pinned host memory, no
 * allocating library routine): its workspace is a static device array of
 * 64 MiB that the library holds on every GPU it runs on until the process
 * ends, and the launch descriptors reach that array as kernel arguments. The
 * caller passes the volume and the output as for drt3d_forward (same layouts
 * and dtypes, bit-identical results).
 * Limit: drt3d_workspace_bytes(N, mask, dtype) <= 64 MiB, i.e. N <= 64 for all
 * 12 dodecants; larger requests return DRT3D_EINVAL before any device work.
 * Every call on one GPU uses that GPU's single array, which keeps the last
 * call's contents: calls that overlap in time on one GPU (on different streams,
 * or from several host threads) race on it and give undefined results, so
 * order them, e.g. on one stream. */
int drt3d_forward_noalloc(const void* vol, void* out, int N, uint32_t mask, int dtype, void* stream);

/* 3D DJT of lines, Algorithm 3 (stage map eq. (15)), driving axis z', over the
 * dodecants of `mask`. out: djt3d_out_elems(N, mask) elements, overwritten.
 * N <= 256 (DRT3D_EUNSUPPORTED above: the output alone is 48 GiB at N = 256). */
int djt3d_forward(const void* vol, void* out, int N, uint32_t mask, int dtype,
                  void* workspace, size_t workspace_bytes, void* stream);

/* DRT adjoint (backprojection), Algorithm 1 reversed with eq. (17) (Sec. 5.1),
 * summed over the dodecants of `mask`. proj: the drt3d_forward layout for the
 * same (N, mask); vol_out: [N][N][N], overwritten. */
int drt3d_adjoint(const void* proj, void* vol_out, int N, uint32_t mask, int dtype,
                  void* workspace, size_t workspace_bytes, void* stream);

/* DJT adjoint (backprojection of lines), Alg. 3 reversed with eq. (18)
 * (Sec. 5.1), summed over the dodecants of `mask`: the exact transpose of
 * djt3d_forward for the same (N, mask), i.e. of eq. (13), with no
 * normalisation. vol_out[x][y][z] = sum over the selected dodecants and slope
 * pairs of the DJT value of the one line through the voxel that is driven along
 * z' with those slopes. proj: the djt3d_forward layout; entries outside the
 * support e <= N-1+s of a slope lie on no line through the cube and are
 * ignored. vol_out: [N][N][N], overwritten. N <= 256. */
int djt3d_adjoint(const void* proj, void* vol_out, int N, uint32_t mask, int dtype,
                  void* workspace, size_t workspace_bytes, void* stream);

/* ---- batched variants ----------------------------------------------------- */
/* `count` independent transforms of possibly different N in one set of
 * persistent launches (one per pass slot), replayed from a cached hipGraph
 * when the same shapes, mask, dtype and workspace recur. vols/outs (device
 * pointers) and Ns live in host memory; every volume uses the same mask and
 * dtype. Results are bit-identical to the single-volume calls. */
int drt3d_forward_batched(int count, const void* const* vols, void* const* outs,
                          const int* Ns, uint32_t mask, int dtype,
                          void* workspace, size_t workspace_bytes, void* stream);
int djt3d_forward_batched(int count, const void* const* vols, void* const* outs,
                          const int* Ns, uint32_t mask, int dtype,
                          void* workspace, size_t workspace_bytes, void* stream);
int drt3d_adjoint_batched(int count, const void* const* projs, void* const* vols_out,
                          const int* Ns, uint32_t mask, int dtype,
                          void* workspace, size_t workspace_bytes, void* stream);
int djt3d_adjoint_batched(int count, const void* const* projs, void* const* vols_out,
                          const int* Ns, uint32_t mask, int dtype,
                          void* workspace, size_t workspace_bytes, void* stream);

/* ---- merged output (Algorithm 2) ---------------------------------------------- */
/* Elements of the merged net: 16 * N * N * (3N-2); 0 if N is invalid. */
size_t drt3d_net_elems(int N);
/* Algorithm 2's global output (Sec. 3.2): each of the 12 dodecants' outputs
 * (proj: the drt3d_forward layout for DRT3D_ALL) is rotated by its OutOrder row
 * (axes (s1, s2) permuted by |OutOrder|, then each axis with a negative entry
 * flipped; dd is never moved) and placed at block DodecantCoords(k) of the
 * net [4N][4N][3N-2]: net[bi*N + i][bj*N + j][dd]. The four corner blocks, which
 * no dodecant fills, are written as zeros; net is fully overwritten. A layout
 * transform on the GPU (one read of proj, one write of net); the net is not
 * claimed to be continuous across block edges. */
int drt3d_merge_net(const void* proj, void* net, int N, int dtype, void* stream);

/* ---- plane detection (Sec. 6.1) ------------------------------------------------ */
/* The application of Sec. 6.1 on a DRT output proj ([count][N][N][3N-2] in the
 * drt3d_forward layout of mask, int32 or float32, device memory):
 *   1. the dominant plane is the largest bin (ties: the smallest flat index;
 *      int32 compares as signed; NaN inputs are not supported);
 *   2. a bin (j, s1, s2, dd) qualifies when its plane is orthogonal to the
 *      dominant one, |cos| <= cos_tol between the integer normals of
 *      drt3d_plane_normal, decided as (a.b)^2 <= cos_tol^2 |a|^2 |b|^2 in
 *      float64; it is a relative maximum of its dodecant's output: over the
 *      26 neighbours (s1+a, s2+b, dd+c) that exist, those earlier in the layout
 *      are strictly below it and those later are not above it; and its value is
 *      >= rel_threshold x the dominant value, in float64.
 * bins (device, cap >= 1 entries of int64): bins[0] = the dominant bin's flat
 * index, then the qualifying bins' flat indices in ascending order, as many as
 * fit. count (device, one int64) = 1 + the number of qualifying bins, which may
 * exceed cap. cos_tol in [0, 1). Stream-ordered, no host synchronisation.
 * Workspace: drt3d_detect_planes_workspace_bytes(N, mask, dtype), 256-byte
 * aligned (about 12 bytes per output column). */
size_t drt3d_detect_planes_workspace_bytes(int N, uint32_t mask, int dtype);
int drt3d_detect_planes(const void* proj, int N, uint32_t mask, int dtype, double cos_tol, double rel_threshold,
                        long long* bins, long long cap, long long* count, void* workspace, size_t workspace_bytes,
                        void* stream);
/* vol_out ([N][N][N], dtype, overwritten) = the adjoint (drt3d_adjoint) of the
 * projection holding 1 at each of the first min(count[0], cap) flat indices of
 * bins (device memory, as drt3d_detect_planes writes them) and 0 elsewhere:
 * per voxel, the number of listed planes through it. Indices outside the
 * output are skipped. Workspace: drt3d_backproject_bins_workspace_bytes
 * (a 0/1 projection of 4 bytes per bin plus the adjoint's workspace). */
size_t drt3d_backproject_bins_workspace_bytes(int N, uint32_t mask, int dtype);
int drt3d_backproject_bins(const long long* bins, const long long* count, long long cap, void* vol_out, int N,
                           uint32_t mask, int dtype, void* workspace, size_t workspace_bytes, void* stream);
/* Integer normal (x, y, z) of dodecant k's planes at slopes (s1, s2), scaled by
 * N-1: in the dodecant's frame the planes z' = s1 x'/(N-1) + s2 y'/(N-1) + d
 * (up to the discrete lines) have the normal (-s1, -s2, N-1) (Sec. 3); the
 * frame table of drt3d_frame_map carries it to the original axes. Host only. */
int drt3d_plane_normal(int k, int s1, int s2, int N, int out[3]);

/* ---- inverse ---------------------------------------------------------------- */
/* Iterative inverse of the 12-dodecant DRT (Sec. 5.2), float32 only: given
 * proj = drt3d_forward(f) for all 12 dodecants ([12][N][N][3N-2] float32),
 * vol_out ([N][N][N] float32, overwritten) approaches f over the cycles.
 * The scheme is Press's iterative improvement with the approximate inverse
 * H A^T, H the 3x3x3 high-pass filter of Sec. 5.2 (borders reflected), run in
 * multigrid V-cycles with the restriction S (Radon domain) and prolongation P
 * (image domain) of Sec. 5.2. Each size smooths with three step sizes (the
 * Chebyshev nodes of [L/10, L], L = 1.02 x the largest eigenvalue of
 * H A^T A at that size) before and after its coarse correction; size 1 takes
 * the mean of its 12 values. cycles = 0 writes zeros.
 * lams: NULL, or the eigenvalues for sizes 2, 4, ..., N (log2 N values), as
 * drt3d_inverse_lambdas returns them. With NULL the library computes them
 * by power iteration (30 steps from a fixed start vector) the first time a
 * size is used on a device, which synchronises `stream`, and keeps them for
 * the process.
 * Workspace: drt3d_inverse_workspace_bytes(N), 256-byte aligned. */
size_t drt3d_inverse_workspace_bytes(int N);
int drt3d_inverse(const void* proj, void* vol_out, int N, int cycles, const double* lams,
                  void* workspace, size_t workspace_bytes, void* stream);
/* The eigenvalues the inverse uses for sizes 2, 4, ..., N, written to lams
 * (log2 N doubles); computes the missing ones (synchronises `stream`). */
int drt3d_inverse_lambdas(int N, double* lams, void* workspace, size_t workspace_bytes, void* stream);

/* ---- tuning ----------------------------------------------------------------- */
/* Pick the stage grouping (stages fused per pass), tile width and LDS budget
 * (hence work groups per dodecant) and the wavefronts per work group for size
 * class N and dtype by timing candidates on the GPU with the given buffers
 * (vol: N^3, out: drt3d_out_elems(N, DRT3D_ALL), workspace of
 * drt3d_workspace_bytes(N, DRT3D_ALL, dtype)); `out` is clobbered. The time
 * minimised is the forward's for DRT3D_I32 and forward plus adjoint for
 * DRT3D_F32; for the latter the call allocates (and frees) the adjoint's
 * volume and workspace itself. The choice is kept for the process and, if the
 * environment variable DRT3D_TUNE_CACHE names a file, appended there. int32
 * results are bit-identical under every candidate; float32 results differ only
 * by the order in which the stage sums are rounded. */
int drt3d_autotune(int N, int dtype, const void* vol, void* out,
                   void* workspace, size_t workspace_bytes, void* stream);
/* Current tuning choice of size class N as text (for logs and tests):
 * "p=<kx>.<ky>,...;lds=<elements>;waves=<w>[;alds=<elements>]", the stages
 * per axis of each pass, the LDS budget of a work group in 4-byte elements,
 * the wavefronts per work group, and optionally a separate LDS budget for the
 * adjoint's passes other than a fused last pass. */
const char* drt3d_tuning_string(int N, int dtype);
/* Force a tuning choice from its text form (as printed by drt3d_tuning_string;
 * every pass of forward and adjoint must fit its LDS budget, else
 * DRT3D_EINVAL); used by determinism tests. */
int drt3d_set_tuning(int N, int dtype, const char* text);

/* ---- profiling -------------------------------------------------------------- */
/* When enabled (nonzero), each pass launch of the calls that follow records a
 * HIP event pair on the call's stream; drt3d_pass_times reports, per kernel
 * name (e.g. "drt_fwd_y2"), the summed milliseconds, the launch count and the
 * algorithmic bytes (reads of each pass's input extent plus writes of its
 * output extent) since the last reset. Synchronises the recorded events. */
int drt3d_profile_enable(int on);
int drt3d_profile_reset(void);
/* Writes up to `cap` records; returns the number of distinct kernel names. */
int drt3d_pass_times(char* names /* cap x 32 chars */, double* ms, long long* launches,
                     double* bytes, int cap);

/* ---- reference stream -------------------------------------------------------- */
/* Not part of any transform: the practical HBM ceiling a pass is measured
 * against. Reads read_bytes of src and writes write_bytes of dst (device
 * buffers, 16-byte aligned, byte counts multiples of 16 in [16, 32 GiB]),
 * interleaved in proportion, 16 bytes per lane, with the non-temporal store
 * policy of the DRT passes and no arithmetic. Asynchronous on `stream`; time it
 * with events. DRT3D_EINVAL for bad sizes or pointers. */
int drt3d_stream_probe(const void* src, size_t read_bytes, void* dst, size_t write_bytes, void* stream);

/* ---- plans ------------------------------------------------------------------ */
/* A plan fixes the shape of one of the four transforms (op as for
 * drt3d_plan_text: 0 drt3d_forward, 1 drt3d_adjoint, 2 djt3d_forward,
 * 3 djt3d_adjoint) for size N, dodecant mask and dtype (DRT3D_U8: op 0 only,
 * N >= 32), and for the DRT the tuning of size class N in force when it is
 * created (the pass grouping of Algorithm 1's stages, tile width, LDS budget,
 * wavefronts), so that later drt3d_autotune or drt3d_set_tuning calls leave its
 * launches unchanged. A plan is a host object: creating, querying and
 * destroying it does no GPU work, and one plan may run on any device, from
 * any thread, with any buffers. Arguments are checked as by the op's own call;
 * a bad one returns DRT3D_EINVAL and leaves *plan NULL. The caller owns the plan
 * and releases it with drt3d_plan_destroy (NULL is accepted there). */
typedef struct drt3d_plan_s* drt3d_plan;
int drt3d_plan_create(drt3d_plan* plan, int op, int N, uint32_t mask, int dtype);
/* Workspace bytes the plan's execution needs (0 for a NULL plan). */
size_t drt3d_plan_workspace_bytes(drt3d_plan plan);
/* Runs the planned transform: in and out as for the op's own call (volume or
 * projections, in that call's layout and dtype), the workspace at least
 * drt3d_plan_workspace_bytes(plan) bytes, asynchronous on `stream`. Results
 * equal the op's own call under the plan's tuning (bit for bit). */
int drt3d_plan_execute(drt3d_plan plan, const void* in, void* out, void* workspace, size_t workspace_bytes,
                       void* stream);
int drt3d_plan_destroy(drt3d_plan plan);

/* ---- introspection (host only, no GPU work) --------------------------------- */
/* Frame view of dodecant k (0..11) at size N as an affine element offset
 * out = {base, sx, sy, sd, group}:
 *   kind 0 (DRT):  g_k(x', y', N-1-dd) = V_group[base + sx*x' + sy*y' + sd*dd],
 *                  V_0 = [x][y][z] (the volume), V_1 = [x][z][y], V_2 = [y][z][x];
 *   kind 1 (DJT):  g_k(N-1-e1, N-1-e2, v) = vol[base + sx*e1 + sy*e2 + sd*v].  */
int drt3d_frame_map(int k, int N, int kind, int out[5]);
/* Text description of the launches one call would make (op 0: drt3d_forward,
 * 1: drt3d_adjoint, 2: djt3d_forward, 3: djt3d_adjoint), one line per launch:
 * "name kind=<k> wg=<work groups> block=<threads> lds=<bytes> bytes=<algorithmic>
 * kernel=<K>", where K names the DRT pass kernel: "fastA.BxW" (the pass kernel
 * specialised for A.B stages and W wavefronts), "groupA.BxW" (the adjoint's last
 * pass fused over each volume layout group), "generic", or "-" for other kinds.
 * Returns the number of launches, or a negative status. */
int drt3d_plan_text(int op, int N, uint32_t mask, int dtype, char* buf, size_t cap);

#ifdef __cplusplus
}
#endif
#endif /* DRT3D_H */
