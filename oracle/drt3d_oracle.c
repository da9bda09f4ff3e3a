/*
 * CPU oracle for the 3D multiscale discrete Radon (DRT) and John (DJT) transforms
 * of Marichal-Hernandez et al., "Three-dimensional multiscale discrete Radon and
 * John transforms" (arXiv 2501.13664).
 *
 * THIS IS TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it. The GPU library never links it and
 * shares no code, table or header with it.
 *
 * Two independent routes are provided for every transform:
 *   - the plain definitions (sums over the digital plane / line sets, Sec. 3.1
 *     eq. (9), Sec. 4.1 eq. (13), and the adjoint as the exact transpose of
 *     eq. (9), Sec. 5.1), evaluated either per output element or in scatter form;
 *   - the paper's multiscale recursions done naively on full-extent buffers
 *     (Algorithm 1 with the stage map of eq. (11), Algorithm 3 with eq. (15),
 *     and Algorithm 1 reversed with eq. (17)).
 * The tests pin each route against the other and against closed forms and
 * invariants; neither route is trusted on its own.
 *
 * Index conventions (readings of the paper, listed with reasons in the design notes):
 *   - primed frame k: the input is seen through the InOrder row k of Algorithm 2,
 *     read as "mirror every original axis |o_j| with o_j<0, then send original
 *     axis i to primed axis |o_i|";
 *   - DRT output R_k[s1][s2][dd], dd in [0,3N-2), dd = N-1-d where d is the
 *     displacement of eq. (9); the support of (s1,s2) is dd <= N-1+s1+s2;
 *   - DJT output J_k[s1][s2][e1][e2], e in [0,2N-1), e = N-1-d for each of the
 *     two displacements of eq. (13); the driving (summed) axis is z'.
 * Integer inputs accumulate in int64; floating inputs are given as double and
 * accumulate in double.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Discrete line, eq. (4), closed form: l^n_s(x) = sum_i bit_{n-1-i}(x) *
 * floor((floor(s/2^i)+1)/2), where bit_0 is the least significant bit (lambda of
 * Sec. 2.1 weights u_i by 2^i).                                               */
int orc_line(int n, int s, int x)
{
    int acc = 0;
    for (int i = 0; i < n; ++i) {
        int bit = (x >> (n - 1 - i)) & 1;
        acc += bit * (((s >> i) + 1) >> 1);
    }
    return acc;
}

/* Discrete line, eq. (4), recursive form: l^n_s(u_0..u_{n-1}) =
 * l^{n-1}_{floor(s/2)}(u_0..u_{n-2}) + u_{n-1} * floor((s+1)/2); l^0 = 0.    */
int orc_line_recursive(int n, int s, int x)
{
    if (n == 0) return 0;
    int top = (x >> (n - 1)) & 1;
    int low = x & ((1 << (n - 1)) - 1);
    return orc_line_recursive(n - 1, s >> 1, low) + top * ((s + 1) >> 1);
}

static int ilog2_exact(int N)
{
    int n = 0;
    while ((1 << n) < N) ++n;
    return ((1 << n) == N) ? n : -1;
}

/* ------------------------------------------------------------------------- */
/* The 12 dodecant frames: InOrder of Algorithm 2, as printed (1-based signed
 * axis numbers, row k = dodecant k).                                         */
static const int IN_ORDER[12][3] = {
    { 1,  2,  3}, {-2,  1,  3}, {-1, -2,  3}, { 2, -1,  3},
    {-1, -3, -2}, {-3, -1,  2}, { 3, -1, -2}, { 1,  3, -2},
    {-3, -2, -1}, {-2, -3,  1}, {-2,  3, -1}, { 3,  2, -1},
};

/* Reading of a row o = InOrder[k]: every original axis |o_j| with o_j < 0 is
 * mirrored (a -> N-1-a), then original axis i is sent to primed axis |o_i|
 * (the inverse permutation). This is the one reading under which the 12 frames
 * tile the hemisphere of plane normals and of line directions, which Sec. 3.2
 * and Sec. 4.1 state they do.                                                */
static int axis_mirrored(int k, int i)
{
    for (int j = 0; j < 3; ++j)
        if (IN_ORDER[k][j] < 0 && -IN_ORDER[k][j] == i + 1) return 1;
    return 0;
}

/* Primed -> original coordinates: original axis i carries primed axis
 * |o_i|-1, mirrored when axis i is in the flipped set.                     */
void orc_frame_to_orig(int k, int N, const int primed[3], int orig[3])
{
    for (int i = 0; i < 3; ++i) {
        int o = IN_ORDER[k][i];
        int p = primed[(o < 0 ? -o : o) - 1];
        orig[i] = axis_mirrored(k, i) ? (N - 1 - p) : p;
    }
}

/* Row k of the InOrder table as the oracle holds it (for the test that pins
 * this transcription against a golden copy of the printed table).          */
void orc_in_order_row(int k, int row[3])
{
    for (int i = 0; i < 3; ++i) row[i] = IN_ORDER[k][i];
}

/* Linear part of the original -> primed map as a signed permutation matrix
 * M (row-major, primed = M * orig + offset); used by the tiling tests.      */
void orc_frame_matrix(int k, int M[9])
{
    memset(M, 0, 9 * sizeof(int));
    for (int i = 0; i < 3; ++i) {
        int o = IN_ORDER[k][i];
        int j = (o < 0 ? -o : o) - 1;
        M[j * 3 + i] = axis_mirrored(k, i) ? -1 : 1;
    }
}

static inline int64_t vol_index(int N, const int c[3])
{
    return ((int64_t)c[0] * N + c[1]) * N + c[2];
}

/* g_k(x',y',z') for an in-range primed point. */
#define FRAME_VALUE(vol, k, N, xp, yp, zp, out)                                \
    do {                                                                       \
        int p_[3] = {(xp), (yp), (zp)}, o_[3];                                 \
        orc_frame_to_orig((k), (N), p_, o_);                                   \
        (out) = (vol)[vol_index((N), o_)];                                     \
    } while (0)

/* Table of l^n_s(x), [s][x]. Caller frees. */
static int* line_table(int N, int n)
{
    int* L = (int*)malloc(sizeof(int) * (size_t)N * N);
    if (!L) return NULL;
    for (int s = 0; s < N; ++s)
        for (int x = 0; x < N; ++x) L[s * N + x] = orc_line(n, s, x);
    return L;
}

static int mask_count(unsigned mask)
{
    int c = 0;
    for (int k = 0; k < 12; ++k) c += (mask >> k) & 1;
    return c;
}

/* ========================================================================= */
/* Definitions, written once for int64 (int32 input) and double (double input). */
#define DEFINE_DEFINITIONS(SUF, IN_T, ACC_T)                                    \
/* eq. (9): R_k[s1][s2][dd] = sum over x',y' of g_k(x',y',                       \
 *   l_{s1}(x') + l_{s2}(y') + N-1-dd), terms with z' outside [0,N) dropped.    */\
ACC_T orc_drt_point_##SUF(const IN_T* vol, int N, int k, int s1, int s2, int dd)\
{                                                                              \
    int n = ilog2_exact(N);                                                    \
    ACC_T acc = 0;                                                             \
    for (int xp = 0; xp < N; ++xp)                                             \
        for (int yp = 0; yp < N; ++yp) {                                       \
            int zp = orc_line(n, s1, xp) + orc_line(n, s2, yp) + N - 1 - dd;   \
            if (zp < 0 || zp >= N) continue;                                   \
            IN_T v;                                                            \
            FRAME_VALUE(vol, k, N, xp, yp, zp, v);                             \
            acc += (ACC_T)v;                                                   \
        }                                                                      \
    return acc;                                                                \
}                                                                              \
/* eq. (9) in scatter form: every voxel of frame k is added to the plane        \
 * (s1,s2,dd) it lies on, for every slope pair. out: [popcount][N][N][3N-2].   */\
int orc_drt_def_##SUF(const IN_T* vol, int N, unsigned mask, ACC_T* out)       \
{                                                                              \
    int n = ilog2_exact(N);                                                    \
    if (n < 1) return -1;                                                      \
    int* L = line_table(N, n);                                                 \
    if (!L) return -2;                                                         \
    const int64_t D = 3 * (int64_t)N - 2;                                      \
    memset(out, 0, sizeof(ACC_T) * (size_t)mask_count(mask) * N * N * D);      \
    int j = 0;                                                                 \
    for (int k = 0; k < 12; ++k) {                                             \
        if (!((mask >> k) & 1)) continue;                                      \
        ACC_T* R = out + (int64_t)j * N * N * D;                               \
        for (int xp = 0; xp < N; ++xp)                                         \
            for (int yp = 0; yp < N; ++yp)                                     \
                for (int zp = 0; zp < N; ++zp) {                               \
                    IN_T v;                                                    \
                    FRAME_VALUE(vol, k, N, xp, yp, zp, v);                     \
                    if (v == 0) continue;                                      \
                    for (int s1 = 0; s1 < N; ++s1)                             \
                        for (int s2 = 0; s2 < N; ++s2) {                       \
                            int dd = N - 1 + L[s1 * N + xp] + L[s2 * N + yp] - zp; \
                            R[((int64_t)s1 * N + s2) * D + dd] += (ACC_T)v;    \
                        }                                                      \
                }                                                              \
        ++j;                                                                   \
    }                                                                          \
    free(L);                                                                   \
    return 0;                                                                  \
}                                                                              \
/* eq. (13) with the driving axis z': J_k[s1][s2][e1][e2] = sum over u of       \
 *   g_k(l_{s1}(u) + N-1-e1, l_{s2}(u) + N-1-e2, u), out-of-cube terms dropped. */\
ACC_T orc_djt_point_##SUF(const IN_T* vol, int N, int k, int s1, int s2,       \
                          int e1, int e2)                                      \
{                                                                              \
    int n = ilog2_exact(N);                                                    \
    ACC_T acc = 0;                                                             \
    for (int u = 0; u < N; ++u) {                                              \
        int xp = orc_line(n, s1, u) + N - 1 - e1;                              \
        int yp = orc_line(n, s2, u) + N - 1 - e2;                              \
        if (xp < 0 || xp >= N || yp < 0 || yp >= N) continue;                  \
        IN_T v;                                                                \
        FRAME_VALUE(vol, k, N, xp, yp, u, v);                                  \
        acc += (ACC_T)v;                                                       \
    }                                                                          \
    return acc;                                                                \
}                                                                              \
/* eq. (13) in scatter form. out: [popcount][N][N][2N-1][2N-1].                */\
int orc_djt_def_##SUF(const IN_T* vol, int N, unsigned mask, ACC_T* out)       \
{                                                                              \
    int n = ilog2_exact(N);                                                    \
    if (n < 1) return -1;                                                      \
    int* L = line_table(N, n);                                                 \
    if (!L) return -2;                                                         \
    const int64_t E = 2 * (int64_t)N - 1;                                      \
    memset(out, 0, sizeof(ACC_T) * (size_t)mask_count(mask) * N * N * E * E);  \
    int j = 0;                                                                 \
    for (int k = 0; k < 12; ++k) {                                             \
        if (!((mask >> k) & 1)) continue;                                      \
        ACC_T* J = out + (int64_t)j * N * N * E * E;                           \
        for (int xp = 0; xp < N; ++xp)                                         \
            for (int yp = 0; yp < N; ++yp)                                     \
                for (int u = 0; u < N; ++u) {                                  \
                    IN_T v;                                                    \
                    FRAME_VALUE(vol, k, N, xp, yp, u, v);                      \
                    if (v == 0) continue;                                      \
                    for (int s1 = 0; s1 < N; ++s1)                             \
                        for (int s2 = 0; s2 < N; ++s2) {                       \
                            int e1 = N - 1 + L[s1 * N + u] - xp;               \
                            int e2 = N - 1 + L[s2 * N + u] - yp;               \
                            J[(((int64_t)s1 * N + s2) * E + e1) * E + e2] += (ACC_T)v; \
                        }                                                      \
                }                                                              \
        ++j;                                                                   \
    }                                                                          \
    free(L);                                                                   \
    return 0;                                                                  \
}                                                                              \
/* Adjoint (backprojection) of eq. (9), Sec. 5.1: every voxel receives, from    \
 * every dodecant in the mask and every slope pair, the value of the one plane  \
 * through it. No normalisation. proj: [popcount][N][N][3N-2].                 */\
ACC_T orc_adj_point_##SUF(const IN_T* proj, int N, unsigned mask,              \
                          int x, int y, int z)                                 \
{                                                                              \
    int n = ilog2_exact(N);                                                    \
    const int64_t D = 3 * (int64_t)N - 2;                                      \
    ACC_T acc = 0;                                                             \
    int j = 0;                                                                 \
    for (int k = 0; k < 12; ++k) {                                             \
        if (!((mask >> k) & 1)) continue;                                      \
        /* primed coordinates of (x,y,z): invert the frame by search */         \
        int o[3] = {x, y, z}, p[3] = {0, 0, 0};                                \
        for (int i = 0; i < 3; ++i) {                                          \
            int oo = IN_ORDER[k][i];                                           \
            int a = (oo < 0 ? -oo : oo) - 1;                                   \
            p[a] = axis_mirrored(k, i) ? (N - 1 - o[i]) : o[i];                \
        }                                                                      \
        const IN_T* P = proj + (int64_t)j * N * N * D;                         \
        for (int s1 = 0; s1 < N; ++s1)                                         \
            for (int s2 = 0; s2 < N; ++s2) {                                   \
                int dd = N - 1 + orc_line(n, s1, p[0]) + orc_line(n, s2, p[1]) - p[2]; \
                acc += (ACC_T)P[((int64_t)s1 * N + s2) * D + dd];              \
            }                                                                  \
        ++j;                                                                   \
    }                                                                          \
    return acc;                                                                \
}                                                                              \
/* Full adjoint by the definition (gather per voxel). vol_out: [N][N][N].      */\
int orc_adj_def_##SUF(const IN_T* proj, int N, unsigned mask, ACC_T* vol_out)  \
{                                                                              \
    if (ilog2_exact(N) < 1) return -1;                                         \
    for (int x = 0; x < N; ++x)                                                \
        for (int y = 0; y < N; ++y)                                            \
            for (int z = 0; z < N; ++z)                                        \
                vol_out[((int64_t)x * N + y) * N + z] =                        \
                    orc_adj_point_##SUF(proj, N, mask, x, y, z);               \
    return 0;                                                                  \
}                                                                              \
/* Adjoint of eq. (13) (the backprojection of lines, Sec. 5.1, which eq. (18)  \
 * computes stage by stage), by its definition: every voxel receives, from     \
 * each selected dodecant, the sum over all slope pairs of the one line        \
 * through it: with primed coordinates (x', y', u), the entry                  \
 * J[s1][s2][N-1 + l_{s1}(u) - x'][N-1 + l_{s2}(u) - y'].                      */\
ACC_T orc_djt_adj_point_##SUF(const IN_T* proj, int N, unsigned mask,          \
                              int x, int y, int z)                             \
{                                                                              \
    int n = ilog2_exact(N);                                                    \
    const int64_t E = 2 * (int64_t)N - 1;                                      \
    ACC_T acc = 0;                                                             \
    int j = 0;                                                                 \
    for (int k = 0; k < 12; ++k) {                                             \
        if (!((mask >> k) & 1)) continue;                                      \
        int o[3] = {x, y, z}, p[3] = {0, 0, 0};                                \
        for (int i = 0; i < 3; ++i) {                                          \
            int oo = IN_ORDER[k][i];                                           \
            int a = (oo < 0 ? -oo : oo) - 1;                                   \
            p[a] = axis_mirrored(k, i) ? (N - 1 - o[i]) : o[i];                \
        }                                                                      \
        const IN_T* P = proj + (int64_t)j * N * N * E * E;                     \
        for (int s1 = 0; s1 < N; ++s1)                                         \
            for (int s2 = 0; s2 < N; ++s2) {                                   \
                int e1 = N - 1 + orc_line(n, s1, p[2]) - p[0];                 \
                int e2 = N - 1 + orc_line(n, s2, p[2]) - p[1];                 \
                acc += (ACC_T)P[(((int64_t)s1 * N + s2) * E + e1) * E + e2];   \
            }                                                                  \
        ++j;                                                                   \
    }                                                                          \
    return acc;                                                                \
}                                                                              \
/* Full DJT adjoint by the definition (gather per voxel). vol_out: [N][N][N].  */\
int orc_djt_adj_def_##SUF(const IN_T* proj, int N, unsigned mask, ACC_T* vol_out) \
{                                                                              \
    if (ilog2_exact(N) < 1) return -1;                                         \
    for (int x = 0; x < N; ++x)                                                \
        for (int y = 0; y < N; ++y)                                            \
            for (int z = 0; z < N; ++z)                                        \
                vol_out[((int64_t)x * N + y) * N + z] =                        \
                    orc_djt_adj_point_##SUF(proj, N, mask, x, y, z);           \
    return 0;                                                                  \
}

DEFINE_DEFINITIONS(i, int32_t, int64_t)
DEFINE_DEFINITIONS(f, double, double)

/* ========================================================================= */
/* The paper's recursions, naive, on full-extent buffers.                    */
#define DEFINE_RECURSIONS(SUF, IN_T, ACC_T)                                     \
/* Algorithm 1 (one dodecant) with the stage map of eq. (11). Buffers are       \
 * N x N x 3N indexed (c1, c2, D); the frame-k input sits at D = 2N + z'.       \
 * At stage m a column index c = sigma + (v << m) carries an m-bit slope sigma  \
 * and an (n-m)-bit block index v; the new slope is a + 2*sigma (the slope's    \
 * new least significant bit a, Sec. 4.1), the two halves v_m = 0,1 of the     \
 * block are merged with the second one read at D + sigma + a, and reads past   \
 * the buffer end are zero. Output dd = 3N-1-D, dd in [0,3N-2).               */\
int orc_drt_rec_##SUF(const IN_T* vol, int N, unsigned mask, ACC_T* out)       \
{                                                                              \
    int n = ilog2_exact(N);                                                    \
    if (n < 1) return -1;                                                      \
    const int64_t W = 3 * (int64_t)N;                                          \
    const int64_t D = 3 * (int64_t)N - 2;                                      \
    size_t cells = (size_t)N * N * W;                                          \
    ACC_T* A = (ACC_T*)malloc(cells * sizeof(ACC_T));                          \
    ACC_T* B = (ACC_T*)malloc(cells * sizeof(ACC_T));                          \
    if (!A || !B) { free(A); free(B); return -2; }                             \
    int j = 0;                                                                 \
    for (int k = 0; k < 12; ++k) {                                             \
        if (!((mask >> k) & 1)) continue;                                      \
        memset(A, 0, cells * sizeof(ACC_T));                                   \
        for (int xp = 0; xp < N; ++xp)                                         \
            for (int yp = 0; yp < N; ++yp)                                     \
                for (int zp = 0; zp < N; ++zp) {                               \
                    IN_T v;                                                    \
                    FRAME_VALUE(vol, k, N, xp, yp, zp, v);                     \
                    A[((int64_t)xp * N + yp) * W + 2 * N + zp] = (ACC_T)v;     \
                }                                                              \
        for (int m = 0; m < n; ++m) {                                          \
            int h = 1 << m;                                                    \
            for (int c1 = 0; c1 < N; ++c1) {                                   \
                int a = c1 & 1, sig1 = (c1 >> 1) & (h - 1), blk1 = c1 >> (m + 1); \
                int lo1 = sig1 + (blk1 << (m + 1)), hi1 = lo1 + h;             \
                int sh1 = sig1 + a;                                            \
                for (int c2 = 0; c2 < N; ++c2) {                               \
                    int b = c2 & 1, sig2 = (c2 >> 1) & (h - 1), blk2 = c2 >> (m + 1); \
                    int lo2 = sig2 + (blk2 << (m + 1)), hi2 = lo2 + h;         \
                    int sh2 = sig2 + b;                                        \
                    const ACC_T* f00 = A + ((int64_t)lo1 * N + lo2) * W;       \
                    const ACC_T* f10 = A + ((int64_t)hi1 * N + lo2) * W;       \
                    const ACC_T* f01 = A + ((int64_t)lo1 * N + hi2) * W;       \
                    const ACC_T* f11 = A + ((int64_t)hi1 * N + hi2) * W;       \
                    ACC_T* o = B + ((int64_t)c1 * N + c2) * W;                 \
                    for (int64_t d = 0; d < W; ++d) {                          \
                        ACC_T s = f00[d];                                      \
                        if (d + sh1 < W) s += f10[d + sh1];                    \
                        if (d + sh2 < W) s += f01[d + sh2];                    \
                        if (d + sh1 + sh2 < W) s += f11[d + sh1 + sh2];        \
                        o[d] = s;                                              \
                    }                                                          \
                }                                                              \
            }                                                                  \
            ACC_T* t = A; A = B; B = t;                                        \
        }                                                                      \
        ACC_T* R = out + (int64_t)j * N * N * D;                               \
        for (int64_t c = 0; c < (int64_t)N * N; ++c)                           \
            for (int64_t dd = 0; dd < D; ++dd)                                 \
                R[c * D + dd] = A[c * W + (W - 1 - dd)];                       \
        ++j;                                                                   \
    }                                                                          \
    free(A); free(B);                                                          \
    return 0;                                                                  \
}                                                                              \
/* Algorithm 3 (one dodecant) with the stage map of eq. (15), driving axis z'.  \
 * Stage m holds (N >> m) blocks v and 4^m slope pairs, each a 2N x 2N plane    \
 * indexed (D1, D2); the input sits at D1 = N + x', D2 = N + y' of block u=z'.  \
 * Block halves 2v and 2v+1 merge, the second read at (D1 + s1', D2 + s2')      \
 * with s' = sigma + new-lsb; reads past the plane are zero. Output              \
 * e = 2N-1-D, e in [0,2N-1).                                                  */\
int orc_djt_rec_##SUF(const IN_T* vol, int N, unsigned mask, ACC_T* out)       \
{                                                                              \
    int n = ilog2_exact(N);                                                    \
    if (n < 1) return -1;                                                      \
    const int64_t W = 2 * (int64_t)N, E = 2 * (int64_t)N - 1;                  \
    const int64_t plane = W * W;                                               \
    size_t cells = (size_t)N * N * plane; /* N*2^m planes at most N*N */       \
    ACC_T* A = (ACC_T*)malloc(cells * sizeof(ACC_T));                          \
    ACC_T* B = (ACC_T*)malloc(cells * sizeof(ACC_T));                          \
    if (!A || !B) { free(A); free(B); return -2; }                             \
    int j = 0;                                                                 \
    for (int k = 0; k < 12; ++k) {                                             \
        if (!((mask >> k) & 1)) continue;                                      \
        /* stage 0: plane index = v (= z'), no slope bits */                    \
        memset(A, 0, (size_t)N * plane * sizeof(ACC_T));                       \
        for (int xp = 0; xp < N; ++xp)                                         \
            for (int yp = 0; yp < N; ++yp)                                     \
                for (int u = 0; u < N; ++u) {                                  \
                    IN_T v;                                                    \
                    FRAME_VALUE(vol, k, N, xp, yp, u, v);                      \
                    A[(int64_t)u * plane + (N + xp) * W + (N + yp)] = (ACC_T)v; \
                }                                                              \
        for (int m = 0; m < n; ++m) {                                          \
            int h = 1 << m;             /* slopes per axis at stage m   */     \
            int Vm = N >> m, Vn = N >> (m + 1);                                \
            /* plane index at stage m: (sig1 * h + sig2) * Vm + v */            \
            for (int s1 = 0; s1 < 2 * h; ++s1)                                 \
                for (int s2 = 0; s2 < 2 * h; ++s2) {                           \
                    int a = s1 & 1, sig1 = s1 >> 1;                            \
                    int b = s2 & 1, sig2 = s2 >> 1;                            \
                    int sh1 = sig1 + a, sh2 = sig2 + b;                        \
                    for (int v = 0; v < Vn; ++v) {                             \
                        const ACC_T* f0 = A + ((int64_t)(sig1 * h + sig2) * Vm + 2 * v) * plane; \
                        const ACC_T* f1 = A + ((int64_t)(sig1 * h + sig2) * Vm + 2 * v + 1) * plane; \
                        ACC_T* o = B + ((int64_t)(s1 * 2 * h + s2) * Vn + v) * plane; \
                        for (int64_t d1 = 0; d1 < W; ++d1)                     \
                            for (int64_t d2 = 0; d2 < W; ++d2) {               \
                                ACC_T s = f0[d1 * W + d2];                     \
                                if (d1 + sh1 < W && d2 + sh2 < W)              \
                                    s += f1[(d1 + sh1) * W + d2 + sh2];        \
                                o[d1 * W + d2] = s;                            \
                            }                                                  \
                    }                                                          \
                }                                                              \
            ACC_T* t = A; A = B; B = t;                                        \
        }                                                                      \
        ACC_T* J = out + (int64_t)j * N * N * E * E;                           \
        for (int64_t p = 0; p < (int64_t)N * N; ++p)                           \
            for (int64_t e1 = 0; e1 < E; ++e1)                                 \
                for (int64_t e2 = 0; e2 < E; ++e2)                             \
                    J[(p * E + e1) * E + e2] =                                 \
                        A[p * plane + (W - 1 - e1) * W + (W - 1 - e2)];        \
        ++j;                                                                   \
    }                                                                          \
    free(A); free(B);                                                          \
    return 0;                                                                  \
}                                                                              \
/* Algorithm 1 reversed with eq. (17) (Sec. 5.1): stages run m = n-1 .. 0; a    \
 * child column sigma + (i << m) + (v << (m+1)) gathers the two parents         \
 * a + 2*sigma + (v << (m+1)), read at D - i*(sigma + a); reads below zero are  \
 * zero. The volume receives D = 2N + z' of the last stage, summed over the     \
 * dodecants of the mask. proj: [popcount][N][N][3N-2], vol_out: [N][N][N].    */\
int orc_adj_rec_##SUF(const IN_T* proj, int N, unsigned mask, ACC_T* vol_out)  \
{                                                                              \
    int n = ilog2_exact(N);                                                    \
    if (n < 1) return -1;                                                      \
    const int64_t W = 3 * (int64_t)N;                                          \
    const int64_t D = 3 * (int64_t)N - 2;                                      \
    size_t cells = (size_t)N * N * W;                                          \
    ACC_T* A = (ACC_T*)malloc(cells * sizeof(ACC_T));                          \
    ACC_T* B = (ACC_T*)malloc(cells * sizeof(ACC_T));                          \
    if (!A || !B) { free(A); free(B); return -2; }                             \
    memset(vol_out, 0, sizeof(ACC_T) * (size_t)N * N * N);                    \
    int j = 0;                                                                 \
    for (int k = 0; k < 12; ++k) {                                             \
        if (!((mask >> k) & 1)) continue;                                      \
        const IN_T* P = proj + (int64_t)j * N * N * D;                         \
        memset(A, 0, cells * sizeof(ACC_T));                                   \
        for (int64_t c = 0; c < (int64_t)N * N; ++c)                           \
            for (int64_t dd = 0; dd < D; ++dd)                                 \
                A[c * W + (W - 1 - dd)] = (ACC_T)P[c * D + dd];                \
        for (int m = n - 1; m >= 0; --m) {                                     \
            int h = 1 << m;                                                    \
            for (int c1 = 0; c1 < N; ++c1) {                                   \
                int i = (c1 >> m) & 1, sig1 = c1 & (h - 1), blk1 = c1 >> (m + 1); \
                for (int c2 = 0; c2 < N; ++c2) {                               \
                    int jj = (c2 >> m) & 1, sig2 = c2 & (h - 1), blk2 = c2 >> (m + 1); \
                    ACC_T* o = B + ((int64_t)c1 * N + c2) * W;                 \
                    for (int64_t d = 0; d < W; ++d) o[d] = 0;                  \
                    for (int a = 0; a < 2; ++a)                                \
                        for (int b = 0; b < 2; ++b) {                          \
                            int p1 = a + 2 * sig1 + (blk1 << (m + 1));         \
                            int p2 = b + 2 * sig2 + (blk2 << (m + 1));         \
                            int sh = i * (sig1 + a) + jj * (sig2 + b);         \
                            const ACC_T* f = A + ((int64_t)p1 * N + p2) * W;   \
                            for (int64_t d = sh; d < W; ++d) o[d] += f[d - sh]; \
                        }                                                      \
                }                                                              \
            }                                                                  \
            ACC_T* t = A; A = B; B = t;                                        \
        }                                                                      \
        for (int xp = 0; xp < N; ++xp)                                         \
            for (int yp = 0; yp < N; ++yp)                                     \
                for (int zp = 0; zp < N; ++zp) {                               \
                    int p_[3] = {xp, yp, zp}, o_[3];                           \
                    orc_frame_to_orig(k, N, p_, o_);                           \
                    vol_out[vol_index(N, o_)] +=                               \
                        A[((int64_t)xp * N + yp) * W + 2 * N + zp];            \
                }                                                              \
        ++j;                                                                   \
    }                                                                          \
    free(A); free(B);                                                          \
    return 0;                                                                  \
}

DEFINE_RECURSIONS(i, int32_t, int64_t)
DEFINE_RECURSIONS(f, double, double)
