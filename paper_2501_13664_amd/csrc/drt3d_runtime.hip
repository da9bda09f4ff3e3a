// Host runtime and C ABI of the drt3d library (see include/drt3d.h).
//
// Every call becomes an ordered list of steps; a step is one kernel launch
// (a DRT pass, a DJT stage or a transpose) described by its descriptors. A
// step carries a canonical key; the batched entry points merge the steps of
// all volumes that share a key into a single persistent launch, in key order,
// which preserves each volume's own order.
//
// DRT forward of one cube: transposes that make the y- and x-normal frames'
// displacement axis contiguous, then the x-passes (stages of slope s1) and
// the y-passes (slope s2), each fusing K stages of eq. (11) in LDS. The
// adjoint runs the mirrored passes in reverse (eq. (17)); its last pass adds
// every dodecant into one accumulator per frame group, and the accumulators
// of the y- and x-normal groups are transposed back into the caller's volume.
// The DJT runs one launch per stage of eq. (15).
//
// Single-volume calls process the dodecants in chunks that keep the stage
// buffers under a fixed budget; batched calls keep every dodecant in flight.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/drt3d.h"
#include "drt3d_internal.h"

namespace drt3d {

// ------------------------------------------------------------------ errors
static thread_local std::string g_last_error;

static int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define HIP_TRY(expr)                                                                                \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess)                                                                        \
            return fail(DRT3D_EHIP, "%s failed: %s (%d)", #expr, hipGetErrorString(e_), (int)e_);     \
    } while (0)

#define TRY(expr)                  \
    do {                           \
        int rc_ = (expr);          \
        if (rc_ != DRT3D_OK) return rc_; \
    } while (0)

static int ilog2_exact(int N)
{
    if (N < 2 || N > DRT3D_MAX_N) return -1;
    int n = 0;
    while ((1 << n) < N) ++n;
    return (1 << n) == N ? n : -1;
}

static int popcount12(uint32_t mask)
{
    int c = 0;
    for (int k = 0; k < 12; ++k) c += (mask >> k) & 1u;
    return c;
}

static inline long long round4(long long x) { return (x + 3) & ~3LL; }
static inline long long round32(long long x) { return (x + 31) & ~31LL; }
static inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// ------------------------------------------------------------------ frames
// Row k of Algorithm 2's InOrder table (1-based signed axis numbers).
static const int kInOrder[12][3] = {
    {1, 2, 3},   {-2, 1, 3},   {-1, -2, 3},  {2, -1, 3}, {-1, -3, -2}, {-3, -1, 2},
    {3, -1, -2}, {1, 3, -2},   {-3, -2, -1}, {-2, -3, 1}, {-2, 3, -1}, {3, 2, -1},
};

// Reading of a row: original axis i is mirrored iff some entry o_j < 0 has
// |o_j| = i+1, and original axis i carries primed axis |o_i|-1.
struct AxisMap {
    int primed;  // 0: x', 1: y', 2: z'
    int mirror;
};

static void frame_axes(int k, AxisMap out[3])
{
    for (int i = 0; i < 3; ++i) {
        const int o = kInOrder[k][i];
        out[i].primed = (o < 0 ? -o : o) - 1;
        out[i].mirror = 0;
    }
    for (int j = 0; j < 3; ++j)
        if (kInOrder[k][j] < 0) out[-kInOrder[k][j] - 1].mirror = 1;
}

// DRT frame group of dodecant k: 0 if z' is along z, 1 along y, 2 along x.
static int drt_group(int k)
{
    AxisMap a[3];
    frame_axes(k, a);
    for (int i = 0; i < 3; ++i)
        if (a[i].primed == 2) return i == 2 ? 0 : (i == 1 ? 1 : 2);
    return 0;
}

// Layout V_g[A][B][C] of group g's copy of the volume, C contiguous:
//   g0: [x][y][z] (the caller's volume), g1: [x][z][y], g2: [y][z][x].
static void group_layout(int g, int axes[3])
{
    if (g == 0) { axes[0] = 0; axes[1] = 1; axes[2] = 2; }
    else if (g == 1) { axes[0] = 0; axes[1] = 2; axes[2] = 1; }
    else { axes[0] = 1; axes[1] = 2; axes[2] = 0; }
}

// g_k(x', y', N-1-dd) = V_g[base + sx x' + sy y' + sd dd].
static FrameMap drt_frame_map(int k, int N)
{
    AxisMap ax[3];
    frame_axes(k, ax);
    FrameMap f{};
    f.group = drt_group(k);
    int axes[3];
    group_layout(f.group, axes);
    const long long mult[3] = {(long long)N * N, N, 1};
    long long base = 0, sx = 0, sy = 0, sd = 0;
    for (int r = 0; r < 3; ++r) {
        const AxisMap& m = ax[axes[r]];
        const long long M = mult[r];
        const long long beta = m.mirror ? -1 : 1;
        if (m.mirror) base += M * (N - 1);
        if (m.primed == 0) sx += M * beta;
        else if (m.primed == 1) sy += M * beta;
        else { base += M * beta * (N - 1); sd -= M * beta; }  // z' = N-1-dd
    }
    f.base = (int)base; f.sx = (int)sx; f.sy = (int)sy; f.sd = (int)sd;
    return f;
}

// DJT stage 0: g_k(N-1-e1, N-1-e2, v) = vol[base + sx e1 + sy e2 + sd v].
static FrameMap djt_frame_map(int k, int N)
{
    AxisMap ax[3];
    frame_axes(k, ax);
    FrameMap f{};
    const long long mult[3] = {(long long)N * N, N, 1};
    long long base = 0, sx = 0, sy = 0, sd = 0;
    for (int i = 0; i < 3; ++i) {
        const long long M = mult[i];
        const long long beta = ax[i].mirror ? -1 : 1;
        if (ax[i].mirror) base += M * (N - 1);
        if (ax[i].primed == 0) { base += M * beta * (N - 1); sx -= M * beta; }
        else if (ax[i].primed == 1) { base += M * beta * (N - 1); sy -= M * beta; }
        else sd += M * beta;
    }
    f.base = (int)base; f.sx = (int)sx; f.sy = (int)sy; f.sd = (int)sd;
    return f;
}

// ------------------------------------------------------------------ tuning
// A tuning is the pass list (each pass fuses kx x-stages and ky y-stages, the
// stages of each axis taken in order), the LDS budget of a work group and the
// number of wavefronts per work group.
struct Tuning {
    int np = 0;
    int kx[8] = {0}, ky[8] = {0};
    int lds_elems = 18432;  // LDS budget of one work group, in 4-byte elements (72 KB: two per CU)
    int waves = 8;          // wavefronts per work group (upper bound)
    int adj_lds_elems = 0;  // the adjoint's passes other than a fused last pass; 0: lds_elems
};

// LDS budget of an adjoint pass (the fused last pass keeps lds_elems)
static int adj_lds_of(const Tuning& t) { return t.adj_lds_elems > 0 ? t.adj_lds_elems : t.lds_elems; }

static const int kMaxPassSlots = 256;  // 2^(kx+ky) columns per group at most

// Default: as few passes as fit 64-column groups, stages spread evenly.
static bool tuning_from_string(const char* s, int n, Tuning& t);

// Rule for size classes without a measured entry: passes of at most 3 x- and
// 3 y-stages, as even as possible, the shorter ones first (the early stage
// buffers are the narrow ones).
static Tuning rule_tuning(int n)
{
    Tuning t;
    int P = (n + 2) / 3;
    if (P < 1) P = 1;
    t.np = P;
    for (int i = 0; i < P; ++i) {
        t.kx[i] = n / P + (i >= P - n % P ? 1 : 0);
        t.ky[i] = t.kx[i];
    }
    return t;
}

// Choices of drt3d_autotune on an MI355X (gfx950), per size class and dtype;
// the adjoint budgets (alds) from timing the adjoint's passes alone.
struct MeasuredTuning {
    int n, is_float;
    const char* text;
};
static const MeasuredTuning kMeasured[] = {
    {5, 0, "p=3.3,2.2;lds=13312;waves=8"},     {5, 1, "p=2.2,3.3;lds=16384;waves=8"},
    {6, 0, "p=3.3,3.3;lds=20480;waves=8"},     {6, 1, "p=3.3,3.3;lds=24576;waves=8"},
    {7, 0, "p=2.2,2.3,3.2;lds=12288;waves=8"}, {7, 1, "p=2.2,2.3,3.2;lds=14336;waves=8"},
    {8, 0, "p=3.3,2.3,3.2;lds=14336;waves=8"}, {8, 1, "p=2.3,3.3,3.2;lds=24576;waves=8"},
    {9, 0, "p=3.3,3.3,3.3;lds=14336;waves=8;alds=13312"}, {9, 1, "p=3.3,3.3,3.3;lds=14336;waves=16"},
};

static Tuning default_tuning(int n, int is_float)
{
    for (const MeasuredTuning& m : kMeasured) {
        Tuning t;
        if (m.n == n && m.is_float == is_float && tuning_from_string(m.text, n, t)) return t;
    }
    return rule_tuning(n);
}

static std::string tuning_to_string(const Tuning& t)
{
    std::string s = "p=";
    for (int i = 0; i < t.np; ++i) s += (i ? "," : "") + std::to_string(t.kx[i]) + "." + std::to_string(t.ky[i]);
    s += ";lds=" + std::to_string(t.lds_elems) + ";waves=" + std::to_string(t.waves);
    if (t.adj_lds_elems > 0) s += ";alds=" + std::to_string(t.adj_lds_elems);
    return s;
}

static bool tuning_from_string(const char* s, int n, Tuning& t)
{
    Tuning r;
    const char* p = s;
    char* e = nullptr;
    if (strncmp(p, "p=", 2)) return false;
    p += 2;
    r.np = 0;
    while (*p >= '0' && *p <= '9') {
        if (r.np >= 8) return false;
        r.kx[r.np] = (int)strtol(p, &e, 10);
        p = e;
        if (*p != '.') return false;
        r.ky[r.np] = (int)strtol(p + 1, &e, 10);
        p = e;
        ++r.np;
        if (*p == ',') ++p;
    }
    if (strncmp(p, ";lds=", 5)) return false;
    r.lds_elems = (int)strtol(p + 5, &e, 10);
    p = e;
    if (strncmp(p, ";waves=", 7)) return false;
    r.waves = (int)strtol(p + 7, &e, 10);
    p = e;
    if (!strncmp(p, ";alds=", 6)) {
        r.adj_lds_elems = (int)strtol(p + 6, &e, 10);
        p = e;
        if (r.adj_lds_elems < 1024 || r.adj_lds_elems > 40960) return false;
    }
    if (*p) return false;
    int sx = 0, sy = 0;
    for (int i = 0; i < r.np; ++i) {
        if (r.kx[i] < 0 || r.ky[i] < 0 || r.kx[i] + r.ky[i] < 1) return false;
        if ((1 << (r.kx[i] + r.ky[i])) > kMaxPassSlots) return false;
        sx += r.kx[i];
        sy += r.ky[i];
    }
    if (r.np < 1 || sx != n || sy != n) return false;
    if (r.lds_elems < 1024 || r.lds_elems > 40960) return false;
    if (r.waves < 1 || r.waves > 16) return false;
    t = r;
    return true;
}

static std::mutex g_tune_mu;
static std::map<std::pair<int, int>, Tuning> g_tuning;  // (N, is_float) -> choice

static Tuning get_tuning(int N, int is_float)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuning.find({N, is_float});
    if (it != g_tuning.end()) return it->second;
    const int n = ilog2_exact(N);
    Tuning t = default_tuning(n, is_float);
    if (const char* path = getenv("DRT3D_TUNE_CACHE")) {
        if (FILE* fp = fopen(path, "r")) {
            char line[256];
            while (fgets(line, sizeof line, fp)) {  // the last matching line wins
                int fN = 0, ff = 0;
                char txt[200];
                if (sscanf(line, "%d %d %199s", &fN, &ff, txt) == 3 && fN == N && ff == is_float) {
                    Tuning c;
                    if (tuning_from_string(txt, n, c)) t = c;
                }
            }
            fclose(fp);
        }
    }
    g_tuning[{N, is_float}] = t;
    return t;
}

static void put_tuning(int N, int is_float, const Tuning& t)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuning[{N, is_float}] = t;
}

// ------------------------------------------------------------------ device
struct DeviceInfo {
    int cus = 256;
    int max_lds = 65536;
    int arch_ok = 0;
};
static std::mutex g_dev_mu;
static std::map<int, DeviceInfo> g_devs;

static int device_info(DeviceInfo& out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_dev_mu);
    auto it = g_devs.find(dev);
    if (it == g_devs.end()) {
        DeviceInfo di;
        hipDeviceProp_t prop;
        HIP_TRY(hipGetDeviceProperties(&prop, dev));
        di.cus = prop.multiProcessorCount;
        di.max_lds = (int)prop.sharedMemPerBlock;
        di.arch_ok = strncmp(prop.gcnArchName, "gfx950", 6) == 0;
        if (di.arch_ok && di.max_lds > 65536) {
            if (set_drt_lds_limit(0, di.max_lds) != hipSuccess || set_drt_lds_limit(1, di.max_lds) != hipSuccess)
                di.max_lds = 65536;
            (void)hipGetLastError();
        }
        it = g_devs.emplace(dev, di).first;
    }
    if (!it->second.arch_ok) return fail(DRT3D_EUNSUPPORTED, "this library is built for gfx950 (MI355X) only");
    out = it->second;
    return DRT3D_OK;
}

// ------------------------------------------------------------------ profiling
struct ProfRec {
    std::string name;
    hipEvent_t a, b;
    double bytes;
};
struct ProfSum {
    double ms = 0, bytes = 0;
    long long n = 0;
};
static std::mutex g_prof_mu;
static std::atomic<int> g_prof_on{0};
static std::vector<ProfRec> g_prof_pending;
static std::map<std::string, ProfSum> g_prof_sum;

static int prof_flush()
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto& r : g_prof_pending) {
        HIP_TRY(hipEventSynchronize(r.b));
        float ms = 0;
        HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b));
        ProfSum& s = g_prof_sum[r.name];
        s.ms += ms;
        s.bytes += r.bytes;
        s.n += 1;
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_prof_pending.clear();
    return DRT3D_OK;
}

// ------------------------------------------------------------------ programs
enum StepKind { S_DRT = 0, S_DJT = 1, S_TRANSPOSE = 2, S_SUM = 3 };

// Step keys: a step's position in its volume's sequence, the same for every
// volume of a batched call (forward transposes, passes, adjoint rounds,
// adjoint combines).
static const int kKeyTransY = 0, kKeyTransX = 1, kKeyPass = 10, kKeyRound = 40, kKeyCombine = 60;

struct Step {
    int kind = S_DRT;
    int key = 0;  // canonical position (batched merge key)
    std::string name;
    std::vector<DrtDesc> drt;
    std::vector<DjtDesc> djt;
    int waves = 4;     // wavefronts per work group
    int shape = 0;     // DRT: Kx | Ky << 4 | (L / 64) << 8 (launches merge only equal shapes)
    size_t lds = 0;    // dynamic LDS bytes
    double bytes = 0;  // algorithmic bytes (reads of inputs + writes of outputs)
    // transpose: out[b][c][r] (+)= in[b][r][c]
    const void* t_in = nullptr;
    void* t_out = nullptr;
    int t_R = 0, t_C = 0, t_batches = 0, t_add = 0;
    int t_bytes = 4;  // transpose element bytes (1: an 8-bit volume)
    // sum: t_out[i] = (t_add ? t_out[i] : 0) + sum over p < t_R of t_in[p * sum_n + i]
    long long sum_n = 0;
};

struct Launch {
    int kind;
    std::string name;
    int fast_kx = -1, fast_ky = -1, fast_nch = -1;  // shape-specialised DRT kernel, if any
    int fast_mode = 0;                              // ... 0 forward, 1 forward last pass, 2 adjoint
    int fast_sb = 4, fast_db = 4;                   // ... storage bytes of its source and destination
    int tr_bytes = 4;                               // transposes: element bytes
    int tr_wide = 0;                                // transposes: 128-byte tiles of 8-bit elements
    int adj_group = 0;                              // DRT: drt_adj_last_group (fast_nch chunks)
    int djt_k = 0, djt_ncc = 0, djt_nco = 0;        // DJT: stages fused per pass, LDS/output row chunks
    int djt_adj = 0;                                // DJT: the pass's transpose
    const void* sum_in = nullptr;                   // S_SUM
    void* sum_out = nullptr;
    int sum_parts = 0, sum_accum = 0;
    long long sum_n = 0;
    int first = 0, ndesc = 0;
    long long total_wg = 0;
    int persistent = 0;  // grid capped at a few work groups per CU, looping over the items
    int block = 64;
    size_t lds = 0;
    double bytes = 0;
};

struct Program {
    int is_float = 0;
    int persistent = 0;
    std::vector<DrtDesc> drt;
    std::vector<DjtDesc> djt;
    std::vector<TransDesc> tr;
    std::vector<Launch> launches;
    size_t drt_bytes() const { return align256(drt.size() * sizeof(DrtDesc)); }
    size_t djt_bytes() const { return align256(djt.size() * sizeof(DjtDesc)); }
    size_t desc_bytes() const { return drt_bytes() + djt_bytes() + align256(tr.size() * sizeof(TransDesc)); }
};

// Append the steps as launches, in order (single calls) or merged by key
// (batched calls: all steps with the same key form one launch). The passes of
// volumes marked `solo` are never merged: they run after the merged passes in
// per-volume order, so each volume's freshly written stage buffers are read
// while they may still sit in the memory-side cache. Their volume transposes
// still merge with everyone's: the forward's (keys below kKeyPass) open the
// program, the adjoint's (kKeyCombine and up) close it.
static void build_program(Program& prog, const std::vector<std::vector<Step>>& per_volume, bool merge,
                          const std::vector<char>* solo = nullptr)
{
    std::vector<const Step*> order;
    std::vector<char> mergeable;
    if (!merge) {
        for (auto& v : per_volume)
            for (auto& s : v) { order.push_back(&s); mergeable.push_back(0); }
    } else {
        std::map<int, std::vector<const Step*>> bykey;
        for (size_t i = 0; i < per_volume.size(); ++i) {
            const bool so = solo && (*solo)[i];
            for (auto& s : per_volume[i])
                if (!so || s.kind == S_TRANSPOSE) bykey[s.key].push_back(&s);
        }
        auto take = [&](bool post) {
            for (auto& kv : bykey)
                if ((kv.first >= kKeyCombine) == post)
                    for (auto* s : kv.second) { order.push_back(s); mergeable.push_back(1); }
        };
        take(false);
        if (solo)
            for (size_t i = 0; i < per_volume.size(); ++i)
                if ((*solo)[i])
                    for (auto& s : per_volume[i])
                        if (s.kind != S_TRANSPOSE) { order.push_back(&s); mergeable.push_back(0); }
        take(true);
    }
    size_t i = 0;
    while (i < order.size()) {
        const Step* s0 = order[i];
        size_t j = i + 1;
        if (mergeable[i] && s0->kind != S_SUM)
            while (j < order.size() && mergeable[j] && order[j]->key == s0->key && order[j]->kind == s0->kind &&
                   order[j]->shape == s0->shape)
                ++j;
        // the forward's volume transposes (keys below kKeyPass) all read
        // inputs and write distinct copies: one launch takes the run of them
        if (s0->kind == S_TRANSPOSE && s0->key < kKeyPass)
            while (j < order.size() && order[j]->kind == S_TRANSPOSE && order[j]->key < kKeyPass &&
                   order[j]->t_bytes == s0->t_bytes)
                ++j;
        Launch L;
        L.kind = s0->kind;
        L.name = s0->name;
        L.persistent = prog.persistent && mergeable[i];
        if (s0->kind == S_SUM) {
            L.sum_in = s0->t_in; L.sum_out = s0->t_out; L.sum_parts = s0->t_R; L.sum_accum = s0->t_add;
            L.sum_n = s0->sum_n; L.bytes = s0->bytes; L.block = 256;
            prog.launches.push_back(L);
            i = j;
            continue;
        }
        if (s0->kind == S_TRANSPOSE) {
            // steps of one key write different volumes: one launch is race-free
            L.tr_bytes = s0->t_bytes;
            L.first = (int)prog.tr.size();
            // 8-bit copies move 4-byte words when every row and base is whole words
            L.tr_wide = L.tr_bytes == 1;
            for (size_t q = i; q < j; ++q) {
                const Step* t = order[q];
                if (t->t_add || t->t_R % 4 || t->t_C % 4 || ((uintptr_t)t->t_in & 3) || ((uintptr_t)t->t_out & 3))
                    L.tr_wide = 0;
            }
            const int te = L.tr_wide ? 128 : 64;  // tile edge in elements
            long long wg = 0;
            for (size_t q = i; q < j; ++q) {
                const Step* t = order[q];
                TransDesc d{};
                d.wg_begin = wg;
                d.in = t->t_in; d.out = t->t_out; d.R = t->t_R; d.C = t->t_C;
                d.batches = t->t_batches; d.add = t->t_add;
                d.tiles_r = (t->t_R + te - 1) / te;
                d.tiles_c = (t->t_C + te - 1) / te;
                wg += (long long)d.tiles_r * d.tiles_c * d.batches;
                prog.tr.push_back(d);
                L.bytes += t->bytes;
            }
            L.ndesc = (int)prog.tr.size() - L.first;
            L.total_wg = wg;
            L.block = 256;
            prog.launches.push_back(L);
            i = j;
            continue;
        }
        int waves = 1;
        size_t lds = 0;
        double bytes = 0;
        long long wg = 0;
        L.first = s0->kind == S_DRT ? (int)prog.drt.size() : (int)prog.djt.size();
        for (size_t q = i; q < j; ++q) {
            const Step* s = order[q];
            waves = std::max(waves, s->waves);
            lds = std::max(lds, s->lds);
            bytes += s->bytes;
            if (s->kind == S_DRT) {
                for (DrtDesc d : s->drt) {
                    d.wg_begin = wg;
                    // a fused adjoint item covers a group's four dodecants; an
                    // 8-bit first pass packs two column groups per item
                    wg += ((long long)(d.fused_group ? d.nslots / 4 : d.nslots) * d.groups_x * d.groups_y) >>
                          (d.sb == 1 && d.db == 2 ? 1 : 0);
                    prog.drt.push_back(d);
                }
            } else {
                for (DjtDesc d : s->djt) {
                    d.wg_begin = wg;
                    // a transposed pass takes one tile per work item
                    wg += (long long)d.nslots * d.groups * ((s->shape >> 12) & 1 ? d.ntiles : 1);
                    prog.djt.push_back(d);
                    L.djt_k = d.K;
                    L.djt_ncc = (s->shape >> 4) & 15;
                    L.djt_nco = (s->shape >> 8) & 15;
                    L.djt_adj = s->shape >> 12;
                }
            }
        }
        L.ndesc = (s0->kind == S_DRT ? (int)prog.drt.size() : (int)prog.djt.size()) - L.first;
        L.total_wg = wg;
        L.block = 64 * waves;
        L.lds = lds;
        L.bytes = bytes;
        if (s0->kind == S_DRT && prog.drt[L.first].fused_group) {
            L.adj_group = 1;
            L.fast_kx = L.fast_ky = prog.drt[L.first].Kx;  // the fused kernel's K
            L.fast_nch = prog.drt[L.first].L >> 6;
        } else if (s0->kind == S_DRT && (L.block == 512 || L.block == 1024)) {
            // one shape across the launch's descriptors -> specialised kernel
            const DrtDesc& f = prog.drt[L.first];
            bool same = true, final_pass = true;
            for (int q = L.first; q < L.first + L.ndesc; ++q) {
                const DrtDesc& e = prog.drt[q];
                // the specialised kernel addresses each region with 32-bit
                // byte offsets: N <= 512 keeps every region below 2^31 bytes
                same = same && e.Kx == f.Kx && e.Ky == f.Ky && e.L == f.L && e.N <= 512 && e.adjoint == f.adjoint &&
                       e.sb == f.sb && e.db == f.db;
                final_pass = final_pass && !e.adjoint && e.dst_mode == 0 && e.nt_store;
            }
            const int mode = f.adjoint ? 2 : final_pass ? 1 : 0;
            const int fsb = f.sb ? f.sb : 4, fdb = f.db ? f.db : 4;
            if (same && (f.L & 63) == 0 && drt_fast_available(f.Kx, f.Ky, f.L >> 6, L.block / 64, mode, fsb, fdb)) {
                L.fast_kx = f.Kx;
                L.fast_ky = f.Ky;
                L.fast_nch = f.L >> 6;
                L.fast_mode = mode;
                L.fast_sb = fsb;
                L.fast_db = fdb;
            }
        }
        prog.launches.push_back(L);
        i = j;
    }
}

// Pinned staging ring for descriptor uploads (reused once its copy is done).
struct Staging {
    static constexpr int kSlots = 16;
    void* buf[kSlots] = {nullptr};
    size_t cap[kSlots] = {0};
    hipEvent_t ev[kSlots] = {nullptr};
    int next = 0;
};
static std::mutex g_stage_mu;
static std::map<int, Staging> g_stage;

static int upload_descs(const Program& p, void* d_area, hipStream_t s)
{
    const size_t bytes = p.desc_bytes();
    if (!bytes) return DRT3D_OK;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_stage_mu);
    Staging& st = g_stage[dev];
    const int i = st.next;
    st.next = (st.next + 1) % Staging::kSlots;
    if (st.ev[i]) HIP_TRY(hipEventSynchronize(st.ev[i]));
    else HIP_TRY(hipEventCreateWithFlags(&st.ev[i], hipEventDisableTiming));
    if (st.cap[i] < bytes) {
        if (st.buf[i]) HIP_TRY(hipHostFree(st.buf[i]));
        st.buf[i] = nullptr;
        st.cap[i] = 0;
        const size_t c = std::max(bytes, (size_t)1 << 20);
        HIP_TRY(hipHostMalloc(&st.buf[i], c, hipHostMallocDefault));
        st.cap[i] = c;
    }
    char* h = (char*)st.buf[i];
    memset(h, 0, bytes);
    if (!p.drt.empty()) memcpy(h, p.drt.data(), p.drt.size() * sizeof(DrtDesc));
    if (!p.djt.empty()) memcpy(h + p.drt_bytes(), p.djt.data(), p.djt.size() * sizeof(DjtDesc));
    if (!p.tr.empty())
        memcpy(h + p.drt_bytes() + p.djt_bytes(), p.tr.data(), p.tr.size() * sizeof(TransDesc));
    HIP_TRY(hipMemcpyAsync(d_area, h, bytes, hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(st.ev[i], s));
    return DRT3D_OK;
}

static int grid_for(long long total_wg, const DeviceInfo& di, int persistent)
{
    const long long cap = persistent ? (long long)di.cus * 8 : (1LL << 30);
    return (int)std::max(1LL, std::min(total_wg, cap));
}

// ------------------------------------------------------------------ no-allocation forward
// drt3d_forward_noalloc runs in the file-scope device array `scratch` instead
// of a caller's workspace. Each GPU holds its own copy from the library's load
// until the process ends. In host code the array's name is only a host-side
// stand-in: every kernel argument and copy uses the device address that
// hipGetSymbolAddress returns on each device (taken once per device, with that
// device current, and kept in g_scratch_ptr).
constexpr size_t kNoallocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];
static std::mutex g_scratch_mu;
static std::map<int, void*> g_scratch_ptr;

static int scratch_ptr(void** out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        void* ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(DRT3D_EHIP, "hipGetSymbolAddress gave no address for the static scratch");
        it = g_scratch_ptr.emplace(dev, ptr).first;
    }
    *out = it->second;
    return DRT3D_OK;
}

// Descriptor upload with no staging buffer: the bytes travel as the kernel
// arguments of a one-block copy kernel, kWordsPerPut words per launch.
constexpr int kWordsPerPut = 480;
struct WordPut {
    uint32_t n;
    uint32_t w[kWordsPerPut];
};

__global__ void __launch_bounds__(256) put_words_kernel(WordPut put, uint32_t* __restrict__ dst)
{
    for (uint32_t i = threadIdx.x; i < put.n; i += blockDim.x) dst[i] = put.w[i];
}

static int upload_descs_by_args(const Program& p, void* d_area, hipStream_t s)
{
    const size_t bytes = p.desc_bytes();
    if (!bytes) return DRT3D_OK;
    std::vector<uint32_t> words((bytes + 3) / 4, 0u);
    char* h = reinterpret_cast<char*>(words.data());
    if (!p.drt.empty()) memcpy(h, p.drt.data(), p.drt.size() * sizeof(DrtDesc));
    if (!p.djt.empty()) memcpy(h + p.drt_bytes(), p.djt.data(), p.djt.size() * sizeof(DjtDesc));
    if (!p.tr.empty())
        memcpy(h + p.drt_bytes() + p.djt_bytes(), p.tr.data(), p.tr.size() * sizeof(TransDesc));
    WordPut put;
    for (size_t w0 = 0; w0 < words.size(); w0 += kWordsPerPut) {
        put.n = (uint32_t)std::min<size_t>(kWordsPerPut, words.size() - w0);
        memcpy(put.w, words.data() + w0, put.n * sizeof(uint32_t));
        hipLaunchKernelGGL(put_words_kernel, dim3(1), dim3(256), 0, s, put, reinterpret_cast<uint32_t*>(d_area) + w0);
        HIP_TRY(hipGetLastError());
    }
    return DRT3D_OK;
}

// allow_prof = false: no events are created or recorded (the no-allocation path)
static int run_launches(const Program& p, void* d_area, hipStream_t s, const DeviceInfo& di, bool allow_prof = true)
{
    const DrtDesc* d_drt = reinterpret_cast<const DrtDesc*>(d_area);
    const DjtDesc* d_djt = reinterpret_cast<const DjtDesc*>((char*)d_area + p.drt_bytes());
    const TransDesc* d_tr = reinterpret_cast<const TransDesc*>((char*)d_area + p.drt_bytes() + p.djt_bytes());
    const bool prof = allow_prof && g_prof_on.load() != 0;
    for (const Launch& L : p.launches) {
        hipEvent_t ea = nullptr, eb = nullptr;
        if (prof) {
            HIP_TRY(hipEventCreate(&ea));
            HIP_TRY(hipEventCreate(&eb));
            HIP_TRY(hipEventRecord(ea, s));
        }
        hipError_t e = hipSuccess;
        if (L.kind == S_DRT) {
            if (L.lds > (size_t)di.max_lds)
                return fail(DRT3D_EINVAL, "%s needs %zu bytes of LDS, the device allows %d", L.name.c_str(), L.lds,
                            di.max_lds);
            if (L.adj_group)
                e = launch_drt_adj_group(p.is_float, L.fast_kx, L.fast_nch, L.block / 64, d_drt + L.first, L.ndesc,
                                         L.total_wg, grid_for(L.total_wg, di, L.persistent), L.lds, s);
            else if (L.fast_kx >= 0)
                e = launch_drt_fast(p.is_float, L.fast_kx, L.fast_ky, L.fast_nch, L.fast_mode, L.block / 64, d_drt + L.first, L.ndesc,
                                    L.total_wg, grid_for(L.total_wg, di, L.persistent), L.lds, s, L.fast_sb, L.fast_db);
            else
                e = launch_drt_pass(p.is_float, d_drt + L.first, L.ndesc, L.total_wg, L.block,
                                    grid_for(L.total_wg, di, L.persistent), L.lds, s);
        } else if (L.kind == S_DJT) {
            if (L.lds > (size_t)di.max_lds)
                return fail(DRT3D_EINVAL, "%s needs %zu bytes of LDS, the device allows %d", L.name.c_str(), L.lds,
                            di.max_lds);
            if (L.djt_adj)
                e = launch_djt_adj(p.is_float, L.djt_k, L.djt_ncc, d_djt + L.first, L.ndesc, L.total_wg,
                                   grid_for(L.total_wg, di, L.persistent), L.lds, s);
            else
                e = launch_djt_pass(p.is_float, L.djt_k, L.djt_ncc, L.djt_nco, d_djt + L.first, L.ndesc, L.total_wg,
                                    grid_for(L.total_wg, di, L.persistent), L.lds, s);
        } else if (L.kind == S_SUM) {
            e = launch_sum_parts(p.is_float, L.sum_in, L.sum_parts, L.sum_out, L.sum_n, L.sum_accum, s);
        } else if (L.tr_bytes == 1) {
            e = launch_transpose_u8(d_tr + L.first, L.ndesc, L.total_wg, L.tr_wide, s);
        } else {
            e = launch_transpose(p.is_float, d_tr + L.first, L.ndesc, L.total_wg, s);
        }
        if (e != hipSuccess)
            return fail(DRT3D_EHIP, "launch of %s failed: %s", L.name.c_str(), hipGetErrorString(e));
        if (prof) {
            HIP_TRY(hipEventRecord(eb, s));
            std::lock_guard<std::mutex> lk(g_prof_mu);
            g_prof_pending.push_back({L.name, ea, eb, L.bytes});
        }
    }
    return DRT3D_OK;
}

// ------------------------------------------------------------------ DRT plan
struct PassGeom {
    int mx0, Kx, my0, Ky;  // stage ranges of the pass
    int E_in, E_out;       // forward extents: N + (2^mx - 1) + (2^my - 1)
};

static std::vector<PassGeom> drt_passes(int N, const Tuning& t)
{
    std::vector<PassGeom> v;
    int mx = 0, my = 0;
    for (int i = 0; i < t.np; ++i) {
        PassGeom g;
        g.mx0 = mx; g.Kx = t.kx[i]; g.my0 = my; g.Ky = t.ky[i];
        g.E_in = N + (1 << mx) - 1 + (1 << my) - 1;
        mx += t.kx[i];
        my += t.ky[i];
        g.E_out = N + (1 << mx) - 1 + (1 << my) - 1;
        v.push_back(g);
    }
    return v;
}

// Largest extent of any intermediate (non-final) pass output over every
// admissible pass list, so that buffer sizes never depend on the tuning.
static long long max_intermediate_extent(int N)
{
    const int n = ilog2_exact(N);
    if (n <= 1) return 2LL * N - 1;
    return 2LL * N + (1LL << (n - 1)) - 2;  // all of one axis, all but one stage of the other
}

// Intermediate columns are padded to 32 elements so that each starts on a
// 128-byte line.
static long long drt_stage_elems_per_dod(int N) { return (long long)N * N * round32(max_intermediate_extent(N)); }

static const long long kStageBudget = 16LL << 30;  // stage-buffer bytes of one single-volume call

static int chunk_size(long long per_dod_bytes, int ndod)
{
    const long long c = std::max(1LL, kStageBudget / std::max(1LL, per_dod_bytes));
    return (int)std::min<long long>(ndod, c);
}

// Tile choice of one pass: T (tile width of the displacement written), H
// (local halo), L (LDS column length, a multiple of 64), pad (zeros between
// LDS columns, covering the largest shift of a step), ntiles. The LDS of a
// work item is nslot * (L + pad) + pad elements. The adjoint's outputs are
// skewed by up to `skew`, so it needs extra tiles.
static int pass_pad(const PassGeom& g)
{
    // largest step shift: (2^(Kx-1) - 1) + (2^(Ky-1) - 1) + 2 <= H/2 + 2
    const int H = ((1 << g.Kx) - 1) + ((1 << g.Ky) - 1);
    const int need = H / 2 + 2;
    return need <= 16 ? 16 : need <= 32 ? 32 : 64;
}

static long long lds_elems_of(int nslot, int L, int pad) { return (long long)nslot * (L + pad) + pad; }

// Longest LDS column the shape-specialised kernels of a (Kx, Ky) pass take
// (0: the shape has none). Longer columns would fall back to the generic kernel.
static int fast_max_L(const PassGeom& g)
{
    for (int nch = 16; nch >= 1; --nch)
        if (drt_fast_available(g.Kx, g.Ky, nch, 8)) return 64 * nch;
    return 0;
}

// halign: the halo H rounded up to a multiple of it (every tile then starts
// on a multiple of it, as the 8-bit first pass's word loads need; a larger
// halo only computes a few more positions that the tile drops).
static bool choose_tiles(const PassGeom& g, int adjoint, int lds_elems, int& T, int& H, int& L, int& ntiles,
                         int halign = 1)
{
    const int ns = 1 << (g.Kx + g.Ky);
    if (ns > kMaxPassSlots) return false;
    H = ((1 << g.Kx) - 1) + ((1 << g.Ky) - 1);
    const int pad = pass_pad(g);
    if (H / 2 + 2 > pad) return false;
    H = (H + halign - 1) / halign * halign;
    const int E = adjoint ? g.E_in : g.E_out;  // extent written
    const int skew = adjoint ? ((1 << g.mx0) - 1) * ((1 << g.Kx) - 1) + ((1 << g.my0) - 1) * ((1 << g.Ky) - 1) : 0;
    const int span = E + skew;
    int Lmax = (int)(((lds_elems - pad) / ns - pad) & ~63LL);
    const int Lfast = fast_max_L(g);
    if (Lfast > 0 && Lmax > Lfast && Lfast - H >= 32) Lmax = Lfast;
    if (Lmax - H < 32) return false;  // tiles of at least one 128-byte line
    ntiles = (span + (Lmax - H) - 1) / (Lmax - H);
    const int Tmin = (span + ntiles - 1) / ntiles;
    L = (Tmin + H + 63) & ~63;
    T = L - H;
    ntiles = (span + T - 1) / T;
    return lds_elems_of(ns, L, pad) <= lds_elems;
}


struct DrtIO {
    const void* in;   // forward: volume; adjoint: projection
    void* out;        // forward: projection; adjoint: volume
    char* ws;         // workspace base for this volume's buffers (after descriptors)
};

static size_t drt_ws_volume_bytes(int N, uint32_t mask, int elem, int adjoint, int chunked)
{
    const int nd = popcount12(mask);
    bool g1 = false, g2 = false;
    for (int k = 0; k < 12; ++k)
        if ((mask >> k) & 1) { g1 |= drt_group(k) == 1; g2 |= drt_group(k) == 2; }
    const size_t vol = (size_t)N * N * N * elem;
    const long long per = drt_stage_elems_per_dod(N) * elem;
    const int c = chunked ? chunk_size(2 * per, nd) : nd;
    size_t b = 0;
    b += g1 ? align256(vol) : 0;  // V_Y (forward) or the y-group accumulator (adjoint)
    b += g2 ? align256(vol) : 0;
    b += 2 * align256((size_t)c * per);
    (void)adjoint;
    return b;
}

// Steps of one DRT forward or adjoint over the dodecants of `mask`.
// narrow: the volume is 8-bit (forward only); the first pass writes 16-bit
// partial sums, later passes 32-bit (see drt_pass_fast's SB, DB).
static int drt_steps(std::vector<Step>& steps, int N, uint32_t mask, int is_float, int adjoint, int chunked,
                     const Tuning& t, const DrtIO& io, int narrow = 0)
{
    const int n = ilog2_exact(N);
    const int elem = 4;
    const int nd = popcount12(mask);
    // dodecants grouped by the volume layout they read (z-, y-, x-normal),
    // increasing k inside a group; mrank[k] is k's place in the caller's
    // projections (increasing k over the mask)
    int dods[12], nd2 = 0, mrank[12] = {0}, gcount[3] = {0, 0, 0};
    for (int k = 0, r = 0; k < 12; ++k)
        if ((mask >> k) & 1) mrank[k] = r++;
    for (int g = 0; g < 3; ++g)
        for (int k = 0; k < 12; ++k)
            if (((mask >> k) & 1) && drt_group(k) == g) { dods[nd2++] = k; ++gcount[g]; }
    bool has[3] = {false, false, false};
    for (int i = 0; i < nd; ++i) has[drt_group(dods[i])] = true;
    const size_t vol_bytes = (size_t)N * N * N * elem;
    const long long per = drt_stage_elems_per_dod(N);  // the workspace's bound per dodecant
    const int chunk_ws = chunked ? chunk_size(2 * per * elem, nd) : nd;
    const std::vector<PassGeom> P = drt_passes(N, t);
    const int np = (int)P.size();
    if (narrow && adjoint) return fail(DRT3D_EUNSUPPORTED, "8-bit volumes are taken by the forward only");
    // storage bytes of pass i's source and destination, and the pitch of the
    // stage it writes: columns start on 128-byte lines (32 elements, or 64 of
    // the first stage's 16-bit ones)
    auto src_bytes = [&](int i) { return !narrow ? 4 : i == 0 ? 1 : i == 1 ? 2 : 4; };
    auto dst_bytes = [&](int i) { return !narrow || i == np - 1 ? 4 : i == 0 ? 2 : 4; };
    auto pitch_of = [&](int i) { return dst_bytes(i) == 2 ? (P[i].E_out + 63) & ~63LL : round32(P[i].E_out); };
    // stage elements per dodecant of this tuning
    long long per_t = 1;
    for (int i = 0; i + 1 < np; ++i) per_t = std::max(per_t, (long long)N * N * pitch_of(i));
    if (per_t > per) return fail(DRT3D_EUNSUPPORTED, "stage pitches of this tuning exceed the workspace bound");
    int chunk = (int)std::min<long long>(nd, chunk_ws * per / per_t);
    // whole layout groups per chunk when every group present has all four
    // dodecants: the first pass then shares each group's loads (xcd_run)
    const bool runs4 = (gcount[0] == 0 || gcount[0] == 4) && (gcount[1] == 0 || gcount[1] == 4) &&
                       (gcount[2] == 0 || gcount[2] == 4);
    if (runs4 && chunk >= 4 && !adjoint) chunk -= chunk % 4;
    // The adjoint's last pass (the forward's first, transposed) adds the
    // dodecants of each volume layout group into one volume. When every group
    // present is whole in a single chunk and that pass is square (2.2 or 3.3,
    // eight wavefronts, or sixteen for 3.3), one fused launch sums each
    // group's four dodecants per block (slots in group order); otherwise it runs in rounds, one dodecant of
    // each group per round, and mixing the groups inside a chunk makes fewer,
    // fuller rounds.
    bool fuse_last = false;
    int fuse_waves = 8;
    if (adjoint) {
        const PassGeom& g0 = P[0];
        int T0, H0, L0, nt0;
        int w0 = std::min(t.waves, std::max(1, 1 << (g0.Kx + g0.Ky - 1)));
        if (w0 > 8 && !(g0.Kx == 3 && g0.Ky == 3)) w0 = 8;
        // the tile widths whose sums fit the fused kernel's register budget
        // without spilling (3.3: 80 registers at eight wavefronts, 64 at
        // sixteen; 2.2 keeps 2 columns per wave)
        auto fused_fits = [&](int K, int waves, int nch) {
            if (K == 2) return nch <= 6;
            return waves == 8 ? nch <= 3 : (nch != 2 && nch <= 5);
        };
        // (its volume and slot byte offsets are 32-bit: N <= 512)
        fuse_last = N <= 512 && runs4 && chunk == nd && g0.Kx == g0.Ky && (g0.Kx == 2 || g0.Kx == 3) && (w0 == 8 || w0 == 16) &&
                    choose_tiles(g0, 1, t.lds_elems, T0, H0, L0, nt0) && (L0 & 63) == 0 &&
                    fused_fits(g0.Kx, w0, L0 >> 6) && drt_adj_group_kernel(is_float, g0.Kx, L0 >> 6, w0) != nullptr;
        fuse_waves = w0;
        if (!fuse_last) {
            int by[3][4], c[3] = {0, 0, 0}, q = 0;
            for (int i = 0; i < nd; ++i) { const int g = drt_group(dods[i]); by[g][c[g]++] = dods[i]; }
            for (int r = 0; r < 4; ++r)
                for (int g = 0; g < 3; ++g)
                    if (r < c[g]) dods[q++] = by[g][r];
        }
    }

    char* w = io.ws;
    void* V[3] = {nullptr, nullptr, nullptr};
    V[0] = adjoint ? io.out : const_cast<void*>(io.in);
    if (has[1]) { V[1] = w; w += align256(vol_bytes); }
    if (has[2]) { V[2] = w; w += align256(vol_bytes); }
    void* S[2];
    S[0] = w; w += align256((size_t)chunk_ws * per * elem);
    S[1] = w;

    const long long out_pitch = 3LL * N - 2;
    const long long slot_out = (long long)N * N * out_pitch;

    // forward: the y- and x-normal copies of the volume
    if (!adjoint) {
        const int vb = narrow ? 1 : 4;
        if (has[1]) {  // V_Y[x][z][y] = vol[x][y][z]
            Step s; s.kind = S_TRANSPOSE; s.key = kKeyTransY; s.name = "transpose_in";
            s.t_in = io.in; s.t_out = V[1]; s.t_R = N; s.t_C = N; s.t_batches = N; s.t_add = 0;
            s.t_bytes = vb;
            s.bytes = 2.0 * vb * N * N * N;
            steps.push_back(s);
        }
        if (has[2]) {  // V_X[(y,z)][x] = vol[x][(y,z)]
            Step s; s.kind = S_TRANSPOSE; s.key = kKeyTransX; s.name = "transpose_in";
            s.t_in = io.in; s.t_out = V[2]; s.t_R = N; s.t_C = N * N; s.t_batches = 1; s.t_add = 0;
            s.t_bytes = vb;
            s.bytes = 2.0 * vb * N * N * N;
            steps.push_back(s);
        }
    }

    bool seen_group[3] = {false, false, false};
    for (int c0 = 0; c0 < nd; c0 += chunk) {
        const int ns = std::min(chunk, nd - c0);
        for (int step = 0; step < np; ++step) {
            const int pi = adjoint ? np - 1 - step : step;
            const PassGeom& g = P[pi];
            DrtDesc d{};
            d.N = N; d.n = n; d.adjoint = adjoint;
            d.mx0 = g.mx0; d.Kx = g.Kx; d.my0 = g.my0; d.Ky = g.Ky;
            int T, H, L, ntl;
            const int pass_lds = adjoint && !(step == np - 1 && fuse_last) ? adj_lds_of(t) : t.lds_elems;
            if (!choose_tiles(g, adjoint, pass_lds, T, H, L, ntl, !adjoint && src_bytes(pi) == 1 ? 4 : 1))
                return fail(DRT3D_EINVAL, "tuning %s cannot fit pass %d in LDS", tuning_to_string(t).c_str(), pi);
            d.T = T; d.H = H; d.L = L; d.Lp = L + pass_pad(g); d.ntiles = ntl;
            d.groups_x = N >> g.Kx;
            d.groups_y = N >> g.Ky;
            d.nslots = ns;
            d.E_in = adjoint ? g.E_out : g.E_in;
            d.E_out = adjoint ? g.E_in : g.E_out;
            d.sb = adjoint ? 4 : src_bytes(pi);
            d.db = adjoint ? 4 : dst_bytes(pi);
            const bool first = step == 0, last = step == np - 1;
            for (int s = 0; s < ns; ++s) {
                const int k = dods[c0 + s];
                d.fm[s] = drt_frame_map(k, N);
                d.phys[s] = first && adjoint ? mrank[k] : s;   // projections or stage slots
                d.dphys[s] = last && !adjoint ? mrank[k] : s;  // projections or stage slots
            }
            if (first && !adjoint) {
                d.src_mode = 1;
                for (int i = 0; i < 3; ++i) d.vsrc[i] = V[i];
                const int items = ((N >> g.Kx) * (N >> g.Ky)) >> (d.sb == 1 && d.db == 2 ? 1 : 0);  // per slot
                if (runs4 && ns % 4 == 0 && g.Kx == g.Ky && items % 8 == 0) d.xcd_run = 4;
            } else if (first) {
                d.src = io.in;
                d.src_slot_stride = slot_out;
                d.P_in = (int)out_pitch;
            } else {
                d.src = S[(step - 1) & 1];
                d.src_slot_stride = per_t;
                d.P_in = adjoint ? (int)round32(d.E_in) : (int)pitch_of(pi - 1);
            }
            if (last && !adjoint) {
                d.dst = io.out;
                d.dst_slot_stride = slot_out;
                d.P_out = (int)out_pitch;
                d.nt_store = 1;  // the caller's output is not read back here
            } else if (last) {
                d.dst_mode = 1;
                for (int i = 0; i < 3; ++i) d.vdst[i] = V[i];
            } else {
                d.dst = S[step & 1];
                d.dst_slot_stride = per_t;
                d.P_out = adjoint ? (int)round32(d.E_out) : (int)pitch_of(pi);
            }
            const int K = g.Kx + g.Ky;
            int waves = std::min(t.waves, std::max(1, 1 << (K - 1)));
            // 16 wavefronts only for the shape that has such a kernel
            if (waves > 8 && !(g.Kx == 3 && g.Ky == 3 && drt_fast_available(3, 3, L >> 6, 16))) waves = 8;
            const size_t lds = (size_t)lds_elems_of(1 << K, L, pass_pad(g)) * elem;
            const double cols = (double)N * N;
            char nm[32];
            snprintf(nm, sizeof nm, "drt_%s_p%d", adjoint ? "adj" : "fwd", pi + 1);
            const int shape = g.Kx | (g.Ky << 4) | ((L >> 6) << 8) | (d.sb << 16) | (d.db << 20);
            if (last && adjoint && fuse_last) {
                d.fused_group = 1;
                Step s; s.kind = S_DRT; s.key = kKeyRound; s.name = nm;
                s.waves = fuse_waves; s.lds = lds; s.shape = shape | (1 << 24);
                s.bytes = cols * elem * ((double)ns * d.E_in + (double)(ns / 4) * d.E_out);
                s.drt.push_back(d);
                steps.push_back(s);
            } else if (!(last && adjoint)) {
                Step s; s.kind = S_DRT; s.key = kKeyPass + step; s.name = nm;
                s.waves = waves; s.lds = lds; s.shape = shape;
                s.bytes = (double)ns * cols *
                          ((first && !adjoint ? (double)N : (double)d.E_in) * d.sb + (double)d.E_out * d.db);
                s.drt.push_back(d);
                steps.push_back(s);
            } else {
                // slots of one frame group add into the same volume: one
                // launch per rank within the group keeps the adds ordered
                int rank[kMaxSlots], cnt[3] = {0, 0, 0}, nr = 0;
                for (int s = 0; s < ns; ++s) {
                    rank[s] = cnt[d.fm[s].group]++;
                    nr = std::max(nr, rank[s] + 1);
                }
                for (int r = 0; r < nr; ++r) {
                    DrtDesc e = d;
                    int k = 0;
                    for (int s = 0; s < ns; ++s) {
                        if (rank[s] != r) continue;
                        const int grp = d.fm[s].group;
                        e.phys[k] = d.phys[s];
                        e.dphys[k] = d.dphys[s];
                        e.fm[k] = d.fm[s];
                        e.accum[k] = seen_group[grp] ? 1 : 0;
                        seen_group[grp] = true;
                        ++k;
                    }
                    e.nslots = k;
                    Step s; s.kind = S_DRT; s.key = kKeyRound + r; s.name = nm;
                    s.waves = waves; s.lds = lds; s.shape = shape;
                    double acc_reads = 0;
                    for (int q = 0; q < k; ++q) acc_reads += e.accum[q] ? (double)N : 0.0;
                    s.bytes = cols * elem * ((double)k * (d.E_in + d.E_out) + acc_reads);
                    s.drt.push_back(e);
                    steps.push_back(s);
                }
            }
        }
    }
    if (adjoint) {
        // accumulators of the y- and x-normal groups back into [x][y][z]
        bool written = has[0];
        if (has[1]) {
            Step s; s.kind = S_TRANSPOSE; s.key = kKeyCombine; s.name = "transpose_out";
            s.t_in = V[1]; s.t_out = io.out; s.t_R = N; s.t_C = N; s.t_batches = N; s.t_add = written;
            s.bytes = (written ? 3.0 : 2.0) * vol_bytes;
            steps.push_back(s);
            written = true;
        }
        if (has[2]) {
            Step s; s.kind = S_TRANSPOSE; s.key = kKeyCombine + 1; s.name = "transpose_out";
            s.t_in = V[2]; s.t_out = io.out; s.t_R = N * N; s.t_C = N; s.t_batches = 1; s.t_add = written;
            s.bytes = (written ? 3.0 : 2.0) * vol_bytes;
            steps.push_back(s);
        }
    }
    return DRT3D_OK;
}

// ------------------------------------------------------------------ DJT plan
static long long djt_extent(int N, int m) { return (long long)N + (1LL << m) - 1; }

// Stages per DJT pass, in order: 2 per pass, and a first pass of 1 when n is
// odd. Measured on the int32 forward (ms; adjoint within 1 %): N = 128
// 1,2,2,2 13.6 against 3,2,2 14.7, 2,3,2 14.3, 3,3,1 21.4, 2,2,2,1 19.4;
// N = 64 2,2,2 1.07 against 3,1,2 1.21; N = 32 1,2,2 0.15 against 3,2 0.20.
// A 3-stage pass holds 8 planes of a group in LDS and writes 64, so it
// runs fewer work groups per CU; a 1-stage last pass doubles the largest
// stage buffer.
static std::vector<int> djt_plan(int n)
{
    std::vector<int> ks;
    // DRT3D_DJT_PASSES="k1,k2,..." (each 1..3, summing to n) overrides the rule
    if (const char* env = getenv("DRT3D_DJT_PASSES")) {
        int sum = 0;
        bool ok = true;
        for (const char* p = env; *p; ++p) {
            if (*p == ',') continue;
            if (*p < '1' || *p > '3') { ok = false; break; }
            ks.push_back(*p - '0');
            sum += *p - '0';
        }
        if (ok && sum == n && !ks.empty()) return ks;
        ks.clear();
    }
    if (n & 1) ks.push_back(1);
    for (int i = n & 1; i < n; i += 2) ks.push_back(2);
    return ks;
}

// Elements of one dodecant's stage-m buffer (2^m slope pairs of N >> m blocks
// ... = N * 2^m planes of E_m x E_m).
static long long djt_stage_elems(int N, int m)
{
    const long long E = djt_extent(N, m);
    return (long long)N * (1LL << m) * E * E;
}

// Ping-pong buffer sizes (elements per dodecant) for the outputs of every
// pass but the last.
static void djt_buffer_elems(int N, long long& a, long long& b)
{
    const std::vector<int> ks = djt_plan(ilog2_exact(N));
    a = 0; b = 0;
    int m = 0;
    for (size_t i = 0; i + 1 < ks.size(); ++i) {
        m += ks[i];
        const long long e = djt_stage_elems(N, m);
        if (i & 1) b = std::max(b, e); else a = std::max(a, e);
    }
}

// Per-dodecant workspace of the DJT: the two stage buffers, plus (adjoint) the
// dodecant's own N^3 volume before the dodecants are summed.
static long long djt_per_dod_elems(int N, int adjoint)
{
    long long a, b;
    djt_buffer_elems(N, a, b);
    return a + b + (adjoint ? (long long)N * N * N : 0);
}

static size_t djt_ws_volume_bytes(int N, uint32_t mask, int elem, int chunked, int adjoint = 0)
{
    long long a, b;
    djt_buffer_elems(N, a, b);
    const int nd = popcount12(mask);
    const int c = chunked ? chunk_size(djt_per_dod_elems(N, adjoint) * elem, nd) : nd;
    size_t bytes = align256((size_t)c * a * elem) + align256((size_t)c * b * elem);
    if (adjoint) bytes += align256((size_t)c * N * N * N * elem);
    return bytes;
}

// Steps of one DJT forward, or of its adjoint: the same passes transposed and
// in reverse order, each dodecant backprojected into its own volume and the
// volumes summed into the caller's.
static int djt_steps(std::vector<Step>& steps, int N, uint32_t mask, int chunked, const DrtIO& io, int adjoint = 0)
{
    const int n = ilog2_exact(N);
    const int elem = 4;
    const int nd = popcount12(mask);
    int dods[12], q = 0;
    for (int k = 0; k < 12; ++k)
        if ((mask >> k) & 1) dods[q++] = k;
    long long A, B;
    djt_buffer_elems(N, A, B);
    const int chunk = chunked ? chunk_size(djt_per_dod_elems(N, adjoint) * elem, nd) : nd;
    char* w = io.ws;
    void* buf[2];
    buf[0] = w; w += align256((size_t)chunk * A * elem);
    buf[1] = w; w += align256((size_t)chunk * B * elem);
    void* vparts = w;  // adjoint: [chunk][N^3]
    const long long nvox = (long long)N * N * N;
    const std::vector<int> ks = djt_plan(n);
    const int np = (int)ks.size();
    const long long Ef = 2LL * N - 1;
    const long long slot_out = (long long)N * N * Ef * Ef;
    for (int c0 = 0; c0 < nd; c0 += chunk) {
        const int ns = std::min(chunk, nd - c0);
        std::vector<int> m0s(np);
        for (int i = 0, m = 0; i < np; ++i) { m0s[i] = m; m += ks[i]; }
        for (int step = 0; step < np; ++step) {
            const int i = adjoint ? np - 1 - step : step;  // the forward pass this step runs or transposes
            const int K = ks[i], m0 = m0s[i];
            const int NB = 1 << K, H = NB - 1;
            DjtDesc d{};
            d.N = N; d.n = n; d.m0 = m0; d.K = K;
            d.E_in = (int)djt_extent(N, m0);
            d.E_out = (int)djt_extent(N, m0 + K);
            d.P = d.E_out + H;
            // the adjoint's window rows hold E_out columns: every read whose
            // sum is written, at column c + loc(j, B) with c < E_in + s2 j,
            // stays below E_in + 2^m0 H + H - 1 = E_out - 1
            const int ncc = adjoint ? djt_adj_chunks_for(d.E_out) : djt_chunks_for(d.P);
            if (ncc == 0) return fail(DRT3D_EUNSUPPORTED, "the DJT is built for N <= 256 (got N = %d)", N);
            d.T1 = adjoint ? djt_adj_tile_rows() : djt_tile_rows(K);
            d.ntiles = (d.E_out + d.T1 - 1) / d.T1;
            d.groups = (1 << (2 * m0)) * (N >> (m0 + K));
            d.nslots = ns;
            for (int s = 0; s < ns; ++s) d.fm[s] = djt_frame_map(dods[c0 + s], N);
            // the forward pass i reads `in` and writes `out`; its transpose the reverse
            const void* in_p;
            void* out_p;
            long long in_stride, out_stride;
            if (i == 0) { in_p = io.in; in_stride = 0; }
            else { in_p = buf[(i - 1) & 1]; in_stride = (i - 1) & 1 ? B : A; }
            if (i == np - 1) { out_p = (char*)io.out + (size_t)c0 * slot_out * elem; out_stride = slot_out; }
            else { out_p = buf[i & 1]; out_stride = i & 1 ? B : A; }
            if (adjoint) {
                // reads what the forward pass writes (the caller's projections
                // for the last), writes what it reads (each dodecant's own
                // volume for the first)
                d.src = i == np - 1 ? (const char*)io.in + (size_t)c0 * slot_out * elem : out_p;
                d.src_slot_stride = out_stride;
                if (i == 0) {
                    d.dst_mode = 1;
                    d.dst = vparts;
                    d.dst_slot_stride = nvox;
                } else {
                    d.dst = const_cast<void*>(in_p);
                    d.dst_slot_stride = in_stride;
                }
                d.final_stage = i == np - 1;
            } else {
                d.src_mode = i == 0;
                d.src = in_p;
                d.src_slot_stride = in_stride;
                d.dst = out_p;
                d.dst_slot_stride = out_stride;
                d.final_stage = i == np - 1;
            }
            char nm[32];
            snprintf(nm, sizeof nm, adjoint ? "djt_adj_p%d" : "djt_p%d", i + 1);
            Step st; st.kind = S_DJT; st.key = kKeyPass + step; st.name = nm;
            st.waves = 8;
            // output chunks: a kernel with one chunk fewer than the LDS row
            // exists; otherwise the extra chunks are masked stores
            const int nco = (d.E_out + 63) / 64 == ncc - 1 ? ncc - 1 : ncc;
            st.shape = K | ncc << 4 | nco << 8 | adjoint << 12;
            st.lds = adjoint ? djt_adj_lds_bytes(K, ncc) : (size_t)NB * (d.T1 + H) * d.P * elem;
            const double in_e = i == 0 ? (double)N * N * N : (double)djt_stage_elems(N, m0);
            // the transpose of the last pass reads only the support e <= N-1+s
            // of each slope: (sum over s of N + s)^2 of the (2N-1)^2 entries
            const double sup = (double)N * N + (double)N * (N - 1) / 2;
            const double out_e = adjoint && i == np - 1 ? sup * sup : (double)djt_stage_elems(N, m0 + K);
            st.bytes = (double)ns * elem * (in_e + out_e);
            st.djt.push_back(d);
            steps.push_back(st);
        }
        if (adjoint) {
            Step st; st.kind = S_SUM; st.key = kKeyCombine; st.name = "djt_adj_sum";
            st.t_in = vparts; st.t_out = io.out; st.t_R = ns; st.t_add = c0 > 0; st.sum_n = nvox;
            st.bytes = (double)(ns + 1 + (c0 > 0)) * nvox * elem;
            steps.push_back(st);
        }
    }
    return DRT3D_OK;
}

// ------------------------------------------------------------------ graphs
// At most kMaxGraphs executable graphs are kept; the least recently used one
// is destroyed to make room, once its last replay has finished.
struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;  // recorded after each replay
    unsigned long long last_use = 0;
};
static constexpr size_t kMaxGraphs = 32;
static std::mutex g_graph_mu;
static std::map<std::string, GraphEntry> g_graphs;
static unsigned long long g_graph_clock = 0;

static std::string program_signature(const Program& p, void* d_area, int dev)
{
    std::string sig;
    char buf[128];
    snprintf(buf, sizeof buf, "%d|%p|%d|", dev, d_area, p.is_float);
    sig += buf;
    for (const Launch& L : p.launches) {
        snprintf(buf, sizeof buf, "%d:%d:%d:%lld:%d:%d:%zu:%d.%d.%d:%d%d%d%d:%d%d%d;", L.kind, L.first, L.ndesc,
                 L.total_wg, L.persistent, L.block, L.lds, L.fast_kx, L.fast_ky, L.fast_nch + 8 * L.fast_mode, L.djt_k,
                 L.djt_ncc, L.djt_nco, L.djt_adj, L.fast_sb, L.fast_db, L.tr_bytes + 8 * L.adj_group + 16 * L.tr_wide);
        sig += buf;
        if (L.kind == S_SUM) {
            snprintf(buf, sizeof buf, "%p>%p:%d:%d:%lld;", L.sum_in, L.sum_out, L.sum_parts, L.sum_accum, L.sum_n);
            sig += buf;
        }
    }
    return sig;
}

// Replays a cached graph of the program's launches, capturing it on a miss.
// Descriptors are uploaded before the replay; kernel arguments only hold the
// descriptor area, so a graph stays valid while the workspace does.
static int run_graph(const Program& p, void* d_area, hipStream_t s, const DeviceInfo& di)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    const std::string sig = program_signature(p, d_area, dev);
    std::lock_guard<std::mutex> lk(g_graph_mu);
    auto it = g_graphs.find(sig);
    if (it == g_graphs.end()) {
        if (g_graphs.size() >= kMaxGraphs) {
            auto lru = g_graphs.begin();
            for (auto q = g_graphs.begin(); q != g_graphs.end(); ++q)
                if (q->second.last_use < lru->second.last_use) lru = q;
            if (lru->second.done) HIP_TRY(hipEventSynchronize(lru->second.done));
            HIP_TRY(hipGraphExecDestroy(lru->second.exec));
            if (lru->second.done) (void)hipEventDestroy(lru->second.done);
            g_graphs.erase(lru);
        }
        hipStream_t cs = s;
        bool own = false;
        if (s == nullptr) {  // the legacy default stream cannot be captured
            HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
            own = true;
        }
        HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        const int rc = run_launches(p, d_area, cs, di);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(cs, &graph);
        if (own) (void)hipStreamDestroy(cs);
        if (rc != DRT3D_OK) { if (graph) (void)hipGraphDestroy(graph); return rc; }
        if (e != hipSuccess) return fail(DRT3D_EHIP, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
        GraphEntry ge;
        const hipError_t e2 = hipGraphInstantiate(&ge.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e2 != hipSuccess) return fail(DRT3D_EHIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e2));
        if (hipEventCreateWithFlags(&ge.done, hipEventDisableTiming) != hipSuccess) {
            (void)hipGraphExecDestroy(ge.exec);
            return fail(DRT3D_EHIP, "hipEventCreateWithFlags failed");
        }
        it = g_graphs.emplace(sig, ge).first;
    }
    it->second.last_use = ++g_graph_clock;
    HIP_TRY(hipGraphLaunch(it->second.exec, s));
    HIP_TRY(hipEventRecord(it->second.done, s));
    return DRT3D_OK;
}

// ------------------------------------------------------------------ execution
static int execute(Program& prog, void* ws, hipStream_t s, const DeviceInfo& di, int use_graph)
{
    TRY(upload_descs(prog, ws, s));
    const bool prof = g_prof_on.load() != 0;
    if (use_graph && !prof) return run_graph(prog, ws, s, di);
    return run_launches(prog, ws, s, di);
}

// ------------------------------------------------------------------ validation
static int check_common(int N, uint32_t mask, int dtype)
{
    if (ilog2_exact(N) < 1) return fail(DRT3D_EINVAL, "N must be a power of two in [2, %d], got %d", DRT3D_MAX_N, N);
    if (mask == 0 || (mask & ~DRT3D_ALL)) return fail(DRT3D_EINVAL, "mask must be a nonzero 12-bit set, got 0x%x", mask);
    if (dtype != DRT3D_I32 && dtype != DRT3D_F32) return fail(DRT3D_EINVAL, "unsupported dtype %d", dtype);
    return DRT3D_OK;
}

static int check_ptr(const void* p, const char* what)
{
    if (!p) return fail(DRT3D_EINVAL, "%s is NULL", what);
    if ((uintptr_t)p & 15) return fail(DRT3D_EINVAL, "%s is not 16-byte aligned", what);
    return DRT3D_OK;
}

static int check_ws(void* ws, size_t have, size_t need)
{
    if (!ws) return fail(DRT3D_EINVAL, "workspace is NULL");
    if ((uintptr_t)ws & 255) return fail(DRT3D_EINVAL, "workspace is not 256-byte aligned");
    if (have < need) return fail(DRT3D_ENOMEM, "workspace of %zu bytes is smaller than the %zu required", have, need);
    return DRT3D_OK;
}

// Descriptor area bounds: one DrtDesc/DjtDesc per step, per volume.
static size_t desc_area_bytes(int kind, int N, uint32_t mask, int chunked, int adjoint = 0)
{
    const int nd = popcount12(mask);
    const int n = ilog2_exact(N);
    size_t cnt;
    if (kind == S_DJT) {
        const int c = chunked ? chunk_size(djt_per_dod_elems(N, adjoint) * 4, nd) : nd;
        cnt = (size_t)((nd + c - 1) / c) * n;
        return align256(cnt * sizeof(DjtDesc)) + 256;
    }
    const int c = chunked ? chunk_size(2 * drt_stage_elems_per_dod(N) * 4, nd) : nd;
    cnt = (size_t)((nd + c - 1) / c) * (2 * n + 4);  // passes (<= 2n) + adjoint rounds
    // + the two volume transposes
    return align256(cnt * sizeof(DrtDesc)) + align256(2 * sizeof(TransDesc)) + 256;
}

}  // namespace drt3d

// ======================================================================= ABI
using namespace drt3d;

extern "C" {

const char* drt3d_last_error(void) { return g_last_error.c_str(); }
int drt3d_abi_version(void) { return DRT3D_ABI_VERSION; }

size_t drt3d_out_elems(int N, uint32_t mask)
{
    if (ilog2_exact(N) < 1 || mask == 0 || (mask & ~DRT3D_ALL)) return 0;
    return (size_t)popcount12(mask) * N * N * (3 * (size_t)N - 2);
}

size_t djt3d_out_elems(int N, uint32_t mask)
{
    if (ilog2_exact(N) < 1 || mask == 0 || (mask & ~DRT3D_ALL)) return 0;
    return (size_t)popcount12(mask) * N * N * (2 * (size_t)N - 1) * (2 * (size_t)N - 1);
}

size_t drt3d_workspace_bytes(int N, uint32_t mask, int dtype)
{
    // 8-bit volumes use the int32 forward's workspace (their buffers are smaller)
    if (check_common(N, mask, dtype == DRT3D_U8 ? DRT3D_I32 : dtype) != DRT3D_OK) return 0;
    return desc_area_bytes(S_DRT, N, mask, 1) + drt_ws_volume_bytes(N, mask, 4, 0, 1);
}

size_t drt3d_adjoint_workspace_bytes(int N, uint32_t mask, int dtype)
{
    if (check_common(N, mask, dtype) != DRT3D_OK) return 0;
    return desc_area_bytes(S_DRT, N, mask, 1) + drt_ws_volume_bytes(N, mask, 4, 1, 1);
}

size_t djt3d_workspace_bytes(int N, uint32_t mask, int dtype)
{
    if (check_common(N, mask, dtype) != DRT3D_OK) return 0;
    return desc_area_bytes(S_DJT, N, mask, 1) + djt_ws_volume_bytes(N, mask, 4, 1);
}

size_t djt3d_adjoint_workspace_bytes(int N, uint32_t mask, int dtype)
{
    if (check_common(N, mask, dtype) != DRT3D_OK) return 0;
    return desc_area_bytes(S_DJT, N, mask, 1, 1) + djt_ws_volume_bytes(N, mask, 4, 1, 1);
}

static size_t batched_ws(int kind, int adjoint, int count, const int* Ns, uint32_t mask, int dtype)
{
    if (count < 1 || !Ns) return 0;
    size_t d = 0, v = 0;
    for (int i = 0; i < count; ++i) {
        if (check_common(Ns[i], mask, dtype) != DRT3D_OK) return 0;
        d += desc_area_bytes(kind, Ns[i], mask, 0, adjoint);
        v += kind == S_DJT ? djt_ws_volume_bytes(Ns[i], mask, 4, 0, adjoint)
                           : drt_ws_volume_bytes(Ns[i], mask, 4, adjoint, 0);
    }
    return align256(d) + v;
}

size_t drt3d_forward_batched_workspace_bytes(int count, const int* Ns, uint32_t mask, int dtype)
{
    return batched_ws(S_DRT, 0, count, Ns, mask, dtype);
}
size_t drt3d_adjoint_batched_workspace_bytes(int count, const int* Ns, uint32_t mask, int dtype)
{
    return batched_ws(S_DRT, 1, count, Ns, mask, dtype);
}
size_t djt3d_forward_batched_workspace_bytes(int count, const int* Ns, uint32_t mask, int dtype)
{
    return batched_ws(S_DJT, 0, count, Ns, mask, dtype);
}
size_t djt3d_adjoint_batched_workspace_bytes(int count, const int* Ns, uint32_t mask, int dtype)
{
    return batched_ws(S_DJT, 1, count, Ns, mask, dtype);
}

// One volume, DRT forward or adjoint. noalloc: the forward in the static
// scratch (drt3d_forward_noalloc), which must hold the whole workspace.
// tune: the tuning to run with (a plan's), else the size class's current one
static int drt_single(const void* in, void* out, int N, uint32_t mask, int dtype, void* ws, size_t ws_bytes,
                      void* stream, int adjoint, int noalloc = 0, const Tuning* tune = nullptr)
{
    const int narrow = dtype == DRT3D_U8;
    if (narrow && adjoint) return fail(DRT3D_EUNSUPPORTED, "8-bit data is taken by drt3d_forward only");
    if (narrow && N < 32) return fail(DRT3D_EUNSUPPORTED, "8-bit volumes are taken for N >= 32 (got N = %d)", N);
    TRY(check_common(N, mask, narrow ? DRT3D_I32 : dtype));
    TRY(check_ptr(in, adjoint ? "proj" : "vol"));
    TRY(check_ptr(out, adjoint ? "vol_out" : "out"));
    const size_t need = adjoint ? drt3d_adjoint_workspace_bytes(N, mask, dtype) : drt3d_workspace_bytes(N, mask, dtype);
    if (noalloc) {
        if (need > kNoallocScratchBytes)
            return fail(DRT3D_EINVAL,
                        "drt3d_forward_noalloc: N = %d with %d dodecants needs %zu bytes of scratch, more than the "
                        "static %zu (12 dodecants: N <= 64); use drt3d_forward with a workspace",
                        N, popcount12(mask), need, kNoallocScratchBytes);
        TRY(scratch_ptr(&ws));
        ws_bytes = kNoallocScratchBytes;
    }
    TRY(check_ws(ws, ws_bytes, need));
    DeviceInfo di;
    TRY(device_info(di));
    const int is_float = dtype == DRT3D_F32;
    const Tuning t = tune ? *tune : get_tuning(N, is_float);
    DrtIO io{in, out, (char*)ws + desc_area_bytes(S_DRT, N, mask, 1)};
    std::vector<std::vector<Step>> vols(1);
    TRY(drt_steps(vols[0], N, mask, is_float, adjoint, 1, t, io, narrow));
    Program prog;
    prog.is_float = is_float;
    build_program(prog, vols, false);
    if (prog.desc_bytes() > desc_area_bytes(S_DRT, N, mask, 1))
        return fail(DRT3D_EINVAL, "internal: descriptor area too small");
    if (narrow)  // narrow storage exists in the shape-specialised passes only
        for (const Launch& L : prog.launches)
            if (L.kind == S_DRT && L.fast_kx < 0)
                return fail(DRT3D_EUNSUPPORTED, "8-bit volumes: tuning %s has a pass without a narrow kernel",
                            tuning_to_string(t).c_str());
    if (noalloc) {
        TRY(upload_descs_by_args(prog, ws, (hipStream_t)stream));
        return run_launches(prog, ws, (hipStream_t)stream, di, false);
    }
    return execute(prog, ws, (hipStream_t)stream, di, 0);
}

int drt3d_forward(const void* vol, void* out, int N, uint32_t mask, int dtype, void* workspace,
                  size_t workspace_bytes, void* stream)
{
    return drt_single(vol, out, N, mask, dtype, workspace, workspace_bytes, stream, 0);
}

int drt3d_forward_noalloc(const void* vol, void* out, int N, uint32_t mask, int dtype, void* stream)
{
    return drt_single(vol, out, N, mask, dtype, nullptr, 0, stream, 0, 1);
}

int drt3d_adjoint(const void* proj, void* vol_out, int N, uint32_t mask, int dtype, void* workspace,
                  size_t workspace_bytes, void* stream)
{
    return drt_single(proj, vol_out, N, mask, dtype, workspace, workspace_bytes, stream, 1);
}

// One volume, DJT forward or adjoint.
static int djt_single(const void* in, void* out, int N, uint32_t mask, int dtype, void* ws, size_t ws_bytes,
                      void* stream, int adjoint)
{
    TRY(check_common(N, mask, dtype));
    TRY(check_ptr(in, adjoint ? "proj" : "vol"));
    TRY(check_ptr(out, adjoint ? "vol_out" : "out"));
    const size_t need = adjoint ? djt3d_adjoint_workspace_bytes(N, mask, dtype) : djt3d_workspace_bytes(N, mask, dtype);
    TRY(check_ws(ws, ws_bytes, need));
    DeviceInfo di;
    TRY(device_info(di));
    DrtIO io{in, out, (char*)ws + desc_area_bytes(S_DJT, N, mask, 1, adjoint)};
    std::vector<std::vector<Step>> vols(1);
    TRY(djt_steps(vols[0], N, mask, 1, io, adjoint));
    Program prog;
    prog.is_float = dtype == DRT3D_F32;
    build_program(prog, vols, false);
    if (prog.desc_bytes() > desc_area_bytes(S_DJT, N, mask, 1, adjoint))
        return fail(DRT3D_EINVAL, "internal: descriptor area too small");
    return execute(prog, ws, (hipStream_t)stream, di, 0);
}

int djt3d_forward(const void* vol, void* out, int N, uint32_t mask, int dtype, void* workspace,
                  size_t workspace_bytes, void* stream)
{
    return djt_single(vol, out, N, mask, dtype, workspace, workspace_bytes, stream, 0);
}

int djt3d_adjoint(const void* proj, void* vol_out, int N, uint32_t mask, int dtype, void* workspace,
                  size_t workspace_bytes, void* stream)
{
    return djt_single(proj, vol_out, N, mask, dtype, workspace, workspace_bytes, stream, 1);
}

// Batched calls merge the launches of volumes below this size.
static const int kSoloN = 128;

static int batched(int kind, int adjoint, int count, const void* const* ins, void* const* outs, const int* Ns,
                   uint32_t mask, int dtype, void* ws, size_t ws_bytes, void* stream)
{
    if (count < 1) return fail(DRT3D_EINVAL, "count must be >= 1, got %d", count);
    if (!ins || !outs || !Ns) return fail(DRT3D_EINVAL, "pointer arrays and Ns must not be NULL");
    for (int i = 0; i < count; ++i) {
        TRY(check_common(Ns[i], mask, dtype));
        TRY(check_ptr(ins[i], "input"));
        TRY(check_ptr(outs[i], "output"));
    }
    TRY(check_ws(ws, ws_bytes, batched_ws(kind, adjoint, count, Ns, mask, dtype)));
    DeviceInfo di;
    TRY(device_info(di));
    const int is_float = dtype == DRT3D_F32;
    size_t dsz = 0;
    for (int i = 0; i < count; ++i) dsz += desc_area_bytes(kind, Ns[i], mask, 0, adjoint);
    char* w = (char*)ws + align256(dsz);
    std::vector<std::vector<Step>> vols(count);
    std::vector<char> solo(count, 0);
    const char* se = getenv("DRT3D_SOLO_N");  // tuning override of kSoloN
    const int solo_n = se ? atoi(se) : kSoloN;
    for (int i = 0; i < count; ++i) {
        // a volume this large fills the GPU in every launch on its own:
        // merging it with others only stretches each launch's working set
        solo[i] = Ns[i] >= solo_n;
        DrtIO io{ins[i], outs[i], w};
        if (kind == S_DJT) {
            TRY(djt_steps(vols[i], Ns[i], mask, 0, io, adjoint));
            w += djt_ws_volume_bytes(Ns[i], mask, 4, 0, adjoint);
        } else {
            TRY(drt_steps(vols[i], Ns[i], mask, is_float, adjoint, 0, get_tuning(Ns[i], is_float), io));
            w += drt_ws_volume_bytes(Ns[i], mask, 4, adjoint, 0);
        }
    }
    Program prog;
    prog.is_float = is_float;
    prog.persistent = 1;
    build_program(prog, vols, true, &solo);
    if (prog.desc_bytes() > align256(dsz)) return fail(DRT3D_EINVAL, "internal: descriptor area too small");
    const char* g = getenv("DRT3D_GRAPHS");
    const int use_graph = g ? atoi(g) != 0 : 1;
    return execute(prog, ws, (hipStream_t)stream, di, use_graph);
}

int drt3d_forward_batched(int count, const void* const* vols, void* const* outs, const int* Ns, uint32_t mask,
                          int dtype, void* workspace, size_t workspace_bytes, void* stream)
{
    return batched(S_DRT, 0, count, vols, outs, Ns, mask, dtype, workspace, workspace_bytes, stream);
}

int drt3d_adjoint_batched(int count, const void* const* projs, void* const* vols_out, const int* Ns, uint32_t mask,
                          int dtype, void* workspace, size_t workspace_bytes, void* stream)
{
    return batched(S_DRT, 1, count, projs, vols_out, Ns, mask, dtype, workspace, workspace_bytes, stream);
}

int djt3d_forward_batched(int count, const void* const* vols, void* const* outs, const int* Ns, uint32_t mask,
                          int dtype, void* workspace, size_t workspace_bytes, void* stream)
{
    return batched(S_DJT, 0, count, vols, outs, Ns, mask, dtype, workspace, workspace_bytes, stream);
}

int djt3d_adjoint_batched(int count, const void* const* projs, void* const* vols_out, const int* Ns, uint32_t mask,
                          int dtype, void* workspace, size_t workspace_bytes, void* stream)
{
    return batched(S_DJT, 1, count, projs, vols_out, Ns, mask, dtype, workspace, workspace_bytes, stream);
}

// ------------------------------------------------------------------ merged net ABI
size_t drt3d_net_elems(int N)
{
    if (ilog2_exact(N) < 1 || N > DRT3D_MAX_N) return 0;
    return (size_t)16 * N * N * (3 * (size_t)N - 2);
}

int drt3d_merge_net(const void* proj, void* net, int N, int dtype, void* stream)
{
    TRY(check_common(N, DRT3D_ALL, dtype));
    TRY(check_ptr(proj, "proj"));
    TRY(check_ptr(net, "net"));
    HIP_TRY(launch_merge_net(dtype == DRT3D_F32, proj, net, N, (hipStream_t)stream));
    return DRT3D_OK;
}

// ------------------------------------------------------------------ plane detection ABI
// The application of Sec. 6.1 on the DRT output: the dominant plane (largest
// bin), then the bins orthogonal to it that are relative maxima and reach a
// threshold; backprojection of listed bins through the adjoint.
namespace {
struct DetectLayout {
    size_t pv = 0, pi = 0, top = 0, thr = 0, counts = 0, offsets = 0, csum = 0, total = 0;
};
void detect_layout(int N, uint32_t mask, DetectLayout& L)
{
    const long long n = (long long)popcount12(mask) * N * N * (3 * N - 2);
    const long long ncol = (long long)popcount12(mask) * N * N;
    const int parts = argmax_parts(n);
    size_t o = 0;
    L.pv = o; o = align256(o + 4 * (size_t)parts);
    L.pi = o; o = align256(o + 8 * (size_t)parts);
    L.top = o; o = align256(o + 8);
    L.thr = o; o = align256(o + 8);
    L.counts = o; o = align256(o + 4 * (size_t)ncol);
    L.offsets = o; o = align256(o + 8 * (size_t)ncol);
    L.csum = o; o = align256(o + 8 * (size_t)scan_chunks(ncol));
    L.total = o;
}
void plane_frames(uint32_t mask, PlaneFrames& F)
{
    F = PlaneFrames{};
    int j = 0;
    for (int k = 0; k < 12; ++k) {
        if ((mask >> k) & 1) F.ks[j++] = k;
        AxisMap ax[3];
        frame_axes(k, ax);
        for (int i = 0; i < 3; ++i) {
            F.axis[k][i] = (signed char)ax[i].primed;
            F.sign[k][i] = (signed char)(ax[i].mirror ? -1 : 1);
        }
    }
}
}  // namespace

size_t drt3d_detect_planes_workspace_bytes(int N, uint32_t mask, int dtype)
{
    if (check_common(N, mask, dtype) != DRT3D_OK) return 0;
    DetectLayout L;
    detect_layout(N, mask, L);
    return L.total;
}

int drt3d_detect_planes(const void* proj, int N, uint32_t mask, int dtype, double cos_tol, double rel_threshold,
                        long long* bins, long long cap, long long* count, void* workspace, size_t workspace_bytes,
                        void* stream)
{
    TRY(check_common(N, mask, dtype));
    TRY(check_ptr(proj, "proj"));
    if (!bins || ((uintptr_t)bins & 7)) return fail(DRT3D_EINVAL, "bins is NULL or not 8-byte aligned");
    if (!count || ((uintptr_t)count & 7)) return fail(DRT3D_EINVAL, "count is NULL or not 8-byte aligned");
    if (cap < 1) return fail(DRT3D_EINVAL, "cap must be at least 1, got %lld", cap);
    if (!(cos_tol >= 0.0 && cos_tol < 1.0)) return fail(DRT3D_EINVAL, "cos_tol must lie in [0, 1), got %g", cos_tol);
    if (!std::isfinite(rel_threshold)) return fail(DRT3D_EINVAL, "rel_threshold must be finite");
    DetectLayout L;
    detect_layout(N, mask, L);
    TRY(check_ws(workspace, workspace_bytes, L.total));
    char* w = (char*)workspace;
    const hipStream_t s = (hipStream_t)stream;
    const int is_float = dtype == DRT3D_F32;
    const int nk = popcount12(mask);
    const long long n = (long long)nk * N * N * (3 * N - 2), ncol = (long long)nk * N * N;
    const int parts = argmax_parts(n);
    long long* top = (long long*)(w + L.top);
    double* thr = (double*)(w + L.thr);
    int* counts = (int*)(w + L.counts);
    long long* offsets = (long long*)(w + L.offsets);
    PlaneFrames F;
    plane_frames(mask, F);
    const double tol2 = cos_tol * cos_tol;
    HIP_TRY(launch_argmax(is_float, proj, n, w + L.pv, (long long*)(w + L.pi), parts, rel_threshold, top, thr, bins, s));
    HIP_TRY(launch_plane_peaks(is_float, 0, proj, N, nk, F, top, thr, tol2, counts, offsets, bins, cap, s));
    HIP_TRY(launch_peak_scan(counts, ncol, offsets, (long long*)(w + L.csum), count, s));
    HIP_TRY(launch_plane_peaks(is_float, 1, proj, N, nk, F, top, thr, tol2, counts, offsets, bins, cap, s));
    return DRT3D_OK;
}

size_t drt3d_backproject_bins_workspace_bytes(int N, uint32_t mask, int dtype)
{
    if (check_common(N, mask, dtype) != DRT3D_OK) return 0;
    return align256(drt3d_out_elems(N, mask) * 4) + drt3d_adjoint_workspace_bytes(N, mask, dtype);
}

int drt3d_backproject_bins(const long long* bins, const long long* count, long long cap, void* vol_out, int N,
                           uint32_t mask, int dtype, void* workspace, size_t workspace_bytes, void* stream)
{
    TRY(check_common(N, mask, dtype));
    if (!bins || ((uintptr_t)bins & 7)) return fail(DRT3D_EINVAL, "bins is NULL or not 8-byte aligned");
    if (!count || ((uintptr_t)count & 7)) return fail(DRT3D_EINVAL, "count is NULL or not 8-byte aligned");
    if (cap < 0) return fail(DRT3D_EINVAL, "cap must not be negative, got %lld", cap);
    TRY(check_ptr(vol_out, "vol_out"));
    TRY(check_ws(workspace, workspace_bytes, drt3d_backproject_bins_workspace_bytes(N, mask, dtype)));
    const long long n = (long long)drt3d_out_elems(N, mask);
    const size_t mbytes = align256((size_t)n * 4);
    uint32_t* marker = (uint32_t*)workspace;
    const hipStream_t s = (hipStream_t)stream;
    HIP_TRY(launch_fill((float*)marker, 0.f, n, s));
    if (cap > 0)
        HIP_TRY(launch_scatter_ones(bins, count, cap, marker, n, dtype == DRT3D_F32 ? 0x3f800000u : 1u, s));
    return drt_single(marker, vol_out, N, mask, dtype, (char*)workspace + mbytes, workspace_bytes - mbytes, stream, 1);
}

int drt3d_plane_normal(int k, int s1, int s2, int N, int out[3])
{
    if (k < 0 || k > 11 || ilog2_exact(N) < 1 || s1 < 0 || s1 >= N || s2 < 0 || s2 >= N || !out)
        return fail(DRT3D_EINVAL, "bad arguments to drt3d_plane_normal");
    AxisMap ax[3];
    frame_axes(k, ax);
    const int c[3] = {-s1, -s2, N - 1};
    for (int i = 0; i < 3; ++i) out[i] = (ax[i].mirror ? -1 : 1) * c[ax[i].primed];
    return DRT3D_OK;
}

// ------------------------------------------------------------------ inverse ABI
// Iterative inverse of the 12-dodecant DRT (Sec. 5.2): Press's iterative
// improvement with the approximate inverse H A^T (H the printed 3x3x3
// high-pass filter) inside multigrid V-cycles that restrict the residual with
// S and prolong the coarse correction with P. Each level smooths with three
// Chebyshev step sizes over [L/10, L], L = 1.02 x the largest eigenvalue of
// H A^T A at that size (a power iteration, computed once per size and device).
// At size 1 the coarse problem's least-squares solution is the mean.
namespace {
struct InvLayout {
    int n = 0;
    std::vector<size_t> b, x;          // per level l (size N >> l), l >= 1
    std::vector<size_t> dfwd, dadj;    // per level l < n: descriptor areas of its forward and adjoint
    size_t tproj = 0, tvol = 0, tvol2 = 0, tvol3 = 0, norm = 0, drt = 0, drt_bytes = 0, total = 0;
};
// A level's forward (x_l -> T) or adjoint (T -> V), planned once per call
// with its descriptors uploaded once into its own area: the cycles then only
// launch kernels.
struct InvProg {
    Program p;
    char* area = nullptr;
    bool fused_residual = false;  // forward: its last pass writes b - A x itself
};
struct InvRun {
    const float* proj;
    float* x0;
    char* ws;
    InvLayout L;
    int N;
    std::vector<double> lam;  // per level l < n
    hipStream_t s;
    std::vector<InvProg> fwd, adj;  // per level l < n, once prepared
    DeviceInfo di;
};
constexpr int kInvNu = 3;
constexpr double kInvRatio = 10.0, kInvMargin = 1.02;
constexpr int kInvPowerIters = 30;
std::mutex g_inv_mu;
std::map<std::pair<int, int>, double> g_inv_lam;  // (device, size) -> eigenvalue
}  // namespace

static InvLayout inv_layout(int N)
{
    InvLayout L;
    L.n = ilog2_exact(N);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align256(bytes);
        return o;
    };
    L.b.assign(L.n + 1, 0);
    L.x.assign(L.n + 1, 0);
    L.dfwd.assign(L.n, 0);
    L.dadj.assign(L.n, 0);
    for (int l = 0; l < L.n; ++l) {
        L.dfwd[l] = take(desc_area_bytes(S_DRT, N >> l, DRT3D_ALL, 1, 0));
        L.dadj[l] = take(desc_area_bytes(S_DRT, N >> l, DRT3D_ALL, 1, 1));
    }
    for (int l = 1; l <= L.n; ++l) {
        const size_t Nl = (size_t)N >> l;
        L.b[l] = take(12 * Nl * Nl * (3 * Nl - 2) * sizeof(float));
        L.x[l] = take(Nl * Nl * Nl * sizeof(float));
    }
    const size_t vol = (size_t)N * N * N * sizeof(float);
    L.tproj = take(12 * (size_t)N * N * (3 * (size_t)N - 2) * sizeof(float));
    L.tvol = take(vol);
    L.tvol2 = take(vol);
    L.tvol3 = take(vol);
    L.norm = take(norm_scratch_bytes());
    size_t dw = 0;
    for (int l = 0; l < L.n; ++l) {
        const int Nl = N >> l;
        dw = std::max(dw, std::max(drt3d_workspace_bytes(Nl, DRT3D_ALL, DRT3D_F32),
                                   drt3d_adjoint_workspace_bytes(Nl, DRT3D_ALL, DRT3D_F32)));
    }
    L.drt = take(dw);
    L.drt_bytes = dw;
    L.total = off;
    return L;
}

static int check_inverse_args(int N, void* ws, size_t ws_bytes)
{
    if (ilog2_exact(N) < 1 || N > DRT3D_MAX_N) return fail(DRT3D_EINVAL, "N must be a power of two in [2, %d], got %d", DRT3D_MAX_N, N);
    if (!ws || ((uintptr_t)ws & 255)) return fail(DRT3D_EINVAL, "the inverse workspace must be non-null and 256-byte aligned");
    const size_t need = inv_layout(N).total;
    if (ws_bytes < need) return fail(DRT3D_ENOMEM, "inverse workspace too small: %zu < %zu bytes", ws_bytes, need);
    return DRT3D_OK;
}

static int inv_drt(InvRun& r, int l, const float* in, float* out, int adjoint)
{
    return drt_single(in, out, r.N >> l, DRT3D_ALL, DRT3D_F32, r.ws + r.L.drt, r.L.drt_bytes, r.s, adjoint);
}

static float* inv_b(InvRun& r, int l) { return l == 0 ? const_cast<float*>(r.proj) : (float*)(r.ws + r.L.b[l]); }
static float* inv_x(InvRun& r, int l) { return l == 0 ? r.x0 : (float*)(r.ws + r.L.x[l]); }

// Plans level l's forward (x_l -> T) and adjoint (T -> V) and uploads their
// descriptors; the stage buffers of both live in the shared transform region
// (the calls are stream-ordered).
static int inv_prepare(InvRun& r)
{
    TRY(device_info(r.di));
    r.fwd.assign(r.L.n, InvProg{});
    r.adj.assign(r.L.n, InvProg{});
    for (int l = 0; l < r.L.n; ++l) {
        const int Nl = r.N >> l;
        const Tuning t = get_tuning(Nl, 1);
        for (int adjoint = 0; adjoint < 2; ++adjoint) {
            InvProg& ip = adjoint ? r.adj[l] : r.fwd[l];
            const void* in = adjoint ? (const void*)(r.ws + r.L.tproj) : (const void*)inv_x(r, l);
            void* out = adjoint ? (void*)(r.ws + r.L.tvol) : (void*)(r.ws + r.L.tproj);
            DrtIO io{in, out, r.ws + r.L.drt};
            std::vector<std::vector<Step>> vols(1);
            TRY(drt_steps(vols[0], Nl, DRT3D_ALL, 1, adjoint, 1, t, io));
            ip.p.is_float = 1;
            build_program(ip.p, vols, false);
            if (!adjoint) {
                // the residual b - A x is written by the forward's last pass
                // itself where that pass runs the eight-wavefront specialised
                // kernel (it reads b where it would otherwise store A x)
                const Launch& last = ip.p.launches.back();
                if (last.kind == S_DRT && last.fast_kx >= 0 && last.fast_mode == 1 && last.block == 512) {
                    for (int q = last.first; q < last.first + last.ndesc; ++q) ip.p.drt[q].sub = inv_b(r, l);
                    ip.fused_residual = true;
                }
            }
            ip.area = r.ws + (adjoint ? r.L.dadj[l] : r.L.dfwd[l]);
            if (ip.p.desc_bytes() > desc_area_bytes(S_DRT, Nl, DRT3D_ALL, 1, adjoint))
                return fail(DRT3D_EINVAL, "internal: inverse descriptor area too small");
            TRY(upload_descs(ip.p, ip.area, r.s));
        }
    }
    return DRT3D_OK;
}

// T = b_l - A x_l in the projection temporary
static int inv_residual(InvRun& r, int l)
{
    const long long Nl = r.N >> l;
    float* T = (float*)(r.ws + r.L.tproj);
    TRY(run_launches(r.fwd[l].p, r.fwd[l].area, r.s, r.di));
    if (!r.fwd[l].fused_residual) HIP_TRY(launch_residual(inv_b(r, l), T, T, 12 * Nl * Nl * (3 * Nl - 2), r.s));
    return DRT3D_OK;
}

// x_l += c H A^T (b_l - A x_l)
static int inv_smooth(InvRun& r, int l, float c)
{
    TRY(inv_residual(r, l));
    TRY(run_launches(r.adj[l].p, r.adj[l].area, r.s, r.di));
    HIP_TRY(launch_hp_filter((const float*)(r.ws + r.L.tvol), inv_x(r, l), r.N >> l, c, 1, r.s));
    return DRT3D_OK;
}

static void inv_steps(double lam, double c[kInvNu])
{
    const double b = kInvMargin * lam, a = b / kInvRatio;
    for (int i = 1; i <= kInvNu; ++i)
        c[i - 1] = 1.0 / ((b + a) / 2 + (b - a) / 2 * cos((2 * i - 1) * M_PI / (2 * kInvNu)));
}

static int inv_vcycle(InvRun& r, int l)
{
    const int Nl = r.N >> l;
    if (Nl == 1) {
        HIP_TRY(launch_base_mean(inv_b(r, l), inv_x(r, l), r.s));
        return DRT3D_OK;
    }
    double c[kInvNu];
    inv_steps(r.lam[l], c);
    for (int i = 0; i < kInvNu; ++i) TRY(inv_smooth(r, l, (float)c[i]));
    TRY(inv_residual(r, l));
    HIP_TRY(launch_restrict((const float*)(r.ws + r.L.tproj), inv_b(r, l + 1), Nl, r.s));
    const long long Nc = Nl / 2;
    HIP_TRY(launch_fill(inv_x(r, l + 1), 0.f, Nc * Nc * Nc, r.s));
    TRY(inv_vcycle(r, l + 1));
    HIP_TRY(launch_prolong_add(inv_x(r, l + 1), inv_x(r, l), Nl, r.s));
    for (int i = kInvNu - 1; i >= 0; --i) TRY(inv_smooth(r, l, (float)c[i]));
    return DRT3D_OK;
}

// Largest eigenvalue of H A^T A at size M by power iteration (synchronises).
static int inv_power(InvRun& r, int M, double& lam)
{
    float* v = (float*)(r.ws + r.L.tvol2);
    float* w1 = (float*)(r.ws + r.L.tvol);
    float* w2 = (float*)(r.ws + r.L.tvol3);
    float* T = (float*)(r.ws + r.L.tproj);
    double* scratch = (double*)(r.ws + r.L.norm);
    const long long n = (long long)M * M * M;
    const int l = ilog2_exact(r.N) - ilog2_exact(M);
    HIP_TRY(launch_power_start(v, M, r.s));
    for (int it = 0; it < kInvPowerIters; ++it) {
        TRY(inv_drt(r, l, v, T, 0));
        TRY(inv_drt(r, l, T, w1, 1));
        HIP_TRY(launch_hp_filter(w1, w2, M, 1.f, 0, r.s));
        HIP_TRY(launch_normalize(w2, v, n, scratch, r.s));
    }
    double norm = 0;
    HIP_TRY(hipMemcpyAsync(&norm, (const char*)scratch + norm_scratch_bytes() - sizeof(double), sizeof(double),
                           hipMemcpyDeviceToHost, r.s));
    HIP_TRY(hipStreamSynchronize(r.s));
    if (!(norm > 0) || !std::isfinite(norm)) return fail(DRT3D_EHIP, "power iteration at N = %d gave %g", M, norm);
    lam = norm;  // v was normalised before the last product: |H A^T A v| / |v| = |w2|
    return DRT3D_OK;
}

// Every level's eigenvalue, from the cache or the power iteration.
static int inv_lambdas(InvRun& r)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    r.lam.assign(r.L.n, 0.0);
    for (int l = 0; l < r.L.n; ++l) {
        const int M = r.N >> l;
        {
            std::lock_guard<std::mutex> lk(g_inv_mu);
            auto it = g_inv_lam.find({dev, M});
            if (it != g_inv_lam.end()) {
                r.lam[l] = it->second;
                continue;
            }
        }
        double lam = 0;
        TRY(inv_power(r, M, lam));
        std::lock_guard<std::mutex> lk(g_inv_mu);
        g_inv_lam[{dev, M}] = lam;
        r.lam[l] = lam;
    }
    return DRT3D_OK;
}

size_t drt3d_inverse_workspace_bytes(int N)
{
    if (ilog2_exact(N) < 1 || N > DRT3D_MAX_N) return 0;
    return inv_layout(N).total;
}

int drt3d_inverse_lambdas(int N, double* lams, void* workspace, size_t workspace_bytes, void* stream)
{
    TRY(check_inverse_args(N, workspace, workspace_bytes));
    if (!lams) return fail(DRT3D_EINVAL, "lams must not be NULL");
    InvRun r{nullptr, nullptr, (char*)workspace, inv_layout(N), N, {}, (hipStream_t)stream};
    TRY(inv_lambdas(r));
    for (int l = 0; l < r.L.n; ++l) lams[r.L.n - 1 - l] = r.lam[l];  // sizes 2, 4, ..., N
    return DRT3D_OK;
}

int drt3d_inverse(const void* proj, void* vol_out, int N, int cycles, const double* lams, void* workspace,
                  size_t workspace_bytes, void* stream)
{
    TRY(check_inverse_args(N, workspace, workspace_bytes));
    TRY(check_ptr(proj, "proj"));
    TRY(check_ptr(vol_out, "vol_out"));
    if (cycles < 0) return fail(DRT3D_EINVAL, "cycles must be >= 0, got %d", cycles);
    InvRun r{(const float*)proj, (float*)vol_out, (char*)workspace, inv_layout(N), N, {}, (hipStream_t)stream};
    if (lams) {
        r.lam.assign(r.L.n, 0.0);
        for (int l = 0; l < r.L.n; ++l) {
            const double v = lams[r.L.n - 1 - l];
            if (!(v > 0) || !std::isfinite(v)) return fail(DRT3D_EINVAL, "lams[%d] = %g is not a positive eigenvalue", r.L.n - 1 - l, v);
            r.lam[l] = v;
        }
    } else {
        TRY(inv_lambdas(r));
    }
    HIP_TRY(launch_fill(r.x0, 0.f, (long long)N * N * N, r.s));
    if (cycles > 0) TRY(inv_prepare(r));
    for (int c = 0; c < cycles; ++c) TRY(inv_vcycle(r, 0));
    return DRT3D_OK;
}

// ------------------------------------------------------------------ tuning ABI
const char* drt3d_tuning_string(int N, int dtype)
{
    static thread_local std::string s;
    if (ilog2_exact(N) < 1 || (dtype != DRT3D_I32 && dtype != DRT3D_F32)) return "";
    s = tuning_to_string(get_tuning(N, dtype == DRT3D_F32));
    return s.c_str();
}

int drt3d_set_tuning(int N, int dtype, const char* text)
{
    TRY(check_common(N, DRT3D_ALL, dtype));
    if (!text) return fail(DRT3D_EINVAL, "tuning text is NULL");
    Tuning t;
    if (!tuning_from_string(text, ilog2_exact(N), t)) return fail(DRT3D_EINVAL, "cannot parse tuning '%s'", text);
    // every pass must fit, the adjoint's under both of its budgets
    for (int adj = 0; adj < 3; ++adj)
        for (const PassGeom& g : drt_passes(N, t)) {
            int T, H, L, nt;
            if (!choose_tiles(g, adj > 0, adj == 2 ? adj_lds_of(t) : t.lds_elems, T, H, L, nt))
                return fail(DRT3D_EINVAL, "tuning '%s' does not fit LDS", text);
        }
    put_tuning(N, dtype == DRT3D_F32, t);
    return DRT3D_OK;
}

// Splits of n stages into P passes of 1..3 stages each, in every order.
static void stage_splits(int n, int P, std::vector<std::vector<int>>& out)
{
    std::vector<int> k(P, 1);
    for (;;) {
        int sum = 0;
        for (int v : k) sum += v;
        if (sum == n) out.push_back(k);
        int i = 0;
        while (i < P && k[i] == 3) k[i++] = 1;
        if (i == P) break;
        ++k[i];
    }
}

// Candidate pass lists: ceil(n/3)..ceil(n/3)+1 passes (at most 4); per pass the
// x- and y-stage counts differ by at most one (square-ish column groups).
static void pass_list_candidates(int n, const Tuning& base, std::vector<Tuning>& out)
{
    const int P0 = std::max(1, (n + 2) / 3);
    for (int P = P0; P <= std::min(std::min(4, n), P0 + 1); ++P) {
        std::vector<std::vector<int>> xs;
        stage_splits(n, P, xs);
        for (auto& a : xs)
            for (auto& b : xs) {
                Tuning c = base;
                c.np = P;
                bool ok = true;
                for (int i = 0; i < P; ++i) {
                    c.kx[i] = a[i];
                    c.ky[i] = b[i];
                    if (std::abs(a[i] - b[i]) > 1 || (1 << (a[i] + b[i])) > kMaxPassSlots) ok = false;
                }
                if (ok) out.push_back(c);
            }
    }
}

// Timed search over the tuning space of one size class. Objective: forward
// time for int32, forward + adjoint time for float32 (the differentiable
// transform runs both). Phase 1 times every pass list at two LDS budgets,
// phase 2 every LDS budget for the three best lists, phase 3 the wave count
// (4 and 16 against the default 8; 16 exists for 3.3 passes only).
// The adjoint's buffers are allocated here (a tuning call, not a transform).
int drt3d_autotune(int N, int dtype, const void* vol, void* out, void* workspace, size_t workspace_bytes,
                   void* stream)
{
    TRY(check_common(N, DRT3D_ALL, dtype));
    TRY(check_ptr(vol, "vol"));
    TRY(check_ptr(out, "out"));
    TRY(check_ws(workspace, workspace_bytes, drt3d_workspace_bytes(N, DRT3D_ALL, dtype)));
    DeviceInfo di;
    TRY(device_info(di));
    const int n = ilog2_exact(N);
    const int is_float = dtype == DRT3D_F32;
    hipStream_t s = (hipStream_t)stream;
    void* back = nullptr;
    void* aws = nullptr;
    const size_t aws_bytes = drt3d_adjoint_workspace_bytes(N, DRT3D_ALL, dtype);
    if (is_float) {
        HIP_TRY(hipMalloc(&back, (size_t)N * N * N * 4));
        if (hipMalloc(&aws, aws_bytes) != hipSuccess) {
            (void)hipFree(back);
            return fail(DRT3D_ENOMEM, "autotune: no memory for the adjoint workspace");
        }
    }
    hipEvent_t ea, eb;
    HIP_TRY(hipEventCreate(&ea));
    HIP_TRY(hipEventCreate(&eb));
    auto time_of = [&](const Tuning& t, float& best_ms) -> int {
        put_tuning(N, is_float, t);
        best_ms = 1e30f;
        for (int r = 0; r < 4; ++r) {
            HIP_TRY(hipEventRecord(ea, s));
            TRY(drt3d_forward(vol, out, N, DRT3D_ALL, dtype, workspace, workspace_bytes, stream));
            if (is_float) TRY(drt3d_adjoint(out, back, N, DRT3D_ALL, dtype, aws, aws_bytes, stream));
            HIP_TRY(hipEventRecord(eb, s));
            HIP_TRY(hipEventSynchronize(eb));
            float ms = 0;
            HIP_TRY(hipEventElapsedTime(&ms, ea, eb));
            if (r > 0) best_ms = std::min(best_ms, ms);
        }
        return DRT3D_OK;
    };
    auto fits = [&](const Tuning& t) {
        if ((size_t)std::max(t.lds_elems, adj_lds_of(t)) * 4 > (size_t)di.max_lds) return false;
        for (int adj = 0; adj < 3; ++adj)
            for (const PassGeom& g : drt_passes(N, t)) {
                int T, H, L, nt;
                if (!choose_tiles(g, adj > 0, adj == 2 ? adj_lds_of(t) : t.lds_elems, T, H, L, nt)) return false;
            }
        return true;
    };
    int rc = DRT3D_OK;
    Tuning best = get_tuning(N, is_float);
    if (!fits(best)) best = default_tuning(n, is_float);
    float best_ms = 1e30f;
    std::vector<std::pair<float, Tuning>> scored;
    auto consider = [&](const Tuning& c) -> int {
        if (!fits(c)) return DRT3D_OK;
        float ms;
        TRY(time_of(c, ms));
        scored.push_back({ms, c});
        if (ms < best_ms) { best_ms = ms; best = c; }
        return DRT3D_OK;
    };
    do {
        if ((rc = consider(best)) != DRT3D_OK) break;
        std::vector<Tuning> lists;
        pass_list_candidates(n, best, lists);
        for (Tuning c : lists) {
            for (int l : {16384, 18432}) {
                c.lds_elems = l;
                c.waves = 8;
                if ((rc = consider(c)) != DRT3D_OK) break;
            }
            if (rc != DRT3D_OK) break;
        }
        if (rc != DRT3D_OK) break;
        std::sort(scored.begin(), scored.end(),
                  [](const std::pair<float, Tuning>& x, const std::pair<float, Tuning>& y) { return x.first < y.first; });
        std::vector<Tuning> top;
        for (auto& sc : scored) {
            bool dup = false;
            for (auto& t : top) dup = dup || (t.np == sc.second.np && std::equal(t.kx, t.kx + t.np, sc.second.kx) &&
                                              std::equal(t.ky, t.ky + t.np, sc.second.ky));
            if (!dup) top.push_back(sc.second);
            if (top.size() == 3) break;
        }
        for (Tuning c : top) {
            for (int l : {8192, 12288, 13312, 14336, 20480, 24576, 32768}) {
                c.lds_elems = l;
                if ((rc = consider(c)) != DRT3D_OK) break;
            }
            if (rc != DRT3D_OK) break;
        }
        if (rc != DRT3D_OK) break;
        const Tuning b = best;
        for (int w : {4, 16}) {
            Tuning c = b;
            c.waves = w;
            if ((rc = consider(c)) != DRT3D_OK) break;
        }
    } while (0);
    put_tuning(N, is_float, best);
    (void)hipEventDestroy(ea);
    (void)hipEventDestroy(eb);
    if (back) (void)hipFree(back);
    if (aws) (void)hipFree(aws);
    if (rc != DRT3D_OK) return rc;
    if (const char* path = getenv("DRT3D_TUNE_CACHE")) {
        if (FILE* fp = fopen(path, "a")) {
            fprintf(fp, "%d %d %s\n", N, is_float, tuning_to_string(best).c_str());
            fclose(fp);
        }
    }
    return DRT3D_OK;
}

// ------------------------------------------------------------------ reference stream
int drt3d_stream_probe(const void* src, size_t read_bytes, void* dst, size_t write_bytes, void* stream)
{
    TRY(check_ptr(src, "src"));
    TRY(check_ptr(dst, "dst"));
    const size_t cap = (size_t)32 << 30;
    if (read_bytes < 16 || write_bytes < 16 || read_bytes % 16 || write_bytes % 16 || read_bytes > cap ||
        write_bytes > cap)
        return fail(DRT3D_EINVAL, "stream probe: byte counts must be multiples of 16 in [16, 32 GiB], got %zu and %zu",
                    read_bytes, write_bytes);
    DeviceInfo di;
    TRY(device_info(di));
    const hipError_t e = launch_stream_probe(src, read_bytes, dst, write_bytes, di.cus, (hipStream_t)stream);
    if (e != hipSuccess) return fail(DRT3D_EHIP, "launch of the stream probe failed: %s", hipGetErrorString(e));
    return DRT3D_OK;
}

// ------------------------------------------------------------------ profiling ABI
int drt3d_profile_enable(int on)
{
    g_prof_on.store(on ? 1 : 0);
    return DRT3D_OK;
}

int drt3d_profile_reset(void)
{
    TRY(prof_flush());
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_sum.clear();
    return DRT3D_OK;
}

int drt3d_pass_times(char* names, double* ms, long long* launches, double* bytes, int cap)
{
    TRY(prof_flush());
    std::lock_guard<std::mutex> lk(g_prof_mu);
    int i = 0;
    for (auto& kv : g_prof_sum) {
        if (i < cap) {
            if (names) {
                strncpy(names + 32 * i, kv.first.c_str(), 31);
                names[32 * i + 31] = 0;
            }
            if (ms) ms[i] = kv.second.ms;
            if (launches) launches[i] = kv.second.n;
            if (bytes) bytes[i] = kv.second.bytes;
        }
        ++i;
    }
    return i;
}

// ------------------------------------------------------------------ introspection ABI
int drt3d_frame_map(int k, int N, int kind, int out[5])
{
    if (k < 0 || k > 11 || ilog2_exact(N) < 1 || (kind != 0 && kind != 1) || !out)
        return fail(DRT3D_EINVAL, "bad arguments to drt3d_frame_map");
    const FrameMap f = kind == 0 ? drt_frame_map(k, N) : djt_frame_map(k, N);
    out[0] = f.base; out[1] = f.sx; out[2] = f.sy; out[3] = f.sd; out[4] = kind == 0 ? f.group : 0;
    return DRT3D_OK;
}

}  // extern "C"

struct drt3d_plan_s {
    int op, N, dtype;
    uint32_t mask;
    Tuning t;  // the DRT's tuning at creation
};

extern "C" {

int drt3d_plan_create(drt3d_plan* plan, int op, int N, uint32_t mask, int dtype)
{
    if (!plan) return fail(DRT3D_EINVAL, "plan is NULL");
    *plan = nullptr;
    if (op < 0 || op > 3) return fail(DRT3D_EINVAL, "op must be 0, 1, 2 or 3");
    if (dtype == DRT3D_U8) {
        if (op != 0) return fail(DRT3D_EUNSUPPORTED, "8-bit data is taken by drt3d_forward only");
        if (N < 32) return fail(DRT3D_EUNSUPPORTED, "8-bit volumes are taken for N >= 32 (got N = %d)", N);
        TRY(check_common(N, mask, DRT3D_I32));
    } else {
        TRY(check_common(N, mask, dtype));
    }
    if (op >= 2 && N > 256) return fail(DRT3D_EUNSUPPORTED, "the DJT takes N <= 256 (got N = %d)", N);
    drt3d_plan_s* p = new (std::nothrow) drt3d_plan_s;
    if (!p) return fail(DRT3D_ENOMEM, "plan: host allocation failed");
    p->op = op; p->N = N; p->dtype = dtype; p->mask = mask;
    p->t = get_tuning(N, dtype == DRT3D_F32);
    *plan = p;
    return DRT3D_OK;
}

size_t drt3d_plan_workspace_bytes(drt3d_plan p)
{
    if (!p) return 0;
    switch (p->op) {
    case 0: return drt3d_workspace_bytes(p->N, p->mask, p->dtype);
    case 1: return drt3d_adjoint_workspace_bytes(p->N, p->mask, p->dtype);
    case 2: return djt3d_workspace_bytes(p->N, p->mask, p->dtype);
    default: return djt3d_adjoint_workspace_bytes(p->N, p->mask, p->dtype);
    }
}

int drt3d_plan_execute(drt3d_plan p, const void* in, void* out, void* workspace, size_t workspace_bytes, void* stream)
{
    if (!p) return fail(DRT3D_EINVAL, "plan is NULL");
    if (p->op <= 1)
        return drt_single(in, out, p->N, p->mask, p->dtype, workspace, workspace_bytes, stream, p->op, 0, &p->t);
    return djt_single(in, out, p->N, p->mask, p->dtype, workspace, workspace_bytes, stream, p->op == 3);
}

int drt3d_plan_destroy(drt3d_plan p)
{
    delete p;
    return DRT3D_OK;
}

int drt3d_plan_text(int op, int N, uint32_t mask, int dtype, char* buf, size_t cap)
{
    TRY(check_common(N, mask, dtype));
    if (op < 0 || op > 3) return fail(DRT3D_EINVAL, "op must be 0, 1, 2 or 3");
    const int is_float = dtype == DRT3D_F32;
    // placeholder addresses: the plan's shape does not depend on them
    static char dummy[256] __attribute__((aligned(256)));
    DrtIO io{dummy, dummy, dummy};
    std::vector<std::vector<Step>> vols(1);
    if (op >= 2) TRY(djt_steps(vols[0], N, mask, 1, io, op == 3));
    else TRY(drt_steps(vols[0], N, mask, is_float, op == 1, 1, get_tuning(N, is_float), io));
    Program prog;
    prog.is_float = is_float;
    build_program(prog, vols, false);
    std::string txt;
    char line[256];
    for (const Launch& L : prog.launches) {
        // which DRT pass kernel runs: the fused adjoint group pass, a
        // shape-specialised pass (K1.K2 x wavefronts), or the generic one
        char kern[32] = "-";
        if (L.kind == S_DRT)
            snprintf(kern, sizeof kern, L.adj_group ? "group%d.%dx%d" : L.fast_kx >= 0 ? "fast%d.%dx%d" : "generic",
                     L.fast_kx, L.fast_ky, L.block / 64);
        snprintf(line, sizeof line, "%s kind=%d wg=%lld block=%d lds=%zu bytes=%.0f kernel=%s\n", L.name.c_str(),
                 L.kind, L.total_wg, L.block, L.lds, L.bytes, kern);
        txt += line;
    }
    if (buf && cap) {
        strncpy(buf, txt.c_str(), cap - 1);
        buf[cap - 1] = 0;
    }
    return (int)prog.launches.size();
}

}  // extern "C"
