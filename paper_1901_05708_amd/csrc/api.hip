// api.hip -- host side of libmp: argument validation, the per-device
// workspace, the planner that lays out a launch (one series, or a batch of
// jobs end to end) and picks the sweep kernels and their shape, the batch
// autotuner and graph cache, and the C ABI of include/mp.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <list>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mp.h"
#include "mp_internal.h"

using namespace mpk;

namespace {

thread_local std::string g_err;
thread_local int g_last_code = MP_OK;

int fail(int code, const char *what)
{
    g_last_code = code;
    g_err = what;
    return code;
}

int fail_hip(hipError_t e, const char *where)
{
    g_last_code = MP_EHIP;
    g_err = std::string(where) + ": " + hipGetErrorString(e);
    return MP_EHIP;
}

#define HIP_TRY(expr, where)                     \
    do {                                         \
        hipError_t e__ = (expr);                 \
        if (e__ != hipSuccess) return fail_hip(e__, where); \
    } while (0)

#define RC_TRY(expr)                             \
    do {                                         \
        int rc__ = (expr);                       \
        if (rc__ != MP_OK) return rc__;          \
    } while (0)

// One lock for all library state (workspace, graph and tuning caches,
// profiling records).
std::recursive_mutex g_mu;

// ---------------------------------------------------------------------------
// workspaces (grow-only), one per device and caller stream: the per-window
// arrays of every series of a launch, concatenated. Calls on different
// streams never share one, so they may run concurrently.
// ---------------------------------------------------------------------------
struct Workspace {
    int dev = 0;
    hipStream_t owner = nullptr;       // the caller stream it serves
    int64_t stream_cap = 0;            // stream entries (sum over jobs of N + STREAM_PAD)
    int64_t key_cap = 0;               // windows (sum over jobs of N)
    double *x = nullptr, *y = nullptr, *z = nullptr;
    float *xf = nullptr, *yf = nullptr, *zf = nullptr;
    double *mu = nullptr, *invn = nullptr;
    double *wsum = nullptr;            // 4 x key_cap: window sums of long z-normalized windows
    int32_t *lcount = nullptr, *lhead = nullptr;   // long-window rescoring: runs per block
    double *lanchor = nullptr;         // 2 x key_cap: and their exact first sums
    uint8_t *isconst = nullptr;
    unsigned long long *keys = nullptr;
    // exact-search queue (key_cap entries) and pivot distances
    int32_t *fb_rows = nullptr;
    int32_t *fb_job = nullptr;
    unsigned long long *fb_keys = nullptr;
    double *fb_ub = nullptr;
    float *fb_pd = nullptr;            // FB_PIVOTS x key_cap
    int32_t *counters = nullptr;
    unsigned long long *visits = nullptr;   // pair-visit counter of the test mode
    // tables of single-series calls (one job)
    Job *job1 = nullptr;
    int64_t *row_base1 = nullptr;
    int32_t *flag1 = nullptr;
    int32_t *pivots1 = nullptr;
    int64_t *band1 = nullptr;
    int64_t band1_cap = 0;
    // motif / discord extraction: exclusion mask and per-round scratch
    uint8_t *topk_mask = nullptr;
    int64_t topk_mask_cap = 0;
    unsigned long long *topk_scratch = nullptr;
    int64_t topk_scratch_cap = 0;
    // partial (anytime) sweeps: band slot -> group map, marks of the call's
    // groups, and the call's own profile when it is merged into an earlier one
    int32_t *any_map = nullptr;
    uint8_t *any_ok = nullptr;
    int64_t any_group_cap = 0;
    double *any_P = nullptr;
    int64_t *any_I = nullptr;
    int64_t any_row_cap = 0;
    uint64_t generation = 0;           // unique over all workspaces; renewed whenever
                                       // the arrays above move
    int arch_ok = -1;                  // -1 unknown, 0 no, 1 gfx950
    int cus = 0;
    // library stream and fork / join events of graph launches
    hipStream_t lib_stream = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
};

std::list<Workspace> g_ws;           // stable addresses: graph entries point at them
uint64_t g_generation = 0;

// Per device: is it a gfx950, and its compute-unit count.
struct DevInfo {
    int arch_ok = -1;                  // -1 unknown, 0 no, 1 gfx950
    int cus = 0;
};
std::vector<DevInfo> g_dev;

void free_arrays(Workspace &w)
{
    void *ptrs[] = {w.x,       w.y,      w.z,       w.xf,    w.yf,    w.zf,
                    w.mu,      w.invn,   w.wsum,    w.isconst, w.keys, w.fb_rows,
                    w.fb_job,  w.fb_keys, w.fb_ub,  w.fb_pd, w.counters, w.lcount,
                    w.lhead,   w.lanchor};
    for (void *p : ptrs) hipFree(p);
    w.x = w.y = w.z = w.mu = w.invn = w.wsum = w.fb_ub = w.lanchor = nullptr;
    w.lcount = w.lhead = nullptr;
    w.xf = w.yf = w.zf = w.fb_pd = nullptr;
    w.isconst = nullptr;
    w.keys = w.fb_keys = nullptr;
    w.fb_rows = w.fb_job = w.counters = nullptr;
    w.stream_cap = w.key_cap = 0;
    w.generation = ++g_generation;
}

void free_ws(Workspace &w)
{
    free_arrays(w);
    void *ptrs[] = {w.job1,      w.row_base1,    w.flag1,   w.pivots1, w.band1, w.visits,
                    w.topk_mask, w.topk_scratch, w.any_map, w.any_ok,  w.any_P, w.any_I};
    for (void *p : ptrs) hipFree(p);
    w.any_map = nullptr;
    w.any_ok = nullptr;
    w.any_P = nullptr;
    w.any_I = nullptr;
    w.any_group_cap = w.any_row_cap = 0;
    w.visits = nullptr;
    w.topk_mask = nullptr;
    w.topk_scratch = nullptr;
    w.topk_mask_cap = w.topk_scratch_cap = 0;
    w.job1 = nullptr;
    w.row_base1 = w.band1 = nullptr;
    w.flag1 = w.pivots1 = nullptr;
    w.band1_cap = 0;
    if (w.ev_fork) hipEventDestroy(w.ev_fork);
    if (w.ev_join) hipEventDestroy(w.ev_join);
    if (w.lib_stream) hipStreamDestroy(w.lib_stream);
    w.ev_fork = w.ev_join = nullptr;
    w.lib_stream = nullptr;
}

template <class T>
int grow(T **p, size_t count, const char *what)
{
    hipFree(*p);
    *p = nullptr;
    if (alloc_fail_hook()) return fail(MP_ENOMEM, what);
    hipError_t e = hipMalloc((void **)p, std::max<size_t>(count, 1) * sizeof(T));
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
        (void)hipGetLastError();
        return fail(MP_ENOMEM, what);
    }
    if (e != hipSuccess) return fail_hip(e, what);
    return MP_OK;
}

// The workspace of the current device and the caller's stream (created on
// first use).
int get_ws(hipStream_t st, Workspace **out, int *dev_out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    if ((int)g_dev.size() <= dev) g_dev.resize(dev + 1);
    DevInfo &di = g_dev[dev];
    if (di.arch_ok < 0) {
        hipDeviceProp_t prop;
        HIP_TRY(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
        di.arch_ok = (std::strncmp(prop.gcnArchName, "gfx950", 6) == 0) ? 1 : 0;
        di.cus = prop.multiProcessorCount;
    }
    if (!di.arch_ok) return fail(MP_EUNSUPPORTED, "the current HIP device is not a gfx950 GPU");
    Workspace *wp = nullptr;
    for (Workspace &x : g_ws)
        if (x.dev == dev && x.owner == st) {
            wp = &x;
            break;
        }
    if (!wp) {
        g_ws.emplace_back();
        wp = &g_ws.back();
        wp->dev = dev;
        wp->owner = st;
        wp->arch_ok = 1;
        wp->cus = di.cus;
        wp->generation = ++g_generation;
    }
    Workspace &w = *wp;
    if (!w.job1) {
        RC_TRY(grow(&w.job1, 1, "workspace job table"));
        RC_TRY(grow(&w.row_base1, 4, "workspace job table"));
        RC_TRY(grow(&w.flag1, 1, "workspace job table"));
        RC_TRY(grow(&w.pivots1, FB_PIVOTS, "workspace job table"));
        RC_TRY(grow(&w.visits, 1, "workspace counter"));
    }
    *out = &w;
    *dev_out = dev;
    return MP_OK;
}

int ensure_arrays(Workspace &w, int64_t streams, int64_t keys)
{
    if (w.stream_cap >= streams && w.key_cap >= keys) return MP_OK;
    const int64_t scap = std::max<int64_t>(streams, w.stream_cap + w.stream_cap / 2);
    const int64_t kcap = std::max<int64_t>(keys, w.key_cap + w.key_cap / 2);
    free_arrays(w);
    int rc;
    if ((rc = grow(&w.x, scap, "workspace x")) || (rc = grow(&w.y, scap, "workspace y")) ||
        (rc = grow(&w.z, scap, "workspace z")) || (rc = grow(&w.xf, scap, "workspace xf")) ||
        (rc = grow(&w.yf, scap, "workspace yf")) || (rc = grow(&w.zf, scap, "workspace zf")) ||
        (rc = grow(&w.mu, kcap, "workspace mu")) || (rc = grow(&w.invn, kcap, "workspace invn")) ||
        (rc = grow(&w.wsum, (size_t)kcap * 4, "workspace window sums")) ||
        (rc = grow(&w.lcount, kcap, "workspace rescoring runs")) ||
        (rc = grow(&w.lhead, kcap, "workspace rescoring runs")) ||
        (rc = grow(&w.lanchor, (size_t)kcap * 2, "workspace rescoring anchors")) ||
        (rc = grow(&w.isconst, kcap, "workspace const")) ||
        (rc = grow(&w.keys, kcap, "workspace keys")) ||
        (rc = grow(&w.fb_rows, kcap, "workspace fallback rows")) ||
        (rc = grow(&w.fb_job, kcap, "workspace fallback jobs")) ||
        (rc = grow(&w.fb_keys, kcap, "workspace fallback keys")) ||
        (rc = grow(&w.fb_ub, kcap, "workspace fallback bounds")) ||
        (rc = grow(&w.fb_pd, (size_t)kcap * FB_PIVOTS, "workspace pivot distances")) ||
        (rc = grow(&w.counters, 64, "workspace counters"))) {
        free_arrays(w);
        return rc;
    }
    w.stream_cap = scap;
    w.key_cap = kcap;
    return MP_OK;
}

int ensure_band1(Workspace &w, int64_t entries)
{
    if (w.band1_cap >= entries) return MP_OK;
    const int64_t cap = std::max<int64_t>(entries, 4096);
    int rc = grow(&w.band1, cap, "workspace bands");
    if (rc) {
        w.band1_cap = 0;
        return rc;
    }
    w.band1_cap = cap;
    return MP_OK;
}

int ensure_any(Workspace &w, int64_t groups, int64_t rows)
{
    if (w.any_group_cap < groups) {
        const int64_t cap = std::max<int64_t>(groups, 1024);
        w.any_group_cap = 0;
        RC_TRY(grow(&w.any_map, cap, "workspace group map"));
        RC_TRY(grow(&w.any_ok, cap, "workspace group marks"));
        w.any_group_cap = cap;
    }
    if (w.any_row_cap < rows) {
        w.any_row_cap = 0;
        RC_TRY(grow(&w.any_P, rows, "workspace partial profile"));
        RC_TRY(grow(&w.any_I, rows, "workspace partial profile"));
        w.any_row_cap = rows;
    }
    return MP_OK;
}

int ensure_lib_stream(Workspace &w)
{
    if (w.lib_stream) return MP_OK;
    HIP_TRY(hipStreamCreateWithFlags(&w.lib_stream, hipStreamNonBlocking), "hipStreamCreate");
    HIP_TRY(hipEventCreateWithFlags(&w.ev_fork, hipEventDisableTiming), "hipEventCreate");
    HIP_TRY(hipEventCreateWithFlags(&w.ev_join, hipEventDisableTiming), "hipEventCreate");
    return MP_OK;
}

// ---------------------------------------------------------------------------
// profiling
// ---------------------------------------------------------------------------
struct EvSet {
    hipEvent_t ev[4];
    int32_t *fb_host = nullptr;   // pinned copy of the call's fallback count
    unsigned long long *visits_host = nullptr;   // and of its pair-visit count
};

struct Prof {
    bool on = false;
    std::vector<EvSet> pending;
    mp_stats acc{};
};
Prof g_prof;

int prof_begin(hipStream_t st, EvSet *es, bool *active)
{
    *active = g_prof.on;
    if (!*active) return MP_OK;
    for (int k = 0; k < 4; ++k) HIP_TRY(hipEventCreate(&es->ev[k]), "hipEventCreate");
    HIP_TRY(hipHostMalloc((void **)&es->fb_host, sizeof(int32_t), hipHostMallocDefault),
            "hipHostMalloc");
    HIP_TRY(hipHostMalloc((void **)&es->visits_host, sizeof(unsigned long long),
                          hipHostMallocDefault),
            "hipHostMalloc");
    *es->fb_host = 0;
    *es->visits_host = 0;
    HIP_TRY(hipEventRecord(es->ev[0], st), "hipEventRecord");
    return MP_OK;
}

// ---------------------------------------------------------------------------
// validation and planning
// ---------------------------------------------------------------------------
// Index bits of a global key: 2^gb > N, so the all-ones index field never
// names a window and can mark an illegal winner.
int32_t index_bits(int64_t N)
{
    int32_t b = 1;
    while (b < 40 && ((int64_t)1 << b) <= N) ++b;
    return b;
}

int64_t pair_count(int64_t N, int64_t excl)
{
    if (N <= excl) return 0;
    int64_t k = N - excl;
    return k * (k + 1) / 2;
}

static_assert(ANY_GROUP == MP_ANYTIME_GROUP && ANY_GROUP == 64 * 8,
              "a group of a partial sweep is one band of the FP64 band kernel");

// Diagonal groups of a partial sweep: group g holds diagonals
// [excl + g ANY_GROUP, excl + (g + 1) ANY_GROUP) that are below N.
int64_t any_groups(int64_t N, int64_t excl)
{
    return N - excl > 0 ? (N - excl + ANY_GROUP - 1) / ANY_GROUP : 0;
}

// Pairs of group g: sum over its diagonals d of N - d.
int64_t group_pairs(int64_t N, int64_t excl, int64_t g)
{
    const int64_t d0 = excl + g * ANY_GROUP, d1 = std::min<int64_t>(d0 + ANY_GROUP, N);
    if (d1 <= d0) return 0;
    const int64_t c = d1 - d0;
    return c * N - c * (d0 + d1 - 1) / 2;
}

int32_t pclass_of(double p)
{
    if (p == 1.0) return P_ONE;
    if (p == 2.0) return P_TWO;
    if (p == 3.0) return P_THREE;
    return P_GENERIC;
}

// One validated series request.
struct Spec {
    const double *T;
    int64_t n;
    int32_t m, kind, pclass, excl, R;
    double p;
    double *P;
    int64_t *I;
    // partial sweep: the diagonal groups to visit (host array); ngroups < 0
    // for a whole profile
    const int32_t *groups = nullptr;
    int64_t ngroups = -1;
    int32_t fcmp = 0;          // ACAMP compared on F (Sec. 4.4), FP64 band sweep
};

int make_spec(const double *T, int64_t n, int32_t m, int32_t kind, double p, int32_t excl,
              int32_t R, double *P, int64_t *I, Spec *out)
{
    if (!T || !P || !I) return fail(MP_EINVAL, "null pointer argument");
    if (n < 1) return fail(MP_EINVAL, "n must be >= 1");
    if (n >= MP_MAX_N) return fail(MP_EINVAL, "n must be < 2^31");
    if (m < 1 || (int64_t)m > n) return fail(MP_EINVAL, "m must satisfy 1 <= m <= n");
    if (R < 0) return fail(MP_EINVAL, "R must be >= 0");
    if (kind < AAMP || kind > ACAMP) return fail(MP_EINVAL, "kind must be MP_KIND_*");
    if (kind == PNORM && !(std::isfinite(p) && p >= 1.0))
        return fail(MP_EINVAL, "p must be finite and >= 1");
    Spec s;
    s.T = T;
    s.n = n;
    s.m = m;
    s.kind = (kind == PNORM && p == 2.0) ? AAMP : kind;   // Sec. 3.4: p = 2 is Euclid
    s.p = s.kind == PNORM ? p : 2.0;
    s.pclass = s.kind == PNORM ? pclass_of(p) : P_TWO;
    s.excl = excl > 0 ? excl : (m + 3) / 4;
    s.R = R;
    s.P = P;
    s.I = I;
    *out = s;
    return MP_OK;
}

int check_precision(int32_t precision)
{
    if (precision != MP_FP64 && precision != MP_FP32_REFRESH && precision != MP_FP32_AUTO)
        return fail(MP_EINVAL, "precision must be MP_FP64, MP_FP32_REFRESH or MP_FP32_AUTO");
    return MP_OK;
}

// Shape knobs of a launch: diagonals per lane (band width / 64), the refresh
// interval of jobs that leave R to the library (0: per-distance default), the
// persistent grid as a multiple of the resident waves, and a cap on the waves
// per SIMD of the grid (0: every resident slot).
struct Tuning {
    int32_t kd = 8;
    int32_t R = 0;
    int32_t grid_mult = 1;
    int32_t wps = 0;
    // MP_FP32_AUTO only: sweep every job in FP64, which meets the FP32
    // tolerance; chosen when it times faster than every FP32 candidate
    bool sweep64 = false;
};

// Longest FP64 refresh interval per window length. A step's rounding error is
// relative to the per-sample scale of the streams (offset, low-variance
// windows are the hard case), while the quantity it perturbs grows with m, so
// the drift after R steps falls with m at a fixed R / m. With window means
// summed around each window's first sample, random walks with constant runs
// and planted motifs, and their affine copies with offset / scale = 1e6,
// showed no drift beyond the 1e-9 bound up to R / m = 256 (m = 256, 1024,
// 4096); the cap of 64 leaves a factor 4.
constexpr int64_t FP64_R_PER_M = 64;

// Default refresh intervals. In FP64, 4096, or 16 m for long windows: R only
// trades the restart cost (m per diagonal) against item count. In FP32 every
// step can add 2^-24 relative error; the values below minimise sweep plus
// exact-search time on the series shapes measured.
int32_t default_R(uint32_t sel, bool fp32, int32_t m)
{
    if (!fp32) return (int32_t)std::min<int64_t>(std::max<int64_t>(4096, 16 * (int64_t)m), 1 << 24);
    int64_t r = 256;
    switch (sel) {
    case SEL_ACAMP: r = 512; break;
    case SEL_P1: r = 1024; break;
    default: break;
    }
    // at least 2m rows per restart of m operations per diagonal
    return (int32_t)std::min<int64_t>(std::max<int64_t>(r, 2 * (int64_t)m), 1 << 24);
}

// Where a band's exact restart goes in the split of the row space: a band of
// L rows takes band_cost + L positions, so that a wave whose share holds many
// short bands (the end of every triangle) is not left with all their
// restarts. By instruction count a restart of m samples costs about m / 6
// rows of the sweep (about 11 VALU operations per sample and lane against 71
// per row, Euclidean and z-normalized), but it runs at a lower issue rate;
// measured over m / 8 ... m / 3 on the long windows of the uniform series,
// m / 4 balanced the waves best (m = 16384: 2800 -> 3215 G pairs/s, m = 65536:
// 1455 -> 1575, both Euclidean, against m / 8), with the headline unchanged.
// The p-norm restarts take 2-4 operations per sample, and for other p one pow
// per sample against two per pair, so they are charged in proportion.
int32_t band_cost(uint32_t sel, int32_t m)
{
    if (sel == SEL_PGEN) return m;
    const bool pnorm = sel == SEL_P1 || sel == SEL_P3;
    return pnorm ? (m + 1) / 2 : (m + 3) / 4;
}

// Rows summed over all bands (band b: N - excl - b W rows) and the band count.
int64_t band_rows_total(int64_t N, int64_t excl, int64_t W, int64_t *nbands)
{
    const int64_t nd = N - excl;
    const int64_t nb = (nd + W - 1) / W;
    *nbands = nb;
    return nb * nd - W * (nb * (nb - 1) / 2);
}

// Windows shorter than this are swept in FP64 even under MP_FP32_REFRESH: with
// few terms per window the running sum can shrink by orders of magnitude
// within a few steps, and the error it carried from its larger past is then
// amplified far beyond what the winner's self-check can see.
constexpr int32_t FP32_MIN_M = 32;

// Distances with an FP32 sweep: ACAMP and p = 1. The certification checks the
// winner's FP32 drift only. The AAMP and p = 3 sums cancel large increments
// against small best-match sums, so a row's true best candidate can drift by
// more than its winner and lose unseen: every-row checks against the oracle
// found the 131072-sample walk's row 113495 2.79e-4 above its minimum (AAMP),
// the sines workload's row 30128 1.004e-4 above (p = 3), and five rows of the
// 512-series batch, identically with and without per-item recentring of the
// operands. Replaying the walk's row in single precision on the host put the
// drift of its true best pair at 2.2e-3 rms from the running sum's rounding
// (u |S| per step, S large away from the match) against 1.5e-5 from the
// rounded operands. ACAMP keys 1 - rho next to 1 and met 1e-4 on every row of
// every workload. Other distances run the FP64 sweep under MP_FP32_REFRESH.
constexpr uint32_t SEL_FP32 = SEL_ACAMP | SEL_P1;

// A band sweep of a launch: a contiguous range of the job table, all of one
// distance specialisation and precision, with its own band-row space. Each
// runs the kernel specialised for its distance.
struct Group {
    int32_t first = 0, count = 0;
    int64_t rows = 0;
    int64_t rb_off = 0;        // its row_base entries (count + 1) in the table
    uint32_t sels = 0;
    int32_t grid = 0;
    int32_t kd = 8;            // diagonals per lane
    bool fp32 = false;
    int32_t wpb = 1;           // waves per block of the sweep launch
};

// A launch laid out: the job table (pointers bound to a workspace by bind())
// ordered as [band jobs by group: FP64 groups, then FP32 groups][other jobs],
// each band sweep's row_base prefix, and the sizes of every per-launch array.
struct Layout {
    std::vector<Job> jobs;
    std::vector<int64_t> row_base;       // per group: count + 1 entries
    std::vector<int64_t> stream_off;     // per job (table order)
    std::vector<Group> groups;
    int64_t band_entries = 0;
    int64_t stream_total = 0, key_total = 0;
    int64_t max_N = 0, max_stream = 0, simple_diag = 0, simple_segs = 0;
    uint32_t sels = 0;
    int32_t kd = 8;
    int64_t pairs = 0, items = 0;
    int32_t R_report = 0;
    int32_t band_jobs = 0, fp32_jobs = 0;
    bool count = false;                  // pair-visit counting (test mode)
    // Whether a row can reach the exact search: an ACAMP job (a constant
    // partner can win the sweep), an FP32 sweep (its self-check) or the test
    // hook. FP64 Euclidean and p-norm sweeps key admissible pairs only.
    bool exact_search = false;
};

int env_int(const char *name, int dflt)
{
    const char *e = std::getenv(name);
    return e ? std::atoi(e) : dflt;
}

// Lay out a launch. A job goes to the band kernel when its distance has one
// and it has at least half a band of diagonals; otherwise to the simple
// kernel (FP64 only: a single-precision request on such a job is served
// exactly in FP64). Test hooks: MP_SWEEP=band|simple forces a kernel,
// MP_KD=16 requests 16 diagonals per lane (FP32 only), MP_WPS=k caps the band
// sweeps' grids at k waves per SIMD, MP_FORCE_FALLBACK=1|2 sends every row
// through the exact search, MP_COUNT_PAIRS=1 makes the sweeps count the pairs
// they visit (reported with profiling on).
int make_layout(const std::vector<Spec> &specs, int32_t precision, const Tuning &tu,
                const Workspace &w, Layout *out)
{
    Layout L;
    const bool want32 =
        precision == MP_FP32_REFRESH || (precision == MP_FP32_AUTO && !tu.sweep64);
    const char *sw = std::getenv("MP_SWEEP");
    const std::string choice = sw ? sw : "auto";
    // diagonals per lane of the FP32 sweep; the FP64 sweep always uses 8
    // (16 FP64 diagonals per lane exceed the register file)
    int32_t kd = tu.kd;
    if (env_int("MP_KD", 0) == 16) kd = 16;
    if (!want32) kd = 8;
    int force_fb = env_int("MP_FORCE_FALLBACK", 0);
    if (force_fb != 1 && force_fb != 2) force_fb = 0;
    L.count = env_int("MP_COUNT_PAIRS", 0) == 1;

    // Classes of jobs: band jobs by precision and specialisation (index
    // 128 fp32 + selector and launch-flag bits, so FP64 classes come first),
    // then the rest.
    constexpr int NCLS = 257, OTHER = 256;
    std::vector<Job> cls[NCLS];
    std::vector<int64_t> rows_of[NCLS];  // band rows
    std::vector<int64_t> pos_of[NCLS];   // positions in the row space (rows + restart costs)
    for (const Spec &sp : specs) {
        Job j;
        std::memset(&j, 0, sizeof(j));
        Series &s = j.s;
        s.T = sp.T;
        s.n = sp.n;
        s.N = sp.n - sp.m + 1;
        s.m = sp.m;
        s.kind = sp.kind;
        s.pclass = sp.pclass;
        s.excl = sp.excl;
        s.p = sp.p;
        s.gb = index_bits(s.N);
        s.force_fb = force_fb;
        if (force_fb) L.exact_search = true;
        j.P = sp.P;
        j.I = sp.I;
        const uint32_t sel = sel_of(s.kind, s.pclass);
        const int64_t ndiag = s.N - s.excl;
        const bool partial = sp.ngroups >= 0;     // FP64 band sweep over the listed groups
        // the sweep this job would join decides its band width
        s.fcmp = sp.fcmp;
        const bool single =
            !partial && !sp.fcmp && want32 && s.m >= FP32_MIN_M && (sel & SEL_FP32);
        const int64_t W = 64 * (single ? kd : 8);
        const bool has_band = (sel & SEL_BAND) || (sel == SEL_PGEN && sp.p <= PGEN_BAND_MAX);
        bool band = has_band && ndiag >= W / 2 && choice != "simple";
        if (choice == "band" && has_band && ndiag > 0) band = true;
        if (ndiag <= 0) band = false;
        if (partial) band = true;
        s.fp32 = (single && band) ? 1 : 0;
        if (s.fp32 || s.kind == ACAMP) L.exact_search = true;
        int64_t rows = 0, nb = 0;
        if (partial) {
            nb = sp.ngroups;
            for (int64_t t = 0; t < nb; ++t) rows += s.N - s.excl - (int64_t)sp.groups[t] * W;
        } else if (band) {
            rows = band_rows_total(s.N, s.excl, W, &nb);
        }
        if (band) {
            L.band_jobs += 1;
            L.fp32_jobs += s.fp32;
            j.band_cost = band_cost(sel, s.m);
            int64_t R = sp.R > 0 ? sp.R
                                 : (tu.R > 0 && s.fp32 == want32 ? tu.R : default_R(sel, s.fp32, s.m));
            j.seg_rows = (int32_t)std::min<int64_t>(R, INT32_MAX / 2);
            if (L.R_report == 0) L.R_report = j.seg_rows;
        } else if (ndiag > 0) {
            // the simple kernel's grid has one row of blocks per segment
            int64_t R = sp.R > 0 ? sp.R : 1024;
            R = std::max<int64_t>(R, (ndiag + 65534) / 65535);
            j.seg_rows = (int32_t)R;
            L.simple_diag = std::max(L.simple_diag, ndiag);
            L.simple_segs = std::max(L.simple_segs, (ndiag + R - 1) / R);
        }
        j.nbands = (int32_t)nb;
        L.sels |= sel;
        if (partial)
            for (int64_t t = 0; t < nb; ++t) L.pairs += group_pairs(s.N, s.excl, sp.groups[t]);
        else
            L.pairs += pair_count(s.N, s.excl);
        L.items += nb + (band ? rows / j.seg_rows : 0);
        const bool longw = !s.fp32 && s.m >= LONG_WINDOW && (sel & (SEL_AAMP | SEL_P1 | SEL_P3));
        const int c = band ? 128 * s.fp32 + (int)(sel | (s.fcmp ? SEL_FCMP : 0u) |
                                                  (longw ? SEL_LONG : 0u))
                           : OTHER;
        cls[c].push_back(j);
        rows_of[c].push_back(rows);
        pos_of[c].push_back(rows + nb * (int64_t)j.band_cost);
    }
    for (int c = 0; c < NCLS; ++c) {
        if (cls[c].empty()) continue;
        const bool grp = c != OTHER;
        if (grp) {
            Group g;
            g.first = (int32_t)L.jobs.size();
            g.count = (int32_t)cls[c].size();
            g.rb_off = (int64_t)L.row_base.size();
            g.sels = (uint32_t)(c & 127);
            g.fp32 = c >= 128;
            g.kd = g.fp32 ? kd : 8;
            L.groups.push_back(g);
        }
        int64_t run = 0, real = 0;
        for (size_t k = 0; k < cls[c].size(); ++k) {
            Job j = cls[c][k];
            const Series &s = j.s;
            j.row_start = run;
            if (grp) L.row_base.push_back(run);
            run += pos_of[c][k];
            real += rows_of[c][k];
            j.band_base = L.band_entries;
            L.band_entries += j.nbands + 1;
            j.key_base = L.key_total;
            L.stream_off.push_back(L.stream_total);
            L.key_total += s.N;
            L.stream_total += s.N + STREAM_PAD;
            L.max_N = std::max(L.max_N, s.N);
            L.max_stream = std::max(L.max_stream, s.N + STREAM_PAD);
            L.jobs.push_back(j);
        }
        if (grp) {
            L.row_base.push_back(run);
            L.groups.back().rows = real;
        }
    }
    L.kd = kd;
    for (Group &g : L.groups) {
        if (!g.rows) continue;
        int64_t slots = (int64_t)w.cus * band_blocks_per_cu(g.sels, g.kd, g.fp32);
        const int32_t wps = env_int("MP_WPS", 0) > 0 ? env_int("MP_WPS", 0) : tu.wps;
        if (wps > 0) slots = std::min<int64_t>(slots, (int64_t)w.cus * 4 * wps);
        // at least 64 rows per wave
        g.grid = (int32_t)std::max<int64_t>(
            1, std::min<int64_t>(slots * std::max(1, tu.grid_mult), g.rows / 64));
        // A grid capped below the kernel's occupancy runs in blocks of four
        // waves: blocks of one wave have landed two on one SIMD and none on
        // another (up to 1.4 times the sweep time), a block's four waves go
        // to four SIMDs.
        if (wps > 0 && !L.count && g.grid >= 4 && band_has_wave_blocks(g.sels, g.kd, g.fp32)) {
            g.wpb = 4;
            g.grid -= g.grid % 4;
        }
        L.items += g.grid;
    }
    *out = std::move(L);
    return MP_OK;
}

// Point every job at its slices of the workspace.
void bind(Layout &L, const Workspace &w)
{
    for (size_t b = 0; b < L.jobs.size(); ++b) {
        Series &s = L.jobs[b].s;
        const int64_t so = L.stream_off[b], ko = L.jobs[b].key_base;
        s.x = w.x + so;
        s.y = w.y + so;
        s.z = w.z + so;
        s.xf = w.xf + so;
        s.yf = w.yf + so;
        s.zf = w.zf + so;
        s.mu = w.mu + ko;
        s.invn = w.invn + ko;
        s.wsum = w.wsum + 4 * ko;
        s.lcount = w.lcount + ko;
        s.lhead = w.lhead + ko;
        s.lanchor = w.lanchor + 2 * ko;
        s.isconst = w.isconst + ko;
        s.keys = w.keys + ko;
    }
}

// Device tables of a launch.
struct Tables {
    Job *jobs = nullptr;
    int64_t *row_base = nullptr;
    int64_t *band = nullptr;
    int32_t *flags = nullptr;
    int32_t *pivots = nullptr;
};

Batch make_batch(const Layout &L, const Workspace &w, const Tables &t)
{
    Batch b;
    std::memset(&b, 0, sizeof(b));
    b.jobs = t.jobs;
    b.row_base = t.row_base;
    b.band_start = t.band;
    b.njobs = (int32_t)L.jobs.size();
    b.band_width = 64 * 8;
    b.max_N = L.max_N;
    b.max_stream = L.max_stream;
    b.simple_diag = L.simple_diag;
    b.simple_segs = L.simple_segs;
    Fallback &fb = b.fb;
    fb.count = w.counters;
    fb.rows = w.fb_rows;
    fb.job = w.fb_job;
    fb.keys = w.fb_keys;
    fb.ub = w.fb_ub;
    fb.job_flag = t.flags;
    fb.pivots = t.pivots;
    fb.pd = w.fb_pd;
    fb.pd_stride = w.key_cap;
    fb.capacity = (int32_t)std::min<int64_t>(L.key_total, INT32_MAX);
    b.visits = L.count ? w.visits : nullptr;
    for (const Job &j : L.jobs) b.long_jobs |= j.s.m >= LONG_WINDOW ? 1 : 0;
    return b;
}

// The view of a launch that one band sweep works on.
Batch group_view(const Batch &b, const Group &g)
{
    Batch v = b;
    v.jobs = b.jobs + g.first;
    v.njobs = g.count;
    v.row_base = b.row_base + g.rb_off;
    v.band_width = 64 * g.kd;
    return v;
}

// The pipeline of a launch, enqueued on st: band tables, window statistics and
// difference streams, sweeps, rescoring and the exact search. With es,
// records its events after the preparation, the sweeps and the whole pipeline
// (ev[0] is recorded by the caller).
int enqueue(const Batch &b, const Layout &L, hipStream_t st, EvSet *es)
{
    for (const Group &g : L.groups) HIP_TRY(launch_plan(group_view(b, g), st), "plan launch");
    HIP_TRY(launch_prep(b, L.sels, st), "prep launch");
    if (es) HIP_TRY(hipEventRecord(es->ev[1], st), "hipEventRecord");
    for (const Group &g : L.groups)
        if (g.grid)
            HIP_TRY(launch_sweep_band(group_view(b, g), g.sels, g.kd, g.fp32, g.grid, g.wpb, st),
                    "sweep launch");
    if (L.simple_diag > 0) HIP_TRY(launch_sweep_simple(b, st), "sweep launch");
    if (es) HIP_TRY(hipEventRecord(es->ev[2], st), "hipEventRecord");
    HIP_TRY(launch_finalize(b, st), "finalize launch");
    if (L.exact_search) HIP_TRY(launch_fallback(b, st), "fallback launch");
    return MP_OK;
}

int finish_profile(EvSet &es, const Batch &b, const Layout &L, hipStream_t st)
{
    HIP_TRY(hipMemcpyAsync(es.fb_host, b.fb.count, sizeof(int32_t), hipMemcpyDeviceToHost, st),
            "hipMemcpyAsync");
    if (b.visits)
        HIP_TRY(hipMemcpyAsync(es.visits_host, b.visits, sizeof(unsigned long long),
                               hipMemcpyDeviceToHost, st),
                "hipMemcpyAsync");
    HIP_TRY(hipEventRecord(es.ev[3], st), "hipEventRecord");
    g_prof.pending.push_back(es);
    mp_stats &a = g_prof.acc;
    a.calls += 1;
    int32_t kd = 0;
    for (const Group &g : L.groups) {
        a.sweep_launches += g.grid ? 1 : 0;
        if (g.grid) kd = std::max(kd, g.kd);
    }
    a.sweep_launches += L.simple_diag > 0 ? 1 : 0;
    a.pairs += L.pairs;
    a.refresh_rows = L.R_report;
    a.diags_per_lane = kd;
    a.items = (int32_t)std::min<int64_t>(L.items, INT32_MAX);
    a.band_jobs = L.band_jobs;
    a.fp32_jobs = L.fp32_jobs;
    return MP_OK;
}

// ---------------------------------------------------------------------------
// batches: autotuner, uploaded tables and captured graphs
// ---------------------------------------------------------------------------
struct TuneEntry {
    int dev;
    int32_t precision;
    std::vector<int64_t> shape;   // per job: n, m, kind, excl, R, p bits
    Tuning best;
};
std::vector<TuneEntry> g_tune;

struct GraphEntry {
    int dev = 0;
    int32_t precision = 0;
    std::vector<mp_job> table;
    const double *T = nullptr;
    const double *P = nullptr;
    const int64_t *I = nullptr;
    uint64_t generation = 0;
    const Workspace *ws = nullptr;   // the workspace its pointers point into
    Layout L;
    Tables t;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};
std::list<GraphEntry> g_graphs;      // most recently used first
constexpr size_t GRAPH_CACHE = 16;

void free_tables(Tables &t)
{
    hipFree(t.jobs);
    hipFree(t.row_base);
    hipFree(t.band);
    hipFree(t.flags);
    hipFree(t.pivots);
    t = Tables();
}

void free_entry(GraphEntry &e)
{
    if (e.exec) hipGraphExecDestroy(e.exec);
    if (e.graph) hipGraphDestroy(e.graph);
    e.exec = nullptr;
    e.graph = nullptr;
    free_tables(e.t);
}

bool same_table(const std::vector<mp_job> &a, const mp_job *b, int32_t n)
{
    return (int32_t)a.size() == n && (n == 0 || std::memcmp(a.data(), b, n * sizeof(mp_job)) == 0);
}

std::vector<int64_t> shape_of(const mp_job *jobs, int32_t njobs)
{
    std::vector<int64_t> v;
    v.reserve((size_t)njobs * 6);
    for (int32_t b = 0; b < njobs; ++b) {
        int64_t pb;
        std::memcpy(&pb, &jobs[b].p, sizeof(pb));
        v.insert(v.end(), {jobs[b].n, jobs[b].m, jobs[b].kind, jobs[b].excl, jobs[b].R, pb});
    }
    return v;
}

int upload_tables(const Layout &L, Tables *t)
{
    const size_t nj = L.jobs.size();
    RC_TRY(grow(&t->jobs, nj, "batch job table"));
    RC_TRY(grow(&t->row_base, L.row_base.size(), "batch job table"));
    RC_TRY(grow(&t->band, (size_t)L.band_entries, "batch band table"));
    RC_TRY(grow(&t->flags, nj, "batch job table"));
    RC_TRY(grow(&t->pivots, nj * FB_PIVOTS, "batch job table"));
    HIP_TRY(hipMemcpy(t->jobs, L.jobs.data(), nj * sizeof(Job), hipMemcpyHostToDevice),
            "hipMemcpy job table");
    HIP_TRY(hipMemcpy(t->row_base, L.row_base.data(), L.row_base.size() * sizeof(int64_t),
                      hipMemcpyHostToDevice),
            "hipMemcpy job table");
    return MP_OK;
}

// Candidate shapes of the autotuner: band width (diagonals per lane; 16 only
// fits the register file in FP32) times refresh interval. In FP64 the interval
// stays within FP64_R_PER_M times the shortest window of the launch; long
// windows also try grids of one or two waves per SIMD, since every wave pays
// at least one O(m) restart. MP_FP32_AUTO tries the FP32 and the FP64 shapes.
std::vector<Tuning> tune_candidates(int32_t precision, int32_t m_min)
{
    std::vector<Tuning> c;
    if (precision != MP_FP64) {
        for (int kd : {8, 16})
            for (int R : {256, 512, 1024, 2048}) c.push_back(Tuning{kd, R, 1, 0});
        // long windows: the restart costs about 2m / R operations per pair,
        // so short intervals lose to the FP64 sweep's; the self-check still
        // decides which rows the longer FP32 runs leave uncertified
        if (m_min >= 1024) {
            for (int64_t f : {4, 16})
                c.push_back(Tuning{8, (int32_t)std::min<int64_t>(f * m_min, 1 << 24), 1, 0});
            if (m_min >= 2048)
                for (int wps : {1, 2})
                    c.push_back(
                        Tuning{8, (int32_t)std::min<int64_t>(16 * (int64_t)m_min, 1 << 24), 1, wps});
        }
    }
    if (precision != MP_FP32_REFRESH) {
        const bool sweep64 = precision == MP_FP32_AUTO;
        for (int R : {1024, 2048, 4096}) c.push_back(Tuning{8, R, 1, 0, sweep64});
        const int64_t rmax = std::min<int64_t>(FP64_R_PER_M * m_min, 1 << 24);
        if (rmax / 2 > 4096) c.push_back(Tuning{8, (int32_t)(rmax / 2), 1, 0, sweep64});
        if (rmax > 4096) c.push_back(Tuning{8, (int32_t)rmax, 1, 0, sweep64});
        if (m_min >= 2048)
            for (int wps : {1, 2}) c.push_back(Tuning{8, (int32_t)rmax, 1, wps, sweep64});
    }
    return c;
}

int record(hipEvent_t e, hipStream_t s)
{
    HIP_TRY(hipEventRecord(e, s), "hipEventRecord");
    return MP_OK;
}

// The slower of two timed runs of a candidate (after a first, warming run)
// on stream ls. Grids of one wave per SIMD can run either at full speed or
// about 1.4 times slower from one launch to the next (the same grid measured
// 9.2 and 13.4 ms on long windows: on some launches the hardware puts two of
// the one-wave blocks on one SIMD and none on another; capped grids now run
// in blocks of four waves where the kernel has such an instance), so a
// candidate counts as fast only if both of its runs are; its faster run alone
// would let such a grid win on a lucky trial and then run slow. A candidate
// whose first run already takes 1.5 times the best time so far (best >= 0) is
// not run again: its first time is reported.
int time_candidate(const std::vector<Spec> &specs, int32_t precision, const Tuning &tu,
                   Workspace &w, hipStream_t ls, hipEvent_t e0, hipEvent_t e1, float best,
                   float *ms)
{
    Layout L;
    RC_TRY(make_layout(specs, precision, tu, w, &L));
    RC_TRY(ensure_arrays(w, L.stream_total, L.key_total));
    bind(L, w);
    Tables t;
    int rc = upload_tables(L, &t);
    if (!rc) {
        const Batch b = make_batch(L, w, t);
        auto timed_run = [&](float *out) {
            int r;
            if ((r = record(e0, ls)) || (r = enqueue(b, L, ls, nullptr)) || (r = record(e1, ls)))
                return r;
            hipError_t e = hipEventSynchronize(e1);
            if (e == hipSuccess) e = hipEventElapsedTime(out, e0, e1);
            return e == hipSuccess ? MP_OK : fail_hip(e, "autotune timing");
        };
        float first = 0.0f;
        rc = timed_run(&first);
        const bool hopeless = !rc && best >= 0.0f && first > 1.5f * best;
        if (hopeless) *ms = first;
        for (int rep = 0; rep < 2 && !rc && !hopeless; ++rep) {
            float tr = 0.0f;
            if (!(rc = timed_run(&tr)) && (rep == 0 || tr > *ms)) *ms = tr;
        }
        hipError_t es = hipStreamSynchronize(ls);
        if (!rc && es != hipSuccess) rc = fail_hip(es, "autotune");
    }
    free_tables(t);
    return rc;
}

// Time every candidate on the batch itself, on the library stream after the
// caller's pending work, and keep the fastest. The runs write the caller's
// outputs, which the real run overwrites.
int autotune(const std::vector<Spec> &specs, int32_t precision, Workspace &w, hipStream_t caller,
             Tuning *best)
{
    RC_TRY(ensure_lib_stream(w));
    hipStream_t ls = w.lib_stream;
    HIP_TRY(hipEventRecord(w.ev_fork, caller), "hipEventRecord");
    HIP_TRY(hipStreamWaitEvent(ls, w.ev_fork, 0), "hipStreamWaitEvent");
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0), "hipEventCreate");
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return fail(MP_EHIP, "hipEventCreate");
    }
    float best_ms = -1.0f;
    int rc = MP_OK;
    int32_t m_min = INT32_MAX;
    for (const Spec &sp : specs) m_min = std::min(m_min, sp.m);
    for (const Tuning &tu : tune_candidates(precision, m_min)) {
        float ms = 0.0f;
        if ((rc = time_candidate(specs, precision, tu, w, ls, e0, e1, best_ms, &ms))) break;
        if (best_ms < 0.0f || ms < best_ms) {
            best_ms = ms;
            *best = tu;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return rc;
}

// Tuning of a launch shape: cached per device, precision and shape (the job
// table without offsets); computed by autotune() on first use unless
// MP_AUTOTUNE=0, in which case the defaults apply.
int tuning_for(const std::vector<Spec> &specs, const mp_job *jobs, int32_t njobs,
               int32_t precision, Workspace &w, int dev, hipStream_t st, Tuning *tu)
{
    const std::vector<int64_t> shape = shape_of(jobs, njobs);
    for (const TuneEntry &te : g_tune)
        if (te.dev == dev && te.precision == precision && te.shape == shape) {
            *tu = te.best;
            return MP_OK;
        }
    *tu = Tuning();
    if (env_int("MP_AUTOTUNE", 1) == 0) return MP_OK;
    const auto t0 = std::chrono::steady_clock::now();
    RC_TRY(autotune(specs, precision, w, st, tu));
    const auto t1 = std::chrono::steady_clock::now();
    g_prof.acc.ms_autotune += std::chrono::duration<double, std::milli>(t1 - t0).count();
    g_tune.push_back(TuneEntry{dev, precision, shape, *tu});
    return MP_OK;
}

// ---------------------------------------------------------------------------
// single series: a batch of one job, tables written on the stream
// ---------------------------------------------------------------------------
int run_series(const double *T, int64_t n, int32_t m, int32_t kind, double p, int32_t excl,
               int32_t precision, int32_t R, double *P, int64_t *I, void *stream,
               int32_t fcmp = 0)
{
    Spec sp;
    RC_TRY(make_spec(T, n, m, kind, p, excl, R, P, I, &sp));
    RC_TRY(check_precision(precision));
    sp.fcmp = fcmp;
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    hipStream_t st = (hipStream_t)stream;
    Workspace *w = nullptr;
    int dev = 0;
    RC_TRY(get_ws(st, &w, &dev));

    // R = 0: the refresh interval (and, in FP32, the band width) is tuned per
    // series shape on first use
    Tuning tu;
    if (sp.R == 0) {
        mp_job shape_job;
        std::memset(&shape_job, 0, sizeof(shape_job));
        shape_job.n = sp.n;
        shape_job.m = sp.m;
        shape_job.kind = sp.kind;
        shape_job.excl = sp.excl;
        shape_job.p = sp.p;
        RC_TRY(tuning_for({sp}, &shape_job, 1, precision, *w, dev, st, &tu));
    }
    Layout L;
    RC_TRY(make_layout({sp}, precision, tu, *w, &L));
    RC_TRY(ensure_arrays(*w, L.stream_total, L.key_total));
    RC_TRY(ensure_band1(*w, L.band_entries));
    bind(L, *w);
    Tables t;
    t.jobs = w->job1;
    t.row_base = w->row_base1;
    t.band = w->band1;
    t.flags = w->flag1;
    t.pivots = w->pivots1;
    const Batch b = make_batch(L, *w, t);

    EvSet es;
    bool prof = false;
    RC_TRY(prof_begin(st, &es, &prof));
    RowBase4 rb;
    std::memset(&rb, 0, sizeof(rb));
    rb.count = (int32_t)L.row_base.size();
    for (int32_t k = 0; k < rb.count && k < 4; ++k) rb.v[k] = L.row_base[k];
    HIP_TRY(launch_store_job(L.jobs[0], rb, w->job1, w->row_base1, st), "job table");
    RC_TRY(enqueue(b, L, st, prof ? &es : nullptr));
    if (prof) RC_TRY(finish_profile(es, b, L, st));
    g_last_code = MP_OK;
    return MP_OK;
}

// ---------------------------------------------------------------------------
// partial (anytime) sweeps: one series, the listed diagonal groups only
// ---------------------------------------------------------------------------
int run_anytime(int32_t kind, const double *T, int64_t n, int32_t m, double p, int32_t excl,
                const int32_t *groups, int64_t ngroups, int32_t resume, double *P, int64_t *I,
                void *stream)
{
    Spec sp;
    RC_TRY(make_spec(T, n, m, kind, p, excl, 0, P, I, &sp));
    if (ngroups < 0 || ngroups > INT32_MAX) return fail(MP_EINVAL, "ngroups out of range");
    if (ngroups > 0 && !groups) return fail(MP_EINVAL, "null pointer argument");
    if (resume != 0 && resume != 1) return fail(MP_EINVAL, "resume must be 0 or 1");
    const uint32_t sel = sel_of(sp.kind, sp.pclass);
    if (!(sel & SEL_BAND) && !(sel == SEL_PGEN && sp.p <= PGEN_BAND_MAX))
        return fail(MP_EINVAL, "partial sweeps need a distance with a band kernel (p <= 6)");
    const int64_t N = sp.n - sp.m + 1;
    const int64_t G = any_groups(N, sp.excl);
    std::vector<uint8_t> marks((size_t)std::max<int64_t>(G, 1), 0);
    for (int64_t t = 0; t < ngroups; ++t) {
        if (groups[t] < 0 || groups[t] >= G) return fail(MP_EINVAL, "group index out of range");
        marks[(size_t)groups[t]] = 1;
    }
    sp.groups = groups;
    sp.ngroups = ngroups;

    std::lock_guard<std::recursive_mutex> lk(g_mu);
    hipStream_t st = (hipStream_t)stream;
    Workspace *w = nullptr;
    int dev = 0;
    RC_TRY(get_ws(st, &w, &dev));
    Layout L;
    RC_TRY(make_layout({sp}, MP_FP64, Tuning(), *w, &L));
    RC_TRY(ensure_arrays(*w, L.stream_total, L.key_total));
    RC_TRY(ensure_band1(*w, L.band_entries));
    RC_TRY(ensure_any(*w, std::max<int64_t>(ngroups, G), N));
    bind(L, *w);
    Job &J = L.jobs[0];
    J.band_map = w->any_map;
    J.group_ok = w->any_ok;
    if (resume) {          // the call's own profile first, merged at the end
        J.P = w->any_P;
        J.I = w->any_I;
    }
    // pageable host sources: the copies have read them when they return
    if (ngroups > 0)
        HIP_TRY(hipMemcpyAsync(w->any_map, groups, (size_t)ngroups * sizeof(int32_t),
                               hipMemcpyHostToDevice, st),
                "hipMemcpyAsync");
    if (G > 0)
        HIP_TRY(hipMemcpyAsync(w->any_ok, marks.data(), (size_t)G, hipMemcpyHostToDevice, st),
                "hipMemcpyAsync");
    Tables t;
    t.jobs = w->job1;
    t.row_base = w->row_base1;
    t.band = w->band1;
    t.flags = w->flag1;
    t.pivots = w->pivots1;
    const Batch b = make_batch(L, *w, t);

    EvSet es;
    bool prof = false;
    RC_TRY(prof_begin(st, &es, &prof));
    RowBase4 rb;
    std::memset(&rb, 0, sizeof(rb));
    rb.count = (int32_t)L.row_base.size();
    for (int32_t k = 0; k < rb.count && k < 4; ++k) rb.v[k] = L.row_base[k];
    HIP_TRY(launch_store_job(J, rb, w->job1, w->row_base1, st), "job table");
    RC_TRY(enqueue(b, L, st, prof ? &es : nullptr));
    if (resume) HIP_TRY(launch_any_merge(w->any_P, w->any_I, P, I, N, st), "merge launch");
    if (prof) RC_TRY(finish_profile(es, b, L, st));
    g_last_code = MP_OK;
    return MP_OK;
}

// splitmix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014): a Weyl sequence with step 0x9e3779b97f4a7c15
// through a 64-bit mixing function.
uint64_t splitmix64(uint64_t &state)
{
    uint64_t z = (state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

int run_batch(const double *T_cat, const mp_job *jobs, int32_t njobs, int32_t precision,
              double *P_cat, int64_t *I_cat, void *stream)
{
    if (!T_cat || !P_cat || !I_cat || (!jobs && njobs > 0))
        return fail(MP_EINVAL, "null pointer argument");
    if (njobs < 0 || njobs > 65535) return fail(MP_EINVAL, "njobs must be in [0, 65535]");
    RC_TRY(check_precision(precision));
    std::vector<Spec> specs((size_t)njobs);
    std::vector<std::pair<int64_t, int64_t>> outs((size_t)njobs);
    for (int32_t b = 0; b < njobs; ++b) {
        const mp_job &jb = jobs[b];
        if (jb.t_off < 0 || jb.out_off < 0) return fail(MP_EINVAL, "negative job offset");
        RC_TRY(make_spec(T_cat + jb.t_off, jb.n, jb.m, jb.kind, jb.p, jb.excl, jb.R,
                         P_cat + jb.out_off, I_cat + jb.out_off, &specs[b]));
        outs[b] = {jb.out_off, jb.out_off + (jb.n - jb.m + 1)};
    }
    std::sort(outs.begin(), outs.end());
    for (size_t b = 1; b < outs.size(); ++b)
        if (outs[b].first < outs[b - 1].second)
            return fail(MP_EINVAL, "output ranges of two jobs overlap");
    if (njobs == 0) {
        g_last_code = MP_OK;
        return MP_OK;
    }

    std::lock_guard<std::recursive_mutex> lk(g_mu);
    hipStream_t st = (hipStream_t)stream;
    Workspace *w = nullptr;
    int dev = 0;
    RC_TRY(get_ws(st, &w, &dev));
    RC_TRY(ensure_lib_stream(*w));
    const bool use_graph =
        !g_prof.on && env_int("MP_GRAPH", 1) != 0 && env_int("MP_COUNT_PAIRS", 0) != 1;

    // cached entry for this exact call?
    auto it = g_graphs.begin();
    for (; it != g_graphs.end(); ++it)
        if (it->dev == dev && it->precision == precision && it->T == T_cat && it->P == P_cat &&
            it->I == I_cat && same_table(it->table, jobs, njobs))
            break;
    if (it != g_graphs.end() && (it->ws != w || it->generation != w->generation)) {
        free_entry(*it);
        g_graphs.erase(it);
        it = g_graphs.end();
    }
    if (it == g_graphs.end()) {
        Tuning tu;
        RC_TRY(tuning_for(specs, jobs, njobs, precision, *w, dev, st, &tu));
        GraphEntry e;
        e.dev = dev;
        e.precision = precision;
        e.table.assign(jobs, jobs + njobs);
        e.T = T_cat;
        e.P = P_cat;
        e.I = I_cat;
        RC_TRY(make_layout(specs, precision, tu, *w, &e.L));
        RC_TRY(ensure_arrays(*w, e.L.stream_total, e.L.key_total));
        bind(e.L, *w);
        int rc = upload_tables(e.L, &e.t);
        if (rc) {
            free_entry(e);
            return rc;
        }
        e.generation = w->generation;
        e.ws = w;
        g_graphs.push_front(std::move(e));
        it = g_graphs.begin();
        while (g_graphs.size() > GRAPH_CACHE) {
            free_entry(g_graphs.back());
            g_graphs.pop_back();
        }
    } else if (it != g_graphs.begin()) {
        g_graphs.splice(g_graphs.begin(), g_graphs, it);
        it = g_graphs.begin();
    }
    GraphEntry &e = *it;
    const Batch b = make_batch(e.L, *w, e.t);

    if (!use_graph) {
        EvSet es;
        bool on = false;
        RC_TRY(prof_begin(st, &es, &on));
        RC_TRY(enqueue(b, e.L, st, on ? &es : nullptr));
        if (on) RC_TRY(finish_profile(es, b, e.L, st));
        g_last_code = MP_OK;
        return MP_OK;
    }
    hipStream_t ls = w->lib_stream;
    if (!e.exec) {
        HIP_TRY(hipStreamBeginCapture(ls, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        int rc = enqueue(b, e.L, ls, nullptr);
        hipGraph_t g = nullptr;
        hipError_t ec = hipStreamEndCapture(ls, &g);
        if (rc) {
            if (g) hipGraphDestroy(g);
            return rc;
        }
        if (ec != hipSuccess) return fail_hip(ec, "hipStreamEndCapture");
        e.graph = g;
        HIP_TRY(hipGraphInstantiate(&e.exec, e.graph, nullptr, nullptr, 0), "hipGraphInstantiate");
    } else {
        g_prof.acc.graph_replays += 1;
    }
    HIP_TRY(hipEventRecord(w->ev_fork, st), "hipEventRecord");
    HIP_TRY(hipStreamWaitEvent(ls, w->ev_fork, 0), "hipStreamWaitEvent");
    HIP_TRY(hipGraphLaunch(e.exec, ls), "hipGraphLaunch");
    HIP_TRY(hipEventRecord(w->ev_join, ls), "hipEventRecord");
    HIP_TRY(hipStreamWaitEvent(st, w->ev_join, 0), "hipStreamWaitEvent");
    g_last_code = MP_OK;
    return MP_OK;
}

// ---------------------------------------------------------------------------
// single series without device allocation (mp_profile_noalloc): every array
// of the pipeline is a slice of one static device array
// ---------------------------------------------------------------------------
// Largest window count of mp_profile_noalloc and the size of its array. Per
// window the pipeline needs three FP64 and three FP32 stream entries (plus
// STREAM_PAD per series), the window statistics, the key, the exact-search
// queue entry and FB_PIVOTS pivot distances: 149 bytes, 39.2 MB at the limit.
constexpr int64_t NOALLOC_MAX_N = MP_NOALLOC_MAX_N;
constexpr size_t NOALLOC_BYTES = (size_t)56 << 20;
constexpr size_t NOALLOC_ALIGN = 256;

// Sub-allocator over the array: slices of at least NOALLOC_ALIGN bytes, in
// call order. With base == 0 it only adds up the bytes a layout needs.
struct Carver {
    uintptr_t base = 0;
    size_t used = 0;
    template <class T>
    T *take(int64_t count)
    {
        const size_t bytes = ((size_t)std::max<int64_t>(count, 1) * sizeof(T) + NOALLOC_ALIGN - 1) &
                             ~(NOALLOC_ALIGN - 1);
        T *p = base ? (T *)(base + used) : nullptr;
        used += bytes;
        return p;
    }
};

// The workspace and tables of a one-job layout as slices of the array.
void carve(Carver &c, const Layout &L, Workspace *w, Tables *t)
{
    const int64_t S = L.stream_total, K = L.key_total;
    w->x = c.take<double>(S);
    w->y = c.take<double>(S);
    w->z = c.take<double>(S);
    w->xf = c.take<float>(S);
    w->yf = c.take<float>(S);
    w->zf = c.take<float>(S);
    w->mu = c.take<double>(K);
    w->invn = c.take<double>(K);
    w->wsum = c.take<double>(4 * K);
    w->lcount = c.take<int32_t>(K);
    w->lhead = c.take<int32_t>(K);
    w->lanchor = c.take<double>(2 * K);
    w->isconst = c.take<uint8_t>(K);
    w->keys = c.take<unsigned long long>(K);
    w->fb_rows = c.take<int32_t>(K);
    w->fb_job = c.take<int32_t>(K);
    w->fb_keys = c.take<unsigned long long>(K);
    w->fb_ub = c.take<double>(K);
    w->fb_pd = c.take<float>(K * FB_PIVOTS);
    w->counters = c.take<int32_t>(64);
    w->visits = c.take<unsigned long long>(1);
    w->stream_cap = S;
    w->key_cap = K;
    t->jobs = c.take<Job>(1);
    t->row_base = c.take<int64_t>(4);
    t->band = c.take<int64_t>(L.band_entries);
    t->flags = c.take<int32_t>(1);
    t->pivots = c.take<int32_t>(FB_PIVOTS);
}

// Bytes carve() takes at the window limit: the largest layout is one job of
// NOALLOC_MAX_N windows swept in bands of 512 diagonals (at most
// NOALLOC_MAX_N / 512 + 1 bands, one more band-table entry).
constexpr size_t noalloc_bytes_at_limit()
{
    constexpr size_t A = NOALLOC_ALIGN;
    constexpr size_t S = (size_t)(NOALLOC_MAX_N + STREAM_PAD), K = (size_t)NOALLOC_MAX_N;
    constexpr size_t per_array = A;   // rounding slack of each slice
    return 3 * (8 * S) + 3 * (4 * S) +
           K * (8 + 8 + 32 + 4 + 4 + 16 + 1 + 8 + 4 + 4 + 8 + 8 + 4 * FB_PIVOTS) + 64 * 4 + 8 +
           sizeof(Job) + 4 * 8 + (K / 512 + 2) * 8 + 4 + FB_PIVOTS * 4 + 29 * per_array;
}
static_assert(noalloc_bytes_at_limit() <= NOALLOC_BYTES,
              "the static array holds a series of MP_NOALLOC_MAX_N windows");

}  // namespace

static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {

// Per device: the device address of `scratch` (the array's name is a host
// stand-in, not a device address), looked up on the first call on the device
// with it current, and the architecture facts of the planner.
constexpr int NOALLOC_DEVICES = 64;
struct NoallocDevice {
    void *ptr;
    int ready;   // 0: not looked up, 1: gfx950 and ptr valid, -1: not a gfx950 GPU
    int cus;
};
NoallocDevice g_noalloc[NOALLOC_DEVICES];

int noalloc_device(NoallocDevice **out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= NOALLOC_DEVICES)
        return fail(MP_EUNSUPPORTED, "device ordinal beyond the allocation-free entry's table");
    NoallocDevice &d = g_noalloc[dev];
    if (d.ready == 0) {
        hipDeviceProp_t prop;
        HIP_TRY(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
            d.ready = -1;
        } else {
            void *p = nullptr;
            HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
            if (!p) return fail(MP_EHIP, "hipGetSymbolAddress(scratch) returned no address");
            d.ptr = p;
            d.cus = prop.multiProcessorCount;
            d.ready = 1;
        }
    }
    if (d.ready < 0) return fail(MP_EUNSUPPORTED, "the current HIP device is not a gfx950 GPU");
    *out = &d;
    return MP_OK;
}

int run_noalloc(int32_t kind, const double *T, int64_t n, int32_t m, double p, int32_t excl,
                int32_t precision, int32_t R, double *P, int64_t *I, void *stream)
{
    Spec sp;
    RC_TRY(make_spec(T, n, m, kind, p, excl, R, P, I, &sp));
    RC_TRY(check_precision(precision));
    if (n - m + 1 > NOALLOC_MAX_N)
        return fail(MP_EINVAL, "n - m + 1 exceeds MP_NOALLOC_MAX_N windows");
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    NoallocDevice *d = nullptr;
    RC_TRY(noalloc_device(&d));
    hipStream_t st = (hipStream_t)stream;

    // no trial runs: R = 0 takes the per-distance default interval
    Workspace w;
    w.cus = d->cus;
    w.arch_ok = 1;
    Layout L;
    RC_TRY(make_layout({sp}, precision, Tuning(), w, &L));
    Tables t;
    Carver size_only;
    carve(size_only, L, &w, &t);
    if (size_only.used > NOALLOC_BYTES)
        return fail(MP_EINVAL, "the series needs more than the allocation-free array holds");
    Carver c;
    c.base = (uintptr_t)d->ptr;
    carve(c, L, &w, &t);
    bind(L, w);
    const Batch b = make_batch(L, w, t);
    RowBase4 rb;
    std::memset(&rb, 0, sizeof(rb));
    rb.count = (int32_t)L.row_base.size();
    for (int32_t k = 0; k < rb.count && k < 4; ++k) rb.v[k] = L.row_base[k];
    HIP_TRY(launch_store_job(L.jobs[0], rb, t.jobs, t.row_base, st), "job table");
    RC_TRY(enqueue(b, L, st, nullptr));
    g_last_code = MP_OK;
    return MP_OK;
}

}  // namespace

// Hooks for the other host files of the library (incremental profiles).
namespace mpk {
int report_error(int code, const char *what) { return fail(code, what); }
int report_hip(hipError_t e, const char *where) { return fail_hip(e, where); }
void report_ok() { g_last_code = MP_OK; }
int profile_once(const double *T, int64_t n, int32_t m, int32_t kind, double p, int32_t excl,
                 int32_t R, double *P, int64_t *I, hipStream_t st)
{
    return run_series(T, n, m, kind, p, excl, MP_FP64, R, P, I, (void *)st);
}
}  // namespace mpk

extern "C" {

int mp_aamp(const double *T, int64_t n, int32_t m, int32_t excl, int32_t precision, int32_t R,
            double *P, int64_t *I, void *stream)
{
    return run_series(T, n, m, AAMP, 2.0, excl, precision, R, P, I, stream);
}

int mp_pnorm(const double *T, int64_t n, int32_t m, double p, int32_t excl, int32_t precision,
             int32_t R, double *P, int64_t *I, void *stream)
{
    return run_series(T, n, m, PNORM, p, excl, precision, R, P, I, stream);
}

int mp_acamp(const double *T, int64_t n, int32_t m, int32_t excl, int32_t precision, int32_t R,
             double *P, int64_t *I, void *stream)
{
    return run_series(T, n, m, ACAMP, 2.0, excl, precision, R, P, I, stream);
}

int mp_acamp_fcmp(const double *T, int64_t n, int32_t m, int32_t excl, int32_t R, double *P,
                  int64_t *I, void *stream)
{
    return run_series(T, n, m, ACAMP, 2.0, excl, MP_FP64, R, P, I, stream, 1);
}

int mp_profile_noalloc(int32_t kind, const double *T, int64_t n, int32_t m, double p,
                       int32_t excl, int32_t precision, int32_t R, double *P, int64_t *I,
                       void *stream)
{
    return run_noalloc(kind, T, n, m, p, excl, precision, R, P, I, stream);
}

int mp_anytime(int32_t kind, const double *T, int64_t n, int32_t m, double p, int32_t excl,
               const int32_t *groups, int64_t ngroups, int32_t resume, double *P, int64_t *I,
               void *stream)
{
    return run_anytime(kind, T, n, m, p, excl, groups, ngroups, resume, P, I, stream);
}

int mp_anytime_groups(int64_t n, int32_t m, int32_t excl, int64_t *ngroups)
{
    if (!ngroups) return fail(MP_EINVAL, "null pointer argument");
    if (n < 1 || n >= MP_MAX_N) return fail(MP_EINVAL, "n must satisfy 1 <= n < 2^31");
    if (m < 1 || (int64_t)m > n) return fail(MP_EINVAL, "m must satisfy 1 <= m <= n");
    const int64_t e = excl > 0 ? excl : (m + 3) / 4;
    *ngroups = any_groups(n - m + 1, e);
    g_last_code = MP_OK;
    return MP_OK;
}

int mp_anytime_order(int64_t n, int32_t m, int32_t excl, uint64_t seed, int32_t *order,
                     int64_t *cum_pairs)
{
    int64_t G = 0;
    RC_TRY(mp_anytime_groups(n, m, excl, &G));
    if (G > 0 && !order) return fail(MP_EINVAL, "null pointer argument");
    const int64_t N = n - m + 1, e = excl > 0 ? excl : (m + 3) / 4;
    // Fisher-Yates from the top; the draw for position k is the high word of
    // a 64 x 64-bit product, uniform over [0, k] up to a 2^-64 bias
    for (int64_t k = 0; k < G; ++k) order[k] = (int32_t)k;
    uint64_t state = seed;
    for (int64_t k = G - 1; k > 0; --k) {
        const uint64_t r = splitmix64(state);
        const int64_t u = (int64_t)(((unsigned __int128)r * (uint64_t)(k + 1)) >> 64);
        std::swap(order[k], order[u]);
    }
    if (cum_pairs) {
        int64_t run = 0;
        for (int64_t k = 0; k < G; ++k) cum_pairs[k] = (run += group_pairs(N, e, order[k]));
    }
    g_last_code = MP_OK;
    return MP_OK;
}

int mp_batch(const double *T_cat, const mp_job *jobs, int32_t njobs, int32_t precision,
             double *P_cat, int64_t *I_cat, void *stream)
{
    return run_batch(T_cat, jobs, njobs, precision, P_cat, I_cat, stream);
}

int mp_topk(const double *P, const int64_t *I, int64_t N, int32_t k, int32_t excl, int32_t mode,
            int64_t *out_i, int64_t *out_j, double *out_d, int32_t *out_count, void *stream)
{
    if (!P || !I || !out_i || !out_j || !out_d || !out_count)
        return fail(MP_EINVAL, "null pointer argument");
    if (N < 0 || N >= MP_MAX_N) return fail(MP_EINVAL, "N must be in [0, 2^31)");
    if (k < 0 || k > 65536) return fail(MP_EINVAL, "k must be in [0, 65536]");
    if (excl < 1) return fail(MP_EINVAL, "excl must be >= 1");
    if (mode != MP_MOTIFS && mode != MP_DISCORDS)
        return fail(MP_EINVAL, "mode must be MP_MOTIFS or MP_DISCORDS");
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    Workspace *w = nullptr;
    int dev = 0;
    RC_TRY(get_ws((hipStream_t)stream, &w, &dev));
    if (w->topk_mask_cap < std::max<int64_t>(N, 1)) {
        RC_TRY(grow(&w->topk_mask, (size_t)std::max<int64_t>(N, 1), "top-k mask"));
        w->topk_mask_cap = std::max<int64_t>(N, 1);
    }
    const int64_t sc = 3 * (int64_t)std::max(k, 1);
    if (w->topk_scratch_cap < sc) {
        RC_TRY(grow(&w->topk_scratch, (size_t)sc, "top-k scratch"));
        w->topk_scratch_cap = sc;
    }
    HIP_TRY(launch_topk(P, I, N, k, excl, mode, out_i, out_j, out_d, out_count, w->topk_scratch,
                        w->topk_mask, (hipStream_t)stream),
            "top-k launch");
    g_last_code = MP_OK;
    return MP_OK;
}

const char *mp_strerror(int code)
{
    static thread_local std::string msg;
    const char *base;
    switch (code) {
    case MP_OK: base = "success"; break;
    case MP_EINVAL: base = "invalid argument"; break;
    case MP_ENOMEM: base = "device allocation failed"; break;
    case MP_EHIP: base = "HIP runtime error"; break;
    case MP_EUNSUPPORTED: base = "unsupported device"; break;
    default: base = "unknown error code"; break;
    }
    msg = base;
    if (code != MP_OK && code == g_last_code && !g_err.empty()) msg += ": " + g_err;
    return msg.c_str();
}

void mp_release(void)
{
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (size_t d = 0; d < g_dev.size(); ++d) {
        (void)hipSetDevice((int)d);
        (void)hipDeviceSynchronize();
        for (auto it = g_graphs.begin(); it != g_graphs.end();) {
            if (it->dev == (int)d) {
                free_entry(*it);
                it = g_graphs.erase(it);
            } else {
                ++it;
            }
        }
        for (auto it = g_ws.begin(); it != g_ws.end();) {
            if (it->dev == (int)d) {
                free_ws(*it);
                it = g_ws.erase(it);
            } else {
                ++it;
            }
        }
    }
    (void)hipSetDevice(cur);
}

void mp_set_profiling(int on)
{
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    for (auto &es : g_prof.pending) {
        for (int k = 0; k < 4; ++k) (void)hipEventDestroy(es.ev[k]);
        (void)hipHostFree(es.fb_host);
        (void)hipHostFree(es.visits_host);
    }
    g_prof.pending.clear();
    g_prof.acc = mp_stats{};
    g_prof.on = on != 0;
}

int mp_profile_read(mp_stats *out)
{
    if (!out) return fail(MP_EINVAL, "null pointer argument");
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    for (auto &es : g_prof.pending) {
        float a = 0.f, b = 0.f, c = 0.f;
        HIP_TRY(hipEventSynchronize(es.ev[3]), "hipEventSynchronize");
        HIP_TRY(hipEventElapsedTime(&a, es.ev[0], es.ev[1]), "hipEventElapsedTime");
        HIP_TRY(hipEventElapsedTime(&b, es.ev[1], es.ev[2]), "hipEventElapsedTime");
        HIP_TRY(hipEventElapsedTime(&c, es.ev[2], es.ev[3]), "hipEventElapsedTime");
        g_prof.acc.ms_prep += a;
        g_prof.acc.ms_sweep += b;
        g_prof.acc.ms_finalize += c;
        g_prof.acc.fallback_rows += *es.fb_host;
        g_prof.acc.pairs_visited += (int64_t)*es.visits_host;
        for (int k = 0; k < 4; ++k) (void)hipEventDestroy(es.ev[k]);
        (void)hipHostFree(es.fb_host);
        (void)hipHostFree(es.visits_host);
    }
    g_prof.pending.clear();
    *out = g_prof.acc;
    return MP_OK;
}

}  // extern "C"
