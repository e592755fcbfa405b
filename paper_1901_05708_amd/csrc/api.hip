// api.hip -- host side of libmp: argument validation, per-device workspace,
// the planner that picks the sweep kernel and its shape, and the C ABI of
// include/mp.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
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

// ---------------------------------------------------------------------------
// per-device workspace (grow-only)
// ---------------------------------------------------------------------------
struct Workspace {
    int64_t cap = 0;           // stream entries (N + STREAM_PAD) the buffers hold
    double *x = nullptr, *y = nullptr, *z = nullptr;
    float *xf = nullptr, *yf = nullptr, *zf = nullptr;
    double *mu = nullptr, *invn = nullptr;
    uint8_t *isconst = nullptr;
    unsigned long long *keys = nullptr;
    unsigned long long *fb_keys = nullptr;
    double *fb_ub = nullptr;
    float *fb_pd = nullptr;            // FB_PIVOTS x cap pivot distances
    int32_t *fb_pivots = nullptr;
    int32_t *fb_rows = nullptr;
    int32_t *counters = nullptr;       // [0] fallback count, [1..] spare
    int64_t band_cap = 0;
    int64_t *band_start = nullptr;
    unsigned int *next_item = nullptr;
    int arch_ok = -1;                  // -1 unknown, 0 no, 1 gfx950
};

std::mutex g_mu;
std::vector<Workspace> g_ws;

void free_ws(Workspace &w)
{
    hipFree(w.x);
    hipFree(w.y);
    hipFree(w.z);
    hipFree(w.xf);
    hipFree(w.yf);
    hipFree(w.zf);
    hipFree(w.mu);
    hipFree(w.invn);
    hipFree(w.isconst);
    hipFree(w.keys);
    hipFree(w.fb_keys);
    hipFree(w.fb_ub);
    hipFree(w.fb_pd);
    hipFree(w.fb_pivots);
    hipFree(w.fb_rows);
    hipFree(w.counters);
    hipFree(w.band_start);
    hipFree(w.next_item);
    int arch = w.arch_ok;
    w = Workspace();
    w.arch_ok = arch;
}

int get_ws(Workspace **out, int *dev_out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_mu);
    if ((int)g_ws.size() <= dev) g_ws.resize(dev + 1);
    Workspace &w = g_ws[dev];
    if (w.arch_ok < 0) {
        hipDeviceProp_t prop;
        HIP_TRY(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
        w.arch_ok = (std::strncmp(prop.gcnArchName, "gfx950", 6) == 0) ? 1 : 0;
    }
    if (!w.arch_ok) return fail(MP_EUNSUPPORTED, "the current HIP device is not a gfx950 GPU");
    *out = &w;
    *dev_out = dev;
    return MP_OK;
}

template <class T>
int grow(T **p, size_t count, const char *what)
{
    hipFree(*p);
    *p = nullptr;
    hipError_t e = hipMalloc((void **)p, std::max<size_t>(count, 1) * sizeof(T));
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
        (void)hipGetLastError();
        return fail(MP_ENOMEM, what);
    }
    if (e != hipSuccess) return fail_hip(e, what);
    return MP_OK;
}

int ensure_ws(Workspace &w, int64_t N)
{
    const int64_t need = N + STREAM_PAD;
    if (w.cap >= need) return MP_OK;
    int64_t cap = std::max<int64_t>(need, w.cap + w.cap / 2);
    free_ws(w);
    int rc;
    if ((rc = grow(&w.x, cap, "workspace x")) || (rc = grow(&w.y, cap, "workspace y")) ||
        (rc = grow(&w.z, cap, "workspace z")) || (rc = grow(&w.xf, cap, "workspace xf")) ||
        (rc = grow(&w.yf, cap, "workspace yf")) || (rc = grow(&w.zf, cap, "workspace zf")) ||
        (rc = grow(&w.mu, cap, "workspace mu")) ||
        (rc = grow(&w.invn, cap, "workspace invn")) ||
        (rc = grow(&w.isconst, cap, "workspace const")) ||
        (rc = grow(&w.keys, cap, "workspace keys")) ||
        (rc = grow(&w.fb_keys, cap, "workspace fallback keys")) ||
        (rc = grow(&w.fb_ub, cap, "workspace fallback bounds")) ||
        (rc = grow(&w.fb_pd, (size_t)cap * FB_PIVOTS, "workspace pivot distances")) ||
        (rc = grow(&w.fb_pivots, 64, "workspace pivots")) ||
        (rc = grow(&w.fb_rows, cap, "workspace fallback")) ||
        (rc = grow(&w.counters, 64, "workspace counters")) ||
        (rc = grow(&w.next_item, 64, "workspace counter"))) {
        free_ws(w);
        return rc;
    }
    w.cap = cap;
    return MP_OK;
}

int ensure_bands(Workspace &w, int64_t nbands)
{
    if (w.band_cap >= nbands + 1) return MP_OK;
    int64_t cap = std::max<int64_t>(nbands + 1, 4096);
    int rc = grow(&w.band_start, cap, "workspace bands");
    if (rc) {
        w.band_cap = 0;
        return rc;
    }
    w.band_cap = cap;
    return MP_OK;
}

// ---------------------------------------------------------------------------
// profiling
// ---------------------------------------------------------------------------
struct EvSet {
    hipEvent_t ev[4];
    int32_t *fb_host = nullptr;   // pinned copy of the call's fallback count
};

struct Prof {
    bool on = false;
    std::vector<EvSet> pending;
    mp_stats acc{};
};
std::mutex g_prof_mu;
Prof g_prof;

int prof_begin(hipStream_t st, EvSet *es, bool *active)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    *active = g_prof.on;
    if (!*active) return MP_OK;
    for (int k = 0; k < 4; ++k) HIP_TRY(hipEventCreate(&es->ev[k]), "hipEventCreate");
    HIP_TRY(hipHostMalloc((void **)&es->fb_host, sizeof(int32_t), hipHostMallocDefault),
            "hipHostMalloc");
    *es->fb_host = 0;
    HIP_TRY(hipEventRecord(es->ev[0], st), "hipEventRecord");
    return MP_OK;
}

void prof_end(const EvSet &es, const mp_stats &cfg)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof.pending.push_back(es);
    g_prof.acc.calls += 1;
    g_prof.acc.sweep_launches += cfg.sweep_launches;
    g_prof.acc.pairs += cfg.pairs;
    g_prof.acc.refresh_rows = cfg.refresh_rows;
    g_prof.acc.diags_per_lane = cfg.diags_per_lane;
    g_prof.acc.items = cfg.items;
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

int validate(const double *T, int64_t n, int32_t m, int32_t precision, int32_t R,
             const double *P, const int64_t *I)
{
    if (!T || !P || !I) return fail(MP_EINVAL, "null pointer argument");
    if (n < 1) return fail(MP_EINVAL, "n must be >= 1");
    if (n >= MP_MAX_N) return fail(MP_EINVAL, "n must be < 2^31");
    if (m < 1 || (int64_t)m > n) return fail(MP_EINVAL, "m must satisfy 1 <= m <= n");
    if (precision != MP_FP64 && precision != MP_FP32_REFRESH)
        return fail(MP_EINVAL, "precision must be MP_FP64 or MP_FP32_REFRESH");
    if (R < 0) return fail(MP_EINVAL, "R must be >= 0");
    return MP_OK;
}

int32_t pclass_of(double p)
{
    if (p == 1.0) return P_ONE;
    if (p == 2.0) return P_TWO;
    if (p == 3.0) return P_THREE;
    return P_GENERIC;
}

const char *sweep_choice()
{
    const char *e = std::getenv("MP_SWEEP");
    return e ? e : "auto";
}

struct Plan {
    bool band = false;
    int32_t R = 0;
    int32_t diags_per_lane = 0;
    int32_t grid = 0;
    int64_t nbands = 0;
    int64_t items = 0;
};

struct DevInfo {
    int cus = 0;
};
std::vector<DevInfo> g_dev;

int device_cus(int dev)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if ((int)g_dev.size() <= dev) g_dev.resize(dev + 1);
    if (g_dev[dev].cus == 0) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return 256;
        g_dev[dev].cus = prop.multiProcessorCount;
    }
    return g_dev[dev].cus;
}

// Rows summed over all bands (band b: N - excl - b W rows) and the band count.
int64_t band_rows_total(int64_t N, int64_t excl, int64_t W, int64_t *nbands)
{
    const int64_t nd = N - excl;
    const int64_t nb = (nd + W - 1) / W;
    *nbands = nb;
    // sum_{b < nb} (nd - b W)
    return nb * nd - W * (nb * (nb - 1) / 2);
}

// Kernel and shape. The band kernel needs at least half a band of diagonals.
// Its persistent grid gives every wave an equal share of the band-major row
// space; R bounds the rows between exact FP64 restarts (each restart costs 2m
// operations per diagonal, and longer runs let round-off drift further).
int make_plan(const Series &s, int32_t R_user, int dev, Plan *pl)
{
    const int64_t ndiag = s.N - s.excl;
    Plan p;
    std::string choice = sweep_choice();
    int32_t kd = 8;
    if (const char *e = std::getenv("MP_KD")) kd = (std::atoi(e) == 16) ? 16 : 8;
    const int64_t W = 64 * kd;
    p.band = band_supported(s) && ndiag >= W / 2 && choice != "simple";
    if (choice == "band" && band_supported(s) && ndiag > 0) p.band = true;
    if (ndiag <= 0) p.band = false;
    if (p.band) {
        p.diags_per_lane = kd;
        const int64_t slots = (int64_t)device_cus(dev) * band_blocks_per_cu(s, kd);
        const int64_t rows = band_rows_total(s.N, s.excl, W, &p.nbands);
        // default refresh interval: 4096 rows in FP64; 1024 in FP32, where
        // drift grows 2^29 times faster per step
        int64_t R = R_user > 0 ? R_user : (s.fp32 ? 1024 : 4096);
        p.R = (int32_t)std::min<int64_t>(R, INT32_MAX / 2);
        // at least 64 rows per wave
        p.grid = (int32_t)std::max<int64_t>(1, std::min<int64_t>(slots, rows / 64));
        const int64_t share = (rows + p.grid - 1) / p.grid;
        p.items = (int64_t)p.grid * ((share + p.R - 1) / p.R) + p.nbands;   // upper bound
    } else {
        // the simple kernel is FP64 only; a single-precision request on a
        // series too small for the band kernel is served exactly in FP64
        int32_t R = R_user > 0 ? R_user : 1024;
        // the simple kernel's grid has one row of blocks per segment
        int64_t minR = (ndiag + 65534) / 65535;
        if (R < minR) R = (int32_t)minR;
        p.R = R;
    }
    *pl = p;
    return MP_OK;
}

int run_series(const double *T, int64_t n, int32_t m, int32_t kind, double p, int32_t excl,
               int32_t precision, int32_t R, double *P, int64_t *I, void *stream)
{
    int rc = validate(T, n, m, precision, R, P, I);
    if (rc) return rc;
    if (kind == PNORM && !(std::isfinite(p) && p >= 1.0))
        return fail(MP_EINVAL, "p must be finite and >= 1");
    if (excl <= 0) excl = (m + 3) / 4;
    if (kind == PNORM && p == 2.0) kind = AAMP;  // Sec. 3.3: p = 2 is Euclid

    Workspace *w = nullptr;
    int dev = 0;
    if ((rc = get_ws(&w, &dev))) return rc;
    hipStream_t st = (hipStream_t)stream;
    const int64_t N = n - m + 1;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if ((rc = ensure_ws(*w, N))) return rc;
    }

    Series s;
    std::memset(&s, 0, sizeof(s));
    s.T = T;
    s.n = n;
    s.N = N;
    s.m = m;
    s.kind = kind;
    s.pclass = kind == PNORM ? pclass_of(p) : P_TWO;
    s.excl = excl;
    s.p = p;
    s.gb = index_bits(N);
    s.x = w->x;
    s.y = w->y;
    s.z = w->z;
    s.mu = w->mu;
    s.invn = w->invn;
    s.isconst = w->isconst;
    s.keys = w->keys;
    s.fb_count = w->counters;
    s.xf = w->xf;
    s.yf = w->yf;
    s.zf = w->zf;
    s.fp32 = (precision == MP_FP32_REFRESH) ? 1 : 0;
    // MP_FORCE_FALLBACK (tests): send every row through the exact search.
    if (const char *e = std::getenv("MP_FORCE_FALLBACK")) {
        const int v = std::atoi(e);
        s.force_fb = (v == 1 || v == 2) ? v : 0;
    }

    Fallback fb;
    fb.count = w->counters;
    fb.rows = w->fb_rows;
    fb.keys = w->fb_keys;
    fb.ub = w->fb_ub;
    fb.pivots = w->fb_pivots;
    fb.pd = w->fb_pd;
    fb.pd_stride = w->cap;
    fb.capacity = (int32_t)std::min<int64_t>(N, INT32_MAX);

    Plan pl;
    if ((rc = make_plan(s, R, dev, &pl))) return rc;
    if (!pl.band) s.fp32 = 0;
    BandPlan bp;
    std::memset(&bp, 0, sizeof(bp));
    if (pl.band) {
        {
            std::lock_guard<std::mutex> lk(g_mu);
            if ((rc = ensure_bands(*w, pl.nbands))) return rc;
        }
        bp.band_width = 64 * pl.diags_per_lane;
        bp.seg_rows = pl.R;
        bp.nbands = (int32_t)pl.nbands;
        bp.band_start = w->band_start;
    }

    EvSet es;
    bool prof = false;
    if ((rc = prof_begin(st, &es, &prof))) return rc;

    HIP_TRY(launch_prep(s, st), "prep launch");
    if (pl.band) HIP_TRY(launch_plan(s, bp, st), "plan launch");
    if (prof) HIP_TRY(hipEventRecord(es.ev[1], st), "hipEventRecord");
    if (pl.band) {
        HIP_TRY(launch_sweep_band(s, bp, pl.diags_per_lane, pl.grid, st), "sweep launch");
    } else {
        HIP_TRY(launch_sweep_simple(s, pl.R, st), "sweep launch");
    }
    if (prof) HIP_TRY(hipEventRecord(es.ev[2], st), "hipEventRecord");
    HIP_TRY(launch_finalize(s, fb, P, I, st), "finalize launch");
    HIP_TRY(launch_fallback(s, fb, P, I, st), "fallback launch");
    if (prof) {
        HIP_TRY(hipMemcpyAsync(es.fb_host, fb.count, sizeof(int32_t), hipMemcpyDeviceToHost, st),
                "hipMemcpyAsync");
        HIP_TRY(hipEventRecord(es.ev[3], st), "hipEventRecord");
        mp_stats cfg{};
        cfg.pairs = pair_count(N, excl);
        cfg.sweep_launches = 1;
        cfg.refresh_rows = pl.R;
        cfg.diags_per_lane = pl.band ? pl.diags_per_lane : 0;
        cfg.items = (int32_t)std::min<int64_t>(pl.items, INT32_MAX);
        prof_end(es, cfg);
    }
    g_last_code = MP_OK;
    return MP_OK;
}

}  // namespace

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

int mp_batch(const double *T_cat, const mp_job *jobs, int32_t njobs, int32_t precision,
             double *P_cat, int64_t *I_cat, void *stream)
{
    if (!T_cat || !jobs || !P_cat || !I_cat) return fail(MP_EINVAL, "null pointer argument");
    if (njobs < 0) return fail(MP_EINVAL, "njobs must be >= 0");
    for (int32_t b = 0; b < njobs; ++b) {
        const mp_job &jb = jobs[b];
        if (jb.t_off < 0 || jb.out_off < 0) return fail(MP_EINVAL, "negative job offset");
        if (jb.kind < MP_KIND_AAMP || jb.kind > MP_KIND_ACAMP)
            return fail(MP_EINVAL, "job kind must be MP_KIND_*");
    }
    for (int32_t b = 0; b < njobs; ++b) {
        const mp_job &jb = jobs[b];
        int rc = run_series(T_cat + jb.t_off, jb.n, jb.m, jb.kind, jb.p, jb.excl, precision, jb.R,
                            P_cat + jb.out_off, I_cat + jb.out_off, stream);
        if (rc) return rc;
    }
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
    std::lock_guard<std::mutex> lk(g_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (size_t d = 0; d < g_ws.size(); ++d) {
        if (g_ws[d].cap == 0 && g_ws[d].band_cap == 0) continue;
        (void)hipSetDevice((int)d);
        (void)hipDeviceSynchronize();
        free_ws(g_ws[d]);
    }
    (void)hipSetDevice(cur);
}

void mp_set_profiling(int on)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto &es : g_prof.pending) {
        for (int k = 0; k < 4; ++k) (void)hipEventDestroy(es.ev[k]);
        (void)hipHostFree(es.fb_host);
    }
    g_prof.pending.clear();
    g_prof.acc = mp_stats{};
    g_prof.on = on != 0;
}

int mp_profile_read(mp_stats *out)
{
    if (!out) return fail(MP_EINVAL, "null pointer argument");
    std::lock_guard<std::mutex> lk(g_prof_mu);
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
        for (int k = 0; k < 4; ++k) (void)hipEventDestroy(es.ev[k]);
        (void)hipHostFree(es.fb_host);
    }
    g_prof.pending.clear();
    *out = g_prof.acc;
    return MP_OK;
}

}  // extern "C"
