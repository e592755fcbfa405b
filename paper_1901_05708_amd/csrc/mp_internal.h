// mp_internal.h -- interface between the host side of libmp (api.hip) and its
// HIP kernels. Not installed; the public ABI is include/mp.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstdlib>

namespace mpk {

enum Kind : int32_t { AAMP = 0, PNORM = 1, ACAMP = 2 };

// p-norm specialisations: p = 2 runs the Euclidean kernels, p = 1 and p = 3
// have closed-form power terms, any other p goes through pow().
enum PClass : int32_t { P_GENERIC = 0, P_ONE = 1, P_TWO = 2, P_THREE = 3 };
// Template value of the band kernel only (never a job's pclass): its ACAMP
// pairs are keyed on the comparator F of Sec. 4.4 instead of 1 - rho.
constexpr int P_FCMP = 4;

// Extra stream entries past N so that sweeps may read a little beyond the last
// window (tail rows of a segment, the last diagonals of a band) without any
// bounds check; those entries hold sentinels that make every such pair lose.
constexpr int64_t STREAM_PAD = 2048 + 64;

// Sentinels for out-of-range stream entries (see prep): the squared or p-th
// power sums of any pair touching them exceed 1e190, far above any real sum
// while |t| < 1e30.
constexpr double SENT_EUCLID = -1e100;   // u = v = -1e100: each step adds ~1e200
constexpr double SENT_P1 = -1e200;       // |a_i - a_j| ~ 1e200
constexpr double SENT_P3 = -1e66;        // |a_i - a_j|^3 ~ 1e198
constexpr double SENT_INIT = 1e200;      // start value of a diagonal already past N
// generic p (1 < p <= 6): -(1e30 + 10^(198/p)), so |a_i - a_j|^p ~ 1e198
__host__ __device__ inline double sent_pgen(double p) { return -(1e30 + pow(10.0, 198.0 / p)); }
// float-stream sentinels (the sums of pairs touching them exceed 1e30 or are +inf)
constexpr float SENTF_EUCLID = -1e18f;
constexpr float SENTF_P1 = -1e30f;
constexpr float SENTF_P3 = -1e10f;

// Device views of one prepared series.
struct Series {
    const double *T;       // n samples
    int64_t n;
    int64_t N;             // n - m + 1 windows
    int32_t m;
    int32_t kind;          // Kind
    int32_t pclass;        // PClass (PNORM only)
    int32_t excl;
    double p;
    int32_t gb;            // index bits of a global key
    int32_t fcmp;          // ACAMP: the band sweep compares pairs on F (Sec. 4.4)
    // Difference streams, N + STREAM_PAD entries each.
    //   AAMP:  x = u_j = t[j+m-1] - t[j-1],  y = v_j = t[j+m-1] + t[j-1]
    //   PNORM: x = a_j = t[j+m-1],           y = b_j = t[j-1]
    //   ACAMP: x = df_j = (t[j+m-1] - t[j-1]) / 2,
    //          y = dg_j = (t[j+m-1] - mu_j) + (t[j-1] - mu_{j-1}),
    //          z = -invn_j (invn = 1 / ||window - mean||, 0 for constant windows)
    double *x;
    double *y;
    double *z;
    // Window statistics (ACAMP), N entries.
    double *mu;
    double *invn;
    uint8_t *isconst;
    // ACAMP with m >= LONG_WINDOW: 4 N entries, for window j the double-double
    // sums S = sum u, Q = sum u^2 (hi, lo, hi, lo) of its samples shifted by
    // c = t[256 floor(j / 256)], u = t - c (k_window_stats).
    double *wsum;
    // Rescoring of long windows (m >= LONG_WINDOW), per block of 256 rows
    // from i0: lcount[i0] its number of runs,
    // lhead[i0 + k] the row offset of run k's first row, lanchor[2 (i0 + k)]
    // that row's exact sum (double-double); N entries each (2 N for lanchor).
    int32_t *lcount;
    int32_t *lhead;
    double *lanchor;
    // Packed (value, index) keys, N entries; ~0 = no candidate.
    unsigned long long *keys;
    // FP32 copies of the streams (MP_FP32_REFRESH), recentred before rounding:
    //   AAMP:  xf = u_j, yf = v_j - 2c;  PNORM: xf = a_j - c, yf = b_j - c;
    //   ACAMP: xf = df_j, yf = dg_j, zf = -invn_j; c = t_0.
    // Entries j >= N hold float-range sentinels.
    float *xf;
    float *yf;
    float *zf;
    int32_t fp32;          // 1: sweep in FP32 with FP64 restarts
    int32_t force_fb;      // test hook: 1 queue every row for the exact search seeded
                           // with its winner, 2 queue every row with no seed
};

// Tolerance of the FP32 sweep's self-check: the winner's FP32 key value (its
// index tag alone may move it by 2^-14 relative) against its exact value, in
// units of the minimised sum S. The profile value is S^(1/p), so a relative
// error e in S is e/p in the profile: the tolerance scales with p/2 (AAMP and
// ACAMP count as p = 2). For ACAMP the key is 1 - rho, computed next to 1, so
// its FP32 rounding floor is a few units of 2^-24 absolute.
constexpr double FP32_SELF_CHECK = 1.5e-4;
constexpr double FP32_SELF_CHECK_ABS_Z = 2.5e-7;

// Pivot windows of the exact fallback search (triangle-inequality pruning).
constexpr int FB_PIVOTS = 16;

// Exact-search queue, shared by the jobs of a launch: rows whose winner must
// be recomputed exactly.
struct Fallback {
    int32_t *count;        // one counter, zeroed by the preparation kernel
    int32_t *rows;         // capacity entries: row within its job
    int32_t *job;          // capacity entries: job of the row
    unsigned long long *keys;   // capacity entries: best (value, index) found so far
    double *ub;            // capacity entries: upper bound on the row's distance (+inf: none)
    int32_t *job_flag;     // per job: 1 once a row of the job is queued (zeroed by prep)
    int32_t *pivots;       // FB_PIVOTS per job: window indices (-1: unused)
    float *pd;             // FB_PIVOTS x pd_stride: distance of every window to each
                           // pivot of its job; job b's windows start at its key_base
    int64_t pd_stride;
    int32_t capacity;
    int32_t pad0;
};

// One series of a launch; a single-series call is a batch of one job.
struct Job {
    Series s;              // views of the job's slices of the workspace
    double *P;             // N outputs
    int64_t *I;
    int64_t row_start;     // first position of the job in its sweep's row space
    int64_t band_base;     // first entry of the job's band table
    int64_t key_base;      // offset of the job's windows in the launch's key space
    int32_t nbands;        // bands of the band kernel (0: simple kernel, or no pairs)
    int32_t seg_rows;      // rows between exact restarts (refresh interval R)
    int32_t band_cost;     // positions a band takes in the row space before its rows
    int32_t pad1;
    // Partial (anytime) sweeps; both null for a whole profile. band_map[t] is
    // the diagonal group that band slot t covers (group g: diagonals
    // [excl + g ANY_GROUP, excl + (g + 1) ANY_GROUP)); group_ok[g] != 0 marks
    // the groups of the call, the only ones the exact search may score.
    const int32_t *band_map;
    const uint8_t *group_ok;
};

// Diagonals per group of a partial sweep: the band of the FP64 band kernel.
constexpr int64_t ANY_GROUP = 512;

// Every array the kernels touch lives in device global memory. Addressing it
// through the global address space makes the compiler emit global_* rather
// than flat_* instructions; flat ones also count against the LDS wait
// counter, so a wait for an LDS read would also wait for an outstanding HBM
// load or L2 atomic.
template <class T>
using gptr = const __attribute__((address_space(1))) T *;
template <class T>
__device__ __forceinline__ gptr<T> as_global(const T *p)
{
    return (gptr<T>)p;
}

__device__ __forceinline__ void global_min(unsigned long long *p, unsigned long long v)
{
    typedef __attribute__((address_space(1))) unsigned long long gu64;
    __hip_atomic_fetch_min((gu64 *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Job tables are read-only during a launch: kernels read them through the
// constant address space so that wave-uniform fields become scalar loads.
template <class T>
__device__ __forceinline__ T load_uniform(const T *p)
{
    static_assert(sizeof(T) % 4 == 0, "dword-sized record");
    typedef const __attribute__((address_space(4))) uint32_t cu32;
    const cu32 *src = (const cu32 *)p;
    T v;
    uint32_t *dst = (uint32_t *)&v;
#pragma unroll
    for (int k = 0; k < (int)(sizeof(T) / 4); ++k) dst[k] = src[k];
    return v;
}

// Everything a launch works on. Band-row positions: a band sweep's work is
// the concatenation over its jobs of each job's bands (band t of a job covers
// diagonals [excl + t W, excl + (t+1) W) and has N - excl - t W rows). A
// launch holds one band sweep per distance specialisation and precision
// among its jobs, each over a contiguous range of the job table; a sweep
// sees a Batch restricted to its range.
struct Batch {
    const Job *jobs;           // njobs entries
    const int64_t *row_base;   // band sweeps: njobs + 1 row_start values, then the total
    int64_t *band_start;       // per job nbands + 1 entries from band_base: launch positions
    int32_t njobs;
    int32_t band_width;        // 64 x diagonals per lane
    int64_t max_N;             // largest N of the jobs (grid of per-window kernels)
    int64_t max_stream;        // largest N + STREAM_PAD
    int64_t simple_diag;       // largest diagonal count of the simple kernel's jobs
    int64_t simple_segs;       // largest segment count of the simple kernel's jobs
    Fallback fb;
    unsigned long long *visits;    // pair-visit counter (test mode), else null
    int32_t long_jobs;             // 1: some job has m >= LONG_WINDOW (rescored in three steps)
    int32_t pad2;
};

// Kernel selectors: which distance specialisations a launch contains.
enum Sel : uint32_t {
    SEL_AAMP = 1,
    SEL_ACAMP = 2,
    SEL_P1 = 4,
    SEL_P3 = 8,
    SEL_PGEN = 16,
    SEL_FCMP = 32,     // a launch flag, not a distance: its ACAMP jobs are keyed on F
    SEL_LONG = 64,     // a launch flag: FP64 Euclidean / p = 1, 3 jobs with windows of at
                       // least LONG_WINDOW samples, run at default occupancy with their
                       // restarts' row samples staged in LDS
};

// Window length from which FP64 Euclidean and p = 1, 3 sweeps use the
// SEL_LONG kernels: there the O(m) restarts, not the recurrence, set the time,
// and the autotuner's grids of one or two waves per SIMD leave registers free.
constexpr int32_t LONG_WINDOW = 2048;

__host__ __device__ inline uint32_t sel_of(int32_t kind, int32_t pclass)
{
    if (kind == AAMP) return SEL_AAMP;
    if (kind == ACAMP) return SEL_ACAMP;
    if (pclass == P_ONE) return SEL_P1;
    if (pclass == P_THREE) return SEL_P3;
    return SEL_PGEN;
}

// Band kernels exist for AAMP, ACAMP and p-norm with p in {1, 3} (one kernel
// may hold any mix of them), and for other p up to PGEN_BAND_MAX in kernels
// of their own: a launch whose jobs are all such p-norms. Other p use the
// simple kernel.
constexpr uint32_t SEL_BAND = SEL_AAMP | SEL_ACAMP | SEL_P1 | SEL_P3;
// With |t| < 1e30 a term |a - b|^p stays below (2e30)^6 = 6.4e181 for p <= 6,
// so no real sum reaches the 1e190 of the sentinel sums and nothing in the
// recurrence overflows.
constexpr double PGEN_BAND_MAX = 6.0;

// --- launch wrappers (return the hipError_t of the launch) -------------------
// The row_base table of a one-job launch (at most one band sweep: its start
// and end, 2 entries).
struct RowBase4 {
    int64_t v[4];
    int32_t count;
    int32_t pad0;
};
hipError_t launch_store_job(const Job &j, const RowBase4 &rb, Job *dst, int64_t *row_base,
                            hipStream_t st);
hipError_t launch_prep(const Batch &b, uint32_t sels, hipStream_t st);
hipError_t launch_plan(const Batch &b, hipStream_t st);
// grid waves in blocks of wpb (1, or 4 where band_has_wave_blocks)
hipError_t launch_sweep_band(const Batch &b, uint32_t sels, int32_t diags_per_lane, bool fp32,
                             int32_t grid, int32_t wpb, hipStream_t st);
bool band_has_wave_blocks(uint32_t sels, int32_t diags_per_lane, bool fp32);
hipError_t launch_sweep_simple(const Batch &b, hipStream_t st);
hipError_t launch_finalize(const Batch &b, hipStream_t st);
hipError_t launch_fallback(const Batch &b, hipStream_t st);
hipError_t launch_any_merge(const double *Pn, const int64_t *In, double *P, int64_t *I, int64_t N,
                            hipStream_t st);

// Motifs / discords of a computed profile (k rounds of 3 small kernels).
// scratch holds 3k u64, mask N bytes.
hipError_t launch_topk(const double *P, const int64_t *I, int64_t N, int32_t k, int32_t excl,
                       int32_t mode, int64_t *out_i, int64_t *out_j, double *out_d,
                       int32_t *out_count, unsigned long long *scratch, uint8_t *mask,
                       hipStream_t st);

// Host hooks of api.hip for the other host files: error reporting (the
// thread's last error, read by mp_strerror), a one-shot FP64 profile through
// the normal pipeline, and the library lock.
int report_error(int code, const char *what);
int report_hip(hipError_t e, const char *where);
void report_ok();
int profile_once(const double *T, int64_t n, int32_t m, int32_t kind, double p, int32_t excl,
                 int32_t R, double *P, int64_t *I, hipStream_t st);

// Test hook of the allocation error path: with MP_FAIL_ALLOC=1 in the
// environment every device allocation of the library fails as if the device
// were out of memory (MP_ENOMEM), before any HIP call is made for it.
inline bool alloc_fail_hook()
{
    const char *e = std::getenv("MP_FAIL_ALLOC");
    return e && e[0] == '1' && e[1] == 0;
}

// Band-kernel facts for the planner: resident waves per CU for a selector set,
// and the selector sets that have their own kernel (others use the mixed one).
int32_t band_blocks_per_cu(uint32_t sels, int32_t diags_per_lane, bool fp32);

}  // namespace mpk
