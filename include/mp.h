/*
 * mp.h -- C ABI of libmp: matrix profile of a time series on one MI355X
 * (gfx950) GPU, computed with the diagonal-wise incremental distance sweep of
 * Akbarinia & Cloez, "Efficient Matrix Profile Computation Using Different
 * Distance Functions" (arXiv 1901.05708).
 *
 * Common conventions (every entry point):
 *
 *  - Indexing is 0-based. A series T has n samples t_0..t_{n-1}; the window
 *    T_{i,m} = <t_i .. t_{i+m-1}> exists for 0 <= i < N = n - m + 1
 *    (Def. 2.2). A pair of windows (i, j) is admissible iff |i - j| >= excl.
 *  - Outputs: P[i] is the distance from window i to its nearest admissible
 *    window (Def. 2.4) and I[i] that window's start index. A row with no
 *    admissible finite candidate gets P[i] = +inf and I[i] = -1 (N <= excl,
 *    or, z-normalized, a constant window / only constant candidates).
 *    Every reported P[i] is the distance of the pair (i, I[i]) recomputed
 *    directly in FP64 from T; when several windows are within the precision
 *    bound of the minimum any of them may be reported.
 *  - Pointers T, P, I are DEVICE pointers (hipMalloc or torch CUDA tensors,
 *    on the current HIP device); T holds n doubles, P holds N doubles, I holds
 *    N int64. The caller owns them. T is read-only; P and I are written
 *    entirely. T must be finite with |t| < 1e30 (larger magnitudes could
 *    meet the sentinel values used for out-of-range pairs).
 *  - stream is a hipStream_t (NULL = the legacy default stream). Calls are
 *    stream-ordered and asynchronous: they return after enqueueing the
 *    kernels, and the caller synchronizes before reading P and I.
 *  - excl <= 0 selects the default exclusion ceil(m/4); excl = 1 reproduces
 *    the paper's loops (every window except itself).
 *  - precision: MP_FP64 runs the whole sweep in double precision.
 *    MP_FP32_REFRESH runs the bulk of the recurrence in single precision,
 *    restarted from an exact FP64 value every R rows, with FP64 window
 *    statistics and FP64 rescoring of every winner; a row whose winner's
 *    single-precision value drifted from its exact value by more than the
 *    sweep allows is searched again exactly in FP64. It applies to ACAMP and
 *    p = 1 with m >= 32; AAMP, other p-norms and shorter windows run the
 *    FP64 sweep under MP_FP32_REFRESH.
 *    MP_FP32_AUTO keeps the MP_FP32_RTOL contract but lets the autotuner
 *    (R = 0) time the FP64 sweep beside the FP32 candidates and keep the
 *    faster per shape: near good matches the FP32 sweep's exact search of
 *    uncertified rows can cost more than it saves. With an explicit R (or
 *    MP_AUTOTUNE=0) it behaves as MP_FP32_REFRESH. mp_stats.fp32_jobs
 *    reports which sweep ran.
 *  - R is the refresh interval (rows between exact FP64 restarts of the
 *    recurrence). R = 0 lets the library choose: the first call with a given
 *    series shape (n, m, distance, excl, precision) times a few candidate
 *    refresh intervals, band widths and (for long windows) grid sizes on the
 *    call's own input, on a library
 *    stream ordered after the caller's stream, and caches the fastest (this
 *    first call blocks the host until the trials end; mp_stats.ms_autotune
 *    reports their time). Set R > 0 to skip the trials.
 *  - Errors: functions return MP_OK (0) or a negative code. Arguments are
 *    validated before any HIP call; on error nothing is enqueued and P, I are
 *    left untouched (except MP_EHIP, after which their content is undefined).
 *    No C++ exception crosses the ABI. mp_strerror() describes the last error
 *    of the calling thread.
 *  - Ownership of internal state: the library keeps a grow-only device
 *    workspace per device and caller stream (keyed by the hipStream_t value),
 *    and for mp_batch a cache of captured HIP graphs; mp_release() frees
 *    both. Calls on different streams use different workspaces and may run
 *    concurrently; calls on one stream are ordered by it. Host-side, the
 *    library serialises its calls with one lock, so any thread may call.
 */
#ifndef MP_H
#define MP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MP_OK 0
#define MP_EINVAL (-1)       /* invalid argument                               */
#define MP_ENOMEM (-2)       /* device allocation failed                       */
#define MP_EHIP (-3)         /* a HIP runtime call failed (see mp_strerror)    */
#define MP_EUNSUPPORTED (-4) /* the current device is not a gfx950 GPU         */

#define MP_FP64 0
#define MP_FP32_REFRESH 1
#define MP_FP32_AUTO 2

#define MP_KIND_AAMP 0  /* pure Euclidean                                      */
#define MP_KIND_PNORM 1 /* p-norm                                              */
#define MP_KIND_ACAMP 2 /* z-normalized Euclidean                              */

/* Relative tolerance on profile values targeted by MP_FP32_REFRESH and
 * MP_FP32_AUTO (plus 1e-6 absolute for ACAMP, where the square root
 * amplifies rounding near DZ = 0). The check that enforces it is empirical,
 * not a proven bound: it compares the winner's single-precision value with
 * its exact one, and cannot see a competitor that drifted more than the
 * winner. It has held on every row of every workload tested, for the two
 * distances that have an FP32 sweep; the Euclidean and p = 3 sums, whose
 * competitors can drift further, run in FP64 instead. FP64 results are
 * within 1e-9 relative of the exact profile. For ACAMP an absolute floor
 * applies near DZ = 0: the partner is chosen on the key 1 - rho, so with
 * delta the absolute error of that key the reported pair's DZ^2 exceeds the
 * minimum by at most 4 m delta, and DZ by at most sqrt(4 m delta). In FP64
 * delta is a few units of 2^-53 (the key is formed next to 1) plus the
 * recurrence's drift, which grows like the square root of the rows since the
 * last restart R: with delta = 2^-53 (8 + 2 sqrt(R)) and R = 64 m the floor is
 * 7e-7 at m = 16 and 5e-6 at m = 256; measured errors stay within the
 * smaller of that floor and 1e-6 at every window length tested. */
#define MP_FP32_RTOL 1e-4

/*
 * Largest supported series length (keys pack a window index in 31 bits).
 * The sweep compares candidates on packed keys whose low b = ceil(log2 N)
 * mantissa bits hold the partner index. Two candidates whose minimised
 * values differ by less than 2^-(52 - b) relative therefore count as tied,
 * and the reported partner is within that of the best: 4.7e-10 for
 * N <= 2^21, growing to 4.8e-7 at N = 2^31 (FP64). P is always the exact
 * FP64 distance of the reported pair.
 */
#define MP_MAX_N ((int64_t)1 << 31)

/*
 * mp_aamp -- pure Euclidean matrix profile (AAMP).
 * Distance: D_{i,j} = sqrt(sum_{l<m} (t_{i+l} - t_{j+l})^2)   (Def. 2.5, Eq. 1).
 * Swept with the incremental update of Lemma 1 (Eq. 4) along diagonals,
 * comparing squared distances and taking one square root per output (Sec. 3.2).
 * Requires 1 <= m <= n <= MP_MAX_N.
 */
int mp_aamp(const double *T, int64_t n, int32_t m, int32_t excl, int32_t precision,
            int32_t R, double *P, int64_t *I, void *stream);

/*
 * mp_pnorm -- p-norm matrix profile (AAMP extended to L^p, Sec. 3.4).
 * Distance: DP_{i,j} = (sum_{l<m} |t_{i+l} - t_{j+l}|^p)^(1/p)  (Def. 2.6, Eq. 2,
 * read with an absolute value), real p >= 1; updated with Lemma 2. p = 2 gives
 * exactly the result of mp_aamp. p must be finite and >= 1. p = 1 and 3 have
 * fast paths; other p up to 6 evaluate pow per term in the band sweep; larger
 * p run on a slower one-thread-per-diagonal sweep. Only p = 1 has an FP32
 * sweep: every other p runs in FP64 under MP_FP32_REFRESH too.
 */
int mp_pnorm(const double *T, int64_t n, int32_t m, double p, int32_t excl,
             int32_t precision, int32_t R, double *P, int64_t *I, void *stream);

/*
 * mp_acamp -- z-normalized Euclidean matrix profile (ACAMP, Sec. 4).
 * Distance: DZ_{i,j} = sqrt(sum_l ((t_{i+l}-mu_i)/s_i - (t_{j+l}-mu_j)/s_j)^2)
 * (Def. 2.7, Eq. 3) with population standard deviations; equivalently
 * DZ^2 = 2m(1 - rho_{i,j}) (Lemma 3, Eq. 8). A window whose samples are all
 * equal has s = 0 and infinite distance to everything (Sec. 1).
 */
int mp_acamp(const double *T, int64_t n, int32_t m, int32_t excl, int32_t precision,
             int32_t R, double *P, int64_t *I, void *stream);

/*
 * mp_acamp_fcmp -- mp_acamp in FP64 with the sweep comparing pairs on the
 * quantity F of Sec. 4.4 (Eq. 9) instead of rho. For two windows,
 * F = -m^2 rho |rho|: F grows exactly when DZ does, and
 * DZ^2 = 2m + 2 sign(F) sqrt|F| (Eq. 10, read as the squared distance). The
 * band sweep keys each pair on 1 + F / m^2 = 1 - rho |rho|, one multiply more
 * per pair than mp_acamp's 1 - rho; winners are rescored exactly as there,
 * so (P, I) agree with mp_acamp up to near ties. Series with fewer than 256
 * admissible diagonals run the simple kernel, which compares on rho (the same
 * order). Arguments, layout and errors as for mp_acamp (no precision
 * argument: FP64 only).
 */
int mp_acamp_fcmp(const double *T, int64_t n, int32_t m, int32_t excl, int32_t R, double *P,
                  int64_t *I, void *stream);

/*
 * mp_profile_noalloc -- mp_aamp / mp_pnorm / mp_acamp (selected by kind,
 * MP_KIND_*; p is read for MP_KIND_PNORM only) for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc. It calls no hipMalloc, hipFree or other
 * allocating routine. Every array the pipeline needs lives in one static
 * device array of 56 MiB per GPU, held from the library's load until the
 * process ends; its address is looked up on the first call on each device.
 *
 * Arguments, layout and results are those of the single-series entry points,
 * with three differences:
 *  - the series may have at most MP_NOALLOC_MAX_N windows (n - m + 1);
 *    longer series return MP_EINVAL before anything is enqueued;
 *  - R = 0 takes the library's default refresh interval instead of running
 *    the autotuner (MP_FP32_AUTO then behaves as MP_FP32_REFRESH);
 *  - profiling (mp_set_profiling) records nothing for these calls.
 * All calls on one GPU share its array and leave their contents there; each
 * call clears what it needs cleared. Two calls on one GPU whose kernels can
 * run at the same time (on different streams with no ordering between them)
 * race; calls serialized on one stream do not.
 */
#define MP_NOALLOC_MAX_N ((int64_t)1 << 18)
int mp_profile_noalloc(int32_t kind, const double *T, int64_t n, int32_t m, double p,
                       int32_t excl, int32_t precision, int32_t R, double *P, int64_t *I,
                       void *stream);

/*
 * One series of a batch. Offsets are in elements. Series b occupies
 * T_cat[t_off .. t_off + n) and its N_b = n - m + 1 outputs go to
 * P_cat[out_off ..), I_cat[out_off ..); I values are local to the series.
 * kind is MP_KIND_*; p is used by MP_KIND_PNORM only; excl and R as above.
 */
typedef struct mp_job {
    int64_t t_off;
    int64_t n;
    int64_t out_off;
    int32_t m;
    int32_t kind;
    int32_t excl;
    int32_t R;
    double p;
} mp_job;

/*
 * mp_batch -- matrix profiles of many independent series in one call: for
 * each distance (and precision) among the jobs, one persistent launch of the
 * sweep lays the bands of diagonals of all its series end to end and splits
 * them evenly over the waves of one grid, whatever the mix of lengths and
 * window lengths (the single-series kernels of Algorithms 1-3, extended over
 * a job table).
 *
 * jobs is a HOST array of njobs entries (read during the call only),
 * 0 <= njobs <= 65535. Each job obeys the single-series rules above; output
 * ranges of different jobs must not overlap (MP_EINVAL otherwise). I values
 * are local to their series.
 *
 * The first call with a given batch shape (the job table without its offsets,
 * and the precision) runs the autotuner: a few trial runs of the whole batch
 * with different band widths (diagonals per lane), refresh intervals R (jobs
 * with R = 0 only) and, for long windows, persistent grid sizes, keeping the
 * fastest; its time is reported in
 * mp_stats.ms_autotune. The first call with a given job table, precision and
 * pointers captures the pipeline into a HIP graph; later identical calls
 * replay it (while profiling is on the pipeline is launched directly, so that
 * its phases can be timed). The graph runs on a library stream ordered after
 * the caller's stream and before the caller's later work.
 */
int mp_batch(const double *T_cat, const mp_job *jobs, int32_t njobs, int32_t precision,
             double *P_cat, int64_t *I_cat, void *stream);

/*
 * Partial (anytime) sweeps. Every outer iteration k of Algorithms 1-3 visits
 * the pairs of diagonal k only, and nothing carries from one iteration to the
 * next; the paper calls the algorithms anytime for this reason (Sec. 1,
 * Sec. 7). A sweep stopped after any set of diagonals leaves, for every row,
 * the exact distance to the best partner on those diagonals: an upper bound on
 * the row's profile value that only decreases as more diagonals are visited,
 * and equal to it once all are.
 *
 * The diagonals excl .. N-1 (N = n - m + 1) are cut into groups of
 * MP_ANYTIME_GROUP: group g holds diagonals [excl + g*512, excl + (g+1)*512)
 * that are below N, so there are ceil((N - excl) / 512) groups (0 when
 * N <= excl). Work per group is proportional to its pairs, about 512 (N - d).
 *
 * mp_anytime_groups: *ngroups receives the number of groups of (n, m, excl);
 *   excl <= 0 means ceil(m/4). Host only.
 * mp_anytime_order: writes a uniformly random permutation of the groups to
 *   the HOST array order (mp_anytime_groups entries), drawn by Fisher-Yates
 *   with splitmix64 from seed (STAMP-style random order, Sec. 6), and, if
 *   cum_pairs is not null, the number of admissible pairs covered after each
 *   prefix of it (HOST int64 array of the same size; the last entry is the
 *   total pair count). Host only; never touches the GPU.
 * mp_anytime: the profile over the diagonals of the listed groups. T, P, I
 *   and the distance arguments are as for mp_aamp / mp_pnorm / mp_acamp
 *   (device pointers, FP64 precision, R chosen by the library); kind is
 *   MP_KIND_*; p-norms need p <= 6. groups is a HOST array of ngroups group
 *   indices in [0, mp_anytime_groups) (read during the call only; repeats
 *   cost work but do not change the result); ngroups = 0 visits nothing.
 *   resume = 0: P, I receive the profile over those diagonals (+inf / -1 for
 *     rows without a candidate there).
 *   resume = 1: P, I must hold on entry the output of an earlier mp_anytime
 *     or full-profile call on the same series and arguments; every row keeps
 *     the better of its entry and the new candidates (equal distances: the
 *     smaller index), so a sequence of calls over groups A, B, ... gives the
 *     profile over their union.
 *   Rows are rescored exactly in FP64 as in the full profile; P[i] is the
 *   distance of (i, I[i]). Errors: MP_EINVAL for a bad group index, ngroups
 *   < 0, resume not 0 or 1, p > 6, or the single-series argument errors.
 *   Stream-ordered and asynchronous; uses the workspace of its stream.
 */
#define MP_ANYTIME_GROUP 512
int mp_anytime_groups(int64_t n, int32_t m, int32_t excl, int64_t *ngroups);
int mp_anytime_order(int64_t n, int32_t m, int32_t excl, uint64_t seed, int32_t *order,
                     int64_t *cum_pairs);
int mp_anytime(int32_t kind, const double *T, int64_t n, int32_t m, double p, int32_t excl,
               const int32_t *groups, int64_t ngroups, int32_t resume, double *P, int64_t *I,
               void *stream);

/*
 * mp_topk -- motifs or discords of a computed profile, the two uses of the
 * matrix profile named in Sec. 1. P and I are the N outputs of one mp_aamp /
 * mp_pnorm / mp_acamp call (device pointers).
 *  - mode MP_MOTIFS: k times, the not yet excluded window i with the smallest
 *    finite P[i] (ties: the smallest i) is reported as (i, I[i], P[i]), then
 *    every window x with |x - i| < excl or |x - I[i]| < excl is excluded (a
 *    motif pair is reported once, and its trivially shifted neighbours not).
 *  - mode MP_DISCORDS: the largest finite P[i] instead, excluding the windows
 *    with |x - i| < excl.
 * out_i, out_j (int64) and out_d (double) are device arrays of k entries;
 * *out_count (device int32) receives the number of rounds that found a
 * candidate (fewer than k once every finite window is excluded; entries past
 * it are left untouched). excl >= 1 (typically the profile's exclusion zone
 * or m); 0 <= k <= 65536; 0 <= N < MP_MAX_N. Stream-ordered and
 * asynchronous; 3 small launches per round; uses the workspace of its stream.
 */
#define MP_MOTIFS 0
#define MP_DISCORDS 1
int mp_topk(const double *P, const int64_t *I, int64_t N, int32_t k, int32_t excl, int32_t mode,
            int64_t *out_i, int64_t *out_j, double *out_d, int32_t *out_count, void *stream);

/*
 * Incremental profiles: the profile of a series that grows by appended
 * samples. Appending one sample adds one window w, i.e. one new column of the
 * distance matrix; each entry (i, w) follows from (i - 1, w - 1) in the
 * previous column by the O(1) updates of Lemmas 1-3, so the whole profile is
 * brought up to date in O(N) per added window. Every row whose minimum
 * improves, and every new window, is rescored exactly in FP64, so after any
 * sequence of appends (P, I) is what mp_aamp / mp_pnorm / mp_acamp in FP64
 * would return for the whole series (up to ties). The carried column is
 * recomputed exactly every `refresh` added windows (0: 4096). The first
 * windows, and any append adding more than max(2048, N/8) windows, run the
 * one-shot FP64 pipeline instead.
 *
 * mp_inc_create: m, kind (MP_KIND_*), p, excl (<= 0: ceil(m/4)) as for the
 *   single-series calls; capacity = the largest number of samples the series
 *   will hold (m <= capacity < MP_MAX_N; device buffers of about 70 bytes
 *   per sample are allocated now). *out receives the handle.
 * mp_inc_append: appends count samples from the DEVICE pointer T (copied).
 *   MP_EINVAL if the capacity would be exceeded. Stream-ordered and
 *   asynchronous; calls on one handle must be serialised on one stream.
 * mp_inc_state: the current number of samples and windows, and DEVICE
 *   pointers to the N profile values and indices (owned by the handle, valid
 *   until mp_inc_destroy; read them after the stream has synchronised).
 * mp_inc_read: copies the current N profile values and indices into the
 *   caller's DEVICE arrays, stream-ordered.
 * mp_inc_destroy: waits for the device and frees the handle.
 */
typedef struct mp_inc mp_inc;
int mp_inc_create(int32_t m, int32_t kind, double p, int32_t excl, int64_t capacity,
                  int32_t refresh, mp_inc **out);
int mp_inc_append(mp_inc *h, const double *T, int64_t count, void *stream);
int mp_inc_state(mp_inc *h, int64_t *n, int64_t *N, double **P, int64_t **I);
int mp_inc_read(mp_inc *h, double *P, int64_t *I, void *stream);
void mp_inc_destroy(mp_inc *h);

/* Human-readable description of an error code, including the HIP error text
 * of the calling thread's last MP_EHIP. Never NULL; the string is owned by the
 * library and valid until the next call on the same thread. */
const char *mp_strerror(int code);

/* Free the workspaces and graph cache of every device and stream. Safe to call at
 * any time no call is in flight; later calls re-allocate. */
void mp_release(void);

/*
 * Profiling. mp_set_profiling(1) clears the accumulated figures and from then
 * on every call records HIP events on its own stream around each phase; this
 * adds no host synchronization to the calls. mp_profile_read() waits for the
 * recorded events and returns the figures summed over all calls made since
 * profiling was switched on (timings in milliseconds of GPU time), with the
 * configuration fields of the most recent call. mp_set_profiling(0) stops
 * recording. Returns MP_OK, or MP_EINVAL if out is NULL.
 */
typedef struct mp_stats {
    double ms_prep;          /* window statistics, difference streams, key fill, work plan */
    double ms_sweep;         /* the diagonal sweep kernel(s) alone              */
    double ms_finalize;      /* rescoring, certification and fallback           */
    double ms_autotune;      /* host time spent by the batch autotuner (counted  
                                whether or not profiling is on)                  */
    int64_t pairs;           /* admissible unordered pairs                      */
    int64_t fallback_rows;   /* rows recomputed exactly in FP64                 */
    int64_t pairs_visited;   /* pairs the sweeps visited, counted only in the
                                test mode MP_COUNT_PAIRS=1 (else 0); equals
                                pairs when the work split is exact               */
    int32_t calls;           /* calls accumulated                               */
    int32_t sweep_launches;  /* sweep kernel launches accumulated               */
    int32_t refresh_rows;    /* R of the most recent call (its first band-swept job) */
    int32_t diags_per_lane;  /* diagonals per lane of the band kernel, most recent call */
    int32_t items;           /* work items (diagonal band x row segment), most recent call */
    int32_t graph_replays;   /* mp_batch calls served by replaying a captured graph,
                                since the last mp_set_profiling() (counted whether
                                or not profiling is on)                          */
    int32_t band_jobs;       /* jobs swept by the band kernel, most recent call  */
    int32_t fp32_jobs;       /* of those, jobs swept in FP32, most recent call   */
} mp_stats;

void mp_set_profiling(int on);
int mp_profile_read(mp_stats *out);

#ifdef __cplusplus
}
#endif

#endif /* MP_H */
