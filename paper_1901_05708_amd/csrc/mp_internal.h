// mp_internal.h -- interface between the host side of libmp (api.hip) and its
// HIP kernels. Not installed; the public ABI is include/mp.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpk {

enum Kind : int32_t { AAMP = 0, PNORM = 1, ACAMP = 2 };

// p-norm specialisations: p = 2 runs the Euclidean kernels, p = 1 and p = 3
// have closed-form power terms, any other p goes through pow().
enum PClass : int32_t { P_GENERIC = 0, P_ONE = 1, P_TWO = 2, P_THREE = 3 };

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
    int32_t pad0;
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
    // Packed (value, index) keys, N entries; ~0 = no candidate.
    unsigned long long *keys;
    // Fallback-queue counter, zeroed by the preparation kernel.
    int32_t *fb_count;
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

// Fallback list: rows whose winner must be recomputed exactly.
struct Fallback {
    int32_t *count;        // one counter
    int32_t *rows;         // capacity entries
    unsigned long long *keys;   // capacity entries: best (value, index) found so far
    double *ub;            // capacity entries: upper bound on the row's distance (+inf: none)
    int32_t *pivots;       // FB_PIVOTS window indices (-1: unused)
    float *pd;             // FB_PIVOTS x pd_stride: distance of every window to each pivot
    int64_t pd_stride;
    int32_t capacity;
    int32_t pad0;
};

// Band-sweep work decomposition (computed on the device by launch_plan).
struct BandPlan {
    int32_t band_width;    // diagonals per band = 64 lanes x diagonals per lane
    int32_t seg_rows;      // longest run of rows between exact restarts (refresh interval R)
    int32_t nbands;
    int32_t pad0;
    int64_t *band_start;   // nbands + 1 prefix sums of the rows of each band
};

// --- launch wrappers (return the hipError_t of the launch) -------------------
hipError_t launch_prep(const Series &s, hipStream_t st);
hipError_t launch_sweep_simple(const Series &s, int32_t R, hipStream_t st);
hipError_t launch_plan(const Series &s, const BandPlan &bp, hipStream_t st);
hipError_t launch_sweep_band(const Series &s, const BandPlan &bp, int32_t diags_per_lane,
                             int32_t grid, hipStream_t st);
hipError_t launch_finalize(const Series &s, const Fallback &fb, double *P, int64_t *I,
                           hipStream_t st);
hipError_t launch_fallback(const Series &s, const Fallback &fb, double *P, int64_t *I,
                           hipStream_t st);

int32_t band_lds_bytes(int32_t kind, int32_t diags_per_lane);
int32_t band_blocks_per_cu(const Series &s, int32_t diags_per_lane);

// Band kernels exist for AAMP, ACAMP and p-norm with p in {1, 3}; other p use
// the simple kernel (the sentinel entries are only sized for those powers).
inline bool band_supported(const Series &s)
{
    return s.kind == AAMP || s.kind == ACAMP || (s.kind == PNORM && (s.pclass == P_ONE || s.pclass == P_THREE));
}

}  // namespace mpk
