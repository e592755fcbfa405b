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
};

// Fallback list: rows whose winner must be recomputed exactly.
struct Fallback {
    int32_t *count;        // one counter
    int32_t *rows;         // capacity entries
    int32_t capacity;
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
