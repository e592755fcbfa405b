// k_prep.hip -- per-window preparation that sits outside the sweep's inner
// loop: the O(m (n - m)) part of the method (Secs. 3.3 and 4.3), computed once
// per window in FP64 instead of once per diagonal.
#include "dd.h"
#include "keys.h"
#include "mp_internal.h"

namespace mpk {

// Window mean, exact all-equal flag and inverse centred norm
// invn_j = 1 / sqrt(sum_l (t_{j+l} - mu_j)^2) = 1 / (sqrt(m) sigma_j) with the
// population standard deviation of App. A. Below LONG_WINDOW they are computed
// directly in two passes per window (no running sums, so no cancellation over
// long series); from LONG_WINDOW on, by exact slides from one anchor per block
// (below). A constant window gets invn = 0; its z-normalized distance to
// anything is infinite (Sec. 1) and the sweep never lets it win.
constexpr int STATS_BLOCK = 256;   // windows per block of k_window_stats
constexpr int STATS_CHUNK = 64;    // steps per staged chunk

// ---- long windows: one exact anchor per block, the rest by exact slides ----
//
// For m >= LONG_WINDOW the direct two passes cost O(m) per window. A block of
// 256 windows instead sums its first window (the anchor) exactly and reaches
// the others by adding what enters and leaves, in double-double arithmetic
// (dd.h). With every sample shifted by c = t[j0] (u = t - c, kept exact as a
// double-double), window j has
//   S_j = sum u,  Q_j = sum u^2,  mu_j = c + S_j / m,
//   ||window - mu_j||^2 = (m Q_j - S_j^2) / m,
// where S_j and Q_j are the anchor's sums plus block-wide prefix sums of
// u_in - u_out and u_in^2 - u_out^2. The subtraction cancels, but its inputs
// carry about 2^-104 relative error, so the centred energy keeps about
// 2^-104 (Q / energy) relative error before its final rounding: far below
// the two-pass sums' own m 2^-53 for any series whose windows vary above
// 1e-10 of their offset from c. Constant windows are flagged exactly from
// integer counts of sample changes, never from the energy. S_j and Q_j are
// kept (wsum) for the rescoring of z-normalized pairs.
__device__ __forceinline__ void window_stats_long(const Series &s, int64_t j0, DD *dbuf,
                                                  int *ibuf)
{
    const int t = threadIdx.x;
    const gptr<double> T = as_global(s.T);
    const int64_t tmax = s.n - 1;
    const int m = s.m;
    const double c = T[j0];
    // the anchor window j0: S, Q and the number of sample changes in
    // (j0, j0 + m - 1], each thread over a stride of the window
    DD S = {0.0, 0.0}, Q = {0.0, 0.0};
    int brk = 0;
    for (int l = t; l < m; l += STATS_BLOCK) {
        const double v = T[j0 + l];
        const DD u = dd_two_sum(v, -c);
        dd_acc(S, u);
        dd_acc(Q, dd_mul(u, u));
        if (l > 0) brk += (v != T[j0 + l - 1]) ? 1 : 0;
    }
    // block totals (the last thread of each inclusive scan holds them)
    const DD S0 = dd_block_sum<STATS_BLOCK>(dd_norm(S), dbuf);
    const DD Q0 = dd_block_sum<STATS_BLOCK>(dd_norm(Q), dbuf);
    brk = int_block_scan<STATS_BLOCK>(brk, ibuf);
    const int B0 = ibuf[STATS_BLOCK - 1];
    __syncthreads();
    // window j = j0 + t (t >= 1) differs from window j - 1 by u_in = u[j+m-1]
    // entering and u_out = u[j-1] leaving
    const int64_t j = j0 + t;
    DD dS = {0.0, 0.0}, dQ = {0.0, 0.0};
    int brk_out = 0, brk_in = 0;
    if (t > 0) {
        const double vin = T[min(j + m - 1, tmax)], vout = T[j - 1];
        const DD uin = dd_two_sum(vin, -c), uout = dd_two_sum(vout, -c);
        dS = dd_sub(uin, uout);
        dQ = dd_sub(dd_mul(uin, uin), dd_mul(uout, uout));
        // a change at position j (entering the interval (j0, j]) and at j + m - 1
        brk_out = (T[j] != vout) ? 1 : 0;
        brk_in = (j + m - 1 <= tmax && vin != T[j + m - 2]) ? 1 : 0;
    }
    const DD Sj = dd_add(S0, dd_block_scan<STATS_BLOCK>(dS, dbuf));
    __syncthreads();
    const DD Qj = dd_add(Q0, dd_block_scan<STATS_BLOCK>(dQ, dbuf));
    __syncthreads();
    const int pre = int_block_scan<STATS_BLOCK>(brk_out, ibuf);
    __syncthreads();
    const int post = int_block_scan<STATS_BLOCK>(brk_in, ibuf);
    if (j < s.N) {
        // changes inside (j, j + m - 1]: the anchor's, minus those in (j0, j],
        // plus those in (j0 + m - 1, j + m - 1]
        const bool same = (B0 - pre + post) == 0;
        const double mu = c + dd_val(Sj) / (double)m;
        const DD e = dd_sub(dd_mul(Qj, {(double)m, 0.0}), dd_mul(Sj, Sj));   // m ||w - mu||^2
        const double ss = dd_val(e) / (double)m;
        s.mu[j] = mu;
        s.isconst[j] = same ? 1 : 0;
        s.invn[j] = (same || !(ss > 0.0)) ? 0.0 : 1.0 / sqrt(ss);
        // the exact sums, for the rescoring of long windows
        double *ws = s.wsum + 4 * j;
        ws[0] = Sj.hi;
        ws[1] = Sj.lo;
        ws[2] = Qj.hi;
        ws[3] = Qj.lo;
    }
}

__global__ void __launch_bounds__(STATS_BLOCK) k_window_stats(Batch b)
{
    const Series s = load_uniform(&b.jobs[blockIdx.y]).s;
    if (s.kind != ACAMP) return;
    if (s.m >= LONG_WINDOW) {
        __shared__ DD dbuf[STATS_BLOCK];
        __shared__ int ibuf[STATS_BLOCK];
        const int64_t j0 = (int64_t)blockIdx.x * STATS_BLOCK;
        if (j0 < s.N) window_stats_long(s, j0, dbuf, ibuf);
        return;
    }
    // The block's windows j0 .. j0 + 255 need, at step l, the samples
    // t[j0 + l .. j0 + l + 255]: one contiguous run. Chunks of STATS_CHUNK
    // steps are staged in LDS (the next chunk's loads are issued before the
    // current one is consumed) and each thread reads its window's sample of
    // the step from there, instead of a global load per window and sample.
    constexpr int B = STATS_BLOCK, CH = STATS_CHUNK, SPAN = B + CH;
    __shared__ double st[SPAN];
    const int t = threadIdx.x;
    const int64_t j0 = (int64_t)blockIdx.x * B;
    if (j0 >= s.N) return;
    const int64_t j = j0 + t;
    const gptr<double> T = as_global(s.T);
    const int64_t tmax = s.n - 1;
    const int m = s.m;
    double r0, r1;
    auto fetch = [&](int l0) {
        r0 = T[min(j0 + l0 + t, tmax)];
        r1 = (t + B < SPAN) ? T[min(j0 + l0 + t + B, tmax)] : 0.0;
    };
    auto put = [&]() {
        __syncthreads();
        st[t] = r0;
        if (t + B < SPAN) st[t + B] = r1;
        __syncthreads();
    };
    // f(t[j + l]) for l = 0 .. m-1 in order (every thread of the block takes
    // part, also those past the last window, for the barriers)
    auto walk = [&](auto &&f) {
        fetch(0);
        put();
        for (int l0 = 0; l0 < m; l0 += CH) {
            const bool more = l0 + CH < m;
            if (more) fetch(l0 + CH);
            const int steps = min(CH, m - l0);
            if (steps == CH) {
#pragma unroll 16
                for (int u = 0; u < CH; ++u) f(st[t + u]);
            } else {
                for (int u = 0; u < steps; ++u) f(st[t + u]);
            }
            if (more) put();
        }
    };
    // The mean is summed around the window's first sample, so its rounding
    // error scales with the window's deviations rather than with the series'
    // offset. Neighbouring windows share all but one sample, so a plain sum's
    // offset-scale errors are correlated from window to window, and the
    // covariance recurrence would accumulate them as drift.
    double sum = 0.0;
    bool same = true;
    const double w0 = T[min(j, tmax)];
    walk([&](double v) {
        sum += v - w0;
        same = same && (v == w0);
    });
    const double mu = w0 + sum / (double)m;
    double ss = 0.0;
    walk([&](double v) {
        const double d = v - mu;
        ss = fma(d, d, ss);
    });
    if (j < s.N) {
        s.mu[j] = mu;
        s.isconst[j] = same ? 1 : 0;
        s.invn[j] = (same || !(ss > 0.0)) ? 0.0 : 1.0 / sqrt(ss);
    }
}

// Per-window difference streams used by the O(1) diagonal updates, and the
// key array reset. Entry j describes what changes when a window slides from
// start j-1 to start j: sample t_{j-1} leaves, sample t_{j+m-1} enters.
//
//  AAMP (Lemma 1): D^2_{i,j} - D^2_{i-1,j-1}
//        = (t_{i+m-1} - t_{j+m-1})^2 - (t_{i-1} - t_{j-1})^2
//        = (u_i - u_j)(v_i - v_j),  u = t_{.+m-1} - t_{.-1}, v = t_{.+m-1} + t_{.-1}
//  p-norm (Lemma 2): |a_i - a_j|^p - |b_i - b_j|^p,  a = t_{.+m-1}, b = t_{.-1}
//  ACAMP: the centred cross sum cov_{i,j} = sum_l (t_{i+l}-mu_i)(t_{j+l}-mu_j)
//        (the numerator C - A B / m of Lemma 3) obeys
//        cov_{i,j} = cov_{i-1,j-1} + df_i dg_j + df_j dg_i
//        with df = (t_{.+m-1} - t_{.-1}) / 2 and
//        dg_j = (t_{j+m-1} - mu_j) + (t_{j-1} - mu_{j-1}).
//        Stored with z_j = -invn_j so that -rho = cov invn_i z_j.
// Entries j >= N hold sentinels that make every pair touching them lose.
// Also resets the launch's exact-search queue, the job's queue flag and the
// pair-visit counter of the test mode.
__global__ void k_streams(Batch b)
{
    const Series s = load_uniform(&b.jobs[blockIdx.y]).s;
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = s.N + STREAM_PAD;
    if (j >= total) return;
    if (j < s.N) s.keys[j] = KEY_NONE;
    if (j == 0) {
        b.fb.job_flag[blockIdx.y] = 0;
        if (blockIdx.y == 0) {
            *b.fb.count = 0;
            if (b.visits) *b.visits = 0;
        }
    }
    const int m = s.m;
    double x = 0.0, y = 0.0, z = 0.0;
    if (j >= s.N) {
        if (s.kind == AAMP) {
            x = SENT_EUCLID;
            y = SENT_EUCLID;
        } else if (s.kind == PNORM) {
            x = (s.pclass == P_ONE) ? SENT_P1 : (s.pclass == P_THREE ? SENT_P3 : sent_pgen(s.p));
            y = 0.0;
        }
    } else if (j >= 1) {
        const double tin = s.T[j + m - 1];
        const double tout = s.T[j - 1];
        if (s.kind == AAMP) {
            x = tin - tout;
            y = tin + tout;
        } else if (s.kind == PNORM) {
            x = tin;
            y = tout;
        } else {
            x = 0.5 * (tin - tout);
            y = (tin - s.mu[j]) + (tout - s.mu[j - 1]);
        }
    }
    if (s.kind == ACAMP && j < s.N) z = -s.invn[j];
    s.x[j] = x;
    s.y[j] = y;
    if (s.kind == ACAMP) s.z[j] = z;
    if (s.fp32) {
        // FP32 copies for the single-precision sweep. Values are recentred by
        // c = t_0 before rounding (the recurrence only uses differences of
        // like entries, so the shift cancels), keeping the rounding error
        // relative to the series' spread rather than its offset.
        const double c = s.T[0];
        float xf, yf, zf = (float)z;
        if (j >= s.N) {
            if (s.kind == AAMP) {
                xf = SENTF_EUCLID;
                yf = SENTF_EUCLID;
            } else if (s.kind == PNORM) {
                xf = (s.pclass == P_ONE) ? SENTF_P1 : (s.pclass == P_THREE ? SENTF_P3 : 0.0f);
                yf = 0.0f;
            } else {
                xf = 0.0f;
                yf = 0.0f;
            }
        } else if (j == 0) {
            xf = 0.0f;
            yf = 0.0f;
        } else if (s.kind == AAMP) {
            xf = (float)x;
            yf = (float)(y - 2.0 * c);
        } else if (s.kind == PNORM) {
            xf = (float)(x - c);
            yf = (float)(y - c);
        } else {
            xf = (float)x;
            yf = (float)y;
        }
        s.xf[j] = xf;
        s.yf[j] = yf;
        if (s.kind == ACAMP) s.zf[j] = zf;
    }
}

// Job table of a single-series call, written on the stream from the kernel
// arguments so that consecutive calls never share a host staging buffer.
__global__ void k_store_job(Job j, RowBase4 rb, Job *dst, int64_t *row_base)
{
    if (threadIdx.x == 0) *dst = j;
    if (threadIdx.x < rb.count) row_base[threadIdx.x] = rb.v[threadIdx.x];
}

hipError_t launch_store_job(const Job &j, const RowBase4 &rb, Job *dst, int64_t *row_base,
                            hipStream_t st)
{
    hipLaunchKernelGGL(k_store_job, dim3(1), dim3(64), 0, st, j, rb, dst, row_base);
    return hipGetLastError();
}

hipError_t launch_prep(const Batch &b, uint32_t sels, hipStream_t st)
{
    const int B = 256;
    if (b.njobs <= 0) return hipSuccess;
    if (sels & SEL_ACAMP) {
        dim3 g((unsigned)((b.max_N + STATS_BLOCK - 1) / STATS_BLOCK), (unsigned)b.njobs);
        hipLaunchKernelGGL(k_window_stats, g, dim3(STATS_BLOCK), 0, st, b);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    dim3 g((unsigned)((b.max_stream + B - 1) / B), (unsigned)b.njobs);
    hipLaunchKernelGGL(k_streams, g, dim3(B), 0, st, b);
    return hipGetLastError();
}

}  // namespace mpk
