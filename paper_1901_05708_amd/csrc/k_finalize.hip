// k_finalize.hip -- turn the packed keys into the profile (Algorithm 2's final
// square-root loop, generalised): decode the winning index of every row,
// recompute that one pair's distance directly in FP64, take the root. Rows
// whose winner is not a legal candidate (z-normalized: a constant window), or
// whose FP32 key disagrees with the exact value by more than the single-
// precision sweep allows, are queued and searched again exactly: k_fallback_scan
// scores, straight from the definition, every column that the triangle
// inequality over a few pivot windows cannot exclude.
#include "dd.h"
#include "exact.h"
#include "keys.h"
#include "mp_internal.h"

namespace mpk {

// Queue row i of job jb for the exact search, seeded with its best known
// (key, distance).
__device__ __forceinline__ void enqueue(const Fallback &fb, int32_t jb, int64_t i,
                                        unsigned long long seed, double ub)
{
    const int pos = atomicAdd(fb.count, 1);
    if (pos < fb.capacity) {
        fb.rows[pos] = (int32_t)i;
        fb.job[pos] = jb;
        fb.keys[pos] = seed;
        fb.ub[pos] = ub;
    }
    fb.job_flag[jb] = 1;
}

// First part of a row's finalize: rows without a candidate get +inf / -1,
// rows whose winner is not a legal candidate go to the exact search; returns
// true (with the winner j) when the winner's exact distance is needed.
template <int KIND>
__device__ __forceinline__ bool finalize_decode(const Series &s, const Fallback &fb, int32_t jb,
                                                int64_t i, double *P, int64_t *I, int64_t *j_out)
{
    const unsigned long long mask = (1ull << s.gb) - 1ull;
    const unsigned long long key = s.keys[i];
    if ((KIND == ACAMP && s.isconst[i]) || key == KEY_NONE) {
        P[i] = __longlong_as_double(0x7FF0000000000000ll);
        I[i] = -1;
        return false;
    }
    const int64_t j = (int64_t)(key & mask);
    if (!legal_pair(s, i, j)) {
        enqueue(fb, jb, i, KEY_NONE, __longlong_as_double(0x7FF0000000000000ll));
        return false;
    }
    *j_out = j;
    return true;
}

// Second part, given the exact pre-root distance ex of (i, j).
template <int KIND, int PC>
__device__ __forceinline__ void finalize_finish(const Series &s, const Fallback &fb, int32_t jb,
                                                int64_t i, int64_t j, double ex, double *P,
                                                int64_t *I)
{
    const unsigned long long mask = (1ull << s.gb) - 1ull;
    if (s.force_fb) {
        if (s.force_fb == 1)
            enqueue(fb, jb, i, pack_key(ex, (unsigned long long)j, mask), root_of<KIND, PC>(ex, s.p));
        else
            enqueue(fb, jb, i, KEY_NONE, __longlong_as_double(0x7FF0000000000000ll));
        return;
    }
    if (s.fp32) {
        // Self-check of the single-precision sweep: the winner's key value is
        // its FP32 value (up to the 2^-14 of its index tag); a larger gap to
        // the exact value means FP32 drift on this row, which is then searched
        // again exactly, starting from this winner. The key holds the
        // minimised quantity: the sum (AAMP, p-norm) or 1 - rho = DZ^2 / 2m
        // (ACAMP).
        const double kv = key_value(s.keys[i], mask);
        const double xv = (KIND == ACAMP) ? ex / (2.0 * (double)s.m) : ex;
        const double pscale = (KIND == PNORM) ? 0.5 * s.p : 1.0;
        const double tol = FP32_SELF_CHECK * pscale * fabs(xv) +
                           (KIND == ACAMP ? FP32_SELF_CHECK_ABS_Z : 0.0);
        // A winner at exact distance 0 is a minimum whatever the drift.
        if (ex != 0.0 && !(fabs(kv - xv) <= tol)) {
            enqueue(fb, jb, i, pack_key(ex, (unsigned long long)j, mask), root_of<KIND, PC>(ex, s.p));
            return;
        }
    }
    P[i] = root_of<KIND, PC>(ex, s.p);
    I[i] = j;
}

constexpr int FIN_BLOCK = 256;   // rows per block of k_finalize
constexpr int FIN_CHUNK = 64;    // steps per staged chunk

// LDS of a k_finalize block: the staged row and winner samples and the
// block's range of winner diagonals.
struct FinLds {
    double sa[FIN_BLOCK + FIN_CHUNK];
    double sb[FIN_BLOCK + FIN_CHUNK];
    long long dlo, dhi;
    int any;
};

// Rows i0 .. i0 + 255 of one job, one thread each. At step l the rows need
// the samples t[i0 + l .. i0 + l + 255], one contiguous run, which is staged
// in LDS chunk by chunk (the next chunk's loads issued before the current one
// is consumed). When every winner of the block lies on one diagonal
// (j = i + d, the common case: neighbouring windows' best matches shift
// together), the winners' samples are a contiguous run too and are staged the
// same way; otherwise each thread loads its winner's samples. Every exact sum
// adds its terms in order of l, with the same terms as exact_sum.
// need / j: whether the block's row i0 + threadIdx.x needs its sum, and the
// winner (finalize_decode, already applied).
template <int KIND, int PC>
__device__ __forceinline__ void finalize_block_sums(const Series &s, const Fallback &fb,
                                                    int32_t jb, int64_t i0, bool need, int64_t j,
                                                    double *P, int64_t *I, FinLds &L)
{
    constexpr int B = FIN_BLOCK, CH = FIN_CHUNK, SPAN = B + CH;
    double *sa = L.sa, *sb = L.sb;
    const int t = threadIdx.x;
    const int64_t i = i0 + t;
    if (t == 0) {
        L.dlo = INT64_MAX;
        L.dhi = INT64_MIN;
        L.any = 0;
    }
    __syncthreads();
    if (need) {
        atomicMin(&L.dlo, (long long)(j - i));
        atomicMax(&L.dhi, (long long)(j - i));
        L.any = 1;
    }
    __syncthreads();
    if (!L.any) return;   // block-uniform
    const bool diag = L.dlo == L.dhi;
    const int64_t d = L.dlo;
    const gptr<double> T = as_global(s.T);
    const int64_t tmax = s.n - 1;
    const int m = s.m;
    const double p = s.p;
    double mi = 0.0, mj = 0.0, ni = 0.0, nj = 0.0;
    if (KIND == ACAMP && need) {
        mi = s.mu[i];
        mj = s.mu[j];
        ni = s.invn[i];
        nj = s.invn[j];
    }
    double ra0, ra1, rb0 = 0.0, rb1 = 0.0;
    auto fetch = [&](int l0) {
        ra0 = T[min(i0 + l0 + t, tmax)];
        ra1 = (t + B < SPAN) ? T[min(i0 + l0 + t + B, tmax)] : 0.0;
        if (diag) {
            // rows that need no sum stage samples too; the diagonal may put
            // their positions before the series start, so clamp both ends
            rb0 = T[min(max(i0 + d + l0 + t, (int64_t)0), tmax)];
            rb1 = (t + B < SPAN) ? T[min(max(i0 + d + l0 + t + B, (int64_t)0), tmax)] : 0.0;
        }
    };
    auto put = [&]() {
        __syncthreads();
        sa[t] = ra0;
        if (t + B < SPAN) sa[t + B] = ra1;
        if (diag) {
            sb[t] = rb0;
            if (t + B < SPAN) sb[t + B] = rb1;
        }
        __syncthreads();
    };
    // a winner's own samples, when the block has no common diagonal
    // (rows that need no sum read t[0], which always exists)
    const gptr<double> tb = T + (need ? j : 0);
    double acc = 0.0;
    fetch(0);
    put();
    for (int l0 = 0; l0 < m; l0 += CH) {
        const bool more = l0 + CH < m;
        if (more) fetch(l0 + CH);
        const int steps = min(CH, m - l0);
        if (diag) {
            for (int u = 0; u < steps; ++u)
                acc = exact_term<KIND, PC>(sa[t + u], sb[t + u], mi, ni, mj, nj, p, acc);
        } else if (need) {
            for (int u = 0; u < steps; ++u)
                acc = exact_term<KIND, PC>(sa[t + u], tb[l0 + u], mi, ni, mj, nj, p, acc);
        }
        if (more) put();
    }
    if (need) {
        const double ex = (KIND == ACAMP) ? acc * (double)m : acc;
        finalize_finish<KIND, PC>(s, fb, jb, i, j, ex, P, I);
    }
}

template <int KIND, int PC>
__device__ __forceinline__ void finalize_block(const Series &s, const Fallback &fb, int32_t jb,
                                               int64_t i0, double *P, int64_t *I, FinLds &L)
{
    const int64_t i = i0 + threadIdx.x;
    int64_t j = 0;
    const bool need = i < s.N && finalize_decode<KIND>(s, fb, jb, i, P, I, &j);
    finalize_block_sums<KIND, PC>(s, fb, jb, i0, need, j, P, I, L);
}

// ---- rescoring of long windows --------------------------------------------
//
// For m >= LONG_WINDOW a direct sum per row costs O(m) per row, while
// neighbouring rows usually have their winners on one diagonal (j = i + d):
// then the sum of row i follows from that of row i - 1 by adding the term of
// the pair that enters (i + m - 1, j + m - 1) and subtracting the one that
// leaves (i - 1, j - 1). A block of 256 rows splits into runs of consecutive
// rows with a common winner diagonal; each run's first pair is summed over
// its m terms by one of LONG_ANCHOR_SPLIT blocks set aside for the block of
// rows, and a segmented prefix sum carries it along the run.
// All of it is double-double (dd.h), so the running sums lose about 2^-104 of
// their largest partial sum to cancellation instead of 2^-53. The quantities:
//   AAMP, p-norm: the sum of (a - b)^2 or |a - b|^p (the terms rounded as in
//     the direct sum, their accumulation exact to double-double);
//   ACAMP: with the row samples shifted by c_a = t[i0] and the column
//     samples by c_b, the first sample of the 256-window block of the run's
//     first column window (u = t - c, kept exact as a double-double: rounding
//     it would move rho by 2^-53 times the window's offset from c over its
//     spread, and 2m (1 - rho) near a perfect match turns that into an
//     absolute DZ error), the cross sum C = sum u_a u_b. The window sums
//     S = sum u and Q = sum u^2 come from the window statistics (k_prep keeps
//     them, double-double, shifted by the first sample of each window's
//     256-window block: c_a for the rows of this block, moved to c_b for the
//     column windows by S(c_b) = S(c) + m (c - c_b)). Then
//     m cov = m C - S_a S_b and E = m ||window - mu||^2 = m Q - S^2 (both the
//     same for any shifts, as long as C, S_a and S_b share them), and
//     DZ^2 = 2m (1 - rho) (Lemma 3) with 1 - rho taken without cancellation:
//     (E_a E_b - (m cov)^2) / (sqrt(E_a E_b) (sqrt(E_a E_b) + m cov)) for
//     positive cov.
// The rounded result is at least as close to the exact distance as the direct
// FP64 sum, whose own error grows like m 2^-53.
static_assert(FIN_BLOCK == 256, "the rescoring's row shift is the window statistics' block shift");

struct FinLongLds {
    DD buf[FIN_BLOCK];
    long long diag[FIN_BLOCK];
    int ibuf[FIN_BLOCK];
    double cb[FIN_BLOCK];
};

// Adds the term of the pair of samples (a, b) to the running sum q
// (unnormalised: dd_norm it before other double-double arithmetic).
template <int KIND, int PC>
__device__ __forceinline__ void long_term(DD &q, double a, double b, double ca, double cb,
                                          double p, double sign)
{
    if (KIND == ACAMP) {
        // the shifted samples exactly (two-sum), their product to 2^-106
        const DD ua = dd_two_sum(a, -ca), ub = dd_two_sum(b, -cb);
        dd_acc(q, dd_mul((sign < 0.0) ? dd_neg(ua) : ua, ub));
    } else if (KIND == AAMP) {
        const double d = a - b;
        const DD sq = dd_prod(d, d);
        dd_acc(q, {sign * sq.hi, sign * sq.lo});
    } else {
        dd_acc(q, {sign * pn_term<PC>(a - b, p), 0.0});
    }
}

// The shift of window j's sums in wsum: the first sample of its block.
__device__ __forceinline__ double wsum_shift(const gptr<double> T, int64_t j)
{
    return T[j & ~(int64_t)(FIN_BLOCK - 1)];
}

// Blocks of step 2 per block of rows: block g sums the anchors of runs
// g, g + LONG_ANCHOR_SPLIT, ... of its block of rows (most blocks of rows
// hold a few runs; every run of a block of 256 rows can be a single row).
constexpr int LONG_ANCHOR_SPLIT = 16;

// finalize_decode without its side effects (the later steps of the
// long-window rescoring read the keys again): whether row i has a winner to
// rescore, and which.
template <int KIND>
__device__ __forceinline__ bool decode_quiet(const Series &s, int64_t i, int64_t *j_out)
{
    const unsigned long long mask = (1ull << s.gb) - 1ull;
    const unsigned long long key = s.keys[i];
    if ((KIND == ACAMP && s.isconst[i]) || key == KEY_NONE) return false;
    const int64_t j = (int64_t)(key & mask);
    if (!legal_pair(s, i, j)) return false;
    *j_out = j;
    return true;
}

// Runs of a block: consecutive rows that need a sum and share the winner
// diagonal dg. Returns their number; head / run tell whether this thread's
// row starts a run and the index of its run. Every thread of the block calls it.
__device__ __forceinline__ int long_runs(bool need, long long dg, FinLongLds &L, bool &head,
                                         int &run)
{
    const int t = threadIdx.x;
    const long long d = need ? dg : LLONG_MIN;
    L.diag[t] = d;
    __syncthreads();
    head = need && (t == 0 || L.diag[t - 1] != d);
    run = int_block_scan<FIN_BLOCK>(head ? 1 : 0, L.ibuf) - 1;
    const int nh = L.ibuf[FIN_BLOCK - 1];
    __syncthreads();
    return nh;
}

// Rescoring of long windows, in three launches, so that the runs' exact first
// sums (the anchors) are spread over the GPU instead of being taken one after
// another by the block of their rows:
//  1. (k_finalize) decode the block's winners, find its runs and record them
//     (lcount, lhead);
//  2. (k_long_anchors) LONG_ANCHOR_SPLIT blocks per block of rows sum its
//     runs' first pairs (run k in block k mod LONG_ANCHOR_SPLIT);
//  3. (k_long_finish) each block slides the anchors along its runs and
//     finishes its rows.
template <int KIND, int PC>
__device__ __forceinline__ void finalize_block_long(const Series &s, const Fallback &fb,
                                                    int32_t jb, int64_t i0, double *P,
                                                    int64_t *I, unsigned char *lds)
{
    FinLongLds &L = *reinterpret_cast<FinLongLds *>(lds);
    const int t = threadIdx.x;
    const int64_t i = i0 + t;
    int64_t j = 0;
    const bool need = i < s.N && finalize_decode<KIND>(s, fb, jb, i, P, I, &j);
    bool head;
    int run;
    const int nheads = long_runs(need, (long long)(j - i), L, head, run);
    if (head) s.lhead[i0 + run] = t;
    if (t == 0) s.lcount[i0] = nheads;
}

// Step 2: the exact sum of the first pair of run k of the block of rows from
// i0, by the whole block (two independent partial sums per thread, for
// instruction-level parallelism in the serial double-double chains).
template <int KIND, int PC>
__device__ __forceinline__ void long_anchor(const Series &s, int64_t i0, int k, DD *buf)
{
    constexpr int B = FIN_BLOCK;
    const int t = threadIdx.x;
    const int64_t ih = i0 + s.lhead[i0 + k];
    int64_t jh = 0;
    decode_quiet<KIND>(s, ih, &jh);   // a run's first row has a winner
    const gptr<double> T = as_global(s.T);
    const int m = s.m;
    const double p = s.p;
    const double ca = (KIND == ACAMP) ? T[i0] : 0.0;
    const double cb = (KIND == ACAMP) ? wsum_shift(T, jh) : 0.0;
    DD q = {0.0, 0.0}, q2 = {0.0, 0.0};
    int l = t;
    for (; l + B < m; l += 2 * B) {
        long_term<KIND, PC>(q, T[ih + l], T[jh + l], ca, cb, p, 1.0);
        long_term<KIND, PC>(q2, T[ih + l + B], T[jh + l + B], ca, cb, p, 1.0);
    }
    if (l < m) long_term<KIND, PC>(q, T[ih + l], T[jh + l], ca, cb, p, 1.0);
    const DD tot = dd_block_sum<B>(dd_add(dd_norm(q), dd_norm(q2)), buf);
    if (t == 0) {
        s.lanchor[2 * (i0 + k)] = tot.hi;
        s.lanchor[2 * (i0 + k) + 1] = tot.lo;
    }
}

// Step 3: every other row of a run is its preceding row's sum plus the pair
// entering minus the pair leaving; a segmented prefix sum carries the
// anchors along the runs.
template <int KIND, int PC>
__device__ __forceinline__ void finalize_block_long_finish(const Series &s, const Fallback &fb,
                                                           int32_t jb, int64_t i0, double *P,
                                                           int64_t *I, unsigned char *lds)
{
    FinLongLds &L = *reinterpret_cast<FinLongLds *>(lds);
    constexpr int B = FIN_BLOCK;
    const int t = threadIdx.x;
    const int64_t i = i0 + t;
    int64_t j = 0;
    const bool need = i < s.N && decode_quiet<KIND>(s, i, &j);
    bool head;
    int run;
    long_runs(need, (long long)(j - i), L, head, run);
    const gptr<double> T = as_global(s.T);
    const int m = s.m;
    const double p = s.p;
    const double ca = (KIND == ACAMP) ? T[i0] : 0.0;
    if (KIND == ACAMP && head) L.cb[run] = wsum_shift(T, j);
    __syncthreads();
    const double cbr = (KIND == ACAMP && need) ? L.cb[run] : 0.0;
    DD x = {0.0, 0.0};
    if (head) {
        x = {s.lanchor[2 * (i0 + run)], s.lanchor[2 * (i0 + run) + 1]};
    } else if (need) {
        long_term<KIND, PC>(x, T[i + m - 1], T[j + m - 1], ca, cbr, p, 1.0);
        long_term<KIND, PC>(x, T[i - 1], T[j - 1], ca, cbr, p, -1.0);
        x = dd_norm(x);
    }
    x = dd_segment_scan<B>(head || !need, x, L.buf, L.ibuf);
    if (!need) return;
    double ex;
    if (KIND == ACAMP) {
        // window sums from the statistics: the row's shifted by c_a (its
        // block is this block), the column's moved to the run's c_b
        const double *wa = s.wsum + 4 * i, *wb = s.wsum + 4 * j;
        const DD sa = {wa[0], wa[1]}, qa = {wa[2], wa[3]};
        const DD sj = {wb[0], wb[1]}, qj = {wb[2], wb[3]};
        const DD md = {(double)m, 0.0};
        const DD sb = dd_add(sj, dd_mul(md, dd_two_sum(wsum_shift(T, j), -cbr)));
        const DD mcov = dd_sub(dd_mul(md, x), dd_mul(sa, sb));
        const DD ea = dd_sub(dd_mul(md, qa), dd_mul(sa, sa));
        const DD eb = dd_sub(dd_mul(md, qj), dd_mul(sj, sj));
        const DD eab = dd_mul(ea, eb);
        const double prod = dd_val(eab);
        if (!(prod > 0.0)) {
            ex = exact_sum<KIND, PC>(s, i, j);   // degenerate energies: the direct sum
        } else {
            const double sq = sqrt(prod), c = dd_val(mcov);
            double omr;   // 1 - rho
            if (c <= 0.0) {
                omr = 1.0 - c / sq;
            } else {
                const DD num = dd_sub(eab, dd_mul(mcov, mcov));
                omr = fmax(dd_val(num), 0.0) / (sq * (sq + c));
            }
            ex = 2.0 * (double)m * omr;
        }
    } else {
        ex = fmax(dd_val(x), 0.0);
    }
    finalize_finish<KIND, PC>(s, fb, jb, i, j, ex, P, I);
}

// Grid: x over blocks of FIN_BLOCK windows, y over jobs.
__global__ void __launch_bounds__(FIN_BLOCK) k_finalize(Batch b)
{
    const int32_t jb = blockIdx.y;
    const Job J = load_uniform(&b.jobs[jb]);
    const int64_t i0 = (int64_t)blockIdx.x * FIN_BLOCK;
    if (i0 >= J.s.N) return;   // block-uniform
    constexpr size_t LDS_BYTES = sizeof(FinLds) > sizeof(FinLongLds) ? sizeof(FinLds)
                                                                      : sizeof(FinLongLds);
    __shared__ __align__(16) unsigned char lds[LDS_BYTES];
    if (J.s.m >= LONG_WINDOW) {
        switch (sel_of(J.s.kind, J.s.pclass)) {
        case SEL_AAMP: finalize_block_long<AAMP, P_TWO>(J.s, b.fb, jb, i0, J.P, J.I, lds); break;
        case SEL_ACAMP: finalize_block_long<ACAMP, P_TWO>(J.s, b.fb, jb, i0, J.P, J.I, lds); break;
        case SEL_P1: finalize_block_long<PNORM, P_ONE>(J.s, b.fb, jb, i0, J.P, J.I, lds); break;
        case SEL_P3: finalize_block_long<PNORM, P_THREE>(J.s, b.fb, jb, i0, J.P, J.I, lds); break;
        default: finalize_block_long<PNORM, P_GENERIC>(J.s, b.fb, jb, i0, J.P, J.I, lds); break;
        }
        return;
    }
    FinLds &L = *reinterpret_cast<FinLds *>(lds);
    switch (sel_of(J.s.kind, J.s.pclass)) {
    case SEL_AAMP: finalize_block<AAMP, P_TWO>(J.s, b.fb, jb, i0, J.P, J.I, L); break;
    case SEL_ACAMP: finalize_block<ACAMP, P_TWO>(J.s, b.fb, jb, i0, J.P, J.I, L); break;
    case SEL_P1: finalize_block<PNORM, P_ONE>(J.s, b.fb, jb, i0, J.P, J.I, L); break;
    case SEL_P3: finalize_block<PNORM, P_THREE>(J.s, b.fb, jb, i0, J.P, J.I, L); break;
    default: finalize_block<PNORM, P_GENERIC>(J.s, b.fb, jb, i0, J.P, J.I, L); break;
    }
}

// Step 2 of the long-window rescoring. Grid: x over (g, block of rows), g
// major (the blocks of first runs come first), y over jobs.
__global__ void __launch_bounds__(FIN_BLOCK) k_long_anchors(Batch b, int32_t nblk)
{
    const int32_t jb = blockIdx.y;
    const Job J = load_uniform(&b.jobs[jb]);
    if (J.s.m < LONG_WINDOW) return;
    const int g = (int)(blockIdx.x / (uint32_t)nblk);
    const int64_t i0 = (int64_t)(blockIdx.x - (uint32_t)g * (uint32_t)nblk) * FIN_BLOCK;
    if (i0 >= J.s.N) return;   // block-uniform
    const int nheads = J.s.lcount[i0];
    __shared__ DD buf[FIN_BLOCK];
    for (int k = g; k < nheads; k += LONG_ANCHOR_SPLIT) {
        switch (sel_of(J.s.kind, J.s.pclass)) {
        case SEL_AAMP: long_anchor<AAMP, P_TWO>(J.s, i0, k, buf); break;
        case SEL_ACAMP: long_anchor<ACAMP, P_TWO>(J.s, i0, k, buf); break;
        case SEL_P1: long_anchor<PNORM, P_ONE>(J.s, i0, k, buf); break;
        case SEL_P3: long_anchor<PNORM, P_THREE>(J.s, i0, k, buf); break;
        default: long_anchor<PNORM, P_GENERIC>(J.s, i0, k, buf); break;
        }
    }
}

// Step 3 of the long-window rescoring. Grid as k_finalize's.
__global__ void __launch_bounds__(FIN_BLOCK) k_long_finish(Batch b)
{
    const int32_t jb = blockIdx.y;
    const Job J = load_uniform(&b.jobs[jb]);
    const int64_t i0 = (int64_t)blockIdx.x * FIN_BLOCK;
    if (J.s.m < LONG_WINDOW || i0 >= J.s.N) return;   // block-uniform
    __shared__ __align__(16) unsigned char lds[sizeof(FinLongLds)];
    switch (sel_of(J.s.kind, J.s.pclass)) {
    case SEL_AAMP: finalize_block_long_finish<AAMP, P_TWO>(J.s, b.fb, jb, i0, J.P, J.I, lds); break;
    case SEL_ACAMP:
        finalize_block_long_finish<ACAMP, P_TWO>(J.s, b.fb, jb, i0, J.P, J.I, lds);
        break;
    case SEL_P1: finalize_block_long_finish<PNORM, P_ONE>(J.s, b.fb, jb, i0, J.P, J.I, lds); break;
    case SEL_P3:
        finalize_block_long_finish<PNORM, P_THREE>(J.s, b.fb, jb, i0, J.P, J.I, lds);
        break;
    default:
        finalize_block_long_finish<PNORM, P_GENERIC>(J.s, b.fb, jb, i0, J.P, J.I, lds);
        break;
    }
}

// ---------------------------------------------------------------------------
// Exact search for queued rows.
//
// All three distances are metrics (Euclidean, Minkowski p >= 1, Euclidean
// between z-normalized windows), so for any pivot window c
//     D(i, j) >= |D(i, c) - D(j, c)|.
// k_pivot_dist stores D(c, j) for FB_PIVOTS pivots and every window j; a column
// whose bound exceeds the row's known upper bound (the exact distance of the
// single-precision winner) can be neither the minimum nor tied with it and is
// skipped. The remaining columns are compacted per wavefront and scored
// exactly. Rows without an upper bound (an illegal winner) score every column.
// ---------------------------------------------------------------------------
constexpr int FB_WAVE = 64;
constexpr int FB_ITERS = 64;                       // 64-column steps per work unit
constexpr int FB_CHUNK = FB_WAVE * FB_ITERS;       // columns per work unit
constexpr int FB_MAXM = 1024;                      // longer row windows are read from T
constexpr int FB_UNROLL = 16;
// Slack of the pruning test: the stored pivot distances are FP64 sums rounded
// to FP32 (relative error below 2^-24, plus ~m 2^-53 from the sum).
constexpr double FB_PD_SLACK = 2.5e-7;

// Pivot windows spread evenly over the series; ACAMP skips constant windows
// (looking up to 4096 windows ahead, else the pivot is left unused).
__global__ void k_pick_pivots(Batch b)
{
    const Fallback &fb = b.fb;
    const int32_t jb = blockIdx.x;
    if (fb.job_flag[jb] == 0) return;
    const Job J = load_uniform(&b.jobs[jb]);
    const Series &s = J.s;
    const int lane = threadIdx.x;
    if (J.group_ok) {
        // a partial sweep queues only rows without an upper bound, which no
        // pivot bound can prune: no pivots
        if (lane < FB_PIVOTS) fb.pivots[jb * FB_PIVOTS + lane] = -1;
        return;
    }
    for (int k = 0; k < FB_PIVOTS; ++k) {
        const int64_t c0 = ((2 * (int64_t)k + 1) * s.N) / (2 * FB_PIVOTS);
        int64_t found = -1;
        for (int t = 0; t < 64 && found < 0; ++t) {
            const int64_t c = (c0 + (int64_t)t * FB_WAVE + lane) % s.N;
            const bool ok = !(s.kind == ACAMP && s.isconst[c]);
            const unsigned long long bal = __ballot(ok);
            if (bal) {
                const int first = __ffsll((long long)bal) - 1;
                found = (c0 + (int64_t)t * FB_WAVE + first) % s.N;
            }
        }
        if (lane == 0) fb.pivots[jb * FB_PIVOTS + k] = (int32_t)found;
    }
}

template <int KIND, int PC>
__device__ __forceinline__ float pivot_distance(const Series &s, int32_t c, int64_t j)
{
    return c < 0 ? 0.0f : (float)root_of<KIND, PC>(exact_sum<KIND, PC>(s, c, j), s.p);
}

// Grid: x over windows, y over pivots, z over jobs.
__global__ void __launch_bounds__(256) k_pivot_dist(Batch b)
{
    const Fallback &fb = b.fb;
    const int32_t jb = blockIdx.z;
    if (fb.job_flag[jb] == 0) return;
    const Job J = load_uniform(&b.jobs[jb]);
    const Series &s = J.s;
    const int k = blockIdx.y;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= s.N) return;
    const int32_t c = fb.pivots[jb * FB_PIVOTS + k];
    if (c < 0) return;          // unused pivot: the scan never reads its column
    float d;
    switch (sel_of(s.kind, s.pclass)) {
    case SEL_AAMP: d = pivot_distance<AAMP, P_TWO>(s, c, j); break;
    case SEL_ACAMP: d = pivot_distance<ACAMP, P_TWO>(s, c, j); break;
    case SEL_P1: d = pivot_distance<PNORM, P_ONE>(s, c, j); break;
    case SEL_P3: d = pivot_distance<PNORM, P_THREE>(s, c, j); break;
    default: d = pivot_distance<PNORM, P_GENERIC>(s, c, j); break;
    }
    fb.pd[(int64_t)k * fb.pd_stride + J.key_base + j] = d;
}

__device__ __forceinline__ int lanes_below(unsigned long long mask)
{
    return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// One work unit of the exact search: queue entry r (row i of the job whose
// series is s), columns [c FB_CHUNK, (c + 1) FB_CHUNK). q is the LDS copy of
// the row window (centred and scaled for ACAMP), staged when the row changes;
// queue is the wave's candidate list.
template <int KIND, int PC>
__device__ __forceinline__ void scan_unit(const Series &s, const Fallback &fb, int64_t pd_base,
                                          const int32_t *pivots, const uint8_t *gok, int r,
                                          int64_t c, double *q, int32_t *queue, int64_t &prev_row)
{
    const int lane = threadIdx.x;
    const unsigned long long mask = (1ull << s.gb) - 1ull;
    const int m = s.m;
    const bool staged = m <= FB_MAXM;
    {
        const int64_t i = fb.rows[r];
        if (gok) {
            // a partial sweep: skip a chunk with no column on the call's
            // diagonal groups (diagonals |i - j| over the chunk's columns)
            const int64_t c0 = c * FB_CHUNK, c1 = min(c0 + FB_CHUNK, s.N) - 1;
            int64_t dlo = c0 > i ? c0 - i : (c1 < i ? i - c1 : 0);
            const int64_t dhi = c0 > i ? c1 - i : (c1 < i ? i - c0 : max(i - c0, c1 - i));
            dlo = max(dlo, (int64_t)s.excl);
            bool any = false;
            for (int64_t g = (dlo - s.excl) / ANY_GROUP; dlo <= dhi && g <= (dhi - s.excl) / ANY_GROUP;
                 ++g)
                any = any || as_global(gok)[g] != 0;
            if (!any) return;
        }
        const double thr = fb.ub[r] * (1.0 + 1e-9);
        const double mi = (KIND == ACAMP) ? s.mu[i] : 0.0;
        const double ni = (KIND == ACAMP) ? s.invn[i] : 1.0;
        if (staged && (int64_t)r != prev_row) {
            __syncthreads();
            for (int l = lane; l < m; l += FB_WAVE)
                q[l] = (KIND == ACAMP) ? (as_global(s.T)[i + l] - mi) * ni : as_global(s.T)[i + l];
            __syncthreads();
            prev_row = r;
        }
        unsigned long long best = KEY_NONE;
        int qn = 0;
        // Exact score of column j. The column window is read in batches of
        // FB_UNROLL independent loads so that their latency overlaps.
        const gptr<double> Tg = as_global(s.T);
        auto score = [&](int64_t j) {
            const gptr<double> b = Tg + j;
            const double mj = (KIND == ACAMP) ? as_global(s.mu)[j] : 0.0;
            const double nj = (KIND == ACAMP) ? as_global(s.invn)[j] : 1.0;
            double acc = 0.0;
            auto term = [&](double a, double bv) {
                if (KIND == ACAMP) {
                    const double d = a - (bv - mj) * nj;
                    acc = fma(d, d, acc);
                } else if (KIND == AAMP) {
                    const double d = a - bv;
                    acc = fma(d, d, acc);
                } else {
                    acc += pn_term<PC>(a - bv, s.p);
                }
            };
            auto qa = [&](int l) {
                if (staged) return q[l];
                return (KIND == ACAMP) ? (Tg[i + l] - mi) * ni : Tg[i + l];
            };
            int l = 0;
            for (; l + FB_UNROLL <= m; l += FB_UNROLL) {
                double bb[FB_UNROLL];
#pragma unroll
                for (int u = 0; u < FB_UNROLL; ++u) bb[u] = b[l + u];
#pragma unroll
                for (int u = 0; u < FB_UNROLL; ++u) term(qa(l + u), bb[u]);
            }
            for (; l < m; ++l) term(qa(l), b[l]);
            if (KIND == ACAMP) acc *= (double)m;
            const unsigned long long key = pack_key(acc, (unsigned long long)j, mask);
            best = key < best ? key : best;
        };
        for (int it = 0; it < FB_ITERS; ++it) {
            const int64_t j = c * FB_CHUNK + (int64_t)it * FB_WAVE + lane;
            bool cand = legal_pair(s, i, j);
            if (gok && cand) {      // a partial sweep: only the call's diagonal groups
                const int64_t d = i > j ? i - j : j - i;
                cand = as_global(gok)[(d - s.excl) / ANY_GROUP] != 0;
            }
            for (int k = 0; k < FB_PIVOTS; ++k) {
                if (__ballot(cand) == 0) break;
                if (pivots[k] < 0) continue;
                // the row's own pivot distance is uniform across the wavefront
                const float pa = fb.pd[(int64_t)k * fb.pd_stride + pd_base + i];
                if (cand) {
                    const double a = pa,
                                 b = as_global(fb.pd)[(int64_t)k * fb.pd_stride + pd_base + j];
                    const double lb = fabs(a - b) - FB_PD_SLACK * (a + b);
                    if (lb > thr) cand = false;       // false for NaN bounds: kept
                }
            }
            const unsigned long long bal = __ballot(cand);
            if (cand) queue[qn + lanes_below(bal)] = (int32_t)j;
            qn += __popcll(bal);
            __syncthreads();
            if (qn >= FB_WAVE) {
                score(queue[lane]);
                const int rest = qn - FB_WAVE;
                const int32_t moved = lane < rest ? queue[FB_WAVE + lane] : 0;
                __syncthreads();
                if (lane < rest) queue[lane] = moved;
                qn = rest;
                __syncthreads();
            }
        }
        if (lane < qn) score(queue[lane]);
        __syncthreads();
        for (int off = 32; off > 0; off >>= 1) {
            const unsigned long long o = __shfl_xor(best, off);
            best = o < best ? o : best;
        }
        if (lane == 0 && best != KEY_NONE) global_min(&fb.keys[r], best);
    }
}

// Grid-stride over the work units (queue entry, column chunk); chunks past
// the entry's series end return at once.
__global__ void __launch_bounds__(FB_WAVE) k_fallback_scan(Batch b)
{
    __shared__ double q[FB_MAXM];
    __shared__ int32_t queue[2 * FB_WAVE];
    const Fallback &fb = b.fb;
    const int cnt = min(*fb.count, fb.capacity);
    const int64_t nch = (b.max_N + FB_CHUNK - 1) / FB_CHUNK;
    const int64_t units = (int64_t)cnt * nch;
    int64_t prev_row = -1;
    for (int64_t u = blockIdx.x; u < units; u += gridDim.x) {
        const int r = (int)(u / nch);
        const int64_t c = u - (int64_t)r * nch;
        const int32_t jb = __builtin_amdgcn_readfirstlane(fb.job[r]);
        const Job J = load_uniform(&b.jobs[jb]);
        const Series &s = J.s;
        if (c * FB_CHUNK >= s.N) continue;
        const int32_t *piv = fb.pivots + jb * FB_PIVOTS;
        const uint8_t *gok = J.group_ok;
        switch (sel_of(s.kind, s.pclass)) {
        case SEL_AAMP: scan_unit<AAMP, P_TWO>(s, fb, J.key_base, piv, gok, r, c, q, queue, prev_row); break;
        case SEL_ACAMP: scan_unit<ACAMP, P_TWO>(s, fb, J.key_base, piv, gok, r, c, q, queue, prev_row); break;
        case SEL_P1: scan_unit<PNORM, P_ONE>(s, fb, J.key_base, piv, gok, r, c, q, queue, prev_row); break;
        case SEL_P3: scan_unit<PNORM, P_THREE>(s, fb, J.key_base, piv, gok, r, c, q, queue, prev_row); break;
        default: scan_unit<PNORM, P_GENERIC>(s, fb, J.key_base, piv, gok, r, c, q, queue, prev_row); break;
        }
    }
}

// Rows of the fallback queue: decode the exact search's winner and rescore it.
template <int KIND, int PC>
__device__ __forceinline__ void finish_row(const Job &J, unsigned long long key, int64_t i)
{
    const Series &s = J.s;
    const unsigned long long mask = (1ull << s.gb) - 1ull;
    if (key == KEY_NONE) {
        J.P[i] = __longlong_as_double(0x7FF0000000000000ll);
        J.I[i] = -1;
    } else {
        const int64_t j = (int64_t)(key & mask);
        J.P[i] = root_of<KIND, PC>(exact_sum<KIND, PC>(s, i, j), s.p);
        J.I[i] = j;
    }
}

__global__ void k_fallback_finish(Batch b)
{
    const Fallback &fb = b.fb;
    const int cnt = min(*fb.count, fb.capacity);
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < cnt; r += gridDim.x * blockDim.x) {
        const Job J = b.jobs[fb.job[r]];
        const int64_t i = fb.rows[r];
        const unsigned long long key = fb.keys[r];
        switch (sel_of(J.s.kind, J.s.pclass)) {
        case SEL_AAMP: finish_row<AAMP, P_TWO>(J, key, i); break;
        case SEL_ACAMP: finish_row<ACAMP, P_TWO>(J, key, i); break;
        case SEL_P1: finish_row<PNORM, P_ONE>(J, key, i); break;
        case SEL_P3: finish_row<PNORM, P_THREE>(J, key, i); break;
        default: finish_row<PNORM, P_GENERIC>(J, key, i); break;
        }
    }
}

// Merge of a partial profile (Pn, In) into an earlier one (P, I) of the same
// series: the smaller distance wins, equal distances keep the smaller index.
// Both hold exact FP64 distances of their pairs (+inf / -1: none yet), so the
// result is the profile over the union of the two sets of diagonals.
__global__ void k_any_merge(const double *Pn, const int64_t *In, double *P, int64_t *I, int64_t N)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= N) return;
    const int64_t jn = In[r];
    if (jn < 0) return;
    const double pn = Pn[r], po = P[r];
    const int64_t jo = I[r];
    if (jo < 0 || pn < po || (pn == po && jn < jo)) {
        P[r] = pn;
        I[r] = jn;
    }
}

hipError_t launch_any_merge(const double *Pn, const int64_t *In, double *P, int64_t *I, int64_t N,
                            hipStream_t st)
{
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_any_merge, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, Pn, In,
                       P, I, N);
    return hipGetLastError();
}

hipError_t launch_finalize(const Batch &b, hipStream_t st)
{
    if (b.njobs <= 0) return hipSuccess;
    const int64_t nblk = (b.max_N + FIN_BLOCK - 1) / FIN_BLOCK;
    dim3 g((unsigned)nblk, (unsigned)b.njobs);
    hipLaunchKernelGGL(k_finalize, g, dim3(FIN_BLOCK), 0, st, b);
    if (b.long_jobs) {
        if (nblk * LONG_ANCHOR_SPLIT > INT32_MAX) return hipErrorInvalidValue;
        dim3 ga((unsigned)(nblk * LONG_ANCHOR_SPLIT), (unsigned)b.njobs);
        hipLaunchKernelGGL(k_long_anchors, ga, dim3(FIN_BLOCK), 0, st, b, (int32_t)nblk);
        hipLaunchKernelGGL(k_long_finish, g, dim3(FIN_BLOCK), 0, st, b);
    }
    return hipGetLastError();
}

hipError_t launch_fallback(const Batch &b, hipStream_t st)
{
    // Every kernel returns at once when the queue (or the job's share of it)
    // is empty.
    if (b.njobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pick_pivots, dim3((unsigned)b.njobs), dim3(FB_WAVE), 0, st, b);
    const dim3 gpd((unsigned)((b.max_N + 255) / 256), FB_PIVOTS, (unsigned)b.njobs);
    hipLaunchKernelGGL(k_pivot_dist, gpd, dim3(256), 0, st, b);
    hipLaunchKernelGGL(k_fallback_scan, dim3(8192), dim3(FB_WAVE), 0, st, b);
    hipLaunchKernelGGL(k_fallback_finish, dim3(64), dim3(256), 0, st, b);
    return hipGetLastError();
}

}  // namespace mpk
