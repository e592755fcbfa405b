// k_incremental.hip -- the profile of a growing series, kept up to date as
// samples are appended (mp_inc_* in include/mp.h).
//
// A new sample adds one window w at the end, i.e. one new column of the
// distance matrix. Every entry of that column lies on a diagonal k = w - i
// whose previous entry, (i - 1, w - 1), is in the column before it, so the
// same O(1) updates that drive the sweep (Lemma 1, Lemma 2, the centred form
// of Lemma 3) give the whole new column in O(N) from the previous one. The
// library keeps that last column; each new entry updates the row minimum of
// row i and the column minimum of w (Algorithms 1-3, run along the new
// column instead of along the diagonals).
//
//  * k_inc_stats: window statistics (ACAMP) of the new windows, key reset.
//  * k_inc_columns: one thread per diagonal walks the chunk's new columns,
//    starting from the stored last column or, at a refresh and on diagonals
//    that begin inside the chunk, from an exact FP64 sum. Row keys travel
//    up the lanes of a wave with their row and leave it with one atomic;
//    all threads take the same column at a step, so its key is reduced over
//    the wave before its one atomic.
//  * k_inc_rescore: the new windows and the old rows whose key changed take
//    their exact FP64 distance (as the one-shot path does).
// A first load, and any append longer than a fraction of the series, runs the
// one-shot pipeline instead and rebuilds the state from its profile.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <new>
#include <type_traits>

#include "../../include/mp.h"
#include "exact.h"
#include "keys.h"
#include "mp_internal.h"

namespace mpk {

constexpr int INC_BLOCK = 256;        // threads per block of the column walk
constexpr int64_t INC_COLS = 2048;    // new columns per column launch at most

// Device views of an incremental state; N is the number of windows after the
// chunk being processed.
struct IncState {
    const double *T;
    double *P;
    int64_t *I;
    unsigned long long *keys;
    double *mu;
    double *invn;
    uint8_t *isconst;
    const double *col_old;     // S(r, w0 - 1) for rows r <= w0 - 1 - excl
    double *col_new;           // S(r, w1) after the chunk
    int64_t N;
    int32_t m, kind, pclass, excl;
    double p;
    int32_t gb;
    int32_t pad0;
};

__device__ __forceinline__ Series inc_series(const IncState &s)
{
    Series v;
    v.T = s.T;
    v.n = s.N + s.m - 1;
    v.N = s.N;
    v.m = s.m;
    v.kind = s.kind;
    v.pclass = s.pclass;
    v.excl = s.excl;
    v.p = s.p;
    v.gb = s.gb;
    v.mu = s.mu;
    v.invn = s.invn;
    v.isconst = s.isconst;
    v.keys = s.keys;
    v.x = v.y = v.z = nullptr;
    v.xf = v.yf = v.zf = nullptr;
    v.fp32 = 0;
    v.force_fb = 0;
    v.fcmp = 0;
    return v;
}

constexpr int STATS_WAVES = 4;   // windows per block of k_inc_stats (one wave each)

// Sum over the 64 lanes of the wave, in every lane.
__device__ __forceinline__ double wave_sum(double x)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// Window statistics of windows [w0, w1] (two passes, mean around the first
// sample) and key reset. One wave per window: the lanes take every 64th
// sample, then the wave adds their partial sums.
__global__ void __launch_bounds__(64 * STATS_WAVES) k_inc_stats(IncState s, int64_t w0, int64_t w1)
{
    const int lane = threadIdx.x & 63;
    const int64_t w = w0 + (int64_t)blockIdx.x * STATS_WAVES + (threadIdx.x >> 6);
    if (w > w1) return;                          // the whole wave
    if (lane == 0) s.keys[w] = KEY_NONE;
    if (s.kind != ACAMP) return;
    const gptr<double> x = as_global(s.T) + w;
    const int m = s.m;
    const double x0 = x[0];
    double sum = 0.0;
    bool same = true;
    for (int l = lane; l < m; l += 64) {
        const double v = x[l];
        sum += v - x0;
        same = same && (v == x0);
    }
    sum = wave_sum(sum);
    const bool all_same = __ballot(!same) == 0;
    const double mu = x0 + sum / (double)m;
    double ss = 0.0;
    for (int l = lane; l < m; l += 64) {
        const double d = x[l] - mu;
        ss = fma(d, d, ss);
    }
    ss = wave_sum(ss);
    if (lane == 0) {
        s.mu[w] = mu;
        s.isconst[w] = all_same ? 1 : 0;
        s.invn[w] = (all_same || !(ss > 0.0)) ? 0.0 : 1.0 / sqrt(ss);
    }
}

// The quantity the recurrence carries along a diagonal, directly: the
// pre-root sum (AAMP, p-norm) or the centred cross sum (ACAMP).
template <int KIND, int PC>
__device__ double inc_start(const IncState &s, int64_t i, int64_t j)
{
    const gptr<double> a = as_global(s.T) + i;
    const gptr<double> b = as_global(s.T) + j;
    double acc = 0.0;
    if (KIND == ACAMP) {
        const double mi = s.mu[i], mj = s.mu[j];
        visit_pairs<8>(a, b, s.m, [&](double x, double y) { acc = fma(x - mi, y - mj, acc); });
        return acc;
    }
    const double p = s.p;
    visit_pairs<8>(a, b, s.m, [&](double x, double y) {
        const double d = x - y;
        acc += (KIND == AAMP) ? d * d : pn_term<PC>(d, p);
    });
    return acc;
}

// Operands of the pair (i, j): those of the update from (i - 1, j - 1) and,
// for ACAMP, those of its key.
struct IncOps {
    double ai, bi, aj, bj;     // t[i+m-1], t[i-1], t[j+m-1], t[j-1]
    double mi, mi1, mj, mj1;   // ACAMP: mu_i, mu_{i-1}, mu_j, mu_{j-1}
    double ni, nj;             // ACAMP: invn_i, invn_j
    bool ci, cj;               // ACAMP: constant windows
};

// Loads them. Rows outside [1, N - 1] (a lane whose diagonal has no row at
// this column yet, or row 0, which only takes a start value) read row 1 or
// N - 1 for the update operands and row 0 or N - 1 for the key operands:
// in-bounds values that are never used for the update. Columns satisfy
// 1 <= j < N.
template <int KIND>
__device__ __forceinline__ IncOps inc_load(const IncState &s, int64_t i, int64_t j)
{
    const gptr<double> T = as_global(s.T);
    const int64_t iu = min(max(i, (int64_t)1), s.N - 1);
    const int64_t ik = min(max(i, (int64_t)0), s.N - 1);
    const int m = s.m;
    IncOps o;
    o.ai = T[iu + m - 1];
    o.bi = T[iu - 1];
    o.aj = T[j + m - 1];
    o.bj = T[j - 1];
    if (KIND == ACAMP) {
        const gptr<double> mu = as_global(s.mu);
        o.mi = mu[iu];
        o.mi1 = mu[iu - 1];
        o.mj = mu[j];
        o.mj1 = mu[j - 1];
        o.ni = as_global(s.invn)[ik];
        o.nj = as_global(s.invn)[j];
        o.ci = as_global(s.isconst)[ik] != 0;
        o.cj = as_global(s.isconst)[j] != 0;
    }
    return o;
}

// Update from (i - 1, j - 1) to (i, j).
template <int KIND, int PC>
__device__ __forceinline__ double inc_update(const IncOps &o, double p)
{
    if (KIND == AAMP) return fma(o.ai - o.aj, o.ai - o.aj, -(o.bi - o.bj) * (o.bi - o.bj));
    if (KIND == PNORM) return pn_term<PC>(o.ai - o.aj, p) - pn_term<PC>(o.bi - o.bj, p);
    const double dfi = 0.5 * (o.ai - o.bi), dfj = 0.5 * (o.aj - o.bj);
    const double dgi = (o.ai - o.mi) + (o.bi - o.mi1);
    const double dgj = (o.aj - o.mj) + (o.bj - o.mj1);
    return fma(dfi, dgj, dfj * dgi);
}

template <int KIND, int PC>
__device__ __forceinline__ double inc_step(const IncState &s, int64_t i, int64_t j)
{
    return inc_update<KIND, PC>(inc_load<KIND>(s, i, j), s.p);
}

// Column-walk steps whose operands are loaded together before any is used.
constexpr int INC_BATCH = 4;

// x combined with its DPP-moved copy (ctrl, row mask); lanes outside the row
// mask, and lanes without a source, keep x.
template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned long long dpp_min_u64(unsigned long long x)
{
    const int lo = __builtin_amdgcn_update_dpp((int)(uint32_t)x, (int)(uint32_t)x, CTRL, ROWS,
                                               0xF, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(uint32_t)(x >> 32), (int)(uint32_t)(x >> 32),
                                               CTRL, ROWS, 0xF, false);
    const unsigned long long y = ((unsigned long long)(uint32_t)hi << 32) | (uint32_t)lo;
    return y < x ? y : x;
}

// Smallest key over the 64 lanes of the wave, in lane 63 (every lane takes
// part): within each row of 16 lanes by quad swaps and the half-row and row
// mirrors, then across rows by the row broadcasts of lanes 15 and 31.
__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long x)
{
    x = dpp_min_u64<0xB1, 0xF>(x);     // quad_perm [1,0,3,2]
    x = dpp_min_u64<0x4E, 0xF>(x);     // quad_perm [2,3,0,1]
    x = dpp_min_u64<0x141, 0xF>(x);    // row_half_mirror
    x = dpp_min_u64<0x140, 0xF>(x);    // row_mirror
    x = dpp_min_u64<0x142, 0xA>(x);    // row_bcast:15 into rows 1 and 3
    x = dpp_min_u64<0x143, 0xC>(x);    // row_bcast:31 into rows 2 and 3
    return x;
}

// The row key of lane l - 1 moves to lane l (lane 0 receives none).
__device__ __forceinline__ unsigned long long shift_up_none(unsigned long long x)
{
    const int lo = __builtin_amdgcn_update_dpp((int)0xFFFFFFFF, (int)(uint32_t)x, 0x138, 0xF, 0xF,
                                               false);
    const int hi = __builtin_amdgcn_update_dpp((int)0xFFFFFFFF, (int)(uint32_t)(x >> 32), 0x138,
                                               0xF, 0xF, false);      // 0x138: wave_shr:1
    return ((unsigned long long)(uint32_t)hi << 32) | (uint32_t)lo;
}

// Row r's key takes a candidate. Nothing waits for the old key: an old row
// whose key improved is found afterwards by its index (k_inc_rescore).
__device__ __forceinline__ void flush_row(const IncState &s, int64_t r, unsigned long long key)
{
    atomicMin(&s.keys[r], key);
}

// Diagonal k = excl + thread, over the chunk's new columns [w0, w1]. All
// threads step through the columns together (column j = w0 + t at step t); a
// diagonal joins at its first new column with a row (j = max(k, w0)).
// Rows: lane l of a wave holds row w0 + t - k at step t, which lane l + 1
// holds at step t + 1, so each lane keeps a running row key that moves one
// lane up per step; the key leaving lane 63 is final for this wave and takes
// one atomic. Columns: the column's key is the same for the whole grid at a
// step; it takes the minimum over the wave, then over the block in LDS, and
// the block adds one global atomic per column at the end.
template <int KIND, int PC>
__global__ void __launch_bounds__(INC_BLOCK) k_inc_columns(IncState s, int64_t w0, int64_t w1,
                                                           int32_t refresh)
{
    __shared__ unsigned long long colk[INC_COLS];
    const int64_t steps = w1 - w0 + 1;           // <= INC_COLS, checked by the host
    for (int64_t t = threadIdx.x; t < steps; t += INC_BLOCK) colk[t] = KEY_NONE;

    const int64_t k = (int64_t)s.excl + (int64_t)blockIdx.x * INC_BLOCK + threadIdx.x;
    const bool mine = k <= w1;                    // a diagonal of the chunk
    const unsigned long long mask = (1ull << s.gb) - 1ull;
    const int64_t js = k > w0 ? k : w0;          // first new column with row >= 0
    // The start of every diagonal, taken before the walk so that the lanes
    // of a wave compute theirs together.
    double S = 0.0;
    if (mine) {
        const int64_t i = js - k;
        if (!refresh && js == w0 && i >= 1)
            S = s.col_old[i - 1] + inc_step<KIND, PC>(s, i, js);
        else
            S = inc_start<KIND, PC>(s, i, js);
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    unsigned long long kr = KEY_NONE;             // key of row w0 + t - k
    // One step (column j = w0 + t, operands o); the last step of the chunk
    // keeps its row keys for the final flush.
    auto walk_step = [&](int64_t t, const IncOps &o, bool last) {
        const int64_t j = w0 + t;
        const int64_t i = j - k;
        unsigned long long kc = KEY_NONE;
        if (mine && j >= js) {
            if (j > js) S += inc_update<KIND, PC>(o, s.p);
            bool ok = true;
            double v = S;
            if (KIND == ACAMP) {
                ok = !o.ci && !o.cj;
                v = fma(S * o.ni, -o.nj, 1.0);     // 1 - rho
            }
            if (ok) {
                const unsigned long long ki = pack_key(v, (unsigned long long)j, mask);
                kr = ki < kr ? ki : kr;
                kc = pack_key(v, (unsigned long long)i, mask);
            }
        }
        kc = wave_min_u64(kc);
        if (lane == 63 && kc != KEY_NONE) atomicMin(&colk[t], kc);
        if (!last) {
            if (lane == 63 && kr != KEY_NONE) flush_row(s, i, kr);
            kr = shift_up_none(kr);
        }
    };
    // batches of INC_BATCH steps before the last one, their operands loaded
    // first; then the rest one by one
    constexpr int U = INC_BATCH;
    const int64_t full = (steps - 1) / U * U;
    int64_t t0 = 0;
    for (; t0 < full; t0 += U) {
        IncOps op[U];
#pragma unroll
        for (int u = 0; u < U; ++u) op[u] = inc_load<KIND>(s, w0 + t0 + u - k, w0 + t0 + u);
#pragma unroll
        for (int u = 0; u < U; ++u) walk_step(t0 + u, op[u], false);
    }
    for (; t0 < steps; ++t0) walk_step(t0, inc_load<KIND>(s, w0 + t0 - k, w0 + t0), t0 + 1 == steps);
    // the rows still held: lane l holds row w1 - k
    if (kr != KEY_NONE) flush_row(s, w1 - k, kr);
    if (mine) s.col_new[w1 - k] = S;
    __syncthreads();
    for (int64_t t = threadIdx.x; t < steps; t += INC_BLOCK) {
        const unsigned long long kc = colk[t];
        if (kc != KEY_NONE) atomicMin(&s.keys[w0 + t], kc);
    }
}

// Rows [0, w1]: every new window, and every old row whose key improved, take
// the exact FP64 distance of their winner. Each pair is visited once, so an
// old row's key improved exactly when its index is no longer the stored I.
template <int KIND, int PC>
__global__ void k_inc_rescore(IncState s, int64_t w0, int64_t w1)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r > w1) return;
    const unsigned long long key = s.keys[r];
    const unsigned long long mask = (1ull << s.gb) - 1ull;
    if (r < w0 && (key == KEY_NONE || (int64_t)(key & mask) == s.I[r])) return;
    if (key == KEY_NONE || (KIND == ACAMP && s.isconst[r])) {
        s.P[r] = __longlong_as_double(0x7FF0000000000000ll);
        s.I[r] = -1;
        return;
    }
    const int64_t j = (int64_t)(key & mask);
    const Series v = inc_series(s);
    s.P[r] = root_of<KIND, PC>(exact_sum<KIND, PC>(v, r, j), s.p);
    s.I[r] = j;
}

// After a one-shot profile of the whole series: keys from (P, I) and the last
// column directly.
template <int KIND, int PC>
__global__ void k_inc_rebuild(IncState s)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= s.N) return;
    const unsigned long long mask = (1ull << s.gb) - 1ull;
    const int64_t j = s.I[r];
    if (j < 0) {
        s.keys[r] = KEY_NONE;
    } else {
        const double P = s.P[r];
        double v;
        if (KIND == ACAMP) v = P * P / (2.0 * (double)s.m);
        else if (KIND == AAMP) v = P * P;
        else v = (PC == P_ONE) ? P : (PC == P_THREE ? P * P * P : pow(P, s.p));
        s.keys[r] = pack_key(v, (unsigned long long)j, mask);
    }
    const int64_t w = s.N - 1;
    if (w - r >= s.excl) s.col_new[r] = inc_start<KIND, PC>(s, r, w);
}

template <int KIND, int PC>
static hipError_t launch_chunk(const IncState &s, int64_t w0, int64_t w1, bool refresh,
                               hipStream_t st)
{
    const int B = 256;
    hipLaunchKernelGGL(k_inc_stats, dim3((unsigned)((w1 - w0 + STATS_WAVES) / STATS_WAVES)),
                       dim3(64 * STATS_WAVES), 0, st, s, w0, w1);
    if (w1 >= s.excl) {
        const int64_t nd = w1 - s.excl + 1;
        if (w1 - w0 + 1 > INC_COLS) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_inc_columns<KIND, PC>),
                           dim3((unsigned)((nd + INC_BLOCK - 1) / INC_BLOCK)), dim3(INC_BLOCK), 0,
                           st, s, w0, w1, (int32_t)(refresh ? 1 : 0));
    }
    hipLaunchKernelGGL((k_inc_rescore<KIND, PC>), dim3((unsigned)((w1 + B) / B)), dim3(B), 0, st,
                       s, w0, w1);
    return hipGetLastError();
}

template <int KIND, int PC>
static hipError_t launch_rebuild(const IncState &s, hipStream_t st)
{
    const int B = 256;
    if (s.N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_inc_stats, dim3((unsigned)((s.N + STATS_WAVES - 1) / STATS_WAVES)),
                       dim3(64 * STATS_WAVES), 0, st, s, (int64_t)0, s.N - 1);
    hipLaunchKernelGGL((k_inc_rebuild<KIND, PC>), dim3((unsigned)((s.N + B - 1) / B)), dim3(B), 0,
                       st, s);
    return hipGetLastError();
}

}  // namespace mpk

using namespace mpk;

// Host state of one incremental profile.
struct mp_inc {
    int32_t m, kind, pclass, excl, refresh;
    double p;
    int64_t capacity;            // samples
    int64_t n = 0;               // samples so far
    int64_t since_refresh = 0;   // windows added since the last exact restart
    int32_t gb;
    double *T = nullptr, *P = nullptr, *mu = nullptr, *invn = nullptr;
    double *col[2] = {nullptr, nullptr};
    int cur = 0;                 // col[cur] holds the last column
    int64_t *I = nullptr;
    unsigned long long *keys = nullptr;
    uint8_t *isconst = nullptr;
    std::mutex mu_lock;
};

namespace {

int32_t inc_index_bits(int64_t N)
{
    int32_t b = 1;
    while (b < 40 && ((int64_t)1 << b) <= N) ++b;
    return b;
}

IncState view(mp_inc *h, int64_t N)
{
    IncState s;
    s.T = h->T;
    s.P = h->P;
    s.I = h->I;
    s.keys = h->keys;
    s.mu = h->mu;
    s.invn = h->invn;
    s.isconst = h->isconst;
    s.col_old = h->col[h->cur];
    s.col_new = h->col[1 - h->cur];
    s.N = N;
    s.m = h->m;
    s.kind = h->kind;
    s.pclass = h->pclass;
    s.excl = h->excl;
    s.p = h->p;
    s.gb = h->gb;
    s.pad0 = 0;
    return s;
}

template <class F>
hipError_t dispatch(int32_t kind, int32_t pclass, F &&f)
{
    switch (sel_of(kind, pclass)) {
    case SEL_AAMP: return f(std::integral_constant<int, AAMP>(), std::integral_constant<int, P_TWO>());
    case SEL_ACAMP: return f(std::integral_constant<int, ACAMP>(), std::integral_constant<int, P_TWO>());
    case SEL_P1: return f(std::integral_constant<int, PNORM>(), std::integral_constant<int, P_ONE>());
    case SEL_P3: return f(std::integral_constant<int, PNORM>(), std::integral_constant<int, P_THREE>());
    default: return f(std::integral_constant<int, PNORM>(), std::integral_constant<int, P_GENERIC>());
    }
}

void free_inc(mp_inc *h)
{
    void *ptrs[] = {h->T, h->P, h->mu, h->invn, h->col[0], h->col[1], h->I, h->keys, h->isconst};
    for (void *q : ptrs) hipFree(q);
}

template <class T>
int inc_alloc(T **p, int64_t count)
{
    if (alloc_fail_hook()) return report_error(MP_ENOMEM, "incremental profile buffers");
    hipError_t e = hipMalloc((void **)p, (size_t)std::max<int64_t>(count, 1) * sizeof(T));
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
        (void)hipGetLastError();
        return report_error(MP_ENOMEM, "incremental profile buffers");
    }
    if (e != hipSuccess) return report_hip(e, "incremental profile buffers");
    return MP_OK;
}

}  // namespace

extern "C" {

int mp_inc_create(int32_t m, int32_t kind, double p, int32_t excl, int64_t capacity,
                  int32_t refresh, mp_inc **out)
{
    if (!out) return report_error(MP_EINVAL, "null pointer argument");
    *out = nullptr;
    if (m < 1) return report_error(MP_EINVAL, "m must be >= 1");
    if (kind < AAMP || kind > ACAMP) return report_error(MP_EINVAL, "kind must be MP_KIND_*");
    if (kind == PNORM && !(std::isfinite(p) && p >= 1.0))
        return report_error(MP_EINVAL, "p must be finite and >= 1");
    if (capacity < m || capacity >= MP_MAX_N)
        return report_error(MP_EINVAL, "capacity must satisfy m <= capacity < 2^31");
    if (refresh < 0) return report_error(MP_EINVAL, "refresh must be >= 0");
    mp_inc *h = new (std::nothrow) mp_inc;
    if (!h) return report_error(MP_ENOMEM, "incremental profile handle");
    h->m = m;
    h->kind = (kind == PNORM && p == 2.0) ? AAMP : kind;
    h->p = h->kind == PNORM ? p : 2.0;
    h->pclass = h->kind != PNORM ? P_TWO : (p == 1.0 ? P_ONE : (p == 3.0 ? P_THREE : P_GENERIC));
    h->excl = excl > 0 ? excl : (m + 3) / 4;
    h->refresh = refresh > 0 ? refresh : 4096;
    h->capacity = capacity;
    const int64_t W = capacity - m + 1;
    h->gb = inc_index_bits(W);
    int rc;
    if ((rc = inc_alloc(&h->T, capacity)) || (rc = inc_alloc(&h->P, W)) ||
        (rc = inc_alloc(&h->I, W)) || (rc = inc_alloc(&h->keys, W)) ||
        (rc = inc_alloc(&h->mu, W)) || (rc = inc_alloc(&h->invn, W)) ||
        (rc = inc_alloc(&h->isconst, W)) ||
        (rc = inc_alloc(&h->col[0], W)) || (rc = inc_alloc(&h->col[1], W))) {
        free_inc(h);
        delete h;
        return rc;
    }
    *out = h;
    report_ok();
    return MP_OK;
}

int mp_inc_append(mp_inc *h, const double *T, int64_t count, void *stream)
{
    if (!h || (!T && count > 0)) return report_error(MP_EINVAL, "null pointer argument");
    if (count < 0) return report_error(MP_EINVAL, "count must be >= 0");
    std::lock_guard<std::mutex> lk(h->mu_lock);
    if (count > h->capacity - h->n) return report_error(MP_EINVAL, "append exceeds the capacity");
    if (count == 0) {
        report_ok();
        return MP_OK;
    }
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(h->T + h->n, T, (size_t)count * sizeof(double),
                                  hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return report_hip(e, "hipMemcpyAsync");
    const int64_t n_old = h->n, n_new = h->n + count;
    h->n = n_new;
    if (n_new < h->m) {
        report_ok();
        return MP_OK;
    }
    const int64_t N_old = n_old >= h->m ? n_old - h->m + 1 : 0;
    const int64_t N_new = n_new - h->m + 1;
    const int64_t added = N_new - N_old;
    if (N_old == 0 || added > std::max<int64_t>(INC_COLS, N_old / 8)) {
        // one-shot profile of the whole series, then rebuild the state
        int rc = profile_once(h->T, n_new, h->m, h->kind, h->p, h->excl, 4096, h->P, h->I, st);
        if (rc) return rc;
        const IncState s = view(h, N_new);
        e = dispatch(h->kind, h->pclass, [&](auto K, auto PC) {
            return launch_rebuild<decltype(K)::value, decltype(PC)::value>(s, st);
        });
        if (e != hipSuccess) return report_hip(e, "incremental rebuild launch");
        h->cur = 1 - h->cur;             // the rebuilt last column is in col_new
        h->since_refresh = 0;
        report_ok();
        return MP_OK;
    }
    int64_t w0 = N_old;
    while (w0 < N_new) {
        const bool restart = h->since_refresh == 0;
        const int64_t len = std::min<int64_t>(
            {N_new - w0, INC_COLS, (int64_t)h->refresh - h->since_refresh});
        const int64_t w1 = w0 + len - 1;
        const IncState s = view(h, w1 + 1);
        e = dispatch(h->kind, h->pclass, [&](auto K, auto PC) {
            return launch_chunk<decltype(K)::value, decltype(PC)::value>(s, w0, w1, restart, st);
        });
        if (e != hipSuccess) return report_hip(e, "incremental launch");
        h->cur = 1 - h->cur;
        h->since_refresh += len;
        if (h->since_refresh >= h->refresh) h->since_refresh = 0;
        w0 = w1 + 1;
    }
    report_ok();
    return MP_OK;
}

int mp_inc_state(mp_inc *h, int64_t *n, int64_t *N, double **P, int64_t **I)
{
    if (!h) return report_error(MP_EINVAL, "null pointer argument");
    std::lock_guard<std::mutex> lk(h->mu_lock);
    if (n) *n = h->n;
    if (N) *N = h->n >= h->m ? h->n - h->m + 1 : 0;
    if (P) *P = h->P;
    if (I) *I = h->I;
    report_ok();
    return MP_OK;
}

int mp_inc_read(mp_inc *h, double *P, int64_t *I, void *stream)
{
    if (!h || !P || !I) return report_error(MP_EINVAL, "null pointer argument");
    std::lock_guard<std::mutex> lk(h->mu_lock);
    const int64_t N = h->n >= h->m ? h->n - h->m + 1 : 0;
    if (N > 0) {
        hipStream_t st = (hipStream_t)stream;
        hipError_t e = hipMemcpyAsync(P, h->P, (size_t)N * sizeof(double), hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(I, h->I, (size_t)N * sizeof(int64_t), hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return report_hip(e, "hipMemcpyAsync");
    }
    report_ok();
    return MP_OK;
}

void mp_inc_destroy(mp_inc *h)
{
    if (!h) return;
    (void)hipDeviceSynchronize();
    free_inc(h);
    delete h;
}

}  // extern "C"
