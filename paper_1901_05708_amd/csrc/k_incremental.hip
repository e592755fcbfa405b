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
//    that begin inside the chunk, from an exact FP64 sum; rows whose packed
//    key improves are flagged. All threads take the same column at a step,
//    so its key is reduced over the wave before its one atomic.
//  * k_inc_rescore: flagged rows and the new windows take their exact FP64
//    distance (as the one-shot path does).
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
    uint8_t *dirty;
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

// Window statistics of windows [w0, w1] (two passes, mean around the first
// sample), key reset and cleared flags.
__global__ void k_inc_stats(IncState s, int64_t w0, int64_t w1)
{
    const int64_t w = w0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w > w1) return;
    s.keys[w] = KEY_NONE;
    s.dirty[w] = 0;
    if (s.kind != ACAMP) return;
    const gptr<double> x = as_global(s.T) + w;
    const int m = s.m;
    const double x0 = x[0];
    double sum = 0.0;
    bool same = true;
    visit_window<8>(x, m, [&](double v) {
        sum += v - x0;
        same = same && (v == x0);
    });
    const double mu = x0 + sum / (double)m;
    double ss = 0.0;
    visit_window<8>(x, m, [&](double v) {
        const double d = v - mu;
        ss = fma(d, d, ss);
    });
    s.mu[w] = mu;
    s.isconst[w] = same ? 1 : 0;
    s.invn[w] = (same || !(ss > 0.0)) ? 0.0 : 1.0 / sqrt(ss);
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

// Update from (i - 1, j - 1) to (i, j).
template <int KIND, int PC>
__device__ __forceinline__ double inc_step(const IncState &s, int64_t i, int64_t j)
{
    const gptr<double> T = as_global(s.T);
    const int m = s.m;
    const double ai = T[i + m - 1], aj = T[j + m - 1], bi = T[i - 1], bj = T[j - 1];
    if (KIND == AAMP) return fma(ai - aj, ai - aj, -(bi - bj) * (bi - bj));
    if (KIND == PNORM) return pn_term<PC>(ai - aj, s.p) - pn_term<PC>(bi - bj, s.p);
    const double dfi = 0.5 * (ai - bi), dfj = 0.5 * (aj - bj);
    const double dgi = (ai - s.mu[i]) + (bi - s.mu[i - 1]);
    const double dgj = (aj - s.mu[j]) + (bj - s.mu[j - 1]);
    return fma(dfi, dgj, dfj * dgi);
}

// Smallest key over the 64 lanes of the wave (every lane takes part).
__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long x)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long y = __shfl_xor(x, off, 64);
        x = y < x ? y : x;
    }
    return x;
}

// Diagonal k = excl + thread, over the chunk's new columns [w0, w1]. All
// threads step through the columns together (column j = w0 + t at step t); a
// diagonal joins at its first new column with a row (j = max(k, w0)). Each
// pair updates its row's key with its own atomic. The column's key is the
// same for the whole grid at a step: it takes the minimum over the wave, then
// over the block in LDS, and the block adds one global atomic per column at
// the end.
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
    for (int64_t t = 0; t < steps; ++t) {
        const int64_t j = w0 + t;
        const int64_t i = j - k;
        unsigned long long kc = KEY_NONE;
        if (mine && j >= js) {
            if (j > js) S += inc_step<KIND, PC>(s, i, j);
            bool ok = true;
            double v = S;
            if (KIND == ACAMP) {
                ok = !s.isconst[i] && !s.isconst[j];
                v = fma(S * s.invn[i], -s.invn[j], 1.0);     // 1 - rho
            }
            if (ok) {
                const unsigned long long ki = pack_key(v, (unsigned long long)j, mask);
                const unsigned long long old = atomicMin(&s.keys[i], ki);
                if (ki < old && i < w0) s.dirty[i] = 1;
                kc = pack_key(v, (unsigned long long)i, mask);
            }
        }
        kc = wave_min_u64(kc);
        if ((threadIdx.x & 63) == 0 && kc != KEY_NONE) atomicMin(&colk[t], kc);
    }
    if (mine) s.col_new[w1 - k] = S;
    __syncthreads();
    for (int64_t t = threadIdx.x; t < steps; t += INC_BLOCK) {
        const unsigned long long kc = colk[t];
        if (kc != KEY_NONE) atomicMin(&s.keys[w0 + t], kc);
    }
}

// Rows [0, w1]: flagged old rows and every new window take the exact FP64
// distance of their winner.
template <int KIND, int PC>
__global__ void k_inc_rescore(IncState s, int64_t w0, int64_t w1)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r > w1) return;
    if (r < w0 && !s.dirty[r]) return;
    s.dirty[r] = 0;
    const unsigned long long key = s.keys[r];
    const unsigned long long mask = (1ull << s.gb) - 1ull;
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
    s.dirty[r] = 0;
    const int64_t w = s.N - 1;
    if (w - r >= s.excl) s.col_new[r] = inc_start<KIND, PC>(s, r, w);
}

template <int KIND, int PC>
static hipError_t launch_chunk(const IncState &s, int64_t w0, int64_t w1, bool refresh,
                               hipStream_t st)
{
    const int B = 256;
    hipLaunchKernelGGL(k_inc_stats, dim3((unsigned)((w1 - w0 + B) / B)), dim3(B), 0, st, s, w0, w1);
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
    hipLaunchKernelGGL(k_inc_stats, dim3((unsigned)((s.N + B - 1) / B)), dim3(B), 0, st, s,
                       (int64_t)0, s.N - 1);
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
    uint8_t *isconst = nullptr, *dirty = nullptr;
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
    s.dirty = h->dirty;
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
    void *ptrs[] = {h->T, h->P, h->mu, h->invn, h->col[0], h->col[1], h->I, h->keys, h->isconst,
                    h->dirty};
    for (void *q : ptrs) hipFree(q);
}

template <class T>
int inc_alloc(T **p, int64_t count)
{
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
        (rc = inc_alloc(&h->isconst, W)) || (rc = inc_alloc(&h->dirty, W)) ||
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
