// exact.h -- the exact FP64 distance of one pair, straight from the
// definitions, and the helpers around it: shared by the rescoring / exact
// search (k_finalize.hip) and the incremental profile (k_incremental.hip).
#pragma once

#include "mp_internal.h"

namespace mpk {

template <int PC>
__device__ __forceinline__ double pn_term(double d, double p)
{
    double a = fabs(d);
    if (PC == P_ONE) return a;
    if (PC == P_TWO) return a * a;
    if (PC == P_THREE) return a * a * a;
    return pow(a, p);
}

// Calls f(a[l], b[l]) for l = 0 .. m-1 in order. Samples are loaded U at a
// time and the loads of the next block are issued before the current block is
// consumed, so a thread keeps 2U loads in flight instead of waiting on every
// sample.
template <int U, typename Fn>
__device__ __forceinline__ void visit_pairs(gptr<double> a, gptr<double> b, int m, Fn f)
{
    double a0[U], b0[U], a1[U], b1[U];
    auto load = [&](double (&x)[U], double (&y)[U], int l) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            x[u] = a[l + u];
            y[u] = b[l + u];
        }
    };
    auto run = [&](const double (&x)[U], const double (&y)[U]) {
#pragma unroll
        for (int u = 0; u < U; ++u) f(x[u], y[u]);
    };
    const int nb = m / U;
    if (nb > 0) load(a0, b0, 0);
    for (int k = 0; k < nb; k += 2) {
        if (k + 1 < nb) load(a1, b1, (k + 1) * U);
        run(a0, b0);
        if (k + 1 >= nb) break;
        if (k + 2 < nb) load(a0, b0, (k + 2) * U);
        run(a1, b1);
    }
    for (int l = nb * U; l < m; ++l) f(a[l], b[l]);
}

// One term of the exact sums: the squared difference of the z-normalized
// samples (times 1/m), the squared difference, or |difference|^p.
template <int KIND, int PC>
__device__ __forceinline__ double exact_term(double x, double y, double mi, double ni, double mj,
                                             double nj, double p, double acc)
{
    if (KIND == ACAMP) {
        const double d = (x - mi) * ni - (y - mj) * nj;
        return fma(d, d, acc);
    }
    if (KIND == AAMP) {
        const double d = x - y;
        return fma(d, d, acc);
    }
    return acc + pn_term<PC>(x - y, p);
}

// Exact pre-root distance of one pair, straight from Defs. 2.5-2.7:
// sum of squares (AAMP), of p-th powers (p-norm), or DZ^2 (ACAMP, written
// with invn = sqrt(m) / (sqrt(m) sigma) so that z = sqrt(m) (t - mu) invn).
// Terms are summed in order of l.
template <int KIND, int PC>
__device__ inline double exact_sum(const Series &s, int64_t i, int64_t j)
{
    const gptr<double> a = as_global(s.T) + i;
    const gptr<double> b = as_global(s.T) + j;
    const int m = s.m;
    double acc = 0.0;
    const double p = s.p;
    double mi = 0.0, mj = 0.0, ni = 0.0, nj = 0.0;
    if (KIND == ACAMP) {
        mi = s.mu[i];
        mj = s.mu[j];
        ni = s.invn[i];
        nj = s.invn[j];
    }
    visit_pairs<8>(a, b, m, [&](double x, double y) {
        acc = exact_term<KIND, PC>(x, y, mi, ni, mj, nj, p, acc);
    });
    return (KIND == ACAMP) ? acc * (double)m : acc;
}

template <int KIND, int PC>
__device__ __forceinline__ double root_of(double S, double p)
{
    if (KIND == PNORM) {
        if (PC == P_ONE) return S;
        if (PC == P_TWO) return sqrt(S);
        return pow(S, 1.0 / p);
    }
    return sqrt(fmax(S, 0.0));
}

__device__ __forceinline__ bool legal_pair(const Series &s, int64_t i, int64_t j)
{
    if (j < 0 || j >= s.N) return false;
    int64_t g = i > j ? i - j : j - i;
    if (g < s.excl) return false;
    if (s.kind == ACAMP && as_global(s.isconst)[j]) return false;
    return true;
}

}  // namespace mpk
