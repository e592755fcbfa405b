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

// Exact pre-root distance of one pair, straight from Defs. 2.5-2.7:
// sum of squares (AAMP), of p-th powers (p-norm), or DZ^2 (ACAMP, written
// with invn = sqrt(m) / (sqrt(m) sigma) so that z = sqrt(m) (t - mu) invn).
template <int KIND, int PC>
__device__ inline double exact_sum(const Series &s, int64_t i, int64_t j)
{
    const gptr<double> a = as_global(s.T) + i;
    const gptr<double> b = as_global(s.T) + j;
    const int m = s.m;
    double acc = 0.0;
    if (KIND == ACAMP) {
        const double mi = s.mu[i], mj = s.mu[j], ni = s.invn[i], nj = s.invn[j];
        for (int l = 0; l < m; ++l) {
            double d = (a[l] - mi) * ni - (b[l] - mj) * nj;
            acc = fma(d, d, acc);
        }
        return acc * (double)m;
    }
    if (KIND == AAMP) {
        for (int l = 0; l < m; ++l) {
            double d = a[l] - b[l];
            acc = fma(d, d, acc);
        }
        return acc;
    }
    for (int l = 0; l < m; ++l) acc += pn_term<PC>(a[l] - b[l], s.p);
    return acc;
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
