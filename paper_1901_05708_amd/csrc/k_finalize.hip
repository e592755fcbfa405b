// k_finalize.hip -- turn the packed keys into the profile (Algorithm 2's final
// square-root loop, generalised): decode the winning index of every row,
// recompute that one pair's distance directly in FP64, take the root. Rows
// whose winner is not a legal candidate (z-normalized: a constant window, or a
// row whose every candidate is anti-correlated) are queued and recomputed
// exactly by k_fallback.
#include "keys.h"
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
__device__ double exact_sum(const Series &s, int64_t i, int64_t j)
{
    const double *a = s.T + i;
    const double *b = s.T + j;
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
    if (s.kind == ACAMP && s.isconst[j]) return false;
    return true;
}

template <int KIND, int PC>
__global__ void k_finalize(Series s, Fallback fb, double *P, int64_t *I)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= s.N) return;
    const unsigned long long mask = (1ull << s.gb) - 1ull;
    const unsigned long long key = s.keys[i];
    if ((KIND == ACAMP && s.isconst[i]) || key == KEY_NONE) {
        P[i] = __longlong_as_double(0x7FF0000000000000ll);
        I[i] = -1;
        return;
    }
    const int64_t j = (int64_t)(key & mask);
    if (!legal_pair(s, i, j)) {
        int pos = atomicAdd(fb.count, 1);
        if (pos < fb.capacity) fb.rows[pos] = (int32_t)i;
        return;
    }
    P[i] = root_of<KIND, PC>(exact_sum<KIND, PC>(s, i, j), s.p);
    I[i] = j;
}

// Exact row minimum for queued rows: one block per row, every admissible
// legal column summed directly (the brute force of the definition), ties to
// the smallest index.
template <int KIND, int PC>
__global__ void __launch_bounds__(256) k_fallback(Series s, Fallback fb, double *P, int64_t *I)
{
    __shared__ double rv[256];
    __shared__ int64_t rj[256];
    const int cnt = min(*fb.count, fb.capacity);
    for (int r = blockIdx.x; r < cnt; r += gridDim.x) {
        const int64_t i = fb.rows[r];
        double bv = __longlong_as_double(0x7FF0000000000000ll);
        int64_t bj = -1;
        for (int64_t j = threadIdx.x; j < s.N; j += blockDim.x) {
            if (!legal_pair(s, i, j)) continue;
            double v = exact_sum<KIND, PC>(s, i, j);
            if (v < bv) {   // j ascends within a thread: strict '<' keeps the smallest
                bv = v;
                bj = j;
            }
        }
        rv[threadIdx.x] = bv;
        rj[threadIdx.x] = bj;
        __syncthreads();
        for (int w = blockDim.x / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) {
                double ov = rv[threadIdx.x + w];
                int64_t oj = rj[threadIdx.x + w];
                double mv = rv[threadIdx.x];
                int64_t mj = rj[threadIdx.x];
                if (oj >= 0 && (mj < 0 || ov < mv || (ov == mv && oj < mj))) {
                    rv[threadIdx.x] = ov;
                    rj[threadIdx.x] = oj;
                }
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            const int64_t j = rj[0];
            if (j < 0) {
                P[i] = __longlong_as_double(0x7FF0000000000000ll);
                I[i] = -1;
            } else {
                P[i] = root_of<KIND, PC>(rv[0], s.p);
                I[i] = j;
            }
        }
        __syncthreads();
    }
}

hipError_t launch_finalize(const Series &s, const Fallback &fb, double *P, int64_t *I,
                           hipStream_t st)
{
    const int B = 256;
    dim3 g((unsigned)((s.N + B - 1) / B));
    if (s.kind == AAMP)
        hipLaunchKernelGGL((k_finalize<AAMP, P_TWO>), g, dim3(B), 0, st, s, fb, P, I);
    else if (s.kind == ACAMP)
        hipLaunchKernelGGL((k_finalize<ACAMP, P_TWO>), g, dim3(B), 0, st, s, fb, P, I);
    else if (s.pclass == P_ONE)
        hipLaunchKernelGGL((k_finalize<PNORM, P_ONE>), g, dim3(B), 0, st, s, fb, P, I);
    else if (s.pclass == P_THREE)
        hipLaunchKernelGGL((k_finalize<PNORM, P_THREE>), g, dim3(B), 0, st, s, fb, P, I);
    else
        hipLaunchKernelGGL((k_finalize<PNORM, P_GENERIC>), g, dim3(B), 0, st, s, fb, P, I);
    return hipGetLastError();
}

hipError_t launch_fallback(const Series &s, const Fallback &fb, double *P, int64_t *I,
                           hipStream_t st)
{
    dim3 g(256), b(256);
    if (s.kind == AAMP)
        hipLaunchKernelGGL((k_fallback<AAMP, P_TWO>), g, b, 0, st, s, fb, P, I);
    else if (s.kind == ACAMP)
        hipLaunchKernelGGL((k_fallback<ACAMP, P_TWO>), g, b, 0, st, s, fb, P, I);
    else if (s.pclass == P_ONE)
        hipLaunchKernelGGL((k_fallback<PNORM, P_ONE>), g, b, 0, st, s, fb, P, I);
    else if (s.pclass == P_THREE)
        hipLaunchKernelGGL((k_fallback<PNORM, P_THREE>), g, b, 0, st, s, fb, P, I);
    else
        hipLaunchKernelGGL((k_fallback<PNORM, P_GENERIC>), g, b, 0, st, s, fb, P, I);
    return hipGetLastError();
}

}  // namespace mpk
