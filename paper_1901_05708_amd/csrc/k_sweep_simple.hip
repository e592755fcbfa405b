// k_sweep_simple.hip -- the diagonal sweep at its simplest: one thread per
// (diagonal, row segment), every pair merged into the global keys with two
// 64-bit atomicMin. Used for small series, where the band kernel's
// 64 x diagonals-per-lane wide bands would leave most of the GPU idle.
//
// Per diagonal k = j - i the first pair of a segment is summed directly
// (the exact FP64 restart), every later pair is the O(1) update of
// Lemma 1 / Lemma 2 / the centred form of Lemma 3, and each pair updates both
// its row i and its column j (Algorithms 1-3).
#include "keys.h"
#include "mp_internal.h"

namespace mpk {

template <int PC>
__device__ __forceinline__ double pnorm_term(double d, double p)
{
    double a = fabs(d);
    if (PC == P_ONE) return a;
    if (PC == P_THREE) return a * a * a;
    return pow(a, p);
}

template <int KIND, int PC>
__global__ void k_sweep_simple(Series s, int32_t R)
{
    const int64_t k = (int64_t)s.excl + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= s.N) return;
    const int64_t i0 = (int64_t)blockIdx.y * R;
    const int64_t iend = min(i0 + (int64_t)R, s.N - k);
    if (i0 >= iend) return;
    const unsigned long long mask = (1ull << s.gb) - 1ull;
    const int m = s.m;
    const double *ti = s.T + i0;
    const double *tj = s.T + i0 + k;

    // exact start of the segment
    double S = 0.0;
    if (KIND == ACAMP) {
        const double mi = s.mu[i0], mj = s.mu[i0 + k];
        for (int l = 0; l < m; ++l) S = fma(ti[l] - mi, tj[l] - mj, S);
    } else if (KIND == AAMP) {
        for (int l = 0; l < m; ++l) {
            double d = ti[l] - tj[l];
            S = fma(d, d, S);
        }
    } else {
        for (int l = 0; l < m; ++l) S += pnorm_term<PC>(ti[l] - tj[l], s.p);
    }

    for (int64_t i = i0; i < iend; ++i) {
        const int64_t j = i + k;
        if (i > i0) {
            if (KIND == AAMP) {
                S = fma(s.x[i] - s.x[j], s.y[i] - s.y[j], S);
            } else if (KIND == PNORM) {
                S += pnorm_term<PC>(s.x[i] - s.x[j], s.p) - pnorm_term<PC>(s.y[i] - s.y[j], s.p);
            } else {
                S = fma(s.x[i], s.y[j], S);
                S = fma(s.x[j], s.y[i], S);
            }
        }
        double v;
        if (KIND == ACAMP) {
            if (s.isconst[i] || s.isconst[j]) continue;
            v = 1.0 - S * s.invn[i] * s.invn[j];
        } else {
            v = S;
        }
        atomicMin(&s.keys[i], pack_key(v, (unsigned long long)j, mask));
        atomicMin(&s.keys[j], pack_key(v, (unsigned long long)i, mask));
    }
}

hipError_t launch_sweep_simple(const Series &s, int32_t R, hipStream_t st)
{
    const int64_t ndiag = s.N - s.excl;
    if (ndiag <= 0) return hipSuccess;
    const int B = 256;
    const int64_t nseg = (ndiag + R - 1) / R;
    dim3 grid((unsigned)((ndiag + B - 1) / B), (unsigned)nseg);
    if (s.kind == AAMP) {
        hipLaunchKernelGGL((k_sweep_simple<AAMP, P_TWO>), grid, dim3(B), 0, st, s, R);
    } else if (s.kind == ACAMP) {
        hipLaunchKernelGGL((k_sweep_simple<ACAMP, P_TWO>), grid, dim3(B), 0, st, s, R);
    } else if (s.pclass == P_ONE) {
        hipLaunchKernelGGL((k_sweep_simple<PNORM, P_ONE>), grid, dim3(B), 0, st, s, R);
    } else if (s.pclass == P_THREE) {
        hipLaunchKernelGGL((k_sweep_simple<PNORM, P_THREE>), grid, dim3(B), 0, st, s, R);
    } else {
        hipLaunchKernelGGL((k_sweep_simple<PNORM, P_GENERIC>), grid, dim3(B), 0, st, s, R);
    }
    return hipGetLastError();
}

}  // namespace mpk
