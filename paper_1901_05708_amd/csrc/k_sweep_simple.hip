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
__device__ __forceinline__ void sweep_simple(const Series &s, int32_t R,
                                             unsigned long long *visits)
{
    const int64_t k = (int64_t)s.excl + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= s.N) return;
    const int64_t i0 = (int64_t)blockIdx.y * R;
    const int64_t iend = min(i0 + (int64_t)R, s.N - k);
    if (i0 >= iend) return;
    if (visits) atomicAdd(visits, (unsigned long long)(iend - i0));   // test mode
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

// Grid: x over diagonals, y over row segments, z over jobs; jobs of the band
// kernel (nbands > 0) return at once.
__global__ void k_sweep_simple(Batch b)
{
    const Job J = load_uniform(&b.jobs[blockIdx.z]);
    if (J.nbands > 0) return;
    const Series s = J.s;
    const int32_t R = J.seg_rows;
    switch (sel_of(s.kind, s.pclass)) {
    case SEL_AAMP: sweep_simple<AAMP, P_TWO>(s, R, b.visits); break;
    case SEL_ACAMP: sweep_simple<ACAMP, P_TWO>(s, R, b.visits); break;
    case SEL_P1: sweep_simple<PNORM, P_ONE>(s, R, b.visits); break;
    case SEL_P3: sweep_simple<PNORM, P_THREE>(s, R, b.visits); break;
    default: sweep_simple<PNORM, P_GENERIC>(s, R, b.visits); break;
    }
}

hipError_t launch_sweep_simple(const Batch &b, hipStream_t st)
{
    if (b.simple_diag <= 0 || b.simple_segs <= 0 || b.njobs <= 0) return hipSuccess;
    const int B = 256;
    dim3 grid((unsigned)((b.simple_diag + B - 1) / B), (unsigned)b.simple_segs, (unsigned)b.njobs);
    hipLaunchKernelGGL(k_sweep_simple, grid, dim3(B), 0, st, b);
    return hipGetLastError();
}

}  // namespace mpk
