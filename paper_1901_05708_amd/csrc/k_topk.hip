// k_topk.hip -- motifs and discords from a matrix profile (the two uses of
// the profile named in Sec. 1): greedy extraction of the k smallest (motifs)
// or largest (discords) finite profile values, each followed by an exclusion
// zone so that a match and its trivially shifted neighbours are reported once.
//
// Round r, with every round enqueued back to back on the stream:
//   1. k_topk_extreme: grid-wide min (motifs) or max (discords) of the bit
//      patterns of the finite, not yet excluded values. Non-negative doubles
//      order like their bit patterns, so one 64-bit atomic per block gives
//      the exact extreme.
//   2. k_topk_argext: the smallest index holding exactly that value (a second
//      grid pass and a 64-bit atomicMin), which makes ties deterministic.
//   3. k_topk_commit (one block): record (i, I[i], P[i]) and mark the zone
//      |x - i| < excl (and |x - I[i]| < excl for motifs) as excluded.
// A round that finds no candidate leaves everything unchanged, so rounds
// after exhaustion are no-ops.
#include "mp_internal.h"

namespace mpk {

constexpr unsigned long long TK_NONE_MIN = ~0ull;   // "no candidate" for a minimum
constexpr unsigned long long TK_NONE_MAX = 0ull;    // for a maximum (bits of +0 are 0 too;
                                                    // a found flag disambiguates)

struct TopkState {
    unsigned long long *ext;    // k entries: extreme bit pattern of round r
    unsigned long long *arg;    // k entries: its smallest index
    int32_t *found;             // k entries: 1 if round r had a candidate
    uint8_t *mask;              // N entries: 1 = excluded
    int32_t *count;             // number of rounds with a result
};

__global__ void k_topk_init(TopkState st, int64_t N, int32_t k, int32_t mode)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t x = t; x < N; x += stride) st.mask[x] = 0;
    for (int64_t r = t; r < k; r += stride) {
        st.ext[r] = mode == 0 ? TK_NONE_MIN : TK_NONE_MAX;
        st.arg[r] = TK_NONE_MIN;
        st.found[r] = 0;
    }
    if (t == 0) *st.count = 0;
}

__device__ __forceinline__ bool tk_candidate(const double *P, const uint8_t *mask, int64_t x)
{
    const double v = P[x];
    return !mask[x] && v >= 0.0 && v < __longlong_as_double(0x7FF0000000000000ll);
}

__global__ void __launch_bounds__(256) k_topk_extreme(const double *P, int64_t N, TopkState st,
                                                     int32_t r, int32_t mode)
{
    __shared__ unsigned long long red[4];
    __shared__ int any_s[4];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    unsigned long long best = mode == 0 ? TK_NONE_MIN : TK_NONE_MAX;
    int any = 0;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < N; x += stride) {
        if (!tk_candidate(P, st.mask, x)) continue;
        const unsigned long long b = (unsigned long long)__double_as_longlong(P[x]);
        best = mode == 0 ? (b < best ? b : best) : (b > best ? b : best);
        any = 1;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(best, off);
        best = mode == 0 ? (o < best ? o : best) : (o > best ? o : best);
        any |= __shfl_xor(any, off);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[w] = best;
        any_s[w] = any;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int a = 0;
        for (int q = 0; q < 4; ++q) {
            if (!any_s[q]) continue;
            best = a ? (mode == 0 ? (red[q] < best ? red[q] : best) : (red[q] > best ? red[q] : best))
                     : red[q];
            a = 1;
        }
        if (a) {
            if (mode == 0) atomicMin(&st.ext[r], best);
            else atomicMax(&st.ext[r], best);
            st.found[r] = 1;
        }
    }
}

__global__ void __launch_bounds__(256) k_topk_argext(const double *P, int64_t N, TopkState st,
                                                     int32_t r)
{
    if (!st.found[r]) return;
    const unsigned long long want = st.ext[r];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    unsigned long long best = TK_NONE_MIN;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < N; x += stride) {
        if (tk_candidate(P, st.mask, x) && (unsigned long long)__double_as_longlong(P[x]) == want) {
            best = (unsigned long long)x;
            break;                      // later x of this thread are larger
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(best, off);
        best = o < best ? o : best;
    }
    if ((threadIdx.x & 63) == 0 && best != TK_NONE_MIN) atomicMin(&st.arg[r], best);
}

__global__ void __launch_bounds__(256) k_topk_commit(const double *P, const int64_t *I, int64_t N,
                                                     TopkState st, int32_t r, int32_t excl,
                                                     int32_t mode, int64_t *out_i, int64_t *out_j,
                                                     double *out_d)
{
    if (!st.found[r]) return;
    const int64_t i = (int64_t)st.arg[r];
    const int64_t j = I[i];
    if (threadIdx.x == 0) {
        out_i[r] = i;
        out_j[r] = j;
        out_d[r] = P[i];
        *st.count = r + 1;
    }
    for (int64_t x = max((int64_t)0, i - excl + 1) + threadIdx.x; x < min(N, i + excl);
         x += blockDim.x)
        st.mask[x] = 1;
    if (mode == 0 && j >= 0 && j < N)
        for (int64_t x = max((int64_t)0, j - excl + 1) + threadIdx.x; x < min(N, j + excl);
             x += blockDim.x)
            st.mask[x] = 1;
}

hipError_t launch_topk(const double *P, const int64_t *I, int64_t N, int32_t k, int32_t excl,
                       int32_t mode, int64_t *out_i, int64_t *out_j, double *out_d,
                       int32_t *out_count, unsigned long long *scratch, uint8_t *mask,
                       hipStream_t st)
{
    TopkState s;
    s.ext = scratch;
    s.arg = scratch + k;
    s.found = (int32_t *)(scratch + 2 * (int64_t)k);
    s.mask = mask;
    s.count = out_count;
    const int B = 256;
    const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((N + B - 1) / B, 2048));
    hipLaunchKernelGGL(k_topk_init, dim3(g), dim3(B), 0, st, s, N, k, mode);
    for (int32_t r = 0; r < k; ++r) {
        hipLaunchKernelGGL(k_topk_extreme, dim3(g), dim3(B), 0, st, P, N, s, r, mode);
        hipLaunchKernelGGL(k_topk_argext, dim3(g), dim3(B), 0, st, P, N, s, r);
        hipLaunchKernelGGL(k_topk_commit, dim3(1), dim3(B), 0, st, P, I, N, s, r, excl, mode,
                           out_i, out_j, out_d);
    }
    return hipGetLastError();
}

}  // namespace mpk
