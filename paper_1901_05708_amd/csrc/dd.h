// dd.h -- double-double arithmetic for the exact sums of long windows.
//
// A value is the unevaluated sum hi + lo of two doubles with |lo| <= ulp(hi)/2,
// about 106 significant bits. Sums use Knuth's error-free two-sum, products
// the fused multiply-add residual of a * b (Dekker's exact product without the
// splitting step). No contraction into fused operations is allowed inside the
// transformations, or their error terms would be lost. Used by the window
// statistics and the rescoring of long windows, where an anchor computed
// exactly is carried to the neighbouring windows by adding what enters and
// subtracting what leaves: in double-double the cancellation of that running
// sum costs about 2^-104 of its largest partial sum instead of 2^-53.
#pragma once

#include <hip/hip_runtime.h>

namespace mpk {

struct DD {
    double hi, lo;
};

__device__ __forceinline__ DD dd_two_sum(double a, double b)
{
#pragma clang fp contract(off)
    const double s = a + b;
    const double bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}

// |a| >= |b| (or a == 0)
__device__ __forceinline__ DD dd_quick(double a, double b)
{
#pragma clang fp contract(off)
    const double s = a + b;
    return {s, b - (s - a)};
}

__device__ __forceinline__ DD dd_add(DD a, DD b)
{
#pragma clang fp contract(off)
    DD s = dd_two_sum(a.hi, b.hi);
    const DD t = dd_two_sum(a.lo, b.lo);
    s = dd_quick(s.hi, s.lo + t.hi);
    return dd_quick(s.hi, s.lo + t.lo);
}

// q += v for a running sum q of many terms: the rounding error of the high
// parts' sum goes to q.lo exactly (two-sum), and v.lo is added to q.lo in
// plain precision. q.lo is not renormalised after each term, so it collects
// the errors of all terms; its own rounding is 2^-53 of that collected error,
// which leaves the sum with an error of order 2^-106 times the sum of the
// terms' magnitudes, as in an ordinary double-double sum (the twice-the-
// working-precision summation of Ogita, Rump and Oishi). dd_norm restores
// |lo| <= ulp(hi) / 2 before q is used as a double-double.
__device__ __forceinline__ void dd_acc(DD &q, DD v)
{
#pragma clang fp contract(off)
    const DD s = dd_two_sum(q.hi, v.hi);
    q.hi = s.hi;
    q.lo += s.lo + v.lo;
}

__device__ __forceinline__ DD dd_norm(DD q) { return dd_two_sum(q.hi, q.lo); }

__device__ __forceinline__ DD dd_neg(DD a) { return {-a.hi, -a.lo}; }

__device__ __forceinline__ DD dd_sub(DD a, DD b) { return dd_add(a, dd_neg(b)); }

// exact product of two doubles
__device__ __forceinline__ DD dd_prod(double a, double b)
{
#pragma clang fp contract(off)
    const double p = a * b;
    return {p, fma(a, b, -p)};
}

// product of two double-doubles (the lo * lo term, below 2^-106 relative,
// is dropped)
__device__ __forceinline__ DD dd_mul(DD a, DD b)
{
#pragma clang fp contract(off)
    DD p = dd_prod(a.hi, b.hi);
    const double c = a.hi * b.lo + a.lo * b.hi;
    return dd_quick(p.hi, p.lo + c);
}

__device__ __forceinline__ double dd_val(DD a) { return a.hi + a.lo; }

// Inclusive prefix sums over a block of B threads (one value each), through
// the LDS buffer buf[B]. Every thread of the block must call it.
template <int B>
__device__ __forceinline__ DD dd_block_scan(DD v, DD *buf)
{
    const int t = threadIdx.x;
    buf[t] = v;
    __syncthreads();
    for (int off = 1; off < B; off <<= 1) {
        const DD o = (t >= off) ? buf[t - off] : DD{0.0, 0.0};
        __syncthreads();
        v = dd_add(o, v);
        buf[t] = v;
        __syncthreads();
    }
    return v;
}

template <int B>
__device__ __forceinline__ int int_block_scan(int v, int *buf)
{
    const int t = threadIdx.x;
    buf[t] = v;
    __syncthreads();
    for (int off = 1; off < B; off <<= 1) {
        const int o = (t >= off) ? buf[t - off] : 0;
        __syncthreads();
        v += o;
        buf[t] = v;
        __syncthreads();
    }
    return v;
}

// Segmented inclusive prefix sums over a block of B threads: a segment
// starts wherever start is set (fbuf[B] holds the flags).
template <int B>
__device__ __forceinline__ DD dd_segment_scan(bool start, DD v, DD *buf, int *fbuf)
{
    const int t = threadIdx.x;
    int f = start ? 1 : 0;
    buf[t] = v;
    fbuf[t] = f;
    __syncthreads();
    for (int off = 1; off < B; off <<= 1) {
        const DD o = (t >= off) ? buf[t - off] : DD{0.0, 0.0};
        const int of = (t >= off) ? fbuf[t - off] : 1;
        __syncthreads();
        if (!f) {
            v = dd_add(o, v);
            f = of;
        }
        buf[t] = v;
        fbuf[t] = f;
        __syncthreads();
    }
    return v;
}

// Block-wide sum, returned to every thread.
template <int B>
__device__ __forceinline__ DD dd_block_sum(DD v, DD *buf)
{
    dd_block_scan<B>(v, buf);
    const DD tot = buf[B - 1];
    __syncthreads();
    return tot;
}

}  // namespace mpk
