// k_sweep_band.hip -- the diagonal sweep, wavefront-native.
//
// What is computed is Algorithms 1-3: along every diagonal k = j - i the
// pre-root distance of (i, j) follows from that of (i-1, j-1) in O(1)
// (Lemma 1 / Lemma 2 / the centred form of Lemma 3), and every pair updates the
// minimum of its row i and of its column j. How it is laid out here:
//
//  * A work item is a band of 64*KD consecutive diagonals [k_lo, k_lo + 64 KD)
//    times a run of rows [i0, i1). One wavefront owns one item at a time; each
//    wave of the persistent grid owns an equal share of the band-major rows,
//    where every band also counts the cost of its restart.
//  * Lane l owns the KD diagonals k_lo + KD l + d. All 64 lanes step through
//    the rows together, so the row operands are wave-uniform (scalar loads) and
//    the column operands of a step are KD-strided in the column stream.
//  * Each item starts with FP64 sums of its first row taken over the m samples
//    of each window pair (the refresh), then runs the O(1) recurrence for the
//    remaining rows, in the precision F: double, or float with the start
//    values rounded from the FP64 sums.
//  * Column operands come from an LDS ring: the stream entries of the item's
//    columns are staged once (coalesced, one block of KD entries per KD steps,
//    fetched a block ahead) and each step every lane reads the one entry that
//    enters its register window of KD columns.
//  * Minima are kept as packed keys: the value being minimised (F) with its low
//    log2(64 KD) mantissa bits replaced by the wave-local diagonal index, so one
//    min instruction keeps value and argument together.
//    - row i: min over the lane's KD diagonals in registers, then across the
//      64 lanes through a small LDS transpose every 8 rows (DPP inside groups
//      of 8 lanes), then one global atomicMin per row and item;
//    - column j: the lane keeps a rotating accumulator per column of its
//      window; after a column's last diagonal in lane l it moves to lane l-1
//      (one DPP wave shift per step); the column leaving lane 0 enters a
//      history register (one DPP shift per step) that is flushed with one
//      global atomicMin per column and item every 64 steps.
//  * Pairs past the end of the series read sentinel stream entries (see
//    k_prep) and lose every comparison; rows and columns outside the item or
//    the series are never written.
//
// Local column numbering: c = j - (i0 + k_lo). At step tau (row i0 + 1 + tau)
// lane l diagonal d touches c = tau + 1 + KD l + d; the entering column of a
// step (d = KD - 1) is c = tau + KD (l + 1). Step tau = -1 is the first row.
#include "keys.h"
#include "mp_internal.h"

namespace mpk {

namespace {

constexpr int NRB = 8;  // rows per LDS transpose batch

template <int KD>
struct Log2;
template <>
struct Log2<8> {
    static constexpr int v = 3;
};
template <>
struct Log2<16> {
    static constexpr int v = 4;
};

// XOR term of the ring swizzle for column block u = c / KD: element c is
// stored at c ^ g(u), a permutation inside each aligned block of KD elements.
// One step's reads (consecutive u, same offset in the block) land on distinct
// bank pairs; within a block of steps a lane's address changes by one XOR.
template <int KD>
__device__ __forceinline__ int gxor(int u)
{
    return (u >> (5 - Log2<KD>::v)) & (KD - 1);
}

template <int KD>
__device__ __forceinline__ int ring_pos(int c)
{
    return c ^ gxor<KD>(c >> Log2<KD>::v);
}

constexpr int DPP_WAVE_SHL1 = 0x130;
constexpr int DPP_WAVE_SHR1 = 0x138;
constexpr int DPP_QUAD_XOR1 = 0xB1;       // quad_perm [1,0,3,2]
constexpr int DPP_QUAD_XOR2 = 0x4E;       // quad_perm [2,3,0,1]
constexpr int DPP_ROW_HALF_MIRROR = 0x141;

// --- per-precision key operations -------------------------------------------
// A key is a value of type F whose low mantissa bits carry an index. Keys are
// compared with the plain float min instruction (IEEE mode is off for this
// file; keys are never NaN).
template <typename F>
struct Prec;

template <>
struct Prec<double> {
    __device__ static double inf() { return __longlong_as_double(0x7FF0000000000000ll); }
    __device__ static double key(double v, uint32_t notmask, uint32_t w)
    {
        unsigned long long b = (unsigned long long)__double_as_longlong(v);
        uint32_t lo = ((uint32_t)b & notmask) | w;
        return __longlong_as_double((long long)((b & 0xFFFFFFFF00000000ull) | lo));
    }
    __device__ static uint32_t index(double k)
    {
        return (uint32_t)(unsigned long long)__double_as_longlong(k);
    }
    __device__ static double kmin(double a, double b) { return __builtin_fmin(a, b); }
    template <int CTRL>
    __device__ static double dpp(double v)
    {
        unsigned long long b = (unsigned long long)__double_as_longlong(v);
        int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)b, CTRL, 0xF, 0xF, false);
        int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
        return __longlong_as_double(
            (long long)(((unsigned long long)(uint32_t)hi << 32) | (uint32_t)lo));
    }
    // wave_shl:1, lane 63 receives +inf (high word from `old`, low word zero)
    __device__ static double shift_down_inf(double v)
    {
        unsigned long long b = (unsigned long long)__double_as_longlong(v);
        int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)b, DPP_WAVE_SHL1, 0xF, 0xF, true);
        int hi = __builtin_amdgcn_update_dpp((int)0x7FF00000, (int)(uint32_t)(b >> 32),
                                             DPP_WAVE_SHL1, 0xF, 0xF, false);
        return __longlong_as_double(
            (long long)(((unsigned long long)(uint32_t)hi << 32) | (uint32_t)lo));
    }
    // wave_shr:1 into the register of `keep`: lane l > 0 receives lane l-1's
    // `hist`, lane 0 keeps `keep`
    __device__ static double shift_up_keep(double hist, double keep)
    {
        unsigned long long h = (unsigned long long)__double_as_longlong(hist);
        unsigned long long k = (unsigned long long)__double_as_longlong(keep);
        int lo = __builtin_amdgcn_update_dpp((int)(uint32_t)k, (int)(uint32_t)h, DPP_WAVE_SHR1,
                                             0xF, 0xF, false);
        int hi = __builtin_amdgcn_update_dpp((int)(uint32_t)(k >> 32), (int)(uint32_t)(h >> 32),
                                             DPP_WAVE_SHR1, 0xF, 0xF, false);
        return __longlong_as_double(
            (long long)(((unsigned long long)(uint32_t)hi << 32) | (uint32_t)lo));
    }
    // refresh value of a diagonal already past the end (AAMP / p-norm)
    __device__ static double sentinel() { return SENT_INIT; }
    __device__ static bool flushable(int kind, double v)
    {
        return kind == ACAMP ? (v < 1e300) : (v < 1e190);
    }
};

template <>
struct Prec<float> {
    __device__ static float inf() { return __int_as_float(0x7F800000); }
    __device__ static float key(float v, uint32_t notmask, uint32_t w)
    {
        return __uint_as_float((__float_as_uint(v) & notmask) | w);
    }
    __device__ static uint32_t index(float k) { return __float_as_uint(k); }
    __device__ static float kmin(float a, float b) { return __builtin_fminf(a, b); }
    template <int CTRL>
    __device__ static float dpp(float v)
    {
        return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
    }
    __device__ static float shift_down_inf(float v)
    {
        return __int_as_float(__builtin_amdgcn_update_dpp((int)0x7F800000, __float_as_int(v),
                                                          DPP_WAVE_SHL1, 0xF, 0xF, false));
    }
    __device__ static float shift_up_keep(float hist, float keep)
    {
        return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(keep), __float_as_int(hist),
                                                          DPP_WAVE_SHR1, 0xF, 0xF, false));
    }
    // refresh value of a diagonal already past the end: +inf (the float
    // sentinel increments are positive, so it stays +inf)
    __device__ static float sentinel() { return __int_as_float(0x7F800000); }
    __device__ static bool flushable(int kind, float v)
    {
        (void)kind;
        return v < 1e30f;
    }
};

template <int PC, typename F>
__device__ __forceinline__ F pw(F d, double p)
{
    F a = fabs(d);
    if (PC == P_ONE) return a;
    if (PC == P_THREE) return a * a * a;
    return (F)pow((double)a, p);   // P_GENERIC (FP64 sweeps only)
}

// A workgroup is a single wavefront and LDS executes one wave's accesses in
// issue order, so ordering LDS accesses only needs the compiler not to move
// them; no s_waitcnt drain or s_barrier.
__device__ __forceinline__ void lds_order() { asm volatile("" ::: "memory"); }

// Wave-uniform reads go through the constant address space so that they
// become scalar loads (the data is read-only for the whole launch).
typedef const __attribute__((address_space(4))) double cdouble;
typedef const __attribute__((address_space(4))) float cfloat;
typedef const __attribute__((address_space(4))) int64_t cint64;
__device__ __forceinline__ cdouble *as_const(const double *p) { return (cdouble *)p; }
__device__ __forceinline__ cfloat *as_const(const float *p) { return (cfloat *)p; }
__device__ __forceinline__ cint64 *as_const(const int64_t *p) { return (cint64 *)p; }

__device__ __forceinline__ int64_t uniform64(int64_t v)
{
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

template <typename F>
struct Streams;
template <>
struct Streams<double> {
    __device__ static const double *x(const Series &s) { return s.x; }
    __device__ static const double *y(const Series &s) { return s.y; }
    __device__ static const double *z(const Series &s) { return s.z; }
};
template <>
struct Streams<float> {
    __device__ static const float *x(const Series &s) { return s.xf; }
    __device__ static const float *y(const Series &s) { return s.yf; }
    __device__ static const float *z(const Series &s) { return s.zf; }
};

// LDS doubles the first-row staging uses: the column samples of a 64-step
// chunk (64 KD + 64, one pad slot per KD), then its 64 row samples.
template <int KD>
constexpr int stage_cols()
{
    return (64 * KD + 64) + (64 * KD + 64) / KD;
}
template <int KD>
constexpr int stage_doubles()
{
    return stage_cols<KD>() + 64;
}

}  // namespace

// One work item: the diagonals [k_lo, k_lo + 64 KD) of series s, rows
// [i0, i1). ring (NF x RING entries) and rowbuf (NRB x 64) are the wave's LDS;
// stage (stage_doubles<KD>() entries) overlays them while the first row is
// computed.
// ACAMP key of a pair from its centred cross sum S, invn_i (ri) and -invn_j
// (cj). With q = S ri cj = -rho the default key is 1 - rho. The comparator
// of Sec. 4.4, F = -m^2 rho |rho|, orders pairs as the distance does; its key
// 1 + F / m^2 = 1 - rho |rho| = fma(q, |q|, 1) costs one multiply more.
template <int PC, typename F>
__device__ __forceinline__ F acamp_key(F S, F ri, F cj)
{
    if (PC == P_FCMP) {
        const F q = S * ri * cj;
        return fma(q, fabs(q), (F)1);
    }
    return fma(S * ri, cj, (F)1);
}

// ROWS_LDS: the restart stages each chunk's row samples in LDS and reads them
// back as broadcasts; otherwise it takes them as scalar loads (the kernels
// that run 3 waves per SIMD on 168 registers, where holding them in vector
// registers spills in the recurrence loop).
template <int KIND, int PC, int KD, typename F, bool COUNT, bool ROWS_LDS, int WPB>
__device__ __forceinline__ void band_item(const Series &s, const int64_t k_lo, const int64_t i0,
                                          const int64_t i1, F *ring, F *rowbuf, F *rowop,
                                          double *stage, unsigned long long *visits)
{
    typedef Prec<F> P;
    constexpr int WD = 64 * KD;          // diagonals per item
    constexpr int RING = WD;             // ring entries per field

    // (blocks of one wave use threadIdx.x as it is: masking it changes the
    // schedule of the ring writes)
    const int lane = WPB == 1 ? (int)threadIdx.x : (int)(threadIdx.x & 63);
    const int64_t N = s.N;
    const uint32_t notmask = ~(uint32_t)(WD - 1);
    const unsigned long long gmask = (1ull << s.gb) - 1ull;
    const F INF = P::inf();
    const int m = s.m;

    uint32_t wd[KD];
#pragma unroll
    for (int d = 0; d < KD; ++d) wd[d] = (uint32_t)(lane * KD + d);

    const gptr<F> sx = as_global(Streams<F>::x(s));
    const gptr<F> sy = as_global(Streams<F>::y(s));
    const gptr<F> sz = as_global(Streams<F>::z(s));
    const gptr<double> Tg = as_global(s.T);
    const gptr<double> mug = as_global(s.mu);
    cdouble *Tc = as_const(s.T);
    // Single-precision Euclidean and p-norm sweeps take their sample-valued
    // operands (AAMP: v = t[j+m-1] + t[j-1]; p-norm: both samples) relative to
    // the item's own centre cc = t[i0], converted from the FP64 streams as they
    // are staged: their rounding then scales with the item's local spread, not
    // with the series' offset (both sides of every difference shift alike).
    // Row operands reach the lanes through a small LDS buffer (rowop), since
    // the conversion needs vector instructions. Entries at or past N keep the
    // single-precision sentinels.
    constexpr bool RECENTRE = sizeof(F) == 4 && KIND != ACAMP;
    constexpr bool RX_LDS = RECENTRE && KIND == PNORM;
    const double cc = RECENTRE ? Tc[i0] : 0.0;
    const gptr<double> xg = as_global(s.x);
    const gptr<double> yg = as_global(s.y);
    const F sent_x = (KIND == PNORM) ? (F)(s.pclass == P_ONE ? SENTF_P1 : SENTF_P3)
                                     : (F)SENTF_EUCLID;
    auto col_x = [&](int64_t c) -> F {
        if (!RX_LDS) return sx[c];
        return c < N ? (F)(xg[c] - cc) : sent_x;
    };
    auto col_y = [&](int64_t c) -> F {
        if (!RECENTRE) return sy[c];
        if (KIND == AAMP) return c < N ? (F)(yg[c] - 2.0 * cc) : (F)SENTF_EUCLID;
        return c < N ? (F)(yg[c] - cc) : (F)0;
    };
    const auto xc = as_const(Streams<F>::x(s));
    const auto yc = as_const(Streams<F>::y(s));
    const auto zc = as_const(Streams<F>::z(s));
    {
        const int nsteps = (int)(i1 - i0) - 1;      // recurrence steps after the first row
        const int64_t cb = i0 + k_lo;               // stream index of local column 0

        // ---- FP64 start values of the first row (the refresh) ---------------
        // At step l lane l' needs the samples t[jb + l + d], d < KD, of its
        // diagonals and the row sample t[i0 + l]. Over a chunk of LCH steps the
        // 64 lanes' column samples form one contiguous run, so each chunk is
        // staged in LDS with coalesced loads (the next chunk's loads are issued
        // before the current chunk is consumed); a lane then reads the KD
        // samples entering its register window over the next KD steps at once,
        // from one address with immediate offsets. The chunk's row samples are
        // staged beside them and read back as broadcasts (scalar loads would
        // stall every KD steps on their latency). Column element e of a chunk
        // sits at e + e / KD, so the lanes' reads (KD elements apart) hit
        // distinct banks.
        //
        // Euclidean and z-normalized distances need one FMA per sample and
        // diagonal: with every sample shifted by c = t[i0] (u = t - c),
        //   S(i0, j)   = sum u_i^2 + sum u_j^2 - 2 sum u_i u_j
        //   cov(i0, j) = sum u_i u_j - m (mu_i0 - c)(mu_j - c)
        // (the shift cancels in both). The column energies follow from the
        // lane's first one by sliding the window. Rounding is relative to the
        // windows' spread around c rather than to the series' offset. The
        // p-norms sum |t_i - t_j|^p directly.
        F S[KD];
        {
            constexpr int LCH = 64;                     // steps per staged chunk
            constexpr int NLD = (WD + LCH) / 64;        // loads per lane per chunk
            constexpr bool DOT = KIND != PNORM;
            const int64_t jb = cb + (int64_t)KD * lane;   // this lane's first column
            const int64_t tmax = s.n - 1;
            const double c0 = DOT ? Tc[i0] : 0.0;
            double acc[KD], win[KD];
            double erow = 0.0, ecol = 0.0;   // AAMP: sum u^2 of the row window and of column jb
#pragma unroll
            for (int d = 0; d < KD; ++d) {
                acc[d] = 0.0;
                win[d] = 0.0;
            }
            auto spos = [](int e) { return e + (e >> Log2<KD>::v); };
            double *rowst = stage + stage_cols<KD>();   // the chunk's LCH row samples
            double nc[NLD], nr;
            auto fetch = [&](int l0) {
#pragma unroll
                for (int q = 0; q < NLD; ++q) nc[q] = Tg[min(cb + l0 + 64 * q + lane, tmax)];
                if (ROWS_LDS) nr = Tg[min(i0 + l0 + lane, tmax)];
            };
            auto put = [&]() {
                lds_order();
#pragma unroll
                for (int q = 0; q < NLD; ++q) stage[spos(64 * q + lane)] = nc[q] - c0;
                if (ROWS_LDS) rowst[lane] = nr - c0;
                lds_order();
            };
            fetch(0);
            put();
#pragma unroll
            for (int d = 0; d < KD - 1; ++d) win[d] = stage[spos(KD * lane + d)];
            // One step: w enters slot (q + KD - 1) % KD, q = l % KD; tr is the
            // (shifted) row sample.
            auto step = [&](int q, double w, double tr) {
                win[(q + KD - 1) % KD] = w;
                if (DOT) {
#pragma unroll
                    for (int d = 0; d < KD; ++d) acc[d] = fma(tr, win[(q + d) % KD], acc[d]);
                    if (KIND == AAMP) {
                        erow = fma(tr, tr, erow);
                        ecol = fma(win[q % KD], win[q % KD], ecol);
                    }
                } else {
                    // the KD differences are formed before any is accumulated,
                    // so that they do not share one register
                    double e[KD];
#pragma unroll
                    for (int d = 0; d < KD; ++d) e[d] = tr - win[(q + d) % KD];
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int d = 0; d < KD; ++d) acc[d] += pw<PC, double>(e[d], s.p);
                }
            };
            for (int l0 = 0; l0 < m; l0 += LCH) {
                const bool more = l0 + LCH < m;
                if (more) fetch(l0 + LCH);
                const int steps = min(LCH, m - l0);
                const int full = steps & ~(KD - 1);
                for (int g = 0; g < full; g += KD) {
                    double nw[KD];
                    // spos(KD lane + g + q + KD - 1) for g a multiple of KD:
                    // one base, then q + (q > 0)
                    const int sb = (KD + 1) * lane + g + (g >> Log2<KD>::v) + KD - 1;
#pragma unroll
                    for (int q = 0; q < KD; ++q)
                        nw[q] = ROWS_LDS ? stage[sb + q + (q > 0 ? 1 : 0)]
                                         : stage[spos(KD * lane + g + q + KD - 1)];
                    if (ROWS_LDS) {
#pragma unroll
                        for (int q = 0; q < KD; ++q) step(q, nw[q], rowst[g + q]);
                    } else {
                        double rv[KD];
                        const int64_t rb = uniform64(i0 + l0 + g);
#pragma unroll
                        for (int q = 0; q < KD; ++q) rv[q] = Tc[rb + q] - c0;
#pragma unroll
                        for (int q = 0; q < KD; ++q) step(q, nw[q], rv[q]);
                    }
                }
                if (full < steps) {
#pragma unroll
                    for (int q = 0; q < KD - 1; ++q)
                        if (full + q < steps)
                            step(q, stage[spos(KD * lane + full + q + KD - 1)],
                                 ROWS_LDS ? rowst[full + q] : Tc[i0 + l0 + full + q] - c0);
                }
                // a full chunk leaves the window slots aligned with the next
                // chunk's first step; its entries are already in registers
                if (more) put();
            }
            lds_order();
            if (KIND == AAMP) {
                // column window jb + d drops sample jb + d - 1, takes jb + d - 1 + m
                double ec = ecol;
#pragma unroll
                for (int d = 0; d < KD; ++d) {
                    if (d > 0) {
                        const double uo = Tg[min(jb + d - 1, tmax)] - c0;
                        const double un = Tg[min(jb + d - 1 + m, tmax)] - c0;
                        ec = fma(un, un, fma(-uo, uo, ec));
                    }
                    acc[d] = fma(-2.0, acc[d], erow + ec);
                }
            } else if (KIND == ACAMP) {
                const double am = (double)m * (as_const(s.mu)[i0] - c0);
#pragma unroll
                for (int d = 0; d < KD; ++d) acc[d] = fma(-am, mug[min(jb + d, N - 1)] - c0, acc[d]);
            }
#pragma unroll
            for (int d = 0; d < KD; ++d) {
                const bool valid = (jb + d) <= N - 1;
                S[d] = valid ? (F)acc[d] : (KIND == ACAMP ? (F)0 : P::sentinel());
            }
        }

        // ---- stage the column streams in the LDS ring: local columns [0, RING)
        lds_order();
#pragma unroll
        for (int q = 0; q < RING / 64; ++q) {
            const int c = lane + 64 * q;
            const int e = ring_pos<KD>(c);
            ring[e] = col_x(cb + c);
            ring[RING + e] = col_y(cb + c);
            if (KIND == ACAMP) ring[2 * RING + e] = sz[cb + c];
        }
        lds_order();

        // register window of column operands: slot c % KD holds local column c
        // of this lane's window; slots 1..KD-1 are preloaded for tau = 0
        F cx[KD], cy[KD], cz[KD];
#pragma unroll
        for (int d = 0; d < KD; ++d) {
            cx[d] = (F)0;
            cy[d] = (F)0;
            cz[d] = (F)0;
        }
#pragma unroll
        for (int d = 0; d < KD - 1; ++d) {
            const int c = KD * lane + 1 + d;
            const int e = ring_pos<KD>(c);
            cx[(1 + d) % KD] = ring[e];
            cy[(1 + d) % KD] = ring[RING + e];
            if (KIND == ACAMP) cz[(1 + d) % KD] = ring[2 * RING + e];
        }

        F colacc[KD];
#pragma unroll
        for (int d = 0; d < KD; ++d) colacc[d] = INF;
        F hist = INF;   // lane p: key of the column that left lane 0 p steps ago

        // -------------------------------------------------------------------
        // one step: keys of the current values, row minimum into the LDS
        // transpose, column minima into the rotating accumulators, then the
        // column whose last diagonal in this lane was d = 0 moves one lane
        // down and lane 0's enters the history register.
        // The accumulator of diagonal d lives in slot (sbase + d) % KD.
        auto reduce_step = [&](int row_slot, int sbase, const F (&v)[KD]) {
            F key[KD];
#pragma unroll
            for (int d = 0; d < KD; ++d) {
                key[d] = P::key(v[d], notmask, wd[d]);
                colacc[(sbase + d) % KD] = P::kmin(colacc[(sbase + d) % KD], key[d]);
            }
#pragma unroll
            for (int ww = 1; ww < KD; ww *= 2)
#pragma unroll
                for (int d = 0; d + ww < KD; d += 2 * ww) key[d] = P::kmin(key[d], key[d + ww]);
            rowbuf[row_slot * 64 + lane] = key[0];
            const F done = colacc[sbase % KD];
            colacc[sbase % KD] = P::shift_down_inf(done);
            hist = P::shift_up_keep(hist, done);
        };

        // LDS transpose flush of the rows whose slots are 0..cnt-1; slot 0
        // holds row rbase. Lane l reduces row l / 8 over lanes 8 (l % 8) ..
        // 8 (l % 8) + 7, then the 8 lanes of a group combine with three DPP
        // steps (xor 1, xor 2, half-row mirror).
        auto flush_rows = [&](int64_t rbase, int cnt) {
            lds_order();
            const int r = lane >> 3;
            F v = INF;
#pragma unroll
            for (int q = 0; q < 8; ++q) v = P::kmin(v, rowbuf[lane * 8 + q]);
            v = P::kmin(v, P::template dpp<DPP_QUAD_XOR1>(v));
            v = P::kmin(v, P::template dpp<DPP_QUAD_XOR2>(v));
            v = P::kmin(v, P::template dpp<DPP_ROW_HALF_MIRROR>(v));
            const int64_t row = rbase + r;
            if ((lane & 7) == 0 && r < cnt && row < i1 && P::flushable(KIND, v)) {
                const int64_t j = row + k_lo + (int64_t)(P::index(v) & (uint32_t)(WD - 1));
                const unsigned long long idx = (j < N) ? (unsigned long long)j : gmask;
                global_min(&s.keys[row], pack_key((double)v, idx, gmask));
            }
            lds_order();
        };

        // flush columns from the history register: lane p holds local column
        // cend - p; lanes p < cnt take part.
        auto flush_cols = [&](int cend, int cnt) {
            if (lane < cnt) {
                const F v = hist;
                const int64_t j = cb + cend - lane;
                if (j < N && P::flushable(KIND, v)) {
                    const int64_t i = j - k_lo - (int64_t)(P::index(v) & (uint32_t)(WD - 1));
                    global_min(&s.keys[j], pack_key((double)v, (unsigned long long)i, gmask));
                }
            }
        };

        // ---- first row (tau = -1): start values only ------------------------
        {
            F v[KD];
            const F rinv0 = (KIND == ACAMP) ? -zc[i0] : (F)0;
            const int64_t jb = cb + (int64_t)KD * lane;
#pragma unroll
            for (int d = 0; d < KD; ++d)
                v[d] = (KIND == ACAMP) ? acamp_key<PC, F>(S[d], rinv0, sz[jb + d]) : S[d];
            reduce_step(0, 0, v);
        }
        flush_cols(0, 1);   // column 0 has only the first row's pair
        // Pair-visit count (test mode): the real pairs (j < N) of every step
        // whose row belongs to this item. The last block may run up to KD - 1
        // steps past i1; those rows belong to the next item and are not counted.
        unsigned long long visited = 0;
        auto count_row = [&](int64_t row) {
            if (COUNT && row < i1) {
                const int64_t left = N - (row + k_lo + (int64_t)KD * lane);
                visited += (unsigned long long)max((int64_t)0, min((int64_t)KD, left));
            }
        };
        count_row(i0);

        // ---- recurrence, KD steps per unrolled block --------------------------
        // Block tb needs local columns [tb + RING, tb + RING + KD) in the ring;
        // lanes < KD fetch each block one block ahead.
        const int bl = min(lane, KD - 1);
        F bx = col_x(cb + RING + bl);
        F by = col_y(cb + RING + bl);
        F bz = (KIND == ACAMP) ? sz[cb + RING + bl] : (F)0;
        // recentred row operands of the next block, one row per lane < KD
        F nrx = RX_LDS ? col_x(i0 + 1 + bl) : (F)0;
        F nry = RECENTRE ? col_y(i0 + 1 + bl) : (F)0;
        // the row operands of a block (scalar registers), fetched during the
        // previous block
        F rxs[KD], rys[KD], rzs[KD];
        {
            const auto xr = xc + (i0 + 1);
            const auto yr = yc + (i0 + 1);
            const auto zr = zc + (i0 + 1);
#pragma unroll
            for (int q = 0; q < KD; ++q) {
                rxs[q] = xr[q];
                rys[q] = yr[q];
                rzs[q] = (KIND == ACAMP) ? -zr[q] : (F)0;
            }
        }
        int tb = 0;
        for (; tb < nsteps; tb += KD) {
            tb = __builtin_amdgcn_readfirstlane(tb);
            // row operands of this block: rows i0 + 1 + tb + q, q < KD
            const int64_t rb = uniform64(i0 + 1 + tb);
            const auto xr = xc + rb;
            const auto yr = yc + rb;
            const auto zr = zc + rb;
            lds_order();
            if (lane < KD) {
                const int e = ring_pos<KD>((tb + RING + lane) & (RING - 1));
                ring[e] = bx;
                ring[RING + e] = by;
                if (KIND == ACAMP) ring[2 * RING + e] = bz;
                if (RX_LDS) rowop[lane] = nrx;
                if (RECENTRE) rowop[KD + lane] = nry;
            }
            lds_order();
            {
                const int64_t c = cb + tb + KD + RING + bl;
                bx = col_x(c);
                by = col_y(c);
                if (KIND == ACAMP) bz = sz[c];
                if (RX_LDS) nrx = col_x(rb + KD + bl);
                if (RECENTRE) nry = col_y(rb + KD + bl);
            }
            // this block's entering columns are tb + KD (lane + 1) + q, all in
            // the aligned column block u = tb / KD + lane + 1
            const int ublk = (tb >> Log2<KD>::v) + lane + 1;
            const int ebase = ((ublk * KD) & (RING - 1)) ^ gxor<KD>(ublk);
#pragma unroll
            for (int q = 0; q < KD; ++q) {
                const int tau = tb + q;
                {
                    const int e = ebase ^ q;
                    cx[q] = ring[e];
                    cy[q] = ring[RING + e];
                    if (KIND == ACAMP) cz[q] = ring[2 * RING + e];
                }
                const F rx = RX_LDS ? rowop[q] : rxs[q];
                const F ry = RECENTRE ? rowop[KD + q] : rys[q];
                const F rinv = rzs[q];
                F v[KD];
#pragma unroll
                for (int d = 0; d < KD; ++d) {
                    const int sl = (q + 1 + d) % KD;
                    if (KIND == AAMP) {
                        S[d] = fma(rx - cx[sl], ry - cy[sl], S[d]);
                        v[d] = S[d];
                    } else if (KIND == PNORM) {
                        S[d] += pw<PC, F>(rx - cx[sl], s.p) - pw<PC, F>(ry - cy[sl], s.p);
                        v[d] = S[d];
                    } else {
                        S[d] = fma(rx, cy[sl], S[d]);
                        S[d] = fma(cx[sl], ry, S[d]);
                        // 1 - rho (or 1 - rho |rho|), with cz = -invn_j
                        v[d] = acamp_key<PC, F>(S[d], rinv, cz[sl]);
                    }
                }
                reduce_step((q + 1) & (NRB - 1), q + 1, v);
                count_row(i0 + 1 + tau);
                if (q == KD - 1) {
                    // next block's row operands (rows past i1 read padding entries)
#pragma unroll
                    for (int u = 0; u < KD; ++u) {
                        rxs[u] = xr[KD + u];
                        rys[u] = yr[KD + u];
                        rzs[u] = (KIND == ACAMP) ? -zr[KD + u] : (F)0;
                    }
                }
                // tb is a multiple of KD and NRB divides KD: (tau + 1) % NRB == (q + 1) % NRB
                if (((q + 1) & (NRB - 1)) == NRB - 1) flush_rows(i0 + tau + 2 - NRB, NRB);
            }
            // the column of step tau is tau + 1, so this block completed
            // columns tb + 1 .. tb + KD; flush them 64 at a time
            if (((tb + KD) & 63) == 0) flush_cols(tb + KD, 64);
        }
        // Steps ran for tau = -1 .. tb - 1. Pending: the row of the last step
        // (its transpose slot is 0 since tb is a multiple of 8) and the columns
        // completed since the last 64-column flush: (tb & ~63) + 1 .. tb.
        if (tb & 63) flush_cols(tb, tb & 63);
        flush_rows(i0 + tb, 1);
        // columns still held by the lanes: slot (tb + 1 + d) % KD = (1 + d) % KD
        // holds local column tb + 1 + KD lane + d
#pragma unroll
        for (int d = 0; d < KD; ++d) {
            const F v = colacc[(1 + d) % KD];
            const int64_t j = cb + tb + 1 + (int64_t)KD * lane + d;
            if (j < N && P::flushable(KIND, v)) {
                const int64_t i = j - k_lo - (int64_t)(P::index(v) & (uint32_t)(WD - 1));
                global_min(&s.keys[j], pack_key((double)v, (unsigned long long)i, gmask));
            }
        }
        if (COUNT && visited) {
            typedef __attribute__((address_space(1))) unsigned long long gu64;
            __hip_atomic_fetch_add((gu64 *)visits, visited, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
        lds_order();
    }
}

// Resident waves per SIMD the compiler is asked for. The FP64 AAMP and p = 1,
// 3 kernels fit 3 waves (168 VGPRs) at the cost of a few spills outside the
// inner loop, 2-4 % faster than 2 waves. The FP64 ACAMP kernel holds three
// ring fields (16 KB of LDS per wave), so 12 waves do not fit a CU's 160 KB;
// asking for 3 was 55 % slower. It, the mixed and the generic-p kernels keep
// the default. FP32 with 8 diagonals per lane fits 4 waves without spills.
// Blocks of four waves serve only grids capped at one or two waves per SIMD:
// asking for 4 there held the FP32 kernels to 128 registers and spilled 33-41.
template <uint32_t SELS, int KD, typename F, int WPB>
constexpr int waves_target()
{
    if (WPB == 4) return 2;
    if (KD != 8 || (SELS & SEL_LONG)) return 1;
    if (sizeof(F) == 4) return 4;
    return (SELS == SEL_AAMP || SELS == SEL_P1 || SELS == SEL_P3) ? 3 : 1;
}

// The persistent sweep over every band of every job of a launch. SELS is the
// set of distance specialisations the launch holds: a single one gets a kernel
// of its own; a mix dispatches per item (the branch is wave-uniform). Each
// wave is a persistent worker of its own; a block holds WPB of them (4 for
// grids capped at one or two waves per SIMD: the hardware places a block's
// four waves on four SIMDs, while blocks of one wave can land two on a SIMD
// and none on another).
template <uint32_t SELS, int KD, typename F, bool COUNT, int WPB>
__global__ void __launch_bounds__(64 * WPB)
    __attribute__((amdgpu_waves_per_eu(waves_target<SELS, KD, F, WPB>()))) k_sweep_band(Batch b)
{
    constexpr int RING = 64 * KD;
    constexpr int NF = (SELS & SEL_ACAMP) ? 3 : 2;
    // ring fields, row transpose, recentred row operands (FP32 only)
    constexpr int SWEEP_D = (int)(((NF * RING + NRB * 64 + 2 * KD) * sizeof(F) + 7) / 8);
    constexpr int LDS_D = SWEEP_D > stage_doubles<KD>() ? SWEEP_D : stage_doubles<KD>();
    __shared__ double lds_all[WPB * LDS_D];
    const int wv = WPB == 1 ? 0 : __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    double *lds = lds_all + wv * LDS_D;   // this wave's part
    F *ring = reinterpret_cast<F *>(lds);
    F *rowbuf = ring + NF * RING;
    F *rowop = rowbuf + NRB * 64;
    double *stage = lds;

    constexpr bool RL = waves_target<SELS, KD, F, WPB>() != 3;
    cint64 *row_base = as_const(b.row_base);
    cint64 *band_start = as_const(b.band_start);
    const int64_t total = row_base[b.njobs];   // band-row positions of the launch

    // This wave's share of the row space: every row of a band costs the same
    // (pairs past the series end run on sentinels), and each band is preceded
    // by band_cost positions that stand for its exact restart, so equal
    // position ranges are nearly equal work. share = total / G positions, the
    // first total % G waves take one more.
    const int64_t G = (int64_t)gridDim.x * WPB;
    const int64_t w = (int64_t)blockIdx.x * WPB + wv;
    const int64_t qrows = total / G, rrows = total % G;
    int64_t pos = uniform64(w * qrows + min(w, rrows));
    const int64_t pend = uniform64(pos + qrows + (w < rrows ? 1 : 0));

    while (pos < pend) {
        // job holding position pos: the last job with row_base <= pos (jobs
        // without band rows share their successor's row_base and are skipped)
        int jlo = 0, jhi = b.njobs;
        while (jhi - jlo > 1) {
            const int mid = (jlo + jhi) >> 1;
            if (row_base[mid] <= pos) jlo = mid;
            else jhi = mid;
        }
        jlo = __builtin_amdgcn_readfirstlane(jlo);
        const Job J = load_uniform(&b.jobs[jlo]);
        const Series &s = J.s;
        cint64 *bs = band_start + J.band_base;
        // band of the job holding pos: bs[t] <= pos < bs[t + 1]
        int lo = 0, hi = J.nbands;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (bs[mid] <= pos) lo = mid;
            else hi = mid;
        }
        lo = __builtin_amdgcn_readfirstlane(lo);
        // band lo holds positions [bs[lo], bs[lo + 1]): band_cost positions for
        // its restart, then one per row. One item: the rows of band lo from pos
        // up to the end of the share, the band, or the refresh interval,
        // whichever comes first; a share that ends among the restart positions
        // holds no row of the band.
        const int64_t band = J.band_map ? (int64_t)load_uniform(&J.band_map[lo]) : (int64_t)lo;
        const int64_t k_lo = uniform64((int64_t)s.excl + band * RING);
        const int64_t row0 = uniform64(bs[lo] + J.band_cost);   // position of row 0
        const int64_t i0 = uniform64(max(pos - row0, (int64_t)0));
        const int64_t lim = uniform64(min(pend, bs[lo + 1]) - row0);
        const int64_t i1 = uniform64(min(lim, i0 + (int64_t)J.seg_rows));
        if (i1 <= i0) {
            pos = min(pend, bs[lo + 1]);
            continue;
        }
        pos = row0 + i1;
        const uint32_t sel = sel_of(s.kind, s.pclass);
        if ((SELS & SEL_AAMP) && sel == SEL_AAMP)
            band_item<AAMP, P_TWO, KD, F, COUNT, RL, WPB>(s, k_lo, i0, i1, ring, rowbuf, rowop, stage, b.visits);
        else if ((SELS & SEL_ACAMP) && sel == SEL_ACAMP)
            band_item<ACAMP, (SELS & SEL_FCMP) ? P_FCMP : P_TWO, KD, F, COUNT, RL, WPB>(
                s, k_lo, i0, i1, ring, rowbuf, rowop, stage, b.visits);
        else if ((SELS & SEL_P1) && sel == SEL_P1)
            band_item<PNORM, P_ONE, KD, F, COUNT, RL, WPB>(s, k_lo, i0, i1, ring, rowbuf, rowop, stage, b.visits);
        else if ((SELS & SEL_P3) && sel == SEL_P3)
            band_item<PNORM, P_THREE, KD, F, COUNT, RL, WPB>(s, k_lo, i0, i1, ring, rowbuf, rowop, stage, b.visits);
        else if ((SELS & SEL_PGEN) && sel == SEL_PGEN)
            band_item<PNORM, P_GENERIC, KD, F, COUNT, RL, WPB>(s, k_lo, i0, i1, ring, rowbuf, rowop, stage, b.visits);
    }
}

// Band table of every job (one block per job): bs[t] = row_base of the job +
// positions of its bands before t, where band t covers diagonals from
// excl + g W on (g = t, or band_map[t] in a partial sweep), has N - excl - g W
// rows and takes band_cost more positions; the last entry bs[nbands] is the
// job's end.
__global__ void __launch_bounds__(1024) k_band_plan(Batch b)
{
    __shared__ int64_t wtot[16];
    const Job J = load_uniform(&b.jobs[blockIdx.x]);
    const int64_t base = J.row_start;
    const int64_t N = J.s.N, excl = J.s.excl, W = b.band_width, C = J.band_cost;
    const int nb = J.nbands;
    int64_t *bs = b.band_start + J.band_base;
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    const int per = (nb + 1023) / 1024;
    const int b0 = min(t * per, nb), b1 = min(b0 + per, nb);
    // band slot u covers diagonal group map[u] of a partial sweep, else u
    const int32_t *map = J.band_map;
    int64_t sum = 0;
    for (int u = b0; u < b1; ++u) sum += C + N - excl - (int64_t)(map ? map[u] : u) * W;
    // exclusive prefix of the threads' sums: inclusive scans within each
    // wave, then over the 16 wave totals
    int64_t x = sum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int64_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) wtot[wid] = x;
    __syncthreads();
    if (wid == 0) {
        int64_t w = lane < 16 ? wtot[lane] : 0;
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) {
            const int64_t y = __shfl_up(w, off, 64);
            if (lane >= off) w += y;
        }
        if (lane < 16) wtot[lane] = w;
    }
    __syncthreads();
    int64_t run = base + (wid ? wtot[wid - 1] : 0) + x - sum;
    for (int u = b0; u < b1; ++u) {
        bs[u] = run;
        run += C + N - excl - (int64_t)(map ? map[u] : u) * W;
    }
    if (t == 1023) bs[nb] = base + wtot[15];
}

hipError_t launch_plan(const Batch &b, hipStream_t st)
{
    if (b.njobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_band_plan, dim3((unsigned)b.njobs), dim3(1024), 0, st, b);
    return hipGetLastError();
}

namespace {

// Kernel of a selector set: one of its own for a single specialisation,
// otherwise the mixed kernel holding the specialisations of SEL_BAND. The
// pair-counting test mode uses the mixed kernel, or for generic p its own.
template <int KD, typename F>
const void *band_kernel(uint32_t sels, bool count)
{
    if constexpr (sizeof(F) == 8) {
        if (sels == SEL_PGEN)
            return count ? (const void *)k_sweep_band<SEL_PGEN, KD, F, true, 1>
                         : (const void *)k_sweep_band<SEL_PGEN, KD, F, false, 1>;
        // ACAMP keyed on F: launches of such jobs alone (pair counting runs
        // the mixed kernel, which visits the same pairs)
        if (sels == (SEL_ACAMP | SEL_FCMP) && !count)
            return (const void *)k_sweep_band<SEL_ACAMP | SEL_FCMP, KD, F, false, 1>;
        // long windows of the Euclidean and p = 1, 3 distances
        if ((sels & SEL_LONG) && !count) {
            switch (sels & SEL_BAND) {
            case SEL_AAMP: return (const void *)k_sweep_band<SEL_AAMP | SEL_LONG, KD, F, false, 1>;
            case SEL_P1: return (const void *)k_sweep_band<SEL_P1 | SEL_LONG, KD, F, false, 1>;
            case SEL_P3: return (const void *)k_sweep_band<SEL_P3 | SEL_LONG, KD, F, false, 1>;
            default: break;
            }
        }
    }
    if (count) return (const void *)k_sweep_band<SEL_BAND, KD, F, true, 1>;
    switch (sels & SEL_BAND) {
    case SEL_AAMP: return (const void *)k_sweep_band<SEL_AAMP, KD, F, false, 1>;
    case SEL_ACAMP: return (const void *)k_sweep_band<SEL_ACAMP, KD, F, false, 1>;
    case SEL_P1: return (const void *)k_sweep_band<SEL_P1, KD, F, false, 1>;
    case SEL_P3: return (const void *)k_sweep_band<SEL_P3, KD, F, false, 1>;
    default: return (const void *)k_sweep_band<SEL_BAND, KD, F, false, 1>;
    }
}

// Blocks of four waves, for the selector sets that run on capped grids (long
// windows); null where there is none.
template <int KD, typename F>
const void *band_kernel4(uint32_t sels)
{
    if constexpr (KD == 8 && sizeof(F) == 8) {
        switch (sels) {
        case SEL_AAMP | SEL_LONG: return (const void *)k_sweep_band<SEL_AAMP | SEL_LONG, KD, F, false, 4>;
        case SEL_P1 | SEL_LONG: return (const void *)k_sweep_band<SEL_P1 | SEL_LONG, KD, F, false, 4>;
        case SEL_P3 | SEL_LONG: return (const void *)k_sweep_band<SEL_P3 | SEL_LONG, KD, F, false, 4>;
        case SEL_ACAMP: return (const void *)k_sweep_band<SEL_ACAMP, KD, F, false, 4>;
        case SEL_ACAMP | SEL_FCMP:
            return (const void *)k_sweep_band<SEL_ACAMP | SEL_FCMP, KD, F, false, 4>;
        default: return nullptr;
        }
    } else if constexpr (KD == 8) {
        switch (sels) {
        case SEL_ACAMP: return (const void *)k_sweep_band<SEL_ACAMP, KD, F, false, 4>;
        case SEL_P1: return (const void *)k_sweep_band<SEL_P1, KD, F, false, 4>;
        default: return nullptr;
        }
    }
    return nullptr;
}

const void *band_kernel_for(uint32_t sels, int32_t kd, bool fp32, bool count)
{
    if (fp32)
        return kd == 16 ? band_kernel<16, float>(sels, count) : band_kernel<8, float>(sels, count);
    return band_kernel<8, double>(sels, count);
}

}  // namespace

bool band_has_wave_blocks(uint32_t sels, int32_t diags_per_lane, bool fp32)
{
    if (diags_per_lane != 8) return false;
    return (fp32 ? band_kernel4<8, float>(sels) : band_kernel4<8, double>(sels)) != nullptr;
}

hipError_t launch_sweep_band(const Batch &b, uint32_t sels, int32_t diags_per_lane, bool fp32,
                             int32_t grid, int32_t wpb, hipStream_t st)
{
    if (grid <= 0 || !(sels & (SEL_BAND | SEL_PGEN))) return hipSuccess;
    const void *k = band_kernel_for(sels, diags_per_lane, fp32, b.visits != nullptr);
    if (wpb == 4) {
        k = (diags_per_lane == 8 && b.visits == nullptr)
                ? (fp32 ? band_kernel4<8, float>(sels) : band_kernel4<8, double>(sels))
                : nullptr;
        if (!k || grid % 4) return hipErrorInvalidValue;
    } else if (wpb != 1) {
        return hipErrorInvalidValue;
    }
    Batch arg = b;
    void *args[] = {&arg};
    return hipLaunchKernel(k, dim3(grid / wpb), dim3(64 * wpb), args, 0, st);
}

int32_t band_blocks_per_cu(uint32_t sels, int32_t diags_per_lane, bool fp32)
{
    int nb = 0;
    const void *k = band_kernel_for(sels, diags_per_lane, fp32, false);
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, 64, 0);
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

}  // namespace mpk
