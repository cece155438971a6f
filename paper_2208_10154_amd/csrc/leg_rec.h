// Legendre recursion machinery shared by the contraction kernels (HIP, gfx950).
//
// A fill item is one north ring and one SEG-row segment of l: it starts from the
// seed pair stored for the segment (exponent-scaled, see k_seed.hip) and runs the
// three-term recursion in FP64 registers, handing every row to an emitter that
// stores it into the LDS operand tile in the contraction's format.
#pragma once
#include "leg_common.h"

namespace sht {
namespace {

template <int I>
struct IC {
    static constexpr int v = I;
};
template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (I < N) {
        f(IC<I>{});
        static_for<I + 1, N>(f);
    }
}

// wave index as a scalar (wave-uniform) value
__device__ __forceinline__ int wave_index() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

// sign flip by mask on the top bit (integer op: keeps the FP64 pipe free)
__device__ __forceinline__ double flip(double v, unsigned s)
{
    unsigned long long b = (unsigned long long)__double_as_longlong(v) ^ ((unsigned long long)s << 32);
    return __longlong_as_double((long long)b);
}
__device__ __forceinline__ float flip(float v, unsigned s) { return __uint_as_float(__float_as_uint(v) ^ s); }

// ----------------------------------------------------------------------------
// seeds and recursion state of one fill item (one ring, one SEG-row segment)
// ----------------------------------------------------------------------------
template <int SPIN>
struct Seed;
template <>
struct Seed<0> {
    double v0, v1, t;  // t = 1 - x, x = cos(theta) of the ring
    int k;
};
template <>
struct Seed<2> {
    double p0, p1, q0, q1, t;
    int k;
};

__device__ __forceinline__ void seed_load(Seed<0>& s, const LegArgs& a, int64_t idx, int r)
{
    s.v0 = a.mu[idx];
    s.v1 = a.mu[a.seedstride + idx];
    s.k = a.kk[idx];
    s.t = a.rings[r].omz;
}
__device__ __forceinline__ void seed_load(Seed<2>& s, const LegArgs& a, int64_t idx, int r)
{
    s.p0 = a.mu[idx];
    s.p1 = a.mu[a.seedstride + idx];
    s.q0 = a.mu[2 * a.seedstride + idx];
    s.q1 = a.mu[3 * a.seedstride + idx];
    s.k = a.kk[idx];
    s.t = a.rings[r].omz;
}

template <int SPIN>
struct Rec;
template <>
struct Rec<0> {
    double v0, v1, t;  // lambda at rows t-2, t-1 (scaled by 2^(600k)); t = 1 - x
    int k;
    bool any;  // a lane of the wave carried an exponent at the start (k never grows)
    // w: 1, 0.5 (equator ring in the map2alm fold) or 0 (no ring)
    __device__ __forceinline__ void start(const Seed<0>& s, double w)
    {
        v0 = w * s.v0;
        v1 = w * s.v1;
        t = s.t;
        k = s.k;
        any = __any(k > 0);
    }
};
template <>
struct Rec<2> {
    double a0, a1, b0, b1, t;  // F+ and F- at rows t-2, t-1; t = 1 - x
    int k;
    bool any;  // as in Rec<0>
    // F+- = -(P +- M)/2 from the seed pair (P = lambda_{+2}, M = lambda_{-2})
    __device__ __forceinline__ void start(const Seed<2>& s, double w)
    {
        const double h = -0.5 * w;
        a0 = h * (s.p0 + s.q0);
        a1 = h * (s.p1 + s.q1);
        b0 = h * (s.p0 - s.q0);
        b1 = h * (s.p1 - s.q1);
        t = s.t;
        k = s.k;
        any = __any(k > 0);
    }
};

// Destination of the rows of one fill item: even rows t go to e0, odd ones to e1
// (the two parity classes of l - m), (t >> 1) * STEP further on; the F- row of
// spin 2 sits FOFF after the F+ row.
template <typename T, int STEP, int FOFF>
struct Emit {
    T* e0;
    T* e1;
    template <int R>
    __device__ __forceinline__ void put(double v)
    {
        (R & 1 ? e1 : e0)[(R >> 1) * STEP] = (T)v;
    }
    template <int R>
    __device__ __forceinline__ void put(double p, double q)
    {
        T* d = (R & 1 ? e1 : e0) + (R >> 1) * STEP;
        d[0] = (T)p;
        d[FOFF] = (T)q;
    }
};

// Row R of a segment: rows 0 and 1 are the seed pair, later rows come from the
// recursion with that row's coefficients c (read beforehand from the coefficient
// tile in LDS).  Rows at or past cnt (beyond lmax) and values still carrying an
// exponent (k > 0: below 2^SIG_LOG2) are emitted as zeros.  The exponent handling is
// a branch taken only by waves that had a lane carrying an exponent when the
// segment started, marked unlikely so that the compiler keeps it out of the
// common path instead of evaluating it on every row and selecting.
template <int R, typename E>
__device__ __forceinline__ void rec_row(Rec<0>& f, const double (&c)[3], int cnt, E& em)
{
    double v;
    if constexpr (R == 0) {
        v = f.v0;
    } else if constexpr (R == 1) {
        v = f.v1;
    } else {
        // lambda_l = (a_l x) lambda_{l-1} - (a_l b_l) lambda_{l-2}, with a_l x formed
        // as a_l - a_l (1 - x): a rounded x near a pole would bias every row alike
        v = fma(-c[0], f.t, c[0]) * f.v1 - c[1] * f.v0;
        if (__builtin_expect(f.any, 0)) {
            if (f.k > 0 && fabs(v) > RESCALE_AT) {
                v *= SCALE_DOWN;
                f.v1 *= SCALE_DOWN;
                --f.k;
            }
        }
        f.v0 = f.v1;
        f.v1 = v;
    }
    em.template put<R>((f.k == 0 && R < cnt) ? v : 0.0);
}

template <int R, typename E>
__device__ __forceinline__ void rec_row(Rec<2>& f, const double (&c)[3], int cnt, E& em)
{
    double fp, fm;
    if constexpr (R == 0) {
        fp = f.a0;
        fm = f.b0;
    } else if constexpr (R == 1) {
        fp = f.a1;
        fm = f.b1;
    } else {
        // P_l = (al x + be) P_{l-1} - ga P_{l-2}, M_l = (al x - be) M_{l-1} - ga M_{l-2}
        // in the F+- basis: F+_l = al x F+_{l-1} + be F-_{l-1} - ga F+_{l-2} (and + <-> -)
        const double ax = fma(-c[0], f.t, c[0]), be = c[1], ga = c[2];  // al x as al - al (1 - x)
        fp = fma(ax, f.a1, fma(be, f.b1, -ga * f.a0));
        fm = fma(ax, f.b1, fma(be, f.a1, -ga * f.b0));
        if (__builtin_expect(f.any, 0)) {
            if (f.k > 0 && fmax(fabs(fp), fabs(fm)) > RESCALE_AT) {
                fp *= SCALE_DOWN;
                fm *= SCALE_DOWN;
                f.a1 *= SCALE_DOWN;
                f.b1 *= SCALE_DOWN;
                --f.k;
            }
        }
        f.a0 = f.a1;
        f.a1 = fp;
        f.b0 = f.b1;
        f.b1 = fm;
    }
    const bool z = f.k == 0 && R < cnt;
    em.template put<R>(z ? fp : 0.0, z ? fm : 0.0);
}

// rows RPG * G .. RPG * G + RPG - 1 of a segment (one interleave group): the
// group's coefficients are read from LDS first (one wait), then the rows run.
// cp: the segment's rows of the coefficient tile (CS = 2 doubles a row for spin
// 0, 4 for spin 2); the address is wave-uniform, a broadcast read.
template <int G, int RPG, int SPIN, typename E>
__device__ __forceinline__ void rec_group(Rec<SPIN>& f, const double* cp, int cnt, E& em)
{
    constexpr int CS = SPIN == 0 ? 2 : 4, NC = SPIN == 0 ? 2 : 3;
    double c[RPG][3];
    static_for<0, RPG>([&](auto q) {
        constexpr int R = RPG * G + decltype(q)::v;
        if constexpr (R >= 2) {
#pragma unroll
            for (int i = 0; i < NC; ++i) c[decltype(q)::v][i] = cp[CS * R + i];
        }
    });
    static_for<0, RPG>([&](auto q) { rec_row<RPG * G + decltype(q)::v>(f, c[decltype(q)::v], cnt, em); });
}

// a whole segment (prologue)
template <int SPIN, typename E>
__device__ __forceinline__ void rec_all(Rec<SPIN>& f, const double* cp, int cnt, E& em)
{
    static_assert(SEG % 4 == 0, "segments are run in groups of four rows");
    static_for<0, SEG / 4>([&](auto g) { rec_group<decltype(g)::v, 4>(f, cp, cnt, em); });
}

template <typename T>
__device__ __forceinline__ T* xptr(const LegArgs& a, int comp)
{
    return static_cast<T*>(a.X) + (int64_t)comp * a.xcomp;
}
template <typename T>
__device__ __forceinline__ T* aptr(const LegArgs& a, int comp)
{
    return static_cast<T*>(a.A) + (int64_t)comp * a.acomp;
}

// m2a work decode: logical g -> (m, lt, ct); off[i] = l tiles of the first i m in
// folded order.
__device__ __forceinline__ void decode_tiles(const LegArgs& a, int g, int& m, int& lt, int& ct)
{
    const int* off = a.tiles;
    const int C = a.ctiles;
    int lo = 0, hi = a.mlist ? a.nlist : a.lmax + 1;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (off[mid] * C <= g) lo = mid; else hi = mid;
    }
    m = a.mlist ? a.mlist[lo] : mfold(lo, a.lmax);
    int r = g - off[lo] * C;
    int nlt = off[lo + 1] - off[lo];
    ct = r / nlt;
    lt = r - ct * nlt;
}

// m values an alm2map launch covers (all, or the listed ones)
__host__ __device__ inline int nm_rows(const LegArgs& a) { return a.mlist ? a.nlist : a.lmax + 1; }

// workgroups per reduction range (see LegArgs::ksplit)
__host__ __device__ inline int kparts(const LegArgs& a) { return a.ksplit > 1 ? a.ksplit : 1; }

// part of a split range this workgroup takes; g becomes the unsplit index
__device__ __forceinline__ int split_part(const LegArgs& a, int& g)
{
    if (a.ksplit <= 1) return 0;
    const int s = g % a.ksplit;
    g /= a.ksplit;
    return s;
}

// narrow [b, e) to part s of the split
__device__ __forceinline__ void split_range(const LegArgs& a, int s, int& b, int& e)
{
    if (a.ksplit <= 1) return;
    const int len = (e - b + a.ksplit - 1) / a.ksplit;
    b = min(e, b + s * len);
    e = min(e, b + len);
}

// output store, or an atomic add when the reduction is split over workgroups
template <typename T>
__device__ __forceinline__ void put_out(T* p, T v, bool add)
{
    if (add) atomicAdd(p, v);
    else *p = v;
}

// first ring chunk whose significance bound reaches an l <= lend
__device__ __forceinline__ int first_chunk(const LegArgs& a, int m, int nchunk, int lend)
{
    int rc = 0;
    while (rc < nchunk && a.lsig[(int64_t)m * a.nrc + rc] > lend) ++rc;
    return __builtin_amdgcn_readfirstlane(rc);
}

// fill weight of north ring r in the map2alm fold
__device__ __forceinline__ double m2a_weight(const LegArgs& a, int r)
{
    return (r >= a.rn) ? 0.0 : (2 * r + 1 == a.nring ? 0.5 : 1.0);
}

// alm2map tile bounds shared by both spins: first l tile start (a whole number of
// tiles past lb, at or below the first significant l of the ring tile) and the
// number of l tiles.
__device__ __forceinline__ void a2m_range(const LegArgs& a, int m, int lb, int r0, int tr, int& lfirst, int& nch)
{
    const int L = a.lmax;
    int lsig = L + 1;
    if (lb <= L)
        for (int c = r0 / RCHUNK; c < min(a.nrc, (r0 + tr + RCHUNK - 1) / RCHUNK); ++c)
            lsig = min(lsig, a.lsig[(int64_t)m * a.nrc + c]);
    // the table loads make these look lane-dependent to the compiler; they are
    // wave-uniform, and the coefficient addresses built from them must be too
    lfirst = __builtin_amdgcn_readfirstlane((lsig > L) ? L + 1 : lb + TL * ((lsig - lb) / TL));
    nch = __builtin_amdgcn_readfirstlane((lfirst > L) ? 0 : (L - lfirst) / TL + 1);
}

// Coefficient tile of one 64-row l tile in LDS: row r (l = l0 + r) at
// tile[CS * r .. CS * r + CS - 1], CS = 2 (spin 0) or 4 (spin 2).  Every thread
// issues one unpredicated load (a duplicate for threads past the tile) so the
// load takes its place in the in-order vector-memory queue; only threads inside
// the tile store.  The recursion then reads its coefficients from LDS, whose
// operations complete in order, instead of through scalar loads that share a wait
// counter with LDS and force it to drain.
template <int CS>
struct CoefTile {
    static constexpr int N = TL * CS;
    static_assert((N & (N - 1)) == 0 && N <= 256, "one load per thread");
    __device__ __forceinline__ static double fetch(const LegArgs& a, int64_t first_row)
    {
        return a.coef[first_row * CS + (threadIdx.x & (N - 1))];
    }
    __device__ __forceinline__ static void put(double* tile, double v)
    {
        if (threadIdx.x < N) tile[threadIdx.x] = v;
    }
};

}  // namespace
}  // namespace sht
