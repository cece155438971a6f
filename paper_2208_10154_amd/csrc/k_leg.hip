// Fused Legendre recursion + MFMA contraction (HIP, gfx950).
//
// For every m the paper reduces the transform to dense products over the map
// batch (Sec. 2.2, eq. "matrix form"):
//     map2alm   A_m = P_m T_m      (contracts rings; dsigma is applied later)
//     alm2map   T_m = P_m^t A_m    (contracts l)
// and, for polarisation, the real 2x2 block form of Sec. 2.3,
//     [A^E; iA^B]_m = [[F+, F-], [F-, F+]]_m [Q; iU]_m,   F+- = -lambda+-,
//     lambda+- = (2lambda +- -2lambda)/2 (Appendix A.2),
// with iA^B and iU as the natural real variables (Sec. 3.1 item 1).
//
// The P_m / F+- tiles are never stored in HBM: each workgroup runs the
// three-term recursion in FP64 registers from the plan's seed table
// (exponent-scaled, see k_seed.hip) and writes the tile to a double-buffered LDS
// array in the operand precision; the recursion for the next tile is interleaved
// with the MFMAs of the current one, four recursion rows per MFMA K-step.  The
// other MFMA operand (ring coefficients T_m for map2alm, coefficients A_m for
// alm2map) comes from HBM in the m-major layouts [m][ring][column] and
// [m][l][column], one K-step ahead, straight into registers.  The two
// hemispheres are folded with lambda_lm(-z) = (-1)^{l+m} lambda_lm(z)
// (lambda+-(-z) = +-(-1)^{l+m} lambda+-(z)): only northern rings are contracted,
// rows of even l-m against T_N + T_S and odd ones against T_N - T_S.  Column
// pairs (2k, 2k+1) are the real and imaginary parts of map k.
//
// Structure chosen for CDNA4:
//  * FP64 VALU work and FP64 MFMAs share one pipe, so the recursion is kept to
//    the minimum FP64 instructions per row (spin 2 runs the coupled F+/F-
//    recursion, so emitting a row needs no arithmetic) and its cost is spread
//    over as many MFMA columns per wave as the register file allows.
//  * Recursion coefficients come from a per-(m, l) table through scalar loads:
//    a fill segment is wave-uniform, so every lane of a wave needs the same row.
//  * Every global load is unpredicated (indices clamped into range) and issued in
//    the same order each K-step, so the compiler's wait counts stay exact and a
//    wave only ever waits for the operand it is about to use.  Rows past lmax and
//    rings past the equator read clamped, finite data and meet exact zeros in
//    the recursion tile; the equator ring, whose north and south rows coincide,
//    enters the map2alm fold with its seeds halved.
#include "leg_common.h"

namespace sht {
namespace {

constexpr int NT = 256;
constexpr int HALF = TL / 2;   // rows of one parity class per l tile
constexpr int KS = 8;          // MFMA K-steps per tile (4 rings, or 4 l per class, each)
constexpr int RPK = SEG / KS;  // recursion rows emitted per K-step
static_assert(RPK == 4, "the fill of one segment is spread over the K-steps of a tile");
constexpr int M_TR = 32;       // map2alm: rings per chunk (= RCHUNK, the skip granularity)
static_assert(M_TR == RCHUNK, "ring chunks and skip-table entries coincide");

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

// Read-only table pointer in the constant address space: with a wave-uniform
// address its loads become scalar loads (one per wave, into SGPRs).
using cptr = const __attribute__((address_space(4))) double*;
__device__ __forceinline__ cptr to_const(const double* p)
{
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Wold-style-cast"
    return (cptr)(p);
#pragma clang diagnostic pop
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
    double v0, v1, x;
    int k;
};
template <>
struct Seed<2> {
    double p0, p1, q0, q1, x;
    int k;
};

__device__ __forceinline__ void seed_load(Seed<0>& s, const LegArgs& a, int64_t idx, int r)
{
    s.v0 = a.mu[idx];
    s.v1 = a.mu[a.seedstride + idx];
    s.k = a.kk[idx];
    s.x = a.rings[r].z;
}
__device__ __forceinline__ void seed_load(Seed<2>& s, const LegArgs& a, int64_t idx, int r)
{
    s.p0 = a.mu[idx];
    s.p1 = a.mu[a.seedstride + idx];
    s.q0 = a.mu[2 * a.seedstride + idx];
    s.q1 = a.mu[3 * a.seedstride + idx];
    s.k = a.kk[idx];
    s.x = a.rings[r].z;
}

template <int SPIN>
struct Rec;
template <>
struct Rec<0> {
    double v0, v1, x;  // lambda at rows t-2, t-1 (scaled by 2^(600k))
    int k;
    // w: 1, 0.5 (equator ring in the map2alm fold) or 0 (no ring)
    __device__ __forceinline__ void start(const Seed<0>& s, double w)
    {
        v0 = w * s.v0;
        v1 = w * s.v1;
        x = s.x;
        k = s.k;
    }
};
template <>
struct Rec<2> {
    double a0, a1, b0, b1, x;  // F+ and F- at rows t-2, t-1
    int k;
    // F+- = -(P +- M)/2 from the seed pair (P = lambda_{+2}, M = lambda_{-2})
    __device__ __forceinline__ void start(const Seed<2>& s, double w)
    {
        const double h = -0.5 * w;
        a0 = h * (s.p0 + s.q0);
        a1 = h * (s.p1 + s.q1);
        b0 = h * (s.p0 - s.q0);
        b1 = h * (s.p1 - s.q1);
        x = s.x;
        k = s.k;
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
// recursion with coefficient row R of the segment (cp: wave-uniform pointer).
// Rows at or past cnt (beyond lmax) and values still carrying an exponent
// (k > 0: below 2^-100) are emitted as zeros.
template <int R, typename E>
__device__ __forceinline__ void rec_row(Rec<0>& f, cptr cp, int cnt, E& em)
{
    double v;
    if constexpr (R == 0) {
        v = f.v0;
    } else if constexpr (R == 1) {
        v = f.v1;
    } else {
        // lambda_l = (a_l x) lambda_{l-1} - (a_l b_l) lambda_{l-2}
        v = (cp[2 * R] * f.x) * f.v1 - cp[2 * R + 1] * f.v0;
        if (__any(f.k > 0)) {
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
__device__ __forceinline__ void rec_row(Rec<2>& f, cptr cp, int cnt, E& em)
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
        const double ax = cp[4 * R] * f.x, be = cp[4 * R + 1], ga = cp[4 * R + 2];
        fp = fma(ax, f.a1, fma(be, f.b1, -ga * f.a0));
        fm = fma(ax, f.b1, fma(be, f.a1, -ga * f.b0));
        if (__any(f.k > 0)) {
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

// the RPK rows emitted during K-step KI
template <int KI, int SPIN, typename E>
__device__ __forceinline__ void rec_group(Rec<SPIN>& f, cptr cp, int cnt, E& em)
{
    static_for<0, RPK>([&](auto q) { rec_row<RPK * KI + decltype(q)::v>(f, cp, cnt, em); });
}

// a whole segment (prologue)
template <int SPIN, typename E>
__device__ __forceinline__ void rec_all(Rec<SPIN>& f, cptr cp, int cnt, E& em)
{
    static_for<0, KS>([&](auto ki) { rec_group<decltype(ki)::v>(f, cp, cnt, em); });
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
__device__ __forceinline__ void decode_tiles(const int* off, int lmax, int C, int g, int& m, int& lt, int& ct)
{
    int lo = 0, hi = lmax + 1;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (off[mid] * C <= g) lo = mid; else hi = mid;
    }
    m = mfold(lo, lmax);
    int r = g - off[lo] * C;
    int nlt = off[lo + 1] - off[lo];
    ct = r / nlt;
    lt = r - ct * nlt;
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

// ============================================================================
// map2alm, spin 0: A_l = sum_{north rings} lambda_l (T_N +- T_S), raw sums into
// the m-major coefficient workspace.  Tile: 64 l x 64*NU columns; rings in
// chunks of 32; wave w owns NU column tiles of 16 and all 64 rows.
// ============================================================================
template <typename T, int NU>
__global__ __launch_bounds__(NT, 2) void k_m2a_spin0(LegArgs a)
{
    constexpr int RS = HALF + 1;        // [ring][row/2]
    constexpr int CLS = M_TR * RS, BUF = 2 * CLS;
    __shared__ T lam[2 * BUF];          // [buffer][parity class][ring][row/2]

    int m, lt, ct;
    decode_tiles(a.tiles, a.lmax, a.ctiles, xcd_remap(blockIdx.x, gridDim.x), m, lt, ct);
    const int L = a.lmax, lb = m;
    const int l0 = lb + lt * TL, lend = min(L, l0 + TL - 1);
    const int lane = threadIdx.x & 63, wave = wave_index();
    const int col = ct * (64 * NU) + 16 * NU * wave + (lane & 15);
    // fill items: 32 rings x 2 segments; lanes 0..15 compute, every lane loads
    const bool filler = lane < 16;
    const int frl = 16 * (wave & 1) + (lane & 15);
    const int fs = wave >> 1;
    const int ls = l0 + SEG * fs;
    const int cnt = min(SEG, L - ls + 1);
    const int64_t row0 = a.rowoff[m];
    const cptr cp = to_const(a.coef) + (row0 + (ls - lb)) * 2;
    const int jseg = min(2 * lt + fs, (L - lb) / SEG);
    const int64_t sbase = a.seedoff[m] + (int64_t)jseg * a.rn;

    using MF = Mfma<T>;
    typename MF::acc acc[2][2][NU];  // [parity][row tile][column tile]
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int u = 0; u < NU; ++u) acc[p][t][u] = typename MF::acc{0, 0, 0, 0};

    const int nchunk = (a.rn + M_TR - 1) / M_TR;
    const int rc0 = first_chunk(a, m, nchunk, lend);
    if (rc0 < nchunk) {
        const T* Xm = xptr<T>(a, 0) + (int64_t)m * a.nring * a.ldx + col;
        auto seed_of = [&](Seed<0>& s, int rc) {
            const int r = min(rc * M_TR + frl, a.rn - 1);
            seed_load(s, a, sbase + r, r);
        };
        auto emit_to = [&](int b) {
            Emit<T, 1, 0> e;
            e.e0 = lam + b * BUF + frl * RS + 16 * fs;
            e.e1 = e.e0 + CLS;
            return e;
        };
        // ring operands of one K-step: north / south rows
        T xb[2][2][NU];  // [K-step parity][north, south][column tile]
        auto load_x = [&](int rc, int ks, T (&d)[2][NU]) {
            const int r = min(rc * M_TR + 4 * ks + (lane >> 4), a.rn - 1);
            const T* pn = Xm + (int64_t)r * a.ldx;
            const T* ps = Xm + (int64_t)(a.nring - 1 - r) * a.ldx;
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                d[0][u] = pn[16 * u];
                d[1][u] = ps[16 * u];
            }
        };

        Seed<0> sd;
        Rec<0> f;
        seed_of(sd, rc0);
        if (filler) {
            f.start(sd, m2a_weight(a, rc0 * M_TR + frl));
            auto em = emit_to(0);
            rec_all(f, cp, cnt, em);
        }
        seed_of(sd, min(rc0 + 1, nchunk - 1));
        load_x(rc0, 0, xb[0]);
        __syncthreads();
        for (int rc = rc0; rc < nchunk; ++rc) {
            const int b = (rc - rc0) & 1;
            const int rcn = min(rc + 1, nchunk - 1);
            if (filler) f.start(sd, m2a_weight(a, rcn * M_TR + frl));
            auto em = emit_to(b ^ 1);
            const T* lb_ = lam + b * BUF;
            static_for<0, KS>([&](auto ki) {
                constexpr int ks = decltype(ki)::v;
                if constexpr (ks + 1 < KS) load_x(rc, ks + 1, xb[(ks + 1) & 1]);
                else load_x(rcn, 0, xb[0]);
                if constexpr (ks == KS / 2) seed_of(sd, min(rc + 2, nchunk - 1));
                // keep the prefetch ahead of this step's compute (the scheduler may sink it)
                __builtin_amdgcn_sched_barrier(0);
                const int kr = 4 * ks + (lane >> 4);
                T av[2][2];
#pragma unroll
                for (int p = 0; p < 2; ++p)
#pragma unroll
                    for (int t = 0; t < 2; ++t) av[p][t] = lb_[p * CLS + kr * RS + 16 * t + (lane & 15)];
#pragma unroll
                for (int u = 0; u < NU; ++u) {
                    const T bs = xb[ks & 1][0][u] + xb[ks & 1][1][u];
                    const T bd = xb[ks & 1][0][u] - xb[ks & 1][1][u];
#pragma unroll
                    for (int t = 0; t < 2; ++t) {
                        acc[0][t][u] = MF::run(av[0][t], bs, acc[0][t][u]);
                        acc[1][t][u] = MF::run(av[1][t], bd, acc[1][t][u]);
                    }
                }
                if (filler) rec_group<ks>(f, cp, cnt, em);
            });
            __syncthreads();
        }
    }

    // store raw sums: row index within a parity class -> l
    T* A = aptr<T>(a, 0) + row0 * a.ldx;
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int ci = 16 * t + MF::row(lane, v);
                const int l = l0 + 2 * ci + p;
                if (l > L) continue;
#pragma unroll
                for (int u = 0; u < NU; ++u) A[(int64_t)(l - lb) * a.ldx + col + 16 * u] = (T)acc[p][t][u][v];
            }
}

// ============================================================================
// map2alm, spin 2 (E and iB from Q and iU):
//   even l-m: A_E = F+ SX + F- DY,  iA_B = F+ SY + F- DX
//   odd  l-m: A_E = F+ DX + F- SY,  iA_B = F+ DY + F- SX
// X = Q coefficients, Y = iU; S/D = north +- south.  Tile 64 l x 64*NU columns,
// rings in chunks of 32; wave w owns NU column tiles of 16.
// ============================================================================
template <typename T, int NU>
__global__ __launch_bounds__(NT, 2) void k_m2a_spin2(LegArgs a)
{
    constexpr int RS = HALF + 1;
    constexpr int CLS = M_TR * RS, FOFF = 2 * CLS, BUF = 4 * CLS;
    __shared__ T fpm[2 * BUF];  // [buffer][F+ / F-][parity class][ring][row/2]

    int m, lt, ct;
    decode_tiles(a.tiles, a.lmax, a.ctiles, xcd_remap(blockIdx.x, gridDim.x), m, lt, ct);
    const int L = a.lmax, lb = lbase(2, m);
    const int l0 = lb + lt * TL, lend = min(L, l0 + TL - 1);
    const int po = (lb - m) & 1;
    const int lane = threadIdx.x & 63, wave = wave_index();
    const int col = ct * (64 * NU) + 16 * NU * wave + (lane & 15);
    const int pcol = col ^ 1;                           // Y = iU swaps re/im: partner column
    const unsigned ysg = (col & 1) ? 0u : 0x80000000u;  // Y_re = -U_im, Y_im = U_re
    const bool filler = lane < 16;
    const int frl = 16 * (wave & 1) + (lane & 15);
    const int fs = wave >> 1;
    const int ls = l0 + SEG * fs;
    const int cnt = min(SEG, L - ls + 1);
    const int64_t row0 = a.rowoff[m];
    const cptr cp = to_const(a.coef) + (row0 + (ls - lb)) * 4;
    const int jseg = min(2 * lt + fs, (L - lb) / SEG);
    const int64_t sbase = a.seedoff[m] + (int64_t)jseg * a.rn;

    using MF = Mfma<T>;
    typename MF::acc accE[2][2][NU], accB[2][2][NU];  // [parity][row tile][column tile]
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int u = 0; u < NU; ++u) accE[p][t][u] = accB[p][t][u] = typename MF::acc{0, 0, 0, 0};

    const int nchunk = (a.rn + M_TR - 1) / M_TR;
    const int rc0 = first_chunk(a, m, nchunk, lend);
    if (rc0 < nchunk) {
        const int64_t xm = (int64_t)m * a.nring * a.ldx;
        const T* XQ = xptr<T>(a, 1) + xm + col;
        const T* XU = xptr<T>(a, 2) + xm + pcol;
        auto seed_of = [&](Seed<2>& s, int rc) {
            const int r = min(rc * M_TR + frl, a.rn - 1);
            seed_load(s, a, sbase + r, r);
        };
        auto emit_to = [&](int b) {
            Emit<T, 1, FOFF> e;
            e.e0 = fpm + b * BUF + po * CLS + frl * RS + 16 * fs;
            e.e1 = fpm + b * BUF + (po ^ 1) * CLS + frl * RS + 16 * fs;
            return e;
        };
        T xb[2][4][NU];  // [K-step parity][Q_N, Q_S, U_N, U_S (partner column)][column tile]
        auto load_x = [&](int rc, int ks, T (&d)[4][NU]) {
            const int r = min(rc * M_TR + 4 * ks + (lane >> 4), a.rn - 1);
            const int64_t on = (int64_t)r * a.ldx, os = (int64_t)(a.nring - 1 - r) * a.ldx;
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                d[0][u] = XQ[on + 16 * u];
                d[1][u] = XQ[os + 16 * u];
                d[2][u] = XU[on + 16 * u];
                d[3][u] = XU[os + 16 * u];
            }
        };

        Seed<2> sd;
        Rec<2> f;
        seed_of(sd, rc0);
        if (filler) {
            f.start(sd, m2a_weight(a, rc0 * M_TR + frl));
            auto em = emit_to(0);
            rec_all(f, cp, cnt, em);
        }
        seed_of(sd, min(rc0 + 1, nchunk - 1));
        load_x(rc0, 0, xb[0]);
        __syncthreads();
        for (int rc = rc0; rc < nchunk; ++rc) {
            const int b = (rc - rc0) & 1;
            const int rcn = min(rc + 1, nchunk - 1);
            if (filler) f.start(sd, m2a_weight(a, rcn * M_TR + frl));
            auto em = emit_to(b ^ 1);
            const T* fb = fpm + b * BUF;
            static_for<0, KS>([&](auto ki) {
                constexpr int ks = decltype(ki)::v;
                if constexpr (ks + 1 < KS) load_x(rc, ks + 1, xb[(ks + 1) & 1]);
                else load_x(rcn, 0, xb[0]);
                if constexpr (ks == KS / 2) seed_of(sd, min(rc + 2, nchunk - 1));
                // keep the prefetch ahead of this step's compute (the scheduler may sink it)
                __builtin_amdgcn_sched_barrier(0);
                const int kr = 4 * ks + (lane >> 4);
                T fp[2][2], fm[2][2];  // [parity][row tile]
#pragma unroll
                for (int p = 0; p < 2; ++p)
#pragma unroll
                    for (int t = 0; t < 2; ++t) {
                        fp[p][t] = fb[p * CLS + kr * RS + 16 * t + (lane & 15)];
                        fm[p][t] = fb[FOFF + p * CLS + kr * RS + 16 * t + (lane & 15)];
                    }
#pragma unroll
                for (int u = 0; u < NU; ++u) {
                    const T(&d)[4][NU] = xb[ks & 1];
                    const T sx = d[0][u] + d[1][u], dx = d[0][u] - d[1][u];
                    const T sy = flip((T)(d[2][u] + d[3][u]), ysg), dy = flip((T)(d[2][u] - d[3][u]), ysg);
#pragma unroll
                    for (int t = 0; t < 2; ++t) {
                        accE[0][t][u] = MF::run(fp[0][t], sx, accE[0][t][u]);
                        accB[0][t][u] = MF::run(fp[0][t], sy, accB[0][t][u]);
                        accE[1][t][u] = MF::run(fp[1][t], dx, accE[1][t][u]);
                        accB[1][t][u] = MF::run(fp[1][t], dy, accB[1][t][u]);
                    }
#pragma unroll
                    for (int t = 0; t < 2; ++t) {
                        accE[0][t][u] = MF::run(fm[0][t], dy, accE[0][t][u]);
                        accB[0][t][u] = MF::run(fm[0][t], dx, accB[0][t][u]);
                        accE[1][t][u] = MF::run(fm[1][t], sy, accE[1][t][u]);
                        accB[1][t][u] = MF::run(fm[1][t], sx, accB[1][t][u]);
                    }
                }
                if (filler) rec_group<ks>(f, cp, cnt, em);
            });
            __syncthreads();
        }
    }

    T* AE = aptr<T>(a, 1) + row0 * a.ldx;
    T* AB = aptr<T>(a, 2) + row0 * a.ldx;
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int ci = 16 * t + MF::row(lane, v);
                const int l = l0 + 2 * ci + (p ^ po);
                if (l > L) continue;
#pragma unroll
                for (int u = 0; u < NU; ++u) {
                    const int64_t o = (int64_t)(l - lb) * a.ldx + col + 16 * u;
                    AE[o] = (T)accE[p][t][u][v];
                    AB[o] = (T)accB[p][t][u][v];
                }
            }
}

// alm2map tile bounds shared by both spins: first l tile start (an even number of
// segments past lb, at or below the first significant l of the ring tile) and
// the number of l tiles.
__device__ __forceinline__ void a2m_range(const LegArgs& a, int m, int lb, int r0, int tr, int& lfirst, int& nch)
{
    const int L = a.lmax;
    int lsig = L + 1;
    if (lb <= L)
        for (int c = r0 / RCHUNK; c < min(a.nrc, (r0 + tr + RCHUNK - 1) / RCHUNK); ++c)
            lsig = min(lsig, a.lsig[(int64_t)m * a.nrc + c]);
    // the table loads make these look lane-dependent to the compiler; they are
    // wave-uniform, and the coefficient addresses built from them must be too
    lfirst = __builtin_amdgcn_readfirstlane((lsig > L) ? L + 1 : lb + SEG * (((lsig - lb) / SEG) & ~1));
    nch = __builtin_amdgcn_readfirstlane((lfirst > L) ? 0 : (L - lfirst) / TL + 1);
}

// ============================================================================
// alm2map, spin 0: E = sum_{even l-m} lambda A, O = sum_{odd} lambda A,
// T_N = E + O, T_S = E - O.  Tile: 64 rings x 64*NU columns, l in chunks of 64;
// wave w owns NU column tiles of 16 and all 64 rings.
// ============================================================================
constexpr int A0_TR = 64;

template <typename T, int NU>
__global__ __launch_bounds__(NT, 2) void k_a2m_spin0(LegArgs a)
{
    constexpr int RS = A0_TR + 1;       // [row/2][ring]
    constexpr int CLS = HALF * RS, BUF = 2 * CLS;
    __shared__ T lam[2 * BUF];          // [buffer][parity class][row/2][ring]

    const int nrt = (a.rn + A0_TR - 1) / A0_TR;
    const int g = xcd_remap(blockIdx.x, gridDim.x);
    const int mi = g / (a.ctiles * nrt);
    const int m = mfold(mi, a.lmax);
    const int rem = g - mi * a.ctiles * nrt;
    const int ct = rem / nrt, rt = rem - ct * nrt;
    const int L = a.lmax, lb = m;
    const int r0 = rt * A0_TR;
    const int lane = threadIdx.x & 63, wave = wave_index();
    const int col = ct * (64 * NU) + 16 * NU * wave + (lane & 15);
    // fill items: 64 rings x 2 segments; lanes 0..31 compute, every lane loads
    const bool filler = lane < 32;
    const int frl = 32 * (wave & 1) + (lane & 31);
    const int fs = wave >> 1;
    const int fr = r0 + frl;
    const int frc = min(fr, a.rn - 1);
    const double w = fr < a.rn ? 1.0 : 0.0;

    int lfirst, nch;
    a2m_range(a, m, lb, r0, A0_TR, lfirst, nch);

    using MF = Mfma<T>;
    typename MF::acc accE[4][NU], accO[4][NU];  // [ring tile][column tile]
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int u = 0; u < NU; ++u) accE[t][u] = accO[t][u] = typename MF::acc{0, 0, 0, 0};

    if (nch > 0) {
        const int64_t row0 = a.rowoff[m];
        const T* Am = aptr<T>(a, 0) + row0 * a.ldx + col;
        const cptr cm = to_const(a.coef) + row0 * 2;
        const int64_t sb = a.seedoff[m] + frc;
        const int j0 = (lfirst - lb) / SEG + fs;
        const int jmax = (L - lb) / SEG;  // last segment of this m
        auto seed_of = [&](Seed<0>& s, int c) { seed_load(s, a, sb + (int64_t)min(j0 + 2 * c, jmax) * a.rn, frc); };
        auto ls_of = [&](int c) { return lfirst + TL * c + SEG * fs; };
        auto emit_to = [&](int b) {
            Emit<T, RS, 0> e;
            e.e0 = lam + b * BUF + 16 * fs * RS + frl;
            e.e1 = e.e0 + CLS;
            return e;
        };
        T bb[2][2][NU];  // [K-step parity][even, odd class row][column tile]
        auto load_a = [&](int c, int ks, T (&d)[2][NU]) {
            const int le = lfirst + TL * c + 2 * (4 * ks + (lane >> 4));
            const T* pe = Am + (int64_t)(min(le, L) - lb) * a.ldx;
            const T* pq = Am + (int64_t)(min(le + 1, L) - lb) * a.ldx;
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                d[0][u] = pe[16 * u];
                d[1][u] = pq[16 * u];
            }
        };

        Seed<0> sd;
        Rec<0> f;
        seed_of(sd, 0);
        if (filler) {
            f.start(sd, w);
            auto em = emit_to(0);
            rec_all(f, cm + (int64_t)__builtin_amdgcn_readfirstlane(ls_of(0) - lb) * 2, min(SEG, L - ls_of(0) + 1), em);
        }
        seed_of(sd, min(1, nch - 1));
        load_a(0, 0, bb[0]);
        __syncthreads();
        for (int c = 0; c < nch; ++c) {
            const int b = c & 1;
            const int cn = min(c + 1, nch - 1);
            const cptr cp = cm + (int64_t)__builtin_amdgcn_readfirstlane(ls_of(cn) - lb) * 2;
            const int cnt = min(SEG, L - ls_of(cn) + 1);
            if (filler) f.start(sd, w);
            auto em = emit_to(b ^ 1);
            const T* lb_ = lam + b * BUF;
            static_for<0, KS>([&](auto ki) {
                constexpr int ks = decltype(ki)::v;
                if constexpr (ks + 1 < KS) load_a(c, ks + 1, bb[(ks + 1) & 1]);
                else load_a(cn, 0, bb[0]);
                if constexpr (ks == KS / 2) seed_of(sd, min(c + 2, nch - 1));
                // keep the prefetch ahead of this step's compute (the scheduler may sink it)
                __builtin_amdgcn_sched_barrier(0);
                const int kl = 4 * ks + (lane >> 4);
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const T aE = lb_[kl * RS + 16 * t + (lane & 15)];
                    const T aO = lb_[CLS + kl * RS + 16 * t + (lane & 15)];
#pragma unroll
                    for (int u = 0; u < NU; ++u) {
                        accE[t][u] = MF::run(aE, bb[ks & 1][0][u], accE[t][u]);
                        accO[t][u] = MF::run(aO, bb[ks & 1][1][u], accO[t][u]);
                    }
                }
                if (filler) rec_group<ks>(f, cp, cnt, em);
            });
            __syncthreads();
        }
    }

    T* X = xptr<T>(a, 0) + (int64_t)m * a.nring * a.ldx + col;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = r0 + 16 * t + MF::row(lane, v);
            if (r >= a.rn) continue;
            const int rs = a.nring - 1 - r;
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const T e = accE[t][u][v], o = accO[t][u][v];
                X[(int64_t)r * a.ldx + 16 * u] = e + o;
                if (rs != r) X[(int64_t)rs * a.ldx + 16 * u] = e - o;
            }
        }
}

// ============================================================================
// alm2map, spin 2, with B' = i a_B:
//   U1 = sum_even F+ E + sum_odd F- B',  U2 = sum_odd F+ E + sum_even F- B'
//   V1 = sum_even F+ B' + sum_odd F- E,  V2 = sum_odd F+ B' + sum_even F- E
//   Q_N = U1 + U2, Q_S = U1 - U2;  (iU)_N = V1 + V2, (iU)_S = V1 - V2.
// Tile: 32 rings x 64*NU columns; wave w owns NU column tiles of 16.
// ============================================================================
constexpr int A2_TR = 32;

template <typename T, int NU>
__global__ __launch_bounds__(NT, 2) void k_a2m_spin2(LegArgs a)
{
    constexpr int RS = A2_TR + 1;
    constexpr int CLS = HALF * RS, FOFF = 2 * CLS, BUF = 4 * CLS;
    __shared__ T fpm[2 * BUF];  // [buffer][F+ / F-][parity class][row/2][ring]

    const int nrt = (a.rn + A2_TR - 1) / A2_TR;
    const int g = xcd_remap(blockIdx.x, gridDim.x);
    const int mi = g / (a.ctiles * nrt);
    const int m = mfold(mi, a.lmax);
    const int rem = g - mi * a.ctiles * nrt;
    const int ct = rem / nrt, rt = rem - ct * nrt;
    const int L = a.lmax, lb = lbase(2, m);
    const int po = (lb - m) & 1;
    const int r0 = rt * A2_TR;
    const int lane = threadIdx.x & 63, wave = wave_index();
    const int col = ct * (64 * NU) + 16 * NU * wave + (lane & 15);
    const bool filler = lane < 16;
    const int frl = 16 * (wave & 1) + (lane & 15);
    const int fs = wave >> 1;
    const int fr = r0 + frl;
    const int frc = min(fr, a.rn - 1);
    const double w = fr < a.rn ? 1.0 : 0.0;

    int lfirst, nch;
    a2m_range(a, m, lb, r0, A2_TR, lfirst, nch);

    using MF = Mfma<T>;
    typename MF::acc u1[2][NU], u2[2][NU], v1[2][NU], v2[2][NU];  // [ring tile][column tile]
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < NU; ++u) u1[t][u] = u2[t][u] = v1[t][u] = v2[t][u] = typename MF::acc{0, 0, 0, 0};

    if (nch > 0) {
        const int64_t row0 = a.rowoff[m];
        const T* AE = aptr<T>(a, 1) + row0 * a.ldx + col;
        const T* AB = aptr<T>(a, 2) + row0 * a.ldx + col;
        const cptr cm = to_const(a.coef) + row0 * 4;
        const int64_t sb = a.seedoff[m] + frc;
        const int j0 = (lfirst - lb) / SEG + fs;
        const int jmax = (L - lb) / SEG;  // last segment of this m
        auto seed_of = [&](Seed<2>& s, int c) { seed_load(s, a, sb + (int64_t)min(j0 + 2 * c, jmax) * a.rn, frc); };
        auto ls_of = [&](int c) { return lfirst + TL * c + SEG * fs; };
        auto emit_to = [&](int b) {
            Emit<T, RS, FOFF> e;
            e.e0 = fpm + b * BUF + po * CLS + 16 * fs * RS + frl;
            e.e1 = fpm + b * BUF + (po ^ 1) * CLS + 16 * fs * RS + frl;
            return e;
        };
        T bb[2][4][NU];  // [K-step parity][E even, E odd, B' even, B' odd][column tile]
        auto load_a = [&](int c, int ks, T (&d)[4][NU]) {
            const int lc = lfirst + TL * c + 2 * (4 * ks + (lane >> 4));
            const int64_t oe = (int64_t)(min(lc + po, L) - lb) * a.ldx;
            const int64_t oo = (int64_t)(min(lc + (po ^ 1), L) - lb) * a.ldx;
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                d[0][u] = AE[oe + 16 * u];
                d[1][u] = AE[oo + 16 * u];
                d[2][u] = AB[oe + 16 * u];
                d[3][u] = AB[oo + 16 * u];
            }
        };

        Seed<2> sd;
        Rec<2> f;
        seed_of(sd, 0);
        if (filler) {
            f.start(sd, w);
            auto em = emit_to(0);
            rec_all(f, cm + (int64_t)__builtin_amdgcn_readfirstlane(ls_of(0) - lb) * 4, min(SEG, L - ls_of(0) + 1), em);
        }
        seed_of(sd, min(1, nch - 1));
        load_a(0, 0, bb[0]);
        __syncthreads();
        for (int c = 0; c < nch; ++c) {
            const int b = c & 1;
            const int cn = min(c + 1, nch - 1);
            const cptr cp = cm + (int64_t)__builtin_amdgcn_readfirstlane(ls_of(cn) - lb) * 4;
            const int cnt = min(SEG, L - ls_of(cn) + 1);
            if (filler) f.start(sd, w);
            auto em = emit_to(b ^ 1);
            const T* fb = fpm + b * BUF;
            static_for<0, KS>([&](auto ki) {
                constexpr int ks = decltype(ki)::v;
                if constexpr (ks + 1 < KS) load_a(c, ks + 1, bb[(ks + 1) & 1]);
                else load_a(cn, 0, bb[0]);
                if constexpr (ks == KS / 2) seed_of(sd, min(c + 2, nch - 1));
                // keep the prefetch ahead of this step's compute (the scheduler may sink it)
                __builtin_amdgcn_sched_barrier(0);
                const int kl = 4 * ks + (lane >> 4);
                const T(&d)[4][NU] = bb[ks & 1];
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const int o = kl * RS + 16 * t + (lane & 15);
                    const T pe = fb[o], pd = fb[CLS + o];
                    const T me = fb[FOFF + o], mo = fb[FOFF + CLS + o];
#pragma unroll
                    for (int u = 0; u < NU; ++u) {
                        u1[t][u] = MF::run(pe, d[0][u], u1[t][u]);
                        u2[t][u] = MF::run(pd, d[1][u], u2[t][u]);
                        v1[t][u] = MF::run(pe, d[2][u], v1[t][u]);
                        v2[t][u] = MF::run(pd, d[3][u], v2[t][u]);
                    }
#pragma unroll
                    for (int u = 0; u < NU; ++u) {
                        u1[t][u] = MF::run(mo, d[3][u], u1[t][u]);
                        u2[t][u] = MF::run(me, d[2][u], u2[t][u]);
                        v1[t][u] = MF::run(mo, d[1][u], v1[t][u]);
                        v2[t][u] = MF::run(me, d[0][u], v2[t][u]);
                    }
                }
                if (filler) rec_group<ks>(f, cp, cnt, em);
            });
            __syncthreads();
        }
    }

    // Q = X; U = -i Y: U_re = Y_im, U_im = -Y_re -> this lane's Y value goes to the partner column
    const int64_t xm = (int64_t)m * a.nring * a.ldx;
    T* XQ = xptr<T>(a, 1) + xm + col;
    T* XU = xptr<T>(a, 2) + xm + (col ^ 1);
    const unsigned usg = (col & 1) ? 0u : 0x80000000u;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = r0 + 16 * t + MF::row(lane, v);
            if (r >= a.rn) continue;
            const int rs = a.nring - 1 - r;
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const T U1 = u1[t][u][v], U2 = u2[t][u][v];
                const T V1 = v1[t][u][v], V2 = v2[t][u][v];
                XQ[(int64_t)r * a.ldx + 16 * u] = U1 + U2;
                XU[(int64_t)r * a.ldx + 16 * u] = flip((T)(V1 + V2), usg);
                if (rs != r) {
                    XQ[(int64_t)rs * a.ldx + 16 * u] = U1 - U2;
                    XU[(int64_t)rs * a.ldx + 16 * u] = flip((T)(V1 - V2), usg);
                }
            }
        }
}

// widest column tiling (64 NU columns per workgroup, NU <= NUMAX) that divides ldx
int pick_nu(int numax, int64_t ldx)
{
    int nu = numax;
    while (nu > 2 && ldx % (64 * nu) != 0) nu >>= 1;
    return nu;
}

// Column tiling per kernel: the widest NU whose registers fit two waves per SIMD
// without spilling (spin 0, map2alm FP64: 4; spin-0 FP32: 4; the rest: 2).
template <typename T>
hipError_t launch_m2a_t(const LegArgs& a, hipStream_t st)
{
    LegArgs b = a;
    const dim3 blk(NT);
    if (a.spin == 0) {
        const int nu = pick_nu(4, a.ldx);
        b.ctiles = (int)(a.ldx / (64 * nu));
        const dim3 grid(b.ntiles * b.ctiles);
        if (nu == 4) hipLaunchKernelGGL((k_m2a_spin0<T, 4>), grid, blk, 0, st, b);
        else hipLaunchKernelGGL((k_m2a_spin0<T, 2>), grid, blk, 0, st, b);
    } else {
        b.ctiles = (int)(a.ldx / 128);
        hipLaunchKernelGGL((k_m2a_spin2<T, 2>), dim3(b.ntiles * b.ctiles), blk, 0, st, b);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_a2m_t(const LegArgs& a, hipStream_t st)
{
    LegArgs b = a;
    constexpr bool F64 = sizeof(T) == 8;
    const dim3 blk(NT);
    if (a.spin == 0) {
        const int nu = pick_nu(F64 ? 2 : 4, a.ldx);
        b.ctiles = (int)(a.ldx / (64 * nu));
        const dim3 grid((a.lmax + 1) * b.ctiles * ((a.rn + A0_TR - 1) / A0_TR));
        if constexpr (!F64) {
            if (nu == 4) {
                hipLaunchKernelGGL((k_a2m_spin0<T, 4>), grid, blk, 0, st, b);
                return hipGetLastError();
            }
        }
        hipLaunchKernelGGL((k_a2m_spin0<T, 2>), grid, blk, 0, st, b);
    } else {
        b.ctiles = (int)(a.ldx / 128);
        const dim3 grid((a.lmax + 1) * b.ctiles * ((a.rn + A2_TR - 1) / A2_TR));
        hipLaunchKernelGGL((k_a2m_spin2<T, 2>), grid, blk, 0, st, b);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_leg_m2a(const LegArgs& a, int prec, hipStream_t st)
{
    if (prec == 0) return launch_m2a_t<double>(a, st);
    return launch_m2a_t<float>(a, st);
}

hipError_t launch_leg_a2m(const LegArgs& a, int prec, hipStream_t st)
{
    if (prec == 0) return launch_a2m_t<double>(a, st);
    return launch_a2m_t<float>(a, st);
}

}  // namespace sht
