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
// with the MFMAs of the current one.  The other MFMA operand (ring coefficients
// T_m for map2alm, coefficients A_m for alm2map) comes straight from HBM in the
// m-major layouts [m][ring][column] and [m][l][column] into registers, one tile
// ahead.  The two hemispheres are folded with lambda_lm(-z) = (-1)^{l+m}
// lambda_lm(z) (lambda+-(-z) = +-(-1)^{l+m} lambda+-(z)): only northern rings are
// contracted, rows of even l-m against T_N + T_S and odd ones against T_N - T_S.
// Column pairs (2k, 2k+1) are the real and imaginary parts of map k.
#include "leg_common.h"

namespace sht {
namespace {

constexpr int NT = 256;
constexpr int HALF = TL / 2;   // rows of one parity class per l tile
constexpr int KS = 8;          // MFMA K-steps per tile (32 rings or 32 l of a parity / 4)
constexpr int STEPS_PER_KS = 4;  // recursion steps interleaved per K-step (KS*4 >= SEG-1)
static_assert(KS * STEPS_PER_KS >= SEG - 1, "interleaved fill must finish within one tile");

// ----------------------------------------------------------------------------
// recursion state of one (ring, segment) fill item
// ----------------------------------------------------------------------------
struct Fill0 {
    double v0, v1, x;
    int k, t, cnt;
    bool on;
};
struct Fill2 {
    double p0, p1, q0, q1, x;
    int k, t, cnt;
    bool on;
};

__device__ __forceinline__ void seed_index(const LegArgs& a, int m, int j, int r, int64_t& idx)
{
    idx = a.seedoff[m] + (int64_t)j * a.rn + r;
}

// Starts a fill item: loads its seed (values at rows 0 and 1 of the segment).
__device__ __forceinline__ void fill_start(Fill0& f, const LegArgs& a, int m, int j, int r, int cnt, bool on)
{
    f.on = on && cnt > 0;
    f.cnt = cnt;
    f.t = 0;
    f.v0 = f.v1 = 0.0;
    f.k = 1;
    f.x = 0.0;
    if (f.on) {
        int64_t idx;
        seed_index(a, m, j, r, idx);
        f.v0 = a.mu[idx];
        f.v1 = a.mu[a.seedstride + idx];
        f.k = a.kk[idx];
        f.x = a.rings[r].z;
    }
}
__device__ __forceinline__ void fill_start(Fill2& f, const LegArgs& a, int m, int j, int r, int cnt, bool on)
{
    f.on = on && cnt > 0;
    f.cnt = cnt;
    f.t = 0;
    f.p0 = f.p1 = f.q0 = f.q1 = 0.0;
    f.k = 1;
    f.x = 0.0;
    if (f.on) {
        int64_t idx;
        seed_index(a, m, j, r, idx);
        f.p0 = a.mu[idx];
        f.p1 = a.mu[a.seedstride + idx];
        f.q0 = a.mu[2 * a.seedstride + idx];
        f.q1 = a.mu[3 * a.seedstride + idx];
        f.k = a.kk[idx];
        f.x = a.rings[r].z;
    }
}

// One step: at t = 0 emits rows 0 and 1 (the seed pair), later steps emit row t.
// Rows at or beyond cnt (past lmax) and items that are off emit zeros.
template <typename Emit>
__device__ __forceinline__ void fill_step(Fill0& f, const double* coef, Emit emit)
{
    if (f.t >= SEG) return;
    if (f.t == 0) {
        emit(0, (f.on && f.k == 0) ? f.v0 : 0.0);
        emit(1, (f.on && f.k == 0 && f.cnt > 1) ? f.v1 : 0.0);
        f.t = 2;
        return;
    }
    const int t = f.t;
    double v2 = (coef[2 * t] * f.x) * f.v1 - coef[2 * t + 1] * f.v0;
    if (f.k > 0 && fabs(v2) > RESCALE_AT) {
        v2 *= SCALE_DOWN;
        f.v1 *= SCALE_DOWN;
        --f.k;
    }
    emit(t, (f.on && f.k == 0 && t < f.cnt) ? v2 : 0.0);
    f.v0 = f.v1;
    f.v1 = v2;
    f.t = t + 1;
}

// emit(row, F+, F-) with F+- = -(P +- M)/2
template <typename Emit>
__device__ __forceinline__ void fill_step(Fill2& f, const double* coef, Emit emit)
{
    if (f.t >= SEG) return;
    if (f.t == 0) {
        bool z0 = f.on && f.k == 0, z1 = z0 && f.cnt > 1;
        emit(0, z0 ? -0.5 * (f.p0 + f.q0) : 0.0, z0 ? -0.5 * (f.p0 - f.q0) : 0.0);
        emit(1, z1 ? -0.5 * (f.p1 + f.q1) : 0.0, z1 ? -0.5 * (f.p1 - f.q1) : 0.0);
        f.t = 2;
        return;
    }
    const int t = f.t;
    const double ax = coef[3 * t] * f.x, be = coef[3 * t + 1], ga = coef[3 * t + 2];
    double p2 = (ax + be) * f.p1 - ga * f.p0;
    double q2 = (ax - be) * f.q1 - ga * f.q0;
    if (f.k > 0 && fmax(fabs(p2), fabs(q2)) > RESCALE_AT) {
        p2 *= SCALE_DOWN; f.p1 *= SCALE_DOWN;
        q2 *= SCALE_DOWN; f.q1 *= SCALE_DOWN;
        --f.k;
    }
    bool z = f.on && f.k == 0 && t < f.cnt;
    emit(t, z ? -0.5 * (p2 + q2) : 0.0, z ? -0.5 * (p2 - q2) : 0.0);
    f.p0 = f.p1; f.p1 = p2;
    f.q0 = f.q1; f.q1 = q2;
    f.t = t + 1;
}

// recursion coefficients of row i = l - l0 (i < TL): spin 0 -> 2 per row, spin 2 -> 3
template <int SPIN>
__device__ __forceinline__ void coef_row(double* coef, int i, int l0, int m)
{
    const int l = l0 + i;
    if (SPIN == 0) {
        double a, ab;
        coef_spin0(l, m, a, ab);
        coef[2 * i] = a;
        coef[2 * i + 1] = ab;
    } else {
        double al, be, ga;
        coef_spin2(l, m, al, be, ga);
        coef[3 * i] = al;
        coef[3 * i + 1] = be;
        coef[3 * i + 2] = ga;
    }
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

// m2a work decode: logical g -> (m, lt, ct); tileoff[m] = l tiles of all m' < m.
__device__ __forceinline__ void decode_tiles(const int* off, int lmax, int C, int g, int& m, int& lt, int& ct)
{
    int lo = 0, hi = lmax + 1;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (off[mid] * C <= g) lo = mid; else hi = mid;
    }
    m = lo;
    int r = g - off[m] * C;
    int nlt = off[m + 1] - off[m];
    ct = r / nlt;
    lt = r - ct * nlt;
}

// next ring chunk >= rc whose first significant l is within [.., lend]
__device__ __forceinline__ int next_chunk(const LegArgs& a, int m, int rc, int nchunk, int lend)
{
    while (rc < nchunk && a.lsig[(int64_t)m * a.nrc + rc] > lend) ++rc;
    return rc;
}

// ============================================================================
// map2alm, spin 0: A_l = sum_{north rings} lambda_l (T_N +- T_S), raw sums into
// the m-major coefficient workspace.  Tile: 64 l x 128 columns; rings in chunks
// of 32; wave w owns columns 32w..32w+31 and all 64 rows.
// ============================================================================
constexpr int M0_TR = 32, M0_TC = 128;

template <typename T>
__global__ __launch_bounds__(NT, 2) void k_m2a_spin0(LegArgs a)
{
    __shared__ T lam[2][2][M0_TR][HALF + 1];  // [buffer][parity][ring][row/2]
    __shared__ double coef[2 * TL];

    int m, lt, ct;
    decode_tiles(a.tiles, a.lmax, a.ctiles, xcd_remap(blockIdx.x, gridDim.x), m, lt, ct);
    const int L = a.lmax, lb = m;
    const int l0 = lb + lt * TL, lend = min(L, l0 + TL - 1);
    const int po = (lb - m) & 1;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int cw = ct * M0_TC + 32 * wave;
    const T* X = xptr<T>(a, 0);
    const int64_t xm = (int64_t)m * a.nring * a.ldx;
    // fill item of this lane: lanes 0..15 of each wave, 64 items = 32 rings x 2 segments
    const int item = wave * 16 + (lane & 15);
    const int frl = item & (M0_TR - 1), fs = item / M0_TR;
    const bool filler = lane < 16;
    const int fls = l0 + SEG * fs;
    const int fcnt = (fls <= L) ? min(SEG, L - fls + 1) : 0;

    if (tid < TL) coef_row<0>(coef, tid, l0, m);
    __syncthreads();

    using MF = Mfma<T>;
    typename MF::acc acc[2][2][2];  // [parity][row tile][col tile]
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int u = 0; u < 2; ++u) acc[p][t][u] = typename MF::acc{0, 0, 0, 0};

    const int nchunk = (a.rn + M0_TR - 1) / M0_TR;
    int rc = next_chunk(a, m, 0, nchunk, lend);
    if (rc < nchunk) {
        auto emit_to = [&](int buf) {
            return [&, buf](int i, double v) {
                const int row = SEG * fs + i;
                lam[buf][(row + po) & 1][frl][row >> 1] = (T)v;
            };
        };
        // prologue: whole fill of the first chunk
        Fill0 f;
        if (filler) {
            const int r = rc * M0_TR + frl;
            fill_start(f, a, m, lt * 2 + fs, r, fcnt, r < a.rn);
            auto em = emit_to(0);
            for (int s = 0; s < SEG; ++s) fill_step(f, coef + 2 * SEG * fs, em);
        }
        // operand registers: N and S ring values for 8 K-steps x 2 column tiles
        double xn[KS][2], xs[KS][2];
        auto load_x = [&](int rcn, double (&n)[KS][2], double (&s)[KS][2]) {
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int r = rcn * M0_TR + 4 * ks + (lane >> 4);
                const bool ok = r < a.rn;
                const int rr = ok ? r : 0;
                const int rs = a.nring - 1 - rr;
                const T* pn = X + xm + (int64_t)rr * a.ldx + cw + (lane & 15);
                const T* ps = X + xm + (int64_t)rs * a.ldx + cw + (lane & 15);
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    double vn = (double)pn[16 * u], vs = (double)ps[16 * u];
                    n[ks][u] = ok ? vn : 0.0;
                    s[ks][u] = (ok && rs != rr) ? vs : 0.0;
                }
            }
        };
        load_x(rc, xn, xs);
        __syncthreads();
        int buf = 0;
        while (rc < nchunk) {
            const int rcn = next_chunk(a, m, rc + 1, nchunk, lend);
            const bool more = rcn < nchunk;
            // seed loads first: waiting for them must not wait for the operand prefetch
            if (filler && more) {
                const int r = rcn * M0_TR + frl;
                fill_start(f, a, m, lt * 2 + fs, r, fcnt, r < a.rn);
            }
            double yn[KS][2], ys[KS][2];
            if (more) load_x(rcn, yn, ys);
            auto em = emit_to(buf ^ 1);
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int kr = 4 * ks + (lane >> 4);
                T av[2][2];
#pragma unroll
                for (int p = 0; p < 2; ++p)
#pragma unroll
                    for (int t = 0; t < 2; ++t) av[p][t] = lam[buf][p][kr][16 * t + (lane & 15)];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const T bs = (T)(xn[ks][u] + xs[ks][u]);
                    const T bd = (T)(xn[ks][u] - xs[ks][u]);
#pragma unroll
                    for (int t = 0; t < 2; ++t) {
                        acc[0][t][u] = MF::run(av[0][t], bs, acc[0][t][u]);
                        acc[1][t][u] = MF::run(av[1][t], bd, acc[1][t][u]);
                    }
                }
                if (filler && more) {
#pragma unroll
                    for (int q = 0; q < STEPS_PER_KS; ++q) fill_step(f, coef + 2 * SEG * fs, em);
                }
            }
            if (filler && more)
                while (f.t < SEG) fill_step(f, coef + 2 * SEG * fs, em);
            __syncthreads();
            if (more) {
#pragma unroll
                for (int ks = 0; ks < KS; ++ks)
#pragma unroll
                    for (int u = 0; u < 2; ++u) { xn[ks][u] = yn[ks][u]; xs[ks][u] = ys[ks][u]; }
            }
            buf ^= 1;
            rc = rcn;
        }
    }

    // store raw sums: row index within a parity class -> l
    T* A = aptr<T>(a, 0) + a.rowoff[m] * a.ldx;
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int ci = 16 * t + MF::row(lane, v);
                    const int l = l0 + 2 * ci + (p ^ po);
                    if (l > L) continue;
                    A[(int64_t)(l - lb) * a.ldx + cw + 16 * u + (lane & 15)] = (T)acc[p][t][u][v];
                }
}

// ============================================================================
// map2alm, spin 2 (E and iB from Q and iU):
//   even l-m: A_E = F+ SX + F- DY,  iA_B = F+ SY + F- DX
//   odd  l-m: A_E = F+ DX + F- SY,  iA_B = F+ DY + F- SX
// X = Q coefficients, Y = iU; S/D = north +- south.  Tile 64 l x 64 columns,
// rings in chunks of 32; wave w owns columns 16w..16w+15.
// ============================================================================
constexpr int M2_TR = 32, M2_TC = 64;

template <typename T>
__global__ __launch_bounds__(NT, 2) void k_m2a_spin2(LegArgs a)
{
    __shared__ T fpm[2][2][2][M2_TR][HALF + 1];  // [buffer][F+ / F-][parity][ring][row/2]
    __shared__ double coef[3 * TL];

    int m, lt, ct;
    decode_tiles(a.tiles, a.lmax, a.ctiles, xcd_remap(blockIdx.x, gridDim.x), m, lt, ct);
    const int L = a.lmax, lb = lbase(2, m);
    const int l0 = lb + lt * TL, lend = min(L, l0 + TL - 1);
    const int po = (lb - m) & 1;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int col = ct * M2_TC + 16 * wave + (lane & 15);
    const int pcol = col ^ 1;               // partner column: Y = iU swaps re/im
    const double ysg = (col & 1) ? 1.0 : -1.0;  // Y_re = -U_im, Y_im = U_re
    const T* XQ = xptr<T>(a, 1);
    const T* XU = xptr<T>(a, 2);
    const int64_t xm = (int64_t)m * a.nring * a.ldx;
    const int item = wave * 16 + (lane & 15);
    const int frl = item & (M2_TR - 1), fs = item / M2_TR;
    const bool filler = lane < 16;
    const int fls = l0 + SEG * fs;
    const int fcnt = (fls <= L) ? min(SEG, L - fls + 1) : 0;

    if (tid < TL) coef_row<2>(coef, tid, l0, m);
    __syncthreads();

    using MF = Mfma<T>;
    typename MF::acc accE[2][2], accB[2][2];  // [parity][row tile]
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int t = 0; t < 2; ++t) accE[p][t] = accB[p][t] = typename MF::acc{0, 0, 0, 0};

    const int nchunk = (a.rn + M2_TR - 1) / M2_TR;
    int rc = next_chunk(a, m, 0, nchunk, lend);
    if (rc < nchunk) {
        auto emit_to = [&](int buf) {
            return [&, buf](int i, double fp, double fm) {
                const int row = SEG * fs + i;
                const int c = (row + po) & 1;
                fpm[buf][0][c][frl][row >> 1] = (T)fp;
                fpm[buf][1][c][frl][row >> 1] = (T)fm;
            };
        };
        Fill2 f;
        if (filler) {
            const int r = rc * M2_TR + frl;
            fill_start(f, a, m, lt * 2 + fs, r, fcnt, r < a.rn);
            auto em = emit_to(0);
            for (int s = 0; s < SEG; ++s) fill_step(f, coef + 3 * SEG * fs, em);
        }
        // operand registers: Q_N, Q_S, Y_N, Y_S per K-step
        double qn[KS], qs[KS], yn[KS], ys[KS];
        auto load_x = [&](int rcn, double (&a1)[KS], double (&a2)[KS], double (&b1)[KS], double (&b2)[KS]) {
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int r = rcn * M2_TR + 4 * ks + (lane >> 4);
                const bool ok = r < a.rn;
                const int rr = ok ? r : 0;
                const int rs = a.nring - 1 - rr;
                const bool south = ok && rs != rr;
                const int64_t on = xm + (int64_t)rr * a.ldx, os = xm + (int64_t)rs * a.ldx;
                double v1 = (double)XQ[on + col], v2 = (double)XQ[os + col];
                double v3 = (double)XU[on + pcol], v4 = (double)XU[os + pcol];
                a1[ks] = ok ? v1 : 0.0;
                a2[ks] = south ? v2 : 0.0;
                b1[ks] = ok ? ysg * v3 : 0.0;
                b2[ks] = south ? ysg * v4 : 0.0;
            }
        };
        load_x(rc, qn, qs, yn, ys);
        __syncthreads();
        int buf = 0;
        while (rc < nchunk) {
            const int rcn = next_chunk(a, m, rc + 1, nchunk, lend);
            const bool more = rcn < nchunk;
            if (filler && more) {
                const int r = rcn * M2_TR + frl;
                fill_start(f, a, m, lt * 2 + fs, r, fcnt, r < a.rn);
            }
            double qn2[KS], qs2[KS], yn2[KS], ys2[KS];
            if (more) load_x(rcn, qn2, qs2, yn2, ys2);
            auto em = emit_to(buf ^ 1);
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int kr = 4 * ks + (lane >> 4);
                const T sx = (T)(qn[ks] + qs[ks]), dx = (T)(qn[ks] - qs[ks]);
                const T sy = (T)(yn[ks] + ys[ks]), dy = (T)(yn[ks] - ys[ks]);
                T fp[2][2], fm[2][2];  // [parity][row tile]
#pragma unroll
                for (int p = 0; p < 2; ++p)
#pragma unroll
                    for (int t = 0; t < 2; ++t) {
                        fp[p][t] = fpm[buf][0][p][kr][16 * t + (lane & 15)];
                        fm[p][t] = fpm[buf][1][p][kr][16 * t + (lane & 15)];
                    }
                // first terms of all eight accumulators, then the second terms, so
                // that dependent MFMAs are eight instructions apart
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    accE[0][t] = MF::run(fp[0][t], sx, accE[0][t]);
                    accB[0][t] = MF::run(fp[0][t], sy, accB[0][t]);
                    accE[1][t] = MF::run(fp[1][t], dx, accE[1][t]);
                    accB[1][t] = MF::run(fp[1][t], dy, accB[1][t]);
                }
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    accE[0][t] = MF::run(fm[0][t], dy, accE[0][t]);
                    accB[0][t] = MF::run(fm[0][t], dx, accB[0][t]);
                    accE[1][t] = MF::run(fm[1][t], sy, accE[1][t]);
                    accB[1][t] = MF::run(fm[1][t], sx, accB[1][t]);
                }
                if (filler && more) {
#pragma unroll
                    for (int q = 0; q < STEPS_PER_KS; ++q) fill_step(f, coef + 3 * SEG * fs, em);
                }
            }
            if (filler && more)
                while (f.t < SEG) fill_step(f, coef + 3 * SEG * fs, em);
            __syncthreads();
            if (more) {
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) { qn[ks] = qn2[ks]; qs[ks] = qs2[ks]; yn[ks] = yn2[ks]; ys[ks] = ys2[ks]; }
            }
            buf ^= 1;
            rc = rcn;
        }
    }

    T* AE = aptr<T>(a, 1) + a.rowoff[m] * a.ldx;
    T* AB = aptr<T>(a, 2) + a.rowoff[m] * a.ldx;
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int ci = 16 * t + MF::row(lane, v);
                const int l = l0 + 2 * ci + (p ^ po);
                if (l > L) continue;
                const int64_t o = (int64_t)(l - lb) * a.ldx + col;
                AE[o] = (T)accE[p][t][v];
                AB[o] = (T)accB[p][t][v];
            }
}

// ============================================================================
// alm2map, spin 0: E = sum_{even l-m} lambda A, O = sum_{odd} lambda A,
// T_N = E + O, T_S = E - O.  Tile: 64 rings x 64 columns, l in chunks of 64;
// wave w owns columns 16w..16w+15 and all 64 rings.
// ============================================================================
constexpr int A0_TR = 64, A0_TC = 64;

template <typename T>
__global__ __launch_bounds__(NT, 2) void k_a2m_spin0(LegArgs a)
{
    __shared__ T lam[2][2][HALF][A0_TR + 1];   // [buffer][parity][row/2][ring]
    __shared__ double coef[3][2 * TL];         // coefficients of three consecutive l chunks

    const int nrt = (a.rn + A0_TR - 1) / A0_TR;
    const int g = xcd_remap(blockIdx.x, gridDim.x);
    const int m = g / (a.ctiles * nrt);
    const int rem = g - m * a.ctiles * nrt;
    const int ct = rem / nrt, rt = rem - ct * nrt;
    const int L = a.lmax, lb = m;
    const int po = (lb - m) & 1;
    const int r0 = rt * A0_TR;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int col = ct * A0_TC + 16 * wave + (lane & 15);
    // fill items: lanes 0..31 of each wave, 128 items = 64 rings x 2 segments
    const int item = wave * 32 + (lane & 31);
    const int frl = item & (A0_TR - 1), fs = item / A0_TR;
    const bool filler = lane < 32;
    const int fr = r0 + frl;
    // lanes 32..63 of waves 0 and 1 compute coefficients of the chunk after next
    const bool coefer = lane >= 32 && wave < 2;
    const int crow = (wave * 32) + (lane - 32);

    int lsig = L + 1;
    for (int c = r0 / RCHUNK; c < min(a.nrc, (r0 + A0_TR + RCHUNK - 1) / RCHUNK); ++c)
        lsig = min(lsig, a.lsig[(int64_t)m * a.nrc + c]);
    const int lfirst = (lsig > L) ? L + 1 : lb + SEG * (((lsig - lb) / SEG) & ~1);
    const int nch = (lfirst > L) ? 0 : (L - lfirst) / TL + 1;

    using MF = Mfma<T>;
    typename MF::acc accE[4], accO[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) accE[t] = accO[t] = typename MF::acc{0, 0, 0, 0};

    const T* Am = aptr<T>(a, 0) + a.rowoff[m] * a.ldx;
    if (nch > 0) {
        if (tid < TL) coef_row<0>(coef[0], tid, lfirst, m);
        if (tid >= TL && tid < 2 * TL && nch > 1) coef_row<0>(coef[1], tid - TL, lfirst + TL, m);
        __syncthreads();
        auto emit_to = [&](int buf) {
            return [&, buf](int i, double v) {
                const int row = SEG * fs + i;
                lam[buf][(row + po) & 1][row >> 1][frl] = (T)v;
            };
        };
        auto seg_of = [&](int c) { return (lfirst - lb) / SEG + 2 * c + fs; };
        auto cnt_of = [&](int c) {
            const int ls = lfirst + TL * c + SEG * fs;
            return (ls <= L) ? min(SEG, L - ls + 1) : 0;
        };
        Fill0 f;
        if (filler) {
            fill_start(f, a, m, seg_of(0), fr < a.rn ? fr : 0, cnt_of(0), fr < a.rn);
            auto em = emit_to(0);
            for (int s = 0; s < SEG; ++s) fill_step(f, coef[0] + 2 * SEG * fs, em);
        }
        // operand registers: A rows of even / odd class for 8 K-steps
        double be[KS], bo[KS];
        auto load_a = [&](int c, double (&e)[KS], double (&o)[KS]) {
            const int lc = lfirst + TL * c;
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int kl = 4 * ks + (lane >> 4);
                // class 0 rows are local rows i with (i + po) even
                const int le = lc + 2 * kl + po, lo = lc + 2 * kl + (po ^ 1);
                const int lec = min(le, L), loc = min(lo, L);
                double ve = (double)Am[(int64_t)(lec - lb) * a.ldx + col];
                double vo = (double)Am[(int64_t)(loc - lb) * a.ldx + col];
                e[ks] = (le <= L) ? ve : 0.0;
                o[ks] = (lo <= L) ? vo : 0.0;
            }
        };
        load_a(0, be, bo);
        __syncthreads();
        int buf = 0;
        for (int c = 0; c < nch; ++c) {
            const bool more = c + 1 < nch;
            if (filler && more) fill_start(f, a, m, seg_of(c + 1), fr < a.rn ? fr : 0, cnt_of(c + 1), fr < a.rn);
            double be2[KS], bo2[KS];
            if (more) load_a(c + 1, be2, bo2);
            if (coefer && c + 2 < nch) coef_row<0>(coef[(c + 2) % 3], crow, lfirst + TL * (c + 2), m);
            const double* cf = coef[(c + 1) % 3] + 2 * SEG * fs;
            auto em = emit_to(buf ^ 1);
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int kl = 4 * ks + (lane >> 4);
                const T bE = (T)be[ks], bO = (T)bo[ks];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const T aE = lam[buf][0][kl][16 * t + (lane & 15)];
                    const T aO = lam[buf][1][kl][16 * t + (lane & 15)];
                    accE[t] = MF::run(aE, bE, accE[t]);
                    accO[t] = MF::run(aO, bO, accO[t]);
                }
                if (filler && more) {
#pragma unroll
                    for (int q = 0; q < STEPS_PER_KS; ++q) fill_step(f, cf, em);
                }
            }
            if (filler && more)
                while (f.t < SEG) fill_step(f, cf, em);
            __syncthreads();
            if (more) {
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) { be[ks] = be2[ks]; bo[ks] = bo2[ks]; }
            }
            buf ^= 1;
        }
    }

    T* X = xptr<T>(a, 0);
    const int64_t xm = (int64_t)m * a.nring * a.ldx;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = r0 + 16 * t + MF::row(lane, v);
            if (r >= a.rn) continue;
            const double e = (double)accE[t][v], o = (double)accO[t][v];
            X[xm + (int64_t)r * a.ldx + col] = (T)(e + o);
            const int rs = a.nring - 1 - r;
            if (rs != r) X[xm + (int64_t)rs * a.ldx + col] = (T)(e - o);
        }
}

// ============================================================================
// alm2map, spin 2, with B' = i a_B:
//   U1 = sum_even F+ E + sum_odd F- B',  U2 = sum_odd F+ E + sum_even F- B'
//   V1 = sum_even F+ B' + sum_odd F- E,  V2 = sum_odd F+ B' + sum_even F- E
//   Q_N = U1 + U2, Q_S = U1 - U2;  (iU)_N = V1 + V2, (iU)_S = V1 - V2.
// Tile: 32 rings x 64 columns; wave w owns columns 16w..16w+15.
// ============================================================================
constexpr int A2_TR = 32, A2_TC = 64;

template <typename T>
__global__ __launch_bounds__(NT, 2) void k_a2m_spin2(LegArgs a)
{
    __shared__ T fpm[2][2][2][HALF][A2_TR + 1];   // [buffer][F+/F-][parity][row/2][ring]
    __shared__ double coef[3][3 * TL];

    const int nrt = (a.rn + A2_TR - 1) / A2_TR;
    const int g = xcd_remap(blockIdx.x, gridDim.x);
    const int m = g / (a.ctiles * nrt);
    const int rem = g - m * a.ctiles * nrt;
    const int ct = rem / nrt, rt = rem - ct * nrt;
    const int L = a.lmax, lb = lbase(2, m);
    const int po = (lb - m) & 1;
    const int r0 = rt * A2_TR;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int col = ct * A2_TC + 16 * wave + (lane & 15);
    const int item = wave * 16 + (lane & 15);
    const int frl = item & (A2_TR - 1), fs = item / A2_TR;
    const bool filler = lane < 16;
    const int fr = r0 + frl;
    const bool coefer = lane >= 32 && wave < 2;
    const int crow = (wave * 32) + (lane - 32);

    int lsig = L + 1;
    if (lb <= L) lsig = a.lsig[(int64_t)m * a.nrc + r0 / RCHUNK];
    const int lfirst = (lsig > L) ? L + 1 : lb + SEG * (((lsig - lb) / SEG) & ~1);
    const int nch = (lfirst > L) ? 0 : (L - lfirst) / TL + 1;

    using MF = Mfma<T>;
    typename MF::acc u1[2], u2[2], v1[2], v2[2];  // per row tile
#pragma unroll
    for (int t = 0; t < 2; ++t) u1[t] = u2[t] = v1[t] = v2[t] = typename MF::acc{0, 0, 0, 0};

    const T* AE = aptr<T>(a, 1) + a.rowoff[m] * a.ldx;
    const T* AB = aptr<T>(a, 2) + a.rowoff[m] * a.ldx;
    if (nch > 0) {
        if (tid < TL) coef_row<2>(coef[0], tid, lfirst, m);
        if (tid >= TL && tid < 2 * TL && nch > 1) coef_row<2>(coef[1], tid - TL, lfirst + TL, m);
        __syncthreads();
        auto emit_to = [&](int buf) {
            return [&, buf](int i, double fp, double fm) {
                const int row = SEG * fs + i;
                const int c = (row + po) & 1;
                fpm[buf][0][c][row >> 1][frl] = (T)fp;
                fpm[buf][1][c][row >> 1][frl] = (T)fm;
            };
        };
        auto seg_of = [&](int c) { return (lfirst - lb) / SEG + 2 * c + fs; };
        auto cnt_of = [&](int c) {
            const int ls = lfirst + TL * c + SEG * fs;
            return (ls <= L) ? min(SEG, L - ls + 1) : 0;
        };
        Fill2 f;
        if (filler) {
            fill_start(f, a, m, seg_of(0), fr < a.rn ? fr : 0, cnt_of(0), fr < a.rn);
            auto em = emit_to(0);
            for (int s = 0; s < SEG; ++s) fill_step(f, coef[0] + 3 * SEG * fs, em);
        }
        double ee[KS], eo[KS], he[KS], ho[KS];   // E and B' rows of both parity classes
        auto load_a = [&](int c, double (&e0)[KS], double (&e1)[KS], double (&h0)[KS], double (&h1)[KS]) {
            const int lc = lfirst + TL * c;
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int kl = 4 * ks + (lane >> 4);
                const int le = lc + 2 * kl + po, lo = lc + 2 * kl + (po ^ 1);
                const int64_t oe = (int64_t)(min(le, L) - lb) * a.ldx + col;
                const int64_t oo = (int64_t)(min(lo, L) - lb) * a.ldx + col;
                double w1 = (double)AE[oe], w2 = (double)AE[oo], w3 = (double)AB[oe], w4 = (double)AB[oo];
                e0[ks] = (le <= L) ? w1 : 0.0;
                e1[ks] = (lo <= L) ? w2 : 0.0;
                h0[ks] = (le <= L) ? w3 : 0.0;
                h1[ks] = (lo <= L) ? w4 : 0.0;
            }
        };
        load_a(0, ee, eo, he, ho);
        __syncthreads();
        int buf = 0;
        for (int c = 0; c < nch; ++c) {
            const bool more = c + 1 < nch;
            if (filler && more) fill_start(f, a, m, seg_of(c + 1), fr < a.rn ? fr : 0, cnt_of(c + 1), fr < a.rn);
            double ee2[KS], eo2[KS], he2[KS], ho2[KS];
            if (more) load_a(c + 1, ee2, eo2, he2, ho2);
            if (coefer && c + 2 < nch) coef_row<2>(coef[(c + 2) % 3], crow, lfirst + TL * (c + 2), m);
            const double* cf = coef[(c + 1) % 3] + 3 * SEG * fs;
            auto em = emit_to(buf ^ 1);
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int kl = 4 * ks + (lane >> 4);
                const T bEe = (T)ee[ks], bEo = (T)eo[ks], bBe = (T)he[ks], bBo = (T)ho[ks];
                T pe[2], pd[2], me[2], mo[2];
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    pe[t] = fpm[buf][0][0][kl][16 * t + (lane & 15)];
                    pd[t] = fpm[buf][0][1][kl][16 * t + (lane & 15)];
                    me[t] = fpm[buf][1][0][kl][16 * t + (lane & 15)];
                    mo[t] = fpm[buf][1][1][kl][16 * t + (lane & 15)];
                }
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    u1[t] = MF::run(pe[t], bEe, u1[t]);
                    u2[t] = MF::run(pd[t], bEo, u2[t]);
                    v1[t] = MF::run(pe[t], bBe, v1[t]);
                    v2[t] = MF::run(pd[t], bBo, v2[t]);
                }
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    u1[t] = MF::run(mo[t], bBo, u1[t]);
                    u2[t] = MF::run(me[t], bBe, u2[t]);
                    v1[t] = MF::run(mo[t], bEo, v1[t]);
                    v2[t] = MF::run(me[t], bEe, v2[t]);
                }
                if (filler && more) {
#pragma unroll
                    for (int q = 0; q < STEPS_PER_KS; ++q) fill_step(f, cf, em);
                }
            }
            if (filler && more)
                while (f.t < SEG) fill_step(f, cf, em);
            __syncthreads();
            if (more) {
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) { ee[ks] = ee2[ks]; eo[ks] = eo2[ks]; he[ks] = he2[ks]; ho[ks] = ho2[ks]; }
            }
            buf ^= 1;
        }
    }

    // Q = X; U = -i Y: U_re = Y_im, U_im = -Y_re -> this lane's Y value goes to the partner column
    T* XQ = xptr<T>(a, 1);
    T* XU = xptr<T>(a, 2);
    const int64_t xm = (int64_t)m * a.nring * a.ldx;
    const int pcol = col ^ 1;
    const double usg = (col & 1) ? 1.0 : -1.0;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = r0 + 16 * t + MF::row(lane, v);
            if (r >= a.rn) continue;
            const double U1 = (double)u1[t][v], U2 = (double)u2[t][v];
            const double V1 = (double)v1[t][v], V2 = (double)v2[t][v];
            XQ[xm + (int64_t)r * a.ldx + col] = (T)(U1 + U2);
            XU[xm + (int64_t)r * a.ldx + pcol] = (T)(usg * (V1 + V2));
            const int rs = a.nring - 1 - r;
            if (rs != r) {
                XQ[xm + (int64_t)rs * a.ldx + col] = (T)(U1 - U2);
                XU[xm + (int64_t)rs * a.ldx + pcol] = (T)(usg * (V1 - V2));
            }
        }
}

template <typename T>
hipError_t launch_m2a_t(const LegArgs& a, hipStream_t st)
{
    LegArgs b = a;
    if (a.spin == 0) {
        b.ctiles = (int)((a.ldx + M0_TC - 1) / M0_TC);
        hipLaunchKernelGGL(k_m2a_spin0<T>, dim3(b.ntiles * b.ctiles), dim3(NT), 0, st, b);
    } else {
        b.ctiles = (int)((a.ldx + M2_TC - 1) / M2_TC);
        hipLaunchKernelGGL(k_m2a_spin2<T>, dim3(b.ntiles * b.ctiles), dim3(NT), 0, st, b);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_a2m_t(const LegArgs& a, hipStream_t st)
{
    LegArgs b = a;
    if (a.spin == 0) {
        b.ctiles = (int)((a.ldx + A0_TC - 1) / A0_TC);
        int nrt = (a.rn + A0_TR - 1) / A0_TR;
        hipLaunchKernelGGL(k_a2m_spin0<T>, dim3((a.lmax + 1) * b.ctiles * nrt), dim3(NT), 0, st, b);
    } else {
        b.ctiles = (int)((a.ldx + A2_TC - 1) / A2_TC);
        int nrt = (a.rn + A2_TR - 1) / A2_TR;
        hipLaunchKernelGGL(k_a2m_spin2<T>, dim3((a.lmax + 1) * b.ctiles * nrt), dim3(NT), 0, st, b);
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
