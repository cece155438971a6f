// Fused Legendre recursion + MFMA contraction (HIP, gfx950).
//
// For every m the paper reduces the transform to dense products over the map
// batch (Sec. 2.2, eq. "matrix form"):
//     map2alm   A_m = dsigma P_m T_m      (contracts rings)
//     alm2map   T_m = P_m^t A_m           (contracts l)
// and, for polarisation, the real 2x2 block form of Sec. 2.3,
//     [A^E; iA^B]_m = [[F+, F-], [F-, F+]]_m [Q; iU]_m,   F+- = -lambda+-,
//     lambda+- = (2lambda +- -2lambda)/2 (Appendix A.2),
// with iA^B and iU as the natural real variables (Sec. 3.1 item 1).
//
// Here the P_m / F+- tiles are never stored: each workgroup runs the three-term
// recursion in FP64 registers from the plan's seed table (exponent-scaled, see
// k_seed.hip), writes the tile to LDS in the operand precision and feeds it to
// MFMA against tiles of T_m (map2alm) or A_m (alm2map) staged in LDS.  The two
// hemispheres are folded with lambda_lm(-z) = (-1)^{l+m} lambda_lm(z) (and
// lambda+-(-z) = +-(-1)^{l+m} lambda+-(z)), so only northern rings are contracted:
// rows of even l-m pair with T_N + T_S, odd ones with T_N - T_S.  Column pairs
// (2k, 2k+1) of the T and A tiles are the real and imaginary parts of map k
// (Sec. 3.1 item 1, real-only arithmetic).
#include "leg_common.h"

namespace sht {
namespace {

constexpr int NT = 256;
constexpr int HALF = TL / 2;  // rows of one parity class per tile

// ----------------------------------------------------------------------------
// seed loading and segment fill
// ----------------------------------------------------------------------------
struct Seed0 { double v0, v1; int k; };
struct Seed2 { double p0, p1, q0, q1; int k; };

__device__ __forceinline__ Seed0 load_seed0(const LegArgs& a, int m, int j, int r)
{
    int64_t idx = a.seedoff[m] + (int64_t)j * a.rn + r;
    Seed0 s;
    s.v0 = a.mu[idx];
    s.v1 = a.mu[a.seedstride + idx];
    s.k = a.kk[idx];
    return s;
}
__device__ __forceinline__ Seed2 load_seed2(const LegArgs& a, int m, int j, int r)
{
    int64_t idx = a.seedoff[m] + (int64_t)j * a.rn + r;
    Seed2 s;
    s.p0 = a.mu[idx];
    s.p1 = a.mu[a.seedstride + idx];
    s.q0 = a.mu[2 * a.seedstride + idx];
    s.q1 = a.mu[3 * a.seedstride + idx];
    s.k = a.kk[idx];
    return s;
}

// Fill SEG values of lambda for one (ring, segment) into the two parity classes.
// emit(i, v) receives local row i (0..SEG-1 within the segment) and the value.
template <typename Emit>
__device__ __forceinline__ void fill_spin0(Seed0 s, double x, int cnt, const double* coef, Emit emit)
{
    double v0 = s.v0, v1 = s.v1;
    int k = s.k;
    emit(0, k == 0 ? v0 : 0.0);
    if (cnt > 1) emit(1, k == 0 ? v1 : 0.0);
    for (int t = 2; t < cnt; ++t) {
        double v2 = (coef[2 * t] * x) * v1 - coef[2 * t + 1] * v0;
        if (k > 0 && fabs(v2) > RESCALE_AT) {
            v2 *= SCALE_DOWN;
            v1 *= SCALE_DOWN;
            --k;
        }
        emit(t, k == 0 ? v2 : 0.0);
        v0 = v1;
        v1 = v2;
    }
}

// emit(i, f_plus, f_minus) with F+- = -(P +- M)/2
template <typename Emit>
__device__ __forceinline__ void fill_spin2(Seed2 s, double x, int cnt, const double* coef, Emit emit)
{
    double p0 = s.p0, p1 = s.p1, q0 = s.q0, q1 = s.q1;
    int k = s.k;
    if (k == 0) emit(0, -0.5 * (p0 + q0), -0.5 * (p0 - q0)); else emit(0, 0.0, 0.0);
    if (cnt > 1) {
        if (k == 0) emit(1, -0.5 * (p1 + q1), -0.5 * (p1 - q1)); else emit(1, 0.0, 0.0);
    }
    for (int t = 2; t < cnt; ++t) {
        double ax = coef[3 * t] * x, be = coef[3 * t + 1], ga = coef[3 * t + 2];
        double p2 = (ax + be) * p1 - ga * p0;
        double q2 = (ax - be) * q1 - ga * q0;
        if (k > 0 && fmax(fabs(p2), fabs(q2)) > RESCALE_AT) {
            p2 *= SCALE_DOWN; p1 *= SCALE_DOWN;
            q2 *= SCALE_DOWN; q1 *= SCALE_DOWN;
            --k;
        }
        if (k == 0) emit(t, -0.5 * (p2 + q2), -0.5 * (p2 - q2)); else emit(t, 0.0, 0.0);
        p0 = p1; p1 = p2;
        q0 = q1; q1 = q2;
    }
}

// coefficients for the TL rows starting at l0: spin 0 -> 2 per row, spin 2 -> 3 per row
template <int SPIN>
__device__ __forceinline__ void make_coef(double* coef, int l0, int m)
{
    if (threadIdx.x < TL) {
        int l = l0 + threadIdx.x;
        if (SPIN == 0) {
            double a, ab;
            coef_spin0(l, m, a, ab);
            coef[2 * threadIdx.x] = a;
            coef[2 * threadIdx.x + 1] = ab;
        } else {
            double al, be, ga;
            coef_spin2(l, m, al, be, ga);
            coef[3 * threadIdx.x] = al;
            coef[3 * threadIdx.x + 1] = be;
            coef[3 * threadIdx.x + 2] = ga;
        }
    }
}

// compact-storage address of (l, m, part) relative to the component base;
// part 0 = Re, 1 = Im.  Returns -1 for Im at m = 0 (not stored).
__device__ __forceinline__ int64_t calm(int L, int l, int m, int part)
{
    if (part == 0) return (int64_t)m * (L + 1) + l;
    if (m == 0) return -1;
    return (int64_t)(L + 1 - m) * (L + 1) + (l - m);
}

template <typename T>
__device__ __forceinline__ T* xptr(const LegArgs& a, int comp)
{
    return static_cast<T*>(a.X) + (int64_t)comp * a.xcomp;
}

template <typename T>
__device__ __forceinline__ void ld2(const T* p, double& x, double& y)
{
    if constexpr (sizeof(T) == 8) {
        double2 v = *reinterpret_cast<const double2*>(p);
        x = v.x; y = v.y;
    } else {
        float2 v = *reinterpret_cast<const float2*>(p);
        x = v.x; y = v.y;
    }
}

// m2a work decode: logical g -> (m, lt, ct); tileoff[m] = tiles of all m' < m.
__device__ __forceinline__ void decode_m2a(const LegArgs& a, int g, int& m, int& lt, int& ct)
{
    const int* off = a.tiles;
    int lo = 0, hi = a.lmax + 1;  // find m with off[m]*C <= g < off[m+1]*C
    const int C = a.ctiles;
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

// ============================================================================
// map2alm, spin 0:  A_l = scale * sum_{north rings} lambda_l (T_N +- T_S)
// tile: TL rows of l x 64 columns, rings in chunks of 32
// ============================================================================
constexpr int M2A_TR = 32;
constexpr int M2A_TC = 64;

template <typename T>
__global__ __launch_bounds__(NT) void k_m2a_spin0(LegArgs a)
{
    __shared__ T lam[2][M2A_TR][HALF + 1];
    __shared__ T xt[2][M2A_TR][M2A_TC + 2];
    __shared__ double coef[2 * TL];

    int m, lt, ct;
    decode_m2a(a, xcd_remap(blockIdx.x, gridDim.x), m, lt, ct);
    const int L = a.lmax;
    const int lb = lbase(0, m);
    const int l0 = lb + lt * TL;
    const int lend = min(L, l0 + TL - 1);
    const int po = (lb - m) & 1;
    const int c0 = ct * M2A_TC;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int p = wave & 1, h = wave >> 1;
    const T* X = xptr<T>(a, 0);

    make_coef<0>(coef, l0, m);
    using MF = Mfma<T>;
    typename MF::acc acc[2][2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u) acc[t][u] = typename MF::acc{0, 0, 0, 0};

    const int nchunk = (a.rn + M2A_TR - 1) / M2A_TR;
    for (int rc = 0; rc < nchunk; ++rc) {
        if (a.lsig[(int64_t)m * a.nrc + rc] > lend) continue;  // whole chunk negligible for this tile
        const int r0 = rc * M2A_TR;
        __syncthreads();  // previous chunk's MFMA reads and the coefficients are done
        if (tid < 2 * M2A_TR) {
            const int rl = tid & (M2A_TR - 1), s = tid / M2A_TR;
            const int r = r0 + rl;
            const int ls = l0 + SEG * s;
            const int cnt = (ls <= L) ? min(SEG, L - ls + 1) : 0;
            if (r < a.rn && cnt > 0) {
                Seed0 sd = load_seed0(a, m, lt * 2 + s, r);
                fill_spin0(sd, a.rings[r].z, cnt, coef + 2 * SEG * s, [&](int i, double v) {
                    int row = SEG * s + i;
                    lam[(row + po) & 1][rl][row >> 1] = (T)v;
                });
            }
            for (int i = (r < a.rn ? cnt : 0); i < SEG; ++i) {
                int row = SEG * s + i;
                lam[(row + po) & 1][rl][row >> 1] = (T)0;
            }
        }
        // T tiles: rows = rings r0.., S = T_N + T_S, D = T_N - T_S (equator: S = T_N, D = 0)
        for (int e = tid; e < M2A_TR * (M2A_TC / 2); e += NT) {
            const int rl = e / (M2A_TC / 2), cp = e - rl * (M2A_TC / 2);
            const int r = r0 + rl;
            double nx = 0, ny = 0, sx = 0, sy = 0;
            if (r < a.rn) {
                ld2(X + ((int64_t)m * a.nring + r) * a.ldx + c0 + 2 * cp, nx, ny);
                const int rs = a.nring - 1 - r;
                if (rs != r) ld2(X + ((int64_t)m * a.nring + rs) * a.ldx + c0 + 2 * cp, sx, sy);
            }
            xt[0][rl][2 * cp] = (T)(nx + sx);
            xt[0][rl][2 * cp + 1] = (T)(ny + sy);
            xt[1][rl][2 * cp] = (T)(nx - sx);
            xt[1][rl][2 * cp + 1] = (T)(ny - sy);
        }
        __syncthreads();
#pragma unroll 2
        for (int ks = 0; ks < M2A_TR / 4; ++ks) {
            const int kr = 4 * ks + (lane >> 4);
            T av[2], bv[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) av[t] = lam[p][kr][16 * t + (lane & 15)];
#pragma unroll
            for (int u = 0; u < 2; ++u) bv[u] = xt[p][kr][32 * h + 16 * u + (lane & 15)];
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int u = 0; u < 2; ++u) acc[t][u] = MF::run(av[t], bv[u], acc[t][u]);
        }
    }

    // store: row index within the parity class -> l
    double* alm = a.alm + (int64_t)a.compT * (L + 1) * (L + 1);
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int ci = 16 * t + MF::row(lane, v);
                const int l = l0 + 2 * ci + (p ^ po);
                const int col = c0 + 32 * h + 16 * u + (lane & 15);
                const int k = col >> 1;
                if (l > L || k >= a.nmaps) continue;
                int64_t off = calm(L, l, m, col & 1);
                if (off < 0) continue;
                double* dst = alm + (int64_t)k * a.almstride + off;
                double val = a.scale * (double)acc[t][u][v];
                if (a.accumulate) *dst += val; else *dst = val;
            }
}

// ============================================================================
// map2alm, spin 2 (E, B from Q, U):
//   even l-m: A_E = F+ SX + F- DY,  iA_B = F- DX + F+ SY
//   odd  l-m: A_E = F+ DX + F- SY,  iA_B = F- SX + F+ DY
// X = Q-coefficients, Y = i U-coefficients; S/D = north +- south.
// ============================================================================
constexpr int M2A2_TR = 32;
constexpr int M2A2_TC = 32;

template <typename T>
__global__ __launch_bounds__(NT) void k_m2a_spin2(LegArgs a)
{
    __shared__ T fpm[2][2][M2A2_TR][HALF + 1];        // [F+ / F-][parity][ring][row/2]
    __shared__ T xt[4][M2A2_TR][M2A2_TC + 2];         // SX, DX, SY, DY
    __shared__ double coef[3 * TL];

    int m, lt, ct;
    decode_m2a(a, xcd_remap(blockIdx.x, gridDim.x), m, lt, ct);
    const int L = a.lmax;
    const int lb = lbase(2, m);
    const int l0 = lb + lt * TL;
    const int lend = min(L, l0 + TL - 1);
    const int po = (lb - m) & 1;
    const int c0 = ct * M2A2_TC;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int p = wave & 1;       // parity class of the rows
    const int q = wave >> 1;      // 0: A_E, 1: iA_B
    // (x1, x2) tiles multiplying F+ and F- for this wave
    const int x1 = (q == 0) ? (p == 0 ? 0 : 1) : (p == 0 ? 2 : 3);
    const int x2 = (q == 0) ? (p == 0 ? 3 : 2) : (p == 0 ? 1 : 0);
    const T* XQ = xptr<T>(a, 1);
    const T* XU = xptr<T>(a, 2);

    make_coef<2>(coef, l0, m);
    using MF = Mfma<T>;
    typename MF::acc acc[2][2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u) acc[t][u] = typename MF::acc{0, 0, 0, 0};

    const int nchunk = (a.rn + M2A2_TR - 1) / M2A2_TR;
    for (int rc = 0; rc < nchunk; ++rc) {
        if (a.lsig[(int64_t)m * a.nrc + rc] > lend) continue;
        const int r0 = rc * M2A2_TR;
        __syncthreads();
        if (tid < 2 * M2A2_TR) {
            const int rl = tid & (M2A2_TR - 1), s = tid / M2A2_TR;
            const int r = r0 + rl;
            const int ls = l0 + SEG * s;
            const int cnt = (ls <= L) ? min(SEG, L - ls + 1) : 0;
            if (r < a.rn && cnt > 0) {
                Seed2 sd = load_seed2(a, m, lt * 2 + s, r);
                fill_spin2(sd, a.rings[r].z, cnt, coef + 3 * SEG * s, [&](int i, double fp, double fm) {
                    int row = SEG * s + i;
                    int c = (row + po) & 1;
                    fpm[0][c][rl][row >> 1] = (T)fp;
                    fpm[1][c][rl][row >> 1] = (T)fm;
                });
            }
            for (int i = (r < a.rn ? cnt : 0); i < SEG; ++i) {
                int row = SEG * s + i;
                int c = (row + po) & 1;
                fpm[0][c][rl][row >> 1] = (T)0;
                fpm[1][c][rl][row >> 1] = (T)0;
            }
        }
        for (int e = tid; e < M2A2_TR * (M2A2_TC / 2); e += NT) {
            const int rl = e / (M2A2_TC / 2), cp = e - rl * (M2A2_TC / 2);
            const int r = r0 + rl;
            double qn = 0, qni = 0, qs = 0, qsi = 0, un = 0, uni = 0, us = 0, usi = 0;
            if (r < a.rn) {
                const int64_t on = ((int64_t)m * a.nring + r) * a.ldx + c0 + 2 * cp;
                ld2(XQ + on, qn, qni);
                ld2(XU + on, un, uni);
                const int rs = a.nring - 1 - r;
                if (rs != r) {
                    const int64_t os = ((int64_t)m * a.nring + rs) * a.ldx + c0 + 2 * cp;
                    ld2(XQ + os, qs, qsi);
                    ld2(XU + os, us, usi);
                }
            }
            // Y = i U: (re, im) = (-U_im, U_re)
            double yn = -uni, yni = un, ys = -usi, ysi = us;
            xt[0][rl][2 * cp] = (T)(qn + qs);  xt[0][rl][2 * cp + 1] = (T)(qni + qsi);
            xt[1][rl][2 * cp] = (T)(qn - qs);  xt[1][rl][2 * cp + 1] = (T)(qni - qsi);
            xt[2][rl][2 * cp] = (T)(yn + ys);  xt[2][rl][2 * cp + 1] = (T)(yni + ysi);
            xt[3][rl][2 * cp] = (T)(yn - ys);  xt[3][rl][2 * cp + 1] = (T)(yni - ysi);
        }
        __syncthreads();
#pragma unroll 2
        for (int ks = 0; ks < M2A2_TR / 4; ++ks) {
            const int kr = 4 * ks + (lane >> 4);
            T ap[2], am[2], b1[2], b2[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                ap[t] = fpm[0][p][kr][16 * t + (lane & 15)];
                am[t] = fpm[1][p][kr][16 * t + (lane & 15)];
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                b1[u] = xt[x1][kr][16 * u + (lane & 15)];
                b2[u] = xt[x2][kr][16 * u + (lane & 15)];
            }
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    acc[t][u] = MF::run(ap[t], b1[u], acc[t][u]);
                    acc[t][u] = MF::run(am[t], b2[u], acc[t][u]);
                }
        }
    }

    const int64_t csz = (int64_t)(L + 1) * (L + 1);
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int ci = 16 * t + MF::row(lane, v);
                const int l = l0 + 2 * ci + (p ^ po);
                const int col = c0 + 16 * u + (lane & 15);
                const int k = col >> 1;
                if (l > L || k >= a.nmaps) continue;
                double val = a.scale * (double)acc[t][u][v];
                int64_t off;
                double* base;
                if (q == 0) {  // A_E: column parity is the part
                    base = a.alm + (int64_t)k * a.almstride + 1 * csz;
                    off = calm(L, l, m, col & 1);
                } else {       // iA_B: Re(iA_B) = -Im(a_B), Im(iA_B) = Re(a_B)
                    base = a.alm + (int64_t)k * a.almstride + 2 * csz;
                    if (col & 1) off = calm(L, l, m, 0);
                    else { off = calm(L, l, m, 1); val = -val; }
                }
                if (off < 0) continue;
                if (a.accumulate) base[off] += val; else base[off] = val;
            }
    // E and B have no l < 2 coefficients: clear them once (first l tile of m < 2)
    if (!a.accumulate && m < 2 && lt == 0) {
        for (int e = tid; e < 2 * M2A2_TC * 2; e += NT) {
            const int comp = 1 + (e / (2 * M2A2_TC));
            const int rem = e % (2 * M2A2_TC);
            const int l = m + (rem >> 5 & 1);
            const int col = c0 + (rem & 31);
            const int k = col >> 1;
            if (l >= 2 || k >= a.nmaps) continue;
            int64_t off = calm(L, l, m, col & 1);
            if (off >= 0) a.alm[(int64_t)k * a.almstride + comp * csz + off] = 0.0;
        }
    }
}

// ============================================================================
// alm2map, spin 0:  E = sum_{even l-m} lambda A, O = sum_{odd} lambda A,
// T_N = E + O, T_S = E - O.   tile: 64 rings x 64 columns, l in chunks of TL.
// ============================================================================
constexpr int A2M_TR = 64;
constexpr int A2M_TC = 64;

template <typename T>
__global__ __launch_bounds__(NT) void k_a2m_spin0(LegArgs a)
{
    __shared__ T lam[2][HALF][A2M_TR + 1];   // [parity][row/2][ring]
    __shared__ T at[2][HALF][A2M_TC + 1];    // [parity][row/2][col]
    __shared__ double coef[2 * TL];

    const int nrt = (a.rn + A2M_TR - 1) / A2M_TR;
    const int g = xcd_remap(blockIdx.x, gridDim.x);
    const int m = g / (a.ctiles * nrt);
    const int rem = g - m * a.ctiles * nrt;
    const int ct = rem / nrt, rt = rem - ct * nrt;
    const int L = a.lmax;
    const int lb = lbase(0, m);
    const int po = (lb - m) & 1;
    const int r0 = rt * A2M_TR, c0 = ct * A2M_TC;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int rh = wave & 1, ch = wave >> 1;
    const double* alm = a.alm + (int64_t)a.compT * (L + 1) * (L + 1);

    int lsig = L + 1;
    for (int c = r0 / RCHUNK; c < min(a.nrc, (r0 + A2M_TR + RCHUNK - 1) / RCHUNK); ++c)
        lsig = min(lsig, a.lsig[(int64_t)m * a.nrc + c]);
    const int jstart = (lsig > L) ? 0 : (lsig - lb) / SEG;
    const int lfirst = (lsig > L) ? L + 1 : lb + SEG * (jstart & ~1);

    using MF = Mfma<T>;
    typename MF::acc accE[2][2], accO[2][2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u) accE[t][u] = accO[t][u] = typename MF::acc{0, 0, 0, 0};

    for (int lc = lfirst; lc <= L; lc += TL) {
        const int jc = (lc - lb) / SEG;
        __syncthreads();
        make_coef<0>(coef, lc, m);
        __syncthreads();
        if (tid < 2 * A2M_TR) {
            const int rl = tid & (A2M_TR - 1), s = tid / A2M_TR;
            const int r = r0 + rl;
            const int ls = lc + SEG * s;
            const int cnt = (ls <= L) ? min(SEG, L - ls + 1) : 0;
            if (r < a.rn && cnt > 0) {
                Seed0 sd = load_seed0(a, m, jc + s, r);
                fill_spin0(sd, a.rings[r].z, cnt, coef + 2 * SEG * s, [&](int i, double v) {
                    int row = SEG * s + i;
                    lam[(row + po) & 1][row >> 1][rl] = (T)v;
                });
            }
            for (int i = (r < a.rn ? cnt : 0); i < SEG; ++i) {
                int row = SEG * s + i;
                lam[(row + po) & 1][row >> 1][rl] = (T)0;
            }
        }
        // A tile: wave w loads columns w, w+4, ...; lane = row
        for (int cc = wave; cc < A2M_TC; cc += 4) {
            const int col = c0 + cc, k = col >> 1;
            const int l = lc + lane;
            double v = 0.0;
            if (l <= L && k < a.nmaps) {
                int64_t off = calm(L, l, m, col & 1);
                if (off >= 0) v = alm[(int64_t)k * a.almstride + off];
            }
            at[(lane + po) & 1][lane >> 1][cc] = (T)v;
        }
        __syncthreads();
#pragma unroll 2
        for (int ks = 0; ks < HALF / 4; ++ks) {
            const int kl = 4 * ks + (lane >> 4);
            T aE[2], aO[2], bE[2], bO[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                aE[t] = lam[0][kl][32 * rh + 16 * t + (lane & 15)];
                aO[t] = lam[1][kl][32 * rh + 16 * t + (lane & 15)];
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                bE[u] = at[0][kl][32 * ch + 16 * u + (lane & 15)];
                bO[u] = at[1][kl][32 * ch + 16 * u + (lane & 15)];
            }
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    accE[t][u] = MF::run(aE[t], bE[u], accE[t][u]);
                    accO[t][u] = MF::run(aO[t], bO[u], accO[t][u]);
                }
        }
    }

    T* X = xptr<T>(a, 0);
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = r0 + 32 * rh + 16 * t + MF::row(lane, v);
                const int col = c0 + 32 * ch + 16 * u + (lane & 15);
                if (r >= a.rn) continue;
                const double e = (double)accE[t][u][v], o = (double)accO[t][u][v];
                X[((int64_t)m * a.nring + r) * a.ldx + col] = (T)(e + o);
                const int rs = a.nring - 1 - r;
                if (rs != r) X[((int64_t)m * a.nring + rs) * a.ldx + col] = (T)(e - o);
            }
}

// ============================================================================
// alm2map, spin 2:
//   U1 = sum_even F+ E + sum_odd F- B',  U2 = sum_odd F+ E + sum_even F- B'
//   V1 = sum_even F+ B' + sum_odd F- E,  V2 = sum_odd F+ B' + sum_even F- E
//   X_N = U1 + U2, X_S = U1 - U2 (Q);  Y_N = V1 + V2, Y_S = V1 - V2 (i U)
// with B' = i a_B.  tile: 32 rings x 32 columns; wave w owns U1, U2, V1, V2.
// ============================================================================
constexpr int A2M2_TR = 32;
constexpr int A2M2_TC = 32;

template <typename T>
__global__ __launch_bounds__(NT) void k_a2m_spin2(LegArgs a)
{
    __shared__ T fpm[2][2][HALF][A2M2_TR + 1];   // [F+/F-][parity][row/2][ring]
    __shared__ T at[2][2][HALF][A2M2_TC + 1];    // [E/B'][parity][row/2][col]
    __shared__ double coef[3 * TL];

    const int nrt = (a.rn + A2M2_TR - 1) / A2M2_TR;
    const int g = xcd_remap(blockIdx.x, gridDim.x);
    const int m = g / (a.ctiles * nrt);
    const int rem = g - m * a.ctiles * nrt;
    const int ct = rem / nrt, rt = rem - ct * nrt;
    const int L = a.lmax;
    const int lb = lbase(2, m);
    const int po = (lb - m) & 1;
    const int r0 = rt * A2M2_TR, c0 = ct * A2M2_TC;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t csz = (int64_t)(L + 1) * (L + 1);
    // per wave: first (parity, F, alm) term and second term
    // U1: (0,+,E)(1,-,B')  U2: (1,+,E)(0,-,B')  V1: (0,+,B')(1,-,E)  V2: (1,+,B')(0,-,E)
    const int pa = (wave == 0 || wave == 2) ? 0 : 1;  // parity of the F+ term
    const int aa = (wave < 2) ? 0 : 1;                // alm of the F+ term (0: E, 1: B')

    int lsig = L + 1;
    if (lb <= L) lsig = a.lsig[(int64_t)m * a.nrc + r0 / RCHUNK];
    const int jstart = (lsig > L) ? 0 : (lsig - lb) / SEG;
    const int lfirst = (lsig > L) ? L + 1 : lb + SEG * (jstart & ~1);

    using MF = Mfma<T>;
    typename MF::acc acc[2][2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u) acc[t][u] = typename MF::acc{0, 0, 0, 0};

    for (int lc = lfirst; lc <= L; lc += TL) {
        const int jc = (lc - lb) / SEG;
        __syncthreads();
        make_coef<2>(coef, lc, m);
        __syncthreads();
        if (tid < 2 * A2M2_TR) {
            const int rl = tid & (A2M2_TR - 1), s = tid / A2M2_TR;
            const int r = r0 + rl;
            const int ls = lc + SEG * s;
            const int cnt = (ls <= L) ? min(SEG, L - ls + 1) : 0;
            if (r < a.rn && cnt > 0) {
                Seed2 sd = load_seed2(a, m, jc + s, r);
                fill_spin2(sd, a.rings[r].z, cnt, coef + 3 * SEG * s, [&](int i, double fp, double fm) {
                    int row = SEG * s + i;
                    int c = (row + po) & 1;
                    fpm[0][c][row >> 1][rl] = (T)fp;
                    fpm[1][c][row >> 1][rl] = (T)fm;
                });
            }
            for (int i = (r < a.rn ? cnt : 0); i < SEG; ++i) {
                int row = SEG * s + i;
                int c = (row + po) & 1;
                fpm[0][c][row >> 1][rl] = (T)0;
                fpm[1][c][row >> 1][rl] = (T)0;
            }
        }
        // alm tiles: E and B' = i a_B (Re B' = -Im a_B, Im B' = Re a_B)
        for (int cc = wave; cc < 2 * A2M2_TC; cc += 4) {
            const int which = cc / A2M2_TC;   // 0: E, 1: B'
            const int cl = cc - which * A2M2_TC;
            const int col = c0 + cl, k = col >> 1;
            const int l = lc + lane;
            double v = 0.0;
            if (l <= L && k < a.nmaps) {
                const double* base = a.alm + (int64_t)k * a.almstride + (1 + which) * csz;
                if (which == 0) {
                    int64_t off = calm(L, l, m, col & 1);
                    if (off >= 0) v = base[off];
                } else if (col & 1) {
                    v = base[calm(L, l, m, 0)];
                } else {
                    int64_t off = calm(L, l, m, 1);
                    if (off >= 0) v = -base[off];
                }
            }
            at[which][(lane + po) & 1][lane >> 1][cl] = (T)v;
        }
        __syncthreads();
#pragma unroll 2
        for (int ks = 0; ks < HALF / 4; ++ks) {
            const int kl = 4 * ks + (lane >> 4);
            T a1[2], a2[2], b1[2], b2[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                a1[t] = fpm[0][pa][kl][16 * t + (lane & 15)];
                a2[t] = fpm[1][pa ^ 1][kl][16 * t + (lane & 15)];
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                b1[u] = at[aa][pa][kl][16 * u + (lane & 15)];
                b2[u] = at[aa ^ 1][pa ^ 1][kl][16 * u + (lane & 15)];
            }
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    acc[t][u] = MF::run(a1[t], b1[u], acc[t][u]);
                    acc[t][u] = MF::run(a2[t], b2[u], acc[t][u]);
                }
        }
    }

    // combine U1/U2 and V1/V2 across waves through LDS (reuses the alm tile space)
    __syncthreads();
    double* ex = reinterpret_cast<double*>(&at[0][0][0][0]);  // 4 x 32 x 32 doubles needed
    static_assert(sizeof(at) >= 4 * A2M2_TR * A2M2_TC * sizeof(float), "exchange space");
    constexpr bool fits = sizeof(at) >= 4 * A2M2_TR * A2M2_TC * sizeof(double);
    float* exf = reinterpret_cast<float*>(&at[0][0][0][0]);
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int rl = 16 * t + MF::row(lane, v);
                const int cl = 16 * u + (lane & 15);
                const int idx = (wave * A2M2_TR + rl) * A2M2_TC + cl;
                if constexpr (fits) ex[idx] = (double)acc[t][u][v];
                else exf[idx] = (float)acc[t][u][v];
            }
    __syncthreads();
    T* XQ = xptr<T>(a, 1);
    T* XU = xptr<T>(a, 2);
    for (int e = tid; e < A2M2_TR * (A2M2_TC / 2); e += NT) {
        const int rl = e / (A2M2_TC / 2), cp = e - rl * (A2M2_TC / 2);
        const int r = r0 + rl;
        if (r >= a.rn) continue;
        double w[4][2];
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int z = 0; z < 2; ++z) {
                const int idx = (s * A2M2_TR + rl) * A2M2_TC + 2 * cp + z;
                if constexpr (fits) w[s][z] = ex[idx];
                else w[s][z] = (double)exf[idx];
            }
        // Q = X, U = -i Y: (U_re, U_im) = (Y_im, -Y_re)
        const int64_t on = ((int64_t)m * a.nring + r) * a.ldx + c0 + 2 * cp;
        XQ[on] = (T)(w[0][0] + w[1][0]);
        XQ[on + 1] = (T)(w[0][1] + w[1][1]);
        XU[on] = (T)(w[2][1] + w[3][1]);
        XU[on + 1] = (T)(-(w[2][0] + w[3][0]));
        const int rs = a.nring - 1 - r;
        if (rs != r) {
            const int64_t os = ((int64_t)m * a.nring + rs) * a.ldx + c0 + 2 * cp;
            XQ[os] = (T)(w[0][0] - w[1][0]);
            XQ[os + 1] = (T)(w[0][1] - w[1][1]);
            XU[os] = (T)(w[2][1] - w[3][1]);
            XU[os + 1] = (T)(-(w[2][0] - w[3][0]));
        }
    }
}

template <typename T>
hipError_t launch_m2a_t(const LegArgs& a, hipStream_t st)
{
    if (a.spin == 0) {
        LegArgs b = a;
        b.ctiles = (int)((a.ldx + M2A_TC - 1) / M2A_TC);
        hipLaunchKernelGGL(k_m2a_spin0<T>, dim3(b.ntiles * b.ctiles), dim3(NT), 0, st, b);
    } else {
        LegArgs b = a;
        b.ctiles = (int)((a.ldx + M2A2_TC - 1) / M2A2_TC);
        hipLaunchKernelGGL(k_m2a_spin2<T>, dim3(b.ntiles * b.ctiles), dim3(NT), 0, st, b);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_a2m_t(const LegArgs& a, hipStream_t st)
{
    LegArgs b = a;
    if (a.spin == 0) {
        b.ctiles = (int)((a.ldx + A2M_TC - 1) / A2M_TC);
        int nrt = (a.rn + A2M_TR - 1) / A2M_TR;
        hipLaunchKernelGGL(k_a2m_spin0<T>, dim3((a.lmax + 1) * b.ctiles * nrt), dim3(NT), 0, st, b);
    } else {
        b.ctiles = (int)((a.ldx + A2M2_TC - 1) / A2M2_TC);
        int nrt = (a.rn + A2M2_TR - 1) / A2M2_TR;
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
