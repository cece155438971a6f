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
#include "leg_rec.h"

namespace sht {
namespace {

constexpr int NT = 256;
constexpr int HALF = TL / 2;   // rows of one parity class per l tile
constexpr int KS = 8;          // MFMA K-steps per tile (4 rings, or 4 l per class, each)
constexpr int RPK = SEG / KS;  // recursion rows emitted per K-step
static_assert(RPK * KS == SEG, "the fill of one segment is spread over the K-steps of a tile");
constexpr int M_TR = 32;       // map2alm: rings per chunk (= RCHUNK, the skip granularity)
static_assert(M_TR == RCHUNK, "ring chunks and skip-table entries coincide");

// ============================================================================
// map2alm, spin 0: A_l = sum_{north rings} lambda_l (T_N +- T_S), raw sums into
// the m-major coefficient workspace.  Tile: 64 l x 64*NU columns; rings in
// chunks of 32; wave w owns NU column tiles of 16 and all 64 rows.
// ============================================================================
template <typename T, int NU, bool NW = false>
__global__ __launch_bounds__(NT, 2) void k_m2a_spin0(LegArgs a)
{
    constexpr int RS = HALF + 1;        // [ring][row/2]
    constexpr int CLS = M_TR * RS, BUF = 2 * CLS;
    __shared__ T lam[2 * BUF];          // [buffer][parity class][ring][row/2]

    int m, lt, ct;
    int g = xcd_remap(blockIdx.x, gridDim.x);
    const int sk = split_part(a, g);
    decode_tiles(a, g, m, lt, ct);
    const int L = a.lmax, lb = m;
    const int l0 = lb + lt * TL, lend = min(L, l0 + TL - 1);
    const int lane = threadIdx.x & 63, wave = wave_index();
    const int col = NW ? (lane & 15) : ct * (64 * NU) + 16 * NU * wave + (lane & 15);
    // narrow tile (NW: at most 8 map sets, the first 16 columns): the four waves
    // split the tile's output blocks instead of its columns
    auto mine = [&](int p, int t) { return !NW || (p == (wave >> 1) && t == (wave & 1)); };
    // fill items: 32 rings x SPT segments, one per lane (segment uniform per half-wave)
    static_assert(M_TR * SPT == NT, "one fill item per thread");
    constexpr bool filler = true;
    const int frl = lane & 31;
    const int fs = 2 * wave + (lane >> 5);
    const int ls = l0 + SEG * fs;
    const int cnt = min(SEG, L - ls + 1);
    const int64_t row0 = a.rowoff[m];
    __shared__ double ctile[CoefTile<2>::N];
    CoefTile<2>::put(ctile, CoefTile<2>::fetch(a, row0 + (l0 - lb)));
    __syncthreads();
    const double* cp = ctile + SEG * fs * 2;
    const int jseg = min(SPT * lt + fs, (L - lb) / SEG);
    const int64_t sbase = a.seedoff[m] + (int64_t)jseg * a.rn;

    using MF = Mfma<T>;
    typename MF::acc acc[2][2][NU];  // [parity][row tile][column tile]
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int u = 0; u < NU; ++u) acc[p][t][u] = typename MF::acc{0, 0, 0, 0};

    int nchunk = (a.rn + M_TR - 1) / M_TR;
    int rc0 = first_chunk(a, m, nchunk, lend);
    split_range(a, sk, rc0, nchunk);
    if (rc0 < nchunk) {
        // Ring chunks run from the equator toward the pole (chunk q of the loop is
        // rsum - q): every l tile of an m needs the equator chunks, so the
        // workgroups of one m, launched together, stream the same ring rows in
        // step and share them in L2 instead of each reading its own from HBM.
        const int rsum = rc0 + nchunk - 1;
        const T* Xm = xptr<T>(a, 0) + (int64_t)m * a.nring * a.ldx + col;
        auto seed_of = [&](Seed<0>& s, int rc) {
            rc = rsum - rc;
            const int r = min(rc * M_TR + frl, a.rn - 1);
            seed_load(s, a, sbase + r, r);
        };
        auto emit_to = [&](int b) {
            Emit<T, 1, 0> e;
            e.e0 = lam + b * BUF + frl * RS + (SEG / 2) * fs;
            e.e1 = e.e0 + CLS;
            return e;
        };
        // ring operands, loaded three K-steps before their MFMAs: raw north /
        // south rows of two K-steps in flight, and the folded sums of the
        // current one
        T xb[2][2][NU];  // [K-step parity][north, south][column tile]
        T xs[2][NU];     // [T_N + T_S, T_N - T_S][column tile]
        auto load_x = [&](int rc, int ks, T (&d)[2][NU]) {
            rc = rsum - rc;
            const int r = min(rc * M_TR + 4 * ks + (lane >> 4), a.rn - 1);
            const T* pn = Xm + (int64_t)r * a.ldx;
            const T* ps = Xm + (int64_t)(a.nring - 1 - r) * a.ldx;
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                d[0][u] = pn[16 * u];
                d[1][u] = ps[16 * u];
            }
        };
        auto fold = [&](const T (&d)[2][NU]) {
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                xs[0][u] = d[0][u] + d[1][u];
                xs[1][u] = d[0][u] - d[1][u];
            }
        };
        static_assert(KS % 2 == 0 && KS >= 3, "the raw buffers alternate with the K-step parity");

        Seed<0> sd;
        Rec<0> f;
        seed_of(sd, rc0);
        if (filler) {
            f.start(sd, m2a_weight(a, (rsum - rc0) * M_TR + frl));
            auto em = emit_to(0);
            rec_all(f, cp, cnt, em);
        }
        seed_of(sd, min(rc0 + 1, nchunk - 1));
        load_x(rc0, 0, xb[0]);
        load_x(rc0, 1, xb[1]);
        fold(xb[0]);
        load_x(rc0, 2, xb[0]);
        __syncthreads();
        for (int rc = rc0; rc < nchunk; ++rc) {
            const int b = (rc - rc0) & 1;
            const int rcn = min(rc + 1, nchunk - 1);
            if (filler) f.start(sd, m2a_weight(a, (rsum - rcn) * M_TR + frl));
            auto em = emit_to(b ^ 1);
            const T* lb_ = lam + b * BUF;
            static_for<0, KS>([&](auto ki) {
                constexpr int ks = decltype(ki)::v;
                if constexpr (ks == KS / 2) seed_of(sd, min(rc + 2, nchunk - 1));
                const int kr = 4 * ks + (lane >> 4);
                T av[2][2];
#pragma unroll
                for (int p = 0; p < 2; ++p)
#pragma unroll
                    for (int t = 0; t < 2; ++t)
                        if (mine(p, t)) av[p][t] = lb_[p * CLS + kr * RS + 16 * t + (lane & 15)];
#pragma unroll
                for (int u = 0; u < NU; ++u)
#pragma unroll
                    for (int t = 0; t < 2; ++t) {
                        if (mine(0, t)) acc[0][t][u] = MF::run(av[0][t], xs[0][u], acc[0][t][u]);
                        if (mine(1, t)) acc[1][t][u] = MF::run(av[1][t], xs[1][u], acc[1][t][u]);
                    }
                // sums of the next K-step; its raw buffer then takes the K-step
                // three ahead (in the next chunk for the last three)
                fold(xb[(ks + 1) & 1]);
                if constexpr (ks + 3 < KS) load_x(rc, ks + 3, xb[(ks + 1) & 1]);
                else load_x(rcn, ks + 3 - KS, xb[(ks + 1) & 1]);
                __builtin_amdgcn_sched_barrier(0);
                if (filler) rec_group<ks, RPK>(f, cp, cnt, em);
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
                if (!mine(p, t)) continue;
                const int ci = 16 * t + MF::row(lane, v);
                const int l = l0 + 2 * ci + p;
                if (l > L) continue;
#pragma unroll
                for (int u = 0; u < NU; ++u) put_out(&A[(int64_t)(l - lb) * a.ldx + col + 16 * u], (T)acc[p][t][u][v], a.ksplit > 1);
            }
}

// ============================================================================
// map2alm, spin 2 (E and iB from Q and iU):
//   even l-m: A_E = F+ SX + F- DY,  iA_B = F+ SY + F- DX
//   odd  l-m: A_E = F+ DX + F- SY,  iA_B = F+ DY + F- SX
// X = Q coefficients, Y = iU; S/D = north +- south.  Tile 64 l x 64*NU columns,
// rings in chunks of 32; wave w owns NU column tiles of 16.  EB = 1 (E only) or
// 2 (B only) computes one block row of the transform; the other stays zero.
// ============================================================================
template <typename T, int NU, int EB, bool NW = false>
__global__ __launch_bounds__(NT, 2) void k_m2a_spin2(LegArgs a)
{
    constexpr int RS = HALF + 1;
    constexpr int CLS = M_TR * RS, FOFF = 2 * CLS, BUF = 4 * CLS;
    __shared__ T fpm[2 * BUF];  // [buffer][F+ / F-][parity class][ring][row/2]

    int m, lt, ct;
    int g = xcd_remap(blockIdx.x, gridDim.x);
    const int sk = split_part(a, g);
    decode_tiles(a, g, m, lt, ct);
    const int L = a.lmax, lb = lbase(2, m);
    const int l0 = lb + lt * TL, lend = min(L, l0 + TL - 1);
    const int po = (lb - m) & 1;
    const int lane = threadIdx.x & 63, wave = wave_index();
    const int col = NW ? (lane & 15) : ct * (64 * NU) + 16 * NU * wave + (lane & 15);
    // narrow tile (NW: at most 8 map sets, the first 16 columns): the four waves
    // split the tile's output blocks instead of its columns
    auto mine = [&](int p, int t) { return !NW || (p == (wave >> 1) && t == (wave & 1)); };
    const int pcol = col ^ 1;                           // Y = iU swaps re/im: partner column
    const unsigned ysg = (col & 1) ? 0u : 0x80000000u;  // Y_re = -U_im, Y_im = U_re
    // fill items: 32 rings x SPT segments, one per lane (segment uniform per half-wave)
    static_assert(M_TR * SPT == NT, "one fill item per thread");
    constexpr bool filler = true;
    const int frl = lane & 31;
    const int fs = 2 * wave + (lane >> 5);
    const int ls = l0 + SEG * fs;
    const int cnt = min(SEG, L - ls + 1);
    const int64_t row0 = a.rowoff[m];
    __shared__ double ctile[CoefTile<4>::N];
    CoefTile<4>::put(ctile, CoefTile<4>::fetch(a, row0 + (l0 - lb)));
    __syncthreads();
    const double* cp = ctile + SEG * fs * 4;
    const int jseg = min(SPT * lt + fs, (L - lb) / SEG);
    const int64_t sbase = a.seedoff[m] + (int64_t)jseg * a.rn;

    using MF = Mfma<T>;
    typename MF::acc accE[2][2][NU], accB[2][2][NU];  // [parity][row tile][column tile]
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int u = 0; u < NU; ++u) accE[p][t][u] = accB[p][t][u] = typename MF::acc{0, 0, 0, 0};

    int nchunk = (a.rn + M_TR - 1) / M_TR;
    int rc0 = first_chunk(a, m, nchunk, lend);
    split_range(a, sk, rc0, nchunk);
    if (rc0 < nchunk) {
        // Ring chunks run from the equator toward the pole (chunk q of the loop is
        // rsum - q): every l tile of an m needs the equator chunks, so the
        // workgroups of one m, launched together, stream the same ring rows in
        // step and share them in L2 instead of each reading its own from HBM.
        const int rsum = rc0 + nchunk - 1;
        const int64_t xm = (int64_t)m * a.nring * a.ldx;
        const T* XQ = xptr<T>(a, 1) + xm + col;
        const T* XU = xptr<T>(a, 2) + xm + pcol;
        auto seed_of = [&](Seed<2>& s, int rc) {
            rc = rsum - rc;
            const int r = min(rc * M_TR + frl, a.rn - 1);
            seed_load(s, a, sbase + r, r);
        };
        auto emit_to = [&](int b) {
            Emit<T, 1, FOFF> e;
            e.e0 = fpm + b * BUF + po * CLS + frl * RS + (SEG / 2) * fs;
            e.e1 = fpm + b * BUF + (po ^ 1) * CLS + frl * RS + (SEG / 2) * fs;
            return e;
        };
        T xb[2][4][NU];  // [K-step parity][Q_N, Q_S, U_N, U_S (partner column)][column tile]
        auto load_x = [&](int rc, int ks, T (&d)[4][NU]) {
            rc = rsum - rc;
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
            f.start(sd, m2a_weight(a, (rsum - rc0) * M_TR + frl));
            auto em = emit_to(0);
            rec_all(f, cp, cnt, em);
        }
        seed_of(sd, min(rc0 + 1, nchunk - 1));
        load_x(rc0, 0, xb[0]);
        __syncthreads();
        for (int rc = rc0; rc < nchunk; ++rc) {
            const int b = (rc - rc0) & 1;
            const int rcn = min(rc + 1, nchunk - 1);
            if (filler) f.start(sd, m2a_weight(a, (rsum - rcn) * M_TR + frl));
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
                        if (!mine(p, t)) continue;
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
                        if constexpr (EB != 2) {
                            if (mine(0, t)) accE[0][t][u] = MF::run(fp[0][t], sx, accE[0][t][u]);
                            if (mine(1, t)) accE[1][t][u] = MF::run(fp[1][t], dx, accE[1][t][u]);
                        }
                        if constexpr (EB != 1) {
                            if (mine(0, t)) accB[0][t][u] = MF::run(fp[0][t], sy, accB[0][t][u]);
                            if (mine(1, t)) accB[1][t][u] = MF::run(fp[1][t], dy, accB[1][t][u]);
                        }
                    }
#pragma unroll
                    for (int t = 0; t < 2; ++t) {
                        if constexpr (EB != 2) {
                            if (mine(0, t)) accE[0][t][u] = MF::run(fm[0][t], dy, accE[0][t][u]);
                            if (mine(1, t)) accE[1][t][u] = MF::run(fm[1][t], sy, accE[1][t][u]);
                        }
                        if constexpr (EB != 1) {
                            if (mine(0, t)) accB[0][t][u] = MF::run(fm[0][t], dx, accB[0][t][u]);
                            if (mine(1, t)) accB[1][t][u] = MF::run(fm[1][t], sx, accB[1][t][u]);
                        }
                    }
                }
                if (filler) rec_group<ks, RPK>(f, cp, cnt, em);
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
                if (!mine(p, t)) continue;
                const int ci = 16 * t + MF::row(lane, v);
                const int l = l0 + 2 * ci + (p ^ po);
                if (l > L) continue;
#pragma unroll
                for (int u = 0; u < NU; ++u) {
                    const int64_t o = (int64_t)(l - lb) * a.ldx + col + 16 * u;
                    put_out(&AE[o], (T)accE[p][t][u][v], a.ksplit > 1);
                    put_out(&AB[o], (T)accB[p][t][u][v], a.ksplit > 1);
                }
            }
}

// ============================================================================
// alm2map, spin 0: E = sum_{even l-m} lambda A, O = sum_{odd} lambda A,
// T_N = E + O, T_S = E - O.  Tile: 64 rings x 64*NU columns, l in chunks of 64;
// wave w owns NU column tiles of 16 and all 64 rings.
// ============================================================================
constexpr int A0_TR = 64;

template <typename T, int NU, bool NW = false>
__global__ __launch_bounds__(NT, 2) void k_a2m_spin0(LegArgs a)
{
    constexpr int RS = A0_TR + 1;       // [row/2][ring]
    constexpr int CLS = HALF * RS, BUF = 2 * CLS;
    __shared__ T lam[2 * BUF];          // [buffer][parity class][row/2][ring]
    __shared__ double ctile[2][CoefTile<2>::N];

    const int nrt = (a.rn + A0_TR - 1) / A0_TR;
    int g = xcd_remap(blockIdx.x, gridDim.x);
    const int sk = split_part(a, g);
    const int mi = g / (a.ctiles * nrt);
    const int m = a.mlist ? a.mlist[mi] : mfold(mi, a.lmax);
    const int rem = g - mi * a.ctiles * nrt;
    const int ct = rem / nrt, rt = rem - ct * nrt;
    const int L = a.lmax, lb = m;
    const int r0 = rt * A0_TR;
    const int lane = threadIdx.x & 63, wave = wave_index();
    const int col = NW ? (lane & 15) : ct * (64 * NU) + 16 * NU * wave + (lane & 15);
    // narrow tile (NW: at most 8 map sets, the first 16 columns): the four waves
    // split the tile's output blocks instead of its columns
    auto mine = [&](int t) { return !NW || t == wave; };
    // fill items: 64 rings x SPT segments, two per lane: ring = lane, segments
    // wave and wave + 4 (wave-uniform)
    static_assert(A0_TR * SPT == 2 * NT && SPT == 8, "two fill items per thread");
    const int frl = lane;
    const int fs0 = wave;
    const int fr = r0 + frl;
    const int frc = min(fr, a.rn - 1);
    const double w = fr < a.rn ? 1.0 : 0.0;

    int lfirst, nch;
    a2m_range(a, m, lb, r0, A0_TR, lfirst, nch);
    if (a.ksplit > 1) {
        int c0 = 0, c1 = nch;
        split_range(a, sk, c0, c1);
        lfirst += TL * c0;
        nch = c1 - c0;
    }

    using MF = Mfma<T>;
    typename MF::acc accE[4][NU], accO[4][NU];  // [ring tile][column tile]
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int u = 0; u < NU; ++u) accE[t][u] = accO[t][u] = typename MF::acc{0, 0, 0, 0};

    if (nch > 0) {
        const int64_t row0 = a.rowoff[m];
        const T* Am = aptr<T>(a, 0) + row0 * a.ldx + col;
        const int64_t sb = a.seedoff[m] + frc;
        const int j0 = (lfirst - lb) / SEG + fs0;
        const int jmax = (L - lb) / SEG;  // last segment of this m
        // item i of this lane: segment fs0 + 4 i
        auto seed_of = [&](Seed<0>& s, int c, int i) {
            seed_load(s, a, sb + (int64_t)min(j0 + 4 * i + SPT * c, jmax) * a.rn, frc);
        };
        auto ls_of = [&](int c, int i) { return lfirst + TL * c + SEG * (fs0 + 4 * i); };
        auto emit_to = [&](int b, int i) {
            Emit<T, RS, 0> e;
            e.e0 = lam + b * BUF + (SEG / 2) * (fs0 + 4 * i) * RS + frl;
            e.e1 = e.e0 + CLS;
            return e;
        };
        // coefficient operands, loaded PD K-steps ahead: two for FP64, one for
        // FP32 (whose widest tiling has no registers for more)
        constexpr int PD = sizeof(T) == 8 ? 2 : 1, NB = 2 * PD;
        static_assert(KS % NB == 0, "the operand buffers cycle with the K-step index");
        T bb[NB][2][NU];  // [K-step mod NB][even, odd class row][column tile]
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

        Seed<0> sd[2];
        Rec<0> f[2];
        using CT = CoefTile<2>;
        auto tile_row = [&](int c) { return row0 + (lfirst + TL * c - lb); };
        CT::put(ctile[0], CT::fetch(a, tile_row(0)));
        CT::put(ctile[1], CT::fetch(a, tile_row(min(1, nch - 1))));
        double cnext = CT::fetch(a, tile_row(min(2, nch - 1)));
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            seed_of(sd[i], 0, i);
            f[i].start(sd[i], w);
            auto em = emit_to(0, i);
            rec_all(f[i], ctile[0] + SEG * (fs0 + 4 * i) * 2, min(SEG, L - ls_of(0, i) + 1), em);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i) seed_of(sd[i], min(1, nch - 1), i);
#pragma unroll
        for (int k = 0; k < PD; ++k) load_a(0, k, bb[k]);
        __syncthreads();
        for (int c = 0; c < nch; ++c) {
            const int b = c & 1;
            const int cn = min(c + 1, nch - 1);
            const double* cp0 = ctile[(c + 1) & 1] + SEG * fs0 * 2;
            const double* cp1 = cp0 + SEG * 4 * 2;
            const int cnt0 = min(SEG, L - ls_of(cn, 0) + 1), cnt1 = min(SEG, L - ls_of(cn, 1) + 1);
#pragma unroll
            for (int i = 0; i < 2; ++i) f[i].start(sd[i], w);
            auto em0 = emit_to(b ^ 1, 0);
            auto em1 = emit_to(b ^ 1, 1);
            const T* lb_ = lam + b * BUF;
            // recursion operands of one K-step from the LDS tile, read one K-step
            // ahead within the chunk where the registers allow (wide FP64 tiles)
            constexpr bool RA = sizeof(T) == 8 && !NW;
            T aw[RA ? 2 : 1][4][2];  // [K-step parity][ring tile][even, odd class row]
            auto read_lam = [&](int ks, T (&d)[4][2]) {
                const int kl = 4 * ks + (lane >> 4);
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    if (!mine(t)) continue;
                    d[t][0] = lb_[kl * RS + 16 * t + (lane & 15)];
                    d[t][1] = lb_[CLS + kl * RS + 16 * t + (lane & 15)];
                }
            };
            if constexpr (RA) read_lam(0, aw[0]);
            static_for<0, KS>([&](auto ki) {
                constexpr int ks = decltype(ki)::v;
                if constexpr (ks + PD < KS) load_a(c, ks + PD, bb[(ks + PD) % NB]);
                else load_a(cn, ks + PD - KS, bb[(ks + PD) % NB]);
                if constexpr (RA && ks + 1 < KS) read_lam(ks + 1, aw[(ks + 1) & 1]);
                if constexpr (ks == KS / 2) {
#pragma unroll
                    for (int i = 0; i < 2; ++i) seed_of(sd[i], min(c + 2, nch - 1), i);
                }
                // keep the prefetch ahead of this step's compute (the scheduler may sink it)
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    if (!mine(t)) continue;
                    T aE, aO;
                    if constexpr (RA) {
                        aE = aw[ks & 1][t][0];
                        aO = aw[ks & 1][t][1];
                    } else {
                        const int kl = 4 * ks + (lane >> 4);
                        aE = lb_[kl * RS + 16 * t + (lane & 15)];
                        aO = lb_[CLS + kl * RS + 16 * t + (lane & 15)];
                    }
#pragma unroll
                    for (int u = 0; u < NU; ++u) {
                        accE[t][u] = MF::run(aE, bb[ks % NB][0][u], accE[t][u]);
                        accO[t][u] = MF::run(aO, bb[ks % NB][1][u], accO[t][u]);
                    }
                }
                rec_group<ks, RPK>(f[0], cp0, cnt0, em0);
                rec_group<ks, RPK>(f[1], cp1, cnt1, em1);
            });
            CT::put(ctile[c & 1], cnext);  // tile of chunk c + 2
            cnext = CT::fetch(a, tile_row(min(c + 3, nch - 1)));
            __syncthreads();
        }
    }

    T* X = xptr<T>(a, 0) + (int64_t)m * a.nring * a.ldx + col;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            if (!mine(t)) continue;
            const int r = r0 + 16 * t + MF::row(lane, v);
            if (r >= a.rn) continue;
            const int rs = a.nring - 1 - r;
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const T e = accE[t][u][v], o = accO[t][u][v];
                put_out(&X[(int64_t)r * a.ldx + 16 * u], (T)(e + o), a.ksplit > 1);
                if (rs != r) put_out(&X[(int64_t)rs * a.ldx + 16 * u], (T)(e - o), a.ksplit > 1);
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

// EB = 1 (E only) or 2 (B only) drops the other block's loads and products:
// the half-block transforms of pixel-domain E/B separation (Sec. 2.3).
template <typename T, int NU, int EB, bool NW = false>
__global__ __launch_bounds__(NT, 2) void k_a2m_spin2(LegArgs a)
{
    constexpr int RS = A2_TR + 1;
    constexpr int CLS = HALF * RS, FOFF = 2 * CLS, BUF = 4 * CLS;
    __shared__ T fpm[2 * BUF];  // [buffer][F+ / F-][parity class][row/2][ring]
    __shared__ double ctile[2][CoefTile<4>::N];

    const int nrt = (a.rn + A2_TR - 1) / A2_TR;
    int g = xcd_remap(blockIdx.x, gridDim.x);
    const int sk = split_part(a, g);
    const int mi = g / (a.ctiles * nrt);
    const int m = a.mlist ? a.mlist[mi] : mfold(mi, a.lmax);
    const int rem = g - mi * a.ctiles * nrt;
    const int ct = rem / nrt, rt = rem - ct * nrt;
    const int L = a.lmax, lb = lbase(2, m);
    const int po = (lb - m) & 1;
    const int r0 = rt * A2_TR;
    const int lane = threadIdx.x & 63, wave = wave_index();
    const int col = NW ? (lane & 15) : ct * (64 * NU) + 16 * NU * wave + (lane & 15);
    // narrow tile (NW: at most 8 map sets, the first 16 columns): the four waves
    // split the tile's output blocks instead of its columns
    // (waves 0 and 1: the Q sums of ring tiles 0 and 1; waves 2 and 3: the iU sums)
    auto mineq = [&](int t) { return !NW || (t == (wave & 1) && wave < 2); };
    auto mineu = [&](int t) { return !NW || (t == (wave & 1) && wave >= 2); };
    static_assert(A2_TR * SPT == NT, "one fill item per thread");
    constexpr bool filler = true;
    const int frl = lane & 31;
    const int fs = 2 * wave + (lane >> 5);
    const int fr = r0 + frl;
    const int frc = min(fr, a.rn - 1);
    const double w = fr < a.rn ? 1.0 : 0.0;

    int lfirst, nch;
    a2m_range(a, m, lb, r0, A2_TR, lfirst, nch);
    if (a.ksplit > 1) {
        int c0 = 0, c1 = nch;
        split_range(a, sk, c0, c1);
        lfirst += TL * c0;
        nch = c1 - c0;
    }

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
        const int64_t sb = a.seedoff[m] + frc;
        const int j0 = (lfirst - lb) / SEG + fs;
        const int jmax = (L - lb) / SEG;  // last segment of this m
        auto seed_of = [&](Seed<2>& s, int c) { seed_load(s, a, sb + (int64_t)min(j0 + SPT * c, jmax) * a.rn, frc); };
        auto ls_of = [&](int c) { return lfirst + TL * c + SEG * fs; };
        auto emit_to = [&](int b) {
            Emit<T, RS, FOFF> e;
            e.e0 = fpm + b * BUF + po * CLS + (SEG / 2) * fs * RS + frl;
            e.e1 = fpm + b * BUF + (po ^ 1) * CLS + (SEG / 2) * fs * RS + frl;
            return e;
        };
        T bb[2][4][NU];  // [K-step parity][E even, E odd, B' even, B' odd][column tile]
        auto load_a = [&](int c, int ks, T (&d)[4][NU]) {
            const int lc = lfirst + TL * c + 2 * (4 * ks + (lane >> 4));
            const int64_t oe = (int64_t)(min(lc + po, L) - lb) * a.ldx;
            const int64_t oo = (int64_t)(min(lc + (po ^ 1), L) - lb) * a.ldx;
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                if constexpr (EB != 2) {
                    d[0][u] = AE[oe + 16 * u];
                    d[1][u] = AE[oo + 16 * u];
                } else {
                    d[0][u] = d[1][u] = T(0);
                }
                if constexpr (EB != 1) {
                    d[2][u] = AB[oe + 16 * u];
                    d[3][u] = AB[oo + 16 * u];
                } else {
                    d[2][u] = d[3][u] = T(0);
                }
            }
        };

        Seed<2> sd;
        Rec<2> f;
        using CT = CoefTile<4>;
        auto tile_row = [&](int c) { return row0 + (lfirst + TL * c - lb); };
        CT::put(ctile[0], CT::fetch(a, tile_row(0)));
        CT::put(ctile[1], CT::fetch(a, tile_row(min(1, nch - 1))));
        double cnext = CT::fetch(a, tile_row(min(2, nch - 1)));
        __syncthreads();
        seed_of(sd, 0);
        if (filler) {
            f.start(sd, w);
            auto em = emit_to(0);
            rec_all(f, ctile[0] + SEG * fs * 4, min(SEG, L - ls_of(0) + 1), em);
        }
        seed_of(sd, min(1, nch - 1));
        load_a(0, 0, bb[0]);
        __syncthreads();
        for (int c = 0; c < nch; ++c) {
            const int b = c & 1;
            const int cn = min(c + 1, nch - 1);
            const double* cp = ctile[(c + 1) & 1] + SEG * fs * 4;
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
                    if (!mineq(t) && !mineu(t)) continue;
                    const int o = kl * RS + 16 * t + (lane & 15);
                    const T pe = fb[o], pd = fb[CLS + o];
                    const T me = fb[FOFF + o], mo = fb[FOFF + CLS + o];
#pragma unroll
                    for (int u = 0; u < NU; ++u) {
                        if constexpr (EB != 2) {
                            if (mineq(t)) u1[t][u] = MF::run(pe, d[0][u], u1[t][u]);
                            if (mineq(t)) u2[t][u] = MF::run(pd, d[1][u], u2[t][u]);
                        }
                        if constexpr (EB != 1) {
                            if (mineu(t)) v1[t][u] = MF::run(pe, d[2][u], v1[t][u]);
                            if (mineu(t)) v2[t][u] = MF::run(pd, d[3][u], v2[t][u]);
                        }
                    }
#pragma unroll
                    for (int u = 0; u < NU; ++u) {
                        if constexpr (EB != 2) {
                            if (mineu(t)) v1[t][u] = MF::run(mo, d[1][u], v1[t][u]);
                            if (mineu(t)) v2[t][u] = MF::run(me, d[0][u], v2[t][u]);
                        }
                        if constexpr (EB != 1) {
                            if (mineq(t)) u1[t][u] = MF::run(mo, d[3][u], u1[t][u]);
                            if (mineq(t)) u2[t][u] = MF::run(me, d[2][u], u2[t][u]);
                        }
                    }
                }
                if (filler) rec_group<ks, RPK>(f, cp, cnt, em);
            });
            CT::put(ctile[c & 1], cnext);  // tile of chunk c + 2
            cnext = CT::fetch(a, tile_row(min(c + 3, nch - 1)));
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
                if (mineq(t)) {
                    put_out(&XQ[(int64_t)r * a.ldx + 16 * u], (T)(U1 + U2), a.ksplit > 1);
                    if (rs != r) put_out(&XQ[(int64_t)rs * a.ldx + 16 * u], (T)(U1 - U2), a.ksplit > 1);
                }
                if (mineu(t)) {
                    put_out(&XU[(int64_t)r * a.ldx + 16 * u], flip((T)(V1 + V2), usg), a.ksplit > 1);
                    if (rs != r) put_out(&XU[(int64_t)rs * a.ldx + 16 * u], flip((T)(V1 - V2), usg), a.ksplit > 1);
                }
            }
        }
}

// widest column tiling (64 NU columns per workgroup, NU <= NUMAX) that divides ldx
int pick_nu(int numax, int64_t ldx)
{
    int nu = numax;
    while (nu > 1 && ldx % (64 * nu) != 0) nu >>= 1;
    return nu;
}

// Column tiling per kernel: the widest NU whose registers fit two waves per SIMD
// without spilling (spin 0, map2alm FP64: 4; spin-0 FP32: 4; the rest: 2), and
// NU = 1 for batches of at most 32 map sets (64 columns).
template <typename T>
hipError_t launch_m2a_t(const LegArgs& a, hipStream_t st)
{
    LegArgs b = a;
    const dim3 blk(NT);
    if (a.spin == 0) {
        const int nu = pick_nu(4, a.ldx);
        b.ctiles = (int)(a.ldx / (64 * nu));
        const dim3 grid(b.ntiles * b.ctiles * kparts(a));
        if (narrow(a)) hipLaunchKernelGGL((k_m2a_spin0<T, 1, true>), grid, blk, 0, st, b);
        else if (nu == 4) hipLaunchKernelGGL((k_m2a_spin0<T, 4>), grid, blk, 0, st, b);
        else if (nu == 2) hipLaunchKernelGGL((k_m2a_spin0<T, 2>), grid, blk, 0, st, b);
        else hipLaunchKernelGGL((k_m2a_spin0<T, 1>), grid, blk, 0, st, b);
    } else {
        const int nu = pick_nu(2, a.ldx);
        b.ctiles = (int)(a.ldx / (64 * nu));
        const dim3 grid(b.ntiles * b.ctiles * kparts(a));
        if (nu == 2) {
            if (a.eb == 1) hipLaunchKernelGGL((k_m2a_spin2<T, 2, 1>), grid, blk, 0, st, b);
            else if (a.eb == 2) hipLaunchKernelGGL((k_m2a_spin2<T, 2, 2>), grid, blk, 0, st, b);
            else hipLaunchKernelGGL((k_m2a_spin2<T, 2, 0>), grid, blk, 0, st, b);
        } else if (narrow(a)) {
            if (a.eb == 1) hipLaunchKernelGGL((k_m2a_spin2<T, 1, 1, true>), grid, blk, 0, st, b);
            else if (a.eb == 2) hipLaunchKernelGGL((k_m2a_spin2<T, 1, 2, true>), grid, blk, 0, st, b);
            else hipLaunchKernelGGL((k_m2a_spin2<T, 1, 0, true>), grid, blk, 0, st, b);
        } else {
            if (a.eb == 1) hipLaunchKernelGGL((k_m2a_spin2<T, 1, 1>), grid, blk, 0, st, b);
            else if (a.eb == 2) hipLaunchKernelGGL((k_m2a_spin2<T, 1, 2>), grid, blk, 0, st, b);
            else hipLaunchKernelGGL((k_m2a_spin2<T, 1, 0>), grid, blk, 0, st, b);
        }
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
        const dim3 grid(nm_rows(a) * b.ctiles * ((a.rn + A0_TR - 1) / A0_TR) * kparts(a));
        if constexpr (!F64) {
            if (nu == 4) {
                hipLaunchKernelGGL((k_a2m_spin0<T, 4>), grid, blk, 0, st, b);
                return hipGetLastError();
            }
        }
        if (narrow(a)) hipLaunchKernelGGL((k_a2m_spin0<T, 1, true>), grid, blk, 0, st, b);
        else if (nu == 1) hipLaunchKernelGGL((k_a2m_spin0<T, 1>), grid, blk, 0, st, b);
        else hipLaunchKernelGGL((k_a2m_spin0<T, 2>), grid, blk, 0, st, b);
    } else {
        const int nu = pick_nu(2, a.ldx);
        b.ctiles = (int)(a.ldx / (64 * nu));
        const dim3 grid(nm_rows(a) * b.ctiles * ((a.rn + A2_TR - 1) / A2_TR) * kparts(a));
        if (nu == 2) {
            if (a.eb == 1) hipLaunchKernelGGL((k_a2m_spin2<T, 2, 1>), grid, blk, 0, st, b);
            else if (a.eb == 2) hipLaunchKernelGGL((k_a2m_spin2<T, 2, 2>), grid, blk, 0, st, b);
            else hipLaunchKernelGGL((k_a2m_spin2<T, 2, 0>), grid, blk, 0, st, b);
        } else if (narrow(a)) {
            if (a.eb == 1) hipLaunchKernelGGL((k_a2m_spin2<T, 1, 1, true>), grid, blk, 0, st, b);
            else if (a.eb == 2) hipLaunchKernelGGL((k_a2m_spin2<T, 1, 2, true>), grid, blk, 0, st, b);
            else hipLaunchKernelGGL((k_a2m_spin2<T, 1, 0, true>), grid, blk, 0, st, b);
        } else {
            if (a.eb == 1) hipLaunchKernelGGL((k_a2m_spin2<T, 1, 1>), grid, blk, 0, st, b);
            else if (a.eb == 2) hipLaunchKernelGGL((k_a2m_spin2<T, 1, 2>), grid, blk, 0, st, b);
            else hipLaunchKernelGGL((k_a2m_spin2<T, 1, 0>), grid, blk, 0, st, b);
        }
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_leg_m2a(const LegArgs& a, int prec, hipStream_t st)
{
    if (prec == 2) return launch_leg_m2a_bf16(a, st);
    if (prec == 0) return launch_m2a_t<double>(a, st);
    return launch_m2a_t<float>(a, st);
}

hipError_t launch_leg_a2m(const LegArgs& a, int prec, hipStream_t st)
{
    if (prec == 2) return launch_leg_a2m_bf16(a, st);
    if (prec == 0) return launch_a2m_t<double>(a, st);
    return launch_a2m_t<float>(a, st);
}

}  // namespace sht
