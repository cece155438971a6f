// Legendre contraction in split-BF16 precision (HIP, gfx950).
//
// The same products as k_leg.hip (the paper's per-m GEMMs, Sec. 2.2 and the 2x2
// block of Sec. 2.3), with every operand x (rounded to FP32) held exactly as
// three bfloat16 numbers x = hi + mid + lo: hi is x with its significand cut to
// 8 bits, mid the rest rounded to bf16, lo what then remains, which has at most
// 8 significant bits and so is a bf16 itself (|mid| < 2^-7 |x|, |lo| <= 2^-16 |x|).
// Cutting hi costs one AND where rounding costs a conversion and a shift, and
// the rounded mid keeps the dropped terms below free of sign bias.  Every
// product is formed on the BF16 matrix cores with FP32 accumulation from six
// partial products: hi*hi + hi*mid + mid*hi + hi*lo + mid*mid + lo*hi.  The three
// dropped terms (mid*lo, lo*mid, lo*lo) are below 2^-22 of the product, so the
// result has the accuracy of an FP32 contraction.  (Two pieces and three
// products leave about 4e-6 relative RMS error per product, which the B mode, a
// tenth of the E power in typical skies, amplifies past 1e-5.)  The recursion,
// its exponent handling and the data in HBM are the same as in the FP32 path
// (recursion FP64, ring coefficients FP32), so only the MFMA step changes
// precision.
//
// alm2map reads its coefficient rows already split, as 64-bit words holding hi,
// mid and lo (written so by the layout kernel), and only regroups them; map2alm
// splits the ring coefficients itself after folding the hemispheres (north +
// south and north - south in FP32), since splitting north and south apart
// would double its matrix products.
//
// One v_mfma_f32_16x16x32_bf16 covers the whole K extent of a tile (32 rings,
// or the 32 rows of one parity class of a 64-row l tile), so a tile is one burst
// of MFMAs per (class, row tile, column tile).  The bursts are spread over eight
// phases with four recursion rows of the next tile after each, as in the FP64 /
// FP32 kernels.  Operand layouts (measured): A[i][k] from lane i + 16 (k / 8),
// element k % 8 of the lane's 8-vector; B[k][j] likewise with j for i; result
// row 4 (lane / 16) + v, column lane % 16.  The recursion tiles are stored
// K-contiguous in LDS (rows of 32 values padded to 40), one plane per piece, so
// each operand vector is one 16-byte LDS read.
#include <type_traits>

#include "leg_rec.h"

namespace sht {
namespace {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned v4u __attribute__((ext_vector_type(4)));
typedef unsigned v2u __attribute__((ext_vector_type(2)));

constexpr int NT = 256;
constexpr int HALF = TL / 2;
constexpr int KP = HALF + 8;   // padded K row in LDS (bf16 elements, 80 bytes)
constexpr int NPH = 8;         // phases per tile
constexpr int RPP = SEG / NPH; // recursion rows per phase
static_assert(RPP * NPH == SEG, "the fill of one segment is spread over the phases of a tile");
constexpr int M_TR = 32;

// an operand split into three bf16 pieces
struct S3 {
    v8bf h, m, l;
};

// c + a*b over the six partial products of order >= 2^-16, small ones first
__device__ __forceinline__ v4f mfma6(const S3& a, const S3& b, v4f c)
{
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.l, b.h, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.m, b.m, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h, b.l, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.m, b.h, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h, b.m, c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h, b.h, c, 0, 0, 0);
}

// x = hi + mid + lo (see above) as FP32 bit patterns whose upper halves are the
// three bf16 numbers (the lower halves are zero)
struct P3 {
    uint32_t h, m, l;
};
__device__ __forceinline__ P3 split3(float x)
{
    const uint32_t h = __float_as_uint(x) & 0xFFFF0000u;
    const float r = x - __uint_as_float(h);
    const float m = (float)(__bf16)r;
    return P3{h, __float_as_uint(m), __float_as_uint(r - m)};
}

// the three operand vectors of eight FP32 values: upper halves paired per word
__device__ __forceinline__ void split8(const float (&x)[8], S3& s)
{
    v4u h, m, l;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const P3 a = split3(x[2 * j]), b = split3(x[2 * j + 1]);
        h[j] = __builtin_amdgcn_perm(b.h, a.h, 0x07060302u);
        m[j] = __builtin_amdgcn_perm(b.m, a.m, 0x07060302u);
        l[j] = __builtin_amdgcn_perm(b.l, a.l, 0x07060302u);
    }
    s.h = __builtin_bit_cast(v8bf, h);
    s.m = __builtin_bit_cast(v8bf, m);
    s.l = __builtin_bit_cast(v8bf, l);
}

__device__ __forceinline__ v8bf lds8(const __bf16* p) { return *reinterpret_cast<const v8bf*>(p); }

// the three planes of a split tile, PL elements apart
template <int PL>
__device__ __forceinline__ S3 lds3(const __bf16* p)
{
    return S3{lds8(p), lds8(p + PL), lds8(p + 2 * PL)};
}

// Row loads through a buffer descriptor: one per-lane offset for the first row
// and a wave-uniform scalar offset per further row, so a chunk's eight rows cost
// no vector address arithmetic.  Used only where every row lies inside the block
// (the scalar offset is outside the hardware range check); the last, overhanging
// chunk takes the clamped per-row addresses instead.
struct Rows {
    __amdgpu_buffer_rsrc_t r;
    bool ok;  // the block fits 31-bit byte offsets
    __device__ __forceinline__ Rows(const void* base, int64_t bytes)
        : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0,
                                              (int)(bytes < 0x7fffffff ? bytes : 0x7fffffff), 0x00020000)),
          ok(bytes < 0x7fffffff)
    {
    }
    __device__ __forceinline__ uint32_t ld(int voff, int soff) const
    {
        return __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
    }
    __device__ __forceinline__ uint64_t ld64(int voff, int soff) const
    {
        const v2u v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
        return ((uint64_t)v.y << 32) | v.x;
    }
};

// hi, mid and lo operand vectors of eight split-BF16 words (hi in bits 0-15,
// mid in 16-31, lo in 32-47): halves regrouped per output word
__device__ __forceinline__ void unpack8(const uint64_t (&d)[8], S3& s)
{
    v4u h, m, l;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t a0 = (uint32_t)d[2 * j], a1 = (uint32_t)d[2 * j + 1];
        const uint32_t b0 = (uint32_t)(d[2 * j] >> 32), b1 = (uint32_t)(d[2 * j + 1] >> 32);
        h[j] = __builtin_amdgcn_perm(a1, a0, 0x05040100u);
        m[j] = __builtin_amdgcn_perm(a1, a0, 0x07060302u);
        l[j] = __builtin_amdgcn_perm(b1, b0, 0x05040100u);
    }
    s.h = __builtin_bit_cast(v8bf, h);
    s.m = __builtin_bit_cast(v8bf, m);
    s.l = __builtin_bit_cast(v8bf, l);
}

// Emitter for the split tiles: hi at d, mid and lo LOFF and 2 LOFF further on,
// F- FOFF after F+.
template <int STEP, int FOFF, int LOFF>
struct EmitBF {
    __bf16* e0;
    __bf16* e1;
    __device__ __forceinline__ static __bf16 upper(uint32_t w) { return __builtin_bit_cast(__bf16, (uint16_t)(w >> 16)); }
    __device__ __forceinline__ static void put1(__bf16* d, double v)
    {
        const P3 p = split3((float)v);
        d[0] = upper(p.h);
        d[LOFF] = upper(p.m);
        d[2 * LOFF] = upper(p.l);
    }
    template <int R>
    __device__ __forceinline__ void put(double v)
    {
        put1((R & 1 ? e1 : e0) + (R >> 1) * STEP, v);
    }
    template <int R>
    __device__ __forceinline__ void put(double p, double q)
    {
        __bf16* d = (R & 1 ? e1 : e0) + (R >> 1) * STEP;
        put1(d, p);
        put1(d + FOFF, q);
    }
};

// Emitter for the alm2map tiles, whose class rows are K-contiguous in LDS
// (STEP 1): a lane's four rows of one parity class in a segment (rows R = c,
// c + 2, c + 4, c + 6) are four adjacent bf16 of a plane, so they are held in
// registers and leave as one 8-byte store per plane (and F+-) once the fourth
// arrives.  Single 2-byte stores from 32 lanes whose rows lie 80 bytes apart
// fall on a quarter of the banks; the gathered stores issue a quarter as often.
template <int FOFF, int LOFF>
struct EmitBF4 {
    static_assert(SEG == 8, "four rows per parity class and segment");
    __bf16* e0;
    __bf16* e1;
    float v[2][4][2];  // [parity class][row within the class][F+, F-]
    __device__ __forceinline__ static uint32_t pair(uint32_t lo, uint32_t hi)
    {
        return __builtin_amdgcn_perm(hi, lo, 0x07060302u);  // upper halves: lo in bits 0-15
    }
    __device__ __forceinline__ static void store4(__bf16* d, const float (&x)[4])
    {
        const P3 a = split3(x[0]), b = split3(x[1]), c = split3(x[2]), e = split3(x[3]);
        *reinterpret_cast<v2u*>(d) = v2u{pair(a.h, b.h), pair(c.h, e.h)};
        *reinterpret_cast<v2u*>(d + LOFF) = v2u{pair(a.m, b.m), pair(c.m, e.m)};
        *reinterpret_cast<v2u*>(d + 2 * LOFF) = v2u{pair(a.l, b.l), pair(c.l, e.l)};
    }
    template <int C, int NF>
    __device__ __forceinline__ void flush()
    {
        __bf16* d = C ? e1 : e0;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const float x[4] = {v[C][0][f], v[C][1][f], v[C][2][f], v[C][3][f]};
            store4(d + f * FOFF, x);
        }
    }
    template <int R>
    __device__ __forceinline__ void put(double x)
    {
        v[R & 1][R >> 1][0] = (float)x;
        if constexpr ((R >> 1) == 3) flush<R & 1, 1>();
    }
    template <int R>
    __device__ __forceinline__ void put(double p, double q)
    {
        v[R & 1][R >> 1][0] = (float)p;
        v[R & 1][R >> 1][1] = (float)q;
        if constexpr ((R >> 1) == 3) flush<R & 1, 2>();
    }
};

__device__ __forceinline__ const float* fptr(const void* base, int64_t comp, int64_t stride)
{
    return static_cast<const float*>(base) + comp * stride;
}

// ============================================================================
// map2alm, spin 0.  Tile 64 l x 64*NU columns, rings in chunks of 32.
// LDS: [buffer][hi, lo][parity class][class row][ring (K)].
// ============================================================================
template <int NU, bool NW = false>
__global__ __launch_bounds__(NT, 2) void k_m2a_spin0_bf(LegArgs a)
{
    constexpr int CLS = HALF * KP, PL = 2 * CLS, BUF = 3 * PL;
    __shared__ __attribute__((aligned(16))) __bf16 lam[2 * BUF];

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
    const int k0 = 8 * (lane >> 4);
    // fill items: 32 rings x SPT segments, one per lane (segment uniform per half-wave)
    static_assert(32 * SPT == NT, "one fill item per thread");
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

    v4f acc[2][2][NU];  // [class][row tile][column tile]
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int u = 0; u < NU; ++u) acc[p][t][u] = v4f{0, 0, 0, 0};

    int nchunk = (a.rn + M_TR - 1) / M_TR;
    int rc0 = first_chunk(a, m, nchunk, lend);
    split_range(a, sk, rc0, nchunk);
    if (rc0 < nchunk) {
        // Ring chunks run from the equator toward the pole (chunk q of the loop is
        // rsum - q): every l tile of an m needs the equator chunks, so the
        // workgroups of one m, launched together, stream the same ring rows in
        // step and share them in L2 instead of each reading its own from HBM.
        const int rsum = rc0 + nchunk - 1;
        const float* Xm = fptr(a.X, 0, a.xcomp) + (int64_t)m * a.nring * a.ldx + col;
        auto seed_of = [&](Seed<0>& s, int rc) {
            rc = rsum - rc;
            const int r = min(rc * M_TR + frl, a.rn - 1);
            seed_load(s, a, sbase + r, r);
        };
        auto emit_to = [&](int b) {
            EmitBF<KP, 0, PL> e;
            e.e0 = lam + b * BUF + (SEG / 2) * fs * KP + frl;
            e.e1 = e.e0 + CLS;
            return e;
        };
        float xr[2][NU][8];  // [north, south][column tile][ring k0 + e] of the next chunk
        const Rows xb(static_cast<const float*>(a.X) + (int64_t)m * a.nring * a.ldx, (int64_t)a.nring * a.ldx * 4);
        const int rstep = (int)a.ldx * 4;
        auto load_x = [&](int rc) {
            rc = rsum - rc;
            if (xb.ok && (rc + 1) * M_TR <= a.rn) {  // whole chunk inside the hemisphere
                const int vn = ((rc * M_TR + k0) * (int)a.ldx + col) * 4;
                const int vs = ((a.nring - 1 - (rc * M_TR + k0 + 7)) * (int)a.ldx + col) * 4;
#pragma unroll
                for (int e = 0; e < 8; ++e)
#pragma unroll
                    for (int u = 0; u < NU; ++u) {
                        xr[0][u][e] = __builtin_bit_cast(float, xb.ld(vn + 64 * u, e * rstep));
                        xr[1][u][e] = __builtin_bit_cast(float, xb.ld(vs + 64 * u, (7 - e) * rstep));
                    }
                return;
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int r = min(rc * M_TR + k0 + e, a.rn - 1);
                const float* pn = Xm + (int64_t)r * a.ldx;
                const float* ps = Xm + (int64_t)(a.nring - 1 - r) * a.ldx;
#pragma unroll
                for (int u = 0; u < NU; ++u) {
                    xr[0][u][e] = pn[16 * u];
                    xr[1][u][e] = ps[16 * u];
                }
            }
        };

        Seed<0> sd;
        Rec<0> f;
        seed_of(sd, rc0);
        if (filler) {
            f.start(sd, m2a_weight(a, (rsum - rc0) * M_TR + frl));
            auto em = emit_to(0);
            rec_all(f, cp, cnt, em);
        }
        seed_of(sd, min(rc0 + 1, nchunk - 1));
        load_x(rc0);
        __syncthreads();
        for (int rc = rc0; rc < nchunk; ++rc) {
            const int b = (rc - rc0) & 1;
            const int rcn = min(rc + 1, nchunk - 1);
            if (filler) f.start(sd, m2a_weight(a, (rsum - rcn) * M_TR + frl));
            // operands of this chunk: north + south and north - south, split
            S3 bs[2][NU];
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                float s8[8], d8[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    s8[e] = xr[0][u][e] + xr[1][u][e];
                    d8[e] = xr[0][u][e] - xr[1][u][e];
                }
                if (!NW || wave < 2) split8(s8, bs[0][u]);   // narrow: only the waves of the class
                if (!NW || wave >= 2) split8(d8, bs[1][u]);
            }
            load_x(rcn);
            seed_of(sd, min(rc + 2, nchunk - 1));
            __builtin_amdgcn_sched_barrier(0);
            auto em = emit_to(b ^ 1);
            const __bf16* lb_ = lam + b * BUF;
            static_for<0, NPH>([&](auto ph) {
                constexpr int P = decltype(ph)::v;
                if constexpr ((P & 1) == 0) {
                    constexpr int cls = (P >> 2) & 1, t = (P >> 1) & 1;
                    if (mine(cls, t)) {
                        const __bf16* q = lb_ + cls * CLS + (16 * t + (lane & 15)) * KP + k0;
                        const S3 a3 = lds3<PL>(q);
#pragma unroll
                        for (int u = 0; u < NU; ++u) acc[cls][t][u] = mfma6(a3, bs[cls][u], acc[cls][t][u]);
                    }
                }
                if (filler) rec_group<P, RPP>(f, cp, cnt, em);
            });
            __syncthreads();
        }
    }

    float* A = static_cast<float*>(a.A) + row0 * a.ldx;
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                if (!mine(p, t)) continue;
                const int ci = 16 * t + 4 * (lane >> 4) + v;
                const int l = l0 + 2 * ci + p;
                if (l > L) continue;
#pragma unroll
                for (int u = 0; u < NU; ++u) put_out(&A[(int64_t)(l - lb) * a.ldx + col + 16 * u], (float)acc[p][t][u][v], a.ksplit > 1);
            }
}

// ============================================================================
// map2alm, spin 2 (see k_m2a_spin2 in k_leg.hip for the block form and EB).
// LDS: [buffer][hi, lo][F+, F-][parity class][class row][ring (K)].
// ============================================================================
template <int NU, int EB, bool NW = false>
__global__ __launch_bounds__(NT, 2) void k_m2a_spin2_bf(LegArgs a)
{
    constexpr int CLS = HALF * KP, FOFF = 2 * CLS, PL = 2 * FOFF, BUF = 3 * PL;
    __shared__ __attribute__((aligned(16))) __bf16 fpm[2 * BUF];

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
    const int pcol = col ^ 1;
    const unsigned ysg = (col & 1) ? 0u : 0x80000000u;
    const int k0 = 8 * (lane >> 4);
    // fill items: 32 rings x SPT segments, one per lane (segment uniform per half-wave)
    static_assert(32 * SPT == NT, "one fill item per thread");
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

    v4f accE[2][2][NU], accB[2][2][NU];  // [class][row tile][column tile]
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int u = 0; u < NU; ++u) accE[p][t][u] = accB[p][t][u] = v4f{0, 0, 0, 0};

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
        const float* XQ = fptr(a.X, 1, a.xcomp) + xm + col;
        const float* XU = fptr(a.X, 2, a.xcomp) + xm + pcol;
        auto seed_of = [&](Seed<2>& s, int rc) {
            rc = rsum - rc;
            const int r = min(rc * M_TR + frl, a.rn - 1);
            seed_load(s, a, sbase + r, r);
        };
        auto emit_to = [&](int b) {
            EmitBF<KP, FOFF, PL> e;
            e.e0 = fpm + b * BUF + po * CLS + (SEG / 2) * fs * KP + frl;
            e.e1 = fpm + b * BUF + (po ^ 1) * CLS + (SEG / 2) * fs * KP + frl;
            return e;
        };
        float xr[4][NU][8];  // [Q_N, Q_S, U_N, U_S][column tile][ring k0 + e]
        const int64_t xblk = (int64_t)a.nring * a.ldx;
        const Rows qb(static_cast<const float*>(a.X) + a.xcomp + xm, xblk * 4);
        const Rows ub(static_cast<const float*>(a.X) + 2 * a.xcomp + xm, xblk * 4);
        const int rstep = (int)a.ldx * 4;
        auto load_x = [&](int rc) {
            rc = rsum - rc;
            if (qb.ok && (rc + 1) * M_TR <= a.rn) {  // whole chunk inside the hemisphere
                const int rn0 = (rc * M_TR + k0) * (int)a.ldx * 4;
                const int rs0 = (a.nring - 1 - (rc * M_TR + k0 + 7)) * (int)a.ldx * 4;
#pragma unroll
                for (int e = 0; e < 8; ++e)
#pragma unroll
                    for (int u = 0; u < NU; ++u) {
                        xr[0][u][e] = __builtin_bit_cast(float, qb.ld(rn0 + (col + 16 * u) * 4, e * rstep));
                        xr[1][u][e] = __builtin_bit_cast(float, qb.ld(rs0 + (col + 16 * u) * 4, (7 - e) * rstep));
                        xr[2][u][e] = __builtin_bit_cast(float, ub.ld(rn0 + (pcol + 16 * u) * 4, e * rstep));
                        xr[3][u][e] = __builtin_bit_cast(float, ub.ld(rs0 + (pcol + 16 * u) * 4, (7 - e) * rstep));
                    }
                return;
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int r = min(rc * M_TR + k0 + e, a.rn - 1);
                const int64_t on = (int64_t)r * a.ldx, os = (int64_t)(a.nring - 1 - r) * a.ldx;
#pragma unroll
                for (int u = 0; u < NU; ++u) {
                    xr[0][u][e] = XQ[on + 16 * u];
                    xr[1][u][e] = XQ[os + 16 * u];
                    xr[2][u][e] = XU[on + 16 * u];
                    xr[3][u][e] = XU[os + 16 * u];
                }
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
        load_x(rc0);
        __syncthreads();
        for (int rc = rc0; rc < nchunk; ++rc) {
            const int b = (rc - rc0) & 1;
            const int rcn = min(rc + 1, nchunk - 1);
            if (filler) f.start(sd, m2a_weight(a, (rsum - rcn) * M_TR + frl));
            // SX, DX, SY, DY split
            S3 bs[4][NU];
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                float o[4][8];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    o[0][e] = xr[0][u][e] + xr[1][u][e];
                    o[1][e] = xr[0][u][e] - xr[1][u][e];
                    o[2][e] = flip(xr[2][u][e] + xr[3][u][e], ysg);
                    o[3][e] = flip(xr[2][u][e] - xr[3][u][e], ysg);
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) split8(o[i], bs[i][u]);
            }
            load_x(rcn);
            seed_of(sd, min(rc + 2, nchunk - 1));
            __builtin_amdgcn_sched_barrier(0);
            auto em = emit_to(b ^ 1);
            const __bf16* fb = fpm + b * BUF;
            static_for<0, NPH>([&](auto ph) {
                constexpr int P = decltype(ph)::v;
                if constexpr ((P & 1) == 0) {
                    constexpr int cls = (P >> 2) & 1, t = (P >> 1) & 1;
                    if (mine(cls, t)) {
                        const __bf16* q = fb + cls * CLS + (16 * t + (lane & 15)) * KP + k0;
                        const S3 fp = lds3<PL>(q), fm = lds3<PL>(q + FOFF);  // F+, F-
                        // even class: E = F+ SX + F- DY, B' = F+ SY + F- DX; odd: S <-> D
                        constexpr int X1 = cls ? 1 : 0, Y1 = cls ? 3 : 2, X2 = cls ? 0 : 1, Y2 = cls ? 2 : 3;
#pragma unroll
                        for (int u = 0; u < NU; ++u) {
                            if constexpr (EB != 2) {
                                accE[cls][t][u] = mfma6(fp, bs[X1][u], accE[cls][t][u]);
                                accE[cls][t][u] = mfma6(fm, bs[Y2][u], accE[cls][t][u]);
                            }
                            if constexpr (EB != 1) {
                                accB[cls][t][u] = mfma6(fp, bs[Y1][u], accB[cls][t][u]);
                                accB[cls][t][u] = mfma6(fm, bs[X2][u], accB[cls][t][u]);
                            }
                        }
                    }
                }
                if (filler) rec_group<P, RPP>(f, cp, cnt, em);
            });
            __syncthreads();
        }
    }

    float* AE = static_cast<float*>(a.A) + a.acomp + row0 * a.ldx;
    float* AB = static_cast<float*>(a.A) + 2 * a.acomp + row0 * a.ldx;
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                if (!mine(p, t)) continue;
                const int ci = 16 * t + 4 * (lane >> 4) + v;
                const int l = l0 + 2 * ci + (p ^ po);
                if (l > L) continue;
#pragma unroll
                for (int u = 0; u < NU; ++u) {
                    const int64_t o = (int64_t)(l - lb) * a.ldx + col + 16 * u;
                    put_out(&AE[o], (float)accE[p][t][u][v], a.ksplit > 1);
                    put_out(&AB[o], (float)accB[p][t][u][v], a.ksplit > 1);
                }
            }
}

// ============================================================================
// alm2map, spin 0.  Tile 64 rings x 64*NU columns, l in chunks of 64.
// LDS: [buffer][hi, lo][parity class][ring][class row (K)].
// ============================================================================
constexpr int A0_TR = 64;

template <int NU, bool NW = false>
__global__ __launch_bounds__(NT, 2) void k_a2m_spin0_bf(LegArgs a)
{
    constexpr int CLS = A0_TR * KP, PL = 2 * CLS, BUF = 3 * PL;
    __shared__ __attribute__((aligned(16))) __bf16 lam[2 * BUF];
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
    const int k0 = 8 * (lane >> 4);
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

    v4f accE[4][NU], accO[4][NU];  // [ring tile][column tile]
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int u = 0; u < NU; ++u) accE[t][u] = accO[t][u] = v4f{0, 0, 0, 0};

    if (nch > 0) {
        const int64_t row0 = a.rowoff[m];
        const uint64_t* Am = static_cast<const uint64_t*>(a.A) + row0 * a.ldx + col;
        const int64_t sb = a.seedoff[m] + frc;
        const int j0 = (lfirst - lb) / SEG + fs0;
        const int jmax = (L - lb) / SEG;
        auto seed_of = [&](Seed<0>& s, int c, int i) {
            seed_load(s, a, sb + (int64_t)min(j0 + 4 * i + SPT * c, jmax) * a.rn, frc);
        };
        auto ls_of = [&](int c, int i) { return lfirst + TL * c + SEG * (fs0 + 4 * i); };
        // gathered 8-byte stores where the registers allow them (one column tile)
        using EM = typename std::conditional<NU == 1, EmitBF4<0, PL>, EmitBF<1, 0, PL>>::type;
        auto emit_to = [&](int b, int i) {
            EM e;
            e.e0 = lam + b * BUF + frl * KP + (SEG / 2) * (fs0 + 4 * i);
            e.e1 = e.e0 + CLS;
            return e;
        };
        uint64_t ar[2][NU][8];  // [even, odd class][column tile][class row k0 + e] of the next chunk
        // rows of this m through a buffer descriptor: one lane offset for the
        // chunk and a wave-uniform scalar offset per row pair, so the eight rows
        // cost no vector address arithmetic; the last chunk of an m, whose rows
        // may pass lmax, takes the clamped per-row addresses
        const Rows ab(static_cast<const uint64_t*>(a.A) + row0 * a.ldx, (int64_t)(L + 1 - lb) * a.ldx * 8);
        const int rstep = 2 * (int)a.ldx * 8;
        auto load_a = [&](int c) {
            if (ab.ok && lfirst + TL * c + TL - 1 <= L) {
                const int v0 = ((lfirst + TL * c + 2 * k0 - lb) * (int)a.ldx + col) * 8;
#pragma unroll
                for (int e = 0; e < 8; ++e)
#pragma unroll
                    for (int u = 0; u < NU; ++u) {
                        ar[0][u][e] = ab.ld64(v0 + 128 * u, e * rstep);
                        ar[1][u][e] = ab.ld64(v0 + (int)a.ldx * 8 + 128 * u, e * rstep);
                    }
                return;
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int le = lfirst + TL * c + 2 * (k0 + e);
                const uint64_t* pe = Am + (int64_t)(min(le, L) - lb) * a.ldx;
                const uint64_t* pq = Am + (int64_t)(min(le + 1, L) - lb) * a.ldx;
#pragma unroll
                for (int u = 0; u < NU; ++u) {
                    ar[0][u][e] = pe[16 * u];
                    ar[1][u][e] = pq[16 * u];
                }
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
        load_a(0);
        __syncthreads();
        for (int c = 0; c < nch; ++c) {
            const int b = c & 1;
            const int cn = min(c + 1, nch - 1);
            const double* cp0 = ctile[(c + 1) & 1] + SEG * fs0 * 2;
            const double* cp1 = cp0 + SEG * 4 * 2;
            const int cnt0 = min(SEG, L - ls_of(cn, 0) + 1), cnt1 = min(SEG, L - ls_of(cn, 1) + 1);
#pragma unroll
            for (int i = 0; i < 2; ++i) f[i].start(sd[i], w);
            S3 bs[2][NU];
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int u = 0; u < NU; ++u) unpack8(ar[p][u], bs[p][u]);
            load_a(cn);
#pragma unroll
            for (int i = 0; i < 2; ++i) seed_of(sd[i], min(c + 2, nch - 1), i);
            __builtin_amdgcn_sched_barrier(0);
            auto em0 = emit_to(b ^ 1, 0);
            auto em1 = emit_to(b ^ 1, 1);
            const __bf16* lb_ = lam + b * BUF;
            static_for<0, NPH>([&](auto ph) {
                constexpr int P = decltype(ph)::v;
                constexpr int cls = P >> 2, t = P & 3;
                if (mine(t)) {
                    const __bf16* q = lb_ + cls * CLS + (16 * t + (lane & 15)) * KP + k0;
                    const S3 a3 = lds3<PL>(q);
#pragma unroll
                    for (int u = 0; u < NU; ++u) {
                        if constexpr (cls == 0) accE[t][u] = mfma6(a3, bs[0][u], accE[t][u]);
                        else accO[t][u] = mfma6(a3, bs[1][u], accO[t][u]);
                    }
                }
                rec_group<P, RPP>(f[0], cp0, cnt0, em0);
                rec_group<P, RPP>(f[1], cp1, cnt1, em1);
            });
            CT::put(ctile[c & 1], cnext);  // tile of chunk c + 2
            cnext = CT::fetch(a, tile_row(min(c + 3, nch - 1)));
            __syncthreads();
        }
    }

    float* X = static_cast<float*>(a.X) + (int64_t)m * a.nring * a.ldx + col;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            if (!mine(t)) continue;
            const int r = r0 + 16 * t + 4 * (lane >> 4) + v;
            if (r >= a.rn) continue;
            const int rs = a.nring - 1 - r;
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const float e = accE[t][u][v], o = accO[t][u][v];
                put_out(&X[(int64_t)r * a.ldx + 16 * u], (float)(e + o), a.ksplit > 1);
                if (rs != r) put_out(&X[(int64_t)rs * a.ldx + 16 * u], (float)(e - o), a.ksplit > 1);
            }
        }
}

// ============================================================================
// alm2map, spin 2 (see k_a2m_spin2 in k_leg.hip for the block form).
// LDS: [buffer][hi, lo][F+, F-][parity class][ring][class row (K)].
// ============================================================================
constexpr int A2_TR = 32;

// EB = 1 (E only) or 2 (B only): the half-block transforms, as in k_leg.hip
template <int NU, int EB, bool NW = false>
__global__ __launch_bounds__(NT, 2) void k_a2m_spin2_bf(LegArgs a)
{
    constexpr int CLS = A2_TR * KP, FOFF = 2 * CLS, PL = 2 * FOFF, BUF = 3 * PL;
    __shared__ __attribute__((aligned(16))) __bf16 fpm[2 * BUF];
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
    const int k0 = 8 * (lane >> 4);
    // fill items: 32 rings x SPT segments, one per lane (segment uniform per half-wave)
    static_assert(32 * SPT == NT, "one fill item per thread");
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

    v4f u1[2][NU], u2[2][NU], v1[2][NU], v2[2][NU];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < NU; ++u) u1[t][u] = u2[t][u] = v1[t][u] = v2[t][u] = v4f{0, 0, 0, 0};

    if (nch > 0) {
        const int64_t row0 = a.rowoff[m];
        const uint64_t* AE = static_cast<const uint64_t*>(a.A) + a.acomp + row0 * a.ldx + col;
        const uint64_t* AB = static_cast<const uint64_t*>(a.A) + 2 * a.acomp + row0 * a.ldx + col;
        const int64_t sb = a.seedoff[m] + frc;
        const int j0 = (lfirst - lb) / SEG + fs;
        const int jmax = (L - lb) / SEG;
        auto seed_of = [&](Seed<2>& s, int c) { seed_load(s, a, sb + (int64_t)min(j0 + SPT * c, jmax) * a.rn, frc); };
        auto ls_of = [&](int c) { return lfirst + TL * c + SEG * fs; };
        auto emit_to = [&](int b) {
            EmitBF4<FOFF, PL> e;
            e.e0 = fpm + b * BUF + po * CLS + frl * KP + (SEG / 2) * fs;
            e.e1 = fpm + b * BUF + (po ^ 1) * CLS + frl * KP + (SEG / 2) * fs;
            return e;
        };
        uint64_t ar[4][NU][8];  // [E even, E odd, B' even, B' odd][column tile][class row k0 + e]
        // rows through buffer descriptors as in the spin-0 kernel (the last chunk
        // of an m takes the clamped per-row addresses)
        const int64_t mbytes = (int64_t)(L + 1 - lb) * a.ldx * 8;
        const Rows eb(static_cast<const uint64_t*>(a.A) + a.acomp + row0 * a.ldx, mbytes);
        const Rows bb(static_cast<const uint64_t*>(a.A) + 2 * a.acomp + row0 * a.ldx, mbytes);
        const int rstep = 2 * (int)a.ldx * 8;
        auto load_a_tile = [&](int c, int u) {
            if (eb.ok && lfirst + TL * c + TL - 1 <= L) {
                const int ve = ((lfirst + TL * c + 2 * k0 + po - lb) * (int)a.ldx + col + 16 * u) * 8;
                const int vo = ve + (po ? -8 : 8) * (int)a.ldx;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    if constexpr (EB != 2) {
                        ar[0][u][e] = eb.ld64(ve, e * rstep);
                        ar[1][u][e] = eb.ld64(vo, e * rstep);
                    } else {
                        ar[0][u][e] = ar[1][u][e] = 0ull;
                    }
                    if constexpr (EB != 1) {
                        ar[2][u][e] = bb.ld64(ve, e * rstep);
                        ar[3][u][e] = bb.ld64(vo, e * rstep);
                    } else {
                        ar[2][u][e] = ar[3][u][e] = 0ull;
                    }
                }
                return;
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int lc = lfirst + TL * c + 2 * (k0 + e);
                const int64_t oe = (int64_t)(min(lc + po, L) - lb) * a.ldx + 16 * u;
                const int64_t oo = (int64_t)(min(lc + (po ^ 1), L) - lb) * a.ldx + 16 * u;
                if constexpr (EB != 2) {
                    ar[0][u][e] = AE[oe];
                    ar[1][u][e] = AE[oo];
                } else {
                    ar[0][u][e] = ar[1][u][e] = 0ull;
                }
                if constexpr (EB != 1) {
                    ar[2][u][e] = AB[oe];
                    ar[3][u][e] = AB[oo];
                } else {
                    ar[2][u][e] = ar[3][u][e] = 0ull;
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
#pragma unroll
        for (int u = 0; u < NU; ++u) load_a_tile(0, u);
        __syncthreads();
        for (int c = 0; c < nch; ++c) {
            const int b = c & 1;
            const int cn = min(c + 1, nch - 1);
            const double* cp = ctile[(c + 1) & 1] + SEG * fs * 4;
            const int cnt = min(SEG, L - ls_of(cn) + 1);
            if (filler) f.start(sd, w);
            // Phases run column tile by column tile (u = P / (NPH / NU)): a tile's
            // operands are regrouped when its first phase starts and its loads for the
            // next chunk issued right after, so only one tile's split operands and
            // one tile's raw prefetch are live besides the accumulators.
            static_assert(NPH % NU == 0 && NPH / NU >= 4, "four MFMA phases per column tile");
            constexpr int PPU = NPH / NU;  // phases per column tile
            S3 bs[4];
            auto em = emit_to(b ^ 1);
            const __bf16* fb = fpm + b * BUF;
            static_for<0, NPH>([&](auto ph) {
                constexpr int P = decltype(ph)::v;
                constexpr int u = P / PPU, pu = P % PPU;
                if constexpr (pu == 0) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) unpack8(ar[i][u], bs[i]);
                    load_a_tile(cn, u);
                    if constexpr (u == 0) seed_of(sd, min(c + 2, nch - 1));
                    __builtin_amdgcn_sched_barrier(0);
                }
                if constexpr (pu < 4) {
                    constexpr int t = pu & 1, second = pu >> 1;
                    const __bf16* q = fb + (16 * t + (lane & 15)) * KP + k0;
                    if (mineq(t) || mineu(t)) {
                    if constexpr (!second) {
                        // F+ terms: U1 += F+e E_e, U2 += F+o E_o, V1 += F+e B'_e, V2 += F+o B'_o
                        const S3 fe = lds3<PL>(q), fo = lds3<PL>(q + CLS);
                        if constexpr (EB != 2) {
                            if (mineq(t)) u1[t][u] = mfma6(fe, bs[0], u1[t][u]);
                            if (mineq(t)) u2[t][u] = mfma6(fo, bs[1], u2[t][u]);
                        }
                        if constexpr (EB != 1) {
                            if (mineu(t)) v1[t][u] = mfma6(fe, bs[2], v1[t][u]);
                            if (mineu(t)) v2[t][u] = mfma6(fo, bs[3], v2[t][u]);
                        }
                    } else {
                        // F- terms: U1 += F-o B'_o, U2 += F-e B'_e, V1 += F-o E_o, V2 += F-e E_e
                        const S3 fe = lds3<PL>(q + FOFF), fo = lds3<PL>(q + FOFF + CLS);
                        if constexpr (EB != 1) {
                            if (mineq(t)) u1[t][u] = mfma6(fo, bs[3], u1[t][u]);
                            if (mineq(t)) u2[t][u] = mfma6(fe, bs[2], u2[t][u]);
                        }
                        if constexpr (EB != 2) {
                            if (mineu(t)) v1[t][u] = mfma6(fo, bs[1], v1[t][u]);
                            if (mineu(t)) v2[t][u] = mfma6(fe, bs[0], v2[t][u]);
                        }
                    }
                    }
                }
                if (filler) rec_group<P, RPP>(f, cp, cnt, em);
            });
            CT::put(ctile[c & 1], cnext);  // tile of chunk c + 2
            cnext = CT::fetch(a, tile_row(min(c + 3, nch - 1)));
            __syncthreads();
        }
    }

    const int64_t xm = (int64_t)m * a.nring * a.ldx;
    float* XQ = static_cast<float*>(a.X) + a.xcomp + xm + col;
    float* XU = static_cast<float*>(a.X) + 2 * a.xcomp + xm + (col ^ 1);
    const unsigned usg = (col & 1) ? 0u : 0x80000000u;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = r0 + 16 * t + 4 * (lane >> 4) + v;
            if (r >= a.rn) continue;
            const int rs = a.nring - 1 - r;
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const float U1 = u1[t][u][v], U2 = u2[t][u][v];
                const float V1 = v1[t][u][v], V2 = v2[t][u][v];
                if (mineq(t)) {
                    put_out(&XQ[(int64_t)r * a.ldx + 16 * u], (float)(U1 + U2), a.ksplit > 1);
                    if (rs != r) put_out(&XQ[(int64_t)rs * a.ldx + 16 * u], (float)(U1 - U2), a.ksplit > 1);
                }
                if (mineu(t)) {
                    put_out(&XU[(int64_t)r * a.ldx + 16 * u], (float)flip(V1 + V2, usg), a.ksplit > 1);
                    if (rs != r) put_out(&XU[(int64_t)rs * a.ldx + 16 * u], (float)flip(V1 - V2, usg), a.ksplit > 1);
                }
            }
        }
}

}  // namespace

hipError_t launch_leg_m2a_bf16(const LegArgs& a, hipStream_t st)
{
    LegArgs b = a;
    const dim3 blk(NT);
    if (a.spin == 0) {
        if (narrow(a)) {
            b.ctiles = 1;
            hipLaunchKernelGGL((k_m2a_spin0_bf<1, true>), dim3(b.ntiles * kparts(a)), blk, 0, st, b);
        } else if (a.ldx % 128 == 0) {
            b.ctiles = (int)(a.ldx / 128);
            hipLaunchKernelGGL((k_m2a_spin0_bf<2>), dim3(b.ntiles * b.ctiles * kparts(a)), blk, 0, st, b);
        } else {
            b.ctiles = (int)(a.ldx / 64);
            hipLaunchKernelGGL((k_m2a_spin0_bf<1>), dim3(b.ntiles * b.ctiles * kparts(a)), blk, 0, st, b);
        }
    } else {
        // one column tile per workgroup: with three pieces per operand, the
        // split operands of two tiles need more than the 256 registers a wave
        // may hold at two waves per SIMD
        b.ctiles = (int)(a.ldx / 64);
        const dim3 grid(b.ntiles * b.ctiles * kparts(a));
        if (narrow(a)) {
            if (a.eb == 1) hipLaunchKernelGGL((k_m2a_spin2_bf<1, 1, true>), grid, blk, 0, st, b);
            else if (a.eb == 2) hipLaunchKernelGGL((k_m2a_spin2_bf<1, 2, true>), grid, blk, 0, st, b);
            else hipLaunchKernelGGL((k_m2a_spin2_bf<1, 0, true>), grid, blk, 0, st, b);
        } else if (a.eb == 1) hipLaunchKernelGGL((k_m2a_spin2_bf<1, 1>), grid, blk, 0, st, b);
        else if (a.eb == 2) hipLaunchKernelGGL((k_m2a_spin2_bf<1, 2>), grid, blk, 0, st, b);
        else hipLaunchKernelGGL((k_m2a_spin2_bf<1, 0>), grid, blk, 0, st, b);
    }
    return hipGetLastError();
}

hipError_t launch_leg_a2m_bf16(const LegArgs& a, hipStream_t st)
{
    LegArgs b = a;
    const dim3 blk(NT);
    if (a.spin == 0) {
        const int nu = a.ldx % 128 == 0 ? 2 : 1;
        b.ctiles = (int)(a.ldx / (64 * nu));
        const dim3 grid(nm_rows(a) * b.ctiles * ((a.rn + A0_TR - 1) / A0_TR) * kparts(a));
        if (narrow(a)) hipLaunchKernelGGL((k_a2m_spin0_bf<1, true>), grid, blk, 0, st, b);
        else if (nu == 2) hipLaunchKernelGGL((k_a2m_spin0_bf<2>), grid, blk, 0, st, b);
        else hipLaunchKernelGGL((k_a2m_spin0_bf<1>), grid, blk, 0, st, b);
    } else {
        b.ctiles = (int)(a.ldx / 64);
        const dim3 grid(nm_rows(a) * b.ctiles * ((a.rn + A2_TR - 1) / A2_TR) * kparts(a));
        if (narrow(a)) {
            if (a.eb == 1) hipLaunchKernelGGL((k_a2m_spin2_bf<1, 1, true>), grid, blk, 0, st, b);
            else if (a.eb == 2) hipLaunchKernelGGL((k_a2m_spin2_bf<1, 2, true>), grid, blk, 0, st, b);
            else hipLaunchKernelGGL((k_a2m_spin2_bf<1, 0, true>), grid, blk, 0, st, b);
        } else if (a.eb == 1) hipLaunchKernelGGL((k_a2m_spin2_bf<1, 1>), grid, blk, 0, st, b);
        else if (a.eb == 2) hipLaunchKernelGGL((k_a2m_spin2_bf<1, 2>), grid, blk, 0, st, b);
        else hipLaunchKernelGGL((k_a2m_spin2_bf<1, 0>), grid, blk, 0, st, b);
    }
    return hipGetLastError();
}

}  // namespace sht
