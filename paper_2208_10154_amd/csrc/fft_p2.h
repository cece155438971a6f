// Ring FFT machinery shared by the power-of-two and Bluestein kernels
// (k_fft_p2.hip) and the four-step kernels (k_fft_four.hip): compile-time
// radix-8 Stockham passes, the work-item decode, the Bluestein convolution step
// and the fold / unfold between ring spectra and the m-major coefficient rows.
// Each translation unit gets its own copy (internal linkage).
#pragma once
#include "fft_internal.h"

namespace sht {
namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

// forward DFTs (e^{-2 pi i jk/R}) of R values in registers, natural order out
__device__ __forceinline__ void dft2(double2* v)
{
    const double2 t = v[0];
    v[0] = cadd(t, v[1]);
    v[1] = csub(t, v[1]);
}
__device__ __forceinline__ void dft4(double2* v)
{
    const double2 a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
    const double2 a2 = cadd(v[1], v[3]), a3 = csub(v[1], v[3]);
    v[0] = cadd(a0, a2);
    v[2] = csub(a0, a2);
    v[1] = make_double2(a1.x + a3.y, a1.y - a3.x);  // a1 - i a3
    v[3] = make_double2(a1.x - a3.y, a1.y + a3.x);  // a1 + i a3
}
// radix 8 by decimation in frequency: X_{2q} = DFT4(x_n + x_{n+4}),
// X_{2q+1} = DFT4((x_n - x_{n+4}) W^n), W = e^{-2 pi i/8}
__device__ __forceinline__ void dft8(double2* v)
{
    constexpr double H = 0.7071067811865476;  // 1/sqrt(2), correctly rounded
    double2 a[4], b[4];
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        a[n] = cadd(v[n], v[n + 4]);
        b[n] = csub(v[n], v[n + 4]);
    }
    b[1] = make_double2(H * (b[1].x + b[1].y), H * (b[1].y - b[1].x));    // * (1 - i)/sqrt(2)
    b[2] = make_double2(b[2].y, -b[2].x);                                  // * -i
    b[3] = make_double2(H * (b[3].y - b[3].x), -H * (b[3].x + b[3].y));   // * (-1 - i)/sqrt(2)
    dft4(a);
    dft4(b);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        v[2 * q] = a[q];
        v[2 * q + 1] = b[q];
    }
}
template <int R>
__device__ __forceinline__ void dftr(double2* v)
{
    if constexpr (R == 2) dft2(v);
    else if constexpr (R == 4) dft4(v);
    else dft8(v);
}

template <int LOGN>
struct P2 {
    static constexpr int N = 1 << LOGN;
    static constexpr int E = 8;                      // values per thread
    static constexpr int T = N / E;                  // threads per sequence
    // sequences (map pairs) per workgroup: 4096 values (two rings of 2048) per
    // workgroup, at most 16 pairs (the map pairs of the narrowest chunk, 32 map
    // sets).  Two or more pairs give every coefficient row access 64 contiguous
    // bytes or more (a single pair's 32 bytes per row leave every access its own
    // partial line and page translation).
    static constexpr int S = (4096 / N) < 1 ? 1 : ((4096 / N) > 16 ? 16 : 4096 / N);
    static constexpr int LOGS = S == 1 ? 0 : (S == 2 ? 1 : (S == 4 ? 2 : (S == 8 ? 3 : 4)));
    static constexpr int NTH = S * T;                // threads per workgroup
    static constexpr int NP = (LOGN + 2) / 3;        // passes
    static constexpr int LOGRL = LOGN - 3 * (NP - 1);  // log2 of the last radix (1..3)
    static constexpr int SEQ = N + N / 8;            // LDS slots per sequence
    static constexpr int LDS_BYTES = S * SEQ * 16;
};

// LDS position of element pos at the boundary after pass P (radix 8, stride
// 8^P between the values of one butterfly).  After the first pass a thread's
// outputs are 8 consecutive slots, after the second 8 runs of 8 lanes, 64
// slots apart: one pad slot per 8 (resp. 8 per 64) spreads those over the
// banks.  Later boundaries are written in runs of >= 64 lanes and need none.
template <int P>
__device__ __forceinline__ int padp(int pos)
{
    if constexpr (P == 0) return pos + (pos >> 3);
    else if constexpr (P == 1) return pos + ((pos >> 6) << 3);
    else return pos;
}

template <int LOGN, int PASS>
struct Pass {
    using C = P2<LOGN>;
    static constexpr bool LAST = (PASS == C::NP - 1);
    static constexpr int LOGR = LAST ? C::LOGRL : 3;
    static constexpr int R = 1 << LOGR;
    static constexpr int B = 8 / R;                  // butterflies per thread
    static constexpr int LOGNS = 3 * PASS;
    static constexpr int NS = 1 << LOGNS;            // product of the earlier radices
    static constexpr int TWS = 2 * (C::N >> (LOGNS + LOGR));  // twiddle index step in e^{-i pi t/N}
};

// twiddles of pass PASS (>= 1): w^{r k}, w = e^{-2 pi i/(NS R)}, k = j mod NS.
// One table load per butterfly (w^k); the other powers are products.  The
// gathers, not the arithmetic, were the latency of a pass: one load instead of
// seven cut the ring FFT time by a fifth to a quarter, and the products add a few
// ulp to twiddles used once.
template <int LOGN, int PASS>
__device__ __forceinline__ void load_twiddles(double2 (&w)[8], int tl, const double2* tw)
{
    using Q = Pass<LOGN, PASS>;
#pragma unroll
    for (int b = 0; b < Q::B; ++b) {
        const int k = (tl + P2<LOGN>::T * b) & (Q::NS - 1);
#pragma unroll
        for (int r = 1; r < Q::R; ++r)
            w[b * Q::R + r] = r == 1 ? tw[Q::TWS * k] : cmul(w[b * Q::R + r - 1], w[b * Q::R + 1]);
    }
}

// Runs passes PASS..NP-1 on the values in v (inputs of pass PASS, twiddles w
// already loaded).  On return v holds the last pass's outputs: value b*R + r is
// element tl + T*b + r*N/R of the transform.
template <int LOGN, int PASS>
__device__ __forceinline__ void run_passes(double2 (&v)[8], double2 (&w)[8], double2* sb, int tl, const double2* tw)
{
    using C = P2<LOGN>;
    using Q = Pass<LOGN, PASS>;
    if constexpr (PASS > 0) {
#pragma unroll
        for (int b = 0; b < Q::B; ++b) {
#pragma unroll
            for (int r = 1; r < Q::R; ++r) v[b * Q::R + r] = cmul(v[b * Q::R + r], w[b * Q::R + r]);
        }
    }
#pragma unroll
    for (int b = 0; b < Q::B; ++b) dftr<Q::R>(v + b * Q::R);
    if constexpr (!Q::LAST) {
        using Q2 = Pass<LOGN, PASS + 1>;
        load_twiddles<LOGN, PASS + 1>(w, tl, tw);  // in flight across the exchange
        if constexpr (PASS > 0) __syncthreads();    // earlier readers of sb are done
        // outputs y[(j - k) R + k + r NS] (radix 8, one butterfly per thread)
        {
            const int j = tl, k = j & (Q::NS - 1);
            const int pos = (j - k) * 8 + k;
#pragma unroll
            for (int r = 0; r < 8; ++r) sb[padp<PASS>(pos + r * Q::NS)] = v[r];
        }
        __syncthreads();
#pragma unroll
        for (int b = 0; b < Q2::B; ++b) {
#pragma unroll
            for (int r = 0; r < Q2::R; ++r)
                v[b * Q2::R + r] = sb[padp<PASS>(tl + C::T * b + r * (C::N / Q2::R))];
        }
        run_passes<LOGN, PASS + 1>(v, w, sb, tl, tw);
    }
}

// Work item of this workgroup: the grid is one-dimensional over (component,
// item); workgroups are dealt to the 8 XCDs round-robin, so the block index is
// remapped to give each XCD one contiguous range (neighbouring pair groups of a
// ring, which write adjacent columns of the same m-major rows, then share an L2).
// A workgroup whose map pairs all lie past the chunk's map sets returns at once:
// their ring coefficient columns are never read into a result (every later step
// treats the columns of a map set on their own, and pairs the two map sets of one
// FFT sequence only with each other), so a small batch does not pay for the
// padding of its column tile.
struct Item {
    int ring, pair0, comp;
};
__device__ __forceinline__ Item work_item(const FftItem* items, int nitems, int comp0)
{
    const int nb = (int)gridDim.x, b = (int)blockIdx.x;
    const int q = nb >> 3, r = nb & 7, x = b & 7;
    const int idx = x * q + min(x, r) + (b >> 3);
    const int comp = idx / nitems;
    const FftItem it = items[idx - comp * nitems];
    return Item{it.ring, it.pair0, comp0 + comp};
}

// m values per thread and batch in the unfolding (loads of a batch issued first)
constexpr int MB = 8;

template <typename XT>
__device__ __forceinline__ void store4(XT* p, double2 ta, double2 tb)
{
    if constexpr (sizeof(XT) == 4) {
        *reinterpret_cast<float4*>(p) = make_float4((float)ta.x, (float)ta.y, (float)tb.x, (float)tb.y);
    } else {
        reinterpret_cast<double2*>(p)[0] = ta;
        reinterpret_cast<double2*>(p)[1] = tb;
    }
}
template <typename XT>
__device__ __forceinline__ void load4(const XT* p, double2& ta, double2& tb)
{
    if constexpr (sizeof(XT) == 4) {
        const float4 f = *reinterpret_cast<const float4*>(p);
        ta = make_double2(f.x, f.y);
        tb = make_double2(f.z, f.w);
    } else {
        ta = reinterpret_cast<const double2*>(p)[0];
        tb = reinterpret_cast<const double2*>(p)[1];
    }
}

// ----------------------------------------------------------------------------
// Rings whose length n has a prime factor above 7 (most polar-cap rings):
// Bluestein's chirp-z form, y_j = w_j sum_i (x_i w_i) conj(w_{j-i}) with
// w_i = e^{-i pi i^2/n}, the circular convolution taken through a power-of-two
// length M >= 2n - 1 with the compile-time passes above.  The kernel spectrum
// bhat (FFT of conj(w) placed circularly, times 1/M) is precomputed per length.
// The last pass of a length-M transform leaves element tl + T k in register
// slot b R + r with k = b + r B, exactly the pass-0 inputs of the next
// transform: the two transforms are chained in registers.
// ----------------------------------------------------------------------------

// m = m0, m0 + dm, ...: keeps j = m mod n and ph = (m s) mod 2n
struct MStep {
    int j, ph, dj, dph, n, two_n;
    __device__ __forceinline__ MStep(int m0, int dm, int n_, int s)
    {
        n = n_;
        two_n = 2 * n_;
        j = m0 % n;
        ph = (int)(((int64_t)m0 * s) % two_n);
        dj = dm % n;
        dph = (int)(((int64_t)dm * s) % two_n);
    }
    __device__ __forceinline__ void next()
    {
        j += dj;
        if (j >= n) j -= n;
        ph += dph;
        if (ph >= two_n) ph -= two_n;
    }
};

// the registers after a transform, reordered to the pass-0 layout
template <int LOGM>
__device__ __forceinline__ void to_pass0(const double2 (&v)[8], double2 (&u)[8])
{
    using QL = Pass<LOGM, P2<LOGM>::NP - 1>;
#pragma unroll
    for (int b = 0; b < QL::B; ++b) {
#pragma unroll
        for (int r = 0; r < QL::R; ++r) u[b + r * QL::B] = v[b * QL::R + r];
    }
}

// Convolution step of Bluestein on the pass-0 values u (x_i w_i at i = tl + k T,
// zero for i >= n): on return y_j = w_j u[k] for j = tl + k T < n.
template <int LOGM>
__device__ __forceinline__ void blue_core(double2 (&u)[8], double2* sb, int tl, const double2* twM, const double2* bhat)
{
    constexpr int T = P2<LOGM>::T;
    double2 v[8], w[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = u[k];
    run_passes<LOGM, 0>(v, w, sb, tl, twM);
    to_pass0<LOGM>(v, u);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const double2 z = cmul(u[k], bhat[tl + k * T]);
        u[k] = make_double2(z.x, -z.y);
    }
    __syncthreads();  // the first transform's last readers of sb are done
    run_passes<LOGM, 0>(u, w, sb, tl, twM);
    to_pass0<LOGM>(u, v);
#pragma unroll
    for (int k = 0; k < 8; ++k) u[k] = make_double2(v[k].x, -v[k].y);
}

// Output of one ring's forward transform, the spectrum Z of each map pair in LDS
// (natural order, n values at lds + seq * SEQ, all threads past a barrier): the
// data spectra F of the iterative map2alm (halfcomplex, when kept) and the unfold
// T_m = e^{-i m phi0} F_{m mod n} into the X rows, lanes over (m, pair, part).
template <int LOGM, typename XT>
__device__ __forceinline__ void blue_spectrum_out(const FftArgs& a, const Item it, const double2* lds,
                                                  const RingDev& rg, const double2* twn)
{
    using C = P2<LOGM>;
    constexpr int T = C::T, S = C::S;
    const int n = rg.n;
    const int seq = (int)threadIdx.x / T, tl = (int)threadIdx.x % T;
    const double2* sb = lds + seq * C::SEQ;
    const int k = 2 * (it.pair0 + seq);
    if (a.F) {  // data spectra of both maps (iterative map2alm), halfcomplex
        for (int pos = tl; pos < n; pos += T) {
            const int j = (pos == 0) ? 0 : (pos == n - 1 ? n / 2 : (pos + 1) / 2);
            const int jn = j ? n - j : 0;
            const double2 z = sb[j], y = sb[jn];
            const double2 Fa = make_double2(0.5 * (z.x + y.x), 0.5 * (z.y - y.y));
            const double2 Fb = make_double2(0.5 * (z.y + y.y), 0.5 * (y.x - z.x));
            const bool im = (pos != 0) && (pos != n - 1) && ((pos & 1) == 0);
            if (k < a.nmaps) a.F[((int64_t)k * a.ncomp + it.comp) * a.npix + rg.first + pos] = im ? Fa.y : Fa.x;
            if (k + 1 < a.nmaps)
                a.F[((int64_t)(k + 1) * a.ncomp + it.comp) * a.npix + rg.first + pos] = im ? Fb.y : Fb.x;
        }
    }

    constexpr int LP = sizeof(XT) == 8 ? 1 : 0;
    constexpr int MSTEP = C::NTH >> (LP + C::LOGS);
    const int part = (int)threadIdx.x & ((1 << LP) - 1);
    const int sq = ((int)threadIdx.x >> LP) & (S - 1);
    const int mi = (int)threadIdx.x >> (LP + C::LOGS);
    const double2* zs = lds + sq * C::SEQ;
    XT* X = static_cast<XT*>(a.X) + (int64_t)it.comp * a.xcomp + (int64_t)it.ring * a.ldx + 4 * (it.pair0 + sq) + 2 * part;
    const int64_t mrow = (int64_t)a.nring * a.ldx;
    MStep ws(mi, MSTEP, n, rg.s);
    const int mtop = min(a.lmax, rg.mcut);
    for (int m0 = mi; m0 <= mtop; m0 += MB * MSTEP) {
        double2 ph[MB];
        int jj[MB];
#pragma unroll
        for (int q = 0; q < MB; ++q) {
            ph[q] = twn[ws.ph];
            jj[q] = ws.j;
            ws.next();
        }
#pragma unroll
        for (int q = 0; q < MB; ++q) {
            const int m = m0 + q * MSTEP;
            if (m <= mtop) {
                const int j = jj[q], jn = j ? n - j : 0;
                const double2 z = zs[j], y = zs[jn];
                const double2 Fa = make_double2(0.5 * (z.x + y.x), 0.5 * (z.y - y.y));
                const double2 Fb = make_double2(0.5 * (z.y + y.y), 0.5 * (y.x - z.x));
                if constexpr (sizeof(XT) == 8) {
                    *reinterpret_cast<double2*>(X + m * mrow) = cmul(ph[q], part ? Fb : Fa);
                } else {
                    store4<XT>(X + m * mrow, cmul(ph[q], Fa), cmul(ph[q], Fb));
                }
            }
        }
    }
}

// Fold of one ring's X rows into conj(Z_j), j < n, at lds + seq * SEQ after
// clearing the first nclear LDS slots: every m up to the ring's cut lands on bin
// m mod n and its mirror, several terms per bin, so added atomically; lanes over
// (m, pair, part), the map-b lane handing its term to the map-a lane.  Ends with
// a barrier.
template <int LOGM, typename XT>
__device__ __forceinline__ void blue_fold(const FftArgs& a, const Item it, double2* lds, const RingDev& rg,
                                          const double2* twn, int nclear)
{
    using C = P2<LOGM>;
    constexpr int S = C::S;
    const int n = rg.n, lmax = min(a.lmax, rg.mcut);  // rows past the ring's cutoff are zero
    for (int e = (int)threadIdx.x; e < nclear; e += C::NTH) lds[e] = make_double2(0.0, 0.0);
    __syncthreads();
    const int part = (int)threadIdx.x & 1;
    const int sq = ((int)threadIdx.x >> 1) & (S - 1);
    const int mi = (int)threadIdx.x >> (1 + C::LOGS);
    constexpr int MSTEP = C::NTH >> (1 + C::LOGS);
    double2* zs = lds + sq * C::SEQ;
    const XT* X = static_cast<const XT*>(a.X) + (int64_t)it.comp * a.xcomp + (int64_t)it.ring * a.ldx +
                  4 * (it.pair0 + sq) + 2 * part;
    const int64_t mrow = (int64_t)a.nring * a.ldx;
    MStep ws(mi, MSTEP, n, rg.s);
    for (int m0 = mi; m0 <= lmax; m0 += MB * MSTEP) {
        double2 tv[MB], p[MB];
        int jj[MB];
#pragma unroll
        for (int q = 0; q < MB; ++q) {
            const XT* xr = X + min(m0 + q * MSTEP, lmax) * mrow;
            if constexpr (sizeof(XT) == 8) {
                tv[q] = *reinterpret_cast<const double2*>(xr);
            } else {
                const float2 f = *reinterpret_cast<const float2*>(xr);
                tv[q] = make_double2(f.x, f.y);
            }
            p[q] = twn[ws.ph];
            jj[q] = ws.j;
            ws.next();
        }
#pragma unroll
        for (int q = 0; q < MB; ++q) {
            const int m = m0 + q * MSTEP;
            const double2 c = cmul(make_double2(p[q].x, -p[q].y), tv[q]);  // c_m of this lane's map
            const double cbx = __shfl_xor(c.x, 1), cby = __shfl_xor(c.y, 1);
            if (part == 0 && m <= lmax && (!a.mown || a.mown[m])) {
                const double2 ca = c, cb = make_double2(cbx, cby);
                double* z1 = reinterpret_cast<double*>(zs + jj[q]);
                atomicAdd(z1, ca.x - cb.y);
                atomicAdd(z1 + 1, -(ca.y + cb.x));
                if (m >= 1) {
                    double* z2 = reinterpret_cast<double*>(zs + (jj[q] ? n - jj[q] : 0));
                    atomicAdd(z2, ca.x + cb.y);
                    atomicAdd(z2 + 1, -(cb.x - ca.y));
                }
            }
        }
    }
    __syncthreads();
}

}  // namespace
}  // namespace sht
