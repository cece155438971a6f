// Ring FFTs and FFT-mapping for HEALPix rings (HIP, gfx950).
//
// One workgroup transforms one iso-latitude ring of `nseq` map pairs: two real
// maps are packed as one complex sequence z = a + i b, transformed in LDS with a
// mixed-radix Stockham FFT (radices 4, 2, 3, 5, 7) or, for ring lengths with a
// larger prime factor, Bluestein's chirp-z algorithm through a 7-smooth length.
//
// The forward kernel then performs the "FFT mapping" of the paper (Sec. 2.1 eq.
// "mm" and Appendix A.1): for every m = 0..lmax it takes bin m mod N of the ring
// spectrum (the conjugate mirror bin above Nyquist is implied by the real input),
// multiplies by e^{-i m phi0} and writes the result m-major, T[m][ring][column],
// so that the Legendre contraction sees contiguous columns (Sec. 3.1 item 5).
// The inverse kernel folds the m-major coefficients back onto the ring's bins
// (every m with m = j or -m = j mod N, conjugated for negative m) and transforms
// back to pixels.  The residual kernel (iterative map2alm, Algorithm 2) performs
// the same fold, subtracts N times it from the stored data spectrum in FP64 and
// unfolds the difference, never leaving the Fourier domain (Sec. 3.1 item 8).
//
// Index arithmetic is kept off the critical path: ring lengths are runtime
// values, so divisions inside LDS index ranges use an exact multiply-high form,
// and the (un)folding walks m with incrementally updated bin and phase indices
// (one thread per map pair and m, all four output columns at once).  LDS holds
// sequence sq, element i at sq * lstride + i + i / 16: the pad slot every 16
// values and the sequence stride (congruent to 16/nseq modulo 16) spread
// power-of-two strides over the banks.
#include "fft_internal.h"

namespace sht {
namespace {

constexpr int NT = FFT_THREADS;

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 conjd(double2 a) { return make_double2(a.x, -a.y); }

// exact x / d for 0 <= x < 2^16 and 1 <= d < 2^16: with mul = ceil(2^32 / d),
// x * mul / 2^32 exceeds x / d by less than 2^-16 < 1/d, so the floor is exact
struct FastDiv {
    int d;
    unsigned mul;
    __device__ __forceinline__ explicit FastDiv(int dd) : d(dd), mul(dd > 1 ? 0xFFFFFFFFu / (unsigned)dd + 1u : 0u) {}
    __device__ __forceinline__ int div(int x) const { return d == 1 ? x : (int)__umulhi((unsigned)x, mul); }
};

// LDS slot of element i of sequence sq
__device__ __forceinline__ int P(int sq, int i, int ls) { return sq * ls + i + (i >> 4); }

// e^{-2 pi i t / R} for the odd radices: real parts c, imaginary parts s
// (correctly rounded values of the cosines and sines of 2 pi t / R)
template <int R>
struct Roots;
template <>
struct Roots<3> {
    static constexpr double c[3] = {1.0, -0.5, -0.5};
    static constexpr double s[3] = {0.0, -0.8660254037844386, 0.8660254037844386};
};
template <>
struct Roots<5> {
    static constexpr double c[5] = {1.0, 0.30901699437494745, -0.8090169943749475, -0.8090169943749475,
                                    0.30901699437494745};
    static constexpr double s[5] = {0.0, -0.9510565162951535, -0.5877852522924731, 0.5877852522924731,
                                    0.9510565162951535};
};
template <>
struct Roots<7> {
    static constexpr double c[7] = {1.0, 0.6234898018587335, -0.2225209339563144, -0.9009688679024191,
                                    -0.9009688679024191, -0.2225209339563144, 0.6234898018587335};
    static constexpr double s[7] = {0.0, -0.7818314824680298, -0.9749279121818236, -0.4338837391175581,
                                    0.4338837391175581, 0.9749279121818236, 0.7818314824680298};
};

// R-point forward DFT (odd R) in registers, using the conjugate symmetry
// W^{(R-r)q} = conj(W^{rq}) of W = e^{-2 pi i/R}: with s_r = v_r + v_{R-r},
// d_r = v_r - v_{R-r}, out_q = A + iB and out_{R-q} = A - iB where
// A = v_0 + sum_r Re(W^{rq}) s_r and B = sum_r Im(W^{rq}) d_r.
template <int R>
__device__ __forceinline__ void dft(double2* v)
{
    constexpr int H = (R - 1) / 2;
    double2 sv[H], dv[H];
    double2 o0 = v[0];
#pragma unroll
    for (int r = 1; r <= H; ++r) {
        sv[r - 1] = cadd(v[r], v[R - r]);
        dv[r - 1] = csub(v[r], v[R - r]);
        o0 = cadd(o0, sv[r - 1]);
    }
    double2 o[R];
    o[0] = o0;
#pragma unroll
    for (int q = 1; q <= H; ++q) {
        double2 A = v[0], B = make_double2(0.0, 0.0);
#pragma unroll
        for (int r = 1; r <= H; ++r) {
            const double wc = Roots<R>::c[(r * q) % R], ws = Roots<R>::s[(r * q) % R];
            A.x += wc * sv[r - 1].x; A.y += wc * sv[r - 1].y;
            B.x += ws * dv[r - 1].x; B.y += ws * dv[r - 1].y;
        }
        o[q] = make_double2(A.x - B.y, A.y + B.x);
        o[R - q] = make_double2(A.x + B.y, A.y - B.x);
    }
#pragma unroll
    for (int q = 0; q < R; ++q) v[q] = o[q];
}
template <>
__device__ __forceinline__ void dft<2>(double2* v)
{
    double2 t = v[0];
    v[0] = cadd(t, v[1]);
    v[1] = csub(t, v[1]);
}
template <>
__device__ __forceinline__ void dft<4>(double2* v)
{
    double2 a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
    double2 a2 = cadd(v[1], v[3]), a3 = csub(v[1], v[3]);
    v[0] = cadd(a0, a2);
    v[2] = csub(a0, a2);
    v[1] = make_double2(a1.x + a3.y, a1.y - a3.x);  // a1 - i a3
    v[3] = make_double2(a1.x - a3.y, a1.y + a3.x);  // a1 + i a3
}

// One radix-R Stockham step over nseq sequences of length n held in LDS, in
// place: every thread first reads all of its butterfly inputs, then (after a
// barrier) writes all outputs.  Ns = product of the radices already applied.
// One twiddle load per butterfly (w^k; the higher powers are products: the
// gathers, not the arithmetic, are the latency).  For radices 2 and 4 the
// twiddle loads are issued before the LDS reads so that
// their latency overlaps the reads and the barrier (the odd radices, rarer and
// with more registers per butterfly, load them after the barrier); butterfly
// indices past the end are clamped (reads only), so no load sits in a branch.
template <int R, int ELEMS>
__device__ __forceinline__ void stockham_step(double2* buf, int nseq, int n, int ls, int Ns, const double2* tw)
{
    constexpr int MAXB = (ELEMS + R - 1) / R;
    constexpr bool PRE = (R == 2 || R == 4);
    const int nb = n / R;
    const int tot = nseq * nb;
    const int unit = 2 * (n / (Ns * R));
    const FastDiv dnb(nb), dns(Ns);
    double2 v[MAXB][R], wt[MAXB][R - 1];
    int sqs[MAXB], js[MAXB];
#pragma unroll
    for (int q = 0; q < MAXB; ++q) {
        const int w = min((int)threadIdx.x + q * NT, tot - 1);
        const int sq = dnb.div(w), j = w - sq * nb;
        const int k = j - dns.div(j) * Ns;
        sqs[q] = sq;
        js[q] = j;
        if (PRE) {
#pragma unroll
            for (int r = 1; r < R; ++r) wt[q][r - 1] = r == 1 ? tw[k * unit] : cmul(wt[q][r - 2], wt[q][0]);
        }
    }
#pragma unroll
    for (int q = 0; q < MAXB; ++q) {
#pragma unroll
        for (int r = 0; r < R; ++r) v[q][r] = buf[P(sqs[q], js[q] + r * nb, ls)];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MAXB; ++q) {
        if ((int)threadIdx.x + q * NT < tot) {
            const int sq = sqs[q], j = js[q];
            const int k = j - dns.div(j) * Ns;
            if (!PRE) {
#pragma unroll
                for (int r = 1; r < R; ++r) wt[q][r - 1] = r == 1 ? tw[k * unit] : cmul(wt[q][r - 2], wt[q][0]);
            }
#pragma unroll
            for (int r = 1; r < R; ++r) v[q][r] = cmul(v[q][r], wt[q][r - 1]);
            dft<R>(v[q]);
            const int base = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[P(sq, base + r * Ns, ls)] = v[q][r];
        }
    }
    __syncthreads();
}

// Forward DFT (e^{-2 pi i jk/n}) of nseq sequences in LDS.
template <int ELEMS>
__device__ __forceinline__ void fft_lds(double2* buf, int nseq, int n, int ls, int nstage, const int* radix, const double2* tw)
{
    int Ns = 1;
    for (int s = 0; s < nstage; ++s) {
        int R = radix[s];
        switch (R) {
            case 4: stockham_step<4, ELEMS>(buf, nseq, n, ls, Ns, tw); break;
            case 2: stockham_step<2, ELEMS>(buf, nseq, n, ls, Ns, tw); break;
            case 3: stockham_step<3, ELEMS>(buf, nseq, n, ls, Ns, tw); break;
            case 5: stockham_step<5, ELEMS>(buf, nseq, n, ls, Ns, tw); break;
            default: stockham_step<7, ELEMS>(buf, nseq, n, ls, Ns, tw); break;
        }
        Ns *= R;
    }
}

// Ring DFT of length n of the sequences already loaded in LDS (elements i < n).
// Direct: Stockham over n.  Bluestein: y_j = w_j sum_i (x_i w_i) conj(w_{j-i}),
// w_i = e^{-i pi i^2/n}, the convolution done through length m with the
// precomputed kernel spectrum (which carries the 1/m of the inverse).
template <int ELEMS>
__device__ __forceinline__ void ring_dft(double2* buf, int nseq, const FftLen* L, const double2* tw_m, const double2* chirp,
                                         const double2* bhat)
{
    const int n = L->n, ls = L->lstride;
    if (!L->blue) {
        fft_lds<ELEMS>(buf, nseq, n, ls, L->nstage, L->radix, tw_m);
        return;
    }
    const int m = L->m;
    const FastDiv dm(m), dn(n);
    const int totm = nseq * m, totn = nseq * n;
    double2 c[ELEMS];
    // x_i w_i, zero-padded to length m
#pragma unroll
    for (int q = 0; q < ELEMS; ++q) {
        const int e = min((int)threadIdx.x + q * NT, totm - 1);
        const int sq = dm.div(e), i = e - sq * m;
        c[q] = chirp[min(i, n - 1)];
    }
#pragma unroll
    for (int q = 0; q < ELEMS; ++q) {
        const int e = (int)threadIdx.x + q * NT;
        if (e < totm) {
            const int sq = dm.div(e), i = e - sq * m;
            buf[P(sq, i, ls)] = (i < n) ? cmul(buf[P(sq, i, ls)], c[q]) : make_double2(0.0, 0.0);
        }
    }
    __syncthreads();
    fft_lds<ELEMS>(buf, nseq, m, ls, L->nstage, L->radix, tw_m);
#pragma unroll
    for (int q = 0; q < ELEMS; ++q) {
        const int e = min((int)threadIdx.x + q * NT, totm - 1);
        const int sq = dm.div(e), i = e - sq * m;
        c[q] = bhat[i];
    }
#pragma unroll
    for (int q = 0; q < ELEMS; ++q) {
        const int e = (int)threadIdx.x + q * NT;
        if (e < totm) {
            const int sq = dm.div(e), i = e - sq * m;
            buf[P(sq, i, ls)] = conjd(cmul(buf[P(sq, i, ls)], c[q]));
        }
    }
    __syncthreads();
    fft_lds<ELEMS>(buf, nseq, m, ls, L->nstage, L->radix, tw_m);
#pragma unroll
    for (int q = 0; q < ELEMS; ++q) {
        const int e = min((int)threadIdx.x + q * NT, totn - 1);
        const int sq = dn.div(e), j = e - sq * n;
        c[q] = chirp[j];
    }
#pragma unroll
    for (int q = 0; q < ELEMS; ++q) {
        const int e = (int)threadIdx.x + q * NT;
        if (e < totn) {
            const int sq = dn.div(e), j = e - sq * n;
            buf[P(sq, j, ls)] = cmul(c[q], conjd(buf[P(sq, j, ls)]));
        }
    }
    __syncthreads();
}

// Walks m = m0, m0 + dm, ... for one thread, keeping j = m mod n and
// ph = (m s) mod 2n (the phase e^{-i m phi0} = tw_n[ph]) up to date.
struct MWalk {
    int j, ph, dj, dph, n, two_n;
    __device__ __forceinline__ MWalk(int m0, int dm, int n_, int s)
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

__device__ __forceinline__ int64_t xidx(const FftArgs& a, int comp, int m, int ring, int col)
{
    return (int64_t)comp * a.xcomp + ((int64_t)m * a.nring + ring) * a.ldx + col;
}

// the four columns (re a, im a, re b, im b) of one map pair at one (m, ring)
__device__ __forceinline__ void store_x4(const FftArgs& a, int64_t idx, double2 ta, double2 tb)
{
    if (a.x32) {
        *reinterpret_cast<float4*>(static_cast<float*>(a.X) + idx) =
            make_float4((float)ta.x, (float)ta.y, (float)tb.x, (float)tb.y);
    } else {
        double2* p = reinterpret_cast<double2*>(static_cast<double*>(a.X) + idx);
        p[0] = ta;
        p[1] = tb;
    }
}
__device__ __forceinline__ void load_x4(const FftArgs& a, int64_t idx, double2& ta, double2& tb)
{
    if (a.x32) {
        const float4 f = *reinterpret_cast<const float4*>(static_cast<const float*>(a.X) + idx);
        ta = make_double2(f.x, f.y);
        tb = make_double2(f.z, f.w);
    } else {
        const double2* p = reinterpret_cast<const double2*>(static_cast<const double*>(a.X) + idx);
        ta = p[0];
        tb = p[1];
    }
}

// m values a thread handles per batch in the (un)folding: the global loads of a
// batch (phase factors, and coefficients when folding) are all issued before
// the first is used, so a thread waits for memory once per batch, not per m.
constexpr int MB = 8;

// Unfold the packed spectrum Z = A + i B (both Hermitian) of each sequence onto
// T_m = e^{-i m phi0} F_{m mod n} for m = 0..lmax and store m-major.  Lanes run
// over (m, sequence, part): an FP64 row takes two 16-byte parts per map pair
// (map a, map b), an FP32 row one, so a wave stores contiguous row segments of
// all nseq pairs of the ring.
__device__ __forceinline__ void unfold_store(const FftArgs& a, const double2* buf, const FftLen* L, int s, int ring, int pair0,
                                             int comp, const double2* tw_n)
{
    const int n = L->n, ls = L->lstride;
    const int lp = a.x32 ? 0 : 1;  // log2 parts per pair
    const int part = (int)threadIdx.x & ((1 << lp) - 1);
    const int sq = ((int)threadIdx.x >> lp) & (L->nseq - 1);
    const int m0 = (int)threadIdx.x >> (lp + L->lgseq), dm = NT >> (lp + L->lgseq);
    const int col = 4 * (pair0 + sq) + 2 * part;
    const int64_t xstep = (int64_t)dm * a.nring * a.ldx;
    int64_t xi = xidx(a, comp, m0, ring, col);
    const int mtop = min(a.lmax, a.rings[ring].mcut);
    MWalk w(m0, dm, n, s);
    for (int mb = m0; mb <= mtop; mb += MB * dm) {
        double2 t[MB];
        int jj[MB];
#pragma unroll
        for (int u = 0; u < MB; ++u) {
            t[u] = tw_n[w.ph];
            jj[u] = w.j;
            w.next();
        }
#pragma unroll
        for (int u = 0; u < MB; ++u) {
            if (mb + u * dm <= mtop) {
                const int j = jj[u], jn = j ? n - j : 0;
                const double2 z = buf[P(sq, j, ls)], y = buf[P(sq, jn, ls)];
                const double2 Fa = make_double2(0.5 * (z.x + y.x), 0.5 * (z.y - y.y));
                const double2 Fb = make_double2(0.5 * (z.y + y.y), 0.5 * (y.x - z.x));
                if (a.x32) {
                    store_x4(a, xi + u * xstep, cmul(t[u], Fa), cmul(t[u], Fb));
                } else {
                    *reinterpret_cast<double2*>(static_cast<double*>(a.X) + xi + u * xstep) = cmul(t[u], part ? Fb : Fa);
                }
            }
        }
        xi += MB * xstep;
    }
}

// Fold the m-major coefficients of each sequence's two maps onto the ring bins:
// Z_j = C^a_j + i C^b_j with C_j = sum_{m = j} c_m + sum_{m >= 1, -m = j} conj(c_m),
// c_m = e^{i m phi0} T_m.  CONJ accumulates conj(Z) instead (the input of an
// inverse DFT taken as conj(DFT(conj Z))).  Lanes run over (m, sequence, part)
// as in the unfolding, so a wave reads contiguous row segments; the map-b lane
// of each pair hands its term to the map-a lane, which adds both.
template <bool CONJ>
__device__ __forceinline__ void fold_load(const FftArgs& a, double2* buf, const FftLen* L, int s, int ring, int pair0, int comp,
                                          const double2* tw_n)
{
    const int n = L->n, ls = L->lstride;
    for (int e = threadIdx.x; e < L->nseq * ls; e += NT) buf[e] = make_double2(0.0, 0.0);
    __syncthreads();
    const int part = (int)threadIdx.x & 1;
    const int sq = ((int)threadIdx.x >> 1) & (L->nseq - 1);
    const int m0 = (int)threadIdx.x >> (1 + L->lgseq), dm = NT >> (1 + L->lgseq);
    const int col = 4 * (pair0 + sq) + 2 * part;
    const int64_t xstep = (int64_t)dm * a.nring * a.ldx;
    const int mtop = min(a.lmax, a.rings[ring].mcut);  // rows past the ring's cutoff are zero
    const int64_t xlast = xidx(a, comp, mtop, ring, col);
    int64_t xi = xidx(a, comp, m0, ring, col);
    const double sg = CONJ ? -1.0 : 1.0;
    MWalk w(m0, dm, n, s);
    for (int mb = m0; mb <= mtop; mb += MB * dm) {
        double2 tv[MB], t[MB];
        int jj[MB];
#pragma unroll
        for (int u = 0; u < MB; ++u) {
            const int64_t xu = min(xi + u * xstep, xlast);  // rows past lmax: clamped, unused
            if (a.x32) {
                const float2 f = *reinterpret_cast<const float2*>(static_cast<const float*>(a.X) + xu);
                tv[u] = make_double2(f.x, f.y);
            } else {
                tv[u] = *reinterpret_cast<const double2*>(static_cast<const double*>(a.X) + xu);
            }
            t[u] = tw_n[w.ph];
            jj[u] = w.j;
            w.next();
        }
#pragma unroll
        for (int u = 0; u < MB; ++u) {
            const int mm = mb + u * dm;
            const double2 ph = conjd(t[u]);
            const double2 c = cmul(ph, tv[u]);  // c_m of this lane's map
            // the map-b lane's term, received by the map-a lane (lanes differ in bit 0)
            const double cbx = __shfl_xor(c.x, 1), cby = __shfl_xor(c.y, 1);
            if (part == 0 && mm <= mtop && (!a.mown || a.mown[mm])) {
                const double2 ca = c, cb = make_double2(cbx, cby);
                double* p1 = reinterpret_cast<double*>(buf + P(sq, jj[u], ls));
                atomicAdd(p1, ca.x - cb.y);
                atomicAdd(p1 + 1, sg * (ca.y + cb.x));
                if (mm >= 1) {
                    const int jn = jj[u] ? n - jj[u] : 0;
                    double* p2 = reinterpret_cast<double*>(buf + P(sq, jn, ls));
                    atomicAdd(p2, ca.x + cb.y);
                    atomicAdd(p2 + 1, sg * (cb.x - ca.y));
                }
            }
        }
        xi += MB * xstep;
    }
    __syncthreads();
}

// Halfcomplex storage of the spectrum of a real sequence of even length n:
// [re F0, re F1, im F1, ..., re F(n/2-1), im F(n/2-1), re F(n/2)].  Positions of
// the real and imaginary parts of bin j (0 <= j < n, bins above n/2 are the
// conjugates of n - j); hc_im is -1 where the imaginary part is zero.
__device__ __forceinline__ int hc_re(int n, int j)
{
    const int h = (2 * j > n) ? n - j : j;
    return h == 0 ? 0 : (2 * h == n ? n - 1 : 2 * h - 1);
}
__device__ __forceinline__ int hc_im(int n, int j)
{
    const int h = (2 * j > n) ? n - j : j;
    return (h == 0 || 2 * h == n) ? -1 : 2 * h;
}

// ssum[2 sq] += va, ssum[2 sq + 1] += vb, called by every lane of the wave:
// one LDS atomic per wave when all lanes hold the same sequence
__device__ __forceinline__ void add_norms(double* ssum, int sq, double va, double vb)
{
    const int s0 = __builtin_amdgcn_readfirstlane(sq);
    if (__all(sq == s0)) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            va += __shfl_xor(va, o);
            vb += __shfl_xor(vb, o);
        }
        if ((threadIdx.x & 63) == 0) {
            atomicAdd(&ssum[2 * s0], va);
            atomicAdd(&ssum[2 * s0 + 1], vb);
        }
    } else {
        atomicAdd(&ssum[2 * sq], va);
        atomicAdd(&ssum[2 * sq + 1], vb);
    }
}

struct RingCtx {
    FftItem it;
    int comp;
    RingDev rg;
    const FftLen* L;
    const double2* tw_n;   // e^{-i pi j / n}
    const double2* tw_m;   // twiddles of the transform length actually run
    const double2* chirp;
    const double2* bhat;
};
// Work item of this workgroup.  The grid is one-dimensional over (component,
// item); workgroups are dealt to the 8 XCDs round-robin, so the linear index is
// remapped to give each XCD one contiguous range: the pair groups of a ring,
// which write neighbouring columns of the same m-major rows, then share an L2.
__device__ __forceinline__ RingCtx ring_ctx(const FftArgs& a, const FftItem* items, int nitems)
{
    const int nb = (int)gridDim.x, b = (int)blockIdx.x;
    const int q = nb >> 3, r = nb & 7, x = b & 7;
    const int idx = x * q + min(x, r) + (b >> 3);
    const int comp = idx / nitems;
    RingCtx c;
    c.it = items[idx - comp * nitems];
    c.comp = a.comp0 + comp;
    c.rg = a.rings[c.it.ring];
    c.L = a.lens + c.rg.len;
    c.tw_n = a.tw + c.L->tw;
    c.tw_m = c.L->blue ? a.tw + c.L->twm : c.tw_n;
    c.chirp = a.tw + c.L->chirp;
    c.bhat = a.bhat + c.L->bhat;
    return c;
}

template <int ELEMS>
__global__ __launch_bounds__(NT, ELEMS == 16 ? 2 : 4) void k_fft_fwd(FftArgs a, const FftItem* items, int nitems)
{
    extern __shared__ double2 lds[];
    const RingCtx c = ring_ctx(a, items, nitems);
    if (2 * c.it.pair0 >= a.nmaps) return;  // only padding map sets (see k_fft_p2.hip)
    const int n = c.rg.n, nseq = c.L->nseq, ls = c.L->lstride;
    const FastDiv dn(n);

    {
        // all pixel loads of the thread first (indices clamped, so none sits in
        // a branch), then the LDS writes: one wait for memory
        const int tot = nseq * n;
        const double* base = a.maps_in + (int64_t)c.comp * a.npix + c.rg.first;
        const int64_t mstride = (int64_t)a.ncomp * a.npix;
        double re[ELEMS], im[ELEMS];
#pragma unroll
        for (int q = 0; q < ELEMS; ++q) {
            const int e = min((int)threadIdx.x + q * NT, tot - 1);
            const int sq = dn.div(e), i = e - sq * n;
            const int k = 2 * (c.it.pair0 + sq);
            re[q] = base[min(k, a.nmaps - 1) * mstride + i];
            im[q] = base[min(k + 1, a.nmaps - 1) * mstride + i];
        }
#pragma unroll
        for (int q = 0; q < ELEMS; ++q) {
            const int e = (int)threadIdx.x + q * NT;
            if (e < tot) {
                const int sq = dn.div(e), i = e - sq * n;
                const int k = 2 * (c.it.pair0 + sq);
                lds[P(sq, i, ls)] = make_double2(k < a.nmaps ? re[q] : 0.0, k + 1 < a.nmaps ? im[q] : 0.0);
            }
        }
    }
    __syncthreads();
    ring_dft<ELEMS>(lds, nseq, c.L, c.tw_m, c.chirp, c.bhat);

    if (a.F) {  // keep the data spectra of both maps (iterative map2alm)
        for (int e = threadIdx.x; e < nseq * n; e += NT) {
            const int sq = dn.div(e), pos = e - sq * n;
            const int j = (pos == 0) ? 0 : (pos == n - 1 ? n / 2 : (pos + 1) / 2);
            const int jn = j ? n - j : 0;
            const double2 z = lds[P(sq, j, ls)], y = lds[P(sq, jn, ls)];
            const double2 Fa = make_double2(0.5 * (z.x + y.x), 0.5 * (z.y - y.y));
            const double2 Fb = make_double2(0.5 * (z.y + y.y), 0.5 * (y.x - z.x));
            const bool im = (pos != 0) && (pos != n - 1) && ((pos & 1) == 0);
            const int k = 2 * (c.it.pair0 + sq);
            if (k < a.nmaps) a.F[((int64_t)k * a.ncomp + c.comp) * a.npix + c.rg.first + pos] = im ? Fa.y : Fa.x;
            if (k + 1 < a.nmaps) a.F[((int64_t)(k + 1) * a.ncomp + c.comp) * a.npix + c.rg.first + pos] = im ? Fb.y : Fb.x;
        }
    }
    unfold_store(a, lds, c.L, c.rg.s, c.it.ring, c.it.pair0, c.comp, c.tw_n);
}

template <int ELEMS>
__global__ __launch_bounds__(NT, ELEMS == 16 ? 2 : 4) void k_fft_inv(FftArgs a, const FftItem* items, int nitems)
{
    extern __shared__ double2 lds[];
    const RingCtx c = ring_ctx(a, items, nitems);
    if (2 * c.it.pair0 >= a.nmaps) return;  // only padding map sets (see k_fft_p2.hip)
    const int n = c.rg.n, nseq = c.L->nseq, ls = c.L->lstride;
    const FastDiv dn(n);

    // inverse DFT as conj(DFT(conj(Z))): the fold accumulates conj(Z)
    fold_load<true>(a, lds, c.L, c.rg.s, c.it.ring, c.it.pair0, c.comp, c.tw_n);
    ring_dft<ELEMS>(lds, nseq, c.L, c.tw_m, c.chirp, c.bhat);
    for (int e = threadIdx.x; e < nseq * n; e += NT) {
        const int sq = dn.div(e), i = e - sq * n;
        const int k = 2 * (c.it.pair0 + sq);
        const double2 z = lds[P(sq, i, ls)];
        if (k < a.nmaps) a.maps_out[((int64_t)k * a.ncomp + c.comp) * a.npix + c.rg.first + i] = z.x;
        if (k + 1 < a.nmaps) a.maps_out[((int64_t)(k + 1) * a.ncomp + c.comp) * a.npix + c.rg.first + i] = -z.y;
    }
}

// Residual of the iterative map2alm in the Fourier domain, FP64:
// R_j = F_j - n C_j  (data spectrum minus the synthesised ring spectrum), then
// T^res_m = e^{-i m phi0} R_{m mod n} written over X; sum |r|^2 = (1/n) sum_j |R_j|^2
// is accumulated per map (Parseval).
template <int ELEMS>
__global__ __launch_bounds__(NT, ELEMS == 16 ? 2 : 4) void k_residual(FftArgs a, const FftItem* items, int nitems)
{
    extern __shared__ double2 lds[];
    const RingCtx c = ring_ctx(a, items, nitems);
    if (2 * c.it.pair0 >= a.nmaps) return;  // only padding map sets (see k_fft_p2.hip)
    const int n = c.rg.n, nseq = c.L->nseq, ls = c.L->lstride;
    const FastDiv dn(n);

    // residual sums of squares per map of each sequence: reduced over the wave
    // when the wave holds one sequence, accumulated in LDS within the workgroup,
    // then one global atomic per map (same-address global atomics from every
    // element serialise in the L2)
    __shared__ double ssum[2 * 16];
    if (threadIdx.x < 2 * 16) ssum[threadIdx.x] = 0.0;
    fold_load<false>(a, lds, c.L, c.rg.s, c.it.ring, c.it.pair0, c.comp, c.tw_n);
    const int tot = nseq * n;
    const double dnn = (double)n;
    const double* fbase = a.F + (int64_t)c.comp * a.npix + c.rg.first;
    const int64_t mstride = (int64_t)a.ncomp * a.npix;
    // stored data spectra of both maps at bin j: all loads first
    double fa[ELEMS][2], fb[ELEMS][2];
#pragma unroll
    for (int q = 0; q < ELEMS; ++q) {
        const int e = min((int)threadIdx.x + q * NT, tot - 1);
        const int sq = dn.div(e), j = e - sq * n;
        const int k = 2 * (c.it.pair0 + sq);
        const int ir = hc_re(n, j), ii = max(hc_im(n, j), 0);
        const double* f0 = fbase + min(k, a.nmaps - 1) * mstride;
        const double* f1 = fbase + min(k + 1, a.nmaps - 1) * mstride;
        fa[q][0] = f0[ir];
        fa[q][1] = f0[ii];
        fb[q][0] = f1[ir];
        fb[q][1] = f1[ii];
    }
    double2 res[ELEMS];
    double ssa[ELEMS], ssb[ELEMS];
#pragma unroll
    for (int q = 0; q < ELEMS; ++q) {
        const int e = min((int)threadIdx.x + q * NT, tot - 1);
        const int sq = dn.div(e), j = e - sq * n;
        const int jn = j ? n - j : 0;
        const double2 z = lds[P(sq, j, ls)], y = lds[P(sq, jn, ls)];
        const double2 Ca = make_double2(0.5 * (z.x + y.x), 0.5 * (z.y - y.y));
        const double2 Cb = make_double2(0.5 * (z.y + y.y), 0.5 * (y.x - z.x));
        const int k = 2 * (c.it.pair0 + sq);
        const double isg = hc_im(n, j) < 0 ? 0.0 : (2 * j > n ? -1.0 : 1.0);
        const double2 Fa = make_double2(fa[q][0], isg * fa[q][1]), Fb = make_double2(fb[q][0], isg * fb[q][1]);
        double2 Ra = make_double2(Fa.x - dnn * Ca.x, Fa.y - dnn * Ca.y);
        double2 Rb = make_double2(Fb.x - dnn * Cb.x, Fb.y - dnn * Cb.y);
        if (k >= a.nmaps) Ra = make_double2(0.0, 0.0);
        if (k + 1 >= a.nmaps) Rb = make_double2(0.0, 0.0);
        const bool live = (int)threadIdx.x + q * NT < tot;
        ssa[q] = live ? (Ra.x * Ra.x + Ra.y * Ra.y) / dnn : 0.0;
        ssb[q] = live ? (Rb.x * Rb.x + Rb.y * Rb.y) / dnn : 0.0;
        if (a.store_res && live && 2 * j <= n) {
            // the stored bins (2j <= n) of both maps into R, maps contiguous per bin
            const int ir = hc_re(n, j), ii = hc_im(n, j);
            double* r0 = a.R + ((int64_t)c.comp * a.npix + c.rg.first) * a.nmaps + k;
            if (k < a.nmaps) {
                r0[(int64_t)ir * a.nmaps] = Ra.x;
                if (ii >= 0) r0[(int64_t)ii * a.nmaps] = Ra.y;
            }
            if (k + 1 < a.nmaps) {
                r0[(int64_t)ir * a.nmaps + 1] = Rb.x;
                if (ii >= 0) r0[(int64_t)ii * a.nmaps + 1] = Rb.y;
            }
        }
        res[q] = make_double2(Ra.x - Rb.y, Ra.y + Rb.x);  // pack as Ra + i Rb
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < ELEMS; ++q) {
        const int e = (int)threadIdx.x + q * NT;
        const int sq = dn.div(min(e, tot - 1));
        if (e < tot) lds[P(sq, e - sq * n, ls)] = res[q];
        if (a.norms) add_norms(ssum, sq, ssa[q], ssb[q]);
    }
    __syncthreads();
    if (a.norms && threadIdx.x < 2 * nseq) {
        const int sq = threadIdx.x >> 1, k = 2 * (c.it.pair0 + sq) + (threadIdx.x & 1);
        if (k < a.nmaps) atomicAdd(a.norms + (int64_t)k * a.ncomp + c.comp, ssum[threadIdx.x]);
    }
    if (a.iteration_sub) unfold_store(a, lds, c.L, c.rg.s, c.it.ring, c.it.pair0, c.comp, c.tw_n);
}

// Bluestein kernel spectra: b_k = e^{+i pi k^2/n} for |k| < n placed circularly
// in length m, transformed forward and divided by m.  One workgroup per length.
template <int ELEMS>
__global__ __launch_bounds__(NT) void k_bluestein_init(const FftLen* lens, const int* blue_lens, const double2* tw,
                                                       double2* bhat)
{
    extern __shared__ double2 lds[];
    const FftLen* L = lens + blue_lens[blockIdx.x];
    const int n = L->n, m = L->m, ls = L->lstride;
    const double2* chirp = tw + L->chirp;
    for (int i = threadIdx.x; i < m; i += NT) {
        const int k = (i < n) ? i : (i > m - n ? m - i : -1);
        double2 v = make_double2(0.0, 0.0);
        if (k >= 0) v = conjd(chirp[k]);
        lds[P(0, i, ls)] = v;
    }
    __syncthreads();
    fft_lds<ELEMS>(lds, 1, m, ls, L->nstage, L->radix, tw + L->twm);
    const double inv = 1.0 / (double)m;
    for (int i = threadIdx.x; i < m; i += NT) {
        const double2 v = lds[P(0, i, ls)];
        bhat[L->bhat + i] = make_double2(v.x * inv, v.y * inv);
    }
}

enum class Kind { Fwd, Inv, Res };

template <int E>
hipError_t launch_one(Kind kind, const FftArgs& a, const FftClass& c, int ncompl, hipStream_t st)
{
    size_t sh = (size_t)c.lds * sizeof(double2);
    dim3 grid(c.nitems * ncompl);
    if (sh > 65536) {
        const void* f = (kind == Kind::Fwd) ? (const void*)k_fft_fwd<E>
                        : (kind == Kind::Inv) ? (const void*)k_fft_inv<E> : (const void*)k_residual<E>;
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
        if (e != hipSuccess) return e;
    }
    if (kind == Kind::Fwd) hipLaunchKernelGGL(k_fft_fwd<E>, grid, dim3(NT), sh, st, a, c.items, c.nitems);
    else if (kind == Kind::Inv) hipLaunchKernelGGL(k_fft_inv<E>, grid, dim3(NT), sh, st, a, c.items, c.nitems);
    else hipLaunchKernelGGL(k_residual<E>, grid, dim3(NT), sh, st, a, c.items, c.nitems);
    return hipGetLastError();
}

hipError_t launch_classes(Kind kind, const FftArgs& a, const FftClass* cls, int ncls, int ncompl, hipStream_t st)
{
    for (int i = 0; i < ncls; ++i) {
        if (cls[i].nitems <= 0) continue;
        hipError_t e;
        if (cls[i].four)  // the residual kernel of the iteration does not cover these rings
            e = kind == Kind::Res ? hipErrorNotSupported : launch_fft_four(kind == Kind::Fwd, a, cls[i], ncompl, st);
        else if (cls[i].p2 && kind != Kind::Res) e = launch_fft_p2(kind == Kind::Fwd, a, cls[i], ncompl, st);
        else if (cls[i].elems <= 2) e = launch_one<2>(kind, a, cls[i], ncompl, st);
        else if (cls[i].elems <= 8) e = launch_one<8>(kind, a, cls[i], ncompl, st);
        else e = launch_one<16>(kind, a, cls[i], ncompl, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

hipError_t launch_fft_forward(const FftArgs& a, const FftClass* cls, int ncls, int ncompl, hipStream_t st)
{
    return launch_classes(Kind::Fwd, a, cls, ncls, ncompl, st);
}

hipError_t launch_fft_inverse(const FftArgs& a, const FftClass* cls, int ncls, int ncompl, hipStream_t st)
{
    return launch_classes(Kind::Inv, a, cls, ncls, ncompl, st);
}

hipError_t launch_residual(const FftArgs& a, const FftClass* cls, int ncls, int ncompl, hipStream_t st)
{
    return launch_classes(Kind::Res, a, cls, ncls, ncompl, st);
}

hipError_t launch_bluestein_init(const FftLen* lens, const int* blue_lens, int nblue, const double2* tw,
                                 double2* bhat, int lds, hipStream_t st)
{
    if (nblue <= 0) return hipSuccess;
    if ((size_t)lds * sizeof(double2) > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)k_bluestein_init<16>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)((size_t)lds * sizeof(double2)));
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_bluestein_init<16>, dim3(nblue), dim3(NT), (size_t)lds * sizeof(double2), st, lens,
                       blue_lens, tw, bhat);
    return hipGetLastError();
}

}  // namespace sht
