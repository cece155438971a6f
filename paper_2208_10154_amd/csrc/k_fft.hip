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
#include "sht_internal.h"

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

// R-point forward DFT (odd R) in registers with W[t] = e^{-2 pi i t/R}, using
// the conjugate symmetry W^{(R-r)q} = conj(W^{rq}): with s_r = v_r + v_{R-r},
// d_r = v_r - v_{R-r}, out_q = A + iB and out_{R-q} = A - iB where
// A = v_0 + sum_r Re(W^{rq}) s_r and B = sum_r Im(W^{rq}) d_r.
template <int R>
__device__ __forceinline__ void dft(double2* v, const double2* W)
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
            const double2 w = W[(r * q) % R];
            A.x += w.x * sv[r - 1].x; A.y += w.x * sv[r - 1].y;
            B.x += w.y * dv[r - 1].x; B.y += w.y * dv[r - 1].y;
        }
        o[q] = make_double2(A.x - B.y, A.y + B.x);
        o[R - q] = make_double2(A.x + B.y, A.y - B.x);
    }
#pragma unroll
    for (int q = 0; q < R; ++q) v[q] = o[q];
}
template <>
__device__ __forceinline__ void dft<2>(double2* v, const double2*)
{
    double2 t = v[0];
    v[0] = cadd(t, v[1]);
    v[1] = csub(t, v[1]);
}
template <>
__device__ __forceinline__ void dft<4>(double2* v, const double2*)
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
template <int R, int ELEMS>
__device__ __forceinline__ void stockham_step(double2* buf, int nseq, int n, int len, int Ns, const double2* tw)
{
    constexpr int MAXB = (ELEMS + R - 1) / R;
    const int nb = n / R;
    const int tot = nseq * nb;
    const int unit = 2 * (n / (Ns * R));
    double2 W[R];
    if (R != 2 && R != 4) {
#pragma unroll
        for (int t = 0; t < R; ++t) W[t] = tw[(2 * n / R) * t];
    }
    double2 v[MAXB][R];
#pragma unroll
    for (int q = 0; q < MAXB; ++q) {
        int w = threadIdx.x + q * NT;
        if (w < tot) {
            int sq = w / nb, j = w - sq * nb;
#pragma unroll
            for (int r = 0; r < R; ++r) v[q][r] = buf[sq * len + j + r * nb];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MAXB; ++q) {
        int w = threadIdx.x + q * NT;
        if (w < tot) {
            int sq = w / nb, j = w - sq * nb;
            int k = j % Ns;
#pragma unroll
            for (int r = 1; r < R; ++r) v[q][r] = cmul(v[q][r], tw[r * k * unit]);
            dft<R>(v[q], W);
            int base = (j / Ns) * Ns * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[sq * len + base + r * Ns] = v[q][r];
        }
    }
    __syncthreads();
}

// Forward DFT (e^{-2 pi i jk/n}) of nseq sequences (stride len) in LDS.
template <int ELEMS>
__device__ __forceinline__ void fft_lds(double2* buf, int nseq, int n, int len, int nstage, const int* radix, const double2* tw)
{
    int Ns = 1;
    for (int s = 0; s < nstage; ++s) {
        int R = radix[s];
        switch (R) {
            case 4: stockham_step<4, ELEMS>(buf, nseq, n, len, Ns, tw); break;
            case 2: stockham_step<2, ELEMS>(buf, nseq, n, len, Ns, tw); break;
            case 3: stockham_step<3, ELEMS>(buf, nseq, n, len, Ns, tw); break;
            case 5: stockham_step<5, ELEMS>(buf, nseq, n, len, Ns, tw); break;
            default: stockham_step<7, ELEMS>(buf, nseq, n, len, Ns, tw); break;
        }
        Ns *= R;
    }
}

// Ring DFT of length n of the sequences already loaded in buf[sq*len + i], i < n.
// Direct: Stockham over n.  Bluestein: y_j = w_j sum_i (x_i w_i) conj(w_{j-i}),
// w_i = e^{-i pi i^2/n}, the convolution done through length m with the
// precomputed kernel spectrum (which carries the 1/m of the inverse).
template <int ELEMS>
__device__ __forceinline__ void ring_dft(double2* buf, int nseq, const FftLen* L, const double2* tw_n, const double2* tw_m,
                         const double2* bhat)
{
    const int n = L->n;
    if (!L->blue) {
        fft_lds<ELEMS>(buf, nseq, n, n, L->nstage, L->radix, tw_n);
        return;
    }
    const int m = L->m;
    const int two_n = 2 * n;
    for (int e = threadIdx.x; e < nseq * m; e += NT) {
        int sq = e / m, i = e - sq * m;
        double2 v = make_double2(0.0, 0.0);
        if (i < n) v = cmul(buf[sq * m + i], tw_n[(int)(((unsigned)(i * i)) % (unsigned)two_n)]);
        buf[sq * m + i] = v;
    }
    __syncthreads();
    fft_lds<ELEMS>(buf, nseq, m, m, L->nstage, L->radix, tw_m);
    for (int e = threadIdx.x; e < nseq * m; e += NT) {
        int i = e % m;
        buf[e] = conjd(cmul(buf[e], bhat[i]));
    }
    __syncthreads();
    fft_lds<ELEMS>(buf, nseq, m, m, L->nstage, L->radix, tw_m);
    for (int e = threadIdx.x; e < nseq * n; e += NT) {
        int sq = e / n, j = e - sq * n;
        buf[sq * m + j] = cmul(tw_n[(int)(((unsigned)(j * j)) % (unsigned)two_n)], conjd(buf[sq * m + j]));
    }
    __syncthreads();
}

__device__ __forceinline__ int64_t xidx(const FftArgs& a, int comp, int m, int ring, int col)
{
    return (int64_t)comp * a.xcomp + ((int64_t)m * a.nring + ring) * a.ldx + col;
}

__device__ __forceinline__ double2 load_x2(const FftArgs& a, int64_t idx)
{
    if (a.x32) {
        float2 f = *reinterpret_cast<const float2*>(static_cast<const float*>(a.X) + idx);
        return make_double2(f.x, f.y);
    }
    return *reinterpret_cast<const double2*>(static_cast<const double*>(a.X) + idx);
}

// Unfold the packed spectrum Z = A + i B (both Hermitian) of each sequence onto
// T_m = e^{-i m phi0} F_{m mod n} for m = 0..lmax and store m-major.
__device__ __forceinline__ void unfold_store(const FftArgs& a, const double2* buf, int len, int nseq, int n, int s, int ring,
                             int pair0, int comp, const double2* tw_n)
{
    const int per_m = 4 * nseq;
    const int tot = (a.lmax + 1) * per_m;
    const int two_n = 2 * n;
    for (int e = threadIdx.x; e < tot; e += NT) {
        int mm = e / per_m, q = e - mm * per_m;
        int sq = q >> 2, w = q & 3;
        int j = mm % n, jn = (n - j) % n;
        double2 z = buf[sq * len + j], y = buf[sq * len + jn];
        double2 F = (w < 2) ? make_double2(0.5 * (z.x + y.x), 0.5 * (z.y - y.y))
                            : make_double2(0.5 * (z.y + y.y), 0.5 * (y.x - z.x));
        double2 T = cmul(tw_n[(int)(((unsigned)(mm * s)) % (unsigned)two_n)], F);
        double val = (w & 1) ? T.y : T.x;
        int64_t idx = xidx(a, comp, mm, ring, 4 * (pair0 + sq) + w);
        if (a.x32) static_cast<float*>(a.X)[idx] = (float)val;
        else static_cast<double*>(a.X)[idx] = val;
    }
}

// Fold the m-major coefficients of each sequence's two maps onto the ring bins:
// Z_j = C^a_j + i C^b_j with C_j = sum_{m = j} c_m + sum_{m >= 1, -m = j} conj(c_m),
// c_m = e^{i m phi0} T_m.
__device__ __forceinline__ void fold_load(const FftArgs& a, double2* buf, int len, int nseq, int n, int s, int ring, int pair0,
                          int comp, const double2* tw_n)
{
    for (int e = threadIdx.x; e < nseq * len; e += NT) buf[e] = make_double2(0.0, 0.0);
    __syncthreads();
    const int two_n = 2 * n;
    const int tot = (a.lmax + 1) * nseq;
    for (int e = threadIdx.x; e < tot; e += NT) {
        int mm = e / nseq, sq = e - mm * nseq;
        int64_t idx = xidx(a, comp, mm, ring, 4 * (pair0 + sq));
        double2 ta = load_x2(a, idx), tb = load_x2(a, idx + 2);
        double2 ph = conjd(tw_n[(int)(((unsigned)(mm * s)) % (unsigned)two_n)]);
        double2 ca = cmul(ph, ta), cb = cmul(ph, tb);
        int j1 = mm % n;
        double* p1 = reinterpret_cast<double*>(buf + sq * len + j1);
        atomicAdd(p1, ca.x - cb.y);
        atomicAdd(p1 + 1, ca.y + cb.x);
        if (mm >= 1) {
            int j2 = (n - j1) % n;
            double* p2 = reinterpret_cast<double*>(buf + sq * len + j2);
            atomicAdd(p2, ca.x + cb.y);
            atomicAdd(p2 + 1, cb.x - ca.y);
        }
    }
    __syncthreads();
}

// halfcomplex position of bin j (0 <= j <= n/2) of a real length-n sequence:
// [re F0, re F1, im F1, ..., re F(n/2-1), im F(n/2-1), re F(n/2)]
__device__ __forceinline__ double2 hc_get(const double* f, int n, int j)
{
    bool conj = false;
    if (j > n / 2) { j = n - j; conj = true; }
    double re, im;
    if (j == 0) { re = f[0]; im = 0.0; }
    else if (2 * j == n) { re = f[n - 1]; im = 0.0; }
    else { re = f[2 * j - 1]; im = f[2 * j]; }
    return make_double2(re, conj ? -im : im);
}

template <int ELEMS>
__global__ __launch_bounds__(NT) void k_fft_fwd(FftArgs a, const FftItem* items)
{
    extern __shared__ double2 lds[];
    const FftItem it = items[blockIdx.x];
    const int comp = a.comp0 + blockIdx.y;
    const RingDev rg = a.rings[it.ring];
    const FftLen* L = a.lens + rg.len;
    const int n = rg.n;
    const int nseq = min(L->nseq, a.npairs - it.pair0);
    const int len = L->blue ? L->m : n;
    const double2* tw_n = a.tw + L->tw;

    for (int e = threadIdx.x; e < nseq * n; e += NT) {
        int sq = e / n, i = e - sq * n;
        int k = 2 * (it.pair0 + sq);
        double re = 0.0, im = 0.0;
        if (k < a.nmaps) re = a.maps_in[((int64_t)k * a.ncomp + comp) * a.npix + rg.first + i];
        if (k + 1 < a.nmaps) im = a.maps_in[((int64_t)(k + 1) * a.ncomp + comp) * a.npix + rg.first + i];
        lds[sq * len + i] = make_double2(re, im);
    }
    __syncthreads();
    ring_dft<ELEMS>(lds, nseq, L, tw_n, a.tw + L->twm, a.bhat + L->bhat);

    if (a.F) {  // keep the data spectra of both maps (iterative map2alm)
        for (int e = threadIdx.x; e < nseq * n; e += NT) {
            int sq = e / n, pos = e - sq * n;
            int j = (pos == 0) ? 0 : (pos == n - 1 ? n / 2 : (pos + 1) / 2);
            int jn = (n - j) % n;
            double2 z = lds[sq * len + j], y = lds[sq * len + jn];
            double2 Fa = make_double2(0.5 * (z.x + y.x), 0.5 * (z.y - y.y));
            double2 Fb = make_double2(0.5 * (z.y + y.y), 0.5 * (y.x - z.x));
            bool im = (pos != 0) && (pos != n - 1) && ((pos & 1) == 0);
            int k = 2 * (it.pair0 + sq);
            if (k < a.nmaps) a.F[((int64_t)k * a.ncomp + comp) * a.npix + rg.first + pos] = im ? Fa.y : Fa.x;
            if (k + 1 < a.nmaps) a.F[((int64_t)(k + 1) * a.ncomp + comp) * a.npix + rg.first + pos] = im ? Fb.y : Fb.x;
        }
    }
    unfold_store(a, lds, len, nseq, n, rg.s, it.ring, it.pair0, comp, tw_n);
}

template <int ELEMS>
__global__ __launch_bounds__(NT) void k_fft_inv(FftArgs a, const FftItem* items)
{
    extern __shared__ double2 lds[];
    const FftItem it = items[blockIdx.x];
    const int comp = a.comp0 + blockIdx.y;
    const RingDev rg = a.rings[it.ring];
    const FftLen* L = a.lens + rg.len;
    const int n = rg.n;
    const int nseq = min(L->nseq, a.npairs - it.pair0);
    const int len = L->blue ? L->m : n;
    const double2* tw_n = a.tw + L->tw;

    fold_load(a, lds, len, nseq, n, rg.s, it.ring, it.pair0, comp, tw_n);
    // inverse DFT as conj(DFT(conj(Z)))
    for (int e = threadIdx.x; e < nseq * n; e += NT) {
        int sq = e / n, j = e - sq * n;
        lds[sq * len + j] = conjd(lds[sq * len + j]);
    }
    __syncthreads();
    ring_dft<ELEMS>(lds, nseq, L, tw_n, a.tw + L->twm, a.bhat + L->bhat);
    for (int e = threadIdx.x; e < nseq * n; e += NT) {
        int sq = e / n, i = e - sq * n;
        int k = 2 * (it.pair0 + sq);
        double2 z = lds[sq * len + i];
        if (k < a.nmaps) a.maps_out[((int64_t)k * a.ncomp + comp) * a.npix + rg.first + i] = z.x;
        if (k + 1 < a.nmaps) a.maps_out[((int64_t)(k + 1) * a.ncomp + comp) * a.npix + rg.first + i] = -z.y;
    }
}

// Residual of the iterative map2alm in the Fourier domain, FP64:
// R_j = F_j - n C_j  (data spectrum minus the synthesised ring spectrum), then
// T^res_m = e^{-i m phi0} R_{m mod n} written over X; sum |r|^2 = (1/n) sum_j |R_j|^2
// is accumulated per map (Parseval).
template <int ELEMS>
__global__ __launch_bounds__(NT) void k_residual(FftArgs a, const FftItem* items)
{
    extern __shared__ double2 lds[];
    const FftItem it = items[blockIdx.x];
    const int comp = a.comp0 + blockIdx.y;
    const RingDev rg = a.rings[it.ring];
    const FftLen* L = a.lens + rg.len;
    const int n = rg.n;
    const int nseq = min(L->nseq, a.npairs - it.pair0);
    const int len = L->blue ? L->m : n;
    const double2* tw_n = a.tw + L->tw;

    fold_load(a, lds, len, nseq, n, rg.s, it.ring, it.pair0, comp, tw_n);
    constexpr int PER = (ELEMS + 0);
    double2 res[PER];
    double ssa[PER], ssb[PER];
    const double dn = (double)n;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        int e = threadIdx.x + q * NT;
        ssa[q] = ssb[q] = 0.0;
        if (e < nseq * n) {
            int sq = e / n, j = e - sq * n;
            int jn = (n - j) % n;
            double2 z = lds[sq * len + j], y = lds[sq * len + jn];
            double2 Ca = make_double2(0.5 * (z.x + y.x), 0.5 * (z.y - y.y));
            double2 Cb = make_double2(0.5 * (z.y + y.y), 0.5 * (y.x - z.x));
            int k = 2 * (it.pair0 + sq);
            double2 Fa = make_double2(0.0, 0.0), Fb = make_double2(0.0, 0.0);
            if (k < a.nmaps) Fa = hc_get(a.F + ((int64_t)k * a.ncomp + comp) * a.npix + rg.first, n, j);
            if (k + 1 < a.nmaps) Fb = hc_get(a.F + ((int64_t)(k + 1) * a.ncomp + comp) * a.npix + rg.first, n, j);
            double2 Ra = make_double2(Fa.x - dn * Ca.x, Fa.y - dn * Ca.y);
            double2 Rb = make_double2(Fb.x - dn * Cb.x, Fb.y - dn * Cb.y);
            if (k >= a.nmaps) Ra = make_double2(0.0, 0.0);
            if (k + 1 >= a.nmaps) Rb = make_double2(0.0, 0.0);
            ssa[q] = (Ra.x * Ra.x + Ra.y * Ra.y) / dn;
            ssb[q] = (Rb.x * Rb.x + Rb.y * Rb.y) / dn;
            res[q] = make_double2(Ra.x - Rb.y, Ra.y + Rb.x);  // pack as Ra + i Rb
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        int e = threadIdx.x + q * NT;
        if (e < nseq * n) {
            int sq = e / n, j = e - sq * n;
            lds[sq * len + j] = res[q];
            int k = 2 * (it.pair0 + sq);
            if (a.norms) {
                if (ssa[q] != 0.0) atomicAdd(a.norms + (int64_t)k * a.ncomp + comp, ssa[q]);
                if (ssb[q] != 0.0) atomicAdd(a.norms + (int64_t)(k + 1) * a.ncomp + comp, ssb[q]);
            }
        }
    }
    __syncthreads();
    if (a.iteration_sub) unfold_store(a, lds, len, nseq, n, rg.s, it.ring, it.pair0, comp, tw_n);
}

// Bluestein kernel spectra: b_k = e^{+i pi k^2/n} for |k| < n placed circularly
// in length m, transformed forward and divided by m.  One workgroup per length.
template <int ELEMS>
__global__ __launch_bounds__(NT) void k_bluestein_init(const FftLen* lens, const int* blue_lens, const double2* tw,
                                                       double2* bhat)
{
    extern __shared__ double2 lds[];
    const FftLen* L = lens + blue_lens[blockIdx.x];
    const int n = L->n, m = L->m;
    const double2* tw_n = tw + L->tw;
    for (int i = threadIdx.x; i < m; i += NT) {
        int k = (i < n) ? i : (i > m - n ? m - i : -1);
        double2 v = make_double2(0.0, 0.0);
        if (k >= 0) v = conjd(tw_n[(int)(((unsigned)(k * k)) % (unsigned)(2 * n))]);
        lds[i] = v;
    }
    __syncthreads();
    fft_lds<ELEMS>(lds, 1, m, m, L->nstage, L->radix, tw + L->twm);
    const double inv = 1.0 / (double)m;
    for (int i = threadIdx.x; i < m; i += NT) bhat[L->bhat + i] = make_double2(lds[i].x * inv, lds[i].y * inv);
}

enum class Kind { Fwd, Inv, Res };

template <int E>
hipError_t launch_one(Kind kind, const FftArgs& a, const FftClass& c, int ncompl, hipStream_t st)
{
    size_t sh = (size_t)c.lds * sizeof(double2);
    dim3 grid(c.nitems, ncompl);
    if (sh > 65536) {
        const void* f = (kind == Kind::Fwd) ? (const void*)k_fft_fwd<E>
                        : (kind == Kind::Inv) ? (const void*)k_fft_inv<E> : (const void*)k_residual<E>;
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
        if (e != hipSuccess) return e;
    }
    if (kind == Kind::Fwd) hipLaunchKernelGGL(k_fft_fwd<E>, grid, dim3(NT), sh, st, a, c.items);
    else if (kind == Kind::Inv) hipLaunchKernelGGL(k_fft_inv<E>, grid, dim3(NT), sh, st, a, c.items);
    else hipLaunchKernelGGL(k_residual<E>, grid, dim3(NT), sh, st, a, c.items);
    return hipGetLastError();
}

hipError_t launch_classes(Kind kind, const FftArgs& a, const FftClass* cls, int ncls, int ncompl, hipStream_t st)
{
    for (int i = 0; i < ncls; ++i) {
        if (cls[i].nitems <= 0) continue;
        hipError_t e;
        if (cls[i].elems <= 2) e = launch_one<2>(kind, a, cls[i], ncompl, st);
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
