// Ring FFTs for power-of-two ring lengths (HIP, gfx950).
//
// Every equatorial-belt ring of a HEALPix grid has N = 4 nside pixels, a power of
// two for the usual resolutions, and those rings hold two thirds of the pixels.
// For them the length is a template parameter, so every stride, pass count and
// LDS offset below is a compile-time constant: the index arithmetic that the
// runtime-length kernels (k_fft.hip) spend most of their instructions on folds
// into immediate offsets, and what remains is the butterflies themselves.
//
// Transform: two real maps are packed as z = a + i b (forward) and the length-N
// DFT is a Stockham autosort FFT of radix-8 passes with one final radix-2, -4 or
// -8 pass.  Each thread owns 8 values of one sequence: the first pass reads them
// straight from global memory (forward) or gathers them from the m-major
// coefficients (inverse), later passes exchange through LDS, and the last pass
// leaves its outputs in natural order.  The FFT mapping is that of the paper
// (Sec. 2.1 eq. "mm", Appendix A.1): T_m = e^{-i m phi0} F_{m mod N} forward, and
// C_j = sum_{m = j} c_m + sum_{m >= 1, -m = j} conj(c_m), c_m = e^{i m phi0} T_m,
// backward (mod N), with the inverse DFT taken as conj(DFT(conj C)).
#include "fft_p2.h"

namespace sht {
namespace {

template <int LOGN, typename XT>
__device__ __forceinline__ void fwd_item(const FftArgs& a, const Item it, double2* lds)
{
    using C = P2<LOGN>;
    constexpr int N = C::N, T = C::T, S = C::S;
    const RingDev rg = a.rings[it.ring];
    const double2* tw = a.tw + a.lens[rg.len].tw;  // e^{-i pi t/N}, t < 2N
    const int seq = (int)threadIdx.x / T, tl = (int)threadIdx.x % T;
    double2* sb = lds + seq * C::SEQ;
    const int k = 2 * (it.pair0 + seq);

    // pass-0 inputs x[tl + r T] of map pair (k, k+1), straight from global memory
    double2 v[8], w[8];
    {
        const int64_t ms = (int64_t)a.ncomp * a.npix;
        const double* pa = a.maps_in + (int64_t)it.comp * a.npix + rg.first + min(k, a.nmaps - 1) * ms;
        const double* pb = a.maps_in + (int64_t)it.comp * a.npix + rg.first + min(k + 1, a.nmaps - 1) * ms;
#pragma unroll
        for (int r = 0; r < 8; ++r) v[r] = make_double2(pa[tl + r * T], pb[tl + r * T]);
#pragma unroll
        for (int r = 0; r < 8; ++r)
            v[r] = make_double2(k < a.nmaps ? v[r].x : 0.0, k + 1 < a.nmaps ? v[r].y : 0.0);
    }
    run_passes<LOGN, 0>(v, w, sb, tl, tw);

    // spectrum Z in natural order into LDS
    using QL = Pass<LOGN, C::NP - 1>;
    __syncthreads();
#pragma unroll
    for (int b = 0; b < QL::B; ++b) {
#pragma unroll
        for (int r = 0; r < QL::R; ++r) sb[tl + T * b + r * (N / QL::R)] = v[b * QL::R + r];
    }
    __syncthreads();

    if (a.F) {  // keep the data spectra of both maps (iterative map2alm), halfcomplex
        for (int pos = tl; pos < N; pos += T) {
            const int j = (pos == 0) ? 0 : (pos == N - 1 ? N / 2 : (pos + 1) / 2);
            const int jn = (N - j) & (N - 1);
            const double2 z = sb[j], y = sb[jn];
            const double2 Fa = make_double2(0.5 * (z.x + y.x), 0.5 * (z.y - y.y));
            const double2 Fb = make_double2(0.5 * (z.y + y.y), 0.5 * (y.x - z.x));
            const bool im = (pos != 0) && (pos != N - 1) && ((pos & 1) == 0);
            if (k < a.nmaps) a.F[((int64_t)k * a.ncomp + it.comp) * a.npix + rg.first + pos] = im ? Fa.y : Fa.x;
            if (k + 1 < a.nmaps)
                a.F[((int64_t)(k + 1) * a.ncomp + it.comp) * a.npix + rg.first + pos] = im ? Fb.y : Fb.x;
        }
    }

    // unfold T_m = e^{-i m phi0} F_{m mod N}.  Lanes run over (m, pair, part):
    // FP64 rows take two 16-byte parts per pair (map k, map k+1), FP32 rows one,
    // so the lanes of a wave store contiguous row segments of all S pairs.
    constexpr int LP = sizeof(XT) == 8 ? 1 : 0;  // log2 parts per pair
    constexpr int MSTEP = C::NTH >> (LP + C::LOGS);
    const int part = (int)threadIdx.x & ((1 << LP) - 1);
    const int sq = ((int)threadIdx.x >> LP) & (S - 1);
    const int mi = (int)threadIdx.x >> (LP + C::LOGS);
    const double2* zs = lds + sq * C::SEQ;
    XT* X = static_cast<XT*>(a.X) + (int64_t)it.comp * a.xcomp + (int64_t)it.ring * a.ldx + 4 * (it.pair0 + sq) + 2 * part;
    const int64_t mrow = (int64_t)a.nring * a.ldx;
    const int s = rg.s, mtop = min(a.lmax, rg.mcut);
    for (int m0 = mi; m0 <= mtop; m0 += MB * MSTEP) {
        double2 ph[MB];
#pragma unroll
        for (int u = 0; u < MB; ++u) ph[u] = tw[((m0 + u * MSTEP) * s) & (2 * N - 1)];
#pragma unroll
        for (int u = 0; u < MB; ++u) {
            const int m = m0 + u * MSTEP;
            if (m <= mtop) {
                const int j = m & (N - 1), jn = (N - j) & (N - 1);
                const double2 z = zs[j], y = zs[jn];
                const double2 Fa = make_double2(0.5 * (z.x + y.x), 0.5 * (z.y - y.y));
                const double2 Fb = make_double2(0.5 * (z.y + y.y), 0.5 * (y.x - z.x));
                if constexpr (sizeof(XT) == 8) {
                    *reinterpret_cast<double2*>(X + m * mrow) = cmul(ph[u], part ? Fb : Fa);
                } else {
                    store4<XT>(X + m * mrow, cmul(ph[u], Fa), cmul(ph[u], Fb));
                }
            }
        }
    }
}

template <int LOGN, typename XT>
__global__ __launch_bounds__(P2<LOGN>::NTH, 4) void k_fft_fwd_p2(FftArgs a, const FftItem* items, int nitems)
{
    extern __shared__ double2 lds[];
    const Item it = work_item(items, nitems, a.comp0);
    if (2 * it.pair0 >= a.nmaps) return;  // only padding map sets: nothing reads them
    fwd_item<LOGN, XT>(a, it, lds);
}

template <int LOGN, typename XT>
__device__ __forceinline__ void inv_item(const FftArgs& a, const Item it, double2* lds)
{
    using C = P2<LOGN>;
    constexpr int N = C::N, T = C::T, S = C::S;
    constexpr int MSTEP = C::NTH >> C::LOGS;  // = T
    const RingDev rg = a.rings[it.ring];
    const double2* tw = a.tw + a.lens[rg.len].tw;
    const int s = rg.s, lmax = min(a.lmax, rg.mcut);  // rows past the ring's cutoff are zero

    // Fold: C_j = sum_{m = j} c_m + sum_{m >= 1, -m = j} conj(c_m) of both maps,
    // Z = C^a + i C^b, into LDS in natural order.  Lanes run over (m, pair) so a
    // wave reads contiguous row segments of all S pairs.  d_m = c^a_m + i c^b_m is
    // the direct term, e_m = conj(c^a_m) + i conj(c^b_m) the mirror term.
    {
        const int sq = (int)threadIdx.x & (S - 1);
        const int mi = (int)threadIdx.x >> C::LOGS;
        double2* zs = lds + sq * C::SEQ;
        const XT* X = static_cast<const XT*>(a.X) + (int64_t)it.comp * a.xcomp + (int64_t)it.ring * a.ldx +
                      4 * (it.pair0 + sq);
        const int64_t mrow = (int64_t)a.nring * a.ldx;
        if (lmax < N) {
            // every bin has at most one direct and one mirror term: bins j = m
            // take d_m (zero beyond lmax), then bins N - m add e_m
            double2 e[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {  // m = mi + u T covers 0..N-1
                const int m = mi + u * MSTEP;
                double2 ta, tb;
                load4<XT>(X + min(m, lmax) * mrow, ta, tb);
                const double2 p = tw[(m * s) & (2 * N - 1)];
                const double2 ph = make_double2(p.x, -p.y);  // e^{+i m phi0}
                const double2 ca = cmul(ph, ta), cb = cmul(ph, tb);
                const bool live = m <= lmax && (!a.mown || a.mown[min(m, lmax)]);
                zs[m] = live ? make_double2(ca.x - cb.y, ca.y + cb.x) : make_double2(0.0, 0.0);
                e[u] = (live && m >= 1) ? make_double2(ca.x + cb.y, cb.x - ca.y) : make_double2(0.0, 0.0);
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int m = mi + u * MSTEP;
                if (m >= 1 && m <= lmax && (!a.mown || a.mown[m])) {
                    double2& z = zs[N - m];
                    z = make_double2(z.x + e[u].x, z.y + e[u].y);
                }
            }
        } else {
            // aliased rows (lmax >= N): several terms per bin, added atomically
            for (int e = (int)threadIdx.x; e < S * C::SEQ; e += C::NTH) lds[e] = make_double2(0.0, 0.0);
            __syncthreads();
            for (int m0 = mi; m0 <= lmax; m0 += MB * MSTEP) {
                double2 ta[MB], tb[MB], p[MB];
#pragma unroll
                for (int u = 0; u < MB; ++u) {
                    const int m = m0 + u * MSTEP;
                    load4<XT>(X + min(m, lmax) * mrow, ta[u], tb[u]);
                    p[u] = tw[(m * s) & (2 * N - 1)];
                }
#pragma unroll
                for (int u = 0; u < MB; ++u) {
                    const int m = m0 + u * MSTEP;
                    if (m <= lmax && (!a.mown || a.mown[m])) {
                        const double2 ph = make_double2(p[u].x, -p[u].y);
                        const double2 ca = cmul(ph, ta[u]), cb = cmul(ph, tb[u]);
                        double* z1 = reinterpret_cast<double*>(zs + (m & (N - 1)));
                        atomicAdd(z1, ca.x - cb.y);
                        atomicAdd(z1 + 1, ca.y + cb.x);
                        if (m >= 1) {
                            double* z2 = reinterpret_cast<double*>(zs + ((N - (m & (N - 1))) & (N - 1)));
                            atomicAdd(z2, ca.x + cb.y);
                            atomicAdd(z2 + 1, cb.x - ca.y);
                        }
                    }
                }
            }
        }
        __syncthreads();
    }

    // pass-0 inputs conj(Z_j) at bins j = tl + r T; the inverse DFT is conj(DFT(conj Z))
    const int seq = (int)threadIdx.x / T, tl = (int)threadIdx.x % T;
    double2* sb = lds + seq * C::SEQ;
    double2 v[8], w[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const double2 z = sb[tl + r * T];
        v[r] = make_double2(z.x, -z.y);
    }
    __syncthreads();  // pass 0 overwrites the buffer
    run_passes<LOGN, 0>(v, w, sb, tl, tw);

    // natural-order outputs: map k = Re, map k+1 = -Im (conjugate of the DFT)
    using QL = Pass<LOGN, C::NP - 1>;
    const int k = 2 * (it.pair0 + seq);
    const int64_t ms = (int64_t)a.ncomp * a.npix;
    double* oa = a.maps_out + (int64_t)it.comp * a.npix + rg.first + (int64_t)k * ms;
    if (k < a.nmaps) {
#pragma unroll
        for (int b = 0; b < QL::B; ++b) {
#pragma unroll
            for (int r = 0; r < QL::R; ++r) oa[tl + T * b + r * (N / QL::R)] = v[b * QL::R + r].x;
        }
    }
    if (k + 1 < a.nmaps) {
#pragma unroll
        for (int b = 0; b < QL::B; ++b) {
#pragma unroll
            for (int r = 0; r < QL::R; ++r) oa[ms + tl + T * b + r * (N / QL::R)] = -v[b * QL::R + r].y;
        }
    }
}

template <int LOGN, typename XT>
__global__ __launch_bounds__(P2<LOGN>::NTH, 4) void k_fft_inv_p2(FftArgs a, const FftItem* items, int nitems)
{
    extern __shared__ double2 lds[];
    const Item it = work_item(items, nitems, a.comp0);
    if (2 * it.pair0 >= a.nmaps) return;  // only padding map sets: nothing reads them
    inv_item<LOGN, XT>(a, it, lds);
}

template <int LOGM, typename XT>
__device__ __forceinline__ void fwd_item_blue(const FftArgs& a, const Item it, double2* lds)
{
    using C = P2<LOGM>;
    constexpr int T = C::T, S = C::S;
    const RingDev rg = a.rings[it.ring];
    const FftLen* L = a.lens + rg.len;
    const int n = rg.n;
    const double2* twn = a.tw + L->tw;      // e^{-i pi t/n}, t < 2n
    const double2* twM = a.tw + L->twm;     // e^{-i pi t/M}, t < 2M
    const double2* chirp = a.tw + L->chirp;
    const double2* bhat = a.bhat + L->bhat;
    const int seq = (int)threadIdx.x / T, tl = (int)threadIdx.x % T;
    double2* sb = lds + seq * C::SEQ;
    const int k = 2 * (it.pair0 + seq);

    double2 u[8];
    {
        const int64_t ms = (int64_t)a.ncomp * a.npix;
        const double* pa = a.maps_in + (int64_t)it.comp * a.npix + rg.first + min(k, a.nmaps - 1) * ms;
        const double* pb = a.maps_in + (int64_t)it.comp * a.npix + rg.first + min(k + 1, a.nmaps - 1) * ms;
        double2 c[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int i = min(tl + q * T, n - 1);
            u[q] = make_double2(pa[i], pb[i]);
            c[q] = chirp[i];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const bool live = tl + q * T < n;
            const double2 x = make_double2(k < a.nmaps ? u[q].x : 0.0, k + 1 < a.nmaps ? u[q].y : 0.0);
            u[q] = live ? cmul(x, c[q]) : make_double2(0.0, 0.0);
        }
    }
    blue_core<LOGM>(u, sb, tl, twM, bhat);

    // spectrum y_j = w_j u[k] (j = tl + k T < n) into LDS in natural order
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int j = tl + q * T;
        if (j < n) sb[j] = cmul(chirp[j], u[q]);
    }
    __syncthreads();

    blue_spectrum_out<LOGM, XT>(a, it, lds, rg, twn);
}

template <int LOGM, typename XT>
__device__ __forceinline__ void inv_item_blue(const FftArgs& a, const Item it, double2* lds)
{
    using C = P2<LOGM>;
    constexpr int T = C::T, S = C::S;
    const RingDev rg = a.rings[it.ring];
    const FftLen* L = a.lens + rg.len;
    const int n = rg.n;
    const double2* twn = a.tw + L->tw;
    const double2* twM = a.tw + L->twm;
    const double2* chirp = a.tw + L->chirp;
    const double2* bhat = a.bhat + L->bhat;

    blue_fold<LOGM, XT>(a, it, lds, rg, twn, S * C::SEQ);

    // Bluestein on conj(Z): pass-0 values conj(Z_i) w_i
    const int seq = (int)threadIdx.x / T, tl = (int)threadIdx.x % T;
    double2* sb = lds + seq * C::SEQ;
    double2 u[8];
    {
        double2 c[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) c[q] = chirp[min(tl + q * T, n - 1)];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int i = tl + q * T;
            u[q] = i < n ? cmul(sb[i], c[q]) : make_double2(0.0, 0.0);
        }
    }
    __syncthreads();  // pass 0 overwrites the buffer
    blue_core<LOGM>(u, sb, tl, twM, bhat);

    // pixels: y_j = w_j u[k] = DFT(conj Z)_j; map k = Re(conj y), map k+1 = Im(conj y)
    const int k = 2 * (it.pair0 + seq);
    const int64_t ms = (int64_t)a.ncomp * a.npix;
    double* oa = a.maps_out + (int64_t)it.comp * a.npix + rg.first + (int64_t)k * ms;
    double2 c[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) c[q] = chirp[min(tl + q * T, n - 1)];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int j = tl + q * T;
        const double2 y = cmul(c[q], u[q]);
        if (j < n) {
            if (k < a.nmaps) oa[j] = y.x;
            if (k + 1 < a.nmaps) oa[ms + j] = -y.y;
        }
    }
}

template <int LOGM, typename XT>
__global__ __launch_bounds__(P2<LOGM>::NTH, 4) void k_fft_fwd_blue(FftArgs a, const FftItem* items, int nitems)
{
    extern __shared__ double2 lds[];
    const Item it = work_item(items, nitems, a.comp0);
    if (2 * it.pair0 >= a.nmaps) return;  // only padding map sets: nothing reads them
    fwd_item_blue<LOGM, XT>(a, it, lds);
}

template <int LOGM, typename XT>
__global__ __launch_bounds__(P2<LOGM>::NTH, 4) void k_fft_inv_blue(FftArgs a, const FftItem* items, int nitems)
{
    extern __shared__ double2 lds[];
    const Item it = work_item(items, nitems, a.comp0);
    if (2 * it.pair0 >= a.nmaps) return;  // only padding map sets: nothing reads them
    inv_item_blue<LOGM, XT>(a, it, lds);
}

template <int LOGN, typename XT>
hipError_t launch_p2(bool fwd, const FftArgs& a, const FftClass& c, int ncompl, hipStream_t st)
{
    using C = P2<LOGN>;
    const dim3 grid(c.nitems * ncompl);
    if (C::LDS_BYTES > 65536) {
        const void* f = c.blue ? (fwd ? (const void*)k_fft_fwd_blue<LOGN, XT> : (const void*)k_fft_inv_blue<LOGN, XT>)
                               : (fwd ? (const void*)k_fft_fwd_p2<LOGN, XT> : (const void*)k_fft_inv_p2<LOGN, XT>);
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, C::LDS_BYTES);
        if (e != hipSuccess) return e;
    }
    if (c.blue) {
        if (fwd) hipLaunchKernelGGL((k_fft_fwd_blue<LOGN, XT>), grid, dim3(C::NTH), C::LDS_BYTES, st, a, c.items, c.nitems);
        else hipLaunchKernelGGL((k_fft_inv_blue<LOGN, XT>), grid, dim3(C::NTH), C::LDS_BYTES, st, a, c.items, c.nitems);
    } else {
        if (fwd) hipLaunchKernelGGL((k_fft_fwd_p2<LOGN, XT>), grid, dim3(C::NTH), C::LDS_BYTES, st, a, c.items, c.nitems);
        else hipLaunchKernelGGL((k_fft_inv_p2<LOGN, XT>), grid, dim3(C::NTH), C::LDS_BYTES, st, a, c.items, c.nitems);
    }
    return hipGetLastError();
}

template <typename XT>
hipError_t launch_p2_x(bool fwd, const FftArgs& a, const FftClass& c, int ncompl, hipStream_t st)
{
    switch (c.p2) {
        case 6: return launch_p2<6, XT>(fwd, a, c, ncompl, st);
        case 7: return launch_p2<7, XT>(fwd, a, c, ncompl, st);
        case 8: return launch_p2<8, XT>(fwd, a, c, ncompl, st);
        case 9: return launch_p2<9, XT>(fwd, a, c, ncompl, st);
        case 10: return launch_p2<10, XT>(fwd, a, c, ncompl, st);
        case 11: return launch_p2<11, XT>(fwd, a, c, ncompl, st);
        case 12: return launch_p2<12, XT>(fwd, a, c, ncompl, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

int p2_seqs_per_group(int logn)
{
    switch (logn) {
        case 6: return P2<6>::S;
        case 7: return P2<7>::S;
        case 8: return P2<8>::S;
        case 9: return P2<9>::S;
        case 10: return P2<10>::S;
        case 11: return P2<11>::S;
        case 12: return P2<12>::S;
        default: return 0;
    }
}

hipError_t launch_fft_p2(bool forward, const FftArgs& a, const FftClass& c, int ncompl, hipStream_t st)
{
    if (c.nitems <= 0) return hipSuccess;
    return a.x32 ? launch_p2_x<float>(forward, a, c, ncompl, st) : launch_p2_x<double>(forward, a, c, ncompl, st);
}

}  // namespace sht
