// Four-step ring FFTs (HIP, gfx950) for the rings whose Bluestein convolution
// would not fit the LDS: n = 4j pixels, four Bluestein DFTs of length j through
// 4096 points on the compile-time passes of fft_p2.h and one radix-4 step.  In a
// translation unit of their own, so that these kernels, which hold 16 spectrum
// values per thread at two waves per SIMD, do not move the register allocation
// of the power-of-two and Bluestein kernels.
#include <algorithm>

#include "fft_p2.h"

namespace sht {
namespace {

// ----------------------------------------------------------------------------
// Rings of n = 4j pixels whose Bluestein convolution would not fit the LDS (the
// polar rings longer than 4096 pixels without a 7-smooth length, nside >= 2048).
// Decimation in time splits the length-n DFT into the four length-j DFTs of the
// pixels 4s + r, each taken by Bluestein through 4096 points (j <= 2047) with the
// compile-time passes of fft_p2.h, and one radix-4 step:
//   Z[k1 + j k2] = sum_r e^{-2 pi i r k1 / n} (-i)^{r k2} Y_r[k1].
// One map pair per workgroup of 512 threads; thread tl keeps the outputs of
// k1 = tl + 512 q (q < 4) for the four k2 in registers while the LDS holds the
// Bluestein buffer, so the LDS never needs more than max(4608, n) values.
// ----------------------------------------------------------------------------
constexpr int FOUR_Q = 4;  // k1 values per thread (j < 4 x 512)

// z[q][k2] += e^{-2 pi i r k1 / n} (-i)^{r k2} Y_r[k1] for k1 = tl + 512 q < j, with
// Y_r[k1] = w_{k1} u[q] the result of blue_core on the r-th decimated sequence
__device__ __forceinline__ void four_accumulate(double2 (&z)[FOUR_Q][4], const double2 (&u)[8], int r, int tl,
                                                int j, int n, const double2* chirp, const double2* twn)
{
    constexpr int T = P2<12>::T;
#pragma unroll
    for (int q = 0; q < FOUR_Q; ++q) {
        const int k1 = tl + q * T;
        if (k1 < j) {
            const double2 y = cmul(chirp[k1], u[q]);
            const double2 t = cmul(twn[(2 * r * k1) % (2 * n)], y);  // e^{-i pi t / n} at t = 2 r k1
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) {
                const int pw = (r * k2) & 3;  // (-i)^pw
                const double2 v = pw == 0   ? t
                                  : pw == 1 ? make_double2(t.y, -t.x)
                                  : pw == 2 ? make_double2(-t.x, -t.y)
                                            : make_double2(-t.y, t.x);
                z[q][k2] = cadd(z[q][k2], v);
            }
        }
    }
}

template <typename XT>
__device__ __forceinline__ void fwd_item_four(const FftArgs& a, const Item it, double2* lds)
{
    constexpr int T = P2<12>::T;
    const RingDev rg = a.rings[it.ring];
    const FftLen* L = a.lens + rg.len;
    const FftLen* LJ = a.lens + L->sub;  // Bluestein data of length j
    const int n = rg.n, j = n >> 2;
    const double2* twn = a.tw + L->tw;
    const double2* twM = a.tw + LJ->twm;
    const double2* chirp = a.tw + LJ->chirp;
    const double2* bhat = a.bhat + LJ->bhat;
    const int tl = (int)threadIdx.x;
    const int k = 2 * it.pair0;
    const int64_t ms = (int64_t)a.ncomp * a.npix;
    const double* pa = a.maps_in + (int64_t)it.comp * a.npix + rg.first + min(k, a.nmaps - 1) * ms;
    const double* pb = a.maps_in + (int64_t)it.comp * a.npix + rg.first + min(k + 1, a.nmaps - 1) * ms;

    double2 z[FOUR_Q][4];
#pragma unroll
    for (int q = 0; q < FOUR_Q; ++q)
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) z[q][k2] = make_double2(0.0, 0.0);
    for (int r = 0; r < 4; ++r) {
        // pass-0 values x_s w_s of the sequence x_s = z_{4s + r}, s = tl + 512 q < j
        double2 u[8], c[FOUR_Q];
#pragma unroll
        for (int q = 0; q < FOUR_Q; ++q) {
            const int sq = min(tl + q * T, j - 1);
            u[q] = make_double2(pa[4 * sq + r], pb[4 * sq + r]);
            c[q] = chirp[sq];
        }
#pragma unroll
        for (int q = 0; q < FOUR_Q; ++q) {
            const double2 x = make_double2(k < a.nmaps ? u[q].x : 0.0, k + 1 < a.nmaps ? u[q].y : 0.0);
            u[q] = tl + q * T < j ? cmul(x, c[q]) : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int q = FOUR_Q; q < 8; ++q) u[q] = make_double2(0.0, 0.0);
        blue_core<12>(u, lds, tl, twM, bhat);
        four_accumulate(z, u, r, tl, j, n, chirp, twn);
        __syncthreads();  // the next sequence's first pass overwrites the buffer
    }
    // spectrum Z in natural order into LDS, then the output of k_fft_fwd_blue
#pragma unroll
    for (int q = 0; q < FOUR_Q; ++q) {
        const int k1 = tl + q * T;
        if (k1 < j) {
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) lds[k1 + j * k2] = z[q][k2];
        }
    }
    __syncthreads();
    blue_spectrum_out<12, XT>(a, it, lds, rg, twn);
}

template <typename XT>
__device__ __forceinline__ void inv_item_four(const FftArgs& a, const Item it, double2* lds)
{
    constexpr int T = P2<12>::T;
    const RingDev rg = a.rings[it.ring];
    const FftLen* L = a.lens + rg.len;
    const FftLen* LJ = a.lens + L->sub;
    const int n = rg.n, j = n >> 2;
    const double2* twn = a.tw + L->tw;
    const double2* twM = a.tw + LJ->twm;
    const double2* chirp = a.tw + LJ->chirp;
    const double2* bhat = a.bhat + LJ->bhat;
    const int tl = (int)threadIdx.x;

    // conj(Z) in LDS, then the four decimated sequences into registers (the
    // inverse DFT is conj(DFT(conj Z)))
    blue_fold<12, XT>(a, it, lds, rg, twn, n);
    double2 x[FOUR_Q][4];
#pragma unroll
    for (int q = 0; q < FOUR_Q; ++q) {
        const int sq = min(tl + q * T, j - 1);
#pragma unroll
        for (int r = 0; r < 4; ++r) x[q][r] = lds[4 * sq + r];
    }
    __syncthreads();  // the LDS becomes the Bluestein buffer

    double2 z[FOUR_Q][4];
#pragma unroll
    for (int q = 0; q < FOUR_Q; ++q)
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) z[q][k2] = make_double2(0.0, 0.0);
    for (int r = 0; r < 4; ++r) {
        // sequence r sits in x[.][0]: the registers rotate after each sequence (a
        // register array indexed by the loop counter would live in scratch memory)
        double2 u[8];
#pragma unroll
        for (int q = 0; q < FOUR_Q; ++q) {
            const int sq = min(tl + q * T, j - 1);
            u[q] = tl + q * T < j ? cmul(x[q][0], chirp[sq]) : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int q = FOUR_Q; q < 8; ++q) u[q] = make_double2(0.0, 0.0);
#pragma unroll
        for (int q = 0; q < FOUR_Q; ++q) {
            x[q][0] = x[q][1];
            x[q][1] = x[q][2];
            x[q][2] = x[q][3];
        }
        blue_core<12>(u, lds, tl, twM, bhat);
        four_accumulate(z, u, r, tl, j, n, chirp, twn);
        __syncthreads();
    }
    // pixels k1 + j k2: y = DFT(conj Z); map k = Re y, map k+1 = -Im y
    const int k = 2 * it.pair0;
    const int64_t ms = (int64_t)a.ncomp * a.npix;
    double* oa = a.maps_out + (int64_t)it.comp * a.npix + rg.first + (int64_t)k * ms;
#pragma unroll
    for (int q = 0; q < FOUR_Q; ++q) {
        const int k1 = tl + q * T;
        if (k1 < j) {
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) {
                if (k < a.nmaps) oa[k1 + j * k2] = z[q][k2].x;
                if (k + 1 < a.nmaps) oa[ms + k1 + j * k2] = -z[q][k2].y;
            }
        }
    }
}

template <typename XT>
__global__ __launch_bounds__(P2<12>::T, 2) void k_fft_fwd_four(FftArgs a, const FftItem* items, int nitems)
{
    extern __shared__ double2 lds[];
    const Item it = work_item(items, nitems, a.comp0);
    if (2 * it.pair0 >= a.nmaps) return;  // only padding map sets: nothing reads them
    fwd_item_four<XT>(a, it, lds);
}

template <typename XT>
__global__ __launch_bounds__(P2<12>::T, 2) void k_fft_inv_four(FftArgs a, const FftItem* items, int nitems)
{
    extern __shared__ double2 lds[];
    const Item it = work_item(items, nitems, a.comp0);
    if (2 * it.pair0 >= a.nmaps) return;
    inv_item_four<XT>(a, it, lds);
}

template <typename XT>
hipError_t launch_four_x(bool fwd, const FftArgs& a, const FftClass& c, int ncompl, hipStream_t st)
{
    const dim3 grid(c.nitems * ncompl);
    const size_t sh = (size_t)std::max(c.lds, P2<12>::SEQ) * sizeof(double2);
    const void* f = fwd ? (const void*)k_fft_fwd_four<XT> : (const void*)k_fft_inv_four<XT>;
    if (sh > 65536) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
        if (e != hipSuccess) return e;
    }
    if (fwd) hipLaunchKernelGGL((k_fft_fwd_four<XT>), grid, dim3(P2<12>::T), sh, st, a, c.items, c.nitems);
    else hipLaunchKernelGGL((k_fft_inv_four<XT>), grid, dim3(P2<12>::T), sh, st, a, c.items, c.nitems);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_fft_four(bool forward, const FftArgs& a, const FftClass& c, int ncompl, hipStream_t st)
{
    if (c.nitems <= 0) return hipSuccess;
    return a.x32 ? launch_four_x<float>(forward, a, c, ncompl, st) : launch_four_x<double>(forward, a, c, ncompl, st);
}


}  // namespace sht
