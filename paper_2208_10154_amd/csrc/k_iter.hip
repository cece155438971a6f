// Fourier-side kernels of the immediate iteration (Sec. 4, Algorithm 3), HIP for
// gfx950.
//
// The immediate mode updates the coefficients of each m inside the m-loop, so
// every later m works on a residual that already holds those updates.  The
// residual is kept as ring spectra R (halfcomplex per ring as the forward ring
// FFT stores spectra, bin-major with the maps of the chunk contiguous, so a wave
// touches one bin of 64 maps in one run), R = F - n C with C the folded ring
// coefficients of the current synthesis:
//   unfold:  T_m(ring) = e^{-i m phi0} R_{m mod n}      (the map2alm input of m)
//   fold:    R_{m mod n} -= n e^{i m phi0} dS_m,  R_{-m mod n} -= n conj(...)
// with dS_m the synthesis of the update of m on that ring.  Modes processed
// together (one level of the schedule) never share a bin of a ring on which
// both carry data, so each thread owns the bins it updates.
#include "fft_internal.h"

namespace sht {
namespace {

constexpr int NT = 256;
constexpr int RB = NT / 64;  // rings per workgroup in the level kernels: one wave per ring, 64 maps

// halfcomplex position of Re / Im of bin j (j and n - j share one slot; Im is
// -1 where it is identically zero), as the ring FFT stores the spectra
__device__ __forceinline__ int hre(int n, int j)
{
    const int h = (2 * j > n) ? n - j : j;
    return h == 0 ? 0 : (2 * h == n ? n - 1 : 2 * h - 1);
}
__device__ __forceinline__ int him(int n, int j)
{
    const int h = (2 * j > n) ? n - j : j;
    return (h == 0 || 2 * h == n) ? -1 : 2 * h;
}

struct LevelItem {
    int m, ring, comp, k;  // k: map of the thread
    bool live;             // ring carries data for m
};

// grid: x = list entry * ring groups + group of RB rings, y = component,
// z = block of 64 maps; wave w of the workgroup takes ring RB * group + w
__device__ __forceinline__ int ring_groups(int nring) { return (nring + RB - 1) / RB; }

__device__ __forceinline__ LevelItem level_item(const FftArgs& a, const int* mlist, const int* cmin)
{
    LevelItem it;
    const int ng = ring_groups(a.nring);
    const int i = blockIdx.x / ng;
    it.ring = (blockIdx.x - i * ng) * RB + (int)(threadIdx.x >> 6);
    it.m = mlist[i];
    it.comp = a.comp0 + blockIdx.y;
    it.k = blockIdx.z * 64 + (int)(threadIdx.x & 63);
    const int rn = min(it.ring, a.nring - 1 - it.ring);
    it.live = it.ring < a.nring && rn / RCHUNK >= cmin[it.m];
    return it;
}

// e^{-i m phi0} with phi0 = pi s / n (first pixel of the ring)
__device__ __forceinline__ void phase(int m, int s, int n, double& c, double& sn)
{
    const int t = (int)(((int64_t)m * s) % (2 * n));
    sincospi((double)t / (double)n, &sn, &c);
    sn = -sn;
}

template <typename XT>
__global__ __launch_bounds__(NT) void k_level_unfold(FftArgs a, const int* mlist, const int* cmin)
{
    const LevelItem it = level_item(a, mlist, cmin);
    if (!it.live || 2 * it.k >= a.ldx) return;
    XT* X = static_cast<XT*>(a.X) + (int64_t)it.comp * a.xcomp + ((int64_t)it.m * a.nring + it.ring) * a.ldx + 2 * it.k;
    double tr = 0.0, ti = 0.0;
    if (it.k < a.nmaps) {
        const RingDev rg = a.rings[it.ring];
        const int n = rg.n, j = it.m % n;
        const double* R = a.R + ((int64_t)it.comp * a.npix + rg.first) * a.nmaps + it.k;
        const double re = R[(int64_t)hre(n, j) * a.nmaps];
        const int pi = him(n, j);
        const double im = pi < 0 ? 0.0 : (2 * j > n ? -R[(int64_t)pi * a.nmaps] : R[(int64_t)pi * a.nmaps]);
        double c, s;
        phase(it.m, rg.s, n, c, s);
        tr = c * re - s * im;
        ti = c * im + s * re;
    }
    X[0] = (XT)tr;
    X[1] = (XT)ti;
}

template <typename XT>
__global__ __launch_bounds__(NT) void k_level_fold(FftArgs a, const int* mlist, const int* cmin)
{
    const LevelItem it = level_item(a, mlist, cmin);
    if (!it.live || it.k >= a.nmaps) return;
    const XT* X = static_cast<const XT*>(a.X) + (int64_t)it.comp * a.xcomp + ((int64_t)it.m * a.nring + it.ring) * a.ldx +
                  2 * it.k;
    const double dr = (double)X[0], di = (double)X[1];
    const RingDev rg = a.rings[it.ring];
    const int n = rg.n, j = it.m % n;
    double c, s;
    phase(it.m, rg.s, n, c, s);  // e^{-i m phi0}; the fold takes its conjugate
    const double cr = c * dr + s * di, ci = c * di - s * dr;
    const double dn = (double)n;
    double* R = a.R + ((int64_t)it.comp * a.npix + rg.first) * a.nmaps + it.k;
    if (j == 0 || 2 * j == n) {
        // the direct and the mirror term meet in a real bin (only c_0 itself at m = 0)
        R[(int64_t)hre(n, j) * a.nmaps] -= (it.m == 0 ? 1.0 : 2.0) * dn * cr;
    } else {
        R[(int64_t)hre(n, j) * a.nmaps] -= dn * cr;
        R[(int64_t)him(n, j) * a.nmaps] -= (2 * j > n ? -dn : dn) * ci;
    }
}

// clear the X rows of the listed m before a split alm2map adds into them
template <typename XT>
__global__ __launch_bounds__(NT) void k_level_zero(FftArgs a, const int* mlist)
{
    const int ng = ring_groups(a.nring);
    const int i = blockIdx.x / ng;
    const int ring = (blockIdx.x - i * ng) * RB + (int)(threadIdx.x >> 6);
    const int k = blockIdx.z * 64 + (int)(threadIdx.x & 63);
    if (ring >= a.nring || 2 * k >= a.ldx) return;
    XT* X = static_cast<XT*>(a.X) + (int64_t)(a.comp0 + blockIdx.y) * a.xcomp +
            ((int64_t)mlist[i] * a.nring + ring) * a.ldx + 2 * k;
    X[0] = XT(0);
    X[1] = XT(0);
}

// sum over the ring of |r|^2 = (1/n) sum_j |R_j|^2 from the halfcomplex spectra
// (bins 0 and n/2 once, the others twice), per map and component.  Lanes run
// over maps, the waves over the ring's slots.
// grid: x = ring, y = component, z = block of 64 maps
__global__ __launch_bounds__(NT) void k_hc_norms(FftArgs a)
{
    __shared__ double part[RB][64];
    const RingDev rg = a.rings[blockIdx.x];
    const int comp = a.comp0 + blockIdx.y, n = rg.n;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int k = blockIdx.z * 64 + lane;
    double acc = 0.0;
    if (k < a.nmaps) {
        const double* R = a.R + ((int64_t)comp * a.npix + rg.first) * a.nmaps + k;
        for (int p = wave; p < n; p += RB) {
            const double v = R[(int64_t)p * a.nmaps];
            acc += (p == 0 || p == n - 1 ? 1.0 : 2.0) * v * v;
        }
    }
    part[wave][lane] = acc;
    __syncthreads();
    if (wave == 0 && k < a.nmaps) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < RB; ++w) t += part[w][lane];
        atomicAdd(a.norms + (int64_t)k * a.ncomp + comp, t / (double)n);
    }
}

dim3 level_grid(const FftArgs& a, int nlist, int ncompl)
{
    return dim3((unsigned)(nlist * ((a.nring + RB - 1) / RB)), (unsigned)ncompl, (unsigned)((a.ldx / 2 + 63) / 64));
}

}  // namespace

hipError_t launch_level_unfold(const FftArgs& a, const int* mlist, int nlist, const int* cmin, int ncompl, hipStream_t st)
{
    if (nlist <= 0) return hipSuccess;
    if (a.x32) hipLaunchKernelGGL(k_level_unfold<float>, level_grid(a, nlist, ncompl), dim3(NT), 0, st, a, mlist, cmin);
    else hipLaunchKernelGGL(k_level_unfold<double>, level_grid(a, nlist, ncompl), dim3(NT), 0, st, a, mlist, cmin);
    return hipGetLastError();
}

hipError_t launch_level_fold(const FftArgs& a, const int* mlist, int nlist, const int* cmin, int ncompl, hipStream_t st)
{
    if (nlist <= 0) return hipSuccess;
    if (a.x32) hipLaunchKernelGGL(k_level_fold<float>, level_grid(a, nlist, ncompl), dim3(NT), 0, st, a, mlist, cmin);
    else hipLaunchKernelGGL(k_level_fold<double>, level_grid(a, nlist, ncompl), dim3(NT), 0, st, a, mlist, cmin);
    return hipGetLastError();
}

hipError_t launch_level_zero(const FftArgs& a, const int* mlist, int nlist, int ncompl, hipStream_t st)
{
    if (nlist <= 0) return hipSuccess;
    if (a.x32) hipLaunchKernelGGL(k_level_zero<float>, level_grid(a, nlist, ncompl), dim3(NT), 0, st, a, mlist);
    else hipLaunchKernelGGL(k_level_zero<double>, level_grid(a, nlist, ncompl), dim3(NT), 0, st, a, mlist);
    return hipGetLastError();
}

hipError_t launch_hc_norms(const FftArgs& a, int ncompl, hipStream_t st)
{
    hipLaunchKernelGGL(k_hc_norms, dim3((unsigned)a.nring, (unsigned)ncompl, (unsigned)((a.nmaps + 63) / 64)), dim3(NT), 0,
                       st, a);
    return hipGetLastError();
}

}  // namespace sht
