// Internal types of the ring FFT stage (plan tables, argument blocks, launch
// wrappers), shared by the host plan code and the FFT / iteration kernels.
#pragma once
#include "sht_internal.h"

namespace sht {

// ----------------------------------------------------------------------------
// FFT tables
// ----------------------------------------------------------------------------
constexpr int MAX_STAGES = 16;
struct FftLen {
    int n;                  // ring length
    int blue;               // 1: Bluestein through length m
    int m;                  // Bluestein FFT length (0 if none)
    int nstage;             // stages of the FFT actually run (length n or m)
    int radix[MAX_STAGES];
    int64_t tw;             // offset of e^{-i pi j / n}, j < 2n
    int64_t twm;            // offset of e^{-i pi j / m}, j < 2m (Bluestein)
    int64_t bhat;           // offset of the Bluestein kernel spectrum (m entries, scaled by 1/m)
    int64_t chirp;          // offset of the Bluestein chirp e^{-i pi j^2 / n}, j < n (in the twiddle pool)
    int nseq;               // map pairs per workgroup (a power of two)
    int lgseq;              // log2(nseq)
    int ldsc;               // complex values per workgroup = nseq * (blue ? m : n)
    int lstride;            // LDS stride between sequences: >= len + len/16, = 16/nseq mod 16 (see k_fft.hip)
    int lds;                // complex LDS slots per workgroup = nseq * lstride
    int p2;                 // log2(n) when n is a power of two handled by k_fft_p2.hip, else 0
    int bp2;                // log2(m) when a Bluestein length m = 2^bp2 is handled by k_fft_p2.hip, else 0
    int four;               // 1: n = 4j, four Bluestein DFTs of length j and a radix-4 step (Bluestein of
                            // length n would need a convolution beyond the LDS); k_fft_four.hip
    int sub;                // four: index of the length-j Bluestein entry (chirp, kernel spectrum, twiddles)
};

struct FftItem {
    int ring;
    int pair0;
};

// ----------------------------------------------------------------------------
// Kernel argument block
// ----------------------------------------------------------------------------
struct FftArgs {
    const RingDev* rings;
    const FftLen* lens;
    const FftItem* items;
    const double2* tw;      // twiddle pool
    const double2* bhat;    // Bluestein spectra pool
    const double* maps_in;  // forward: maps of the chunk (component stride npix, map-set stride ncomp*npix)
    double* maps_out;       // inverse: output maps
    void* X;                // ring Fourier coefficients, [m][ring][ldx] (double or float)
    double* F;              // optional halfcomplex spectra [map-set][comp][npix] (iteration data)
    double* norms;          // optional per map-set/comp residual sum of squares (K_RES)
    int64_t npix;
    int ncomp;
    int comp0;              // first component index handled by this launch (blockIdx.y adds to it)
    int nmaps;              // map sets in the chunk
    int npairs;             // padded map-set pairs (ldx / 4)
    int lmax;
    int nring;
    int64_t ldx;            // columns of X (2 * padded map sets)
    int64_t xcomp;          // element stride between the X arrays of consecutive components
    int x32;                // X stored as float
    int iteration_sub;      // K_RES: subtract N*C from F into X
    int store_res;          // K_RES: write the residual spectra to R
    // immediate iteration: residual spectra, halfcomplex per ring, bin-major with the
    // maps of the chunk contiguous: R[(comp * npix + pixel slot) * nmaps + map]
    double* R;
    // optional 0/1 per m (lmax + 1 entries): the inverse transforms fold only the
    // rows of m marked 1 (a plan that owns a subset of the m)
    const unsigned char* mown;
};

// ----------------------------------------------------------------------------
// Launch wrappers (defined in the .hip files)
// ----------------------------------------------------------------------------
// FFT work is launched per LDS class so that small rings are not held to the
// occupancy of the largest ones.  Workgroups have FFT_THREADS threads;
// elems = complex values per thread per FFT stage (lds / FFT_THREADS).
constexpr int FFT_THREADS = 512;
struct FftClass {
    const FftItem* items;
    int nitems;
    int lds;     // complex LDS elements per workgroup
    int elems;   // 2, 8 or 16
    int p2;      // 0: runtime-length kernels; else log2 of the (convolution) length (k_fft_p2.hip)
    int blue;    // with p2: Bluestein rings through a power-of-two convolution
    int four;    // rings of FftLen::four, one map pair per workgroup
};
// power-of-two ring lengths 2^6 .. 2^12: map pairs per workgroup (0: not handled)
int p2_seqs_per_group(int logn);
hipError_t launch_fft_p2(bool forward, const FftArgs& a, const FftClass& c, int ncompl, hipStream_t st);
// the four-step class (FftLen::four): forward and inverse only
hipError_t launch_fft_four(bool forward, const FftArgs& a, const FftClass& c, int ncompl, hipStream_t st);
hipError_t launch_fft_forward(const FftArgs& a, const FftClass* cls, int ncls, int ncompl, hipStream_t st);
hipError_t launch_fft_inverse(const FftArgs& a, const FftClass* cls, int ncls, int ncompl, hipStream_t st);
hipError_t launch_residual(const FftArgs& a, const FftClass* cls, int ncls, int ncompl, hipStream_t st);
hipError_t launch_bluestein_init(const FftLen* lens, const int* blue_lens, int nblue, const double2* tw,
                                 double2* bhat, int lds, hipStream_t st);

// immediate iteration, Fourier side (k_iter.hip), on the residual spectra
// FftArgs::R; cmin[m] is the first ring chunk
// where some Legendre value of m is significant (rings before it carry no data for m).
hipError_t launch_level_unfold(const FftArgs& a, const int* mlist, int nlist, const int* cmin, int ncompl, hipStream_t st);
hipError_t launch_level_fold(const FftArgs& a, const int* mlist, int nlist, const int* cmin, int ncompl, hipStream_t st);
hipError_t launch_hc_norms(const FftArgs& a, int ncompl, hipStream_t st);
// zero the ring coefficient rows of the listed m, every ring and column
hipError_t launch_level_zero(const FftArgs& a, const int* mlist, int nlist, int ncompl, hipStream_t st);

}  // namespace sht
