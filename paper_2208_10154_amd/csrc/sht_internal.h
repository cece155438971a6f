// Internal types shared by the host plan code and the HIP kernels of libsht.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace sht {

// ----------------------------------------------------------------------------
// Scaled representation of Legendre values: true value = mu * 2^(-SCALE_BITS*k).
// k >= 1 means |true| < 2^SIG_LOG2, which is treated as exactly zero when the
// value is fed to the contraction (ring skipping, the safe starting positions
// and underflow handling in one rule).  The threshold is the paper's example
// for the safe positions (Sec. 3.1: amplitudes above about 1e-20; 2^-67 is
// 6.8e-21): a dropped value is below 1e-16 of FP64 resolution at O(1) peaks.
// ----------------------------------------------------------------------------
constexpr int SCALE_BITS = 600;
constexpr double SCALE_DOWN = 0x1p-600;   // 2^-SCALE_BITS
constexpr int SIG_LOG2 = -67;             // values below 2^SIG_LOG2 count as zero
constexpr double RESCALE_AT = 0x1p533;    // 2^(SIG_LOG2 + SCALE_BITS): rescale when |mu| exceeds this and k >= 1

// Legendre tiling: l segments of SEG values start at lb(m) + SEG*j (one stored
// seed pair each, so SEG rows of one ring can be generated independently);
// contraction tiles cover TL = SPT * SEG values of l.
constexpr int SEG = 8;
constexpr int TL = 64;
constexpr int SPT = TL / SEG;  // segments per tile
constexpr int RCHUNK = 32;   // ring granularity of the skip table

// ----------------------------------------------------------------------------
// Split-BF16 operands: x (rounded to FP32) = hi + mid + lo with hi = bf16(x),
// mid = bf16(x - hi), lo = bf16(x - hi - mid): three bfloat16 numbers carry the
// 24 significant bits of the FP32 value.  Stored as one 64-bit word, hi in bits
// 0-15, mid in 16-31, lo in 32-47.  The layout kernel writes the coefficient rows
// of the split-BF16 alm2map contraction in this form, so that kernel only
// regroups halves instead of splitting every operand in every tile.
// ----------------------------------------------------------------------------
__device__ __forceinline__ uint64_t pack_bf16_triple(float x)
{
    const __bf16 h = (__bf16)x;
    const float r = x - (float)h;
    const __bf16 m = (__bf16)r;
    const __bf16 l = (__bf16)(r - (float)m);
    const uint32_t w0 = (uint32_t)__builtin_bit_cast(unsigned short, h) | ((uint32_t)__builtin_bit_cast(unsigned short, m) << 16);
    return (uint64_t)w0 | ((uint64_t)__builtin_bit_cast(unsigned short, l) << 32);
}

// ----------------------------------------------------------------------------
// Rings
// ----------------------------------------------------------------------------
struct RingDev {
    double z;               // cos(theta)
    double omz;             // 1 - |z| from the exact rational: near the poles z rounded to FP64
                            // loses the relative precision of 1 - z that the recursion needs
    double sth;             // sin(theta)
    int64_t first;          // first pixel
    int n;                  // pixels
    int s;                  // phase shift: first pixel at phi = pi s / n
    int len;                // index into FftLen table
    int mcut;               // highest m whose Legendre rows on this ring are not all
                            // negligible (ring skip table); the FFT mapping stops there
};

// ----------------------------------------------------------------------------
// Kernel argument blocks
// ----------------------------------------------------------------------------
struct LegArgs {
    const RingDev* rings;   // all rings; north ring r (0-based) is rings[r]
    // seeds: for (m, segment j, north ring r): index seedoff[m] + j*rn + r
    const double* mu;       // spin 0: 2 values (l, l+1); spin 2: 4 values (P_l, P_l+1, M_l, M_l+1), SoA
    const int* kk;          // exponent counter k at the segment start
    const int64_t* seedoff;
    int64_t seedstride;     // distance between SoA arrays of mu
    const int* lsig;        // [m][ring chunk of RCHUNK]: first l with a significant value (or lmax+1)
    int nrc;                // ring chunks of RCHUNK per m
    // map2alm work list: l tiles of the m in folded order (see mfold), prefix sums:
    // tiles[i] = l tiles of mfold(0..i-1) (lmax+2 entries)
    const int* tiles;
    int ntiles;             // map2alm: total l tiles (tiles[lmax+1])
    void* X;                // [m][ring][ldx], component arrays xcomp apart (T | Q | U)
    int64_t xcomp;
    void* A;                // m-major coefficients [rowoff[m] + l - lb(m)][ldx], arrays acomp apart (T | E | iB)
    int64_t acomp;
    const int64_t* rowoff;  // first row of each m in A for this spin
    // recursion coefficients per (m, l), row rowoff[m] + l - lb(m): spin 0 {a, ab}
    // (2 doubles a row), spin 2 {alpha, beta, gamma, 0} (4 doubles); TL zero rows
    // follow the last m so that a segment may run past lmax
    const double* coef;
    int64_t ldx;            // columns of X and A (2 * padded map sets, multiple of 64)
    int lmax, rn, nring, spin;
    int ctiles;             // column tiles
    int eb;                 // spin-2 alm2map: 0 E and B, 1 E only, 2 B only (the other block skipped)
    // optional list of m values to transform instead of all m (immediate-mode
    // iteration); tiles then holds the prefix sums over the list entries and
    // ntiles their total
    const int* mlist;
    int nlist;
    // > 1: each workgroup's reduction range (map2alm: ring chunks, alm2map: l
    // tiles) is split over ksplit workgroups that add into pre-zeroed outputs
    // (list mode, where one level's grid is too small to fill the chip)
    int ksplit;
    int ncols;              // columns holding map sets in this chunk (2 per map set); the rest pad
};

// Narrow tiles: a chunk of at most 8 map sets (16 columns, inside one 64-column
// tile) runs Legendre kernels whose four waves split the tile's output blocks
// instead of its columns, so a small batch is not charged for the 24 padding map
// sets of the tile.
__host__ __device__ inline bool narrow(const LegArgs& a) { return a.ldx == 64 && a.ncols > 0 && a.ncols <= 16; }

// Layout change compact alm <-> m-major rows (one spin's components per launch).
struct AlmArgs {
    const double* alm_in;   // compact alm of the chunk (to m-major)
    double* alm_out;        // compact alm of the chunk (from m-major)
    void* A;                // rows the map2alm contraction writes (double or float)
    void* Aop;              // rows the alm2map contraction reads: A itself, except for
                            // split BF16, whose 64-bit words sit in a region of their own
    int64_t acomp;
    const int64_t* rowoff;
    const int* tileoff;     // l tiles of 64 per m for this spin
    int ntiles;
    int kblocks;            // blocks of 32 map sets (ldx / 64)
    int64_t ldx;
    int64_t almstride;      // doubles between consecutive map sets
    int lmax, spin, nmaps;
    int comp0;              // first component of the launch (blockIdx.y adds)
    double scale;           // from m-major: alm = scale * A
    int accumulate;         // from m-major: alm += scale * A
    const int* mlist;       // optional m list (tileoff then over the list entries, ntiles its total)
    int nlist;
};
hipError_t launch_alm_to_mmajor(const AlmArgs& a, int ncompl, int prec, hipStream_t st);
hipError_t launch_alm_from_mmajor(const AlmArgs& a, int ncompl, int prec, hipStream_t st);
// base[i*stride + j] = 0 for i < rows, j < len
hipError_t launch_zero_strided(double* base, int rows, int64_t stride, int64_t len, hipStream_t st);
// immediate iteration: A rows of the listed m (m2a output) -> scale * rows, in
// place, with the parts the compact storage lacks (m = 0) zeroed; scale = 0
// clears them (before a split map2alm adds into them)
hipError_t launch_level_rows(const AlmArgs& a, int ncompl, int prec, hipStream_t st);
// immediate iteration: alm += scale * rows (as launch_alm_from_mmajor with
// accumulate) and scale * rows written as the alm2map operand (Aop, m = 0 parts
// without a compact slot zeroed), in one pass
hipError_t launch_level_commit(const AlmArgs& a, int ncompl, int prec, hipStream_t st);


// Folded m order 0, lmax, 1, lmax-1, ...: work per m falls linearly with m, so any
// run of consecutive folded indices carries about the same work per index.  Each
// XCD takes a contiguous run of workgroups, which keeps the XCDs balanced while
// the workgroups of one m stay on one XCD (and its L2).
__host__ __device__ inline int mfold(int i, int lmax) { return (i & 1) ? lmax - (i >> 1) : (i >> 1); }

// first l of the recursion for (spin, m)
__host__ __device__ inline int lbase(int spin, int m) { return spin == 2 ? (m > 2 ? m : 2) : m; }
__host__ __device__ inline int nsegs(int spin, int lmax, int m)
{
    int lb = lbase(spin, m);
    return lb > lmax ? 0 : (lmax - lb + SEG) / SEG;
}

// ----------------------------------------------------------------------------
// Launch wrappers (defined in the .hip files)
// ----------------------------------------------------------------------------

struct SeedArgs {
    const RingDev* rings;
    const double* start;    // spin 0: lambda_lb (scaled mantissa); spin 2: P, M; [m][r] (SoA for spin 2)
    const int* startk;      // [m][r]
    double* mu;
    int* kk;
    const int64_t* seedoff;
    int64_t seedstride;
    int* lsig;
    int nrc;
    int lmax, rn, spin;
};
hipError_t launch_seeds(const SeedArgs& a, hipStream_t st);
// recursion coefficient table (layout of LegArgs::coef); rows must be zeroed first
hipError_t launch_coefs(double* coef, const int64_t* rowoff, int lmax, int spin, hipStream_t st);

// prec: 0 FP64, 1 FP32, 2 split BF16 (FP32 ring coefficients and map2alm rows,
// 64-bit split words as the alm2map operand rows)
hipError_t launch_leg_m2a(const LegArgs& a, int prec, hipStream_t st);
hipError_t launch_leg_a2m(const LegArgs& a, int prec, hipStream_t st);
hipError_t launch_leg_m2a_bf16(const LegArgs& a, hipStream_t st);
hipError_t launch_leg_a2m_bf16(const LegArgs& a, hipStream_t st);

}  // namespace sht
