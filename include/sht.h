/*
 * sht.h -- C ABI of the batched HEALPix spherical harmonic transform for
 * AMD Instinct MI355X (gfx950).
 *
 * The operations are those of Tian, Li & Liu, "Accelerating spherical harmonic
 * transforms for a large number of sky maps" (arXiv:2208.10154):
 *
 *   map2alm   a_lm = dsigma sum_p T(p) Y*_lm(p), dsigma = 4 pi / Npix
 *             (Sec. 2.1, eq. 1 and eq. "mm"; Algorithm 1); for polarisation the
 *             E/B coefficients of Sec. 2.3 (eqs. alm-EB and the 2x2 block form).
 *   alm2map   T(p) = sum_{l,m} a_lm Y_lm(p) (Sec. 2.1, backward equation), and the
 *             transposed block form of Sec. 2.3 for Q/U.
 *   map2alm_iter  the "traditional" iteration of Sec. 4 / Algorithm 2:
 *             a_0 = A m, a_n = a_{n-1} + A (m - Y a_{n-1}), run between the
 *             ring Fourier coefficients and a_lm (Sec. 3.1 item 8).
 *
 * Problem statement (Algorithm 1 "Data"/"Result"): a batch of sky maps in, their
 * spherical harmonic coefficients out, or the reverse.
 *
 * Layouts (all boundary data is FP64 in every precision mode):
 *   maps : double[nmaps][ncomp][12 nside^2], HEALPix RING order, ncomp = 1 (T)
 *          for spin 0 and 3 (I, Q, U) for spin 2.
 *   alm  : double[nmaps][ncomp][lmax+1][lmax+1] in the paper's compact real
 *          storage (Appendix A.2): component (T) or (T, E, B); within one
 *          component, column-major with flat index col*(lmax+1) + row, where
 *          Re a_lm sits at (row l, col m) and Im a_lm (m >= 1) at
 *          (row l-m, col lmax+1-m).  All a_lm with l < 2 of E and B are zero.
 *
 * All data pointers passed to the transform calls are DEVICE pointers on the
 * plan's device; the caller owns them.  Calls are asynchronous and ordered on
 * the plan's stream.  The plan owns its tables and (unless one is supplied) its
 * workspace.  A plan is not thread safe: use one plan per host thread/stream.
 *
 * Every call returns SHT_OK (0) or a negative status; sht_last_error() gives a
 * message (thread local).  Argument errors are detected before any device work
 * and leave the plan unchanged.  Asynchronous device faults surface at the next
 * call or at sht_plan_sync().
 */
#ifndef SHT_H
#define SHT_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sht_plan_s* sht_plan;

enum sht_status {
    SHT_OK = 0,
    SHT_ERR_ARG = -1,         /* invalid argument: nothing was done */
    SHT_ERR_NOMEM = -2,       /* device or host allocation failed */
    SHT_ERR_DEVICE = -3,      /* a HIP call or kernel failed */
    SHT_ERR_UNSUPPORTED = -4  /* valid request outside what this library implements */
};

/* Precision of the Legendre contraction.  The recursion (with its exponent
 * rescaling), dsigma, the FFTs and the iteration residual are FP64 in all modes. */
enum sht_precision {
    SHT_FP64 = 0,   /* FP64 MFMA, FP64 ring Fourier coefficients */
    SHT_FP32 = 1,   /* FP32 MFMA, FP32 ring Fourier coefficients */
    SHT_BF16X3 = 2  /* split BF16: each operand (rounded to FP32) as three bf16 numbers
                     * hi + mid + lo, products from the six partial products of order
                     * >= 2^-16 on the BF16 matrix cores, accumulated in FP32 (the
                     * accuracy of an FP32 contraction) */
};

/* Create a plan for HEALPix resolution nside, band limit lmax and spin 0 (T maps)
 * or 2 (IQU map triples), for batches of up to nmaps map sets per call.
 * Requires 1 <= nside <= 8192, 0 <= lmax <= 4*nside-1 (spin 2: lmax >= 2),
 * nmaps >= 1 (SHT_ERR_ARG otherwise); this library supports nside <= 2048
 * (SHT_ERR_UNSUPPORTED beyond).  Builds the ring tables, FFT plans and Legendre
 * seed tables on the current HIP device (the paper's once-only initialisation,
 * Sec. 3.3) and allocates the workspace for one chunk of map sets (see
 * sht_plan_set_chunk).  The seed tables hold about 80 nside lmax^2 / 8 bytes
 * (spin 2: three times that), 8.6 GB at nside 512 / lmax 1535; a plan whose
 * tables do not fit the device gives SHT_ERR_NOMEM (sht_plan_create_part splits
 * them). */
int sht_plan_create(sht_plan* out, int nside, int lmax, int spin, int nmaps);

/* Create a plan that owns part `part` (0 <= part < nparts) of the orders m: the
 * pairs (q, lmax - q) of m are dealt to the parts in turn (q mod nparts == part),
 * which balances the triangle of (l, m) work between parts.  This is one GPU's
 * share of the split by m that resolutions beyond one GPU's memory need (Sec. 5:
 * nside >= 2048; the Legendre step of each part needs nothing from the others).
 * The plan's seed and coefficient tables cover its own m only.  Its transforms:
 *   sht_map2alm  writes the a_lm of its own m and leaves every other a_lm entry
 *                of the output unchanged (so the parts can fill one array);
 *   sht_alm2map  writes the maps synthesised from the a_lm of its own m only
 *                (the sum over the parts' maps is the full synthesis).
 * The ring FFTs are computed for all rings on the plan's GPU (the exchange
 * between ring and m layouts that splits them across GPUs is not part of this
 * library).  Iterations, E/B separation, component selections and
 * sht_alm2map_noalloc need a plan of all m (SHT_ERR_UNSUPPORTED).  Arguments as
 * for sht_plan_create; SHT_ERR_ARG if part is out of range or owns no m. */
int sht_plan_create_part(sht_plan* out, int nside, int lmax, int spin, int nmaps, int part, int nparts);

/* Release every device and host resource of the plan (NULL is accepted). */
int sht_plan_destroy(sht_plan plan);

/* Select the contraction precision (enum sht_precision).  Default SHT_FP64.
 * Reallocates the workspace when the element size changes. */
int sht_plan_set_precision(sht_plan plan, int precision);

/* Stream on which all later calls of this plan are enqueued (a hipStream_t;
 * NULL = the default stream). */
int sht_plan_set_stream(sht_plan plan, void* hip_stream);

/* Number of map sets processed by the next calls, 1 <= n <= the nmaps given at
 * creation.  Default: that nmaps. */
int sht_plan_set_nmaps(sht_plan plan, int n);

/* Map sets transformed per internal chunk (bounds the workspace).  The default
 * keeps the workspace under about 8 GB.  Reallocates the workspace. */
int sht_plan_set_chunk(sht_plan plan, int maps_per_chunk);

/* Bytes of device workspace the plan uses with its current chunk and precision
 * (for admission control by a caller). */
size_t sht_plan_workspace_bytes(sht_plan plan);

/* Bytes of device memory held by the plan's own tables (excluding workspace). */
size_t sht_plan_table_bytes(sht_plan plan);

/* Ring coefficient rows (m, ring) the ring FFTs write (map2alm) or read
 * (alm2map) per component map: over all rings, 1 + the highest m whose Legendre
 * values on that ring are significant (the ring optimisation of Sec. 3.1 item 10
 * applied to the FFT mapping), at most (lmax + 1) * (4 nside - 1).  Each row is
 * one complex value per map.  0 for a NULL plan. */
long long sht_plan_ring_rows(sht_plan plan);

/* Use caller-owned device memory of at least sht_plan_workspace_bytes() bytes as
 * workspace (the plan frees its own).  dev_ptr must be 256-byte aligned, as
 * hipMalloc returns it: the operand rows inside are laid out for aligned vector
 * access.  A misaligned or too small buffer gives SHT_ERR_ARG and leaves the plan
 * as it was.  The buffer must stay allocated while the plan uses it; a later
 * sht_plan_set_chunk or sht_plan_set_precision that needs more gives SHT_ERR_ARG
 * and keeps the old setting.
 * Passing NULL returns to a plan-owned workspace. */
int sht_plan_set_workspace(sht_plan plan, void* dev_ptr, size_t bytes);

/* Backward transform (alm -> maps) of the current batch.  Device pointers. */
int sht_alm2map(sht_plan plan, const double* alm, double* map);

/* Backward transform (alm -> maps) of the current batch, as sht_alm2map, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid allocation): this call allocates nothing.
 * Its workspace is a static device array of SHT_NOALLOC_WORKSPACE_BYTES bytes
 * that each GPU the library runs on holds until the process ends (the plan's own
 * workspace is not used).  The batch runs in chunks of as many map sets as fit
 * that array at the plan's precision; if one map set does not fit (for example
 * nside 256, lmax 767, spin 0 in FP64) the call returns SHT_ERR_ARG and does
 * nothing.  All calls on one GPU share the array: calls that overlap in time on
 * one GPU (two streams, two host threads) race and give undefined results;
 * calls ordered on one stream are safe.  Every workspace element a chunk reads
 * is written earlier in the same chunk, so nothing is cleared between calls.
 * Same layouts and results as sht_alm2map (the same kernels). */
#define SHT_NOALLOC_WORKSPACE_BYTES (256u << 20)
int sht_alm2map_noalloc(sht_plan plan, const double* alm, double* map);

/* Forward transform (maps -> alm) of the current batch.  Device pointers. */
int sht_map2alm(sht_plan plan, const double* map, double* alm);

/* Iterative forward transform with niter >= 0 correction rounds (Algorithm 2).
 * If resid is not NULL it receives niter+1 host doubles: the RMS over all pixels
 * of all maps of the residual m - Y a_n after estimate n (n = 0 .. niter),
 * computed in FP64 from the ring Fourier coefficients (Parseval); this call then
 * synchronises the stream. */
int sht_map2alm_iter(sht_plan plan, const double* map, double* alm, int niter, double* resid);

/* Iterative forward transform in the "immediate" mode of Sec. 4 / Algorithm 3:
 * after a_0 = A m, each of the niter >= 0 sweeps updates the coefficients m by m
 * in increasing m, each update computed from the residual that already holds
 * the updates of the earlier m (a Gauss-Seidel sweep; the traditional mode of
 * sht_map2alm_iter is the Jacobi form).  The residual is kept as FP64 ring
 * spectra; m that share no ring bin run together, in schedule levels built once
 * per plan, which leaves the result of the sweep unchanged.  resid as for
 * sht_map2alm_iter (RMS over all pixels after estimate n, n = 0 .. niter; the
 * call then synchronises the stream).  Same layouts and errors as
 * sht_map2alm_iter.  The plan allocates, on the first call, a residual buffer
 * of the iteration buffer's size (8 * chunk * ncomp * 12 nside^2 bytes). */
int sht_map2alm_immediate(sht_plan plan, const double* map, double* alm, int niter, double* resid);

/* Components of the selective transforms (bit mask). */
enum sht_comp {
    SHT_COMP_T = 1,   /* temperature / intensity: the spin-0 part */
    SHT_COMP_E = 2,   /* E mode of a spin-2 plan */
    SHT_COMP_B = 4,   /* B mode of a spin-2 plan */
    SHT_COMP_ALL = 7
};

/* Backward transform of the selected components only: the coefficients of the
 * components left out are not read (they act as zero), so the maps hold the
 * synthesis of the selected ones; a map component with nothing selected (I when
 * T is left out, Q and U when E and B are) is written as zero.  With E or B alone
 * the spin-2 contraction keeps one half of the 0/1 diagonal selector lambda^{E,B}
 * of Sec. 2.3 and does half of its products (Sec. 3.1 asks for E and B to be
 * transformable on their own, in both directions).
 * comps: nonzero mask of enum sht_comp; a spin-0 plan accepts only SHT_COMP_T.
 * SHT_ERR_ARG otherwise.  sht_alm2map is this call with every component. */
int sht_alm2map_sel(sht_plan plan, int comps, const double* alm, double* map);

/* Forward transform of the selected components only: the coefficients of the
 * components left out are written as zero, and only the map components the
 * selection needs are read (I for T, Q and U for E or B).  Same comps rules as
 * sht_alm2map_sel; sht_map2alm is this call with every component. */
int sht_map2alm_sel(sht_plan plan, int comps, const double* map, double* alm);

/* Pixel-domain E/B separation of IQU map triples, S^{E,B} = F^t lambda^{E,B} F S
 * (Sec. 2.3, the block-matrix form with the 0/1 diagonal selector):
 *   alm   <- map2alm(map) (T, E, B; as sht_map2alm),
 *   map_e <- alm2map of (T, E, 0): Q/U are the E-mode part of the polarisation,
 *            I is the band-limited intensity,
 *   map_b <- alm2map of (0, 0, B): Q/U are the B-mode part, I is zero,
 * so map_e + map_b = alm2map(alm).  The coefficient rows are laid out once and
 * the E and B syntheses each run the half-block contraction.  Spin-2 plans only;
 * map_e and map_b must be distinct and must not overlap alm or map (map_e may be
 * map itself: each chunk is read before it is overwritten).  Device pointers,
 * layouts as above. */
int sht_eb_split(sht_plan plan, const double* map, double* alm, double* map_e, double* map_b);

/* Stages timed by the optional profiler. */
enum sht_stage {
    SHT_STAGE_FFT_FWD = 0,     /* ring FFT + m-unfold (maps -> ring coefficients) */
    SHT_STAGE_FFT_INV = 1,     /* alias fold + inverse ring FFT */
    SHT_STAGE_RESIDUAL = 2,    /* iteration residual in the Fourier domain */
    SHT_STAGE_M2A_SPIN0 = 3,   /* Legendre contraction, map2alm, T */
    SHT_STAGE_M2A_SPIN2 = 4,   /* Legendre contraction, map2alm, E/B */
    SHT_STAGE_A2M_SPIN0 = 5,   /* Legendre contraction, alm2map, T */
    SHT_STAGE_A2M_SPIN2 = 6,   /* Legendre contraction, alm2map, Q/U */
    SHT_STAGE_ALM_LAYOUT = 7,  /* compact <-> m-major coefficient layout (with dsigma) */
    SHT_NSTAGE = 8
};

/* Enable (1) or disable (0) per-stage timing: when enabled every stage's kernel
 * launches are bracketed by HIP events on the plan's stream.  Off by default. */
int sht_plan_set_profiling(sht_plan plan, int enable);

/* Synchronise the plan's stream and return, per stage (arrays of SHT_NSTAGE),
 * the summed device time in milliseconds and the number of timed launches since
 * the last reset; reset != 0 clears the record. */
int sht_plan_get_profile(sht_plan plan, double* ms, long long* launches, int reset);

/* Wait for the plan's stream and report any asynchronous device error. */
int sht_plan_sync(sht_plan plan);

/* Message describing the last error on this thread ("" if none). */
const char* sht_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SHT_H */
