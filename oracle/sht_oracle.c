/*
 * sht_oracle.c -- TEST INFRASTRUCTURE ONLY (parity oracle, never a product path).
 *
 * A plain, slow, obviously-correct CPU implementation of the spherical harmonic
 * transforms of HEALPix ring-ordered sky maps, written from the definitions in
 * Tian, Li & Liu, "Accelerating spherical harmonic transforms for a large number
 * of sky maps" (arXiv:2208.10154):
 *
 *   forward  a_lm = dsigma * sum_p T(p) Y*_lm(p),  dsigma = 4 pi / Npix   (Sec. 2.1, eq. 1 and eq. "mm")
 *   backward T(p) = sum_{l<=lmax} sum_{|m|<=l} a_lm Y_lm(p)              (Sec. 2.1, backward equation)
 *   spin 2   Q +/- iU = sum a_{+/-2,lm} {}_{+/-2}Y_lm,
 *            a_E = -(a_2 + a_-2)/2,  a_B = i (a_2 - a_-2)/2               (Sec. 2.3, eqs. Q+-iU and alm-EB)
 *
 * Everything is evaluated by direct summation in long double (x87, 64-bit
 * mantissa, 15-bit exponent, so sin^m(theta) of the highest m used here does not
 * underflow before it matters). There is no FFT, no matrix product, no batching
 * trick and no compact alm storage: the azimuthal sum is a literal DFT with
 * e^{-i m phi} evaluated per pixel (aliasing of m onto ring bins therefore happens
 * by itself), and the only re-association of the defining sum is the grouping of
 * the pixel sum by iso-latitude ring (the first three rows of eq. "mm").
 *
 * It shares no code with the GPU path: geometry, Legendre functions, phases and
 * storage conversions are all written here independently.
 *
 * alm arrays are complex, stored as interleaved (re, im) doubles indexed
 * [map][l][m] on an (lmax+1) x (lmax+1) grid (entries with m > l are ignored and
 * written as zero); only m >= 0 is stored, the negative-m coefficients of a real
 * field being a_{l,-m} = (-1)^m conj(a_lm).  Maps are double[map][Npix] in HEALPix
 * RING order.  Spin-2 routines take/return the E and B coefficients and the Q and
 * U maps.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef long double ld;
static const ld PI_L = 3.141592653589793238462643383279502884197L;

/* ------------------------------------------------------------------------- */
/* HEALPix RING geometry, from the published definition of the pixelisation  */
/* (Gorski et al. 2005, cited in Sec. 1). Rings i = 1 .. 4 nside - 1 from the */
/* north pole. Pixel n (0-based) of a ring sits at phi = pi (2n + s) / N.     */
/* ------------------------------------------------------------------------- */
typedef struct {
    ld z;       /* cos(theta) */
    ld sth;     /* sin(theta) */
    long n;     /* pixels in the ring */
    int s;      /* phase shift: first pixel at phi = pi s / N */
    long first; /* index of the first pixel of the ring */
} oring;

static oring ring_of(long nside, long i)
{
    oring r;
    ld ns = (ld)nside;
    if (i < nside || i > 3 * nside) {              /* polar caps */
        long j = (i < nside) ? i : 4 * nside - i;  /* ring counted from the nearer pole */
        ld onemz = (ld)(j * j) / (3.0L * ns * ns); /* 1 - |z| */
        r.z = 1.0L - onemz;
        r.sth = sqrtl(onemz * (2.0L - onemz));
        r.n = 4 * j;
        r.s = 1;
        if (i < nside) r.first = 2 * j * (j - 1);
        else { r.first = 12 * nside * nside - 2 * j * (j + 1); r.z = -r.z; }
    } else {                                       /* equatorial belt */
        r.z = (ld)(4 * nside - 2 * i) / (3.0L * ns);
        r.sth = sqrtl((1.0L - r.z) * (1.0L + r.z));
        r.n = 4 * nside;
        r.s = ((i - nside) % 2 == 0) ? 1 : 0;
        r.first = 2 * nside * (nside - 1) + (i - nside) * 4 * nside;
    }
    return r;
}

/* exact phase: m * phi_n = pi * (m (2n+s) mod 2N) / N, reduced in integers */
static void phase(long m, long n, const oring* r, ld* c, ld* s)
{
    long twoN = 2 * r->n;
    long q = ((m % twoN) * ((2 * n + r->s) % twoN)) % twoN;
    if (q < 0) q += twoN;
    ld ang = PI_L * (ld)q / (ld)r->n;
    *c = cosl(ang);
    *s = sinl(ang);
}

/* ------------------------------------------------------------------------- */
/* Normalised associated Legendre functions lambda_lm(theta), with           */
/* Y_lm = lambda_lm e^{i m phi} (Sec. 2.1 footnote: |P| = |Y|), orthonormal, */
/* Condon-Shortley phase.  Standard three-term recursion in l from l = m.    */
/* ------------------------------------------------------------------------- */
static void lam_spin0(long lmax, long m, ld z, ld sth, ld* out)
{
    ld v = 1.0L / sqrtl(4.0L * PI_L);
    for (long k = 1; k <= m; ++k) v *= -sqrtl((ld)(2 * k + 1) / (ld)(2 * k)) * sth;
    out[m] = v;
    if (m + 1 <= lmax) out[m + 1] = sqrtl((ld)(2 * m + 3)) * z * v;
    for (long l = m + 2; l <= lmax; ++l) {
        ld a = sqrtl((ld)(4 * l * l - 1) / (ld)(l * l - m * m));
        ld b = sqrtl((ld)((l - 1) * (l - 1) - m * m) / (ld)(4 * (l - 1) * (l - 1) - 1));
        out[l] = a * (z * out[l - 1] - b * out[l - 2]);
    }
}

/* Wigner small-d d^j_{a b}(beta) by its explicit finite sum, with
 * c = cos(beta/2), s = sin(beta/2) (both > 0 on HEALPix ring centres). */
static ld lfact(long n) { return lgammal((ld)n + 1.0L); }
static ld wigner_d(long j, long a, long b, ld c, ld s)
{
    long kmin = 0, kmax = j + b;
    if (b - a > kmin) kmin = b - a;
    if (j - a < kmax) kmax = j - a;
    ld pre = 0.5L * (lfact(j + a) + lfact(j - a) + lfact(j + b) + lfact(j - b));
    ld lc = logl(c), ls = logl(s), sum = 0.0L;
    for (long k = kmin; k <= kmax; ++k) {
        ld lg = pre - lfact(j + b - k) - lfact(k) - lfact(a - b + k) - lfact(j - a - k)
              + (ld)(2 * j + b - a - 2 * k) * lc + (ld)(a - b + 2 * k) * ls;
        ld t = expl(lg);
        sum += (((a - b + k) & 1) ? -t : t);
    }
    return sum;
}

/* Spin-weighted functions {}_s lambda_lm(theta) = sqrt((2l+1)/4pi) d^l_{m,-s}(theta),
 * so that {}_sY_lm = {}_s lambda_lm e^{i m phi} (Goldberg et al. 1967 form; for
 * s = +-2 the (-1)^s factor of some conventions is 1).  Any sign of m.  Filled for
 * l = max(|m|,|s|) .. lmax, zero below.  Three-term recursion of d^l in l. */
static void lam_spin(long lmax, long m, long s, ld z, ld* out)
{
    long mp = -s;
    long l0 = labs(m) > labs(mp) ? labs(m) : labs(mp);
    for (long l = 0; l <= lmax && l < l0; ++l) out[l] = 0.0L;
    if (l0 > lmax) return;
    ld c = sqrtl((1.0L + z) / 2.0L), sn = sqrtl((1.0L - z) / 2.0L);
    ld dprev = 0.0L, d = wigner_d(l0, m, mp, c, sn);
    out[l0] = sqrtl((ld)(2 * l0 + 1) / (4.0L * PI_L)) * d;
    for (long l = l0; l < lmax; ++l) {
        ld num1 = (ld)(2 * l + 1) * ((ld)(l * (l + 1)) * z - (ld)(m * mp)) * d;
        ld num2 = (ld)(l + 1) * sqrtl((ld)(l * l - m * m) * (ld)(l * l - mp * mp)) * dprev;
        ld den = (ld)l * sqrtl((ld)((l + 1) * (l + 1) - m * m) * (ld)((l + 1) * (l + 1) - mp * mp));
        ld dn = (num1 - num2) / den;
        dprev = d;
        d = dn;
        out[l + 1] = sqrtl((ld)(2 * l + 3) / (4.0L * PI_L)) * d;
    }
}

/* ------------------------------------------------------------------------- */
/* exported helpers (used by the pin tests)                                  */
/* ------------------------------------------------------------------------- */
long orc_npix(long nside) { return 12 * nside * nside; }

void orc_ring(long nside, long i, double* z, double* sth, long* n, int* s, long* first)
{
    oring r = ring_of(nside, i);
    *z = (double)r.z; *sth = (double)r.sth; *n = r.n; *s = r.s; *first = r.first;
}

void orc_lambda0(long lmax, long m, double theta, double* out)
{
    ld* buf = (ld*)calloc((size_t)lmax + 2, sizeof(ld));
    ld th = (ld)theta;
    lam_spin0(lmax, m, cosl(th), sinl(th), buf);
    for (long l = 0; l <= lmax; ++l) out[l] = (l < m) ? 0.0 : (double)buf[l];
    free(buf);
}

void orc_lambda_spin(long lmax, long m, long s, double theta, double* out)
{
    ld* buf = (ld*)calloc((size_t)lmax + 2, sizeof(ld));
    lam_spin(lmax, m, s, cosl((ld)theta), buf);
    for (long l = 0; l <= lmax; ++l) out[l] = (double)buf[l];
    free(buf);
}

/* ------------------------------------------------------------------------- */
/* spin 0                                                                    */
/* ------------------------------------------------------------------------- */
#define ALM(a, k, l, m, L) ((a) + 2 * (((size_t)(k) * ((L) + 1) + (size_t)(l)) * ((L) + 1) + (size_t)(m)))

/* backward transform: T(p) = sum_m e^{i m phi} sum_l a_lm lambda_lm, m = -lmax..lmax,
 * written over m >= 0 with the reality condition (weight 1 for m = 0, 2 for m > 0). */
/* rstep > 1 evaluates only every rstep-th ring (a timing sample; other rings untouched) */
void orc_alm2map_spin0_strided(long nside, long lmax, long nmaps, const double* alm, double* map, long rstep)
{
    long nring = 4 * nside - 1, npix = 12 * nside * nside, L = lmax;
#pragma omp parallel
    {
        ld* lam = (ld*)malloc(sizeof(ld) * (L + 2));
        ld* cre = (ld*)malloc(sizeof(ld) * nmaps * (L + 1));
        ld* cim = (ld*)malloc(sizeof(ld) * nmaps * (L + 1));
#pragma omp for schedule(dynamic)
        for (long i = 1; i <= nring; i += rstep) {
            oring r = ring_of(nside, i);
            for (long m = 0; m <= L; ++m) {
                lam_spin0(L, m, r.z, r.sth, lam);
                for (long k = 0; k < nmaps; ++k) {
                    ld sr = 0.0L, si = 0.0L;
                    for (long l = m; l <= L; ++l) {
                        sr += (ld)ALM(alm, k, l, m, L)[0] * lam[l];
                        si += (ld)ALM(alm, k, l, m, L)[1] * lam[l];
                    }
                    cre[k * (L + 1) + m] = sr;
                    cim[k * (L + 1) + m] = si;
                }
            }
            for (long n = 0; n < r.n; ++n) {
                for (long k = 0; k < nmaps; ++k) {
                    ld t = 0.0L;
                    for (long m = 0; m <= L; ++m) {
                        ld c, s;
                        phase(m, n, &r, &c, &s);
                        ld w = (m == 0) ? 1.0L : 2.0L;
                        t += w * (cre[k * (L + 1) + m] * c - cim[k * (L + 1) + m] * s);
                    }
                    map[(size_t)k * npix + r.first + n] = (double)t;
                }
            }
        }
        free(lam); free(cre); free(cim);
    }
}

void orc_alm2map_spin0(long nside, long lmax, long nmaps, const double* alm, double* map)
{
    orc_alm2map_spin0_strided(nside, lmax, nmaps, alm, map, 1);
}

/* forward transform: a_lm = dsigma sum_rings lambda_lm(theta_i) sum_n T(i,n) e^{-i m phi_n};
 * mstep > 1 evaluates only every mstep-th m (a timing sample) */
void orc_map2alm_spin0_strided(long nside, long lmax, long nmaps, const double* map, double* alm, long mstep)
{
    long nring = 4 * nside - 1, npix = 12 * nside * nside, L = lmax;
    ld dsig = 4.0L * PI_L / (ld)npix;
    memset(alm, 0, sizeof(double) * 2 * nmaps * (L + 1) * (L + 1));
#pragma omp parallel
    {
        ld* lam = (ld*)malloc(sizeof(ld) * (L + 2));
        ld* are = (ld*)malloc(sizeof(ld) * nmaps * (L + 1));
        ld* aim = (ld*)malloc(sizeof(ld) * nmaps * (L + 1));
        ld* cs = (ld*)malloc(sizeof(ld) * 2 * 4 * nside);
#pragma omp for schedule(dynamic)
        for (long m = 0; m <= L; m += mstep) {
            for (long j = 0; j < nmaps * (L + 1); ++j) are[j] = aim[j] = 0.0L;
            for (long i = 1; i <= nring; ++i) {
                oring r = ring_of(nside, i);
                lam_spin0(L, m, r.z, r.sth, lam);
                for (long n = 0; n < r.n; ++n) phase(m, n, &r, &cs[2 * n], &cs[2 * n + 1]);
                for (long k = 0; k < nmaps; ++k) {
                    ld gr = 0.0L, gi = 0.0L;
                    const double* t = map + (size_t)k * npix + r.first;
                    for (long n = 0; n < r.n; ++n) { gr += t[n] * cs[2 * n]; gi -= t[n] * cs[2 * n + 1]; }
                    for (long l = m; l <= L; ++l) {
                        are[k * (L + 1) + l] += lam[l] * gr;
                        aim[k * (L + 1) + l] += lam[l] * gi;
                    }
                }
            }
            for (long k = 0; k < nmaps; ++k)
                for (long l = m; l <= L; ++l) {
                    ALM(alm, k, l, m, L)[0] = (double)(dsig * are[k * (L + 1) + l]);
                    ALM(alm, k, l, m, L)[1] = (double)(dsig * aim[k * (L + 1) + l]);
                }
        }
        free(lam); free(are); free(aim); free(cs);
    }
}

void orc_map2alm_spin0(long nside, long lmax, long nmaps, const double* map, double* alm)
{
    orc_map2alm_spin0_strided(nside, lmax, nmaps, map, alm, 1);
}

/* ------------------------------------------------------------------------- */
/* spin 2: Q + iU = sum_{l>=2} sum_{m=-l..l} a_{2,lm} {}_2Y_lm with           */
/* a_{2,lm} = -(a_E,lm + i a_B,lm) (inverse of eq. alm-EB), all m.            */
/* ------------------------------------------------------------------------- */
static void get_eb(const double* aE, const double* aB, long k, long l, long m, long L,
                   ld* er, ld* ei, ld* br, ld* bi)
{
    long am = labs(m);
    ld sg = ((am & 1) && m < 0) ? -1.0L : 1.0L;         /* (-1)^m for negative m */
    ld cj = (m < 0) ? -1.0L : 1.0L;                       /* conjugate for negative m */
    *er = sg * (ld)ALM(aE, k, l, am, L)[0];
    *ei = sg * cj * (ld)ALM(aE, k, l, am, L)[1];
    *br = sg * (ld)ALM(aB, k, l, am, L)[0];
    *bi = sg * cj * (ld)ALM(aB, k, l, am, L)[1];
}

void orc_alm2map_spin2_strided(long nside, long lmax, long nmaps, const double* aE, const double* aB,
                               double* Q, double* U, long rstep)
{
    long nring = 4 * nside - 1, npix = 12 * nside * nside, L = lmax;
    long nm = 2 * L + 1;
#pragma omp parallel
    {
        ld* lam = (ld*)malloc(sizeof(ld) * (L + 2));
        ld* cre = (ld*)malloc(sizeof(ld) * nmaps * nm);
        ld* cim = (ld*)malloc(sizeof(ld) * nmaps * nm);
#pragma omp for schedule(dynamic)
        for (long i = 1; i <= nring; i += rstep) {
            oring r = ring_of(nside, i);
            for (long m = -L; m <= L; ++m) {
                lam_spin(L, m, 2, r.z, lam);
                for (long k = 0; k < nmaps; ++k) {
                    ld sr = 0.0L, si = 0.0L;
                    long lo = labs(m) > 2 ? labs(m) : 2;
                    for (long l = lo; l <= L; ++l) {
                        ld er, ei, br, bi;
                        get_eb(aE, aB, k, l, m, L, &er, &ei, &br, &bi);
                        /* a_2 = -(E + i B) */
                        ld a2r = -(er - bi), a2i = -(ei + br);
                        sr += a2r * lam[l];
                        si += a2i * lam[l];
                    }
                    cre[k * nm + (m + L)] = sr;
                    cim[k * nm + (m + L)] = si;
                }
            }
            for (long n = 0; n < r.n; ++n)
                for (long k = 0; k < nmaps; ++k) {
                    ld pr = 0.0L, pi = 0.0L;
                    for (long m = -L; m <= L; ++m) {
                        ld c, s;
                        phase(m, n, &r, &c, &s);
                        ld xr = cre[k * nm + (m + L)], xi = cim[k * nm + (m + L)];
                        pr += xr * c - xi * s;
                        pi += xr * s + xi * c;
                    }
                    Q[(size_t)k * npix + r.first + n] = (double)pr;
                    U[(size_t)k * npix + r.first + n] = (double)pi;
                }
        }
        free(lam); free(cre); free(cim);
    }
}

void orc_alm2map_spin2(long nside, long lmax, long nmaps, const double* aE, const double* aB,
                       double* Q, double* U)
{
    orc_alm2map_spin2_strided(nside, lmax, nmaps, aE, aB, Q, U, 1);
}

/* a_{+-2,lm} = dsigma sum_p (Q +- iU)(p) {}_{+-2}Y*_lm(p); then eq. alm-EB. m >= 0. */
void orc_map2alm_spin2_strided(long nside, long lmax, long nmaps, const double* Q, const double* U,
                               double* aE, double* aB, long mstep)
{
    long nring = 4 * nside - 1, npix = 12 * nside * nside, L = lmax;
    ld dsig = 4.0L * PI_L / (ld)npix;
    memset(aE, 0, sizeof(double) * 2 * nmaps * (L + 1) * (L + 1));
    memset(aB, 0, sizeof(double) * 2 * nmaps * (L + 1) * (L + 1));
#pragma omp parallel
    {
        ld* lp = (ld*)malloc(sizeof(ld) * (L + 2));
        ld* lm = (ld*)malloc(sizeof(ld) * (L + 2));
        ld* acc = (ld*)malloc(sizeof(ld) * 4 * nmaps * (L + 1)); /* a_2 re,im ; a_-2 re,im */
        ld* cs = (ld*)malloc(sizeof(ld) * 2 * 4 * nside);
#pragma omp for schedule(dynamic)
        for (long m = 0; m <= L; m += mstep) {
            for (long j = 0; j < 4 * nmaps * (L + 1); ++j) acc[j] = 0.0L;
            for (long i = 1; i <= nring; ++i) {
                oring r = ring_of(nside, i);
                lam_spin(L, m, 2, r.z, lp);
                lam_spin(L, m, -2, r.z, lm);
                for (long n = 0; n < r.n; ++n) phase(m, n, &r, &cs[2 * n], &cs[2 * n + 1]);
                for (long k = 0; k < nmaps; ++k) {
                    const double* q = Q + (size_t)k * npix + r.first;
                    const double* u = U + (size_t)k * npix + r.first;
                    /* G+- = sum_n (Q +- iU) e^{-i m phi} */
                    ld gpr = 0, gpi = 0, gmr = 0, gmi = 0;
                    for (long n = 0; n < r.n; ++n) {
                        ld c = cs[2 * n], s = cs[2 * n + 1];
                        gpr += q[n] * c + u[n] * s;  gpi += u[n] * c - q[n] * s;
                        gmr += q[n] * c - u[n] * s;  gmi += -u[n] * c - q[n] * s;
                    }
                    ld* a = acc + 4 * k * (L + 1);
                    for (long l = (m > 2 ? m : 2); l <= L; ++l) {
                        a[4 * l + 0] += lp[l] * gpr;
                        a[4 * l + 1] += lp[l] * gpi;
                        a[4 * l + 2] += lm[l] * gmr;
                        a[4 * l + 3] += lm[l] * gmi;
                    }
                }
            }
            for (long k = 0; k < nmaps; ++k)
                for (long l = (m > 2 ? m : 2); l <= L; ++l) {
                    ld* a = acc + 4 * k * (L + 1) + 4 * l;
                    ld a2r = dsig * a[0], a2i = dsig * a[1], amr = dsig * a[2], ami = dsig * a[3];
                    /* a_E = -(a_2 + a_-2)/2 ; a_B = i (a_2 - a_-2)/2 */
                    ALM(aE, k, l, m, L)[0] = (double)(-(a2r + amr) / 2.0L);
                    ALM(aE, k, l, m, L)[1] = (double)(-(a2i + ami) / 2.0L);
                    ALM(aB, k, l, m, L)[0] = (double)(-(a2i - ami) / 2.0L);
                    ALM(aB, k, l, m, L)[1] = (double)((a2r - amr) / 2.0L);
                }
        }
        free(lp); free(lm); free(acc); free(cs);
    }
}

void orc_map2alm_spin2(long nside, long lmax, long nmaps, const double* Q, const double* U,
                       double* aE, double* aB)
{
    orc_map2alm_spin2_strided(nside, lmax, nmaps, Q, U, aE, aB, 1);
}

/* ------------------------------------------------------------------------- */
/* sampled evaluations, for checks at sizes where a full transform is slow   */
/* ------------------------------------------------------------------------- */
static long ring_of_pixel(long nside, long p)
{
    /* smallest ring i whose first pixel exceeds p, minus one; plain linear scan */
    long nring = 4 * nside - 1;
    for (long i = 1; i <= nring; ++i) {
        oring r = ring_of(nside, i);
        if (p < r.first + r.n) return i;
    }
    return nring;
}

/* T at selected pixels of one map (spin 0) */
void orc_synth_pixels_spin0(long nside, long lmax, const double* alm, long npts, const long* pix, double* out)
{
    long L = lmax;
#pragma omp parallel
    {
        ld* lam = (ld*)malloc(sizeof(ld) * (L + 2));
#pragma omp for schedule(dynamic)
        for (long q = 0; q < npts; ++q) {
            long i = ring_of_pixel(nside, pix[q]);
            oring r = ring_of(nside, i);
            long n = pix[q] - r.first;
            ld t = 0.0L;
            for (long m = 0; m <= L; ++m) {
                lam_spin0(L, m, r.z, r.sth, lam);
                ld sr = 0.0L, si = 0.0L;
                for (long l = m; l <= L; ++l) { sr += ALM(alm, 0, l, m, L)[0] * lam[l]; si += ALM(alm, 0, l, m, L)[1] * lam[l]; }
                ld c, s;
                phase(m, n, &r, &c, &s);
                t += ((m == 0) ? 1.0L : 2.0L) * (sr * c - si * s);
            }
            out[q] = (double)t;
        }
        free(lam);
    }
}

/* Q, U at selected pixels of one map (spin 2) */
void orc_synth_pixels_spin2(long nside, long lmax, const double* aE, const double* aB, long npts,
                            const long* pix, double* outQ, double* outU)
{
    long L = lmax;
#pragma omp parallel
    {
        ld* lam = (ld*)malloc(sizeof(ld) * (L + 2));
#pragma omp for schedule(dynamic)
        for (long q = 0; q < npts; ++q) {
            long i = ring_of_pixel(nside, pix[q]);
            oring r = ring_of(nside, i);
            long n = pix[q] - r.first;
            ld pr = 0.0L, pi = 0.0L;
            for (long m = -L; m <= L; ++m) {
                lam_spin(L, m, 2, r.z, lam);
                ld sr = 0.0L, si = 0.0L;
                for (long l = (labs(m) > 2 ? labs(m) : 2); l <= L; ++l) {
                    ld er, ei, br, bi;
                    get_eb(aE, aB, 0, l, m, L, &er, &ei, &br, &bi);
                    sr += -(er - bi) * lam[l];
                    si += -(ei + br) * lam[l];
                }
                ld c, s;
                phase(m, n, &r, &c, &s);
                pr += sr * c - si * s;
                pi += sr * s + si * c;
            }
            outQ[q] = (double)pr;
            outU[q] = (double)pi;
        }
        free(lam);
    }
}

/* a_lm of one map at selected (l, m), spin 0 */
void orc_analyze_lm_spin0(long nside, long lmax, const double* map, long npts, const long* ls,
                          const long* ms, double* out /* re,im */)
{
    long nring = 4 * nside - 1, npix = 12 * nside * nside, L = lmax;
    ld dsig = 4.0L * PI_L / (ld)npix;
#pragma omp parallel
    {
        ld* lam = (ld*)malloc(sizeof(ld) * (L + 2));
#pragma omp for schedule(dynamic)
        for (long q = 0; q < npts; ++q) {
            long l = ls[q], m = ms[q];
            ld ar = 0.0L, ai = 0.0L;
            for (long i = 1; i <= nring; ++i) {
                oring r = ring_of(nside, i);
                lam_spin0(l, m, r.z, r.sth, lam);
                ld gr = 0.0L, gi = 0.0L;
                for (long n = 0; n < r.n; ++n) {
                    ld c, s;
                    phase(m, n, &r, &c, &s);
                    gr += map[r.first + n] * c;
                    gi -= map[r.first + n] * s;
                }
                ar += lam[l] * gr;
                ai += lam[l] * gi;
            }
            out[2 * q] = (double)(dsig * ar);
            out[2 * q + 1] = (double)(dsig * ai);
        }
        free(lam);
    }
}

/* a_E, a_B of one Q/U map pair at selected (l, m), spin 2 */
void orc_analyze_lm_spin2(long nside, long lmax, const double* Q, const double* U, long npts,
                          const long* ls, const long* ms, double* outE, double* outB)
{
    long nring = 4 * nside - 1, npix = 12 * nside * nside;
    ld dsig = 4.0L * PI_L / (ld)npix;
    (void)lmax;
#pragma omp parallel
    {
        ld* lp = (ld*)malloc(sizeof(ld) * (lmax + 2));
        ld* lm = (ld*)malloc(sizeof(ld) * (lmax + 2));
#pragma omp for schedule(dynamic)
        for (long q = 0; q < npts; ++q) {
            long l = ls[q], m = ms[q];
            ld a2r = 0, a2i = 0, amr = 0, ami = 0;
            for (long i = 1; i <= nring; ++i) {
                oring r = ring_of(nside, i);
                lam_spin(l, m, 2, r.z, lp);
                lam_spin(l, m, -2, r.z, lm);
                ld gpr = 0, gpi = 0, gmr = 0, gmi = 0;
                for (long n = 0; n < r.n; ++n) {
                    ld c, s;
                    phase(m, n, &r, &c, &s);
                    ld qq = Q[r.first + n], uu = U[r.first + n];
                    gpr += qq * c + uu * s;  gpi += uu * c - qq * s;
                    gmr += qq * c - uu * s;  gmi += -uu * c - qq * s;
                }
                a2r += lp[l] * gpr; a2i += lp[l] * gpi;
                amr += lm[l] * gmr; ami += lm[l] * gmi;
            }
            a2r *= dsig; a2i *= dsig; amr *= dsig; ami *= dsig;
            outE[2 * q] = (double)(-(a2r + amr) / 2.0L);
            outE[2 * q + 1] = (double)(-(a2i + ami) / 2.0L);
            outB[2 * q] = (double)(-(a2i - ami) / 2.0L);
            outB[2 * q + 1] = (double)((a2r - amr) / 2.0L);
        }
        free(lp); free(lm);
    }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
