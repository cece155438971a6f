// Legendre seed tables (plan creation).
//
// The contraction kernels generate lambda_lm(theta) on the fly with the
// three-term recursion in l (the paper's Algorithm 1 recomputes P_m(l, theta) for
// every m rather than caching it, Sec. 3.3).  To let many threads run the
// recursion of one (m, ring) in parallel, this kernel runs it once per plan and
// records the pair (lambda_ls, lambda_ls+1) at every segment start
// ls = lb(m) + SEG j, in the scaled form mu * 2^(-600 k).  The exponent counter
// replaces the paper's "safe positions" table (Sec. 3.1 item 11): values below
// 2^SIG_LOG2 are carried exactly in scaled form and count as zero, which also gives
// the ring-skipping bounds (Sec. 3.1 item 10) recorded in lsig.
#include "leg_common.h"

namespace sht {
namespace {

__global__ __launch_bounds__(128) void k_seeds(SeedArgs a)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const int m = blockIdx.y;
    if (r >= a.rn) return;
    const int L = a.lmax;
    const int lb = lbase(a.spin, m);
    if (lb > L) return;
    if (a.seedoff[m + 1] == a.seedoff[m]) return;  // an m the plan does not own: no seeds
    // x = cos(theta) enters as 1 - t with t = 1 - x exact to rounding: products
    // a x are formed as a - a t, so a pole ring's rounded z biases no row
    const double t = a.rings[r].omz;
    const int64_t base = a.seedoff[m] + r;
    const int64_t st = a.seedstride;
    int lsig = L + 1;

    if (a.spin == 0) {
        double v0 = a.start[(int64_t)m * a.rn + r];
        int k = a.startk[(int64_t)m * a.rn + r];
        const double s3 = sqrt(2.0 * m + 3.0);
        double v1 = fma(-s3, t, s3) * v0;  // lambda_{m+1,m} = sqrt(2m+3) x lambda_mm
        if (k == 0) lsig = lb;
        int j = 0;
        for (int l = lb; l <= L; ++l) {
            // state: v0 = lambda_l, v1 = lambda_{l+1}
            if (l == lb + SEG * j) {
                int64_t idx = base + (int64_t)j * a.rn;
                a.mu[idx] = v0;
                a.mu[st + idx] = v1;
                a.kk[idx] = k;
                ++j;
            }
            if (l + 1 >= L) {  // nothing further to compute; still reach l = L for its seed
                v0 = v1;
                continue;
            }
            double ca, cab;
            coef_spin0(l + 2, m, ca, cab);
            double v2 = fma(-ca, t, ca) * v1 - cab * v0;
            if (k > 0 && fabs(v2) > RESCALE_AT) {
                v2 *= SCALE_DOWN;
                v1 *= SCALE_DOWN;
                if (--k == 0 && lsig > L) lsig = l + 2;
            }
            v0 = v1;
            v1 = v2;
        }
    } else {
        double p0 = a.start[(int64_t)m * a.rn + r];
        double q0 = a.start[(int64_t)(a.lmax + 1) * a.rn + (int64_t)m * a.rn + r];
        int k = a.startk[(int64_t)m * a.rn + r];
        double al, be, ga;
        coef_spin2(lb + 1, m, al, be, ga);
        const double ax1 = fma(-al, t, al);
        double p1 = (ax1 + be) * p0;  // gamma(lb) = 0
        double q1 = (ax1 - be) * q0;
        if (k == 0) lsig = lb;
        int j = 0;
        for (int l = lb; l <= L; ++l) {
            if (l == lb + SEG * j) {
                int64_t idx = base + (int64_t)j * a.rn;
                a.mu[idx] = p0;
                a.mu[st + idx] = p1;
                a.mu[2 * st + idx] = q0;
                a.mu[3 * st + idx] = q1;
                a.kk[idx] = k;
                ++j;
            }
            if (l + 1 >= L) {
                p0 = p1;
                q0 = q1;
                continue;
            }
            coef_spin2(l + 2, m, al, be, ga);
            double ax = fma(-al, t, al);
            double p2 = (ax + be) * p1 - ga * p0;
            double q2 = (ax - be) * q1 - ga * q0;
            if (k > 0 && fmax(fabs(p2), fabs(q2)) > RESCALE_AT) {
                p2 *= SCALE_DOWN; p1 *= SCALE_DOWN;
                q2 *= SCALE_DOWN; q1 *= SCALE_DOWN;
                if (--k == 0 && lsig > L) lsig = l + 2;
            }
            p0 = p1; p1 = p2;
            q0 = q1; q1 = q2;
        }
    }
    atomicMin(a.lsig + (int64_t)m * a.nrc + r / RCHUNK, lsig);
}

// One row per (m, l >= lb): the coefficients the recursion uses to produce
// lambda_l, from the same formulas the seed recursion above evaluates.
__global__ __launch_bounds__(256) void k_coefs(double* coef, const int64_t* rowoff, int lmax, int spin)
{
    const int m = blockIdx.y;
    const int lb = lbase(spin, m);
    const int l = lb + blockIdx.x * blockDim.x + threadIdx.x;
    if (l > lmax) return;
    if (rowoff[m + 1] == rowoff[m]) return;  // an m the plan does not own: no rows
    if (spin == 0) {
        double* c = coef + (rowoff[m] + (l - lb)) * 2;
        coef_spin0(l, m, c[0], c[1]);
    } else {
        double* c = coef + (rowoff[m] + (l - lb)) * 4;
        coef_spin2(l, m, c[0], c[1], c[2]);
        c[3] = 0.0;
    }
}

}  // namespace

hipError_t launch_coefs(double* coef, const int64_t* rowoff, int lmax, int spin, hipStream_t st)
{
    dim3 grid((lmax + 1 + 255) / 256, lmax + 1);
    hipLaunchKernelGGL(k_coefs, grid, dim3(256), 0, st, coef, rowoff, lmax, spin);
    return hipGetLastError();
}

hipError_t launch_seeds(const SeedArgs& a, hipStream_t st)
{
    dim3 grid((a.rn + 127) / 128, a.lmax + 1);
    hipLaunchKernelGGL(k_seeds, grid, dim3(128), 0, st, a);
    return hipGetLastError();
}

}  // namespace sht
