// Device helpers shared by the Legendre seed and contraction kernels.
#pragma once
#include "sht_internal.h"

namespace sht {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// MFMA 16x16x4 policy for FP64 / FP32 operands.  Operands (both types): A[i][k]
// from lane 16k + i, B[k][j] from lane 16k + j.  Results: D[i][j] sits in lane
// 16*(i & 3) + j, register i >> 2 for FP64, and in lane 16*(i >> 2) + j,
// register i & 3 for FP32 (measured on gfx950); row(lane, v) gives i.
template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
    using acc = v4d;
    __device__ static __forceinline__ acc run(double a, double b, acc c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ int row(int lane, int v) { return 4 * v + (lane >> 4); }
};
template <>
struct Mfma<float> {
    using acc = v4f;
    __device__ static __forceinline__ acc run(float a, float b, acc c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

// Spin-0 recursion coefficients producing lambda_l from lambda_{l-1}, lambda_{l-2}:
// lambda_l = (a_l x) lambda_{l-1} - (a_l b_l) lambda_{l-2},
// a_l = sqrt((4l^2-1)/(l^2-m^2)), b_l = sqrt(((l-1)^2-m^2)/(4(l-1)^2-1)).
__device__ __forceinline__ void coef_spin0(int l, int m, double& a, double& ab)
{
    if (l <= m) { a = 0.0; ab = 0.0; return; }
    double dl = l, dm = m, t = (dl - 1.0) * (dl - 1.0);
    a = sqrt((4.0 * dl * dl - 1.0) / (dl * dl - dm * dm));
    ab = a * sqrt((t - dm * dm) / (4.0 * t - 1.0));
}

// Spin +-2 recursion (Wigner d^l_{m,-+2} normalised by sqrt((2l+1)/4pi)) producing
// lambda_l from lambda_{l-1}, lambda_{l-2}:
//   P_l = (alpha x + beta) P_{l-1} - gamma P_{l-2}   (s = +2)
//   M_l = (alpha x - beta) M_{l-1} - gamma M_{l-2}   (s = -2)
// with, for j = l-1 and c(j) = sqrt((j^2-m^2)(j^2-4)):
//   alpha = sqrt((2j+3)(2j+1)) (j+1) / c(j+1)
//   beta  = 2 m sqrt((2j+3)(2j+1)) / (j c(j+1))
//   gamma = sqrt((2j+3)/(2j-1)) (j+1) c(j) / (j c(j+1))
__device__ __forceinline__ void coef_spin2(int l, int m, double& al, double& be, double& ga)
{
    int lb = m > 2 ? m : 2;
    if (l <= lb) { al = be = ga = 0.0; return; }
    double j = l - 1, dm = m;
    double cj = sqrt((j * j - dm * dm) * (j * j - 4.0));
    double cj1 = sqrt(((j + 1) * (j + 1) - dm * dm) * ((j + 1) * (j + 1) - 4.0));
    double q = sqrt((2.0 * j + 3.0) * (2.0 * j + 1.0));
    al = q * (j + 1.0) / cj1;
    be = 2.0 * dm * q / (j * cj1);
    ga = sqrt((2.0 * j + 3.0) / (2.0 * j - 1.0)) * (j + 1.0) * cj / (j * cj1);
}

// XCD-aware block order: consecutive blocks are dealt round-robin to the 8 XCDs;
// give the blocks of one XCD consecutive logical indices so that tiles sharing
// operands run on the same XCD (and L2) at about the same time.
__device__ __forceinline__ int xcd_remap(int b, int B)
{
    int nx = B >> 3, rem = B & 7, x = b & 7, pos = b >> 3;
    return (x < rem) ? x * (nx + 1) + pos : rem * (nx + 1) + (x - rem) * nx + pos;
}

}  // namespace sht
