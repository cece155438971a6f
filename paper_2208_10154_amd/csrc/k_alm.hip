// Coefficient layout changes between the paper's compact storage and the m-major
// operand layout of the Legendre kernels (HIP, gfx950).
//
// The compact storage (Appendix A.2) keeps, per map and component, the real part
// of a_lm at (row l, col m) and the imaginary part at (row l-m, col lmax+1-m) of an
// (lmax+1)^2 column-major square, so for one m each part is a contiguous run in l.
// The contraction wants, per m, rows of l with the maps of the batch along the
// row: A[m][l][2k + part].  These kernels move 64 l x 32 maps tiles through LDS so
// both sides are read and written in contiguous runs.  They also carry the scalar
// work of the boundary: dsigma and accumulation for map2alm (the paper's GEMM
// alpha/beta, Sec. 3.1 item 7) and the B <-> iB change of variable of Sec. 2.3.
#include <algorithm>

#include "sht_internal.h"

namespace sht {
namespace {

constexpr int NT = 256;
constexpr int TLB = 64;  // l per tile (= TL)
constexpr int TK = 32;   // maps per tile
constexpr int PER = 2 * TK * TLB / NT;  // tile elements per thread

__device__ __forceinline__ int64_t calm(int L, int l, int m, int part)
{
    if (part == 0) return (int64_t)m * (L + 1) + l;
    if (m == 0) return -1;
    return (int64_t)(L + 1 - m) * (L + 1) + (l - m);
}

__device__ __forceinline__ void decode(const int* off, int lmax, const int* mlist, int nlist, int C, int g, int& m,
                                       int& lt, int& kb)
{
    int lo = 0, hi = mlist ? nlist : lmax + 1;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (off[mid] * C <= g) lo = mid; else hi = mid;
    }
    m = mlist ? mlist[lo] : lo;
    int r = g - off[lo] * C;
    int nlt = off[lo + 1] - off[lo];
    kb = r / nlt;
    lt = r - kb * nlt;
}

// compact (FP64) -> m-major operand rows (T = double or float).
// comp: component of the alm array; kind 0 = plain (T or E), 1 = B stored as B' = i a_B.
template <typename T>
__global__ __launch_bounds__(NT) void k_to_mmajor(AlmArgs a)
{
    __shared__ double tile[TLB][2 * TK + 1];
    const int comp = a.comp0 + blockIdx.y;
    const int kind = (a.spin == 2 && comp == 2) ? 1 : 0;
    int m, lt, kb;
    decode(a.tileoff, a.lmax, a.mlist, a.nlist, a.kblocks, blockIdx.x, m, lt, kb);
    const int L = a.lmax;
    const int lb = lbase(a.spin, m);
    const int l0 = lb + lt * TLB;
    const int64_t csz = (int64_t)(L + 1) * (L + 1);
    // Every load of a thread is issued before the first is used: addresses are
    // clamped into the arrays (so the loads need no predicate) and the values
    // that lie outside the tile are replaced by zero afterwards.  B' = i a_B takes
    // Re B' = -Im a_B and Im B' = Re a_B (the parts swap); m = 0 has no Im slot.
    double v[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int e = (int)threadIdx.x + i * NT;
        const int part = e / (TK * TLB), kk = (e / TLB) % TK, li = e % TLB;
        const int l = min(l0 + li, L), k = min(kb * TK + kk, a.nmaps - 1);
        const int src = kind ? (part ^ 1) : part;
        const int64_t o = calm(L, l, m, (src && m == 0) ? 0 : src);
        v[i] = a.alm_in[(int64_t)k * a.almstride + comp * csz + o];
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int e = (int)threadIdx.x + i * NT;
        const int part = e / (TK * TLB), kk = (e / TLB) % TK, li = e % TLB;
        const int src = kind ? (part ^ 1) : part;
        const bool live = l0 + li <= L && kb * TK + kk < a.nmaps && !(src && m == 0);
        const double x = (kind && part == 0) ? -v[i] : v[i];
        tile[li][2 * kk + part] = live ? x : 0.0;
    }
    __syncthreads();
    T* A = static_cast<T*>(a.Aop) + comp * a.acomp + (a.rowoff[m] + (l0 - lb)) * a.ldx + kb * 2 * TK;
    if constexpr (sizeof(T) == 4) {
        // four columns per lane, one 16-byte store (4-byte stores left the kernel
        // latency-bound); rows start on 64-column boundaries of a 256-byte aligned
        // workspace, so every vector is aligned
        struct alignas(16) V4 { T v[4]; };
#pragma unroll
        for (int i = 0; i < PER / 4; ++i) {
            const int e = (int)threadIdx.x + i * NT;
            const int li = e / (TK / 2), c = 4 * (e % (TK / 2));
            if (l0 + li > L) continue;
            V4 w;
#pragma unroll
            for (int q = 0; q < 4; ++q) w.v[q] = (T)tile[li][c + q];
            *reinterpret_cast<V4*>(A + (int64_t)li * a.ldx + c) = w;
        }
    } else if constexpr (__is_same(T, uint64_t)) {
        // split-BF16 words: two columns per lane, one 16-byte store
        struct alignas(16) W2 { uint64_t v[2]; };
#pragma unroll
        for (int i = 0; i < PER / 2; ++i) {
            const int e = (int)threadIdx.x + i * NT;
            const int li = e / TK, c = 2 * (e % TK);
            if (l0 + li > L) continue;
            W2 w;
            w.v[0] = pack_bf16_triple((float)tile[li][c]);
            w.v[1] = pack_bf16_triple((float)tile[li][c + 1]);
            *reinterpret_cast<W2*>(A + (int64_t)li * a.ldx + c) = w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = (int)threadIdx.x + i * NT;
            const int li = e / (2 * TK), c = e % (2 * TK);
            if (l0 + li > L) continue;
            A[(int64_t)li * a.ldx + c] = (T)tile[li][c];
        }
    }
}

// m-major rows -> compact (FP64): alm = scale * A (or alm += scale * A).
// kind 1 converts B' back: Re a_B = Im B', Im a_B = -Re B'.  Spin-2 components
// have no l < 2 coefficients: the first tile of m < 2 clears them (store mode).
// TO != void: also write scale * rows as the alm2map operand of the same update
// (at Aop, in TO's format), from the tile already in LDS.
template <typename T, typename TO = void>
__global__ __launch_bounds__(NT) void k_from_mmajor(AlmArgs a)
{
    __shared__ double tile[TLB][2 * TK + 1];
    const int comp = a.comp0 + blockIdx.y;
    const int kind = (a.spin == 2 && comp == 2) ? 1 : 0;
    int m, lt, kb;
    decode(a.tileoff, a.lmax, a.mlist, a.nlist, a.kblocks, blockIdx.x, m, lt, kb);
    const int L = a.lmax;
    const int lb = lbase(a.spin, m);
    const int l0 = lb + lt * TLB;
    const int64_t csz = (int64_t)(L + 1) * (L + 1);
    const T* A = static_cast<const T*>(a.A) + comp * a.acomp + (a.rowoff[m] + (l0 - lb)) * a.ldx + kb * 2 * TK;
    // all loads of a thread first (rows clamped into the m's block, rows past
    // lmax then read as zero), as in k_to_mmajor
    if constexpr (sizeof(T) == 4) {
        // four columns per lane, one 16-byte load (aligned as in k_to_mmajor)
        float4 v[PER / 4];
#pragma unroll
        for (int i = 0; i < PER / 4; ++i) {
            const int e = (int)threadIdx.x + i * NT;
            const int li = e / (TK / 2), c = 4 * (e % (TK / 2));
            v[i] = *reinterpret_cast<const float4*>(A + (int64_t)min(li, L - l0) * a.ldx + c);
        }
#pragma unroll
        for (int i = 0; i < PER / 4; ++i) {
            const int e = (int)threadIdx.x + i * NT;
            const int li = e / (TK / 2), c = 4 * (e % (TK / 2));
            const bool live = l0 + li <= L;
            tile[li][c] = live ? v[i].x : 0.0;
            tile[li][c + 1] = live ? v[i].y : 0.0;
            tile[li][c + 2] = live ? v[i].z : 0.0;
            tile[li][c + 3] = live ? v[i].w : 0.0;
        }
    } else {
        T v[PER];
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = (int)threadIdx.x + i * NT;
            const int li = e / (2 * TK), c = e % (2 * TK);
            v[i] = A[(int64_t)min(li, L - l0) * a.ldx + c];
        }
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = (int)threadIdx.x + i * NT;
            const int li = e / (2 * TK), c = e % (2 * TK);
            tile[li][c] = (l0 + li <= L) ? (double)v[i] : 0.0;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int e = (int)threadIdx.x + i * NT;
        const int part = e / (TK * TLB);
        const int kk = (e / TLB) % TK;
        const int li = e % TLB;
        const int l = l0 + li, k = kb * TK + kk;
        if (l > L || k >= a.nmaps) continue;
        double* base = a.alm_out + (int64_t)k * a.almstride + comp * csz;
        double v;
        int64_t o;
        if (kind == 0) {
            v = tile[li][2 * kk + part];
            o = calm(L, l, m, part);
        } else if (part == 0) {  // Re a_B = Im B'
            v = tile[li][2 * kk + 1];
            o = calm(L, l, m, 0);
        } else {                 // Im a_B = -Re B'
            v = -tile[li][2 * kk];
            o = calm(L, l, m, 1);
        }
        if (o < 0) continue;
        v *= a.scale;
        if (a.accumulate) base[o] += v; else base[o] = v;
    }
    if constexpr (!__is_same(TO, void)) {
        // tile reads all happened before the barrier above (Aop is A itself
        // unless the operand words have a region of their own)
        TO* out = static_cast<TO*>(a.Aop) + comp * a.acomp + (a.rowoff[m] + (l0 - lb)) * a.ldx + kb * 2 * TK;
        const int drop = (m == 0) ? (kind == 0 ? 1 : 0) : -1;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = (int)threadIdx.x + i * NT;
            const int li = e / (2 * TK), c = e % (2 * TK);
            if (l0 + li > L) continue;
            const bool keep = (c & 1) != drop && kb * TK + (c >> 1) < a.nmaps;
            const double v = keep ? a.scale * tile[li][c] : 0.0;
            if constexpr (__is_same(TO, uint64_t)) out[(int64_t)li * a.ldx + c] = pack_bf16_triple((float)v);
            else out[(int64_t)li * a.ldx + c] = (TO)v;
        }
    }
    if (a.spin == 2 && !a.accumulate && m < 2 && lt == 0) {
        for (int e = threadIdx.x; e < TK * 2 * 2; e += NT) {
            const int kk = e / 4, part = (e >> 1) & 1, l = m + (e & 1);
            const int k = kb * TK + kk;
            if (l >= 2 || k >= a.nmaps) continue;
            int64_t o = calm(L, l, m, part);
            if (o >= 0) a.alm_out[(int64_t)k * a.almstride + comp * csz + o] = 0.0;
        }
    }
}

// Immediate iteration: the map2alm rows of the listed m become scale * A, in
// place; the parts the compact storage has no slot for (Im of T and E at m = 0,
// Re of B' = i a_B at m = 0) and the padding maps are zeroed.  scale = 0 clears
// the rows without reading them (before a split map2alm adds into them).
template <typename T>
__global__ __launch_bounds__(NT) void k_level_rows(AlmArgs a)
{
    const int comp = a.comp0 + blockIdx.y;
    const int kind = (a.spin == 2 && comp == 2) ? 1 : 0;
    int m, lt, kb;
    decode(a.tileoff, a.lmax, a.mlist, a.nlist, a.kblocks, blockIdx.x, m, lt, kb);
    const int L = a.lmax;
    const int lb = lbase(a.spin, m);
    const int l0 = lb + lt * TLB;
    const int64_t o0 = comp * a.acomp + (a.rowoff[m] + (l0 - lb)) * a.ldx + kb * 2 * TK;
    T* rows = static_cast<T*>(a.A) + o0;
    const int drop = (m == 0) ? (kind == 0 ? 1 : 0) : -1;  // part without a compact slot
    for (int e = threadIdx.x; e < 2 * TK * TLB; e += NT) {
        const int li = e / (2 * TK), c = e % (2 * TK);
        if (l0 + li > L) continue;
        const int64_t o = (int64_t)li * a.ldx + c;
        const bool keep = (c & 1) != drop && kb * TK + (c >> 1) < a.nmaps;
        rows[o] = (keep && a.scale != 0.0) ? (T)(a.scale * (double)rows[o]) : (T)0;
    }
}

// Zero len doubles at base + i*stride for i < rows (components a selective
// transform leaves out); a kernel rather than a memset so the call may be captured.
__global__ __launch_bounds__(NT) void k_zero_strided(double* base, int rows, int64_t stride, int64_t len)
{
    for (int i = blockIdx.y; i < rows; i += gridDim.y) {
        double* r = base + (int64_t)i * stride;
        for (int64_t j = (int64_t)blockIdx.x * NT + threadIdx.x; j < len; j += (int64_t)gridDim.x * NT) r[j] = 0.0;
    }
}

}  // namespace

hipError_t launch_zero_strided(double* base, int rows, int64_t stride, int64_t len, hipStream_t st)
{
    if (rows <= 0 || len <= 0) return hipSuccess;
    const int64_t bx = std::min<int64_t>((len + NT - 1) / NT, 1024);
    const dim3 grid((unsigned)bx, (unsigned)std::min(rows, 1024));
    hipLaunchKernelGGL(k_zero_strided, grid, dim3(NT), 0, st, base, rows, stride, len);
    return hipGetLastError();
}

hipError_t launch_level_rows(const AlmArgs& a, int ncompl, int prec, hipStream_t st)
{
    dim3 grid(a.ntiles * a.kblocks, ncompl);
    if (prec == 0) hipLaunchKernelGGL(k_level_rows<double>, grid, dim3(NT), 0, st, a);
    else hipLaunchKernelGGL(k_level_rows<float>, grid, dim3(NT), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_level_commit(const AlmArgs& a, int ncompl, int prec, hipStream_t st)
{
    dim3 grid(a.ntiles * a.kblocks, ncompl);
    if (prec == 0) hipLaunchKernelGGL((k_from_mmajor<double, double>), grid, dim3(NT), 0, st, a);
    else if (prec == 2) hipLaunchKernelGGL((k_from_mmajor<float, uint64_t>), grid, dim3(NT), 0, st, a);
    else hipLaunchKernelGGL((k_from_mmajor<float, float>), grid, dim3(NT), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_alm_to_mmajor(const AlmArgs& a, int ncompl, int prec, hipStream_t st)
{
    dim3 grid(a.ntiles * a.kblocks, ncompl);
    if (prec == 0) hipLaunchKernelGGL(k_to_mmajor<double>, grid, dim3(NT), 0, st, a);
    else if (prec == 2) hipLaunchKernelGGL(k_to_mmajor<uint64_t>, grid, dim3(NT), 0, st, a);  // split-BF16 words
    else hipLaunchKernelGGL(k_to_mmajor<float>, grid, dim3(NT), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_alm_from_mmajor(const AlmArgs& a, int ncompl, int prec, hipStream_t st)
{
    dim3 grid(a.ntiles * a.kblocks, ncompl);
    if (prec == 0) hipLaunchKernelGGL(k_from_mmajor<double>, grid, dim3(NT), 0, st, a);
    else hipLaunchKernelGGL(k_from_mmajor<float>, grid, dim3(NT), 0, st, a);
    return hipGetLastError();
}

}  // namespace sht
