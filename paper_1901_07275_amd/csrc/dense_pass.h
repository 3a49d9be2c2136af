// Dense axis pass on the matrix cores: for short lines the plan keeps the
// whole n x n transform matrix (the direct block covers every degree, no FFT
// terms), and a pass over many lines is a small matrix product
//   forward:  out[line][j] = sum_k WV[k][j] in[line][k]   (Out = In * WV)
//   inverse:  out[line][k] = sum_j WV[k][j] in[line][j]   (Out = In * WV^T)
// computed with 16 x 16 x 4 MFMA tiles: 16 lines by 16 outputs per wave,
// accumulating over the degrees four at a time (fp32 tiles for the fp32-bulk
// path, fp64 tiles for the fp64 path).  A block first stages its 16 input
// lines in LDS, so passes that work in place are safe.
#pragma once

#include <hip/hip_runtime.h>

#include "launch.h"

namespace jt {
namespace dev {

typedef float mf32x4 __attribute__((ext_vector_type(4)));
typedef double mf64x4 __attribute__((ext_vector_type(4)));

template <class T>
struct Mfma;

// Lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; it receives
// D[4 (l / 16) + i][l % 16] (fp32) or D[l / 16 + 4 i][l % 16] (fp64), i < 4.
template <>
struct Mfma<float> {
    using acc = mf32x4;
    static __device__ __forceinline__ acc step(float a, float b, acc c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int i) { return 4 * (lane >> 4) + i; }
};
template <>
struct Mfma<double> {
    using acc = mf64x4;
    static __device__ __forceinline__ acc step(double a, double b, acc c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int i) { return (lane >> 4) + 4 * i; }
};

// Lines of a dense pass held by one block, and the longest dense line.
constexpr int kDenseLines = 16;
constexpr int kDenseMax = 1024;
// LDS row stride (elements) of the staged lines: odd, against bank conflicts.
__host__ __device__ constexpr int dense_ld(int n) { return n | 1; }
// Dynamic LDS a dense block needs.
__host__ __device__ constexpr size_t dense_lds_bytes(int n, bool fp32)
{
    return (size_t)kDenseLines * (size_t)dense_ld(n) * (fp32 ? 4 : 8);
}

// All threads of the block: lines line0 .. line0 + 15 (those below line_end).
// smem holds dense_lds_bytes(n) bytes.
template <class T, int FWD>
__device__ __forceinline__ void dense_lines(const AxisLaunch &a, unsigned line0, unsigned line_end, T *smem)
{
    using M = Mfma<T>;
    const int n = a.n, ld = dense_ld(n);
    const unsigned stride = (unsigned)a.stride;
    // stage the lines (zero past the end); consecutive threads read along the
    // axis for contiguous lines, across lines for strided ones
    const int total = kDenseLines * n;
    for (int e = (int)threadIdx.x; e < total; e += (int)blockDim.x) {
        int r, k;
        if (stride == 1u) {
            r = e / n;
            k = e - r * n;
        } else {
            k = e / kDenseLines;
            r = e - k * kDenseLines;
        }
        const unsigned line = line0 + (unsigned)r;
        T v = 0;
        if (line < line_end) {
            const unsigned outer = line / stride;
            const unsigned idx = outer * (unsigned)n * stride + (line - outer * stride) + (unsigned)k * stride;
            v = a.in_f64 ? (T) reinterpret_cast<const double *>(a.in)[idx]
                         : (T) reinterpret_cast<const float *>(a.in)[idx];
        }
        smem[r * ld + k] = v;
    }
    __syncthreads();
    const T *wv = reinterpret_cast<const T *>(a.wv);
    const int lane = (int)(threadIdx.x & 63u);
    const int waves = (int)(blockDim.x >> 6);
    const int arow = lane & 15, kl = lane >> 4;
    for (int c0 = 16 * (int)(threadIdx.x >> 6); c0 < n; c0 += 16 * waves) {
        const int bcol = c0 + (lane & 15);
        const bool bcol_ok = bcol < n;
        typename M::acc c = {0, 0, 0, 0};
        for (int k0 = 0; k0 < n; k0 += 4) {
            const int k = k0 + kl;
            T av = 0, bv = 0;
            if (k < n) {
                av = smem[arow * ld + k];
                if (bcol_ok) bv = FWD ? wv[k * n + bcol] : wv[bcol * n + k];
            }
            c = M::step(av, bv, c);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const unsigned line = line0 + (unsigned)M::row(lane, i);
            if (line < line_end && bcol_ok) {
                const unsigned outer = line / stride;
                const unsigned o = outer * (unsigned)n * stride + (line - outer * stride) + (unsigned)bcol * stride;
                if (a.out_f64)
                    reinterpret_cast<double *>(a.out)[o] = (double)c[i];
                else
                    reinterpret_cast<float *>(a.out)[o] = (float)c[i];
            }
        }
    }
}

}  // namespace dev
}  // namespace jt
