// Dense axis pass on the matrix cores: for short lines the plan keeps the
// whole n x n transform matrix (the direct block covers every degree, no FFT
// terms), and a pass over many lines is a small matrix product
//   forward:  out[line][j] = sum_k WV[k][j] in[line][k]   (Out = In * WV)
//   inverse:  out[line][k] = sum_j WV[k][j] in[line][j]   (Out = In * WV^T)
// computed with 16 x 16 x 4 MFMA tiles (16 lines by 16 outputs), accumulating
// over the degrees four at a time (fp32 tiles for the fp32-bulk path, fp64
// tiles for the fp64 path).  A block first stages its 16, 32 or 64 input
// lines in LDS (as many as fit), so passes that work in place are safe.
#pragma once

#include <hip/hip_runtime.h>

#include "dense_shape.h"
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

// All threads of the block: lines line0 .. line0 + rows - 1 (those below
// line_end), rows = 16 * RT.  smem holds dense_lds_bytes(n, rows) bytes.  Each
// wave takes 16-column tiles of the output and computes the RT row tiles of
// a column tile together, so a loaded matrix column serves RT MFMAs.
template <class T, int FWD, int RT>
__device__ __forceinline__ void dense_tiles(const AxisLaunch &a, unsigned line0, unsigned line_end, T *smem)
{
    using M = Mfma<T>;
    constexpr int R = 16 * RT;
    const int n = a.n, ld = dense_ld(n);
    const unsigned stride = (unsigned)a.stride;
    // stage the lines (zero past the end); consecutive threads read along the
    // axis for contiguous lines, across lines for strided ones
    const int total = R * n;
    for (int e = (int)threadIdx.x; e < total; e += (int)blockDim.x) {
        int r, k;
        if (stride == 1u) {
            r = e / n;
            k = e - r * n;
        } else {
            k = e / R;
            r = e - k * R;
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
        const typename M::acc zero = {0, 0, 0, 0};
        typename M::acc c[RT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) c[rt] = zero;
        // eight k-steps (32 degrees) at a time: their matrix values are
        // requested together, so the MFMAs wait for one L2 round trip per
        // eight steps instead of one per step; out-of-range operands load
        // from a clamped address and are replaced by zero (no branches)
        constexpr int U = 8;
        for (int k0 = 0; k0 < n; k0 += 4 * U) {
            T bv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int k = k0 + 4 * u + kl;
                const bool ok = k < n && bcol_ok;
                const T w = wv[ok ? (FWD ? k * n + bcol : bcol * n + k) : 0];
                bv[u] = ok ? w : (T)0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int k = k0 + 4 * u + kl;
                const bool k_ok = k < n;
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) {
                    const T a = smem[(rt * 16 + arow) * ld + (k_ok ? k : 0)];
                    c[rt] = M::step(k_ok ? a : (T)0, bv[u], c[rt]);
                }
            }
        }
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const unsigned line = line0 + (unsigned)(rt * 16 + M::row(lane, i));
                if (line < line_end && bcol_ok) {
                    const unsigned outer = line / stride;
                    const unsigned o = outer * (unsigned)n * stride + (line - outer * stride) + (unsigned)bcol * stride;
                    if (a.out_f64)
                        reinterpret_cast<double *>(a.out)[o] = (double)c[rt][i];
                    else
                        reinterpret_cast<float *>(a.out)[o] = (float)c[rt][i];
                }
            }
    }
}

// Dispatch on the block's line count (16, 32 or 64).
template <class T, int FWD>
__device__ __forceinline__ void dense_lines(const AxisLaunch &a, unsigned line0, unsigned line_end, int rows,
                                            T *smem)
{
    if (rows == 64) dense_tiles<T, FWD, 4>(a, line0, line_end, smem);
    else if (rows == 32) dense_tiles<T, FWD, 2>(a, line0, line_end, smem);
    else dense_tiles<T, FWD, 1>(a, line0, line_end, smem);
}

}  // namespace dev
}  // namespace jt
