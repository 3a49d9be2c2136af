// Internal interface between the C ABI layer and the HIP axis-pass kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace jt {

// One axis pass over all lines of a row-major tensor.  A line is the set of
// n elements base + k*stride (k < n) with
//   line = outer * stride + inner,  base = outer * n * stride + inner.
struct AxisLaunch {
    const void *in = nullptr;   // input tensor (device)
    void *out = nullptr;        // output tensor (device), may alias `in`
    int in_f64 = 1, out_f64 = 1;
    long long lines = 0;        // number of lines
    long long stride = 1;       // element stride along the axis
    int n = 0, L = 0, nu0 = 0, rank = 0;
    int max_per_bin = 0;        // most nodes sharing one DFT bin
    int forward = 1;            // 1: W J alpha, 0: (W J)^T g
    int fp32 = 0;               // 0: fp64 arithmetic, 1: fp32 bulk (fp64 accumulation)
    // factor sections (device pointers inside the bound plan blob)
    const void *tw = nullptr;    // L complex, exp(+2 pi i p / L)
    const int *bins = nullptr;   // n
    const int *binptr = nullptr; // L/2 + 2
    const void *wv = nullptr;    // nu0 x n   (WV[k*n + j])
    const void *u = nullptr;     // rank x n complex
    const void *v = nullptr;     // rank x L complex
};

// Launch on `stream`; returns hipSuccess or the launch error.
hipError_t launch_axis(const AxisLaunch &a, hipStream_t stream);

}  // namespace jt
