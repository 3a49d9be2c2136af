// Fused axis-pass kernels for the fast uniform Jacobi transform on gfx950.
//
// One pass applies W J_n^(a,b) (forward) or its transpose (inverse) along one
// axis of a row-major tensor, independently on every line (Section 3.1 for a
// single line; Sections 3.2-3.3 apply it axis by axis, eqs. (54)-(55),
// (59)-(60)).  Per line, the forward pass computes eq. (50):
//
//   out_j = sum_{k<nu0} (WV)_{jk} alpha_k
//         + Re sum_l u_{l,j} * y_l[m_j],   y_l[m] = sum_k v_{l,k} alpha_k e^{+2 pi i m k / L}
//
// and the inverse pass computes eq. (51):
//
//   alpha_k = sum_j (WV)_{jk} g_j                       (k < nu0)
//   alpha_k = Re sum_l v_{l,k} * Y_l[k],  Y_l[k] = sum_m e^{+2 pi i m k / L} z_l[m],
//             z_l[m] = sum_{j : m_j = m} u_{l,j} g_j     (k >= nu0)
//
// Layout of a line inside the kernel: P = L/16 lanes per line, lane p holds
// the 16 elements p + P*q (q = 0..15) in registers.  The L-point DFT is a
// Stockham radix-16 FFT (with one final radix-2/4/8 pass when log2 L is not a
// multiple of 4): the first pass starts from registers (no LDS read), the
// last pass ends in registers in the same lane-owned layout, and the passes
// in between exchange through a padded LDS line buffer.  The gather of
// y[m_j] (forward) and the bin sums of z (inverse) also go through that
// buffer.  The rank sum is accumulated in fp64 in both precisions.
#include <hip/hip_runtime.h>

#include "launch.h"

#include "dense_pass.h"
#include "fft_line.h"

namespace jt {
namespace {

using namespace dev;

// Blocks that share an XCD get neighbouring lines, so that the strided passes
// reuse cache lines within one L2.
__device__ __forceinline__ unsigned block_line(unsigned lpb)
{
    const unsigned b = blockIdx.x, g = gridDim.x;
    unsigned lb = b;
    if ((g & 7u) == 0u) lb = (b & 7u) * (g >> 3) + (b >> 3);
    return lb * lpb;
}

// The one-pass kernel: a block holds S split groups that share the same
// lines (rank split, only for lines held by a single wave).  WIDE: blocks of
// up to eight single-wave groups, for passes with too few lines to fill the
// chip (a 1D transform is one line), where more groups per line shorten it.
// Waves per SIMD the single-wave-line kernels are compiled for (1: as many
// registers as the compiler wants).
#ifndef JT_F32_FWD_MIN_WAVES
#define JT_F32_FWD_MIN_WAVES 1
#endif
#ifndef JT_F32_INV_MIN_WAVES
#define JT_F32_INV_MIN_WAVES 1
#endif
template <class T, int LOG2L, int FWD>
constexpr int min_waves()
{
    if constexpr (Geo<LOG2L>::BLOCK > 64 || sizeof(T) == 8) return 1;
    else return FWD ? JT_F32_FWD_MIN_WAVES : JT_F32_INV_MIN_WAVES;
}

template <class T, int LOG2L, int FWD, int WIDE>
__global__ void __launch_bounds__(WIDE ? 512 : (Geo<LOG2L>::BLOCK == 64 ? 256 : Geo<LOG2L>::BLOCK),
                                  (WIDE ? 1 : min_waves<T, LOG2L, FWD>()))
    axis_pass(AxisLaunch a)
{
    using G = Geo<LOG2L>;
    extern __shared__ unsigned char lds_raw[];
    cpx<T> *smem = reinterpret_cast<cpx<T> *>(lds_raw);
    const int S = (int)(blockDim.x / G::BLOCK);
    const cpx<T> *tw = reinterpret_cast<const cpx<T> *>(a.tw);
    if constexpr (tw_mode<T, LOG2L, FWD>() == 1) {
        cpx<T> *tws = smem + S * G::LPB * G::BUF;
        for (int i = (int)threadIdx.x; i < G::L; i += (int)blockDim.x) tws[i] = tw[i];
        __syncthreads();
        tw = tws;
    }
    pass_lines<T, LOG2L, FWD>(a, block_line(G::LPB), (unsigned)a.lines, S, (int)threadIdx.x / G::BLOCK,
                              (int)threadIdx.x % G::BLOCK, smem, tw);
}

// Dense pass (every degree in the direct block): 16, 32 or 64 lines per
// block of four waves, on the matrix cores.
template <class T, int FWD>
__global__ void __launch_bounds__(256) dense_pass(AxisLaunch a)
{
    extern __shared__ unsigned char lds_raw[];
    const int rows = dense_rows(a.n, (int)sizeof(T), kDenseLdsOnePass, a.lines);
    const unsigned line0 = blockIdx.x * (unsigned)rows;
    const unsigned end = line0 + rows < (unsigned)a.lines ? line0 + rows : (unsigned)a.lines;
    dense_lines<T, FWD>(a, line0, end, rows, reinterpret_cast<T *>(lds_raw));
}

template <class T>
hipError_t launch_dense(const AxisLaunch &a, hipStream_t s)
{
    const int rows = dense_rows(a.n, (int)sizeof(T), kDenseLdsOnePass, a.lines);
    const long long blocks = (a.lines + rows - 1) / rows;
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    const size_t lds = dense_lds_bytes(a.n, rows, (int)sizeof(T));
    static bool attr_set[2] = {false, false};
    if (!attr_set[a.forward ? 1 : 0]) {
        const void *fn = a.forward ? reinterpret_cast<const void *>(&dense_pass<T, 1>)
                                   : reinterpret_cast<const void *>(&dense_pass<T, 0>);
        (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        (void)hipGetLastError();
        attr_set[a.forward ? 1 : 0] = true;
    }
    if (a.forward)
        hipLaunchKernelGGL((dense_pass<T, 1>), dim3((unsigned)blocks), dim3(256), lds, s, a);
    else
        hipLaunchKernelGGL((dense_pass<T, 0>), dim3((unsigned)blocks), dim3(256), lds, s, a);
    return hipGetLastError();
}

// Rank split S for lines held by a single wave (S waves share each line and
// take every S-th term).  A pass costs about rounds(S) * ceil(rank / S) term
// iterations, rounds(S) being how often its waves (blocks * S) fill the chip
// at two waves per SIMD, the occupancy the kernels' register use allows.
// Ties go to S = 2 in fp32; in fp64 to the larger S when the waves fill the
// chip at most twice (balance across SIMDs) and to the smaller otherwise
// (less partial-sum reduction).  At most 4 ways, never beyond the rank.
// Measured on 1024^2 (ranks 19, 18) and 256^3 (rank 10): fp32 picks 2
// everywhere, fp64 2 and 4 on 1024^2 and 1 on 256^3.  Passes of at most 256
// blocks (fewer than the compute units) may go to 8 ways in the wide kernel.
constexpr long long kWideBlocks = 256;
int rank_split(long long blocks, int rank, bool fp32)
{
    const long long slots = 2LL * 4 * 256;
    const int smax = blocks <= kWideBlocks ? 8 : 4;
    int best = 1;
    long long best_cost = -1;
    for (int S = 1; S <= smax && S <= (rank > 1 ? rank : 1); ++S) {
        const long long rounds = (blocks * S + slots - 1) / slots;
        const long long cost = rounds * ((rank + S - 1) / S);
        bool take = best_cost < 0 || cost < best_cost;
        if (cost == best_cost) take = fp32 ? (S > 2 ? S - 2 : 2 - S) < (best > 2 ? best - 2 : 2 - best) : rounds <= 2;
        if (take) {
            best = S;
            best_cost = cost;
        }
    }
    return best;
}

template <class T, int LOG2L>
hipError_t launch_t(const AxisLaunch &a, hipStream_t s)
{
    using G = Geo<LOG2L>;
    const long long blocks = (a.lines + G::LPB - 1) / G::LPB;
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    const int S = G::BLOCK == 64 ? rank_split(blocks, a.rank, sizeof(T) == 4) : 1;
    const int twm = a.forward ? tw_mode<T, LOG2L, 1>() : tw_mode<T, LOG2L, 0>();
    const size_t lds = ((size_t)S * G::LPB * G::BUF + (twm == 1 ? G::L : 0)) * sizeof(cpx<T>);
    const dim3 grid((unsigned)blocks), block((unsigned)(G::BLOCK * S));
    const void *fn;
    int which;
    if constexpr (G::BLOCK == 64) {
        const bool wide = S > 4;
        which = (wide ? 2 : 0) + (a.forward ? 1 : 0);
        fn = wide ? (a.forward ? reinterpret_cast<const void *>(&axis_pass<T, LOG2L, 1, 1>)
                               : reinterpret_cast<const void *>(&axis_pass<T, LOG2L, 0, 1>))
                  : (a.forward ? reinterpret_cast<const void *>(&axis_pass<T, LOG2L, 1, 0>)
                               : reinterpret_cast<const void *>(&axis_pass<T, LOG2L, 0, 0>));
    } else {
        which = a.forward ? 1 : 0;
        fn = a.forward ? reinterpret_cast<const void *>(&axis_pass<T, LOG2L, 1, 0>)
                       : reinterpret_cast<const void *>(&axis_pass<T, LOG2L, 0, 0>);
    }
    // allow dynamic LDS beyond 64 KB (gfx950 has 160 KB per CU); once per kernel
    static bool attr_set[4] = {false, false, false, false};
    if (!attr_set[which]) {
        (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        (void)hipGetLastError();
        attr_set[which] = true;
    }
    if constexpr (G::BLOCK == 64) {
        if (which >= 2) {
            if (a.forward)
                hipLaunchKernelGGL((axis_pass<T, LOG2L, 1, 1>), grid, block, lds, s, a);
            else
                hipLaunchKernelGGL((axis_pass<T, LOG2L, 0, 1>), grid, block, lds, s, a);
            return hipGetLastError();
        }
    }
    if (a.forward)
        hipLaunchKernelGGL((axis_pass<T, LOG2L, 1, 0>), grid, block, lds, s, a);
    else
        hipLaunchKernelGGL((axis_pass<T, LOG2L, 0, 0>), grid, block, lds, s, a);
    return hipGetLastError();
}

template <class T>
hipError_t launch_prec(const AxisLaunch &a, hipStream_t s)
{
    if (a.nu0 == a.n) {
        if (a.n > kDenseMax) return hipErrorInvalidValue;
        return launch_dense<T>(a, s);
    }
    switch (a.L) {
    case 64: return launch_t<T, 6>(a, s);
    case 128: return launch_t<T, 7>(a, s);
    case 256: return launch_t<T, 8>(a, s);
    case 512: return launch_t<T, 9>(a, s);
    case 1024: return launch_t<T, 10>(a, s);
    case 2048: return launch_t<T, 11>(a, s);
    case 4096: return launch_t<T, 12>(a, s);
    case 8192: return launch_t<T, 13>(a, s);
    default: break;
    }
    if constexpr (sizeof(T) == 4) {
        if (a.L == 16384) return launch_t<T, 14>(a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_axis(const AxisLaunch &a, hipStream_t stream)
{
    return a.fp32 ? launch_prec<float>(a, stream) : launch_prec<double>(a, stream);
}

}  // namespace jt
