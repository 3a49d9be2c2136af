// Persistent batch kernel: one launch runs every axis pass of every item of
// a batch of independent transforms (uneven n, d and (a, b)), pulling work
// units from a device queue.  Each unit runs the same fused per-line body as
// the one-pass kernel (eqs. (50) and (51)).
//
// Block shape: 512 threads (8 waves).  For a unit of FFT length L the block
// is cut into groups of Geo<L>::BLOCK threads (one wave, or P = L/16 lanes
// for longer lines; a 16384-point line puts two lanes on each of the 512
// threads); S consecutive groups share one set of LPB lines (rank split), so
// a unit holds (groups / S) * LPB lines.
#include <hip/hip_runtime.h>

#include <mutex>

#include "batch.h"
#include "dense_pass.h"
#include "fft_line.h"

namespace jt {

// The counters of runs that bring none of their own (jt_batch_run_static).
// In host code this name is only a handle for the symbol lookup below; the
// array's device address comes from hipGetSymbolAddress, per device.
static __device__ __align__(256) uint32_t scratch[kStaticCounterWords];

namespace {

using namespace dev;

// Bounded wait for a pass to complete (about 4 s at most): on timeout the
// error word gets kBatchErrWaitTimeout and the unit proceeds, so the grid
// always drains.
__device__ void wait_done(const uint32_t *ctr, uint32_t need, uint32_t *err)
{
    for (uint32_t spins = 0;; ++spins) {
        const uint32_t v = __hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        if (v >= need) return;
        if (spins > (1u << 23)) {
            atomicOr(err, kBatchErrWaitTimeout);
            return;
        }
        __builtin_amdgcn_s_sleep(8);
    }
}

// The unit functions receive the descriptors by reference, so the compiler
// cannot see that every field is the same in all lanes; reading each one
// through readfirstlane keeps it in scalar registers (scalar loop control and
// address arithmetic, fewer vector registers).
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
template <class P>
__device__ __forceinline__ P *uni(P *p)
{
    const unsigned long long v = reinterpret_cast<unsigned long long>(p);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return reinterpret_cast<P *>(((unsigned long long)hi << 32) | lo);
}

// One variant per length, kept out of line: inlined together, the nine
// variants of both directions would share one register allocation and spill.
__device__ __forceinline__ AxisLaunch launch_of(const PassDesc &d, const BatchLaunch &b, bool fp32)
{
    AxisLaunch a;
    a.in = uni((d.in_from_out ? (const unsigned char *)b.out_base : b.in_base) + d.in_off);
    a.out = uni(b.out_base + d.out_off);
    a.in_f64 = uni(d.in_f64);
    a.out_f64 = uni(d.out_f64);
    a.lines = uni(d.lines);
    a.stride = uni(d.stride);
    a.n = uni(d.n);
    a.L = uni(d.L);
    a.nu0 = uni(d.nu0);
    a.rank = uni(d.rank);
    a.max_per_bin = uni(d.max_per_bin);
    a.forward = uni(d.forward);
    a.fp32 = fp32;
    a.tw = uni(d.tw);
    a.bins = uni(d.bins);
    a.binptr = uni(d.binptr);
    a.wv = uni(d.wv);
    a.u = uni(d.u);
    a.v = uni(d.v);
    return a;
}

// A dense unit: 16 lines on the matrix cores (every degree in the direct block).
template <class T>
__device__ __attribute__((noinline)) void run_dense(const PassDesc &d, const WorkUnit &w, const BatchLaunch &b,
                                                    cpx<T> *smem)
{
    const AxisLaunch a = launch_of(d, b, sizeof(T) == 4);
    const unsigned end = (unsigned)uni(w.line0 + w.nlines);
    const int rows = uni(d.cap);  // lines per dense unit: 16, 32 or 64
    if (a.forward)
        dense_lines<T, 1>(a, (unsigned)uni(w.line0), end, rows, reinterpret_cast<T *>(smem));
    else
        dense_lines<T, 0>(a, (unsigned)uni(w.line0), end, rows, reinterpret_cast<T *>(smem));
}

// Options of the forward FFT units (pass_lines' OPT bits).  The kernel's
// occupancy is fixed at two waves per SIMD by its block size and LDS, so
// registers up to 256 per thread cost nothing here, unlike in the one-pass
// kernel.  fp32 single-lane lines request u_l before the FFT (4096-item
// ragged 1D batch: 3.16 -> 2.99 ms) and, up to JT_BATCH_PF_V_MAX = log2 L,
// also load the next v_l during the gather (the same batch's 2D items on the
// FFT path: 21.0 -> 17.0 ms); fp64 has no registers to spare.  fp32 units
// also take the direct block in its node-contiguous form (the ragged 1D
// batch: 2.99 -> 2.80 ms; fp64 always does).
#ifndef JT_BATCH_PF_V_MAX
#define JT_BATCH_PF_V_MAX 12
#endif
#ifndef JT_BATCH_PF_U
#define JT_BATCH_PF_U 1
#endif
template <class T, int LOG2L>
constexpr int batch_fwd_opts()
{
    if constexpr (sizeof(T) != 4) return 0;
    else return (LOG2L <= JT_BATCH_PF_V_MAX ? 1 : 0) | (JT_BATCH_PF_U ? 2 : 0) | 8;
}

// Inverse FFT units: fp32 single-lane lines up to JT_BATCH_PF_INV_MAX =
// log2 L request the term's v_l before the FFT (the 4096-item ragged
// batches run inverse: 1D 3.59 -> 3.51 ms, 2D on the FFT path 24.9 -> 21.5
// ms).
#ifndef JT_BATCH_PF_INV_MAX
#define JT_BATCH_PF_INV_MAX 13
#endif
template <class T, int LOG2L>
constexpr int batch_inv_opts()
{
    return (sizeof(T) == 4 && LOG2L <= JT_BATCH_PF_INV_MAX) ? 4 : 0;
}

template <class T, int LOG2L>
__device__ __attribute__((noinline)) void run_unit(const PassDesc &d, const WorkUnit &w, const BatchLaunch &b, cpx<T> *smem)
{
    constexpr int NT = kBatchThreads;
    constexpr int VL = ((1 << LOG2L) / 16 > NT) ? ((1 << LOG2L) / 16) / NT : 1;
    using G = Geo<LOG2L, VL>;
    if constexpr (sizeof(T) == 8 && LOG2L > 13) {
        return;  // rejected on the host (the line buffer would not fit in LDS)
    } else {
        const AxisLaunch a = launch_of(d, b, sizeof(T) == 4);
        const int S = uni(w.split);
        const int wl0 = uni(w.line0);
        const int grp = (int)threadIdx.x / G::BLOCK;
        const int vb = grp / S, sgrp = grp % S;
        const unsigned line0 = (unsigned)wl0 + (unsigned)(vb * G::LPB);
        const unsigned line_end = (unsigned)(wl0 + uni(w.nlines));
        cpx<T> *vs = smem + vb * S * G::LPB * G::BUF;
        const cpx<T> *tw = reinterpret_cast<const cpx<T> *>(a.tw);
        if (a.forward)
            pass_lines<T, LOG2L, 1, VL, false, batch_fwd_opts<T, LOG2L>()>(a, line0, line_end, S, sgrp,
                                                                           (int)threadIdx.x % G::BLOCK, vs, tw);
        else
            pass_lines<T, LOG2L, 0, VL, false, batch_inv_opts<T, LOG2L>()>(a, line0, line_end, S, sgrp,
                                                                               (int)threadIdx.x % G::BLOCK, vs, tw);
    }
}

// One chunk of lines of one pass, by length class.
template <class T>
__device__ __forceinline__ void run_chunk(const PassDesc &d, const WorkUnit &w, const BatchLaunch &b, cpx<T> *smem,
                                          uint32_t *err)
{
    if (d.nu0 == d.n) {
        run_dense<T>(d, w, b, smem);
        return;
    }
    switch (d.L) {
    case 64: run_unit<T, 6>(d, w, b, smem); break;
    case 128: run_unit<T, 7>(d, w, b, smem); break;
    case 256: run_unit<T, 8>(d, w, b, smem); break;
    case 512: run_unit<T, 9>(d, w, b, smem); break;
    case 1024: run_unit<T, 10>(d, w, b, smem); break;
    case 2048: run_unit<T, 11>(d, w, b, smem); break;
    case 4096: run_unit<T, 12>(d, w, b, smem); break;
    case 8192: run_unit<T, 13>(d, w, b, smem); break;
    case 16384: run_unit<T, 14>(d, w, b, smem); break;
    default:
        if (threadIdx.x == 0) atomicOr(err, kBatchErrBadLength);
        break;
    }
}

template <class T>
__global__ void __launch_bounds__(kBatchThreads) batch_kernel(BatchLaunch b)
{
    // The line buffers start at LDS offset 0 and the dequeued unit index sits
    // after them: a static __shared__ variable would be placed first and
    // shift the dynamic buffer off 8-byte alignment, which turns every fp64
    // LDS access into a misaligned one.
    extern __shared__ unsigned char lds_raw[];
    cpx<T> *smem = reinterpret_cast<cpx<T> *>(lds_raw);
    int &s_unit = *reinterpret_cast<int *>(lds_raw + batch_lds_bytes(sizeof(T) == 4));
    uint32_t *head = b.counters;
    uint32_t *err = b.counters + 1;
    uint32_t *done = b.counters + 2;
    for (;;) {
        if (threadIdx.x == 0) s_unit = (int)atomicAdd(head, 1u);
        __syncthreads();
        const int u = s_unit;
        __syncthreads();  // every thread has read s_unit before it is overwritten
        if (u >= b.nunits) break;
        const WorkUnit w = b.units[u];
        if (w.npass > 0) {
            // a whole small item: its passes in order, every line, inside this
            // block; the barrier after each chunk also publishes its stores to
            // the block's later passes
            for (int p = w.pass; p < w.pass + w.npass; ++p) {
                const PassDesc d = b.passes[p];
                for (int l0 = 0; l0 < d.lines; l0 += d.cap) {
                    WorkUnit c;
                    c.pass = p;
                    c.line0 = l0;
                    c.nlines = d.lines - l0 < d.cap ? d.lines - l0 : d.cap;
                    c.split = d.split;
                    run_chunk<T>(d, c, b, smem, err);
                    __syncthreads();
                }
            }
            continue;
        }
        const PassDesc d = b.passes[w.pass];
        if (w.wait_pass >= 0) {
            if (threadIdx.x == 0) wait_done(done + w.wait_pass, (uint32_t)w.wait_count, err);
            __syncthreads();
            // the previous pass's results were written by other blocks (other XCDs)
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        run_chunk<T>(d, w, b, smem, err);
        if (d.publish) {
            // publish this unit's stores device-wide, then count it done
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __syncthreads();
            if (threadIdx.x == 0)
                __hip_atomic_fetch_add(done + w.pass, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __syncthreads();  // the LDS is free for the next unit
        }
    }
}

// Counters are cleared by a kernel (not a memset node), so that a captured
// graph of a run replays correctly.
__global__ void __launch_bounds__(256) clear_words(uint32_t *w, int count)
{
    for (int i = (int)threadIdx.x; i < count; i += (int)blockDim.x) w[i] = 0u;
}

template <class T>
hipError_t launch_t(const BatchLaunch &b, hipStream_t s)
{
    constexpr bool f32 = sizeof(T) == 4;
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&batch_kernel<T>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)batch_lds_total(f32));
        (void)hipGetLastError();
        attr_set = true;
    }
    hipLaunchKernelGGL(batch_kernel<T>, dim3((unsigned)b.grid), dim3(kBatchThreads), batch_lds_total(f32), s, b);
    return hipGetLastError();
}

__global__ void __launch_bounds__(64) copy_word_kernel(uint32_t *dst, const uint32_t *src)
{
    if (threadIdx.x == 0) *dst = *src;
}

}  // namespace

hipError_t static_counters(uint32_t **ptr)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static uint32_t *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = static_cast<uint32_t *>(p);
    }
    *ptr = addr[dev];
    return hipSuccess;
}

hipError_t copy_word(uint32_t *dst, const uint32_t *src, hipStream_t stream)
{
    hipLaunchKernelGGL(copy_word_kernel, dim3(1), dim3(64), 0, stream, dst, src);
    return hipGetLastError();
}

hipError_t launch_batch(const BatchLaunch &b, hipStream_t stream)
{
    if (b.nunits <= 0) return hipSuccess;
    if (b.grid <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(clear_words, dim3(1), dim3(256), 0, stream, b.counters, 2 + b.npasses);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return b.fp32 ? launch_t<float>(b, stream) : launch_t<double>(b, stream);
}

}  // namespace jt
