// Device building blocks of the axis pass, shared by the one-pass kernel and
// the persistent batch kernel: radix-16 Stockham FFT of a line held in
// registers (lane-owned layout) and the fused scale -> FFT -> gather ->
// accumulate body of eqs. (50) and (51).
#pragma once

#include <hip/hip_runtime.h>

#include "launch.h"

namespace jt {
namespace dev {


// Aligned to its size, so that LDS and global accesses of one complex value
// are single 8- or 16-byte operations with immediate offsets.
#ifndef JT_CPX_ALIGN
#define JT_CPX_ALIGN 1
#endif
template <class T>
struct alignas(JT_CPX_ALIGN ? 2 * sizeof(T) : sizeof(T)) cpx {
    T x, y;
};

template <class T>
__device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <class T>
__device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <class T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b)
{
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <class T>
__device__ __forceinline__ cpx<T> muli(cpx<T> a) { return {-a.y, a.x}; }

// exp(2 pi i e / 16) for e = 0..15
constexpr double kW16c[16] = {
    1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
    0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
    -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173,
    0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};
constexpr double kW16s[16] = {
    0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613,
    1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
    0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
    -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173};

template <class T, int E>
__device__ __forceinline__ cpx<T> w16(cpx<T> a)
{
    constexpr int e = E & 15;
    if constexpr (e == 0) {
        return a;
    } else if constexpr (e == 4) {
        return {-a.y, a.x};
    } else if constexpr (e == 8) {
        return {-a.x, -a.y};
    } else if constexpr (e == 12) {
        return {a.y, -a.x};
    } else if constexpr (e == 2 || e == 6 || e == 10 || e == 14) {
        // (c, s) with |c| = |s| = sqrt(2)/2
        constexpr T r = (T)0.70710678118654752440;
        constexpr T cs = (e == 2 || e == 14) ? r : -r;
        constexpr T sn = (e == 2 || e == 6) ? r : -r;
        return {cs * a.x - sn * a.y, sn * a.x + cs * a.y};
    } else {
        constexpr T c = (T)kW16c[e], s = (T)kW16s[e];
        return {c * a.x - s * a.y, s * a.x + c * a.y};
    }
}

// a * exp(2 pi i e / 16) for an e that is known after unrolling
template <class T>
__device__ __forceinline__ cpx<T> rot16(cpx<T> a, int e)
{
    switch (e & 15) {
    case 0: return a;
    case 1: return w16<T, 1>(a);
    case 2: return w16<T, 2>(a);
    case 3: return w16<T, 3>(a);
    case 4: return w16<T, 4>(a);
    case 5: return w16<T, 5>(a);
    case 6: return w16<T, 6>(a);
    case 7: return w16<T, 7>(a);
    case 8: return w16<T, 8>(a);
    case 9: return w16<T, 9>(a);
    case 10: return w16<T, 10>(a);
    case 11: return w16<T, 11>(a);
    case 12: return w16<T, 12>(a);
    case 13: return w16<T, 13>(a);
    case 14: return w16<T, 14>(a);
    default: return w16<T, 15>(a);
    }
}

// The value itself, hidden from the optimiser (an empty asm statement that
// claims to change it): twiddles derived from it are then recomputed in every
// pass instead of being hoisted out of the term loop, where the 27 derived
// factors of a 1024-point FFT would hold 108 extra registers in fp64.
template <class T>
__device__ __forceinline__ cpx<T> opaque(cpx<T> a)
{
    asm volatile("" : "+v"(a.x), "+v"(a.y));
    return a;
}

template <class T>
__device__ __forceinline__ cpx<T> csq(cpx<T> a)
{
    return {a.x * a.x - a.y * a.y, (T)2 * a.x * a.y};
}

template <class T>
__device__ __forceinline__ void dft2(cpx<T> &a0, cpx<T> &a1)
{
    cpx<T> t = a0;
    a0 = t + a1;
    a1 = t - a1;
}

// sign +:  X_m = sum_k a_k i^{k m}
template <class T>
__device__ __forceinline__ void dft4(cpx<T> &a0, cpx<T> &a1, cpx<T> &a2, cpx<T> &a3)
{
    cpx<T> t0 = a0 + a2, t1 = a0 - a2, t2 = a1 + a3, t3 = muli(a1 - a3);
    a0 = t0 + t2;
    a2 = t0 - t2;
    a1 = t1 + t3;
    a3 = t1 - t3;
}

// In-place 8-point DFT (sign +), natural order in and out: 8 = 2 x 4.
template <class T>
__device__ __forceinline__ void dft8(cpx<T> *v)
{
    // k = k1 + 2 k2:  4-point DFTs over k2 for k1 = 0, 1
    dft4(v[0], v[2], v[4], v[6]);
    dft4(v[1], v[3], v[5], v[7]);
    // twiddle omega_8^{k1 m2} = omega_16^{2 k1 m2}
    v[3] = w16<T, 2>(v[3]);
    v[5] = w16<T, 4>(v[5]);
    v[7] = w16<T, 6>(v[7]);
    // X[m2 + 4 m1] = 2-point DFT over k1 of Y[k1][m2] (stored at v[k1 + 2 m2])
    cpx<T> o[8];
#pragma unroll
    for (int m2 = 0; m2 < 4; ++m2) {
        cpx<T> a = v[2 * m2], b = v[2 * m2 + 1];
        o[m2] = a + b;
        o[m2 + 4] = a - b;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = o[i];
}

// In-place 16-point DFT (sign +), natural order in and out: 16 = 4 x 4.
template <class T>
__device__ __forceinline__ void dft16(cpx<T> *v)
{
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) dft4(v[k1], v[k1 + 4], v[k1 + 8], v[k1 + 12]);
    v[5] = w16<T, 1>(v[5]);
    v[9] = w16<T, 2>(v[9]);
    v[13] = w16<T, 3>(v[13]);
    v[6] = w16<T, 2>(v[6]);
    v[10] = w16<T, 4>(v[10]);
    v[14] = w16<T, 6>(v[14]);
    v[7] = w16<T, 3>(v[7]);
    v[11] = w16<T, 6>(v[11]);
    v[15] = w16<T, 9>(v[15]);
    cpx<T> o[16];
#pragma unroll
    for (int m2 = 0; m2 < 4; ++m2) {
        cpx<T> a0 = v[4 * m2], a1 = v[4 * m2 + 1], a2 = v[4 * m2 + 2], a3 = v[4 * m2 + 3];
        dft4(a0, a1, a2, a3);
        o[m2] = a0;
        o[m2 + 4] = a1;
        o[m2 + 8] = a2;
        o[m2 + 12] = a3;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = o[i];
}

template <class T, int R>
__device__ __forceinline__ void dftR(cpx<T> *v)
{
    if constexpr (R == 2) dft2(v[0], v[1]);
    else if constexpr (R == 4) dft4(v[0], v[1], v[2], v[3]);
    else if constexpr (R == 8) dft8(v);
    else dft16(v);
}

// Synchronisation of the lanes that share one line buffer.  A line of up to
// 1024 points lives in one wave: its lanes exchange data through LDS in
// program order, so a wave-scope fence (no instruction, it only stops the
// compiler from moving LDS accesses across it) is enough, and the other waves
// of the block keep running.  Longer lines span several waves and need the
// block barrier.
template <int TPL>
__device__ __forceinline__ void sync_line()
{
    if constexpr (TPL <= 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// padded LDS index: one spare slot every 16 elements
__device__ __forceinline__ int pad(int i) { return i + (i >> 4); }

// Sum v[0..K-1] over the TPL threads of one line; every thread of the line
// gets the totals.  Inside a wave: butterfly over lanes (the line's lanes
// form an aligned segment of TPL lanes).  A line over several waves adds the
// per-wave totals through red (K doubles per wave, in LDS) in wave order.
// Every thread of the line must call it.
template <int TPL, int K>
__device__ __forceinline__ void line_sum(double *v, double *red, int t)
{
    constexpr int W = TPL < 64 ? TPL : 64;
#pragma unroll
    for (int off = W / 2; off >= 1; off /= 2)
#pragma unroll
        for (int c = 0; c < K; ++c) v[c] += __shfl_xor(v[c], off, W);
    if constexpr (TPL > 64) {
        constexpr int NW = TPL / 64;
        const int w = t / 64;
        __syncthreads();  // previous readers of red are done
        if ((t & 63) == 0)
#pragma unroll
            for (int c = 0; c < K; ++c) red[w * K + c] = v[c];
        __syncthreads();
#pragma unroll
        for (int c = 0; c < K; ++c) {
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < NW; ++i) s += red[i * K + c];
            v[c] = s;
        }
    }
}

// Four consecutive values from a 16-byte aligned address (global or LDS).
template <class T>
__device__ __forceinline__ void load4(const T *p, T (&o)[4])
{
    if constexpr (sizeof(T) == 4) {
        const float4 v = *reinterpret_cast<const float4 *>(p);
        o[0] = v.x, o[1] = v.y, o[2] = v.z, o[3] = v.w;
    } else {
        const double2 a = reinterpret_cast<const double2 *>(p)[0], b = reinterpret_cast<const double2 *>(p)[1];
        o[0] = a.x, o[1] = a.y, o[2] = b.x, o[3] = b.y;
    }
}

// Shape of one line of length L = 2^LOG2L: P = L/16 lanes, each holding 16
// elements.  A thread carries VL lanes (p and p + TPL, ...), so a line takes
// TPL = P / VL threads; lines shorter than a wave share one (LPB lines per
// group of BLOCK threads).
template <int LOG2L, int VL = 1>
struct Geo {
    static constexpr int L = 1 << LOG2L;
    static constexpr int P = L / 16;                     // lanes per line
    static constexpr int TPL = P / VL;                   // threads per line
    static constexpr int S16 = LOG2L / 4;                // radix-16 passes
    static constexpr int F = LOG2L % 4;
    static constexpr int RF = 1 << F;                    // final radix (1: none)
    static constexpr int NMID = S16 - 1;                 // radix-16 passes after the first
    static constexpr int BLOCK = (TPL < 64) ? 64 : TPL;  // threads per group
    static constexpr int LPB = BLOCK / TPL;              // lines per group
    static constexpr int BUF = L + L / 16;               // padded line buffer (complex)
    static_assert(VL == 1 || TPL >= 64, "several lanes per thread only for lines spanning whole waves");
};

// Twiddles of all passes after the first.  They depend only on the lane, so
// the fp32 kernels keep them in registers for the whole kernel; the fp64
// kernels (twice the register cost) and blocks of 512+ threads read them from
// the L-entry table when a pass needs them.
// Where the per-pass twiddles come from: 0 = registers (loaded once), 1 = a
// copy of the table in LDS (loaded once per block), 2 = the table in global
// memory (L1/L2 resident), 3 = computed in registers from two values per lane
// loaded once: the twiddles of a radix-16 pass are the powers w^r (r < 16) of
// one root of unity w per lane, built by squarings and products (at most four
// roundings deep), and those of the final radix-2/4/8 pass are b^r times a
// sixteenth root of unity known at compile time, with b = exp(2 pi i p / L).
// Loading a twiddle per factor held the fp64 kernels at 256 registers, where
// the compiler issues each load and waits for it before the next (27
// round trips to L1/L2 per FFT); mode 3 needs no loads after the first and
// frees the registers that held the 27 load addresses.
#ifndef JT_TW_MODE_F64
#define JT_TW_MODE_F64 3
#endif
#ifndef JT_TW_MODE_F32_FWD
#define JT_TW_MODE_F32_FWD 3
#endif
// fp64 lines of up to 256 points (one radix-16 pass after the first, many
// lines per pass): computed twiddles in both directions, measured on 256^3.
// Forward passes took 532 us with the twiddles from global memory against
// 980 us computed when first measured; with the node-contiguous direct
// block they take 500-520 us from global memory and 465-478 us computed.
// Inverse passes: 1081 against 1130 us, computed ones faster.
#ifndef JT_TW_MODE_F64_SHORT_FWD
#define JT_TW_MODE_F64_SHORT_FWD 3
#endif
#ifndef JT_TW_MODE_F64_SHORT_INV
#define JT_TW_MODE_F64_SHORT_INV 3
#endif
// fp32 inverse passes over lines of up to 256 points: computed twiddles
// (mode 3) keep the kernel at 162 registers, three waves per SIMD (on
// 1024-point lines the same change, for three waves there too, was measured
// slower: 59/64 -> 85/99 us per inverse pass)
#ifndef JT_TW_MODE_F32_SHORT_INV
#define JT_TW_MODE_F32_SHORT_INV 3
#endif
template <class T, int LOG2L, int FWD>
constexpr int tw_mode()
{
    if constexpr (sizeof(T) == 8)
        return LOG2L <= 8 ? (FWD ? JT_TW_MODE_F64_SHORT_FWD : JT_TW_MODE_F64_SHORT_INV) : JT_TW_MODE_F64;
    else if constexpr (Geo<LOG2L>::BLOCK > 256) return 3;  // big lines: too few registers per lane
    else if constexpr (!FWD) return LOG2L <= 8 ? JT_TW_MODE_F32_SHORT_INV : 0;
    else return LOG2L <= 8 ? 1 : JT_TW_MODE_F32_FWD;
}

template <class T, int LOG2L, int FWD>
struct Twiddles {
    using G = Geo<LOG2L>;
    static constexpr int kMode = tw_mode<T, LOG2L, FWD>();
    static constexpr bool kHoist = kMode == 0;
    static constexpr bool kComp = kMode == 3;
    cpx<T> mid_[(kHoist && G::NMID > 0) ? G::NMID : 1][15];
    cpx<T> fin_[(kHoist && G::RF > 1) ? 16 / G::RF : 1][(G::RF > 1) ? G::RF - 1 : 1];
    cpx<T> wb_[(kComp && G::NMID > 0) ? G::NMID : 1];  // root of pass i+1: omega_{16 Ns}^{p mod Ns}
    cpx<T> fb_;                                         // omega_L^p (final pass)
    const cpx<T> *tw;
    int p;

    static __device__ __forceinline__ constexpr int pass_ns(int i)
    {
        int ns = 16;
        for (int k = 0; k < i; ++k) ns *= 16;
        return ns;
    }
    // pass i+1 has Ns = 16^(i+1); factor omega_{16 Ns}^{(p mod Ns) r} = tw[(p mod Ns) r L / (16 Ns)]
    static __device__ __forceinline__ int mid_index(int i, int r, int p)
    {
        const int ns = pass_ns(i);
        return (p & (ns - 1)) * r * (G::L / (16 * ns));
    }
    // final pass (radix RF, Ns = L/RF): task j = p + P t, factor omega_L^{j r}
    static __device__ __forceinline__ int fin_index(int t, int r, int p) { return (p + G::P * t) * r; }

    __device__ __forceinline__ void load(const cpx<T> *table, int lane)
    {
        tw = table;
        p = lane;
        if constexpr (kHoist) {
#pragma unroll
            for (int i = 0; i < G::NMID; ++i)
#pragma unroll
                for (int r = 1; r < 16; ++r) mid_[i][r - 1] = tw[mid_index(i, r, p)];
            if constexpr (G::RF > 1) {
#pragma unroll
                for (int t = 0; t < 16 / G::RF; ++t)
#pragma unroll
                    for (int r = 1; r < G::RF; ++r) fin_[t][r - 1] = tw[fin_index(t, r, p)];
            }
        }
        if constexpr (kComp) {
#pragma unroll
            for (int i = 0; i < G::NMID; ++i) wb_[i] = tw[mid_index(i, 1, p)];
            if constexpr (G::RF > 1) fb_ = tw[p];
        }
    }
    __device__ __forceinline__ cpx<T> mid(int i, int r) const
    {
        if constexpr (kHoist) return mid_[i][r - 1];
        else return tw[mid_index(i, r, p)];
    }
    __device__ __forceinline__ cpx<T> fin(int t, int r) const
    {
        if constexpr (kHoist) return fin_[t][r - 1];
        else return tw[fin_index(t, r, p)];
    }
    // v[r] *= (twiddle of pass i+1, factor r) for r = 1..15
    __device__ __forceinline__ void apply_mid(int i, cpx<T> *v) const
    {
        if constexpr (kComp) {
            const cpx<T> w1 = opaque(wb_[i]), w2 = csq(w1), w3 = cmul(w2, w1), w4 = csq(w2);
            const cpx<T> w8 = csq(w4), w12 = cmul(w8, w4);
            v[1] = cmul(v[1], w1);
            v[2] = cmul(v[2], w2);
            v[3] = cmul(v[3], w3);
            v[4] = cmul(v[4], w4);
            v[8] = cmul(v[8], w8);
            v[12] = cmul(v[12], w12);
            v[5] = cmul(v[5], cmul(w4, w1));
            v[6] = cmul(v[6], cmul(w4, w2));
            v[7] = cmul(v[7], cmul(w4, w3));
            v[9] = cmul(v[9], cmul(w8, w1));
            v[10] = cmul(v[10], cmul(w8, w2));
            v[11] = cmul(v[11], cmul(w8, w3));
            v[13] = cmul(v[13], cmul(w12, w1));
            v[14] = cmul(v[14], cmul(w12, w2));
            v[15] = cmul(v[15], cmul(w12, w3));
        } else {
#pragma unroll
            for (int r = 1; r < 16; ++r) v[r] = cmul(v[r], mid(i, r));
        }
    }
    // powers b^r (r < RF) of the final pass's per-lane root (mode 3 only)
    __device__ __forceinline__ void fin_powers(cpx<T> *bp) const
    {
        if constexpr (kComp && G::RF > 1) {
            bp[1] = opaque(fb_);
#pragma unroll
            for (int r = 2; r < G::RF; ++r) bp[r] = (r % 2 == 0) ? csq(bp[r / 2]) : cmul(bp[r - 1], bp[1]);
        }
    }
    // w[r] *= (twiddle of task t, factor r) for r = 1..RF-1
    __device__ __forceinline__ void apply_fin(int t, cpx<T> *w, const cpx<T> *bp) const
    {
#pragma unroll
        for (int r = 1; r < G::RF; ++r) {
            if constexpr (kComp) {
                // omega_L^{(p + P t) r} = b^r omega_16^{t r}  (P = L / 16)
                w[r] = cmul(w[r], rot16(bp[r], t * r));
            } else {
                w[r] = cmul(w[r], fin(t, r));
            }
        }
    }
};

// L-point DFT (sign +) of the line held in v (lane-owned layout: lane p = pv[h]
// holds v[h][q] = x[p + P q]); on return v[h][q] = X[p + P q].  buf is this
// line's LDS buffer.  Every thread of the line must call it (it contains the
// line's barriers); the VL lanes of a thread are processed between the same
// barriers.
template <class T, int LOG2L, int VL, class TW>
__device__ __forceinline__ void fft_line(cpx<T> (*v)[16], cpx<T> *buf, const int *pv, const TW *tw)
{
    using G = Geo<LOG2L, VL>;
    static_assert(G::L >= 64, "lines shorter than 64 use the dense path with L = 64");
    // pass 0: Ns = 1, no twiddles, inputs are already v[r] = x[p + r P]
#pragma unroll
    for (int h = 0; h < VL; ++h) {
        dft16(v[h]);
#pragma unroll
        for (int r = 0; r < 16; ++r) buf[pad(pv[h] * 16 + r)] = v[h][r];
    }
    int ns = 16;
#pragma unroll
    for (int i = 0; i < G::NMID; ++i) {
        sync_line<G::TPL>();
#pragma unroll
        for (int h = 0; h < VL; ++h) {
#pragma unroll
            for (int r = 0; r < 16; ++r) v[h][r] = buf[pad(pv[h] + r * G::P)];
            tw[h].apply_mid(i, v[h]);
            dft16(v[h]);
        }
        const bool last = (G::RF == 1) && (i == G::NMID - 1);
        if (!last) {
            sync_line<G::TPL>();
#pragma unroll
            for (int h = 0; h < VL; ++h) {
                const int p = pv[h];
                const int base = (p / ns) * ns * 16 + (p & (ns - 1));
#pragma unroll
                for (int r = 0; r < 16; ++r) buf[pad(base + r * ns)] = v[h][r];
            }
        }
        ns *= 16;
    }
    if constexpr (G::RF > 1) {
        constexpr int RF = G::RF, NT = 16 / RF;
        sync_line<G::TPL>();
#pragma unroll
        for (int h = 0; h < VL; ++h) {
            cpx<T> bp[RF];
            tw[h].fin_powers(bp);
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                cpx<T> w[RF];
                const int j = pv[h] + G::P * t;
#pragma unroll
                for (int r = 0; r < RF; ++r) w[r] = buf[pad(j + r * (G::L / RF))];
                tw[h].apply_fin(t, w, bp);
                dftR<T, RF>(w);
                // output index j + r * (L/RF) = p + P (t + r * NT)
#pragma unroll
                for (int r = 0; r < RF; ++r) v[h][t + r * NT] = w[r];
            }
        }
    }
}

// Everything one split group does for its LPB lines.  The caller arranges
// the threads: S split groups of G::BLOCK threads share lines line0 ..
// line0 + LPB - 1 (lines at or past line_end are inactive); group sgrp takes
// the terms l = sgrp, sgrp + S, ... and the S partial sums are added in LDS
// at the end (fixed order, so results do not depend on timing).  Every group
// runs the same number of iterations (ceil(rank / S)) so that all of them
// meet every block barrier; a group whose term index runs past the rank
// computes a term it then discards.  smem holds S * LPB line buffers for
// these groups; tw is the L-entry twiddle table (global or LDS).  Every
// thread of the block must call this with the same S and the same rank.
// A thread carries VL lanes of its line (VL > 1 only when S == 1).
// OWN_SUM: each group adds up only the partial sums of the slots it stores
// (the one-pass kernel; measured slower inside the persistent batch kernel,
// whose register allocation it changes, so that one sums every slot).
// OPT bits.  Prefetch (single-lane threads; each holds 16 more complex
// values per thread across the FFT): forward, 1 loads the next term's v_l
// while the current term gathers and 2 requests the term's u_l before its
// FFT; inverse, 4 requests the term's v_l before its FFT.  8: the fp32
// forward direct block in its node-contiguous form (always so in fp64).
template <class T, int LOG2L, int FWD, int VL = 1, bool OWN_SUM = true, int OPT = 0>
__device__ __forceinline__ void pass_lines(const AxisLaunch &a, unsigned line0, unsigned line_end, int S, int sgrp,
                                           int tid, cpx<T> *smem, const cpx<T> *tw)
{
    using G = Geo<LOG2L, VL>;
    const int slot = tid / G::TPL;
    int pv[VL];
#pragma unroll
    for (int h = 0; h < VL; ++h) pv[h] = tid % G::TPL + h * G::TPL;
    cpx<T> *buf = smem + (sgrp * G::LPB + slot) * G::BUF;
    T *sbuf = reinterpret_cast<T *>(buf);

    // the host guarantees lines * n < 2^31, so 32-bit indexing is exact
    const unsigned line = line0 + (unsigned)slot;
    const bool active = line < line_end;
    const unsigned stride = (unsigned)a.stride;
    const unsigned outer = active ? line / stride : 0u;
    const unsigned inner = active ? line - outer * stride : 0u;
    const unsigned base = outer * (unsigned)a.n * stride + inner;
    const int n = a.n, nu0 = a.nu0, rank = a.rank;

    const cpx<T> *uf = reinterpret_cast<const cpx<T> *>(a.u);
    const cpx<T> *vf = reinterpret_cast<const cpx<T> *>(a.v);
    const T *wv = reinterpret_cast<const T *>(a.wv);

    Twiddles<T, LOG2L, FWD> twd[VL];
#pragma unroll
    for (int h = 0; h < VL; ++h) twd[h].load(tw, pv[h]);

    // the line, in the lane-owned layout (zero beyond n); dtype branch is uniform
    T x[VL][16];
#ifndef JT_SHARED_STRIDED_LOAD
#define JT_SHARED_STRIDED_LOAD 1
#endif
    if (JT_SHARED_STRIDED_LOAD && VL == 1 && S > 1 && stride > 1u) {
        // Strided line: every element is its own cache line, so the S split
        // groups that share the line each load a 1/S share (the slots they
        // also store) into group 0's line buffer, and all of them read the
        // whole line back from there.  Uniform branch; block barriers.
        T *stage = reinterpret_cast<T *>(smem + slot * G::BUF);
        __syncthreads();  // the buffer's previous users are done
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            if (q % S != sgrp) continue;
            const int k = pv[0] + G::P * q;
            T v = (T)0;
            if (active && k < n)
                v = a.in_f64 ? (T) reinterpret_cast<const double *>(a.in)[base + (unsigned)k * stride]
                             : (T) reinterpret_cast<const float *>(a.in)[base + (unsigned)k * stride];
            stage[k] = v;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 16; ++q) x[0][q] = stage[pv[0] + G::P * q];
        __syncthreads();  // group 0 reuses the buffer from here on
    } else if (a.in_f64) {
        const double *src = reinterpret_cast<const double *>(a.in);
#pragma unroll
        for (int h = 0; h < VL; ++h)
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int k = pv[h] + G::P * q;
                x[h][q] = (active && k < n) ? (T)src[base + (unsigned)k * stride] : (T)0;
            }
    } else {
        const float *src = reinterpret_cast<const float *>(a.in);
#pragma unroll
        for (int h = 0; h < VL; ++h)
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int k = pv[h] + G::P * q;
                x[h][q] = (active && k < n) ? (T)src[base + (unsigned)k * stride] : (T)0;
            }
    }
    double acc[VL][16];
    const int iters = (rank + S - 1) / S;
#ifndef JT_FULL_FAST
#define JT_FULL_FAST 1
#endif
    const bool full = JT_FULL_FAST && (n == G::L);  // uniform: the line fills every owned slot

    if constexpr (FWD) {
        // ---- direct block: out_j = sum_{k<nu0} WV[k][j] alpha_k (degrees split over the groups)
#pragma unroll
        for (int h = 0; h < VL; ++h)
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int k = pv[h] + G::P * q;
                if (k < nu0) sbuf[k] = x[h][q];
            }
        sync_line<G::TPL>();
        // Node-contiguous form: when n is a multiple of 4 and the sums fit
        // behind the staged coefficients, each thread takes groups of four
        // consecutive nodes, so a degree's row of WV is read with 16-byte
        // loads (the block re-reads WV for every line), and the sums reach
        // the lane-owned layout through the line buffer.  Same arithmetic,
        // in the same order, as the per-lane form below.  Measured: 2D
        // 1024^2 fp64 forward passes 73.5/94.6 -> 60.8/74.6 us, 3D 256^3
        // fp64 about 15 us faster per pass, the 4096-item ragged 1D batch
        // (fp32) 2.99 -> 2.80 ms; slower in the one-pass fp32 kernels (2D
        // 45.8/51.2 -> 49.5/62.0 us), which keep the per-lane form.
        constexpr bool kVec4Fwd = sizeof(T) == 8 || (OPT & 8);
        constexpr int NI4 = G::L / (4 * G::TPL);  // four-node groups per thread
        const int ost_off = ((nu0 * (int)sizeof(T) + 15) / 16) * 16;  // bytes, after sbuf
        const bool vec4f = kVec4Fwd && (n & 3) == 0 &&
                           ost_off + n * (int)sizeof(T) <= G::BUF * (int)sizeof(cpx<T>);  // uniform
        if (vec4f) {
            T *ost = reinterpret_cast<T *>(reinterpret_cast<unsigned char *>(buf) + ost_off);
            const int t = tid % G::TPL;
            T s4[NI4][4];
#pragma unroll
            for (int i = 0; i < NI4; ++i)
#pragma unroll
                for (int e = 0; e < 4; ++e) s4[i][e] = 0;
            for (int k = sgrp; k < nu0; k += S) {
                const T ak = sbuf[k];
#pragma unroll
                for (int i = 0; i < NI4; ++i) {
                    const int j = 4 * (t + G::TPL * i);
                    if (j < n) {
                        T w4[4];
                        load4(wv + k * n + j, w4);
#pragma unroll
                        for (int e = 0; e < 4; ++e) s4[i][e] += w4[e] * ak;
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < NI4; ++i) {
                const int j = 4 * (t + G::TPL * i);
                if (j < n)
#pragma unroll
                    for (int e = 0; e < 4; ++e) ost[j + e] = s4[i][e];
            }
            sync_line<G::TPL>();
#pragma unroll
            for (int h = 0; h < VL; ++h)
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int j = pv[h] + G::P * q;
                    acc[h][q] = j < n ? (double)ost[j] : 0.0;
                }
        } else if (full) {
            // all 16 outputs exist: one batch of 16 loads per degree k
            T s[VL][16];
#pragma unroll
            for (int h = 0; h < VL; ++h)
#pragma unroll
                for (int q = 0; q < 16; ++q) s[h][q] = 0;
            // degrees k = sgrp, sgrp + S, ...: the split groups share the block
            for (int k = sgrp; k < nu0; k += S) {
                const T ak = sbuf[k];
#pragma unroll
                for (int h = 0; h < VL; ++h)
#pragma unroll
                    for (int q = 0; q < 16; ++q) s[h][q] += wv[k * n + pv[h] + G::P * q] * ak;
            }
#pragma unroll
            for (int h = 0; h < VL; ++h)
#pragma unroll
                for (int q = 0; q < 16; ++q) acc[h][q] = (double)s[h][q];
        } else {
#pragma unroll
            for (int h = 0; h < VL; ++h)
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int j = pv[h] + G::P * q;
                    T s = 0;
                    if (j < n)
                        for (int k = sgrp; k < nu0; k += S) s += wv[k * n + j] * sbuf[k];
                    acc[h][q] = (double)s;
                }
        }
#ifndef JT_HOIST_BINS
#define JT_HOIST_BINS 1
#endif
        constexpr bool kPFV = (OPT & 1) && VL == 1, kPFU = (OPT & 2) && VL == 1;
        // LDS slots of y[m_j] for the owned nodes (the same for every term);
        // kept in registers except on the longest lines, which have none to spare
#ifndef JT_HOIST_F64
#define JT_HOIST_F64 1
#endif
        // (fp64 only from 512 points: measured slower on 256-point lines)
#ifndef JT_HB_F64_MIN
#define JT_HB_F64_MIN 9
#endif
        constexpr bool kHB = JT_HOIST_BINS && Geo<LOG2L>::BLOCK <= 256 && (sizeof(T) == 4 || (JT_HOIST_F64 && LOG2L >= JT_HB_F64_MIN));
        int bix[VL][kHB ? 16 : 1];
        if constexpr (kHB) {
#pragma unroll
            for (int h = 0; h < VL; ++h)
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int j = pv[h] + G::P * q;
                    bix[h][q] = pad(j < n ? a.bins[j] : 0);
                }
        }
        // factors v_l of the next term, loaded while the current term gathers
        cpx<T> fv[VL][16];
        if constexpr (kPFV) {
            const int l = (sgrp < rank) ? sgrp : rank - 1;
#pragma unroll
            for (int h = 0; h < VL; ++h)
#pragma unroll
                for (int q = 0; q < 16; ++q) fv[h][q] = vf[l * G::L + pv[h] + G::P * q];
        }
        for (int it = 0; it < iters; ++it) {
            const int l0 = it * S + sgrp;
            const bool keep = l0 < rank;
            const int l = keep ? l0 : rank - 1;
            cpx<T> v[VL][16];
#pragma unroll
            for (int h = 0; h < VL; ++h)
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const cpx<T> f = kPFV ? fv[h][q] : vf[l * G::L + pv[h] + G::P * q];
                    v[h][q] = {f.x * x[h][q], f.y * x[h][q]};
                }
            // u_l for the gather, requested before the FFT so that it arrives meanwhile
            cpx<T> uu[VL][kPFU ? 16 : 1];
            if constexpr (kPFU) {
                const cpx<T> *ul = uf + l * n;
#pragma unroll
                for (int h = 0; h < VL; ++h)
#pragma unroll
                    for (int q = 0; q < 16; ++q) {
                        const int j = pv[h] + G::P * q;
                        uu[h][q] = (full || j < n) ? ul[j] : cpx<T>{(T)0, (T)0};
                    }
            }
            sync_line<G::TPL>();  // previous users of buf are done
            fft_line<T, LOG2L, VL>(v, buf, pv, twd);
            sync_line<G::TPL>();
#pragma unroll
            for (int h = 0; h < VL; ++h)
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int m = pv[h] + G::P * q;
                    if (m <= G::L / 2) buf[pad(m)] = v[h][q];
                }
            if constexpr (kPFV) {
                const int ln0 = (it + 1) * S + sgrp;
                const int ln = ln0 < rank ? ln0 : rank - 1;
#pragma unroll
                for (int h = 0; h < VL; ++h)
#pragma unroll
                    for (int q = 0; q < 16; ++q) fv[h][q] = vf[ln * G::L + pv[h] + G::P * q];
            }
            sync_line<G::TPL>();
            if (keep) {
                const cpx<T> *ul = uf + l * n;
                if (full) {
                    // every owned node exists: no per-element guards, loads batch
#pragma unroll
                    for (int h = 0; h < VL; ++h)
#pragma unroll
                        for (int q = 0; q < 16; ++q) {
                            const int j = pv[h] + G::P * q;
                            const cpx<T> y = buf[kHB ? bix[h][q % (kHB ? 16 : 1)] : pad(a.bins[j])];
                            const cpx<T> u = kPFU ? uu[h][q % (kPFU ? 16 : 1)] : ul[j];
                            acc[h][q] += (double)(u.x * y.x - u.y * y.y);
                        }
                } else {
#pragma unroll
                    for (int h = 0; h < VL; ++h)
#pragma unroll
                        for (int q = 0; q < 16; ++q) {
                            const int j = pv[h] + G::P * q;
                            if (j < n) {
                                const cpx<T> y = buf[kHB ? bix[h][q % (kHB ? 16 : 1)] : pad(a.bins[j])];
                                const cpx<T> u = kPFU ? uu[h][q % (kPFU ? 16 : 1)] : ul[j];
                                acc[h][q] += (double)(u.x * y.x - u.y * y.y);
                            }
                        }
                }
            }
        }
    } else {
        // ---- direct block: alpha_k = sum_j WV[k][j] g_j for k < nu0.  The
        // degrees go in chunks of KC, chunk c to split group c mod S.  Every
        // lane sums over its own nodes (coalesced rows of WV), the partial sums
        // are added across the line's lanes, and the totals wait in the
        // group's line buffer until the lanes that own those degrees pick them
        // up.  All groups run the same number of rounds (line_sum may hold a
        // block barrier).
#pragma unroll
        for (int h = 0; h < VL; ++h)
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[h][q] = 0.0;
        // degrees per chunk: 4 in the one-pass kernel (against 8: 2D 1024^2
        // fp64 inverse passes 80.9/97.7 -> 79.2/96.3 us, 3D 256^3 fp64 about
        // 12 us faster per pass; 16 took the fp32 256-point inverse over 170
        // registers), 8 in the persistent kernel (OWN_SUM false), whose
        // 2048- and 4096-point units spill more with 4, and 2 on the
        // register-poor long lines
        constexpr int KC = Geo<LOG2L>::BLOCK <= 256 ? (OWN_SUM ? 4 : 8) : 2;
        const int nchunks = (nu0 + KC - 1) / KC;
        const int rounds = (nchunks + S - 1) / S;
        // The line buffer is free until the first term.  It holds, in order:
        // the per-degree sums red[0, nu0) (rounded up to 16 bytes), the
        // per-wave partials of line_sum (lines over several waves), and the
        // staged line gs.  The host caps nu0 at 64, so red and the partials
        // always fit (512 + 256 bytes against at least 544 bytes of buffer).
        // When n is a multiple of 4 and the staged line fits behind them, each
        // thread takes groups of four consecutive nodes, so a degree's row of
        // WV is read with 16-byte loads: the block re-reads WV for every line,
        // and four times fewer (wider) loads is what this block's time depends
        // on.  Otherwise the lanes sum over the nodes they own.
        double *red = reinterpret_cast<double *>(buf);
        const int red_n = (nu0 + 1) & ~1;
        constexpr int LSUM = G::TPL > 64 ? (G::TPL / 64) * KC : 0;
        double *lsum = red + red_n;
        const int gs_off = 8 * (red_n + LSUM);  // bytes; a multiple of 16
        const bool vec4 = (n & 3) == 0 && gs_off + G::L * (int)sizeof(T) <= G::BUF * (int)sizeof(cpx<T>);  // uniform
        T *gs = reinterpret_cast<T *>(reinterpret_cast<unsigned char *>(buf) + gs_off);
        if (vec4) {
#pragma unroll
            for (int h = 0; h < VL; ++h)
#pragma unroll
                for (int q = 0; q < 16; ++q) gs[pv[h] + G::P * q] = x[h][q];  // zero beyond n
            sync_line<G::TPL>();
        }
        constexpr int NI = G::L / (4 * G::TPL);  // four-node groups per thread
        for (int rd = 0; rd < rounds; ++rd) {
            const int ch = rd * S + sgrp;
            const int k0 = ch * KC;
            double part[KC];
#pragma unroll
            for (int c = 0; c < KC; ++c) part[c] = 0.0;
            if (ch < nchunks && vec4) {
                const int t = tid % G::TPL;
#pragma unroll
                for (int i = 0; i < NI; ++i) {
                    const int j = 4 * (t + G::TPL * i);
                    if (j < n) {
                        T g4[4];
                        load4(gs + j, g4);
#pragma unroll
                        for (int c = 0; c < KC; ++c)
                            if (k0 + c < nu0) {
                                T w4[4];
                                load4(wv + (k0 + c) * n + j, w4);
#pragma unroll
                                for (int e = 0; e < 4; ++e) part[c] += (double)w4[e] * (double)g4[e];
                            }
                    }
                }
            } else if (ch < nchunks) {
#pragma unroll
                for (int h = 0; h < VL; ++h)
#pragma unroll
                    for (int q = 0; q < 16; ++q) {
                        const int j = pv[h] + G::P * q;
                        if (j < n) {
                            const double g = (double)x[h][q];
#pragma unroll
                            for (int c = 0; c < KC; ++c)
                                if (k0 + c < nu0) part[c] += (double)wv[(k0 + c) * n + j] * g;
                        }
                    }
            }
            line_sum<G::TPL, KC>(part, lsum, tid % G::TPL);
            if (ch < nchunks && tid % G::TPL == 0)
#pragma unroll
                for (int c = 0; c < KC; ++c)
                    if (k0 + c < nu0) red[k0 + c] = part[c];
        }
        sync_line<G::TPL>();
#pragma unroll
        for (int h = 0; h < VL; ++h)
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int k = pv[h] + G::P * q;
                if (k < nu0 && (k / KC) % S == sgrp) acc[h][q] = red[k];
            }
        // the nodes of each owned bin m (at most two in almost every plan), as
        // padded LDS slots packed j_a | j_b << 16 (0xffff: none); the same for
        // every term, so they are read once.  Only where 16 more registers
        // keep the kernel's occupancy: fp32, and fp64 below 256 points and at
        // 1024 (2D 1024^2 fp64 inverse passes 81.0/99.2 -> 80.5/98.1 us).  At
        // 256 points they would take the fp64 inverse over 256 registers (one
        // wave per SIMD instead of two) and the fp32 inverse over 170 (two
        // instead of three): measured on 256^3, 1100 -> 910 us (fp64) and
        // 640 -> 495 us (fp32, with computed twiddles) per inverse pass
        // without them.
#ifndef JT_BP_L256_F64
#define JT_BP_L256_F64 0
#endif
#ifndef JT_BP_L256_F32
#define JT_BP_L256_F32 0
#endif
        constexpr bool kBP = Geo<LOG2L>::BLOCK <= 256 && (sizeof(T) == 4 || LOG2L <= 8 || LOG2L == 10) &&
                             (LOG2L != 8 || (sizeof(T) == 4 ? JT_BP_L256_F32 : JT_BP_L256_F64));
        const bool two = kBP && a.max_per_bin <= 2;
        unsigned bpair[VL][kBP ? 16 : 1];
#pragma unroll
        for (int h = 0; h < VL; ++h)
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int m = pv[h] + G::P * q;
                unsigned w = 0xffffffffu;
                if (two && m <= G::L / 2) {
                    const int j0 = a.binptr[m], j1 = a.binptr[m + 1];
                    const unsigned ja = (j1 > j0) ? (unsigned)pad(j0) : 0xffffu;
                    const unsigned jb = (j1 > j0 + 1) ? (unsigned)pad(j0 + 1) : 0xffffu;
                    w = ja | (jb << 16);
                }
                bpair[h][q % (kBP ? 16 : 1)] = w;
            }
        constexpr bool kPFI = (OPT & 4) && VL == 1;
        for (int it = 0; it < iters; ++it) {
            const int l0 = it * S + sgrp;
            const bool keep = l0 < rank;
            const int l = keep ? l0 : rank - 1;
            sync_line<G::TPL>();  // previous users of buf are done
            if (full) {
#pragma unroll
                for (int h = 0; h < VL; ++h)
#pragma unroll
                    for (int q = 0; q < 16; ++q) {
                        const int j = pv[h] + G::P * q;
                        const cpx<T> u = uf[l * n + j];
                        buf[pad(j)] = {u.x * x[h][q], u.y * x[h][q]};
                    }
            } else {
#pragma unroll
                for (int h = 0; h < VL; ++h)
#pragma unroll
                    for (int q = 0; q < 16; ++q) {
                        const int j = pv[h] + G::P * q;
                        if (j < n) {
                            const cpx<T> u = uf[l * n + j];
                            buf[pad(j)] = {u.x * x[h][q], u.y * x[h][q]};
                        }
                    }
            }
            sync_line<G::TPL>();
            cpx<T> v[VL][16];
            if (two) {
#pragma unroll
                for (int h = 0; h < VL; ++h)
#pragma unroll
                    for (int q = 0; q < 16; ++q) {
                        const unsigned w = bpair[h][q % (kBP ? 16 : 1)];
                        const unsigned ja = w & 0xffffu, jb = w >> 16;
                        cpx<T> z = {(T)0, (T)0};
                        if (ja != 0xffffu) z = buf[ja];
                        if (jb != 0xffffu) z = z + buf[jb];
                        v[h][q] = z;
                    }
            } else if ((sizeof(T) == 4 || LOG2L > 8) && a.max_per_bin <= 2) {
                // at most two nodes per bin (uniform): both slots are read
                // unconditionally (slot 0 stands in for an absent node) and
                // selected, with no per-bin loop and no registers held
                // across terms.  Measured against the loop: 2D 1024^2 fp64
                // inverse passes 87/106 -> 81/102 us, 3D 256^3 fp32 490 ->
                // 450 us; slower on 256-point fp64 lines (910 -> 1108 us),
                // which keep the loop
#pragma unroll
                for (int h = 0; h < VL; ++h)
#pragma unroll
                    for (int q = 0; q < 16; ++q) {
                        const int m = pv[h] + G::P * q;
                        cpx<T> z = {(T)0, (T)0};
                        if (m <= G::L / 2) {
                            const int j0 = a.binptr[m], j1 = a.binptr[m + 1];
                            const bool ha = j1 > j0, hb = j1 > j0 + 1;
                            const cpx<T> ya = buf[ha ? pad(j0) : 0], yb = buf[hb ? pad(j0 + 1) : 0];
                            z.x = (ha ? ya.x : (T)0) + (hb ? yb.x : (T)0);
                            z.y = (ha ? ya.y : (T)0) + (hb ? yb.y : (T)0);
                        }
                        v[h][q] = z;
                    }
            } else {
#pragma unroll
                for (int h = 0; h < VL; ++h)
#pragma unroll
                    for (int q = 0; q < 16; ++q) {
                        const int m = pv[h] + G::P * q;
                        cpx<T> z = {(T)0, (T)0};
                        if (m <= G::L / 2) {
                            const int j0 = a.binptr[m], j1 = a.binptr[m + 1];
                            for (int jj = j0; jj < j1; ++jj) z = z + buf[pad(jj)];
                        }
                        v[h][q] = z;
                    }
            }
            // v_l of this term, requested before the FFT (OPT bit 4)
            cpx<T> fi[VL][kPFI ? 16 : 1];
            if constexpr (kPFI) {
#pragma unroll
                for (int h = 0; h < VL; ++h)
#pragma unroll
                    for (int q = 0; q < 16; ++q) fi[h][q] = vf[l * G::L + pv[h] + G::P * q];
            }
            sync_line<G::TPL>();
            fft_line<T, LOG2L, VL>(v, buf, pv, twd);
            if (keep) {
#pragma unroll
                for (int h = 0; h < VL; ++h)
#pragma unroll
                    for (int q = 0; q < 16; ++q) {
                        const int k = pv[h] + G::P * q;
                        const cpx<T> f = kPFI ? fi[h][q % (kPFI ? 16 : 1)] : vf[l * G::L + k];
                        acc[h][q] += (double)(f.x * v[h][q].x - f.y * v[h][q].y);
                    }
            }
        }
    }
    // ---- sum the S partial results in LDS (fixed order), then store.
    // All reads of the input happened before the first barrier, so the output
    // may alias the input (in-place passes).
    double *part = reinterpret_cast<double *>(buf);  // L doubles fit in one line buffer
    if (S > 1) {
        __syncthreads();
#pragma unroll
        for (int h = 0; h < VL; ++h)
#pragma unroll
            for (int q = 0; q < 16; ++q) part[pv[h] + G::P * q] = acc[h][q];
        __syncthreads();
        // with OWN_SUM, each group adds up (and below stores) only the slots
        // q = sgrp mod S
#pragma unroll
        for (int h = 0; h < VL; ++h)
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                if (OWN_SUM && (q % S) != sgrp) continue;  // uniform
                double t = 0.0;
                for (int s2 = 0; s2 < S; ++s2)
                    t += reinterpret_cast<const double *>(smem + (s2 * G::LPB + slot) * G::BUF)[pv[h] + G::P * q];
                acc[h][q] = t;
            }
    }
    if (a.out_f64) {
        double *dst = reinterpret_cast<double *>(a.out);
#pragma unroll
        for (int h = 0; h < VL; ++h)
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int i = pv[h] + G::P * q;
                if (active && i < n && (q % S) == sgrp) dst[base + (unsigned)i * stride] = acc[h][q];
            }
    } else {
        float *dst = reinterpret_cast<float *>(a.out);
#pragma unroll
        for (int h = 0; h < VL; ++h)
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int i = pv[h] + G::P * q;
                if (active && i < n && (q % S) == sgrp) dst[base + (unsigned)i * stride] = (float)acc[h][q];
            }
    }
}

}  // namespace dev
}  // namespace jt
