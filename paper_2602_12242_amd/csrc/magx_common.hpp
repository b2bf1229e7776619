// Shared device-side building blocks for the magx kernels (gfx950, wave64).
//
// Complex arithmetic on float2/double2, the twiddle table, radix-2/4/8
// butterflies and an LDS-resident Stockham FFT used by every FFT pass of the
// demag convolution (Section II-B: FFT convolution on the extended grid).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/magx.h"

namespace magx {

constexpr int kNT = 256;          // threads per block for every FFT/pencil kernel
constexpr int kTwLog = 12;        // twiddle table covers lengths up to 4096
constexpr int kTwN = 1 << kTwLog;

template <typename R> struct vec2;
template <> struct vec2<float> { using type = float2; };
template <> struct vec2<double> { using type = double2; };
template <typename R> using cx = typename vec2<R>::type;

template <typename R> __device__ __forceinline__ cx<R> mk(R a, R b) { cx<R> r; r.x = a; r.y = b; return r; }
template <typename R> __device__ __forceinline__ cx<R> cadd(cx<R> a, cx<R> b) { return mk<R>(a.x + b.x, a.y + b.y); }
template <typename R> __device__ __forceinline__ cx<R> csub(cx<R> a, cx<R> b) { return mk<R>(a.x - b.x, a.y - b.y); }
template <typename R> __device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
    return mk<R>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename R> __device__ __forceinline__ cx<R> cconj(cx<R> a) { return mk<R>(a.x, -a.y); }
template <typename R> __device__ __forceinline__ cx<R> cscale(cx<R> a, R s) { return mk<R>(a.x * s, a.y * s); }
// multiply by -i (forward) or +i (inverse)
template <typename R, bool INV> __device__ __forceinline__ cx<R> mul_mi(cx<R> a) {
    return INV ? mk<R>(-a.y, a.x) : mk<R>(a.y, -a.x);
}

// exp(-2 pi i k / 4096), k in [0, 4096), filled once per device at context
// creation (double-precision sincospi, rounded once for the float table).
extern __device__ float2 g_tw32[kTwN];
extern __device__ double2 g_tw64[kTwN];

template <typename R> __device__ __forceinline__ cx<R> tw_fwd(int k);
template <> __device__ __forceinline__ float2 tw_fwd<float>(int k) { return g_tw32[k]; }
template <> __device__ __forceinline__ double2 tw_fwd<double>(int k) { return g_tw64[k]; }
// w^k for a transform of direction INV; k indexes the 4096-point table.
template <typename R, bool INV> __device__ __forceinline__ cx<R> tw(int k) {
    cx<R> w = tw_fwd<R>(k);
    return INV ? cconj<R>(w) : w;
}

// ---- small DFTs in registers --------------------------------------------------
template <typename R, bool INV> __device__ __forceinline__ void dft2(cx<R>* v) {
    cx<R> a = v[0], b = v[1];
    v[0] = cadd<R>(a, b);
    v[1] = csub<R>(a, b);
}

template <typename R, bool INV> __device__ __forceinline__ void dft4(cx<R>* v) {
    cx<R> a0 = cadd<R>(v[0], v[2]), a1 = csub<R>(v[0], v[2]);
    cx<R> a2 = cadd<R>(v[1], v[3]), a3 = mul_mi<R, INV>(csub<R>(v[1], v[3]));
    v[0] = cadd<R>(a0, a2);
    v[2] = csub<R>(a0, a2);
    v[1] = cadd<R>(a1, a3);
    v[3] = csub<R>(a1, a3);
}

template <typename R, bool INV> __device__ __forceinline__ void dft8(cx<R>* v) {
    const R h = (R)0.70710678118654752440;
    cx<R> e[4] = {v[0], v[2], v[4], v[6]};
    cx<R> o[4] = {v[1], v[3], v[5], v[7]};
    dft4<R, INV>(e);
    dft4<R, INV>(o);
    // o[k] *= w8^k (forward w8 = (1 - i)/sqrt2, inverse its conjugate)
    cx<R> o1 = INV ? mk<R>((o[1].x - o[1].y) * h, (o[1].x + o[1].y) * h)
                   : mk<R>((o[1].x + o[1].y) * h, (o[1].y - o[1].x) * h);
    cx<R> o2 = mul_mi<R, INV>(o[2]);
    cx<R> o3 = INV ? mk<R>(-(o[3].x + o[3].y) * h, (o[3].x - o[3].y) * h)
                   : mk<R>((o[3].y - o[3].x) * h, -(o[3].x + o[3].y) * h);
    v[0] = cadd<R>(e[0], o[0]);
    v[4] = csub<R>(e[0], o[0]);
    v[1] = cadd<R>(e[1], o1);
    v[5] = csub<R>(e[1], o1);
    v[2] = cadd<R>(e[2], o2);
    v[6] = csub<R>(e[2], o2);
    v[3] = cadd<R>(e[3], o3);
    v[7] = csub<R>(e[3], o3);
}

template <typename R, int RAD, bool INV> __device__ __forceinline__ void dft(cx<R>* v) {
    if constexpr (RAD == 2) dft2<R, INV>(v);
    else if constexpr (RAD == 4) dft4<R, INV>(v);
    else dft8<R, INV>(v);
}

// ---- Stockham FFTs in LDS ----------------------------------------------------------
// nseq independent sequences of length L = 2^lgL (1 <= L <= 4096).  Two LDS
// layouts:
//  * columns (LAYOUT = kCols): nseq = NC << lgT sequences, element j of
//    sequence b at b + j*nseq; consecutive threads take consecutive b
//    (coalesced column tiles; NC = 1 or 3 is a compile-time constant so the
//    thread -> (b, j) split needs no runtime division);
//  * lines (LAYOUT = kLines): element j of sequence b at (b << lgL) + j;
//    consecutive threads take consecutive j.
// Each thread holds at most EMAX elements (nseq * L <= kNT * EMAX).
// load(b, j) / store(b, j, v) are used instead of LDS by the first / last
// pass when SRC_LDS / DST_LDS is false.  The remainder radix (2 or 4) comes
// first, then radix-8 passes.  Radix-8 twiddles w^{rk} come from three table
// reads (w^k, w^2k, w^4k) and their products.  A barrier follows every pass
// that writes LDS (and precedes a pass reading and writing LDS in place).
// Unnormalised; the inverse uses conjugate twiddles.
constexpr int kCols = 0;
constexpr int kLines = 1;

__device__ __forceinline__ int mul24(int a, int b) { return __mul24(a, b); }

template <typename R, bool INV>
__device__ __forceinline__ void twiddle_apply(cx<R>* v, int RAD, int k, int twshift) {
    if (!k) return;
    const cx<R> w1 = tw<R, INV>(k << twshift);
    if (RAD == 2) { v[1] = cmul<R>(v[1], w1); return; }
    const cx<R> w2 = tw<R, INV>((2 * k) << twshift);
    if (RAD == 4) {
        v[1] = cmul<R>(v[1], w1);
        v[2] = cmul<R>(v[2], w2);
        v[3] = cmul<R>(v[3], cmul<R>(w2, w1));
        return;
    }
    const cx<R> w4 = tw<R, INV>((4 * k) << twshift);
    const cx<R> w3 = cmul<R>(w2, w1);
    v[1] = cmul<R>(v[1], w1);
    v[2] = cmul<R>(v[2], w2);
    v[3] = cmul<R>(v[3], w3);
    v[4] = cmul<R>(v[4], w4);
    v[5] = cmul<R>(v[5], cmul<R>(w4, w1));
    v[6] = cmul<R>(v[6], cmul<R>(w4, w2));
    v[7] = cmul<R>(v[7], cmul<R>(w4, w3));
}

template <int LAYOUT, int NC>
__device__ __forceinline__ void seq_split(int t, int lgT, int lgnb, int nseq, int& b, int& j) {
    if constexpr (LAYOUT == kLines) {
        b = t >> lgnb;
        j = t & ((1 << lgnb) - 1);
    } else if constexpr (NC == 1) {
        b = t & (nseq - 1);
        j = t >> lgT;
    } else {
        j = (t >> lgT) / NC;
        b = t - mul24(j, nseq);
    }
}

template <typename R, int RAD, bool INV, int EMAX, bool SRC_LDS, bool DST_LDS, int LAYOUT, int NC, class Load,
          class Store>
__device__ __forceinline__ void stockham_io_pass(cx<R>* __restrict__ buf, int lgL, int lgNs, int lgT, int nseq,
                                                 Load& load, Store& store) {
    constexpr int PER = EMAX / RAD > 0 ? EMAX / RAD : 1;
    constexpr int LGR = RAD == 2 ? 1 : (RAD == 4 ? 2 : 3);
    const int lgnb = lgL - LGR;
    const int nb = 1 << lgnb;
    const int total = nb * nseq;
    const int Ns = 1 << lgNs;
    const int twshift = kTwLog - LGR - lgNs;
    // uniform strides between the RAD inputs / outputs of one butterfly
    const int in_stride = LAYOUT == kLines ? nb : (nb * nseq);
    const int out_stride = LAYOUT == kLines ? Ns : (Ns * nseq);
    cx<R> v[PER][RAD];
    int seqv[PER], pos0[PER], obase[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int t = threadIdx.x + i * kNT;
        if (t < total) {
            int b, j;
            seq_split<LAYOUT, NC>(t, lgT, lgnb, nseq, b, j);
            seqv[i] = b;
            if constexpr (SRC_LDS) {
                const int ib = LAYOUT == kLines ? (b << lgL) + j : b + mul24(j, nseq);
#pragma unroll
                for (int r = 0; r < RAD; ++r) v[i][r] = buf[ib + r * in_stride];
            } else {
#pragma unroll
                for (int r = 0; r < RAD; ++r) v[i][r] = load(b, j + (r << lgnb));
            }
            const int k = j & (Ns - 1);
            pos0[i] = ((j >> lgNs) << (lgNs + LGR)) + k;
            obase[i] = LAYOUT == kLines ? (b << lgL) + pos0[i] : b + mul24(pos0[i], nseq);
            twiddle_apply<R, INV>(v[i], RAD, k, twshift);
            dft<R, RAD, INV>(v[i]);
        }
    }
    if constexpr (SRC_LDS && DST_LDS) __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int t = threadIdx.x + i * kNT;
        if (t < total) {
#pragma unroll
            for (int r = 0; r < RAD; ++r) {
                if constexpr (DST_LDS) buf[obase[i] + r * out_stride] = v[i][r];
                else store(seqv[i], pos0[i] + r * Ns, v[i][r]);
            }
        }
    }
    if constexpr (DST_LDS) __syncthreads();
}

template <typename R, bool INV, int EMAX, bool SRC_LDS, bool DST_LDS, int LAYOUT, int NC, class Load, class Store>
__device__ __forceinline__ void fft_io(cx<R>* __restrict__ buf, int lgL, int lgT, int nseq, Load load, Store store) {
    if (lgL == 0) {   // length 1: the transform is the identity
        for (int b = threadIdx.x; b < nseq; b += kNT) {
            cx<R> x;
            if constexpr (SRC_LDS) x = buf[b];
            else x = load(b, 0);
            if constexpr (DST_LDS) buf[b] = x;
            else store(b, 0, x);
        }
        if constexpr (DST_LDS) __syncthreads();
        return;
    }
    const int rem = lgL % 3;
    int lgNs = 0, left = lgL;
    bool first = true;
#define MAGX_PASS(RADIX, S, D) \
    stockham_io_pass<R, RADIX, INV, EMAX, S, D, LAYOUT, NC>(buf, lgL, lgNs, lgT, nseq, load, store)
    if (rem) {
        const bool last = (left == rem);
        if (rem == 1) {
            if (last) MAGX_PASS(2, SRC_LDS, DST_LDS);
            else MAGX_PASS(2, SRC_LDS, true);
        } else {
            if (last) MAGX_PASS(4, SRC_LDS, DST_LDS);
            else MAGX_PASS(4, SRC_LDS, true);
        }
        lgNs += rem;
        left -= rem;
        first = false;
    }
    while (left > 0) {
        const bool last = (left == 3);
        if (first) {
            if (last) MAGX_PASS(8, SRC_LDS, DST_LDS);
            else MAGX_PASS(8, SRC_LDS, true);
            first = false;
        } else {
            if (last) MAGX_PASS(8, true, DST_LDS);
            else MAGX_PASS(8, true, true);
        }
        lgNs += 3;
        left -= 3;
    }
#undef MAGX_PASS
}

// Workgroups are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b % 8), each with its own L2.  This bijection of [0, nblocks) gives every XCD
// a contiguous range of logical blocks, so neighbouring tiles (which share
// cache lines, stencil rows or tensor rows) meet in the same L2.
__device__ __forceinline__ int xcd_logical_block(int b, int nblocks) {
    const int q = nblocks >> 3, r = nblocks & 7;
    const int x = b & 7, i = b >> 3;
    return x * q + min(x, r) + i;
}

__host__ __device__ inline int ilog2(int v) {
    int r = 0;
    while ((1 << r) < v) ++r;
    return r;
}

}  // namespace magx
