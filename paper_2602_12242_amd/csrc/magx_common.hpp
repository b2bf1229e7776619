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
// pass when SRC_LDS / DST_LDS is false.  HALF_IN: elements j >= L/2 of every
// input sequence are zero (zero padding of the extended grid), so the first
// pass neither reads them nor spends arithmetic on them; HALF_OUT: only
// outputs j < L/2 are wanted, so the last pass computes and writes no others.  The remainder radix (2 or 4) comes
// first, then radix-8 passes.  Radix-8 twiddles w^{rk} come from three table
// reads (w^k, w^2k, w^4k) and their products.  A barrier follows every pass
// that writes LDS (and precedes a pass reading and writing LDS in place).
// Unnormalised; the inverse uses conjugate twiddles.
constexpr int kCols = 0;
constexpr int kLines = 1;

__device__ __forceinline__ int mul24(int a, int b) { return __mul24(a, b); }

// threadIdx.x behind an empty volatile asm statement: index arithmetic derived
// from it is recomputed in each pass instead of being hoisted out of a tile
// loop and held in registers across it.
__device__ __forceinline__ int tid_opaque() {
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

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

// Source of a pass's inputs: the load functor, LDS, or registers filled
// beforehand by first_pass_load (first pass only).
constexpr int kSrcFn = 0;
constexpr int kSrcLds = 1;
constexpr int kSrcReg = 2;

// Inputs of the first pass of one tile held in registers, so that the loads
// of the next tile can be in flight while this one is transformed: EMAX
// values per thread for any first radix (EMAX/2 when the upper half is zero).
template <typename R, int EMAX, bool HALF_IN>
struct FirstIn {
    static constexpr int N = HALF_IN ? EMAX / 2 : EMAX;
    cx<R> v[N];
};

template <typename R, int RAD, bool INV, int EMAX, int SRC, bool DST_LDS, int LAYOUT, int NC, bool HIN,
          bool HOUT, class Load, class Store, class In>
__device__ __forceinline__ void stockham_io_pass(cx<R>* __restrict__ buf, int lgL, int lgNs, int lgT, int nseq,
                                                 Load& load, Store& store, In& in) {
    constexpr bool SRC_LDS = SRC == kSrcLds;
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
    const int tid = tid_opaque();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int t = tid + i * kNT;
        if (t < total) {
            int b, j;
            seq_split<LAYOUT, NC>(t, lgT, lgnb, nseq, b, j);
            seqv[i] = b;
            // with HIN the inputs r >= RAD/2 lie in the zero half (first pass: lgNs = 0)
            constexpr int RIN = HIN ? RAD / 2 : RAD;
            if constexpr (SRC == kSrcReg) {
#pragma unroll
                for (int r = 0; r < RIN; ++r) v[i][r] = in.v[i * RIN + r];
            } else if constexpr (SRC_LDS) {
                const int ib = LAYOUT == kLines ? (b << lgL) + j : b + mul24(j, nseq);
#pragma unroll
                for (int r = 0; r < RIN; ++r) v[i][r] = buf[ib + r * in_stride];
            } else {
#pragma unroll
                for (int r = 0; r < RIN; ++r) v[i][r] = load(b, j + (r << lgnb));
            }
#pragma unroll
            for (int r = RIN; r < RAD; ++r) v[i][r] = mk<R>((R)0, (R)0);
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
        const int t = tid + i * kNT;
        if (t < total) {
#pragma unroll
            // with HOUT the outputs r >= RAD/2 land in the unwanted half (last pass)
            for (int r = 0; r < (HOUT ? RAD / 2 : RAD); ++r) {
                if constexpr (DST_LDS) buf[obase[i] + r * out_stride] = v[i][r];
                else store(seqv[i], pos0[i] + r * Ns, v[i][r]);
            }
        }
    }
    if constexpr (DST_LDS) __syncthreads();
}

template <typename R, bool INV, int EMAX, bool SRC_LDS, bool DST_LDS, int LAYOUT, int NC, bool HALF_IN = false,
          bool HALF_OUT = false, class Load, class Store>
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
    // first pass: source SRC_LDS, zero upper half if HALF_IN; last pass:
    // destination DST_LDS, lower half only if HALF_OUT; LDS in between
    struct NoIn { cx<R> v[1]; } noin;
#define MAGX_PASS(RADIX, S, D, HI, HO) \
    stockham_io_pass<R, RADIX, INV, EMAX, (S) ? kSrcLds : kSrcFn, D, LAYOUT, NC, HI, HO>(buf, lgL, lgNs, lgT, nseq, \
                                                                                      load, store, noin)
    if (rem) {
        const bool last = (left == rem);
        if (rem == 1) {
            if (last) MAGX_PASS(2, SRC_LDS, DST_LDS, HALF_IN, HALF_OUT);
            else MAGX_PASS(2, SRC_LDS, true, HALF_IN, false);
        } else {
            if (last) MAGX_PASS(4, SRC_LDS, DST_LDS, HALF_IN, HALF_OUT);
            else MAGX_PASS(4, SRC_LDS, true, HALF_IN, false);
        }
        lgNs += rem;
        left -= rem;
        first = false;
    }
    while (left > 0) {
        const bool last = (left == 3);
        if (first) {
            if (last) MAGX_PASS(8, SRC_LDS, DST_LDS, HALF_IN, HALF_OUT);
            else MAGX_PASS(8, SRC_LDS, true, HALF_IN, false);
            first = false;
        } else {
            if (last) MAGX_PASS(8, true, DST_LDS, false, HALF_OUT);
            else MAGX_PASS(8, true, true, false, false);
        }
        lgNs += 3;
        left -= 3;
    }
#undef MAGX_PASS
}

// Loads the first pass's inputs of one tile into `in` (lgL >= 1), in the
// order the register-sourced first pass of fft_reg consumes them.
template <typename R, int RAD, int EMAX, int LAYOUT, int NC, bool HIN, class Load>
__device__ __forceinline__ void first_load_rad(FirstIn<R, EMAX, HIN>& in, int lgL, int lgT, int nseq, Load& load) {
    constexpr int PER = EMAX / RAD > 0 ? EMAX / RAD : 1;
    constexpr int LGR = RAD == 2 ? 1 : (RAD == 4 ? 2 : 3);
    constexpr int RIN = HIN ? RAD / 2 : RAD;
    static_assert(PER * RIN <= FirstIn<R, EMAX, HIN>::N, "first-pass register budget");
    const int lgnb = lgL - LGR;
    const int total = (1 << lgnb) * nseq;
    const int tid = tid_opaque();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int t = tid + i * kNT;
        if (t < total) {
            int b, j;
            seq_split<LAYOUT, NC>(t, lgT, lgnb, nseq, b, j);
#pragma unroll
            for (int r = 0; r < RIN; ++r) in.v[i * RIN + r] = load(b, j + (r << lgnb));
        }
    }
}

template <typename R, int EMAX, int LAYOUT, int NC, bool HIN, class Load>
__device__ __forceinline__ void first_load(FirstIn<R, EMAX, HIN>& in, int lgL, int lgT, int nseq, Load load) {
    const int rem = lgL % 3;
    if (rem == 1) first_load_rad<R, 2, EMAX, LAYOUT, NC, HIN>(in, lgL, lgT, nseq, load);
    else if (rem == 2) first_load_rad<R, 4, EMAX, LAYOUT, NC, HIN>(in, lgL, lgT, nseq, load);
    else first_load_rad<R, 8, EMAX, LAYOUT, NC, HIN>(in, lgL, lgT, nseq, load);
}

// fft_io with the first pass taken from registers (filled by first_load);
// after_first() runs once the first pass has consumed them, typically to
// issue the next tile's first_load.  Requires lgL >= 1.
template <typename R, bool INV, int EMAX, bool DST_LDS, int LAYOUT, int NC, bool HALF_IN, bool HALF_OUT, class After,
          class Store>
__device__ __forceinline__ void fft_reg(cx<R>* __restrict__ buf, int lgL, int lgT, int nseq,
                                        FirstIn<R, EMAX, HALF_IN>& in, After after_first, Store store) {
    auto none_load = [](int, int) -> cx<R> { return mk<R>((R)0, (R)0); };
    struct NoIn { cx<R> v[1]; } noin;
    const int rem = lgL % 3;
    int lgNs = 0, left = lgL;
#define MAGX_RPASS(RADIX, S, D, HI, HO, IN) \
    stockham_io_pass<R, RADIX, INV, EMAX, S, D, LAYOUT, NC, HI, HO>(buf, lgL, lgNs, lgT, nseq, none_load, store, IN)
    {
        const int r0 = rem ? rem : 3;
        const bool last = left == r0;
        if (r0 == 1) {
            if (last) MAGX_RPASS(2, kSrcReg, DST_LDS, HALF_IN, HALF_OUT, in);
            else MAGX_RPASS(2, kSrcReg, true, HALF_IN, false, in);
        } else if (r0 == 2) {
            if (last) MAGX_RPASS(4, kSrcReg, DST_LDS, HALF_IN, HALF_OUT, in);
            else MAGX_RPASS(4, kSrcReg, true, HALF_IN, false, in);
        } else {
            if (last) MAGX_RPASS(8, kSrcReg, DST_LDS, HALF_IN, HALF_OUT, in);
            else MAGX_RPASS(8, kSrcReg, true, HALF_IN, false, in);
        }
        lgNs += r0;
        left -= r0;
    }
    after_first();
    while (left > 0) {
        const bool last = (left == 3);
        if (last) MAGX_RPASS(8, kSrcLds, DST_LDS, false, HALF_OUT, noin);
        else MAGX_RPASS(8, kSrcLds, true, false, false, noin);
        lgNs += 3;
        left -= 3;
    }
#undef MAGX_RPASS
}

// Division of 0 <= n < 2^31 by a divisor fixed at launch: with
// l = ceil(log2 d) and m = floor(2^(32+l) / d) - 2^32 + 1,
// n / d = (mulhi(n, m) + n) >> l (mulhi(n, m) < n keeps the sum in 32 bits).
struct FastDiv {
    unsigned m;
    int l;
};

inline FastDiv make_fastdiv(int d) {
    FastDiv f;
    int l = 0;
    while ((1LL << l) < (long long)d) ++l;
    f.l = l;
    f.m = (unsigned)((((unsigned long long)1 << (32 + l)) / (unsigned long long)d) - ((unsigned long long)1 << 32) + 1);
    return f;
}

__device__ __forceinline__ int fdiv(int n, const FastDiv& f) {
    return (int)((__umulhi((unsigned)n, f.m) + (unsigned)n) >> f.l);
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
