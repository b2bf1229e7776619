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

// ---- LDS Stockham FFT ------------------------------------------------------------
// nseq independent sequences of length L = 2^lgL (1 <= L <= 4096) live in LDS;
// element j of sequence b is at buf[b*bs + j*es].  If seq_fast, consecutive
// threads take consecutive sequences (column tiles, es > 1); otherwise
// consecutive positions within a sequence (contiguous lines, es == 1).
// Each thread holds at most EMAX elements, i.e. nseq*L <= kNT*EMAX.  All
// threads of the block must call; the routine begins and ends with a barrier.
// Unnormalised: the inverse is the conjugate-twiddle transform.
template <typename R, int RAD, bool INV, int EMAX>
__device__ __forceinline__ void stockham_pass(cx<R>* buf, int lgL, int lgNs, int nseq, int bs,
                                              int es, bool seq_fast) {
    constexpr int PER = EMAX / RAD > 0 ? EMAX / RAD : 1;
    constexpr int LGR = RAD == 2 ? 1 : (RAD == 4 ? 2 : 3);
    const int lgnb = lgL - LGR;          // log2 butterflies per sequence
    const int nb = 1 << lgnb;
    const int total = nb * nseq;
    const int Ns = 1 << lgNs;
    const int twshift = kTwLog - LGR - lgNs;   // w_{RAD*Ns}^{rk} = table[(r*k) << twshift]
    cx<R> v[PER][RAD];
    int base[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int t = threadIdx.x + i * kNT;
        if (t < total) {
            int b, j;
            if (seq_fast) { b = t % nseq; j = t / nseq; }
            else { b = t >> lgnb; j = t & (nb - 1); }
            base[i] = b * bs;
            const cx<R>* src = buf + b * bs + j * es;
#pragma unroll
            for (int r = 0; r < RAD; ++r) v[i][r] = src[(r << lgnb) * es];
            // twiddle and butterfly in registers
            const int k = j & (Ns - 1);
#pragma unroll
            for (int r = 1; r < RAD; ++r) {
                if (k) v[i][r] = cmul<R>(v[i][r], tw<R, INV>((r * k) << twshift));
            }
            dft<R, RAD, INV>(v[i]);
            // destination index of output r: ((j >> lgNs) * RAD + r) * Ns + k
            base[i] += (((j >> lgNs) * RAD) * Ns + k) * es;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int t = threadIdx.x + i * kNT;
        if (t < total) {
            cx<R>* dst = buf + base[i];
#pragma unroll
            for (int r = 0; r < RAD; ++r) dst[(r * Ns) * es] = v[i][r];
        }
    }
    __syncthreads();
}

template <typename R, bool INV, int EMAX>
__device__ __forceinline__ void lds_fft(cx<R>* buf, int lgL, int nseq, int bs, int es, bool seq_fast) {
    __syncthreads();
    int lgNs = 0;
    int rem = lgL;
    while (rem >= 3) {
        stockham_pass<R, 8, INV, EMAX>(buf, lgL, lgNs, nseq, bs, es, seq_fast);
        lgNs += 3;
        rem -= 3;
    }
    if (rem == 2) stockham_pass<R, 4, INV, EMAX>(buf, lgL, lgNs, nseq, bs, es, seq_fast);
    else if (rem == 1) stockham_pass<R, 2, INV, EMAX>(buf, lgL, lgNs, nseq, bs, es, seq_fast);
}

__host__ __device__ inline int ilog2(int v) {
    int r = 0;
    while ((1 << r) < v) ++r;
    return r;
}

}  // namespace magx
