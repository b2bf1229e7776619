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

constexpr int kNT = 256;          // threads per block of the pencil kernels (and default of the FFT core)
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
template <> __device__ __forceinline__ float2 tw_fwd<float>(int k) { return g_tw32[(unsigned)k]; }
template <> __device__ __forceinline__ double2 tw_fwd<double>(int k) { return g_tw64[(unsigned)k]; }
// w^k for a transform of direction INV; k indexes the 4096-point table.
template <typename R, bool INV> __device__ __forceinline__ cx<R> tw(int k) {
    cx<R> w = tw_fwd<R>(k);
    return INV ? cconj<R>(w) : w;
}

// Two-level copy of the twiddle table in LDS for the FFT passes of a block:
// W^k = W^(64 (k >> 6)) W^(k & 63) (W = exp(-2 pi i / 4096)), 128 entries.
// A pass twiddle then costs two LDS reads and a complex product instead of a
// global (L2) load.  Every kernel that asks the passes for it (TWL) fills it
// with tw_lds_fill before its first barrier.
template <typename R> __device__ __forceinline__ cx<R>* tw_lds() {
    __shared__ cx<R> t[128];
    return t;
}
template <typename R> __device__ __forceinline__ void tw_lds_fill() {
    cx<R>* t = tw_lds<R>();
    for (int i = threadIdx.x; i < 128; i += blockDim.x) t[i] = tw_fwd<R>(i < 64 ? i : (i - 64) << 6);
}
template <typename R, bool INV, bool TWL> __device__ __forceinline__ cx<R> tw_pass(int k) {
    if constexpr (TWL) {
        const cx<R>* t = tw_lds<R>();
        const cx<R> w = cmul<R>(t[64 + (k >> 6)], t[k & 63]);
        return INV ? cconj<R>(w) : w;
    } else {
        return tw<R, INV>(k);
    }
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

// cos(pi j / 16), j = 0..8 (the 32nd roots of unity follow by symmetry)
constexpr double kCos16[9] = {1.0,
                              0.98078528040323044913,
                              0.92387953251128675613,
                              0.83146961230254523708,
                              0.70710678118654752440,
                              0.55557023301960222474,
                              0.38268343236508977173,
                              0.19509032201612826785,
                              0.0};

// cos and sin of 2 pi m / 32 for 0 <= m < 32
constexpr double cos32(int m) {
    m &= 31;
    return m <= 8 ? kCos16[m] : (m <= 16 ? -kCos16[16 - m] : (m <= 24 ? -kCos16[m - 16] : kCos16[32 - m]));
}
constexpr double sin32(int m) { return cos32(m - 8); }

// a * W_32^M with W_32 = exp(-2 pi i / 32) (forward) or its conjugate
// (inverse); the quarter turns are exact.
template <typename R, bool INV, int M>
__device__ __forceinline__ cx<R> mul_w32(cx<R> a) {
    constexpr int m = M & 31;
    if constexpr (m == 0) return a;
    else if constexpr (m == 8) return mul_mi<R, INV>(a);
    else if constexpr (m == 16) return mk<R>(-a.x, -a.y);
    else if constexpr (m == 24) return mul_mi<R, !INV>(a);
    else {
        constexpr R c = (R)cos32(m);
        constexpr R sn = INV ? (R)sin32(m) : (R)-sin32(m);
        return mk<R>(a.x * c - a.y * sn, a.x * sn + a.y * c);
    }
}

// Length 16 = 4 x 4 and 32 = 8 x 4 (Cooley-Tukey, n = 4 n1 + n2,
// k = k1 + N1 k2): DFTs of length N1 over n1, twiddles W_N^(n2 k1), DFTs of
// length 4 over n2.  Natural order in and out.
template <typename R, bool INV> __device__ __forceinline__ void dft16(cx<R>* v) {
    cx<R> y[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
#pragma unroll
        for (int n1 = 0; n1 < 4; ++n1) y[n2][n1] = v[4 * n1 + n2];
        dft4<R, INV>(y[n2]);
    }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        cx<R> u[4];
        u[0] = y[0][k1];
        if (k1 == 0) { u[1] = y[1][0]; u[2] = y[2][0]; u[3] = y[3][0]; }
        else if (k1 == 1) { u[1] = mul_w32<R, INV, 2>(y[1][1]); u[2] = mul_w32<R, INV, 4>(y[2][1]); u[3] = mul_w32<R, INV, 6>(y[3][1]); }
        else if (k1 == 2) { u[1] = mul_w32<R, INV, 4>(y[1][2]); u[2] = mul_w32<R, INV, 8>(y[2][2]); u[3] = mul_w32<R, INV, 12>(y[3][2]); }
        else { u[1] = mul_w32<R, INV, 6>(y[1][3]); u[2] = mul_w32<R, INV, 12>(y[2][3]); u[3] = mul_w32<R, INV, 18>(y[3][3]); }
        dft4<R, INV>(u);
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = u[k2];
    }
}

template <typename R, bool INV, int N2, int K1>
__device__ __forceinline__ cx<R> tw32_n2k1(cx<R> a) {
    return mul_w32<R, INV, N2 * K1>(a);
}

template <typename R, bool INV> __device__ __forceinline__ void dft32(cx<R>* v) {
    cx<R> y[4][8];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
#pragma unroll
        for (int n1 = 0; n1 < 8; ++n1) y[n2][n1] = v[4 * n1 + n2];
        dft8<R, INV>(y[n2]);
    }
    // W_32^(n2 k1) with compile-time exponents
#define MAGX_TW(K1)                                       \
    {                                                     \
        cx<R> u[4];                                       \
        u[0] = y[0][K1];                                  \
        u[1] = tw32_n2k1<R, INV, 1, K1>(y[1][K1]);        \
        u[2] = tw32_n2k1<R, INV, 2, K1>(y[2][K1]);        \
        u[3] = tw32_n2k1<R, INV, 3, K1>(y[3][K1]);        \
        dft4<R, INV>(u);                                  \
        for (int k2 = 0; k2 < 4; ++k2) v[K1 + 8 * k2] = u[k2]; \
    }
    MAGX_TW(0) MAGX_TW(1) MAGX_TW(2) MAGX_TW(3) MAGX_TW(4) MAGX_TW(5) MAGX_TW(6) MAGX_TW(7)
#undef MAGX_TW
}

template <typename R, int RAD, bool INV> __device__ __forceinline__ void dft(cx<R>* v) {
    if constexpr (RAD == 2) dft2<R, INV>(v);
    else if constexpr (RAD == 4) dft4<R, INV>(v);
    else if constexpr (RAD == 8) dft8<R, INV>(v);
    else if constexpr (RAD == 16) dft16<R, INV>(v);
    else dft32<R, INV>(v);
}

constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v >> 1); }

// ---- Stockham FFTs in LDS ----------------------------------------------------------
// nseq independent sequences of length L = 2^lgL (1 <= L <= 4096).  Two LDS
// layouts:
//  * columns (LAYOUT = kCols): nseq = NC << lgT sequences, element j of
//    sequence b at b + j*nseq; consecutive threads take consecutive b
//    (coalesced column tiles; NC = 1 or 3 is a compile-time constant so the
//    thread -> (b, j) split needs no runtime division);
//  * lines (LAYOUT = kLines): element j of sequence b at (b << lgL) + j;
//    consecutive threads take consecutive j.
// Each of the NT threads of the block holds at most EMAX elements
// (nseq * L <= NT * EMAX).
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
__device__ __forceinline__ unsigned umul24(unsigned a, unsigned b) { return __umul24(a, b); }

// threadIdx.x behind an empty volatile asm statement: index arithmetic derived
// from it is recomputed in each pass instead of being hoisted out of a tile
// loop and held in registers across it.
__device__ __forceinline__ int tid_opaque() {
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// v[r] *= w^(r k), r = 1..RAD-1, for the pass twiddle w: w^k, w^2k, w^4k, ...
// come from the table and every other power is a product of those (at most
// log2(RAD) - 1 products deep).
template <typename R, bool INV, int RAD, bool TWL = false>
__device__ __forceinline__ void twiddle_apply(cx<R>* v, int k, int twshift) {
    if (!k) return;
    cx<R> w[RAD];
#pragma unroll
    for (int p = 1; p < RAD; p <<= 1) w[p] = tw_pass<R, INV, TWL>((p * k) << twshift);
#pragma unroll
    for (int r = 3; r < RAD; ++r) {
        if ((r & (r - 1)) == 0) continue;
        const int hi = 1 << ilog2c(r);
        w[r] = cmul<R>(w[hi], w[r - hi]);
    }
#pragma unroll
    for (int r = 1; r < RAD; ++r) v[r] = cmul<R>(v[r], w[r]);
}

// Thread slot t -> (sequence b, butterfly j); unsigned arithmetic throughout
// (no sign fix-ups in shifts and divisions).
template <int LAYOUT, int NC>
__device__ __forceinline__ void seq_split(unsigned t, int lgT, int lgnb, unsigned nseq, unsigned& b, unsigned& j) {
    if constexpr (LAYOUT == kLines) {
        b = t >> lgnb;
        j = t & ((1u << lgnb) - 1u);
    } else if constexpr (NC == 1) {
        b = t & (nseq - 1u);
        j = t >> lgT;
    } else {
        j = (t >> lgT) / (unsigned)NC;
        b = t - umul24(j, nseq);
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
          bool HOUT, int NT, bool TWL, class Load, class Store, class In>
__device__ __forceinline__ void stockham_io_pass(cx<R>* __restrict__ buf, int lgL, int lgNs, int lgT, int nseq,
                                                 Load& load, Store& store, In& in) {
    constexpr bool SRC_LDS = SRC == kSrcLds;
    constexpr int PER = EMAX / RAD > 0 ? EMAX / RAD : 1;
    constexpr int LGR = ilog2c(RAD);
    const int lgnb = lgL - LGR;
    const unsigned nb = 1u << lgnb;
    const unsigned total = nb * (unsigned)nseq;
    const unsigned Ns = 1u << lgNs;
    const int twshift = kTwLog - LGR - lgNs;
    // uniform strides between the RAD inputs / outputs of one butterfly
    const unsigned in_stride = LAYOUT == kLines ? nb : (nb * (unsigned)nseq);
    const unsigned out_stride = LAYOUT == kLines ? Ns : (Ns * (unsigned)nseq);
    cx<R> v[PER][RAD];
    unsigned seqv[PER], pos0[PER], obase[PER];
    const unsigned tid = (unsigned)tid_opaque();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const unsigned t = tid + (unsigned)(i * NT);
        if (t < total) {
            unsigned b, j;
            seq_split<LAYOUT, NC>(t, lgT, lgnb, (unsigned)nseq, b, j);
            seqv[i] = b;
            // with HIN the inputs r >= RAD/2 lie in the zero half (first pass: lgNs = 0)
            constexpr int RIN = HIN ? RAD / 2 : RAD;
            if constexpr (SRC == kSrcReg) {
#pragma unroll
                for (int r = 0; r < RIN; ++r) v[i][r] = in.v[i * RIN + r];
            } else if constexpr (SRC_LDS) {
                const unsigned ib = LAYOUT == kLines ? (b << lgL) + j : b + umul24(j, (unsigned)nseq);
#pragma unroll
                for (int r = 0; r < RIN; ++r) v[i][r] = buf[ib + (unsigned)r * in_stride];
            } else {
#pragma unroll
                for (int r = 0; r < RIN; ++r) v[i][r] = load((int)b, (int)(j + ((unsigned)r << lgnb)));
            }
#pragma unroll
            for (int r = RIN; r < RAD; ++r) v[i][r] = mk<R>((R)0, (R)0);
            const unsigned k = j & (Ns - 1u);
            pos0[i] = ((j >> lgNs) << (lgNs + LGR)) + k;
            obase[i] = LAYOUT == kLines ? (b << lgL) + pos0[i] : b + umul24(pos0[i], (unsigned)nseq);
            twiddle_apply<R, INV, RAD, TWL>(v[i], (int)k, twshift);
            dft<R, RAD, INV>(v[i]);
        }
    }
    if constexpr (SRC_LDS && DST_LDS) __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const unsigned t = tid + (unsigned)(i * NT);
        if (t < total) {
#pragma unroll
            // with HOUT the outputs r >= RAD/2 land in the unwanted half (last pass)
            for (int r = 0; r < (HOUT ? RAD / 2 : RAD); ++r) {
                if constexpr (DST_LDS) buf[obase[i] + (unsigned)r * out_stride] = v[i][r];
                else store((int)seqv[i], (int)(pos0[i] + (unsigned)r * Ns), v[i][r]);
            }
        }
    }
    if constexpr (DST_LDS) __syncthreads();
}

// Pass plan: radices up to 2^lgmax<EMAX>() (32 when a thread holds 32
// elements, 16 for 16, else 8); the remainder radix 2^(lgL mod lgmax) comes
// first, then full-size passes.  Fewer, larger passes mean fewer LDS round
// trips and barriers per transform.
template <int EMAX> constexpr int lgmax() { return EMAX >= 32 ? 5 : (EMAX >= 16 ? 4 : 3); }

// Calls MAGX_BODY(RAD) with RAD = 2^lg for a runtime lg in [1, LGM].
#define MAGX_RADIX_SWITCH(lg, LGM)                        \
    switch (lg) {                                         \
        case 1: MAGX_BODY(2); break;                      \
        case 2: MAGX_BODY(4); break;                      \
        case 3: MAGX_BODY(8); break;                      \
        case 4: if constexpr ((LGM) >= 4) { MAGX_BODY(16); } break; \
        default: if constexpr ((LGM) >= 5) { MAGX_BODY(32); } break; \
    }

template <typename R, bool INV, int EMAX, bool SRC_LDS, bool DST_LDS, int LAYOUT, int NC, bool HALF_IN = false,
          bool HALF_OUT = false, int LGM = lgmax<EMAX>(), int NT = kNT, bool TWL = false, class Load, class Store>
__device__ __forceinline__ void fft_io(cx<R>* __restrict__ buf, int lgL, int lgT, int nseq, Load load, Store store) {
    if (lgL == 0) {   // length 1: the transform is the identity
        for (int b = threadIdx.x; b < nseq; b += NT) {
            cx<R> x;
            if constexpr (SRC_LDS) x = buf[b];
            else x = load(b, 0);
            if constexpr (DST_LDS) buf[b] = x;
            else store(b, 0, x);
        }
        if constexpr (DST_LDS) __syncthreads();
        return;
    }
    static_assert(LGM >= 3 && LGM <= lgmax<EMAX>(), "pass radix beyond the register budget");
    const int rem = lgL % LGM;
    int lgNs = 0, left = lgL;
    // first pass: source SRC_LDS, zero upper half if HALF_IN; last pass:
    // destination DST_LDS, lower half only if HALF_OUT; LDS in between
    struct NoIn { cx<R> v[1]; } noin;
    {
        const int g = rem ? rem : LGM;
        const bool last = left == g;
#define MAGX_BODY(RADIX)                                                                                          \
    if (last)                                                                                                     \
        stockham_io_pass<R, RADIX, INV, EMAX, SRC_LDS ? kSrcLds : kSrcFn, DST_LDS, LAYOUT, NC, HALF_IN, HALF_OUT, NT, TWL>(  \
            buf, lgL, lgNs, lgT, nseq, load, store, noin);                                                        \
    else                                                                                                          \
        stockham_io_pass<R, RADIX, INV, EMAX, SRC_LDS ? kSrcLds : kSrcFn, true, LAYOUT, NC, HALF_IN, false, NT, TWL>(      \
            buf, lgL, lgNs, lgT, nseq, load, store, noin);
        MAGX_RADIX_SWITCH(g, LGM)
#undef MAGX_BODY
        lgNs += g;
        left -= g;
    }
    while (left > 0) {
        constexpr int RADIX = 1 << LGM;
        if (left == LGM)
            stockham_io_pass<R, RADIX, INV, EMAX, kSrcLds, DST_LDS, LAYOUT, NC, false, HALF_OUT, NT, TWL>(
                buf, lgL, lgNs, lgT, nseq, load, store, noin);
        else
            stockham_io_pass<R, RADIX, INV, EMAX, kSrcLds, true, LAYOUT, NC, false, false, NT, TWL>(
                buf, lgL, lgNs, lgT, nseq, load, store, noin);
        lgNs += LGM;
        left -= LGM;
    }
}

// Loads the first pass's inputs of one tile into `in` (lgL >= 1), in the
// order the register-sourced first pass of fft_reg consumes them.
template <typename R, int RAD, int EMAX, int LAYOUT, int NC, bool HIN, int NT, class Load>
__device__ __forceinline__ void first_load_rad(FirstIn<R, EMAX, HIN>& in, int lgL, int lgT, int nseq, Load& load) {
    constexpr int PER = EMAX / RAD > 0 ? EMAX / RAD : 1;
    constexpr int LGR = ilog2c(RAD);
    constexpr int RIN = HIN ? RAD / 2 : RAD;
    static_assert(PER * RIN <= FirstIn<R, EMAX, HIN>::N, "first-pass register budget");
    const int lgnb = lgL - LGR;
    const unsigned total = (1u << lgnb) * (unsigned)nseq;
    const unsigned tid = (unsigned)tid_opaque();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const unsigned t = tid + (unsigned)(i * NT);
        if (t < total) {
            unsigned b, j;
            seq_split<LAYOUT, NC>(t, lgT, lgnb, (unsigned)nseq, b, j);
#pragma unroll
            for (int r = 0; r < RIN; ++r) in.v[i * RIN + r] = load((int)b, (int)(j + ((unsigned)r << lgnb)));
        }
    }
}

template <typename R, int EMAX, int LAYOUT, int NC, bool HIN, int LGM = lgmax<EMAX>(), int NT = kNT, class Load>
__device__ __forceinline__ void first_load(FirstIn<R, EMAX, HIN>& in, int lgL, int lgT, int nseq, Load load) {
    const int rem = lgL % LGM;
    const int g = rem ? rem : LGM;
#define MAGX_BODY(RADIX) first_load_rad<R, RADIX, EMAX, LAYOUT, NC, HIN, NT>(in, lgL, lgT, nseq, load);
    MAGX_RADIX_SWITCH(g, LGM)
#undef MAGX_BODY
}

// Replaces every value held for the first pass by f(b, j, value), where
// (b, j) is the sequence and the element index first_load gave it; entries
// first_load did not fill are left alone.
template <typename R, int RAD, int EMAX, int LAYOUT, int NC, bool HIN, int NT, class F>
__device__ __forceinline__ void first_apply_rad(FirstIn<R, EMAX, HIN>& in, int lgL, int lgT, int nseq, F& f) {
    constexpr int PER = EMAX / RAD > 0 ? EMAX / RAD : 1;
    constexpr int LGR = ilog2c(RAD);
    constexpr int RIN = HIN ? RAD / 2 : RAD;
    const int lgnb = lgL - LGR;
    const unsigned total = (1u << lgnb) * (unsigned)nseq;
    const unsigned tid = (unsigned)tid_opaque();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const unsigned t = tid + (unsigned)(i * NT);
        if (t < total) {
            unsigned b, j;
            seq_split<LAYOUT, NC>(t, lgT, lgnb, (unsigned)nseq, b, j);
#pragma unroll
            for (int r = 0; r < RIN; ++r)
                in.v[i * RIN + r] = f((int)b, (int)(j + ((unsigned)r << lgnb)), in.v[i * RIN + r]);
        }
    }
}

template <typename R, int EMAX, int LAYOUT, int NC, bool HIN, int LGM = lgmax<EMAX>(), int NT = kNT, class F>
__device__ __forceinline__ void first_apply(FirstIn<R, EMAX, HIN>& in, int lgL, int lgT, int nseq, F f) {
    const int rem = lgL % LGM;
    const int g = rem ? rem : LGM;
#define MAGX_BODY(RADIX) first_apply_rad<R, RADIX, EMAX, LAYOUT, NC, HIN, NT>(in, lgL, lgT, nseq, f);
    MAGX_RADIX_SWITCH(g, LGM)
#undef MAGX_BODY
}

// fft_io with the first pass taken from registers (filled by first_load);
// after_first() runs once the first pass has consumed them, typically to
// issue the next tile's first_load.  Requires lgL >= 1.
template <typename R, bool INV, int EMAX, bool DST_LDS, int LAYOUT, int NC, bool HALF_IN, bool HALF_OUT,
          int LGM = lgmax<EMAX>(), int NT = kNT, bool TWL = false, class After, class Store>
__device__ __forceinline__ void fft_reg(cx<R>* __restrict__ buf, int lgL, int lgT, int nseq,
                                        FirstIn<R, EMAX, HALF_IN>& in, After after_first, Store store) {
    static_assert(LGM >= 3 && LGM <= lgmax<EMAX>(), "pass radix beyond the register budget");
    auto none_load = [](int, int) -> cx<R> { return mk<R>((R)0, (R)0); };
    struct NoIn { cx<R> v[1]; } noin;
    const int rem = lgL % LGM;
    int lgNs = 0, left = lgL;
    {
        const int g = rem ? rem : LGM;
        const bool last = left == g;
#define MAGX_BODY(RADIX)                                                                                     \
    if (last)                                                                                                \
        stockham_io_pass<R, RADIX, INV, EMAX, kSrcReg, DST_LDS, LAYOUT, NC, HALF_IN, HALF_OUT, NT, TWL>(              \
            buf, lgL, lgNs, lgT, nseq, none_load, store, in);                                                \
    else                                                                                                     \
        stockham_io_pass<R, RADIX, INV, EMAX, kSrcReg, true, LAYOUT, NC, HALF_IN, false, NT, TWL>(buf, lgL, lgNs, lgT, \
                                                                                         nseq, none_load,    \
                                                                                         store, in);
        MAGX_RADIX_SWITCH(g, LGM)
#undef MAGX_BODY
        lgNs += g;
        left -= g;
    }
    after_first();
    while (left > 0) {
        constexpr int RADIX = 1 << LGM;
        if (left == LGM)
            stockham_io_pass<R, RADIX, INV, EMAX, kSrcLds, DST_LDS, LAYOUT, NC, false, HALF_OUT, NT, TWL>(
                buf, lgL, lgNs, lgT, nseq, none_load, store, noin);
        else
            stockham_io_pass<R, RADIX, INV, EMAX, kSrcLds, true, LAYOUT, NC, false, false, NT, TWL>(
                buf, lgL, lgNs, lgT, nseq, none_load, store, noin);
        lgNs += LGM;
        left -= LGM;
    }
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

// Streaming (non-temporal) global accesses of complex values.  A pass whose
// output is read only by the next pass stores it this way, and the inverse y
// pass loads its input this way: measured at 512 x 512 x 32, the consumer of
// streamed data runs faster (inverse y pass 155 -> 126 us, z pass 229 -> 217 us)
// than when the same lines are written through the caches.
template <typename R> __device__ __forceinline__ void st_stream(cx<R>* p, cx<R> v) {
    typedef R V __attribute__((ext_vector_type(2)));
    V t;
    t.x = v.x;
    t.y = v.y;
    __builtin_nontemporal_store(t, reinterpret_cast<V*>(p));
}
template <typename R> __device__ __forceinline__ cx<R> ld_stream(const cx<R>* p) {
    typedef R V __attribute__((ext_vector_type(2)));
    const V t = __builtin_nontemporal_load(reinterpret_cast<const V*>(p));
    return mk<R>(t.x, t.y);
}

// Element at a 32-bit byte offset from a base pointer: with a uniform base
// the access is one scalar-base + 32-bit vector-offset instruction, without
// 64-bit address arithmetic per lane.  The caller guarantees off < 2^32.
template <typename R> __device__ __forceinline__ R ld_off(const R* base, unsigned off) {
    return *reinterpret_cast<const R*>(reinterpret_cast<const char*>(base) + off);
}

// A complex value that is the same in every lane of the wave, moved to
// scalar registers (operands of vector instructions without occupying
// vector registers).
__device__ __forceinline__ unsigned uniform_u32(unsigned v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uniform_r(float v) { return __uint_as_float(uniform_u32(__float_as_uint(v))); }
__device__ __forceinline__ double uniform_r(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned long long lo = uniform_u32((unsigned)b), hi = uniform_u32((unsigned)(b >> 32));
    return __longlong_as_double((long long)((hi << 32) | lo));
}
template <typename R> __device__ __forceinline__ cx<R> wave_uniform(cx<R> v) {
    return mk<R>(uniform_r(v.x), uniform_r(v.y));
}

// An empty statement that takes v in vector registers and may change it: the
// computation of v stays before this point (the compiler may otherwise sink
// pure arithmetic past a barrier, keeping all of its inputs live instead).
template <typename R> __device__ __forceinline__ void keep_in_regs(cx<R>& v) {
    asm volatile("" : "+v"(v.x), "+v"(v.y));
}

__host__ __device__ inline int ilog2(int v) {
    int r = 0;
    while ((1 << r) < v) ++r;
    return r;
}

}  // namespace magx
