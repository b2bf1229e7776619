// Strided passes of the demag FFT convolution (Section II-B, Eq. (3)).
//
// Each block owns a tile of T consecutive kx columns (contiguous in memory,
// coalesced row segments) and transforms them along y or z in LDS.
//  * yfwd : rows y < ny are loaded, rows ny..Py-1 are the zero padding and
//           never read from memory; all Py output rows are written.
//  * zconv: for one ky, all three components: forward z FFT (rows z >= nz
//           are zero padding), then the pointwise product with the real
//           symmetric tensor spectrum, H_a = -Ms sum_b N_ab M_b (tensor values
//           held in registers), then the inverse z FFT; only rows z < nz are
//           written back (in place).  Single precision with Pz = 8 ... 64
//           has a register-resident variant (zconvr).
//  * yinv : inverse y FFT; only rows y < ny (inside the box) are written.
// FFT pass twiddles come from a two-level LDS table filled by each block.
// yfwd, zconv and yinv write their outputs with streaming stores, and yinv
// reads its input with streaming loads (see st_stream).
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

#include "magx_internal.hpp"

namespace magx {

// EM: FFT elements held per thread (T * L <= kNT * EM); 16 or 32.
//
// Every kernel is persistent: the launch has as many blocks as can be
// resident, and block lb walks the contiguous tile range
// [ntiles*lb/G, ntiles*(lb+1)/G) (logical blocks of one XCD are contiguous,
// so neighbouring tiles share its L2).  The first FFT pass of a tile takes its
// inputs from registers, and right after it the next tile's inputs are
// requested, so the loads of tile t+1 are in flight while tile t finishes.

// Walk of a block of a pair over the y-pass tiles (plane, tx): units are
// (plane, txp) with txp = tx / 2; a pair of blocks (adjacent logical indices,
// one XCD) shares a contiguous unit range and its even / odd block takes
// column tile 2 txp / 2 txp + 1 (skipped when past the last tile).
struct PairWalk {
    int ntx, ntxp, side, u0, u1;
    __device__ PairWalk(int ntiles, int ntx_) : ntx(ntx_) {
        ntxp = (ntx + 1) >> 1;
        const int lbp = xcd_logical_block(blockIdx.x, gridDim.x);
        side = lbp & 1;
        const int npairs = gridDim.x >> 1, pr = lbp >> 1;
        const long long nunits = (long long)(ntiles / ntx) * ntxp;
        u0 = (int)(nunits * pr / npairs);
        u1 = (int)(nunits * (pr + 1) / npairs);
    }
    __device__ bool valid(int u) const { return 2 * (u % ntxp) + side < ntx; }
    __device__ int first() const {
        int u = u0;
        while (u < u1 && !valid(u)) ++u;
        return u;
    }
    __device__ int next(int u) const {
        ++u;
        while (u < u1 && !valid(u)) ++u;
        return u;
    }
    __device__ int tile(int u) const { return (u / ntxp) * ntx + 2 * (u % ntxp) + side; }
};

// Compile-time geometry of the y passes for square power-of-two grids,
// nx = ny = 2^(LG-1) (Px = Py = 2^LG): every size of the pass (row stride,
// tile width, tile count) becomes a constant, so the FFT strides and row
// offsets are immediates.  LG = 0 keeps runtime sizes.  The tile width is the
// plan's, ty = min(16, budget / Py) with a budget of 2^14 complex values in
// single precision and in double precision 2^13 for Py >= 1024, 2^12 below
// (128 KiB and 64 KiB of LDS; at Py = 512 the smaller tile measured faster).
template <typename R> constexpr int ytile_lg(int LG) {
    constexpr int lgb = sizeof(R) == 4 ? 14 : 13;
    if constexpr (sizeof(R) == 8) {
        if (LG <= 9) return LG >= 8 ? 12 - LG : 4;
    }
    return LG >= lgb - 4 ? lgb - LG : 4;
}

template <typename R, int LG>
__device__ __forceinline__ void ygeom_fix(int& ny, int& lgPy, int& Hx, int& Sx, int& lgT, int& ntx) {
    if constexpr (LG > 0) {
        ny = 1 << (LG - 1);
        lgPy = LG;
        Hx = (1 << (LG - 1)) + 1;
        Sx = (1 << (LG - 1)) + 16;
        lgT = ytile_lg<R>(LG);
        ntx = (Hx + (1 << lgT) - 1) >> lgT;
    }
}

// Packed Nyquist column (plans with the single-precision register z pass,
// Py <= 1024): the value of row ky at column Lh = Hx - 1 is kept at row prow,
// column Lh + i instead.  Rows ky = q < Py/2 and the mirrored rows (q = Py - ky,
// q = 0 for ky = Py/2) go, 16 consecutive q at a time, to the padding columns
// Lh ... Lh + 15 of one row: prow = 16 floor(q/16) for the first kind,
// Py - 1 - 16 floor(q/16) for the second, i = q mod 16.  The z pass then reads
// 16 Nyquist values of a plane as one 128-byte segment.  Returns the element
// offset from column Lh of row 0.
__device__ __forceinline__ unsigned nyq_pack(int ky, int Py, unsigned Sx) {
    const int h = Py >> 1;
    const bool mirrored = ky >= h;
    const int q = ky < h ? ky : (ky == h ? 0 : Py - ky);
    const int k = q >> 4;
    const int prow = mirrored ? Py - 1 - 16 * k : 16 * k;
    return (unsigned)prow * Sx + (unsigned)(q & 15);
}

template <typename R, int EM, int NT, int LG>
__global__ void __launch_bounds__(NT) yfwd_kernel(const cx<R>* __restrict__ X1, cx<R>* __restrict__ X2, int ny,
                                                  int lgPy, int Hx, int Sx, int lgT, int ntx, int ntiles, int nyq) {
    ygeom_fix<R, LG>(ny, lgPy, Hx, Sx, lgT, ntx);
    tw_lds_fill<R>();   // read by the second pass, after the first barrier
    extern __shared__ unsigned char smem_raw[];
    cx<R>* buf = reinterpret_cast<cx<R>*>(smem_raw);
    const int T = 1 << lgT;
    const int Py = 1 << lgPy;
    // block pairs: unit u = (plane, column-tile pair); the even block of a pair
    // takes column tile 2 txp, the odd one 2 txp + 1, at the same time, so the
    // two halves of every 128-byte row segment are requested together
    const PairWalk pw(ntiles, ntx);
    // tile t: plane t / ntx (= c * nz + z), columns (t % ntx) * T ...
    // sequence b = column kx0 + b; rows >= ny are the zero padding, never read
    auto loader = [=](int t) {
        const int tx = t % ntx;
        const long long plane = t / ntx;
        const int kx0 = tx * T;
        const cx<R>* src = X1 + plane * ny * (long long)Sx + kx0;
        const int ncol = min(T, Hx - kx0);
        return [=](int b, int j) -> cx<R> {
            if (j < ny && b < ncol) return src[umul24((unsigned)j, (unsigned)Sx) + (unsigned)b];
            return mk<R>(0, 0);
        };
    };
    FirstIn<R, EM, true> in;
    int u = pw.first();
    if (u < pw.u1) first_load<R, EM, kCols, 1, true, lgmax<EM>(), NT>(in, lgPy, lgT, T, loader(pw.tile(u)));
    while (u < pw.u1) {
        const int un = pw.next(u);
        const int t = pw.tile(u);
        const int tx = t % ntx;
        const long long plane = t / ntx;
        const int kx0 = tx * T;
        cx<R>* dst = X2 + plane * Py * (long long)Sx + kx0;
        const int ncol = min(T, Hx - kx0);
        // with a packed Nyquist column, column Hx - 1 (b = ncol - 1 of the last tile) moves
        const int bnyq = nyq && kx0 + ncol == Hx ? ncol - 1 : -1;
        auto store = [&](int b, int j, cx<R> v) {
            if (b < ncol) {
                const unsigned off = b == bnyq ? nyq_pack(j, Py, (unsigned)Sx) : umul24((unsigned)j, (unsigned)Sx);
                st_stream<R>(&dst[off + (unsigned)b], v);
            }
        };
        auto next = [&]() {
            if (un < pw.u1)
                first_load<R, EM, kCols, 1, true, lgmax<EM>(), NT>(in, lgPy, lgT, T, loader(pw.tile(un)));
        };
        fft_reg<R, false, EM, false, kCols, 1, true, false, lgmax<EM>(), NT, true>(buf, lgPy, lgT, T, in, next, store);
        __syncthreads();   // the last pass read LDS; the next tile's first pass writes it
        u = un;
    }
}

template <typename R, int EM, int NT, int LG>
__global__ void __launch_bounds__(NT) yinv_kernel(const cx<R>* __restrict__ X2, cx<R>* __restrict__ Y1, int ny,
                                                  int lgPy, int Hx, int Sx, int lgT, int ntx, int ntiles, int nyq) {
    ygeom_fix<R, LG>(ny, lgPy, Hx, Sx, lgT, ntx);
    tw_lds_fill<R>();   // read by the second pass, after the first barrier
    extern __shared__ unsigned char smem_raw[];
    cx<R>* buf = reinterpret_cast<cx<R>*>(smem_raw);
    const int T = 1 << lgT;
    const int Py = 1 << lgPy;
    const PairWalk pw(ntiles, ntx);
    auto loader = [=](int t) {
        const int tx = t % ntx;
        const long long plane = t / ntx;
        const int kx0 = tx * T;
        const cx<R>* src = X2 + plane * Py * (long long)Sx + kx0;
        const int ncol = min(T, Hx - kx0);
        const int bnyq = nyq && kx0 + ncol == Hx ? ncol - 1 : -1;   // packed Nyquist column
        return [=](int b, int j) -> cx<R> {
            if (b < ncol) {
                const unsigned off = b == bnyq ? nyq_pack(j, Py, (unsigned)Sx) : umul24((unsigned)j, (unsigned)Sx);
                return ld_stream<R>(&src[off + (unsigned)b]);
            }
            return mk<R>(0, 0);
        };
    };
    FirstIn<R, EM, false> in;
    int u = pw.first();
    if (u < pw.u1) first_load<R, EM, kCols, 1, false, lgmax<EM>(), NT>(in, lgPy, lgT, T, loader(pw.tile(u)));
    while (u < pw.u1) {
        const int un = pw.next(u);
        const int t = pw.tile(u);
        const int tx = t % ntx;
        const long long plane = t / ntx;
        const int kx0 = tx * T;
        cx<R>* dst = Y1 + plane * ny * (long long)Sx + kx0;
        const int ncol = min(T, Hx - kx0);
        // only rows inside the box are written
        auto store = [&](int b, int j, cx<R> v) {
            if (j < ny && b < ncol) st_stream<R>(&dst[umul24((unsigned)j, (unsigned)Sx) + (unsigned)b], v);
        };
        auto next = [&]() {
            if (un < pw.u1)
                first_load<R, EM, kCols, 1, false, lgmax<EM>(), NT>(in, lgPy, lgT, T, loader(pw.tile(un)));
        };
        fft_reg<R, true, EM, false, kCols, 1, false, true, lgmax<EM>(), NT, true>(buf, lgPy, lgT, T, in, next, store);
        __syncthreads();
        u = un;
    }
}

// y passes for Py = 2048 (ny = 513 ... 1024) as two transforms of length 1024
// each, so a tile of 2^14 (single) or 2^13 (double) values spans 16 or 8
// columns instead of 8 or 4 (whole 128-byte row segments).
//  * forward, input rows n < ny: X[2k] = DFT_1024(x)[k] and
//    X[2k+1] = DFT_1024(x W_2048^n)[k]; the tile's inputs stay in registers
//    for the second transform, twiddled there.
//  * inverse, output rows n < ny <= 1024, by decimation in frequency:
//    x[2n] = IDFT_1024(X[k] + X[k+1024])[n] and
//    x[2n+1] = IDFT_1024((X[k] - X[k+1024]) W_2048^-k)[n], n < 512 (the last
//    pass computes only that half); both halves of the input are combined in
//    registers, the second waits there while the first is transformed, and
//    the next tile's input is fetched while the transforms run.  Radix-8
//    passes keep the two register sets within 128 registers (1024 threads).
template <typename R, int EM, int NT>
__global__ void __launch_bounds__(NT) yfwd2_kernel(const cx<R>* __restrict__ X1, cx<R>* __restrict__ X2, int ny,
                                                   int Hx, int Sx, int lgT, int ntx, int ntiles) {
    constexpr int LGL = 10, PY = 2048;
    tw_lds_fill<R>();   // read by the second pass, after the first barrier
    extern __shared__ unsigned char smem_raw[];
    cx<R>* buf = reinterpret_cast<cx<R>*>(smem_raw);
    const int T = 1 << lgT;
    const PairWalk pw(ntiles, ntx);
    auto loader = [=](int t) {
        const int tx = t % ntx;
        const long long plane = t / ntx;
        const int kx0 = tx * T;
        const cx<R>* src = X1 + plane * ny * (long long)Sx + kx0;
        const int ncol = min(T, Hx - kx0);
        return [=](int b, int j) -> cx<R> {
            if (j < ny && b < ncol) return src[umul24((unsigned)j, (unsigned)Sx) + (unsigned)b];
            return mk<R>(0, 0);
        };
    };
    FirstIn<R, EM, false> in;
    int u = pw.first();
    if (u < pw.u1) first_load<R, EM, kCols, 1, false, lgmax<EM>(), NT>(in, LGL, lgT, T, loader(pw.tile(u)));
    while (u < pw.u1) {
        const int un = pw.next(u);
        const int t = pw.tile(u);
        const int tx = t % ntx;
        const long long plane = t / ntx;
        const int kx0 = tx * T;
        cx<R>* dst = X2 + plane * PY * (long long)Sx + kx0;
        const int ncol = min(T, Hx - kx0);
        auto store_even = [&](int b, int j, cx<R> v) {
            if (b < ncol) st_stream<R>(&dst[umul24((unsigned)(2 * j), (unsigned)Sx) + (unsigned)b], v);
        };
        auto store_odd = [&](int b, int j, cx<R> v) {
            if (b < ncol) st_stream<R>(&dst[umul24((unsigned)(2 * j + 1), (unsigned)Sx) + (unsigned)b], v);
        };
        auto none = [&]() {};
        fft_reg<R, false, EM, false, kCols, 1, false, false, lgmax<EM>(), NT, true>(buf, LGL, lgT, T, in, none,
                                                                                     store_even);
        __syncthreads();   // the last pass read LDS; the second transform's first pass writes it
        // x[n] W_2048^n: entry 2n of the 4096-point table
        first_apply<R, EM, kCols, 1, false, lgmax<EM>(), NT>(
            in, LGL, lgT, T, [](int, int j, cx<R> v) { return cmul<R>(v, tw_pass<R, false, true>(j << 1)); });
        auto next = [&]() {
            if (un < pw.u1)
                first_load<R, EM, kCols, 1, false, lgmax<EM>(), NT>(in, LGL, lgT, T, loader(pw.tile(un)));
        };
        fft_reg<R, false, EM, false, kCols, 1, false, false, lgmax<EM>(), NT, true>(buf, LGL, lgT, T, in, next,
                                                                                     store_odd);
        __syncthreads();
        u = un;
    }
}

template <typename R, int EM, int NT>
__global__ void __launch_bounds__(NT) yinv2_kernel(const cx<R>* __restrict__ X2, cx<R>* __restrict__ Y1, int ny,
                                                   int Hx, int Sx, int lgT, int ntx, int ntiles) {
    constexpr int LGL = 10, PY = 2048;
    tw_lds_fill<R>();   // read by the second pass and by the twiddles W_2048^-k, after the first barrier
    extern __shared__ unsigned char smem_raw[];
    cx<R>* buf = reinterpret_cast<cx<R>*>(smem_raw);
    const int T = 1 << lgT;
    const PairWalk pw(ntiles, ntx);
    // rows k (half 0) or k + 1024 (half 1) of a tile: sequence b = column, element k
    auto loader = [=](int t, int half) {
        const int tx = t % ntx;
        const long long plane = t / ntx;
        const int kx0 = tx * T;
        const cx<R>* src = X2 + plane * PY * (long long)Sx + kx0 + (long long)half * 1024 * Sx;
        const int ncol = min(T, Hx - kx0);
        return [=](int b, int k) -> cx<R> {
            if (b < ncol) return ld_stream<R>(&src[umul24((unsigned)k, (unsigned)Sx) + (unsigned)b]);
            return mk<R>(0, 0);
        };
    };
    FirstIn<R, EM, false> lo, hi;
    int u = pw.first();
    if (u < pw.u1) {
        first_load<R, EM, kCols, 1, false, 3, NT>(lo, LGL, lgT, T, loader(pw.tile(u), 0));
        first_load<R, EM, kCols, 1, false, 3, NT>(hi, LGL, lgT, T, loader(pw.tile(u), 1));
    }
    bool first_tile = true;
    while (u < pw.u1) {
        const int un = pw.next(u);
        const int t = pw.tile(u);
        const int tx = t % ntx;
        const long long plane = t / ntx;
        const int kx0 = tx * T;
        cx<R>* dst = Y1 + plane * ny * (long long)Sx + kx0;
        const int ncol = min(T, Hx - kx0);
        if (first_tile) __syncthreads();   // the LDS twiddle table is complete
        first_tile = false;
        // u = X[k] + X[k + 1024] (in lo), v = (X[k] - X[k + 1024]) W_2048^-k (in hi)
#pragma unroll
        for (int e = 0; e < FirstIn<R, EM, false>::N; ++e) {
            const cx<R> a = lo.v[e], b = hi.v[e];
            lo.v[e] = cadd<R>(a, b);
            hi.v[e] = csub<R>(a, b);
        }
        first_apply<R, EM, kCols, 1, false, 3, NT>(
            hi, LGL, lgT, T, [](int, int k, cx<R> v) { return cmul<R>(v, tw_pass<R, true, true>(k << 1)); });
        // even output rows 2n = IDFT_1024(u)[n], odd rows 2n + 1 = IDFT_1024(v)[n], n < 512
        auto store_even = [&](int b, int n, cx<R> v) {
            if (2 * n < ny && b < ncol) st_stream<R>(&dst[umul24((unsigned)(2 * n), (unsigned)Sx) + (unsigned)b], v);
        };
        auto store_odd = [&](int b, int n, cx<R> v) {
            if (2 * n + 1 < ny && b < ncol)
                st_stream<R>(&dst[umul24((unsigned)(2 * n + 1), (unsigned)Sx) + (unsigned)b], v);
        };
        auto next_lo = [&]() {
            if (un < pw.u1)
                first_load<R, EM, kCols, 1, false, 3, NT>(lo, LGL, lgT, T, loader(pw.tile(un), 0));
        };
        auto next_hi = [&]() {
            if (un < pw.u1)
                first_load<R, EM, kCols, 1, false, 3, NT>(hi, LGL, lgT, T, loader(pw.tile(un), 1));
        };
        fft_reg<R, true, EM, false, kCols, 1, false, true, 3, NT, true>(buf, LGL, lgT, T, lo, next_lo,
                                                                                   store_even);
        __syncthreads();   // the last pass read LDS; the second transform's first pass writes it
        fft_reg<R, true, EM, false, kCols, 1, false, true, 3, NT, true>(buf, LGL, lgT, T, hi, next_hi,
                                                                                   store_odd);
        __syncthreads();
        u = un;
    }
}

// LDS layout: element (z, c, col) at (z * 3 + c) * T + col, i.e. sequence
// b = c*T + col with unit sequence stride and element stride 3T.
//
// The tensor values of the spectral product stay in registers: item
// e = threadIdx.x + it * kNT of a tile is the pair (kzo, col) =
// (e >> lgT, e & (T-1)); the same thread loads the six components of its items
// (at most kTensorIt per thread, guaranteed by the plan) right after the
// previous tile's product, so the loads are in flight during that tile's
// inverse and this tile's forward transform.  The z FFT uses radix-8 passes
// (two for Pz = 64).
constexpr int kTensorIt = 4;

template <typename R, int EM>
__global__ void __launch_bounds__(kNT) zconv_kernel(cx<R>* __restrict__ X2, const R* __restrict__ spec, R Ms,
                                                    int nz, int lgPz, int Py, int Hx, int Hz, int Sx, int lgT,
                                                    int ntx, int units_per_member, int nunits) {
    tw_lds_fill<R>();   // read from the second pass on, after the first barrier
    extern __shared__ unsigned char smem_raw[];
    cx<R>* buf = reinterpret_cast<cx<R>*>(smem_raw);
    const int T = 1 << lgT;
    const int T3 = 3 * T;
    const int Pz = 1 << lgPz;
    const int H2 = Pz >> 1;
    const int plane_stride = Py * Sx;     // one z row of X2 (< 2^23, checked in the plan)
    const int comp_stride = nz * plane_stride;
    // Work unit u -> member mb, row pair q, column tile tx (tx fastest).  The
    // blocks of a launch come in pairs with adjacent logical indices (one XCD,
    // the same unit range, started together): the even block of a pair takes
    // row ky = q, the odd one row Py - q (q = 0 pairs rows 0 and Py/2).  Rows q
    // and Py - q read the same tensor octant values, so the pair's second
    // request for them finds them in L2.
    struct Tile {
        int mb, kx0, ky, tx, kyo;
    };
    const int lbp = xcd_logical_block(blockIdx.x, gridDim.x);
    const int side = lbp & 1;
    auto tile_of = [=](int u) {
        Tile d;
        d.mb = u / units_per_member;
        const int r = u - d.mb * units_per_member;
        const int q = r / ntx;
        d.tx = r - q * ntx;
        d.kyo = side ? (q == 0 ? Py >> 1 : q) : q;
        d.ky = side ? (q == 0 ? Py >> 1 : Py - q) : q;
        d.kx0 = d.tx * T;
        return d;
    };
    auto base_of = [=](const Tile& d) {
        return X2 + (long long)d.mb * 3 * comp_stride + (long long)d.ky * Sx + d.kx0;
    };
    // rows z >= nz are the zero padding (never read) and are never written back
    auto loader = [=](int t) {
        const Tile d = tile_of(t);
        const cx<R>* base = base_of(d);
        const int ncol = min(T, Hx - d.kx0);
        return [=](int b, int j) -> cx<R> {
            const int c = b >> lgT, col = b & (T - 1);
            if (j < nz && col < ncol) return base[(unsigned)c * (unsigned)comp_stride + umul24((unsigned)j, (unsigned)plane_stride) + (unsigned)col];
            return mk<R>(0, 0);
        };
    };
    const int tslab = (H2 + 1) * T;      // tensor values of one component and tile
    R tv[kTensorIt][6];
    // the tile's tensor block [6][Hz][T] is contiguous (row kyo, column tile tx)
    auto tensor_load = [&](int u) {
        const Tile d = tile_of(u);
        const R* blk = spec + (long long)(d.kyo * ntx + d.tx) * 6 * tslab;
        const int tid = tid_opaque();
        const bool okx = d.kx0 + (tid & (T - 1)) < Hx;
#pragma unroll
        for (int it = 0; it < kTensorIt; ++it) {
            const int e = tid + it * kNT;
            if (e < tslab) {
#pragma unroll
                for (int c6 = 0; c6 < 6; ++c6) tv[it][c6] = okx ? blk[c6 * tslab + e] : (R)0;
            }
        }
    };
    // unit range of this block's pair
    const int npairs = gridDim.x >> 1;
    const int pr = lbp >> 1;
    const int t0 = (int)((long long)nunits * pr / npairs);
    const int t1 = (int)((long long)nunits * (pr + 1) / npairs);
    FirstIn<R, EM, true> in;
    if (t0 < t1) {
        first_load<R, EM, kCols, 3, true, 3>(in, lgPz, lgT, T3, loader(t0));
        tensor_load(t0);
    }
    for (int t = t0; t < t1; ++t) {
        const Tile d = tile_of(t);
        const R sy = d.ky <= Py / 2 ? (R)1 : (R)-1;
        cx<R>* base = base_of(d);
        const int ncol = min(T, Hx - d.kx0);
        auto store = [&](int b, int j, cx<R> v) {
            const int c = b >> lgT, col = b & (T - 1);
            if (j < nz && col < ncol)
                st_stream<R>(&base[(unsigned)c * (unsigned)comp_stride + umul24((unsigned)j, (unsigned)plane_stride) + (unsigned)col], v);
        };
        auto none_load = [&](int, int) -> cx<R> { return mk<R>(0, 0); };
        auto none_store = [&](int, int, cx<R>) {};
        auto next = [&]() {
            if (t + 1 < t1) first_load<R, EM, kCols, 3, true, 3>(in, lgPz, lgT, T3, loader(t + 1));
        };
        fft_reg<R, false, EM, true, kCols, 3, true, false, 3, kNT, true>(buf, lgPz, lgT, T3, in, next, none_store);
        // 3x3 symmetric product with the real spectrum: H_a = -Ms sum_b N_ab M_b.
        // Item (kzo, col) serves kz = kzo and its mirror Pz - kzo, where the
        // components odd in z (xz, yz) change sign.
        const R s = -Ms;
        const int tid = tid_opaque();
#pragma unroll
        for (int it = 0; it < kTensorIt; ++it) {
            const int e = tid + it * kNT;
            if (e >= tslab) continue;
            const int kzo = e >> lgT, col = e & (T - 1);
            const R nxx = tv[it][0], nyy = tv[it][1], nzz = tv[it][2];
            const R nxy = sy * tv[it][3], nxz = tv[it][4], nyz = sy * tv[it][5];
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                if (m == 1 && (kzo == 0 || kzo == H2)) break;
                const int kz = m ? Pz - kzo : kzo;
                const R sz = m ? (R)-1 : (R)1;
                const R xz = sz * nxz, yz = sz * nyz;
                cx<R>* p = buf + kz * T3 + col;
                const cx<R> mx = p[0], my = p[T], mz = p[2 * T];
                p[0] = mk<R>(s * (nxx * mx.x + nxy * my.x + xz * mz.x), s * (nxx * mx.y + nxy * my.y + xz * mz.y));
                p[T] = mk<R>(s * (nxy * mx.x + nyy * my.x + yz * mz.x), s * (nxy * mx.y + nyy * my.y + yz * mz.y));
                p[2 * T] =
                    mk<R>(s * (xz * mx.x + yz * my.x + nzz * mz.x), s * (xz * mx.y + yz * my.y + nzz * mz.y));
            }
        }
        if (t + 1 < t1) tensor_load(t + 1);
        __syncthreads();
        fft_io<R, true, EM, true, false, kCols, 3, false, true, 3, kNT, true>(buf, lgPz, lgT, T3, none_load, store);
        __syncthreads();   // LDS is rewritten by the next tile
    }
}

// Register-resident z pass for Pz = 8 G, G = 1, 2, 4, 8 (single precision).
// Thread (col, g), col < T, g < G, of a T-column tile (G T threads) holds
// the elements z = g + G r (r < 8) of all three components.  Forward: a
// length-8 DFT over r, the twiddles W_Pz^(g k1), one LDS exchange, and
// length-G DFTs over g: the thread then owns k1 = g + G j (j < 8/G) and
// kz = k1 + 8 k2 (k2 < G) of all three components, eight values each, so the
// 3x3 spectral product runs in registers.  The inverse retraces the steps with
// conjugate twiddles.  Rows z >= nz (nz <= Pz/2, so r < 4) are the zero
// padding and are not written back.  The tensor spectrum is the tile-major
// layout of the generic pass with a tile width of T.  G = 8 is the 8 x 8
// split of Pz = 64; G = 1 needs no exchange.
template <typename R, int T, int G>
__global__ void __launch_bounds__(G * T) zconvr_kernel(cx<R>* __restrict__ X2, const R* __restrict__ spec, R Ms,
                                                       int nz, int Py, int Hx, int Sx, int ntx, int ntxn,
                                                       int upm, int ngm, int nbatch, int gw, long long tn_off) {
    constexpr int PZ = 8 * G, H2 = PZ / 2, Hz = H2 + 1, J = 8 / G;
    constexpr int LGPZ = ilog2c(PZ);
    extern __shared__ unsigned char smem_raw[];
    cx<R>* E = reinterpret_cast<cx<R>*>(smem_raw);   // [3][8][G][T]
    const int tid = threadIdx.x;
    const int col = tid & (T - 1);
    const int g = tid / T;
    __builtin_assume(g >= 0 && g < G);
    const unsigned plane_stride = (unsigned)Py * (unsigned)Sx;
    const unsigned comp_stride = (unsigned)nz * plane_stride;
    // w1[k1] = W_Pz^(g k1) (forward pass over r); w2[j][q] = W_Pz^(q (g + G j))
    // (the twiddles between the length-G DFTs of the items k1 = g + G j);
    // the inverse uses the conjugates.  w1[0] = 1 and w2[j][0] = 1: those
    // products are skipped.  (for G = 8, J = 1 and w2[0] = w1)
    const R s = -Ms;
    cx<R> w1[8], w2[J][G];
#pragma unroll
    for (int k1 = 0; k1 < 8; ++k1) w1[k1] = tw_fwd<R>(((g * k1) & (PZ - 1)) << (kTwLog - LGPZ));
#pragma unroll
    for (int jj = 0; jj < J; ++jj)
#pragma unroll
        for (int q = 0; q < G; ++q)
            w2[jj][q] = G == 8 ? w1[q] : tw_fwd<R>(((q * (g + G * jj)) & (PZ - 1)) << (kTwLog - LGPZ));
    // Units: upm = ntxn column tiles for each row pair q < Py/2 of a member
    // and, with a packed Nyquist column (ntxn = ntx - 1, ngm > 0), ngm Nyquist
    // units per member, each the column kx = Hx - 1 of T row pairs (lane col
    // takes q = q0 + col: 16 consecutive q are one 128-byte segment of X2, and
    // the tensor's Nyquist copy has the column tiles' block layout with q as
    // the column), instead of one whole tile per row pair.
    // The two blocks of a pair take the rows ky = q and Py - q (q = 0: 0 and
    // Py/2) of the same units.  A pair's list is its Nyquist units (spread
    // evenly over the pairs, each counted as gw column tiles), then a
    // contiguous range of column tiles (the host picks gw = 2 only when every
    // pair has at least gw column tiles, which keeps the ranges ordered).
    struct Tile {
        int mb, kx0, ky, tx, kyo, nyq, q0;
        bool ok;        // this lane's column exists
        unsigned off;   // this lane's element offset in its plane
    };
    const int lbp = xcd_logical_block(blockIdx.x, gridDim.x);
    const int side = lbp & 1;
    const int npairs = gridDim.x >> 1;
    const int pr = lbp >> 1;
    const int half = Py >> 1;
    const long long NN = (long long)upm * nbatch, NG = (long long)ngm * nbatch, S = NN + gw * NG;
    auto gstart = [=](long long p) { return (p * NG + npairs - 1) / npairs; };
    auto nstart = [=](long long p) { return min(NN, max(0LL, p * S / npairs - gw * gstart(p))); };
    const int kg0 = (int)gstart(pr), ng = (int)gstart(pr + 1) - kg0;
    const int n0 = (int)nstart(pr), nn = (int)nstart(pr + 1) - n0;
    // a unit of the pair's list (uniform): member, row pair q (column tiles),
    // column tile tx, or Nyquist unit of rows q0 ...
    struct Unit {
        int mb, q, tx, nyq, q0;
    };
    auto unit_at = [=](int u) {
        Unit a;
        a.nyq = u < ng;
        a.q0 = 0;
        if (a.nyq) {
            const int k = kg0 + u;
            a.mb = k / ngm;
            a.q0 = (k - a.mb * ngm) * T;
            a.q = 0;
            a.tx = ntx - 1;
        } else {
            const int n = n0 + u - ng;
            a.mb = n / upm;
            const int r = n - a.mb * upm;
            a.q = r / ntxn;
            a.tx = r - a.q * ntxn;
        }
        return a;
    };
    // the unit after a (unit u of the list): column tiles follow each other
    // in (member, q, tx) order, so only the first one needs divisions
    auto unit_next = [=](const Unit& a, int u) {
        if (u <= ng) return unit_at(u);
        Unit b = a;
        if (++b.tx == ntxn) {
            b.tx = 0;
            if (++b.q == half) {
                b.q = 0;
                ++b.mb;
            }
        }
        return b;
    };
    auto tile_of = [=](const Unit& a) {
        Tile d;
        d.nyq = a.nyq;
        d.mb = a.mb;
        d.q0 = a.q0;
        d.tx = a.tx;
        const int qu = a.q;   // the row pair of a column tile (uniform)
        d.kx0 = d.tx * T;
        d.kyo = side ? (qu == 0 ? half : qu) : qu;   // column tiles only
        // this lane's row pair: a Nyquist unit's lanes take consecutive ones
        int q = d.nyq ? d.q0 + col : qu;
        d.ok = d.nyq ? q < half : d.kx0 + col < Hx;
        if (d.nyq && !d.ok) q = 0;   // a valid element; its results are never stored
        d.ky = side ? (q == 0 ? half : Py - q) : q;
        // columns beyond Hx read at the clamped column Hx - 1 of the same row
        d.off = d.nyq ? nyq_pack(d.ky, Py, (unsigned)Sx) + (unsigned)(Hx - 1)
                      : (unsigned)d.ky * (unsigned)Sx + (unsigned)(d.kx0 + min(col, Hx - 1 - d.kx0));
        return d;
    };
    auto base_of = [=](const Tile& d) { return X2 + (long long)d.mb * 3 * comp_stride; };
    // Inputs of a tile: rows g + G r, r < 4, of the three components (scaled
    // by the spectral product's factor s = -Ms when the forward pass takes
    // them: the pass is linear, and there are fewer inputs than spectral
    // values; not at the load, which would make it wait for the data).  Every
    // operation of the pass acts on one column, so a column beyond Hx (read at
    // the clamped column Hx-1 of the same row) only produces values that are
    // never stored; rows z >= nz are the zero padding.
    cx<R> pin[12];
    auto load_tile = [&](const Unit& un) {
        const Tile d = tile_of(un);
        const cx<R>* base = base_of(d);
        const unsigned voff = (unsigned)g * plane_stride + d.off;
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int z = g + G * r;
                const unsigned zoff = (unsigned)min(G * r, nz - 1 - g) * plane_stride;
                const cx<R> v = base[(unsigned)c * comp_stride + zoff + voff];
                pin[c * 4 + r] = z < nz ? v : mk<R>((R)0, (R)0);
            }
    };
    const int t0 = 0, t1 = ng + nn;
    Unit uc = unit_at(t0);
    if (t0 < t1) load_tile(uc);
    for (int t = t0; t < t1; ++t) {
        const Tile d = tile_of(uc);
        const Unit un = unit_next(uc, t + 1);
        const R sy = d.ky <= Py / 2 ? (R)1 : (R)-1;
        // tensor values of this thread's kz = g + G j + 8 k2, read at the
        // octant row kzo = min(kz, Pz - kz); the tile's block [6][Hz][T] of the
        // tile-major spectrum is contiguous and includes the padding columns of
        // the last tile
        R tv[8][6];
        // with g < G, kz <= H2 holds for all g when G j + 8 k2 + G - 1 <= H2 and
        // for none when G j + 8 k2 > H2 (decided at compile time)
        auto kzo_of = [&](int k0) {
            return k0 + G - 1 <= H2 ? g + k0 : (k0 > H2 ? PZ - g - k0 : (g + k0 <= H2 ? g + k0 : PZ - g - k0));
        };
        {
            // a column tile's block [6][Hz][T] of the tile-major spectrum, or for
            // a Nyquist unit the block of the tensor's Nyquist copy whose column
            // col holds row pair q0 + col (the extra last block: the mirrored
            // side's first block, where q = 0 is row Py/2)
            const int nblk = (half + T - 1) / T;
            const long long bidx = d.nyq ? (side && d.q0 == 0 ? nblk : d.q0 / T) : (long long)d.kyo * ntx + d.tx;
            const R* blk = spec + (d.nyq ? tn_off : 0LL) + bidx * 6 * (Hz * T);
#pragma unroll
            for (int jj = 0; jj < J; ++jj)
#pragma unroll
                for (int k2 = 0; k2 < G; ++k2) {
                    const int o = kzo_of(G * jj + 8 * k2) * T + col;
#pragma unroll
                    for (int c6 = 0; c6 < 6; ++c6)
                        tv[jj * G + k2][c6] = ld_off<R>(blk, (unsigned)(c6 * (Hz * T) + o) * (unsigned)sizeof(R));
                }
        }
        // forward: DFT over r, twiddles, exchange
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            cx<R> v[8];
#pragma unroll
            for (int r = 0; r < 4; ++r) v[r] = cscale<R>(pin[c * 4 + r], s);
#pragma unroll
            for (int r = 4; r < 8; ++r) v[r] = mk<R>((R)0, (R)0);
            dft8<R, false>(v);
#pragma unroll
            for (int k1 = 0; k1 < 8; ++k1)
                E[((c * 8 + k1) * G + g) * T + col] = (k1 == 0 || G == 1) ? v[k1] : cmul<R>(v[k1], w1[k1]);
        }
        if constexpr (G > 1) __syncthreads();
        // length-G DFTs over g: X[c][j G + k2] is the spectrum at kz = g + G j + 8 k2
        cx<R> X[3][8];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int jj = 0; jj < J; ++jj) {
                const int k1 = g + G * jj;
#pragma unroll
                for (int q = 0; q < G; ++q) X[c][jj * G + q] = E[((c * 8 + k1) * G + q) * T + col];
                if constexpr (G > 1) dft<R, G, false>(&X[c][jj * G]);
            }
        // spectral product N M (its factor -Ms was applied to the inputs)
#pragma unroll
        for (int jj = 0; jj < J; ++jj)
#pragma unroll
            for (int k2 = 0; k2 < G; ++k2) {
                const int e = jj * G + k2;
                const int kz = g + G * jj + 8 * k2;
                const R sz = kz <= H2 ? (R)1 : (R)-1;
                const R nxx = tv[e][0], nyy = tv[e][1], nzz = tv[e][2];
                const R nxy = sy * tv[e][3], nxz = sz * tv[e][4], nyz = sy * sz * tv[e][5];
                const cx<R> mx = X[0][e], my = X[1][e], mz = X[2][e];
                X[0][e] = mk<R>(nxx * mx.x + nxy * my.x + nxz * mz.x, nxx * mx.y + nxy * my.y + nxz * mz.y);
                X[1][e] = mk<R>(nxy * mx.x + nyy * my.x + nyz * mz.x, nxy * mx.y + nyy * my.y + nyz * mz.y);
                X[2][e] = mk<R>(nxz * mx.x + nyz * my.x + nzz * mz.x, nxz * mx.y + nyz * my.y + nzz * mz.y);
            }
        // the next tile's inputs are in flight during the inverse transform
        if (t + 1 < t1) load_tile(un);
        // inverse: length-G DFTs over k2, conjugate twiddles, exchange back
        if constexpr (G > 1) __syncthreads();
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int jj = 0; jj < J; ++jj) {
                const int k1 = g + G * jj;
                if constexpr (G > 1) dft<R, G, true>(&X[c][jj * G]);
#pragma unroll
                for (int q = 0; q < G; ++q)
                    E[((c * 8 + k1) * G + q) * T + col] =
                        q == 0 ? X[c][jj * G] : cmul<R>(X[c][jj * G + q], cconj<R>(w2[jj][q]));
            }
        if constexpr (G > 1) __syncthreads();
        cx<R>* base = base_of(d);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            cx<R> v[8];
#pragma unroll
            for (int k1 = 0; k1 < 8; ++k1) v[k1] = E[((c * 8 + k1) * G + g) * T + col];
            dft8<R, true>(v);
            // rows z = g + G n1 >= Pz/2 >= nz are never needed
#pragma unroll
            for (int n1 = 0; n1 < 4; ++n1) {
                const int z = g + G * n1;
                if (d.ok && z < nz)
                    st_stream<R>(&base[(unsigned)c * comp_stride + (unsigned)z * plane_stride + d.off], v[n1]);
            }
        }
        __syncthreads();   // the next tile's forward exchange rewrites E
        uc = un;
    }
}

// Copy of nbytes (a multiple of 16) from 16-byte aligned global memory to LDS
// without registers: each wave moves 64 x 16 bytes per instruction
// (global_load_lds_dwordx4 writes lane i's 16 bytes at the wave's LDS address
// + 16 i).  Completion is counted by the vector memory counter: the caller
// waits for it and synchronises the block before the copy is read.
template <int NT>
__device__ __forceinline__ void lds_copy_async(const void* src, void* lds, int nbytes) {
    const int lane = (int)threadIdx.x & 63;
    const int w0 = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6) * 64;
    const int n16 = nbytes >> 4;
    for (int base = w0; base < n16; base += NT) {
        const int piece = base + lane;
        if (piece < n16)
            __builtin_amdgcn_global_load_lds(
                static_cast<const char*>(src) + (size_t)piece * 16,
                (__attribute__((address_space(3))) void*)(static_cast<char*>(lds) + (size_t)base * 16), 16, 0, 0);
    }
}

// s_waitcnt vmcnt(0): every vector memory access of the wave has completed
__device__ __forceinline__ void wait_vm_all() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Register-resident z pass for Pz = 128 (single precision, nz = 33 ... 64).
// Sixteen threads per column, T = 16 columns per tile (256 threads).
// Thread (col, g), g < 16, holds the elements z = g + 16 r (r < 8; r < 4 are
// inside the box) of all three components.  Forward: a length-8 DFT over r,
// the twiddles W_128^(g k1) (k1 < 8), one LDS exchange, then the length-16
// DFT over g split by decimation in frequency: thread (col, h) with
// k1 = h & 7 and parity p = h >> 3 (one parity per wave) forms
// u[g'] + (-1)^p u[g' + 8], multiplies by W_16^(p g') and takes a length-8
// DFT over g', which gives the spectrum at kz = k1 + 8 (2 m + p), m < 8, of
// all three components: the 3x3 product runs on registers.  The inverse
// retraces the steps (length-8 inverse DFTs over m, W_16^(-p g'), exchange,
// recombination a + (-1)^h W_16^(-g') c of the two parities, conjugate
// twiddles, length-8 inverse DFT over k1); rows z >= nz are not written.
// The tensor spectrum is in the tile-major layout with a tile width of 16; a
// tile's block is copied to LDS by direct global-to-LDS loads, issued one
// tile ahead while the inverse transform runs.
template <typename R>
__global__ void __launch_bounds__(256) zconvr128_kernel(cx<R>* __restrict__ X2, const R* __restrict__ spec, R Ms,
                                                        int nz, int Py, int Hx, int Sx, int ntx,
                                                        int units_per_member, int nunits) {
    constexpr int T = 16, PZ = 128, Hz = PZ / 2 + 1;
    constexpr int LGPZ = 7;
    constexpr int TSB = 6 * Hz * T * (int)sizeof(R);
    extern __shared__ unsigned char smem_raw[];
    R* TS = reinterpret_cast<R*>(smem_raw);                        // [6][Hz][T]
    cx<R>* E = reinterpret_cast<cx<R>*>(smem_raw + TSB);          // [3][8][16][T]
    const int tid = threadIdx.x;
    const int col = tid & (T - 1);
    const int g = tid / T;                          // forward layout: row phase g < 16
    __builtin_assume(g >= 0 && g < 16);
    const int k1h = g & 7, par = g >> 3;            // spectral layout: (k1, parity), parity uniform per wave
    const unsigned plane_stride = (unsigned)Py * (unsigned)Sx;
    const unsigned comp_stride = (unsigned)nz * plane_stride;
    const R s = -Ms;
    // W_128^(g k1), k1 = 1 ... 7 (w1[0] = 1 is not used)
    cx<R> w1[8];
#pragma unroll
    for (int k1 = 0; k1 < 8; ++k1) w1[k1] = tw_fwd<R>(((g * k1) & (PZ - 1)) << (kTwLog - LGPZ));
    struct Tile {
        int mb, kx0, ky, tx, kyo;
    };
    const int lbp = xcd_logical_block(blockIdx.x, gridDim.x);
    const int side = lbp & 1;
    auto tile_of = [=](int u) {
        Tile d;
        d.mb = u / units_per_member;
        const int r = u - d.mb * units_per_member;
        const int q = r / ntx;
        d.tx = r - q * ntx;
        d.kyo = side ? (q == 0 ? Py >> 1 : q) : q;
        d.ky = side ? (q == 0 ? Py >> 1 : Py - q) : q;
        d.kx0 = d.tx * T;
        return d;
    };
    auto base_of = [=](const Tile& d) {
        return X2 + (long long)d.mb * 3 * comp_stride + (long long)d.ky * Sx + d.kx0;
    };
    // inputs: rows g + 16 r, r < 4 (the rest is zero padding), columns beyond
    // Hx read at the clamped column (their values are never stored)
    cx<R> pin[12];
    auto load_tile = [&](int u) {
        const Tile d = tile_of(u);
        const cx<R>* base = base_of(d);
        const unsigned voff = (unsigned)g * plane_stride + (unsigned)min(col, Hx - 1 - d.kx0);
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int z = g + 16 * r;
                const unsigned zoff = (unsigned)min(16 * r, nz - 1 - g) * plane_stride;
                const cx<R> v = base[(unsigned)c * comp_stride + zoff + voff];
                pin[c * 4 + r] = z < nz ? v : mk<R>((R)0, (R)0);
            }
    };
    auto tensor_copy = [&](int u) {
        const Tile d = tile_of(u);
        lds_copy_async<256>(spec + (long long)(d.kyo * ntx + d.tx) * 6 * (Hz * T), TS, TSB);
    };
    const int npairs = gridDim.x >> 1;
    const int pr = lbp >> 1;
    const int t0 = (int)((long long)nunits * pr / npairs);
    const int t1 = (int)((long long)nunits * (pr + 1) / npairs);
    if (t0 < t1) {
        tensor_copy(t0);
        load_tile(t0);
    }
    for (int t = t0; t < t1; ++t) {
        const Tile d = tile_of(t);
        const R sy = d.ky <= Py / 2 ? (R)1 : (R)-1;
        // tensor values of this thread's kz = k1 + 16 m + 8 p: octant row kz
        // for m < 4 and 128 - kz (odd components change sign) for m >= 4
        // forward: length-8 DFT over r, twiddles W_128^(g k1), exchange
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            cx<R> v[8];
#pragma unroll
            for (int r = 0; r < 4; ++r) v[r] = cscale<R>(pin[c * 4 + r], s);
#pragma unroll
            for (int r = 4; r < 8; ++r) v[r] = mk<R>((R)0, (R)0);
            dft8<R, false>(v);
#pragma unroll
            for (int k1 = 0; k1 < 8; ++k1)
                E[((c * 8 + k1) * 16 + g) * T + col] = k1 == 0 ? v[0] : cmul<R>(v[k1], w1[k1]);
        }
        wait_vm_all();
        __syncthreads();
        // length-16 DFT over g, parity p of the outputs: X[c][m] at kz = k1 + 8 (2 m + p)
        cx<R> X[3][8];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const cx<R>* src = E + (c * 8 + k1h) * 16 * T + col;
            cx<R> u[8];
            if (par == 0) {
#pragma unroll
                for (int q = 0; q < 8; ++q) u[q] = cadd<R>(src[q * T], src[(q + 8) * T]);
            } else {
                u[0] = csub<R>(src[0], src[8 * T]);
                u[1] = mul_w32<R, false, 2>(csub<R>(src[1 * T], src[9 * T]));
                u[2] = mul_w32<R, false, 4>(csub<R>(src[2 * T], src[10 * T]));
                u[3] = mul_w32<R, false, 6>(csub<R>(src[3 * T], src[11 * T]));
                u[4] = mul_w32<R, false, 8>(csub<R>(src[4 * T], src[12 * T]));
                u[5] = mul_w32<R, false, 10>(csub<R>(src[5 * T], src[13 * T]));
                u[6] = mul_w32<R, false, 12>(csub<R>(src[6 * T], src[14 * T]));
                u[7] = mul_w32<R, false, 14>(csub<R>(src[7 * T], src[15 * T]));
            }
            dft8<R, false>(u);
#pragma unroll
            for (int m = 0; m < 8; ++m) X[c][m] = u[m];
        }
        // spectral product N M (its factor -Ms was applied to the inputs)
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const R sz = m < 4 ? (R)1 : (R)-1;
            const int kz = k1h + 16 * m + 8 * par;
            const R* tv = TS + (m < 4 ? kz : PZ - kz) * T + col;
            const R nxx = tv[0], nyy = tv[Hz * T], nzz = tv[2 * Hz * T];
            const R nxy = sy * tv[3 * Hz * T], nxz = sz * tv[4 * Hz * T], nyz = sy * sz * tv[5 * Hz * T];
            const cx<R> mx = X[0][m], my = X[1][m], mz = X[2][m];
            X[0][m] = mk<R>(nxx * mx.x + nxy * my.x + nxz * mz.x, nxx * mx.y + nxy * my.y + nxz * mz.y);
            X[1][m] = mk<R>(nxy * mx.x + nyy * my.x + nyz * mz.x, nxy * mx.y + nyy * my.y + nyz * mz.y);
            X[2][m] = mk<R>(nxz * mx.x + nyz * my.x + nzz * mz.x, nxz * mx.y + nyz * my.y + nzz * mz.y);
        }
        // the next tile's inputs are in flight during the inverse transform
        if (t + 1 < t1) load_tile(t + 1);
        // inverse: length-8 inverse DFTs over m, W_16^(-p g'), exchange back
        __syncthreads();   // every thread has read its exchange values
        if (t + 1 < t1) tensor_copy(t + 1);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            cx<R> u[8];
#pragma unroll
            for (int m = 0; m < 8; ++m) u[m] = X[c][m];
            dft8<R, true>(u);
            cx<R>* dst = E + ((c * 8 + k1h) * 2 + par) * 8 * T + col;
            if (par == 0) {
#pragma unroll
                for (int q = 0; q < 8; ++q) dst[q * T] = u[q];
            } else {
                dst[0] = u[0];
                dst[1 * T] = mul_w32<R, true, 2>(u[1]);
                dst[2 * T] = mul_w32<R, true, 4>(u[2]);
                dst[3 * T] = mul_w32<R, true, 6>(u[3]);
                dst[4 * T] = mul_w32<R, true, 8>(u[4]);
                dst[5 * T] = mul_w32<R, true, 10>(u[5]);
                dst[6 * T] = mul_w32<R, true, 12>(u[6]);
                dst[7 * T] = mul_w32<R, true, 14>(u[7]);
            }
        }
        __syncthreads();
        // recombination for row phase g = g' + 8 h: a[g'] + (-1)^h c'[g'], conjugate
        // twiddles, length-8 inverse DFT over k1; rows z = g + 16 n1, n1 < 4
        cx<R>* base = base_of(d);
        const bool okc = d.kx0 + col < Hx;
        const int gl = g & 7;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            cx<R> v[8];
#pragma unroll
            for (int k1 = 0; k1 < 8; ++k1) {
                const cx<R>* src = E + ((c * 8 + k1) * 2) * 8 * T + gl * T + col;
                const cx<R> a = src[0], b = src[8 * T];
                const cx<R> y = par == 0 ? cadd<R>(a, b) : csub<R>(a, b);
                v[k1] = k1 == 0 ? y : cmul<R>(y, cconj<R>(w1[k1]));
            }
            dft8<R, true>(v);
#pragma unroll
            for (int n1 = 0; n1 < 4; ++n1) {
                const int z = g + 16 * n1;
                if (okc && z < nz)
                    st_stream<R>(&base[(unsigned)c * comp_stride + (unsigned)z * plane_stride + (unsigned)col], v[n1]);
            }
        }
        __syncthreads();   // the next tile's forward exchange rewrites E
    }
}

// Register-resident z pass for double precision, Pz = 16 P (P = 1, 2, 4, 8):
// G = 4 P threads per column, each holding four values per component, and
// T = 64 / P columns per tile (8 for P = 8: 256 threads, 128-byte rows).  Row layout: thread (col, g) holds
// z = g + G r, r < 4, of all three components (r < 2 lie inside the box).
// Forward: a length-4 DFT over r, the twiddles W_Pz^(g k1), one LDS exchange.
// The length-G DFT over g at k2 = p + P m is split by decimation in frequency
// with g = g' + 4 h: thread (col, q), k1 = q & 3, p = q >> 2, forms
// b[g'] = W_G^(g' p) sum_h u[g' + 4 h] W_P^(h p) (the length-P DFT over h at
// frequency p) and takes a length-4 DFT over g'; it then owns kz = q + G m
// (m < 4) of all three components, so the 3x3 product runs on registers.
// Inverse: length-4 inverse DFT over m, twiddles W_G^(-g' p), exchange; the
// thread of row phase g = g' + 4 h sums the P parts with W_P^(-h p), applies
// W_Pz^(-g k1) and takes a length-4 inverse DFT over k1 for the rows g and
// g + G.  For P <= 4 a wave spans at most four consecutive g, so p = h = g >> 2
// is the same for the whole wave and the twiddles of the split are uniform
// (scalar registers); for P = 8 they are per lane.
// The tile's tensor block ([6][Hz][T] of the tile-major spectrum, tile width
// T) is copied to LDS by direct global-to-LDS loads, issued one tile ahead
// while the inverse transform runs, so it occupies no registers.
template <int P> struct ZD {
    static constexpr int G = 4 * P, PZ = 4 * G, T = 64 / P, Hz = PZ / 2 + 1, NT = G * T;
    static constexpr bool UNIFORM = 64 / T <= 4;                       // p = g >> 2 uniform per wave
    static constexpr int TS_BYTES = 6 * Hz * T * 8;                    // tensor block (double)
    static constexpr int LDS_BYTES = TS_BYTES + 3 * 4 * G * T * 16;    // + exchange [3][4][G][T] complex
};

template <typename R, int P>
__global__ void __launch_bounds__(ZD<P>::NT)
    zconvd_kernel(cx<R>* __restrict__ X2, const R* __restrict__ spec, R Ms, int nz, int Py, int Hx, int Sx,
                  int ntx, int units_per_member, int nunits) {
    constexpr int G = ZD<P>::G, PZ = ZD<P>::PZ, T = ZD<P>::T, Hz = ZD<P>::Hz, NT = ZD<P>::NT;
    constexpr int LGPZ = ilog2c(PZ), LGG = ilog2c(G), LGP = ilog2c(P), LGT = ilog2c(T);
    extern __shared__ unsigned char smem_raw[];
    R* TS = reinterpret_cast<R*>(smem_raw);                                // [6][Hz][T]
    cx<R>* E = reinterpret_cast<cx<R>*>(smem_raw + ZD<P>::TS_BYTES);    // [3][4][G][T]
    const int tid = threadIdx.x;
    const int col = tid & (T - 1);
    const int g = tid >> LGT;                       // row phase; spectral index q = g
    __builtin_assume(g >= 0 && g < G);
    const int k1s = g & 3;                          // spectral layout: k1 = q & 3
    const int gq = g & 3;                           // inverse gather: g' = g & 3
    const int pu = ZD<P>::UNIFORM ? __builtin_amdgcn_readfirstlane(g >> 2) : (g >> 2);   // p = h = g >> 2
    const unsigned plane_stride = (unsigned)Py * (unsigned)Sx;
    const unsigned comp_stride = (unsigned)nz * plane_stride;
    const R s = -Ms;
    // w1[k1] = W_Pz^(g k1); wp[h] = W_P^(h p); wg[g'] = W_G^(g' p) (index 0 unused)
    cx<R> w1[4], wp[P], wg[4];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) w1[k1] = tw_fwd<R>(((g * k1) & (PZ - 1)) << (kTwLog - LGPZ));
#pragma unroll
    for (int hh = 0; hh < P; ++hh) {
        wp[hh] = tw_fwd<R>(((hh * pu) & (P - 1)) << (kTwLog - LGP));
        if constexpr (ZD<P>::UNIFORM) wp[hh] = wave_uniform<R>(wp[hh]);
    }
#pragma unroll
    for (int gp = 0; gp < 4; ++gp) {
        wg[gp] = tw_fwd<R>(((gp * pu) & (G - 1)) << (kTwLog - LGG));
        if constexpr (ZD<P>::UNIFORM) wg[gp] = wave_uniform<R>(wg[gp]);
    }
    struct Tile {
        int mb, kx0, ky, tx, kyo;
    };
    const int lbp = xcd_logical_block(blockIdx.x, gridDim.x);
    const int side = lbp & 1;
    auto tile_of = [=](int u) {
        Tile d;
        d.mb = u / units_per_member;
        const int r = u - d.mb * units_per_member;
        const int q = r / ntx;
        d.tx = r - q * ntx;
        d.kyo = side ? (q == 0 ? Py >> 1 : q) : q;
        d.ky = side ? (q == 0 ? Py >> 1 : Py - q) : q;
        d.kx0 = d.tx * T;
        return d;
    };
    auto base_of = [=](const Tile& d) {
        return X2 + (long long)d.mb * 3 * comp_stride + (long long)d.ky * Sx + d.kx0;
    };
    auto tensor_copy = [&](int u) {
        const Tile d = tile_of(u);
        lds_copy_async<NT>(spec + (long long)(d.kyo * ntx + d.tx) * 6 * (Hz * T), TS, ZD<P>::TS_BYTES);
    };
    // inputs: rows g (always below nz > G) and g + G of the three components,
    // columns beyond Hx read at the clamped column (their values are never stored)
    cx<R> pin[6];
    auto load_tile = [&](int u) {
        const Tile d = tile_of(u);
        const cx<R>* base = base_of(d);
        const unsigned voff = (unsigned)g * plane_stride + (unsigned)min(col, Hx - 1 - d.kx0);
        const bool two = g + G < nz;
        const unsigned zoff = two ? (unsigned)G * plane_stride : 0u;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            pin[c * 2] = base[(unsigned)c * comp_stride + voff];
            const cx<R> v = base[(unsigned)c * comp_stride + zoff + voff];
            pin[c * 2 + 1] = two ? v : mk<R>((R)0, (R)0);
        }
    };
    const int npairs = gridDim.x >> 1;
    const int pr = lbp >> 1;
    const int t0 = (int)((long long)nunits * pr / npairs);
    const int t1 = (int)((long long)nunits * (pr + 1) / npairs);
    if (t0 < t1) {
        tensor_copy(t0);
        load_tile(t0);
    }
    for (int t = t0; t < t1; ++t) {
        const Tile d = tile_of(t);
        const R sy = d.ky <= Py / 2 ? (R)1 : (R)-1;
        // forward: length-4 DFT over r (two nonzero inputs), twiddles W_Pz^(g k1), exchange
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const cx<R> x0 = cscale<R>(pin[c * 2], s), x1 = cscale<R>(pin[c * 2 + 1], s);
            cx<R> a[4];
            a[0] = cadd<R>(x0, x1);
            a[1] = cadd<R>(x0, mul_mi<R, false>(x1));
            a[2] = csub<R>(x0, x1);
            a[3] = csub<R>(x0, mul_mi<R, false>(x1));
#pragma unroll
            for (int k1 = 0; k1 < 4; ++k1)
                E[((c * 4 + k1) * G + g) * T + col] = k1 == 0 ? a[0] : cmul<R>(a[k1], w1[k1]);
        }
        wait_vm_all();     // this wave's part of the tensor block has arrived
        __syncthreads();
        // length-G DFT over g at k2 = p + P m: X[c][m] at kz = q + G m
        cx<R> X[3][4];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const cx<R>* src = E + (c * 4 + k1s) * G * T + col;
            cx<R> b[4];
#pragma unroll
            for (int gp = 0; gp < 4; ++gp) b[gp] = src[gp * T];
#pragma unroll
            for (int hh = 1; hh < P; ++hh) {
#pragma unroll
                for (int gp = 0; gp < 4; ++gp) b[gp] = cadd<R>(b[gp], cmul<R>(src[(gp + 4 * hh) * T], wp[hh]));
            }
#pragma unroll
            for (int gp = 1; gp < 4; ++gp) b[gp] = cmul<R>(b[gp], wg[gp]);
            dft4<R, false>(b);
#pragma unroll
            for (int m = 0; m < 4; ++m) X[c][m] = b[m];
        }
        // spectral product N M (its factor -Ms was applied to the inputs); the
        // tensor at kz = q + G m sits at the octant rows q, G + q, 2G - q and
        // G - q (the last two mirrored: odd components negated, except at kz = Pz/2)
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int row = m == 0 ? g : (m == 1 ? G + g : (m == 2 ? 2 * G - g : G - g));
            const R* tv = TS + row * T + col;
            const R sz = m < 2 || (m == 2 && g == 0) ? (R)1 : (R)-1;
            const R nxx = tv[0], nyy = tv[Hz * T], nzz = tv[2 * Hz * T];
            const R nxy = sy * tv[3 * Hz * T], nxz = sz * tv[4 * Hz * T], nyz = sy * sz * tv[5 * Hz * T];
            const cx<R> mx = X[0][m], my = X[1][m], mz = X[2][m];
            X[0][m] = mk<R>(nxx * mx.x + nxy * my.x + nxz * mz.x, nxx * mx.y + nxy * my.y + nxz * mz.y);
            X[1][m] = mk<R>(nxy * mx.x + nyy * my.x + nyz * mz.x, nxy * mx.y + nyy * my.y + nyz * mz.y);
            X[2][m] = mk<R>(nxz * mx.x + nyz * my.x + nzz * mz.x, nxz * mx.y + nyz * my.y + nzz * mz.y);
        }
        // the spectra are formed here, not after the barrier (which would keep
        // every exchange value and tensor entry in registers across it)
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int m = 0; m < 4; ++m) keep_in_regs<R>(X[c][m]);
        __syncthreads();   // every thread has read its exchange values and tensor block
        // the next tile's tensor block and inputs are in flight during the inverse transform
        if (t + 1 < t1) {
            tensor_copy(t + 1);
            load_tile(t + 1);
        }
        // inverse: length-4 inverse DFTs over m, W_G^(-g' p), exchange back as [3][4][P][4][T]
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            cx<R> u[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) u[m] = X[c][m];
            dft4<R, true>(u);
            cx<R>* dst = E + (((c * 4 + k1s) * P + pu) * 4) * T + col;
#pragma unroll
            for (int gp = 0; gp < 4; ++gp) dst[gp * T] = gp == 0 ? u[0] : cmul<R>(u[gp], cconj<R>(wg[gp]));
        }
        __syncthreads();
        // row phase g = g' + 4 h: sum over the parts p' with W_P^(-h p'),
        // conjugate twiddles, length-4 inverse DFT over k1; rows g and g + G
        cx<R>* base = base_of(d);
        const bool okc = d.kx0 + col < Hx;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            cx<R> e[4];
#pragma unroll
            for (int k1 = 0; k1 < 4; ++k1) {
                const cx<R>* src = E + ((c * 4 + k1) * P * 4 + gq) * T + col;
                cx<R> acc = src[0];
#pragma unroll
                for (int pp = 1; pp < P; ++pp) acc = cadd<R>(acc, cmul<R>(src[pp * 4 * T], cconj<R>(wp[pp])));
                e[k1] = k1 == 0 ? acc : cmul<R>(acc, cconj<R>(w1[k1]));
            }
            dft4<R, true>(e);
            if (okc) {
                st_stream<R>(&base[(unsigned)c * comp_stride + (unsigned)g * plane_stride + (unsigned)col], e[0]);
                if (g + G < nz)
                    st_stream<R>(&base[(unsigned)c * comp_stride + (unsigned)(g + G) * plane_stride + (unsigned)col],
                                 e[1]);
            }
        }
        __syncthreads();   // the next tile's forward exchange rewrites E
    }
}

static inline bool em_big(long long elements) { return elements > (long long)kNT * 16; }

// Blocks of a persistent launch: as many as can be resident on the device
// (occupancy of this kernel at this LDS size, times the CU count), at most
// one per tile.  Cached per device, kernel and LDS size.
static int persistent_grid(const void* kernel, size_t lds, long long ntiles, int nt = kNT) {
    static std::mutex mu;
    static std::map<std::tuple<int, const void*, size_t>, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -1;
    int resident = 0;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto key = std::make_tuple(dev, kernel, lds + ((size_t)nt << 40));
        auto it = cache.find(key);
        if (it != cache.end()) {
            resident = it->second;
        } else {
            int cus = 0, per_cu = 0;
            // more than 64 KiB of dynamic LDS has to be allowed per kernel first
            if (lds > 65536 &&
                hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
                return -1;
            if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -1;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, nt, lds) != hipSuccess) return -1;
            resident = std::max(1, per_cu) * std::max(1, cus);
            cache.emplace(key, resident);
        }
    }
    return (int)std::min<long long>(ntiles, resident);
}

// Even grid of block pairs (at most one pair per unit); a multiple of 16 when
// large enough, so that no pair straddles two XCDs.
static int pair_grid(int resident, long long nunits) {
    if (resident < 2) return -1;
    long long g = 2 * std::min<long long>(nunits, resident / 2);
    if (g >= 16) g -= g % 16;
    return (int)g;
}

template <typename R, int EM, int NT, int LG = 0>
static hipError_t run_yfwd(const Plan& pl, const void* X1, void* X2, hipStream_t s) {
    const int lgT = ilog2(pl.ty);
    const int ntx = (pl.Hx + pl.ty - 1) / pl.ty;
    const int ntiles = ntx * 3 * pl.nz * pl.nbatch;
    const size_t lds = (size_t)pl.Py * pl.ty * sizeof(cx<R>);
    const int grid = pair_grid(persistent_grid(reinterpret_cast<const void*>(&yfwd_kernel<R, EM, NT, LG>), lds,
                                               1LL << 30, NT),
                               (long long)(ntiles / ntx) * ((ntx + 1) / 2));
    if (grid < 2) return hipErrorInvalidValue;
    hipLaunchKernelGGL((yfwd_kernel<R, EM, NT, LG>), dim3(grid), dim3(NT), lds, s, static_cast<const cx<R>*>(X1),
                       static_cast<cx<R>*>(X2), pl.ny, pl.lgPy, pl.Hx, pl.Sx, lgT, ntx, ntiles, pl.nyqpack);
    return hipGetLastError();
}

template <typename R, int EM, int NT, int LG = 0>
static hipError_t run_yinv(const Plan& pl, const void* X2, void* Y1, hipStream_t s) {
    const int lgT = ilog2(pl.ty);
    const int ntx = (pl.Hx + pl.ty - 1) / pl.ty;
    const int ntiles = ntx * 3 * pl.nz * pl.nbatch;
    const size_t lds = (size_t)pl.Py * pl.ty * sizeof(cx<R>);
    const int grid = pair_grid(persistent_grid(reinterpret_cast<const void*>(&yinv_kernel<R, EM, NT, LG>), lds,
                                               1LL << 30, NT),
                               (long long)(ntiles / ntx) * ((ntx + 1) / 2));
    if (grid < 2) return hipErrorInvalidValue;
    hipLaunchKernelGGL((yinv_kernel<R, EM, NT, LG>), dim3(grid), dim3(NT), lds, s, static_cast<const cx<R>*>(X2),
                       static_cast<cx<R>*>(Y1), pl.ny, pl.lgPy, pl.Hx, pl.Sx, lgT, ntx, ntiles, pl.nyqpack);
    return hipGetLastError();
}

// Py = 2048: two transforms of length 1024 per tile, 16 (single) or 8
// (double) columns, 128 KiB of LDS; 512 threads, 1024 for the inverse (it
// holds two sets of first-pass values).
template <typename R, bool INV>
static hipError_t run_y2(const Plan& pl, const void* in, void* out, hipStream_t s) {
    constexpr int NT = INV ? 1024 : 512;
    constexpr int EM = (sizeof(R) == 4 ? 32 : 16) * 512 / NT;
    constexpr int lgT = sizeof(R) == 4 ? 4 : 3;
    constexpr int T = 1 << lgT;
    if (pl.Py != 2048 || 2 * pl.ny <= 1024) return hipErrorInvalidValue;
    const int ntx = (pl.Hx + T - 1) / T;
    const int ntiles = ntx * 3 * pl.nz * pl.nbatch;
    const size_t lds = (size_t)1024 * T * sizeof(cx<R>);
    const long long units = (long long)(ntiles / ntx) * ((ntx + 1) / 2);
    if constexpr (INV) {
        const int grid = pair_grid(
            persistent_grid(reinterpret_cast<const void*>(&yinv2_kernel<R, EM, NT>), lds, 1LL << 30, NT), units);
        if (grid < 2) return hipErrorInvalidValue;
        hipLaunchKernelGGL((yinv2_kernel<R, EM, NT>), dim3(grid), dim3(NT), lds, s, static_cast<const cx<R>*>(in),
                           static_cast<cx<R>*>(out), pl.ny, pl.Hx, pl.Sx, lgT, ntx, ntiles);
    } else {
        const int grid = pair_grid(
            persistent_grid(reinterpret_cast<const void*>(&yfwd2_kernel<R, EM, NT>), lds, 1LL << 30, NT), units);
        if (grid < 2) return hipErrorInvalidValue;
        hipLaunchKernelGGL((yfwd2_kernel<R, EM, NT>), dim3(grid), dim3(NT), lds, s, static_cast<const cx<R>*>(in),
                           static_cast<cx<R>*>(out), pl.ny, pl.Hx, pl.Sx, lgT, ntx, ntiles);
    }
    return hipGetLastError();
}

// Tiles of more than 256 x 32 elements (up to 128 KiB of LDS, one block per
// CU): 512 threads of 32 elements (two radix-32 passes for Py = 1024).
static bool y_huge(const Plan& pl) { return (long long)pl.Py * pl.ty > (long long)kNT * 32; }

// LG of the compile-time y geometry that matches the plan, 0 if none.
template <typename R>
static int y_lg(const Plan& pl) {
    if (pl.Px != pl.Py || 2 * pl.nx != pl.Px || 2 * pl.ny != pl.Py) return 0;
    if (pl.lgPy < 8 || pl.lgPy > 11) return 0;
    if (pl.ty != (1 << ytile_lg<R>(pl.lgPy)) || pl.Sx != pl.Px / 2 + 16) return 0;
    return pl.lgPy;
}

template <typename R>
hipError_t launch_yfwd(const Plan& pl, const void* X1, void* X2, hipStream_t s) {
    if (pl.Py == 2048) return run_y2<R, false>(pl, X1, X2, s);
    if constexpr (std::is_same<R, float>::value) {
        switch (y_lg<R>(pl)) {
            case 8: return run_yfwd<R, 16, kNT, 8>(pl, X1, X2, s);
            case 9: return run_yfwd<R, 32, kNT, 9>(pl, X1, X2, s);
            case 10: return run_yfwd<R, 32, 512, 10>(pl, X1, X2, s);
            case 11: return run_yfwd<R, 32, 512, 11>(pl, X1, X2, s);
            default: break;
        }
    } else {
        // double precision: tiles of 2^12 values (256 threads of 16) or 2^13 (512 threads of 16)
        switch (y_lg<R>(pl)) {
            case 8: return run_yfwd<R, 16, kNT, 8>(pl, X1, X2, s);
            case 9: return run_yfwd<R, 16, kNT, 9>(pl, X1, X2, s);
            case 10: return run_yfwd<R, 16, 512, 10>(pl, X1, X2, s);
            case 11: return run_yfwd<R, 16, 512, 11>(pl, X1, X2, s);
            default: break;
        }
        // tiles of up to 2^12 values: 256 threads of 16; up to 2^13 (128 KiB): 512 threads of 16
        if (!em_big((long long)pl.Py * pl.ty)) return run_yfwd<R, 16, kNT>(pl, X1, X2, s);
        return run_yfwd<R, 16, 512>(pl, X1, X2, s);
    }
    // tiles of up to 256 x 16 elements: 256 threads of 16; up to 256 x 32
    // (64 KiB in single precision): 256 threads of 32
    if (!em_big((long long)pl.Py * pl.ty)) return run_yfwd<R, 16, kNT>(pl, X1, X2, s);
    if (y_huge(pl)) return run_yfwd<R, 32, 512>(pl, X1, X2, s);
    return run_yfwd<R, 32, kNT>(pl, X1, X2, s);
}

template <typename R>
hipError_t launch_yinv(const Plan& pl, const void* X2, void* Y1, hipStream_t s) {
    if (pl.Py == 2048) return run_y2<R, true>(pl, X2, Y1, s);
    if constexpr (std::is_same<R, float>::value) {
        switch (y_lg<R>(pl)) {
            case 8: return run_yinv<R, 16, kNT, 8>(pl, X2, Y1, s);
            case 9: return run_yinv<R, 32, kNT, 9>(pl, X2, Y1, s);
            case 10: return run_yinv<R, 32, 512, 10>(pl, X2, Y1, s);
            case 11: return run_yinv<R, 32, 512, 11>(pl, X2, Y1, s);
            default: break;
        }
    } else {
        switch (y_lg<R>(pl)) {
            case 8: return run_yinv<R, 16, kNT, 8>(pl, X2, Y1, s);
            case 9: return run_yinv<R, 16, kNT, 9>(pl, X2, Y1, s);
            case 10: return run_yinv<R, 16, 512, 10>(pl, X2, Y1, s);
            case 11: return run_yinv<R, 16, 512, 11>(pl, X2, Y1, s);
            default: break;
        }
        // tiles of up to 2^12 values: 256 threads of 16; up to 2^13 (128 KiB): 512 threads of 16
        if (!em_big((long long)pl.Py * pl.ty)) return run_yinv<R, 16, kNT>(pl, X2, Y1, s);
        return run_yinv<R, 16, 512>(pl, X2, Y1, s);
    }
    if (!em_big((long long)pl.Py * pl.ty)) return run_yinv<R, 16, kNT>(pl, X2, Y1, s);
    if (y_huge(pl)) return run_yinv<R, 32, 512>(pl, X2, Y1, s);
    return run_yinv<R, 32, kNT>(pl, X2, Y1, s);
}

template <typename R, int EM>
static hipError_t run_zconv(const Plan& pl, void* X2, const void* spec, R Ms, hipStream_t s) {
    const int lgT = ilog2(pl.tz);
    const int ntx = pl.ntz;
    const int upm = ntx * (pl.Py / 2);          // units (row pair, column tile) per member
    const long long nunits = (long long)upm * pl.nbatch;
    const size_t lds = (size_t)3 * pl.Pz * pl.tz * sizeof(cx<R>);
    if ((long long)(pl.Pz / 2 + 1) * pl.tz > (long long)kTensorIt * kNT) return hipErrorInvalidValue;
    // block pairs share a unit range; pairs never straddle an XCD when the
    // grid is a multiple of 16
    const int resident = persistent_grid(reinterpret_cast<const void*>(&zconv_kernel<R, EM>), lds, 1LL << 30);
    if (resident < 1) return hipErrorInvalidValue;
    long long grid = 2 * std::min<long long>(nunits, std::max(1, resident / 2));
    if (grid >= 16) grid -= grid % 16;
    hipLaunchKernelGGL((zconv_kernel<R, EM>), dim3((unsigned)grid), dim3(kNT), lds, s, static_cast<cx<R>*>(X2),
                       static_cast<const R*>(spec), Ms, pl.nz, pl.lgPz, pl.Py, pl.Hx, pl.Hz, pl.Sx, lgT, ntx, upm,
                       (int)nunits);
    return hipGetLastError();
}

template <int T, int G>
static hipError_t run_zconvr(const Plan& pl, void* X2, const void* spec, float Ms, hipStream_t s) {
    if (pl.Pz != 8 * G || pl.tz != T || 2 * pl.nz > pl.Pz || 4 * pl.nz <= pl.Pz) return hipErrorInvalidValue;
    const int ntx = pl.ntz;
    const int half = pl.Py / 2;
    const size_t lds = (size_t)3 * 8 * G * T * sizeof(cx<float>);
    const int resident =
        persistent_grid(reinterpret_cast<const void*>(&zconvr_kernel<float, T, G>), lds, 1LL << 30, G * T);
    if (resident < 2) return hipErrorInvalidValue;
    // with a packed Nyquist column the last column tile (only kx = Hx - 1 = Lh)
    // becomes Nyquist units of T row pairs
    if (pl.nyqpack && (ntx < 2 || (ntx - 1) * T != pl.Hx - 1 || half % 16 != 0)) return hipErrorInvalidValue;
    const int ntxn = pl.nyqpack ? ntx - 1 : ntx;
    const int upm = ntxn * half;
    const int ngm = pl.nyqpack ? (half + T - 1) / T : 0;
    const long long nunits = ((long long)upm + ngm) * pl.nbatch;
    long long grid = 2 * std::min<long long>(nunits, std::max(1, resident / 2));
    if (grid >= 16) grid -= grid % 16;
    // a Nyquist unit costs about two column tiles; balance with that weight
    // when every pair gets several column tiles and at most one Nyquist unit
    const long long npairs = grid / 2, NN = (long long)upm * pl.nbatch, NG = (long long)ngm * pl.nbatch;
    const int gw = (NG > 0 && NG <= npairs && NN >= 4 * npairs) ? 2 : 0;
    hipLaunchKernelGGL((zconvr_kernel<float, T, G>), dim3((unsigned)grid), dim3(G * T), lds, s,
                       static_cast<cx<float>*>(X2), static_cast<const float*>(spec), Ms, pl.nz, pl.Py, pl.Hx, pl.Sx,
                       ntx, ntxn, upm, ngm, pl.nbatch, gw, pl.tn_off);
    return hipGetLastError();
}

static hipError_t run_zconvr128(const Plan& pl, void* X2, const void* spec, float Ms, hipStream_t s) {
    if (pl.Pz != 128 || pl.tz != 16 || 2 * pl.nz > pl.Pz || 4 * pl.nz <= pl.Pz ||
        (reinterpret_cast<uintptr_t>(spec) & 15) != 0)
        return hipErrorInvalidValue;
    const int ntx = pl.ntz;
    const int upm = ntx * (pl.Py / 2);
    const long long nunits = (long long)upm * pl.nbatch;
    const size_t lds = (size_t)3 * 8 * 16 * 16 * sizeof(cx<float>) + 6 * 65 * 16 * sizeof(float);   // E + tensor
    const int resident =
        persistent_grid(reinterpret_cast<const void*>(&zconvr128_kernel<float>), lds, 1LL << 30, 256);
    if (resident < 2) return hipErrorInvalidValue;
    long long grid = 2 * std::min<long long>(nunits, std::max(1, resident / 2));
    if (grid >= 16) grid -= grid % 16;
    hipLaunchKernelGGL((zconvr128_kernel<float>), dim3((unsigned)grid), dim3(256), lds, s,
                       static_cast<cx<float>*>(X2), static_cast<const float*>(spec), Ms, pl.nz, pl.Py, pl.Hx, pl.Sx,
                       ntx, upm, (int)nunits);
    return hipGetLastError();
}

template <int P>
static hipError_t run_zconvd(const Plan& pl, void* X2, const void* spec, double Ms, hipStream_t s) {
    constexpr int G = ZD<P>::G, T = ZD<P>::T, NT = ZD<P>::NT;
    if (pl.Pz != 4 * G || pl.tz != T || 2 * pl.nz > pl.Pz || 4 * pl.nz <= pl.Pz ||
        (reinterpret_cast<uintptr_t>(spec) & 15) != 0)
        return hipErrorInvalidValue;
    const int ntx = pl.ntz;
    const int upm = ntx * (pl.Py / 2);
    const long long nunits = (long long)upm * pl.nbatch;
    const size_t lds = ZD<P>::LDS_BYTES;
    const int resident =
        persistent_grid(reinterpret_cast<const void*>(&zconvd_kernel<double, P>), lds, 1LL << 30, NT);
    if (resident < 2) return hipErrorInvalidValue;
    long long grid = 2 * std::min<long long>(nunits, std::max(1, resident / 2));
    if (grid >= 16) grid -= grid % 16;
    hipLaunchKernelGGL((zconvd_kernel<double, P>), dim3((unsigned)grid), dim3(NT), lds, s,
                       static_cast<cx<double>*>(X2), static_cast<const double*>(spec), Ms, pl.nz, pl.Py, pl.Hx,
                       pl.Sx, ntx, upm, (int)nunits);
    return hipGetLastError();
}

static hipError_t run_zregd(const Plan& pl, void* X2, const void* spec, double Ms, hipStream_t s) {
    switch (pl.Pz) {
        case 16: return run_zconvd<1>(pl, X2, spec, Ms, s);
        case 32: return run_zconvd<2>(pl, X2, spec, Ms, s);
        case 64: return run_zconvd<4>(pl, X2, spec, Ms, s);
        case 128: return run_zconvd<8>(pl, X2, spec, Ms, s);
        default: return hipErrorInvalidValue;
    }
}

static hipError_t run_zreg(const Plan& pl, void* X2, const void* spec, float Ms, hipStream_t s) {
    switch (pl.Pz) {
        case 128: return run_zconvr128(pl, X2, spec, Ms, s);
        case 8: return run_zconvr<64, 1>(pl, X2, spec, Ms, s);
        case 16: return run_zconvr<32, 2>(pl, X2, spec, Ms, s);
        case 32: return run_zconvr<32, 4>(pl, X2, spec, Ms, s);
        case 64: return run_zconvr<32, 8>(pl, X2, spec, Ms, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename R>
hipError_t launch_zconv(const Plan& pl, void* X2, const void* spec, R Ms, hipStream_t s) {
    if constexpr (std::is_same<R, float>::value) {
        if (pl.zreg) return run_zreg(pl, X2, spec, Ms, s);
    } else {
        if (pl.zreg) return run_zregd(pl, X2, spec, Ms, s);
    }
    return em_big(3LL * pl.Pz * pl.tz) ? run_zconv<R, 32>(pl, X2, spec, Ms, s) : run_zconv<R, 16>(pl, X2, spec, Ms, s);
}

// ---- films: the y and z passes fused ---------------------------------------------
// With nz = 1 (Pz = 2) the z transform of the single input row is that row
// for both kz = 0 and 1, and the inverse adds the two products, so the z pass
// is the product with N(kz = 0) + N(kz = 1).  One block takes T columns of all
// three components: forward y FFT from X1 (rows >= ny are the zero padding)
// into LDS, the 3x3 product there, inverse y FFT from LDS to Y1 (rows < ny;
// Y1 may be X1: a block reads its columns completely before it writes them).
// Element ky of sequence b = c T + col sits at ky 3T + b.
template <typename R, int EM>
__global__ void __launch_bounds__(kNT) yzfilm_kernel(const cx<R>* X1, cx<R>* Y1, const R* __restrict__ spec, R Ms,
                                                     int ny, int lgPy, int Hx, int Sx, int lgT, int ntx, int tz,
                                                     int ntz, int ntiles) {
    tw_lds_fill<R>();   // read from the second pass on, after the first barrier
    extern __shared__ unsigned char smem_raw[];
    cx<R>* buf = reinterpret_cast<cx<R>*>(smem_raw);
    const int T = 1 << lgT;
    const int T3 = 3 * T;
    const int Py = 1 << lgPy;
    const R s = -Ms;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int mb = t / ntx;
        const int kx0 = (t - mb * ntx) * T;
        const int ncol = min(T, Hx - kx0);
        const long long mrow = (long long)mb * 3 * ny;    // first row of the member's component 0
        auto load = [&](int b, int j) -> cx<R> {
            const int c = b >> lgT, col = b & (T - 1);
            if (j < ny && col < ncol) return X1[(mrow + (long long)c * ny + j) * Sx + kx0 + col];
            return mk<R>((R)0, (R)0);
        };
        auto none_load = [&](int, int) -> cx<R> { return mk<R>((R)0, (R)0); };
        auto none_store = [&](int, int, cx<R>) {};
        fft_io<R, false, EM, false, true, kCols, 3, true, false, lgmax<EM>(), kNT, true>(buf, lgPy, lgT, T3, load,
                                                                                         none_store);
        __syncthreads();
        // product with N(kz = 0) + N(kz = 1) (octant rows 0 and 1, both with
        // the even sign in z); components odd in y change sign for ky > Py/2
        for (int e = threadIdx.x; e < (Py << lgT); e += kNT) {
            const int ky = e >> lgT, col = e & (T - 1);
            if (col >= ncol) continue;
            const int kx = kx0 + col;
            const int kyo = ky <= Py / 2 ? ky : Py - ky;
            const R sy = ky <= Py / 2 ? (R)1 : (R)-1;
            const int txs = kx / tz;
            const R* blk = spec + ((long long)(kyo * ntz + txs) * 6) * (2 * tz) + (kx - txs * tz);
            R n6[6];
#pragma unroll
            for (int c6 = 0; c6 < 6; ++c6) n6[c6] = blk[c6 * 2 * tz] + blk[c6 * 2 * tz + tz];
            const R nxx = s * n6[0], nyy = s * n6[1], nzz = s * n6[2];
            const R nxy = s * sy * n6[3], nxz = s * n6[4], nyz = s * sy * n6[5];
            cx<R>* p = buf + ky * T3 + col;
            const cx<R> mx = p[0], my = p[T], mz = p[2 * T];
            p[0] = mk<R>(nxx * mx.x + nxy * my.x + nxz * mz.x, nxx * mx.y + nxy * my.y + nxz * mz.y);
            p[T] = mk<R>(nxy * mx.x + nyy * my.x + nyz * mz.x, nxy * mx.y + nyy * my.y + nyz * mz.y);
            p[2 * T] = mk<R>(nxz * mx.x + nyz * my.x + nzz * mz.x, nxz * mx.y + nyz * my.y + nzz * mz.y);
        }
        __syncthreads();
        auto store = [&](int b, int j, cx<R> v) {
            const int c = b >> lgT, col = b & (T - 1);
            if (j < ny && col < ncol) Y1[(mrow + (long long)c * ny + j) * Sx + kx0 + col] = v;
        };
        fft_io<R, true, EM, true, false, kCols, 3, false, true, lgmax<EM>(), kNT, true>(buf, lgPy, lgT, T3, none_load,
                                                                                        store);
        __syncthreads();   // the next tile's first pass writes LDS
    }
}

template <typename R>
hipError_t launch_yzfilm(const Plan& pl, void* X1, const void* spec, R Ms, hipStream_t s) {
    if (!pl.yzfilm || pl.nz != 1 || pl.Pz != 2 || pl.Hz != 2) return hipErrorInvalidValue;
    const int T = pl.yzt;
    const int lgT = ilog2(T);
    const int ntx = (pl.Hx + T - 1) / T;
    const int ntiles = ntx * pl.nbatch;
    const long long elems = 3LL * pl.Py * T;
    const size_t lds = (size_t)elems * sizeof(cx<R>);
    const int grid = std::min(ntiles, 4096);
    if (elems <= (long long)kNT * 16)
        hipLaunchKernelGGL((yzfilm_kernel<R, 16>), dim3(grid), dim3(kNT), lds, s, static_cast<const cx<R>*>(X1),
                           static_cast<cx<R>*>(X1), static_cast<const R*>(spec), Ms, pl.ny, pl.lgPy, pl.Hx, pl.Sx,
                           lgT, ntx, pl.tz, pl.ntz, ntiles);
    else
        hipLaunchKernelGGL((yzfilm_kernel<R, 32>), dim3(grid), dim3(kNT), lds, s, static_cast<const cx<R>*>(X1),
                           static_cast<cx<R>*>(X1), static_cast<const R*>(spec), Ms, pl.ny, pl.lgPy, pl.Hx, pl.Sx,
                           lgT, ntx, pl.tz, pl.ntz, ntiles);
    return hipGetLastError();
}

// ---- memory patterns without arithmetic (diagnostics) ---------------------------
// The practical bandwidth of the access patterns of the passes, measured on
// the same buffer: a float4 stream copy, and in-place read + write (scaled by
// a runtime factor 1, so nothing is elided) with the z pass's tiling (tiles
// of 32 columns x the nz rows of three components, rows a plane apart) and
// with the y pass's (16 columns x Py rows of one plane).
__global__ void __launch_bounds__(256) probe_copy_kernel(const float4* __restrict__ a, float4* __restrict__ b,
                                                         long long n4) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n4) b[i] = a[i];
}

__global__ void __launch_bounds__(256) probe_ztile_kernel(float2* X, int nz, int Py, int Hx, int Sx, int ntx,
                                                          float f) {
    const int col = threadIdx.x & 31, g = threadIdx.x >> 5;
    const long long plane = (long long)Py * Sx, comp = (long long)nz * plane;
    const int ky = blockIdx.x / ntx, tx = blockIdx.x % ntx;
    const int kx = tx * 32 + col;
    if (kx >= Hx) return;
    float2* base = X + (long long)ky * Sx + kx;
    for (int z = g; z < nz; z += 8) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float2* q = base + c * comp + z * plane;
            const float2 v = *q;
            *q = make_float2(v.x * f, v.y * f);
        }
    }
}

__global__ void __launch_bounds__(512) probe_ytile_kernel(float2* X, int Py, int Hx, int Sx, int ntx, float f) {
    const int col = threadIdx.x & 15, rg = threadIdx.x >> 4;
    const long long pl = blockIdx.x / ntx;
    const int tx = blockIdx.x % ntx;
    const int kx = tx * 16 + col;
    if (kx >= Hx) return;
    float2* base = X + pl * Py * (long long)Sx + kx;
    for (int r = rg; r < Py; r += 32) {
        float2* q = base + (long long)r * Sx;
        const float2 v = *q;
        *q = make_float2(v.x * f, v.y * f);
    }
}

hipError_t launch_memory_probe(const Plan& pl, int kind, void* X2, hipStream_t s, double* bytes) {
    const long long n2 = 3LL * pl.nbatch * pl.nz * pl.Py * pl.Sx;       // complex values in X2
    const double useful = 2.0 * 3.0 * pl.nbatch * pl.nz * pl.Py * (double)pl.Hx * sizeof(float2);
    if (kind == 0) {
        const long long n4 = n2 / 4;                                     // float4 in each half
        hipLaunchKernelGGL(probe_copy_kernel, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, s,
                           static_cast<const float4*>(X2), static_cast<float4*>(X2) + n4, n4);
        *bytes = 2.0 * n4 * sizeof(float4);
    } else if (kind == 1) {
        const int ntx = (pl.Hx + 31) / 32;
        for (int mb = 0; mb < pl.nbatch; ++mb)
            hipLaunchKernelGGL(probe_ztile_kernel, dim3((unsigned)(pl.Py * ntx)), dim3(256), 0, s,
                               static_cast<float2*>(X2) + (long long)mb * 3 * pl.nz * pl.Py * pl.Sx, pl.nz, pl.Py,
                               pl.Hx, pl.Sx, ntx, 1.0f);
        *bytes = useful;
    } else {
        const int ntx = (pl.Hx + 15) / 16;
        hipLaunchKernelGGL(probe_ytile_kernel, dim3((unsigned)(3 * pl.nbatch * pl.nz * ntx)), dim3(512), 0, s,
                           static_cast<float2*>(X2), pl.Py, pl.Hx, pl.Sx, ntx, 1.0f);
        *bytes = useful;
    }
    return hipGetLastError();
}

template hipError_t launch_yfwd<float>(const Plan&, const void*, void*, hipStream_t);
template hipError_t launch_yfwd<double>(const Plan&, const void*, void*, hipStream_t);
template hipError_t launch_yinv<float>(const Plan&, const void*, void*, hipStream_t);
template hipError_t launch_yinv<double>(const Plan&, const void*, void*, hipStream_t);
template hipError_t launch_zconv<float>(const Plan&, void*, const void*, float, hipStream_t);
template hipError_t launch_zconv<double>(const Plan&, void*, const void*, double, hipStream_t);
template hipError_t launch_yzfilm<float>(const Plan&, void*, const void*, float, hipStream_t);
template hipError_t launch_yzfilm<double>(const Plan&, void*, const void*, double, hipStream_t);

}  // namespace magx
