// Strided passes of the demag FFT convolution (Section II-B, Eq. (3)).
//
// Each block owns a tile of T consecutive kx columns (contiguous in memory,
// coalesced row segments) and transforms them along y or z in LDS.
//  * yfwd : rows y < ny are loaded, rows ny..Py-1 are the zero padding and
//           never read from memory; all Py output rows are written.
//  * zconv: for one ky, all three components: forward z FFT (rows z >= nz
//           are zero padding), then the pointwise product with the real
//           symmetric tensor spectrum, H_a = -Ms sum_b N_ab M_b, then the
//           inverse z FFT; only rows z < nz are written back (in place).
//  * yinv : inverse y FFT; only rows y < ny (inside the box) are written.
#include "magx_internal.hpp"

namespace magx {

// EM: FFT elements held per thread (T * L <= kNT * EM); 16 or 32.

template <typename R, int EM>
__global__ void __launch_bounds__(kNT) yfwd_kernel(const cx<R>* __restrict__ X1, cx<R>* __restrict__ X2, int ny,
                                                   int lgPy, int Hx, int Sx, int lgT, int ntx) {
    extern __shared__ unsigned char smem_raw[];
    cx<R>* buf = reinterpret_cast<cx<R>*>(smem_raw);
    const int T = 1 << lgT;
    const int Py = 1 << lgPy;
    const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int tx = lb % ntx;
    const long long plane = lb / ntx;    // c * nz + z
    const int kx0 = tx * T;
    const cx<R>* src = X1 + plane * ny * (long long)Sx + kx0;
    cx<R>* dst = X2 + plane * Py * (long long)Sx + kx0;
    const int ncol = min(T, Hx - kx0);
    // sequence b = column kx0 + b; rows >= ny are the zero padding, never read
    auto load = [&](int b, int j) -> cx<R> {
        if (j < ny && b < ncol) return src[mul24(j, Sx) + b];
        return mk<R>(0, 0);
    };
    auto store = [&](int b, int j, cx<R> v) {
        if (b < ncol) dst[mul24(j, Sx) + b] = v;
    };
    fft_io<R, false, EM, false, false, kCols, 1>(buf, lgPy, lgT, T, load, store);
}

template <typename R, int EM>
__global__ void __launch_bounds__(kNT) yinv_kernel(const cx<R>* __restrict__ X2, cx<R>* __restrict__ Y1, int ny,
                                                   int lgPy, int Hx, int Sx, int lgT, int ntx) {
    extern __shared__ unsigned char smem_raw[];
    cx<R>* buf = reinterpret_cast<cx<R>*>(smem_raw);
    const int T = 1 << lgT;
    const int Py = 1 << lgPy;
    const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int tx = lb % ntx;
    const long long plane = lb / ntx;
    const int kx0 = tx * T;
    const cx<R>* src = X2 + plane * Py * (long long)Sx + kx0;
    cx<R>* dst = Y1 + plane * ny * (long long)Sx + kx0;
    const int ncol = min(T, Hx - kx0);
    auto load = [&](int b, int j) -> cx<R> {
        if (b < ncol) return src[mul24(j, Sx) + b];
        return mk<R>(0, 0);
    };
    // rows inside the box only
    auto store = [&](int b, int j, cx<R> v) {
        if (j < ny && b < ncol) dst[mul24(j, Sx) + b] = v;
    };
    fft_io<R, true, EM, false, false, kCols, 1>(buf, lgPy, lgT, T, load, store);
}

// LDS layout: element (z, c, col) at (z * 3 + c) * T + col, i.e. sequence
// b = c*T + col with unit sequence stride and element stride 3T; behind it the
// block's tensor tile tl[(comp * (Pz/2+1) + kzo) * T + col].
template <typename R, int EM>
__global__ void __launch_bounds__(kNT) zconv_kernel(cx<R>* __restrict__ X2, const R* __restrict__ spec, R Ms,
                                                    int nz, int lgPz, int Py, int Hx, int Hy, int Hz, int Sx,
                                                    int lgT, int ntx, int blocks_per_member) {
    extern __shared__ unsigned char smem_raw[];
    cx<R>* buf = reinterpret_cast<cx<R>*>(smem_raw);
    const int T = 1 << lgT;
    const int T3 = 3 * T;
    const int Pz = 1 << lgPz;
    const int H2 = Pz >> 1;
    R* tl = reinterpret_cast<R*>(smem_raw + (size_t)Pz * T3 * sizeof(cx<R>));
    // logical order 0, 1, Py-1, 2, Py-2, ..., Py/2: the mirrored rows ky and
    // Py-ky read the same tensor octant rows one after the other on one XCD
    const int lbg = xcd_logical_block(blockIdx.x, gridDim.x);
    const int mb = lbg / blocks_per_member;            // member of a batch of systems
    const int lb = lbg - mb * blocks_per_member;
    const int tx = lb % ntx;
    const int u = lb / ntx;
    const int ky = (u & 1) ? (u + 1) >> 1 : (u == 0 ? 0 : Py - (u >> 1));
    const int kx0 = tx * T;
    const int kyo = ky <= Py / 2 ? ky : Py - ky;
    const R sy = ky <= Py / 2 ? (R)1 : (R)-1;
    // tensor tile -> LDS first; its loads are in flight while the FFT loads X2
    {
        const int ntl = 6 * (H2 + 1) * T;
        const int cstride = Hz * Hy * Sx;
        for (int e0 = threadIdx.x; e0 < ntl; e0 += kNT * 4) {
            R v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int e = e0 + q * kNT;
                const int col = e & (T - 1), rest = e >> lgT;
                const int c6 = rest / (H2 + 1), kzo = rest - c6 * (H2 + 1);
                const int kx = kx0 + col;
                v[q] = (e < ntl && kx < Hx) ? spec[c6 * cstride + mul24(mul24(kzo, Hy) + kyo, Sx) + kx] : (R)0;
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int e = e0 + q * kNT;
                if (e < ntl) tl[e] = v[q];
            }
        }
    }
    const int plane_stride = Py * Sx;     // one z row of X2 (< 2^23, checked in the plan)
    const int comp_stride = nz * plane_stride;
    cx<R>* base = X2 + (long long)mb * 3 * comp_stride + (long long)ky * Sx + kx0;
    const int ncol = min(T, Hx - kx0);
    // rows z >= nz are the zero padding (never read) and are never written back
    auto load = [&](int b, int j) -> cx<R> {
        const int c = b >> lgT, col = b & (T - 1);
        if (j < nz && col < ncol) return base[c * comp_stride + mul24(j, plane_stride) + col];
        return mk<R>(0, 0);
    };
    auto store = [&](int b, int j, cx<R> v) {
        const int c = b >> lgT, col = b & (T - 1);
        if (j < nz && col < ncol) base[c * comp_stride + mul24(j, plane_stride) + col] = v;
    };
    auto none_load = [&](int, int) -> cx<R> { return mk<R>(0, 0); };
    auto none_store = [&](int, int, cx<R>) {};
    fft_io<R, false, EM, false, true, kCols, 3>(buf, lgPz, lgT, T3, load, none_store);
    // 3x3 symmetric product with the real spectrum: H_a = -Ms sum_b N_ab M_b.
    // Item (kzo, col) serves kz = kzo and its mirror Pz - kzo, where the
    // components odd in z (xz, yz) change sign.
    const int tslab = (H2 + 1) * T;
    const R s = -Ms;
    for (int e = threadIdx.x; e < tslab; e += kNT) {
        const int kzo = e >> lgT, col = e & (T - 1);
        const R* t = tl + e;
        const R nxx = t[0], nyy = t[tslab], nzz = t[2 * tslab];
        const R nxy = sy * t[3 * tslab], nxz = t[4 * tslab], nyz = sy * t[5 * tslab];
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
            p[2 * T] = mk<R>(s * (xz * mx.x + yz * my.x + nzz * mz.x), s * (xz * mx.y + yz * my.y + nzz * mz.y));
        }
    }
    __syncthreads();
    fft_io<R, true, EM, true, false, kCols, 3>(buf, lgPz, lgT, T3, none_load, store);
}

static inline bool em_big(long long elements) { return elements > (long long)kNT * 16; }

template <typename R>
hipError_t launch_yfwd(const Plan& pl, const void* X1, void* X2, hipStream_t s) {
    const int lgT = ilog2(pl.ty);
    const int ntx = (pl.Hx + pl.ty - 1) / pl.ty;
    const unsigned blocks = (unsigned)(ntx * 3 * pl.nz * pl.nbatch);
    const size_t lds = (size_t)pl.Py * pl.ty * sizeof(cx<R>);
    if (em_big((long long)pl.Py * pl.ty))
        hipLaunchKernelGGL((yfwd_kernel<R, 32>), dim3(blocks), dim3(kNT), lds, s, static_cast<const cx<R>*>(X1),
                           static_cast<cx<R>*>(X2), pl.ny, pl.lgPy, pl.Hx, pl.Sx, lgT, ntx);
    else
        hipLaunchKernelGGL((yfwd_kernel<R, 16>), dim3(blocks), dim3(kNT), lds, s, static_cast<const cx<R>*>(X1),
                           static_cast<cx<R>*>(X2), pl.ny, pl.lgPy, pl.Hx, pl.Sx, lgT, ntx);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_yinv(const Plan& pl, const void* X2, void* Y1, hipStream_t s) {
    const int lgT = ilog2(pl.ty);
    const int ntx = (pl.Hx + pl.ty - 1) / pl.ty;
    const unsigned blocks = (unsigned)(ntx * 3 * pl.nz * pl.nbatch);
    const size_t lds = (size_t)pl.Py * pl.ty * sizeof(cx<R>);
    if (em_big((long long)pl.Py * pl.ty))
        hipLaunchKernelGGL((yinv_kernel<R, 32>), dim3(blocks), dim3(kNT), lds, s, static_cast<const cx<R>*>(X2),
                           static_cast<cx<R>*>(Y1), pl.ny, pl.lgPy, pl.Hx, pl.Sx, lgT, ntx);
    else
        hipLaunchKernelGGL((yinv_kernel<R, 16>), dim3(blocks), dim3(kNT), lds, s, static_cast<const cx<R>*>(X2),
                           static_cast<cx<R>*>(Y1), pl.ny, pl.lgPy, pl.Hx, pl.Sx, lgT, ntx);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_zconv(const Plan& pl, void* X2, const void* spec, R Ms, hipStream_t s) {
    const int lgT = ilog2(pl.tz);
    const int ntx = (pl.Hx + pl.tz - 1) / pl.tz;
    const int bpm = ntx * pl.Py;
    const unsigned blocks = (unsigned)(bpm * pl.nbatch);
    const size_t lds = (size_t)3 * pl.Pz * pl.tz * sizeof(cx<R>) + (size_t)6 * (pl.Pz / 2 + 1) * pl.tz * sizeof(R);
    if (em_big(3LL * pl.Pz * pl.tz))
        hipLaunchKernelGGL((zconv_kernel<R, 32>), dim3(blocks), dim3(kNT), lds, s, static_cast<cx<R>*>(X2),
                           static_cast<const R*>(spec), Ms, pl.nz, pl.lgPz, pl.Py, pl.Hx, pl.Hy, pl.Hz, pl.Sx, lgT,
                           ntx, bpm);
    else
        hipLaunchKernelGGL((zconv_kernel<R, 16>), dim3(blocks), dim3(kNT), lds, s, static_cast<cx<R>*>(X2),
                           static_cast<const R*>(spec), Ms, pl.nz, pl.lgPz, pl.Py, pl.Hx, pl.Hy, pl.Hz, pl.Sx, lgT,
                           ntx, bpm);
    return hipGetLastError();
}

template hipError_t launch_yfwd<float>(const Plan&, const void*, void*, hipStream_t);
template hipError_t launch_yfwd<double>(const Plan&, const void*, void*, hipStream_t);
template hipError_t launch_yinv<float>(const Plan&, const void*, void*, hipStream_t);
template hipError_t launch_yinv<double>(const Plan&, const void*, void*, hipStream_t);
template hipError_t launch_zconv<float>(const Plan&, void*, const void*, float, hipStream_t);
template hipError_t launch_zconv<double>(const Plan&, void*, const void*, double, hipStream_t);

}  // namespace magx
