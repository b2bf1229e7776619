// Demag tensor setup (Section II-B, Eq. (3)): real-space cell-averaged tensor
// on the non-negative octant of cell offsets, then its spectrum on the
// extended grid of twice the problem size, all in double precision.
//
// Tensor definition (H = -N M): N_ab(R) is minus the target-cell average of
// d_a d_b (1/|x-y|)/(4 pi) integrated over the source cell.
//  * r = |R|/max(dx,dy,dz) < 6: Newell-Williams-Dunlop closed forms (27-point
//    product of (-1, 2, -1) second differences of the auxiliary functions f
//    and g, divided by 4 pi V).
//  * otherwise: N(R) = -(V/4pi) E_v[K(R+v)], K_ab = (3 r_a r_b - r^2 d_ab)/r^5,
//    each v_i with the triangle density (d_i-|v_i|)/d_i^2 (difference of two
//    uniform points of a cell), by Gauss-Legendre on each triangle half with
//    a node count that falls with distance.
//
// Spectrum: every component is even or odd along each axis (odd along two
// axes for the off-diagonal ones) and vanishes at the unreachable offsets
// +-n, so its DFT on the extended grid is real and separable:
//   sum_{X=-(n-1)}^{n-1} N(X) e^{-2 pi i k X/P} = sum_{X>=0} c_X N(X) cos(2 pi k X/P)   (even)
//                                            = -i sum_{X>0} 2 N(X) sin(2 pi k X/P)  (odd)
// with c_0 = 1, c_X = 2; two odd axes give (-i)^2 = -1.  The transform is
// applied axis by axis as a dense product (a contraction over X) on the
// octant, only for k in [0, P/2]; the 1/(Px Py Pz) of the inverse FFT is
// folded in.
#include <math.h>

#include "magx_internal.hpp"

namespace magx {

__device__ float2 g_tw32[kTwN];
__device__ double2 g_tw64[kTwN];

__global__ void twiddle_init_kernel() {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < kTwN) {
        double s, c;
        sincospi(-2.0 * (double)k / (double)kTwN, &s, &c);
        g_tw64[k] = make_double2(c, s);
        g_tw32[k] = make_float2((float)c, (float)s);
    }
}

// ---- Newell auxiliary functions (double) ----------------------------------------
__device__ double newell_f(double x, double y, double z) {
    const double x2 = x * x, y2 = y * y, z2 = z * z;
    const double R = sqrt(x2 + y2 + z2);
    double out = (2.0 * x2 - y2 - z2) * R / 6.0;
    double s = x2 + z2;
    if (s > 0.0) out += 0.5 * y * (z2 - x2) * asinh(y / sqrt(s));
    s = x2 + y2;
    if (s > 0.0) out += 0.5 * z * (y2 - x2) * asinh(z / sqrt(s));
    if (x != 0.0 && R > 0.0) out -= x * y * z * atan(y * z / (x * R));
    return out;
}

__device__ double newell_g(double x, double y, double z) {
    const double x2 = x * x, y2 = y * y, z2 = z * z;
    const double R = sqrt(x2 + y2 + z2);
    double out = -x * y * R / 3.0;
    double s = x2 + y2;
    if (s > 0.0) out += x * y * z * asinh(z / sqrt(s));
    s = y2 + z2;
    if (s > 0.0) out += y / 6.0 * (3.0 * z2 - y2) * asinh(x / sqrt(s));
    s = x2 + z2;
    if (s > 0.0) out += x / 6.0 * (3.0 * z2 - x2) * asinh(y / sqrt(s));
    if (z != 0.0) out -= z2 * z / 6.0 * atan(x * y / (z * R));
    if (y != 0.0) out -= z * y2 / 2.0 * atan(x * z / (y * R));
    if (x != 0.0) out -= z * x2 / 2.0 * atan(y * z / (x * R));
    return out;
}

template <bool G>
__device__ double second_diff(double X, double Y, double Z, double a, double b, double c) {
    const double w[3] = {-1.0, 2.0, -1.0};
    double acc = 0.0;
    for (int i = -1; i <= 1; ++i)
        for (int j = -1; j <= 1; ++j)
            for (int k = -1; k <= 1; ++k) {
                const double f = G ? newell_g(X + i * a, Y + j * b, Z + k * c)
                                   : newell_f(X + i * a, Y + j * b, Z + k * c);
                acc += w[i + 1] * w[j + 1] * w[k + 1] * f;
            }
    return acc / (4.0 * M_PI * a * b * c);
}

struct GaussTable {
    // Gauss-Legendre nodes/weights on [-1, 1] for q = 2..6, packed by q
    double t[21];
    double w[21];
    int off[8];
};

__device__ void far_tensor(double X, double Y, double Z, double dx, double dy, double dz, int q,
                           const GaussTable& gt, double out[6]) {
    // nodes of the triangle density on each axis: v = +-(d/2)(t+1), weight
    // w_GL (d/2) (d - |v|)/d^2 (weights sum to 1 per axis)
    double vx[12], wx[12], vy[12], wy[12], vz[12], wz[12];
    const int o = gt.off[q];
    for (int i = 0; i < q; ++i) {
        const double t = gt.t[o + i], w = gt.w[o + i];
        double v = 0.5 * dx * (t + 1.0);
        vx[i] = -v; vx[q + i] = v; wx[i] = wx[q + i] = w * 0.5 * dx * (dx - v) / (dx * dx);
        v = 0.5 * dy * (t + 1.0);
        vy[i] = -v; vy[q + i] = v; wy[i] = wy[q + i] = w * 0.5 * dy * (dy - v) / (dy * dy);
        v = 0.5 * dz * (t + 1.0);
        vz[i] = -v; vz[q + i] = v; wz[i] = wz[q + i] = w * 0.5 * dz * (dz - v) / (dz * dz);
    }
    double s[6] = {0, 0, 0, 0, 0, 0};
    const int n = 2 * q;
    for (int a = 0; a < n; ++a) {
        const double x = X + vx[a];
        for (int b = 0; b < n; ++b) {
            const double y = Y + vy[b];
            const double wab = wx[a] * wy[b];
            for (int c = 0; c < n; ++c) {
                const double z = Z + vz[c];
                const double r2 = x * x + y * y + z * z;
                const double ir = 1.0 / sqrt(r2);
                const double ir2 = ir * ir;
                const double w = wab * wz[c] * ir2 * ir2 * ir;   // weight / r^5
                s[0] += w * (3.0 * x * x - r2);
                s[1] += w * (3.0 * y * y - r2);
                s[2] += w * (3.0 * z * z - r2);
                s[3] += w * (3.0 * x * y);
                s[4] += w * (3.0 * x * z);
                s[5] += w * (3.0 * y * z);
            }
        }
    }
    const double scale = -(dx * dy * dz) / (4.0 * M_PI);
    for (int c = 0; c < 6; ++c) out[c] = scale * s[c];
}

__device__ int quad_nodes(double r) {
    if (r < 12.0) return 6;
    if (r < 40.0) return 5;
    if (r < 150.0) return 4;
    if (r < 2000.0) return 3;
    return 2;
}

// One thread per non-negative offset (i, j, k); writes oct[c][k][j][i], c = xx yy zz xy xz yz.
__global__ void __launch_bounds__(kNT) newell_octant_kernel(double* __restrict__ oct, int nx, int ny, int nz,
                                                            double dx, double dy, double dz, GaussTable gt) {
    const long long n = (long long)nx * ny * nz;
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n) return;
    const int i = (int)(id % nx);
    const int j = (int)((id / nx) % ny);
    const int k = (int)(id / ((long long)nx * ny));
    const double X = i * dx, Y = j * dy, Z = k * dz;
    const double dmax = fmax(dx, fmax(dy, dz));
    const double r = sqrt(X * X + Y * Y + Z * Z) / dmax;
    double t[6];
    if (r < 6.0) {
        t[0] = second_diff<false>(X, Y, Z, dx, dy, dz);
        t[1] = second_diff<false>(Y, X, Z, dy, dx, dz);
        t[2] = second_diff<false>(Z, Y, X, dz, dy, dx);
        t[3] = second_diff<true>(X, Y, Z, dx, dy, dz);
        t[4] = second_diff<true>(X, Z, Y, dx, dz, dy);
        t[5] = second_diff<true>(Y, Z, X, dy, dz, dx);
    } else {
        far_tensor(X, Y, Z, dx, dy, dz, quad_nodes(r), gt, t);
    }
    for (int c = 0; c < 6; ++c) oct[c * n + id] = t[c];
}

// Axis transform as a tiled dense product.  For each component c:
//   out[c][k][q] = scale_c * sum_{j<J} wgt_j * trig_c(2 pi k j / P) * in[c][q][j],  k < K,
// trig = cos for components even along the axis, sin for odd ones
// (parity bit mask `odd`, bit c), wgt_0 = 1, wgt_j = 2; scale_c = -scale for
// components in the mask `neg`, else scale.  The output row q is
// written at ((q / orow) * ostride + q % orow) inside component c's slab of
// oslab elements.  With TILED (the last pass, q = ky * Hx + kx, k = kz) the
// output is the z pass's layout [Hy][ntz][6][Hz][tz]: for each row ky and
// column tile of tz values, the six components' Hz x tz blocks back to back
// (orow = Hx, ostride = tz, oslab = ntz, and Hz = K).
template <typename TO, bool TILED>
__global__ void __launch_bounds__(kNT) axis_transform_kernel(const double* __restrict__ in, TO* __restrict__ out,
                                                             int Q, int J, int K, int P, int lgP, unsigned odd,
                                                             double scale, unsigned neg, long long islab,
                                                             int orow, int ostride, long long oslab) {
    constexpr int TQ = 64, TK = 32, TJ = 32;
    __shared__ double sIn[TJ][TQ + 1];
    __shared__ double sM[TJ][TK + 1];
    const int c = blockIdx.z;
    const int q0 = blockIdx.x * TQ, k0 = blockIdx.y * TK;
    const bool isodd = (odd >> c) & 1u;
    const double* inc = in + (long long)c * islab;
    const int tq = threadIdx.x & 15;     // 16 x 4 = 64 q
    const int tk = threadIdx.x >> 4;     // 16 x 2 = 32 k
    double acc[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
    const int twshift = kTwLog - lgP;
    for (int j0 = 0; j0 < J; j0 += TJ) {
        for (int e = threadIdx.x; e < TQ * TJ; e += kNT) {
            const int jj = e % TJ, qq = e / TJ;
            const int q = q0 + qq, j = j0 + jj;
            sIn[jj][qq] = (q < Q && j < J) ? inc[(long long)q * J + j] : 0.0;
        }
        for (int e = threadIdx.x; e < TK * TJ; e += kNT) {
            const int kk = e % TK, jj = e / TK;
            const int k = k0 + kk, j = j0 + jj;
            double v = 0.0;
            if (j < J) {
                const int idx = (int)(((long long)k * j) & (P - 1)) << twshift;
                const double2 w = g_tw64[idx];     // (cos t, -sin t)
                v = isodd ? -w.y : w.x;
                if (j > 0) v *= 2.0;
            }
            sM[jj][kk] = v;
        }
        __syncthreads();
#pragma unroll 8
        for (int jj = 0; jj < TJ; ++jj) {
            const double m0 = sM[jj][tk], m1 = sM[jj][tk + 16];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const double x = sIn[jj][tq + 16 * b];
                acc[0][b] += m0 * x;
                acc[1][b] += m1 * x;
            }
        }
        __syncthreads();
    }
    const double sc = ((neg >> c) & 1u) ? -scale : scale;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const int k = k0 + tk + 16 * a;
        if (k >= K) continue;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int q = q0 + tq + 16 * b;
            if (q >= Q) continue;
            long long o;
            if constexpr (TILED) {
                const int ky = q / orow, kx = q % orow;
                const int tile = kx / ostride, col = kx % ostride;
                o = ((((long long)ky * oslab + tile) * 6 + c) * K + k) * ostride + col;
            } else {
                o = (long long)c * oslab + (long long)k * ((long long)(Q / orow) * ostride) +
                    (long long)(q / orow) * ostride + (q % orow);
            }
            out[o] = (TO)(sc * acc[a][b]);
        }
    }
}

// Host: Gauss-Legendre nodes by Newton iteration on P_q.
static GaussTable make_gauss_table() {
    GaussTable gt{};
    int off = 0;
    for (int q = 0; q < 8; ++q) gt.off[q] = 0;
    for (int q = 2; q <= 6; ++q) {
        gt.off[q] = off;
        for (int i = 0; i < q; ++i) {
            double x = cos(M_PI * (i + 0.75) / (q + 0.5));
            for (int it = 0; it < 100; ++it) {
                double p0 = 1.0, p1 = x;
                for (int n = 2; n <= q; ++n) {
                    const double p2 = ((2.0 * n - 1.0) * x * p1 - (n - 1.0) * p0) / n;
                    p0 = p1;
                    p1 = p2;
                }
                const double dp = q * (x * p1 - p0) / (x * x - 1.0);
                const double dx = p1 / dp;
                x -= dx;
                if (fabs(dx) < 1e-17) break;
            }
            double p0 = 1.0, p1 = x;
            for (int n = 2; n <= q; ++n) {
                const double p2 = ((2.0 * n - 1.0) * x * p1 - (n - 1.0) * p0) / n;
                p0 = p1;
                p1 = p2;
            }
            const double dp = q * (x * p1 - p0) / (x * x - 1.0);
            gt.t[off + i] = x;
            gt.w[off + i] = 2.0 / ((1.0 - x * x) * dp * dp);
        }
        off += q;
    }
    return gt;
}

// Parity masks (bit c set = odd) along x, y, z for c = xx yy zz xy xz yz.
static constexpr unsigned kOddX = (1u << 3) | (1u << 4);
static constexpr unsigned kOddY = (1u << 3) | (1u << 5);
static constexpr unsigned kOddZ = (1u << 4) | (1u << 5);

hipError_t launch_twiddle_init(hipStream_t s) {
    hipLaunchKernelGGL(twiddle_init_kernel, dim3(kTwN / kNT), dim3(kNT), 0, s);
    return hipGetLastError();
}

// The tensor's Nyquist column kx = Hx - 1 (column 0 of each row's last tile)
// once more, for the z pass's Nyquist units: blocks [6][Hz][tz] like the
// column tiles', column c of block b holding row q = b tz + c (rows q >= Py/2
// zero), and one extra block that is block 0 with row Py/2 in column 0 (the
// mirrored rows' q = 0).
__global__ void nyquist_copy_kernel(float* spec, int half, int Hz, int tz, int ntz, int nblk, long long tn_off) {
    const long long e = (long long)blockIdx.x * kNT + threadIdx.x;
    const long long per = 6LL * Hz * tz;
    if (e >= (nblk + 1) * per) return;
    const int b = (int)(e / per);
    const int r = (int)(e - b * per);
    const int c6 = r / (Hz * tz), kzo = (r / tz) % Hz, c = r % tz;
    const int q = b < nblk ? b * tz + c : c;
    const int kyo = (b == nblk && c == 0) ? half : q;
    spec[tn_off + e] = (q < half || kyo == half)
                           ? spec[(((long long)kyo * ntz + ntz - 1) * 6 + c6) * Hz * tz + (long long)kzo * tz]
                           : 0.0f;
}

hipError_t build_tensor_spectrum(const Plan& pl, void* spectrum, void* scratch, hipStream_t s) {
    const int nx = pl.nx, ny = pl.ny, nz = pl.nz;
    const long long n = (long long)nx * ny * nz;
    double* oct = static_cast<double*>(scratch);
    double* t1 = oct + pl.scratch_a_elems;     // [6][Hx][nz*ny]
    double* t2 = oct;                          // [6][Hy][Hx*nz] (reuses the octant slab)
    GaussTable gt = make_gauss_table();
    hipLaunchKernelGGL(newell_octant_kernel, dim3((unsigned)((n + kNT - 1) / kNT)), dim3(kNT), 0, s, oct, nx, ny,
                       nz, pl.dx, pl.dy, pl.dz, gt);
    if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
    // x: in [6][nz*ny][nx] -> t1 [6][Hx][nz*ny]
    {
        const int Q = nz * ny, J = nx, K = pl.Hx;
        dim3 grid((Q + 63) / 64, (K + 31) / 32, 6);
        hipLaunchKernelGGL((axis_transform_kernel<double, false>), grid, dim3(kNT), 0, s, oct, t1, Q, J, K, pl.Px, pl.lgPx,
                           kOddX, 1.0, 0u, n, Q, Q, (long long)K * Q);
        if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
    }
    // y: in [6][Hx*nz][ny] -> t2 [6][Hy][Hx*nz]
    {
        const int Q = pl.Hx * nz, J = ny, K = pl.Hy;
        dim3 grid((Q + 63) / 64, (K + 31) / 32, 6);
        hipLaunchKernelGGL((axis_transform_kernel<double, false>), grid, dim3(kNT), 0, s, t1, t2, Q, J, K, pl.Py, pl.lgPy,
                           kOddY, 1.0, 0u, (long long)pl.Hx * nz * ny, Q, Q, (long long)K * Q);
        if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
    }
    // z: in [6][Hy*Hx][nz] -> spectrum in the z pass's layout
    // [Hy][ntz][6][Hz][tz], scaled by 1/(Px Py Pz) and by -1 for the
    // off-diagonal components.  Columns kx >= Hx of the last tile are never read.
    {
        const int Q = pl.Hy * pl.Hx, J = nz, K = pl.Hz;
        dim3 grid((Q + 63) / 64, (K + 31) / 32, 6);
        const double sc = 1.0 / ((double)pl.Px * pl.Py * pl.Pz);
        const unsigned offdiag = (1u << 3) | (1u << 4) | (1u << 5);
        if (pl.dtype == MAGX_F32) {
            hipLaunchKernelGGL((axis_transform_kernel<float, true>), grid, dim3(kNT), 0, s, t2,
                               static_cast<float*>(spectrum), Q, J, K, pl.Pz, pl.lgPz, kOddZ, sc, offdiag,
                               (long long)pl.Hy * pl.Hx * nz, pl.Hx, pl.tz, (long long)pl.ntz);
        } else {
            hipLaunchKernelGGL((axis_transform_kernel<double, true>), grid, dim3(kNT), 0, s, t2,
                               static_cast<double*>(spectrum), Q, J, K, pl.Pz, pl.lgPz, kOddZ, sc, offdiag,
                               (long long)pl.Hy * pl.Hx * nz, pl.Hx, pl.tz, (long long)pl.ntz);
        }
        if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
    }
    // the Nyquist column kx = Hx - 1 (column 0 of the last tile) once more, in
    // blocks along ky for the z pass's Nyquist units
    if (pl.nyqpack) {
        const int half = pl.Py / 2, nblk = (half + pl.tz - 1) / pl.tz;
        const long long n = (nblk + 1) * 6LL * pl.Hz * pl.tz;
        hipLaunchKernelGGL(nyquist_copy_kernel, dim3((unsigned)((n + kNT - 1) / kNT)), dim3(kNT), 0, s,
                           static_cast<float*>(spectrum), half, pl.Hz, pl.tz, pl.ntz, nblk, pl.tn_off);
        if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
    }
    return hipSuccess;
}

}  // namespace magx
