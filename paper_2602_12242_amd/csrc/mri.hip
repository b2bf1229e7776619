// Explicit-explicit multirate stepping of Eq. (1) (Section III-C): the
// torque of the exchange field is the fast partition, everything else (demag,
// DMI, anisotropy, bias) the slow one, and both time scales use the
// three-stage third-order method of Knoth and Wolke in its multirate
// infinitesimal step form.
//
// Per step and slow stage i = 1..3 the slow torque S_i = R(Y_i, H_eff - H_exch)
// is evaluated once (one FFT convolution); the forcing of the following fast
// interval, r_i = sum_j w_ij S_j, is formed in the same kernel.  The fast ODE
// dv/dtau = R(v, H_exch(v)) + r_i is then advanced in equal substeps, each the
// three stages of the method in Williamson's two-register form
//   q <- A_k q + h F(v),  v <- v + B_k q,
// A = (0, -5/9, -153/128), B = (1/3, 15/16, 8/15).  A fast stage is one
// stencil kernel over the grid; the last one of an interval optionally
// renormalises and performs the forward x pass of the next slow evaluation.
#include "cell_ops.hpp"

namespace magx {

// Slow stage: inverse x pass of the convolution output + slow local terms +
// torque; r = wa*Sa + wb*Sb + wn*S (Sa, Sb earlier slow torques or null).
template <typename R, bool BIG>
__global__ void __launch_bounds__(kNT) mri_slow_kernel(const cx<R>* __restrict__ Y1, const R* __restrict__ y,
                                                       PG g, Phys<R> ph, int has_demag, R* __restrict__ S_out,
                                                       const R* __restrict__ Sa, const R* __restrict__ Sb, R wa,
                                                       R wb, R wn, R* __restrict__ r_out) {
    const bool stream = stream_of<BIG>(g);
    extern __shared__ unsigned char smem_raw[];
    cx<R>* buf = reinterpret_cast<cx<R>*>(smem_raw);
    const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int mb = lb / g.bpm;
    int pen0, npen;
    block_pencils(g, lb - mb * g.bpm, pen0, npen);
    const long long mo = (long long)mb * 3 * g.N;
    y += mo;
    r_out += mo;
    if (S_out) S_out += mo;
    if (Sa) Sa += mo;
    if (Sb) Sb += mo;
    R hbv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) hbv[c] = ph.hbm ? ph.hbm[mb * 3 + c] : ph.hb[c];
    const bool vec = (g.nx & 1) == 0;
    if (has_demag) c2r_lines<R, BIG>(buf, Y1, g, mb, pen0, npen);
    for (int e = threadIdx.x; e < npen << g.lgLq; e += kNT) {
        const int p = e >> g.lgLq, n = e & ((1 << g.lgLq) - 1);
        const int x0 = 2 * n;
        if (x0 >= g.nx) continue;
        const bool two = x0 + 1 < g.nx;
        int yy, z;
        pen_coords<R>(g, pen0 + p, yy, z);
        const long long id = ((long long)z * g.ny + yy) * g.nx + x0;
        R m[2][3], H[2][3], ex[2], dm[2], an[2], S[2][3], r[2][3], sw[2];
        local_field_pair<R>(y, g, x0, yy, z, vec, two, ph, m, H, ex, dm, an, false, sw);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            // with a profile: no field outside the magnet
            const R inside = (!ph.msp || sw[q] > (R)0) ? (R)1 : (R)0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (has_demag) H[q][c] += inside * demag_at<R>(buf, 3 * p + c, g.Lh, n, q);
                if (ph.terms & MAGX_ZEEMAN) H[q][c] += inside * hbv[c];
            }
            llg_rhs<R>(m[q], H[q], ph.a, ph.alpha, S[q]);
#pragma unroll
            for (int c = 0; c < 3; ++c) r[q][c] = wn * S[q][c];
        }
        if (Sa) {
            R a0[3], a1[3];
            load_pair(Sa, g.N, id, vec, two, a0, a1);
#pragma unroll
            for (int c = 0; c < 3; ++c) { r[0][c] += wa * a0[c]; r[1][c] += wa * a1[c]; }
        }
        if (Sb) {
            R b0[3], b1[3];
            load_pair(Sb, g.N, id, vec, two, b0, b1);
#pragma unroll
            for (int c = 0; c < 3; ++c) { r[0][c] += wb * b0[c]; r[1][c] += wb * b1[c]; }
        }
        if (ph.nf) note_nonfinite(ph.nf, any_nonfinite<R, 3>(r[0]) || (two && any_nonfinite<R, 3>(r[1])));
        if (S_out) store_pair(S_out, g.N, id, vec, two, S[0], S[1], stream);
        store_pair(r_out, g.N, id, vec, two, r[0], r[1], stream);
    }
}

// One fast stage: F = R(v, H_exch(v)) + r; q <- Ak q + h F (q not read when
// first); v_out = v + Bk q, renormalised if norm; r2c of v_out into X1 if fwd.
template <typename R, bool BIG>
__global__ void __launch_bounds__(kNT) mri_fast_kernel(const R* __restrict__ v, R* __restrict__ vout,
                                                       R* __restrict__ qbuf, const R* __restrict__ rbuf, PG g,
                                                       Phys<R> ph, R Ak, R Bk, R h, int first, int norm, int fwd,
                                                       cx<R>* __restrict__ X1) {
    const bool stream = stream_of<BIG>(g);
    extern __shared__ unsigned char smem_raw[];
    cx<R>* buf = reinterpret_cast<cx<R>*>(smem_raw);
    const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int mb = lb / g.bpm;
    int pen0, npen;
    block_pencils(g, lb - mb * g.bpm, pen0, npen);
    const long long mo = (long long)mb * 3 * g.N;
    v += mo;
    vout += mo;
    qbuf += mo;
    rbuf += mo;
    const bool vec = (g.nx & 1) == 0;
    // v_out also goes into this thread's LDS line entries for the forward x pass
    // one slot (cell pair) per iteration; kept rolled to keep the kernel small
#pragma unroll 1
    for (int i = 0; i < maxslot<BIG>(); ++i) {
        const int e = threadIdx.x + i * kNT;
        if (e >= npen << g.lgLq) continue;
        const int p = e >> g.lgLq, n = e & ((1 << g.lgLq) - 1);
        const int x0 = 2 * n;
        if (x0 >= g.nx) {
            if (fwd) {
#pragma unroll
                for (int c = 0; c < 3; ++c) buf[(3 * p + c) * g.Lh + n] = mk<R>((R)0, (R)0);
            }
            continue;
        }
        const bool two = x0 + 1 < g.nx;
        int yy, z;
        pen_coords<R>(g, pen0 + p, yy, z);
        const long long id = ((long long)z * g.ny + yy) * g.nx + x0;
        R m[2][3], H[2][3], ex[2], dm[2], an[2], r[2][3], q[2][3], k[2][3], xn[2][3], sw[2];
        local_field_pair<R>(v, g, x0, yy, z, vec, two, ph, m, H, ex, dm, an, false, sw);
        load_pair(rbuf, g.N, id, vec, two, r[0], r[1]);
        if (!first) load_pair(qbuf, g.N, id, vec, two, q[0], q[1]);
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            llg_rhs<R>(m[s], H[s], ph.a, ph.alpha, k[s]);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const R F = k[s][c] + r[s][c];
                q[s][c] = first ? h * F : Ak * q[s][c] + h * F;
                xn[s][c] = m[s][c] + Bk * q[s][c];
            }
            if (norm) {
                const R nr = sqrt(dot3(xn[s], xn[s]));
                if (nr > (R)0) {
                    const R inv = (R)1 / nr;
#pragma unroll
                    for (int c = 0; c < 3; ++c) xn[s][c] *= inv;
                }
            }
        }
        if (ph.nf) note_nonfinite(ph.nf, any_nonfinite<R, 3>(xn[0]) || (two && any_nonfinite<R, 3>(xn[1])));
        store_pair(qbuf, g.N, id, vec, two, q[0], q[1], stream);
        store_pair(vout, g.N, id, vec, two, xn[0], xn[1], stream);
        if (fwd) {
            // demag source of the next slow stage: Ms(r) m = Ms s m
#pragma unroll
            for (int c = 0; c < 3; ++c)
                buf[(3 * p + c) * g.Lh + n] = mk<R>(sw[0] * xn[0][c], two ? sw[1] * xn[1][c] : (R)0);
        }
    }
    if (!fwd) return;
    r2c_lines<R, BIG>(buf, X1, g, mb, pen0, npen);
}

template <typename R>
hipError_t launch_mri_slow(const Plan& pl, const Phys<R>& ph, const void* Y1, const R* y, int has_demag, R* S_out,
                           const R* Sa, const R* Sb, R wa, R wb, R wn, R* r_out, hipStream_t s) {
    const PG g = make_pg(pl);
    const size_t lds = has_demag ? pencil_lds(pl) : 0;
    if (pencil_big(pl))
        hipLaunchKernelGGL((mri_slow_kernel<R, true>), dim3(pl.pencil_blocks), dim3(kNT), lds, s,
                           static_cast<const cx<R>*>(Y1), y, g, ph, has_demag, S_out, Sa, Sb, wa, wb, wn, r_out);
    else
        hipLaunchKernelGGL((mri_slow_kernel<R, false>), dim3(pl.pencil_blocks), dim3(kNT), lds, s,
                           static_cast<const cx<R>*>(Y1), y, g, ph, has_demag, S_out, Sa, Sb, wa, wb, wn, r_out);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_mri_fast(const Plan& pl, const Phys<R>& ph, const R* v, R* vout, R* q, const R* r, R Ak, R Bk,
                           R h, int first, int norm, void* X1, hipStream_t s) {
    const PG g = make_pg(pl);
    const int fwd = X1 != nullptr;
    const size_t lds = fwd ? pencil_lds(pl) : 0;
    if (pencil_big(pl))
        hipLaunchKernelGGL((mri_fast_kernel<R, true>), dim3(pl.pencil_blocks), dim3(kNT), lds, s, v, vout, q, r, g,
                           ph, Ak, Bk, h, first, norm, fwd, static_cast<cx<R>*>(X1));
    else
        hipLaunchKernelGGL((mri_fast_kernel<R, false>), dim3(pl.pencil_blocks), dim3(kNT), lds, s, v, vout, q, r,
                           g, ph, Ak, Bk, h, first, norm, fwd, static_cast<cx<R>*>(X1));
    return hipGetLastError();
}

template hipError_t launch_mri_slow<float>(const Plan&, const Phys<float>&, const void*, const float*, int, float*,
                                           const float*, const float*, float, float, float, float*, hipStream_t);
template hipError_t launch_mri_slow<double>(const Plan&, const Phys<double>&, const void*, const double*, int,
                                            double*, const double*, const double*, double, double, double, double*,
                                            hipStream_t);
template hipError_t launch_mri_fast<float>(const Plan&, const Phys<float>&, const float*, float*, float*,
                                           const float*, float, float, float, int, int, void*, hipStream_t);
template hipError_t launch_mri_fast<double>(const Plan&, const Phys<double>&, const double*, double*, double*,
                                            const double*, double, double, double, int, int, void*, hipStream_t);

}  // namespace magx
