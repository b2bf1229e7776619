// x-direction passes of the demag convolution fused with everything that is
// local to a cell (Section II-A/II-B, Eqs. (1), (2), (5), (7), (9), (10)).
//
// A block owns np "pencils" (z, y) and all three components of each: 3*np
// x lines.  The real transform of length Px = 2^k (>= 2 nx, zero padded) is
// done as a complex FFT of length Lh = Px/2 on z[n] = x[2n] + i x[2n+1] plus
// the usual split/merge step, so each thread slot owns a PAIR of cells
// (2n, 2n+1) and LDS line entries are written whole.
//
// Kernels
//  xfwd    r2c of a field (first forward x pass of a step)
//  field   c2r of the demag spectrum + exchange/DMI/anisotropy/Zeeman -> H_eff,
//          or per-block energy sums, or K applied to a cotangent
//  stage   one RK4 stage: H_eff(y_s) -> k_s = R(y_s) -> accumulator, next
//          stage input (renormalised) -> its r2c for the next convolution
//  bstart  reverse of the step's final combination and renormalisation
//  bstage  reverse of one stage: K mu_s + pointwise Jacobian-transpose terms
//
// Boundary condition (Eq. (10) with the outward normal n): one ghost per face,
// m_ghost = m_b + h (-D/2A) (e_z x n) x m_b, shared by the exchange and DMI
// stencils; on z faces and without DMI it is plain zero-flux Neumann.
#include "cell_ops.hpp"

namespace magx {

// ---- kernels -------------------------------------------------------------------

template <typename R, bool BIG, int LG>
__global__ void __launch_bounds__(kNT) xfwd_kernel(const R* __restrict__ f, cx<R>* __restrict__ X1, PG g,
                                                   const R* __restrict__ msp) {
    pg_fix<LG>(g);
    extern __shared__ unsigned char smem_raw[];
    cx<R>* buf = reinterpret_cast<cx<R>*>(smem_raw);
    // logical block -> member mb and its first pencil; members own contiguous block ranges
    const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int mb = lb / g.bpm;
    int pen0, npen;
    block_pencils(g, lb - mb * g.bpm, pen0, npen);
    const long long mo = (long long)mb * 3 * g.N;   // member offset of vector fields
    f += mo;
    const bool vec = (g.nx & 1) == 0;
    const int nitem = npen << g.lgLq;
    // every cell pair of this thread is loaded first (one 8-byte load per
    // component when nx is even), so that their latencies overlap; the LDS
    // line entries are written afterwards
    R va[maxslot<BIG>()][3], vb[maxslot<BIG>()][3], s0[maxslot<BIG>()], s1[maxslot<BIG>()];
#pragma unroll
    for (int i = 0; i < maxslot<BIG>(); ++i) {
        const int e = threadIdx.x + i * kNT;
        s0[i] = s1[i] = (R)1;
#pragma unroll
        for (int c = 0; c < 3; ++c) va[i][c] = vb[i][c] = (R)0;
        if (e >= nitem) continue;
        const int p = e >> g.lgLq, n = e & ((1 << g.lgLq) - 1);
        const int x0 = 2 * n;
        if (x0 >= g.nx) continue;
        int y, z;
        pen_coords<R>(g, pen0 + p, y, z);
        const long long id = ((long long)z * g.ny + y) * g.nx + x0;
        const bool two = x0 + 1 < g.nx;
        load_pair(f, g.N, id, vec, two, va[i], vb[i]);
        // the demag source is Ms(r) m = Ms s m with a magnetisation profile
        if (msp) {
            s0[i] = msp[id];
            s1[i] = two ? msp[id + 1] : (R)0;
        }
    }
#pragma unroll
    for (int i = 0; i < maxslot<BIG>(); ++i) {
        const int e = threadIdx.x + i * kNT;
        if (e >= nitem) continue;
        const int p = e >> g.lgLq, n = e & ((1 << g.lgLq) - 1);
#pragma unroll
        for (int c = 0; c < 3; ++c) buf[(3 * p + c) * g.Lh + n] = mk<R>(s0[i] * va[i][c], s1[i] * vb[i][c]);
    }
    r2c_lines<R, BIG>(buf, X1, g, mb, pen0, npen);
}

// mode: 0 -> write H (with bias if with_bias); 1 -> energy partials (m.H_term).
// RED: the block sums (energy, or the sum of the input field) are wanted; the
// plain field evaluation is a kernel of its own without their accumulators,
// which keeps it within the registers of five waves per SIMD.
template <typename R, bool BIG, int LG, bool RED>
__device__ __forceinline__ void field_body(const cx<R>* __restrict__ Y1, const R* __restrict__ f,
                                           R* __restrict__ H, PG g, Phys<R> ph, int has_demag,
                                           int with_bias, int energy, int sum_input,
                                           double* __restrict__ partials) {
    if constexpr (!RED) energy = sum_input = 0;
    pg_fix<LG>(g);
    const bool stream = stream_of<BIG>(g);
    extern __shared__ unsigned char smem_raw[];
    cx<R>* buf = reinterpret_cast<cx<R>*>(smem_raw);
    __shared__ double red[kNT];
    // logical block -> member mb and its first pencil; members own contiguous block ranges
    const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int mb = lb / g.bpm;
    int pen0, npen;
    block_pencils(g, lb - mb * g.bpm, pen0, npen);
    const long long mo = (long long)mb * 3 * g.N;   // member offset of vector fields
    f += mo;
    if (H) H += mo;
    R hbv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) hbv[c] = ph.hbm ? ph.hbm[mb * 3 + c] : ph.hb[c];
    const bool vec = (g.nx & 1) == 0;
    if (has_demag) c2r_lines<R, BIG>(buf, Y1, g, mb, pen0, npen);
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int e = threadIdx.x; e < npen << g.lgLq; e += kNT) {
        const int p = e >> g.lgLq, n = e & ((1 << g.lgLq) - 1);
        const int x0 = 2 * n;
        if (x0 >= g.nx) continue;
        const bool two = x0 + 1 < g.nx;
        int y, z;
        pen_coords<R>(g, pen0 + p, y, z);
        R m[2][3], hl[2][3], ex[2], dm[2], an[2], out[2][3], sw[2];
        local_field_pair<R>(f, g, x0, y, z, vec, two, ph, m, hl, ex, dm, an, energy != 0, sw);
        const long long id = ((long long)z * g.ny + y) * g.nx + x0;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            R hd[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) hd[c] = has_demag ? demag_at<R>(buf, 3 * p + c, g.Lh, n, q) : (R)0;
            const bool live = q == 0 || two;
            // with a profile: no field outside the magnet, densities weighted by s
            const R inside = sw[q] > (R)0 ? (R)1 : (R)0;
            if (energy) {
                if (live) {
                    const double w = (double)sw[q];
                    acc[0] += w * (double)(inside * dot3(m[q], hd));
                    acc[1] += w * (double)ex[q];
                    acc[2] += w * (double)dm[q];
                    acc[3] += w * (double)an[q];
                    if (ph.terms & MAGX_ZEEMAN) acc[4] += w * (double)dot3(m[q], hbv);
                    acc[5] += (double)inside;
                }
            } else {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    out[q][c] = inside * hd[c] + hl[q][c];
                    if (with_bias && (ph.terms & MAGX_ZEEMAN)) out[q][c] += inside * hbv[c];
                }
                if (sum_input && live) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) acc[c] += (double)m[q][c];
                }
            }
        }
        if (!energy) {
            if (ph.nf) note_nonfinite(ph.nf, any_nonfinite<R, 3>(out[0]) || (two && any_nonfinite<R, 3>(out[1])));
            store_pair(H, g.N, id, vec, two, out[0], out[1], stream);
        }
    }
    if (energy && ph.nf) note_nonfinite(ph.nf, !isfinite(acc[0] + acc[1] + acc[2] + acc[3] + acc[4]));
    if (energy) {
        for (int v = 0; v < 6; ++v) {
            const double sm = block_sum(acc[v], red);
            if (threadIdx.x == 0) partials[lb * 8 + v] = sm;
        }
    } else if (sum_input) {
        for (int v = 0; v < 3; ++v) {
            const double sm = block_sum(acc[v], red);
            if (threadIdx.x == 0) partials[lb * 8 + v] += sm;
        }
    }
}

template <typename R, bool BIG, int LG>
__global__ void __launch_bounds__(kNT) field_kernel(const cx<R>* __restrict__ Y1, const R* __restrict__ f,
                                                    R* __restrict__ H, PG g, Phys<R> ph, int has_demag,
                                                    int with_bias, int energy, int sum_input,
                                                    double* __restrict__ partials) {
    field_body<R, BIG, LG, false>(Y1, f, H, g, ph, has_demag, with_bias, energy, sum_input, partials);
}

template <typename R, bool BIG, int LG>
__global__ void __launch_bounds__(kNT) field_reduce_kernel(const cx<R>* __restrict__ Y1, const R* __restrict__ f,
                                                           R* __restrict__ H, PG g, Phys<R> ph, int has_demag,
                                                           int with_bias, int energy, int sum_input,
                                                           double* __restrict__ partials) {
    field_body<R, BIG, LG, true>(Y1, f, H, g, ph, has_demag, with_bias, energy, sum_input, partials);
}

template <typename R, bool BIG, int LG>
__global__ void __launch_bounds__(kNT) stage_kernel(const cx<R>* Y1, cx<R>* X1, PG g,
                                                    Phys<R> ph, StageArgs<R> a, int has_demag) {
    pg_fix<LG>(g);
    const bool stream = stream_of<BIG>(g);
    extern __shared__ unsigned char smem_raw[];
    cx<R>* buf = reinterpret_cast<cx<R>*>(smem_raw);
    // logical block -> member mb and its first pencil; members own contiguous block ranges
    const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int mb = lb / g.bpm;
    int pen0, npen;
    block_pencils(g, lb - mb * g.bpm, pen0, npen);
    const long long mo = (long long)mb * 3 * g.N;   // member offset of vector fields
    const long long mo1 = (long long)mb * g.N;      // member offset of scalar fields
    a.yin += mo;
    a.mn += mo;
    a.acc += mo;
    a.yout += mo;
    if (a.yout2) a.yout2 += mo;
    if (a.tapeH) a.tapeH += mo;
    if (a.tapeYin) a.tapeYin += mo;
    if (a.tapeNx) a.tapeNx += mo1;
    R hbv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) hbv[c] = ph.hbm ? ph.hbm[mb * 3 + c] : ph.hb[c];
    const bool vec = (g.nx & 1) == 0;
    if (has_demag) c2r_lines<R, BIG>(buf, Y1, g, mb, pen0, npen);
    // classical RK4 tableau
    const R bw[4] = {(R)(1.0 / 6.0), (R)(1.0 / 3.0), (R)(1.0 / 3.0), (R)(1.0 / 6.0)};
    const R cw[4] = {(R)0, (R)0.5, (R)0.5, (R)1};
    const int s = a.stage;
    // stage 0 is a forward Euler step: m_{n+1} = y + dt k, renormalised like a new state
    const bool norm = (s >= 1 && s < 4) ? (ph.renorm == 2) : (ph.renorm >= 1);
    // the next stage input goes straight into this thread's own LDS line
    // entries (the ones it read the demag field from) for the forward x pass
    const bool fwd = a.want_next && has_demag;
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
        int y, z;
        pen_coords<R>(g, pen0 + p, y, z);
        const long long id = ((long long)z * g.ny + y) * g.nx + x0;
        // RK4 registers first, so their loads are in flight with the stencil's
        R k[2][3], mn[2][3], acc[2][3], xn[2][3], nrm[2];
        if (s > 1) {
            load_pair(a.mn, g.N, id, vec, two, mn[0], mn[1], stream);
            load_pair(a.acc, g.N, id, vec, two, acc[0], acc[1], stream);
        }
        R ys[2][3], H[2][3], ex[2], dm[2], an[2], sw[2];
        local_field_pair<R>(a.yin, g, x0, y, z, vec, two, ph, ys, H, ex, dm, an, false, sw);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            // with a profile: no field (so no motion) outside the magnet
            const R inside = (!ph.msp || sw[q] > (R)0) ? (R)1 : (R)0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (has_demag) H[q][c] += inside * demag_at<R>(buf, 3 * p + c, g.Lh, n, q);
                if (ph.terms & MAGX_ZEEMAN) H[q][c] += inside * hbv[c];
            }
        }
        if (a.tapeH) store_pair(a.tapeH, g.N, id, vec, two, H[0], H[1], stream);
        if (a.tapeYin) store_pair(a.tapeYin, g.N, id, vec, two, ys[0], ys[1], stream);
#pragma unroll
        for (int q = 0; q < 2; ++q) llg_rhs<R>(ys[q], H[q], ph.a, ph.alpha, k[q]);
        if (s <= 1) {
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int c = 0; c < 3; ++c) mn[q][c] = ys[q][c];
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (s == 0) {
                    xn[q][c] = mn[q][c] + a.dt * k[q][c];
                } else if (s < 4) {
                    acc[q][c] = (s == 1 ? (R)0 : acc[q][c]) + bw[s - 1] * k[q][c];
                    xn[q][c] = mn[q][c] + cw[s] * a.dt * k[q][c];
                } else {
                    xn[q][c] = mn[q][c] + a.dt * (acc[q][c] + bw[3] * k[q][c]);
                }
            }
            nrm[q] = (R)1;
            if (norm) {
                nrm[q] = sqrt(dot3(xn[q], xn[q]));
                if (nrm[q] > (R)0) {
                    const R inv = (R)1 / nrm[q];
#pragma unroll
                    for (int c = 0; c < 3; ++c) xn[q][c] *= inv;
                }
            }
        }
        if (ph.nf)
            note_nonfinite(ph.nf, any_nonfinite<R, 3>(xn[0]) || any_nonfinite<R, 3>(H[0]) ||
                                      (two && (any_nonfinite<R, 3>(xn[1]) || any_nonfinite<R, 3>(H[1]))));
        if (s >= 1 && s < 4) store_pair(a.acc, g.N, id, vec, two, acc[0], acc[1], stream);
        if (a.tapeNx) {
            if (vec) *reinterpret_cast<cx<R>*>(a.tapeNx + id) = mk<R>(nrm[0], nrm[1]);
            else { a.tapeNx[id] = nrm[0]; if (two) a.tapeNx[id + 1] = nrm[1]; }
        }
        store_pair(a.yout, g.N, id, vec, two, xn[0], xn[1], stream);
        if (a.yout2) store_pair(a.yout2, g.N, id, vec, two, xn[0], xn[1], stream);
        if (fwd) {
            // demag source of the next stage: Ms(r) m = Ms s m
#pragma unroll
            for (int c = 0; c < 3; ++c)
                buf[(3 * p + c) * g.Lh + n] = mk<R>(sw[0] * xn[0][c], two ? sw[1] * xn[1][c] : (R)0);
        }
    }
    if (!fwd) return;
    r2c_lines<R, BIG>(buf, X1, g, mb, pen0, npen);
}

template <typename R, bool BIG, int LG>
__global__ void __launch_bounds__(kNT) bstart_kernel(cx<R>* __restrict__ X1, PG g, Phys<R> ph, StartArgs<R> a,
                                                     int has_demag, double* __restrict__ partials) {
    pg_fix<LG>(g);
    const bool stream = stream_of<BIG>(g);
    extern __shared__ unsigned char smem_raw[];
    cx<R>* buf = reinterpret_cast<cx<R>*>(smem_raw);
    __shared__ double red[kNT];
    // logical block -> member mb and its first pencil; members own contiguous block ranges
    const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int mb = lb / g.bpm;
    int pen0, npen;
    block_pencils(g, lb - mb * g.bpm, pen0, npen);
    const long long mo = (long long)mb * 3 * g.N;   // member offset of vector fields
    const long long mo1 = (long long)mb * g.N;      // member offset of scalar fields
    a.gm += mo;
    a.y5 += mo;
    a.y4 += mo;
    a.xi5 += mo;
    a.kap += mo;
    a.muout += mo;
    a.nx5 += mo1;
    const bool vec = (g.nx & 1) == 0;
    const bool norm = ph.renorm >= 1;
    const R b4 = (R)(1.0 / 6.0);
    double hs[3] = {0, 0, 0};
    // mu_4 goes straight into this thread's LDS line entries for the forward x pass
    // one slot (cell pair) per iteration; kept rolled to keep the kernel small
#pragma unroll 1
    for (int i = 0; i < maxslot<BIG>(); ++i) {
        const int e = threadIdx.x + i * kNT;
        if (e >= npen << g.lgLq) continue;
        const int p = e >> g.lgLq, n = e & ((1 << g.lgLq) - 1);
        const int x0 = 2 * n;
        if (x0 >= g.nx) {
            if (has_demag) {
#pragma unroll
                for (int c = 0; c < 3; ++c) buf[(3 * p + c) * g.Lh + n] = mk<R>((R)0, (R)0);
            }
            continue;
        }
        const bool two = x0 + 1 < g.nx;
        int y, z;
        pen_coords<R>(g, pen0 + p, y, z);
        const long long id = ((long long)z * g.ny + y) * g.nx + x0;
        R lam[2][3], xi[2][3], y5[2][3], y4[2][3], kap[2][3], mu[2][3];
        load_pair(a.gm, g.N, id, vec, two, lam[0], lam[1]);
        load_pair(a.y4, g.N, id, vec, two, y4[0], y4[1]);
        if (norm) {
            load_pair(a.y5, g.N, id, vec, two, y5[0], y5[1]);
            R nx5[2];
            nx5[0] = a.nx5[id];
            const R n1 = a.nx5[id + (two ? 1 : 0)];
            nx5[1] = two ? n1 : (R)1;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const R pl = dot3(y5[q], lam[q]);
                const R inv = nx5[q] > (R)0 ? (R)1 / nx5[q] : (R)1;
#pragma unroll
                for (int c = 0; c < 3; ++c) xi[q][c] = (lam[q][c] - y5[q][c] * pl) * inv;
            }
        } else {
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int c = 0; c < 3; ++c) xi[q][c] = lam[q][c];
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
#pragma unroll
            for (int c = 0; c < 3; ++c) kap[q][c] = b4 * a.dt * xi[q][c];
            rhs_mu<R>(y4[q], kap[q], ph.a, ph.alpha, mu[q]);
        }
        if (ph.nf) note_nonfinite(ph.nf, any_nonfinite<R, 3>(xi[0]) || (two && any_nonfinite<R, 3>(xi[1])));
        store_pair(a.xi5, g.N, id, vec, two, xi[0], xi[1], stream);
        store_pair(a.gm, g.N, id, vec, two, xi[0], xi[1], stream);
        store_pair(a.kap, g.N, id, vec, two, kap[0], kap[1], stream);
        store_pair(a.muout, g.N, id, vec, two, mu[0], mu[1], stream);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const R m1 = two ? mu[1][c] : (R)0;
            hs[c] += (double)mu[0][c] + (double)m1;
            if (has_demag) buf[(3 * p + c) * g.Lh + n] = mk<R>(mu[0][c], m1);
        }
    }
    if (ph.terms & MAGX_ZEEMAN) {
        for (int v = 0; v < 3; ++v) {
            const double sm = block_sum(hs[v], red);
            if (threadIdx.x == 0) partials[lb * 8 + v] += sm;
        }
    }
    if (!has_demag) return;
    r2c_lines<R, BIG>(buf, X1, g, mb, pen0, npen);
}

template <typename R, bool BIG, int LG>
__global__ void __launch_bounds__(kNT) bstage_kernel(const cx<R>* Y1, cx<R>* X1, PG g,
                                                     Phys<R> ph, BackArgs<R> a, int has_demag,
                                                     double* __restrict__ partials) {
    pg_fix<LG>(g);
    const bool stream = stream_of<BIG>(g);
    extern __shared__ unsigned char smem_raw[];
    cx<R>* buf = reinterpret_cast<cx<R>*>(smem_raw);
    __shared__ double red[kNT];
    // logical block -> member mb and its first pencil; members own contiguous block ranges
    const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int mb = lb / g.bpm;
    int pen0, npen;
    block_pencils(g, lb - mb * g.bpm, pen0, npen);
    const long long mo = (long long)mb * 3 * g.N;   // member offset of vector fields
    const long long mo1 = (long long)mb * g.N;      // member offset of scalar fields
    a.mu += mo;
    a.ys += mo;
    a.Hs += mo;
    a.kap += mo;
    a.xi5 += mo;
    a.gm += mo;
    a.muout += mo;
    if (a.yprev) a.yprev += mo;
    if (a.nxs) a.nxs += mo1;
    const bool vec = (g.nx & 1) == 0;
    if (has_demag) c2r_lines<R, BIG>(buf, Y1, g, mb, pen0, npen);
    const R bw[4] = {(R)(1.0 / 6.0), (R)(1.0 / 3.0), (R)(1.0 / 3.0), (R)(1.0 / 6.0)};
    const R cw[4] = {(R)0, (R)0.5, (R)0.5, (R)1};
    const int s = a.stage;
    const bool norm = ph.renorm == 2;
    double hs[3] = {0, 0, 0};
    // mu_{s-1} goes straight into this thread's own LDS line entries (read
    // above for K mu_s) for the forward x pass
    const bool fwd = s > 1 && has_demag;
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
        int y, z;
        pen_coords<R>(g, pen0 + p, y, z);
        const long long id = ((long long)z * g.ny + y) * g.nx + x0;
        R mu[2][3], Kmu[2][3], ex[2], dm[2], an[2];
        R sw[2];
        local_field_pair<R>(a.mu, g, x0, y, z, vec, two, ph, mu, Kmu, ex, dm, an, false, sw);
        if (has_demag) {
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int c = 0; c < 3; ++c) Kmu[q][c] += demag_at<R>(buf, 3 * p + c, g.Lh, n, q);
        }
        R ys[2][3], Hs[2][3], kap[2][3], lam[2][3], yb[2][3];
        load_pair(a.ys, g.N, id, vec, two, ys[0], ys[1]);
        load_pair(a.Hs, g.N, id, vec, two, Hs[0], Hs[1]);
        load_pair(a.kap, g.N, id, vec, two, kap[0], kap[1]);
        load_pair(a.gm, g.N, id, vec, two, lam[0], lam[1]);
        // ybar = a [H x kappa + alpha (H (y.kappa) + kappa (y.H) - 2 y (H.kappa))] + K mu
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            R Hxk[3];
            cross3(Hs[q], kap[q], Hxk);
            const R yk = dot3(ys[q], kap[q]), yH = dot3(ys[q], Hs[q]), Hk = dot3(Hs[q], kap[q]);
#pragma unroll
            for (int c = 0; c < 3; ++c)
                yb[q][c] = ph.a * (Hxk[c] + ph.alpha * (Hs[q][c] * yk + kap[q][c] * yH - (R)2 * ys[q][c] * Hk)) +
                           Kmu[q][c];
        }
        if (s > 1) {
            R xi[2][3], x5[2][3], kp[2][3], yp[2][3], mup[2][3];
            if (norm) {
                R nxs[2];
                nxs[0] = a.nxs[id];
                const R n1 = a.nxs[id + (two ? 1 : 0)];
                nxs[1] = two ? n1 : (R)1;
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const R py = dot3(ys[q], yb[q]);
                    const R inv = nxs[q] > (R)0 ? (R)1 / nxs[q] : (R)1;
#pragma unroll
                    for (int c = 0; c < 3; ++c) xi[q][c] = (yb[q][c] - ys[q][c] * py) * inv;
                }
            } else {
#pragma unroll
                for (int q = 0; q < 2; ++q)
#pragma unroll
                    for (int c = 0; c < 3; ++c) xi[q][c] = yb[q][c];
            }
            load_pair(a.xi5, g.N, id, vec, two, x5[0], x5[1]);
            load_pair(a.yprev, g.N, id, vec, two, yp[0], yp[1]);
#pragma unroll
            for (int q = 0; q < 2; ++q) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    lam[q][c] += xi[q][c];
                    kp[q][c] = bw[s - 2] * a.dt * x5[q][c] + cw[s - 1] * a.dt * xi[q][c];
                }
                rhs_mu<R>(yp[q], kp[q], ph.a, ph.alpha, mup[q]);
            }
            if (ph.nf) note_nonfinite(ph.nf, any_nonfinite<R, 3>(lam[0]) || (two && any_nonfinite<R, 3>(lam[1])));
            store_pair(a.gm, g.N, id, vec, two, lam[0], lam[1], stream);
            store_pair(a.kap, g.N, id, vec, two, kp[0], kp[1], stream);
            store_pair(a.muout, g.N, id, vec, two, mup[0], mup[1], stream);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const R m1 = two ? mup[1][c] : (R)0;
                hs[c] += (double)mup[0][c] + (double)m1;
                if (fwd) buf[(3 * p + c) * g.Lh + n] = mk<R>(mup[0][c], m1);
            }
        } else {
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int c = 0; c < 3; ++c) lam[q][c] += yb[q][c];
            if (ph.nf) note_nonfinite(ph.nf, any_nonfinite<R, 3>(lam[0]) || (two && any_nonfinite<R, 3>(lam[1])));
            store_pair(a.gm, g.N, id, vec, two, lam[0], lam[1], stream);
        }
    }
    if (s > 1 && (ph.terms & MAGX_ZEEMAN)) {
        for (int v = 0; v < 3; ++v) {
            const double sm = block_sum(hs[v], red);
            if (threadIdx.x == 0) partials[lb * 8 + v] += sm;
        }
    }
    if (!fwd) return;
    r2c_lines<R, BIG>(buf, X1, g, mb, pen0, npen);
}

template <typename R>
__global__ void rhs_kernel(const R* __restrict__ m, const R* __restrict__ H, R* __restrict__ out, long long N,
                           R a, R alpha) {
    // grid (cells / kNT, members); member mb's fields start at mb * 3N
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N) return;
    const long long id = (long long)blockIdx.y * 3 * N + t;
    R mm[3], hh[3], k[3];
    load3(m, N, id, mm);
    load3(H, N, id, hh);
    llg_rhs<R>(mm, hh, a, alpha, k);
    store3(out, N, id, k);
}

__global__ void fill_zero_kernel(double* p, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

template <typename R>
__global__ void reduce_partials_kernel(const double* __restrict__ partials, int bpm, int nval, R* out,
                                       int accumulate) {
    __shared__ double red[kNT];
    const int mb = blockIdx.x;
    const double* pp = partials + (long long)mb * bpm * 8;
    for (int v = 0; v < nval; ++v) {
        double acc = 0.0;
        for (int b = threadIdx.x; b < bpm; b += kNT) acc += pp[b * 8 + v];
        const double s = block_sum(acc, red);
        R* o = out + mb * nval + v;
        if (threadIdx.x == 0) *o = accumulate ? (R)((double)*o + s) : (R)s;
    }
}

// e_out[6 mb + ...]: demag, exch, dmi, anis, zeeman, total (J) of member mb.
// pref = -(mu0 Ms V)/2, vku_cell = V Ku (anisotropy constant term per magnetic
// cell; partial 5 counts the magnetic cells).
__global__ void energy_finish_kernel(const double* __restrict__ partials, int bpm, double pref,
                                     double vku_cell, double* e_out) {
    __shared__ double red[kNT];
    const int mb = blockIdx.x;
    const double* pp = partials + (long long)mb * bpm * 8;
    double e[6];
    for (int v = 0; v < 6; ++v) {
        double acc = 0.0;
        for (int b = threadIdx.x; b < bpm; b += kNT) acc += pp[b * 8 + v];
        e[v] = block_sum(acc, red);
    }
    if (threadIdx.x == 0) {
        const double ed = pref * e[0], ee = pref * e[1], em = pref * e[2];
        const double ea = pref * e[3] + vku_cell * e[5], ez = 2.0 * pref * e[4];
        double* o = e_out + 6 * mb;
        o[0] = ed;
        o[1] = ee;
        o[2] = em;
        o[3] = ea;
        o[4] = ez;
        o[5] = ed + ee + em + ea + ez;
    }
}

template <typename R>
__global__ void copy_kernel(const R* __restrict__ src, R* __restrict__ dst, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// ---- launchers -----------------------------------------------------------------

// Pencil kernel launch: the power-of-two line lengths 2^7 ... 2^10 with
// compile-time geometry, every other size with runtime geometry.
#define MAGX_PENCIL_LAUNCH(KERNEL, ...)                                                                 \
    do {                                                                                                \
        const dim3 grid_((unsigned)pl.pencil_blocks), block_(kNT);                                      \
        const size_t lds_ = pencil_lds(pl);                                                             \
        switch (pencil_lg(pl)) {                                                                        \
            case 7: hipLaunchKernelGGL((KERNEL<R, false, 7>), grid_, block_, lds_, s, __VA_ARGS__); break;  \
            case 8: hipLaunchKernelGGL((KERNEL<R, false, 8>), grid_, block_, lds_, s, __VA_ARGS__); break;  \
            case 9: hipLaunchKernelGGL((KERNEL<R, false, 9>), grid_, block_, lds_, s, __VA_ARGS__); break;  \
            case 10: hipLaunchKernelGGL((KERNEL<R, false, 10>), grid_, block_, lds_, s, __VA_ARGS__); break; \
            default:                                                                                    \
                if (pencil_big(pl))                                                                     \
                    hipLaunchKernelGGL((KERNEL<R, true, 0>), grid_, block_, lds_, s, __VA_ARGS__);      \
                else                                                                                    \
                    hipLaunchKernelGGL((KERNEL<R, false, 0>), grid_, block_, lds_, s, __VA_ARGS__);     \
        }                                                                                               \
    } while (0)

template <typename R>
hipError_t launch_xfwd(const Plan& pl, const R* f, void* X1, const R* msp, hipStream_t s) {
    MAGX_PENCIL_LAUNCH(xfwd_kernel, f, static_cast<cx<R>*>(X1), make_pg(pl), msp);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_field(const Plan& pl, const Phys<R>& ph, const void* Y1, const R* f, R* H, int with_bias,
                        int energy, int sum_input, double* partials, hipStream_t s) {
    const int has_demag = (ph.terms & MAGX_DEMAG) ? 1 : 0;
    if (energy || sum_input)
        MAGX_PENCIL_LAUNCH(field_reduce_kernel, static_cast<const cx<R>*>(Y1), f, H, make_pg(pl), ph, has_demag, with_bias, energy, sum_input, partials);
    else
        MAGX_PENCIL_LAUNCH(field_kernel, static_cast<const cx<R>*>(Y1), f, H, make_pg(pl), ph, has_demag, with_bias, energy, sum_input, partials);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_stage(const Plan& pl, const Phys<R>& ph, const void* Y1, void* X1, const StageArgs<R>& a,
                        hipStream_t s) {
    const int has_demag = (ph.terms & MAGX_DEMAG) ? 1 : 0;
    MAGX_PENCIL_LAUNCH(stage_kernel, static_cast<const cx<R>*>(Y1), static_cast<cx<R>*>(X1), make_pg(pl), ph, a, has_demag);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_bstart(const Plan& pl, const Phys<R>& ph, void* X1, const StartArgs<R>& a, double* partials,
                         hipStream_t s) {
    const int has_demag = (ph.terms & MAGX_DEMAG) ? 1 : 0;
    MAGX_PENCIL_LAUNCH(bstart_kernel, static_cast<cx<R>*>(X1), make_pg(pl), ph, a, has_demag, partials);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_bstage(const Plan& pl, const Phys<R>& ph, const void* Y1, void* X1, const BackArgs<R>& a,
                         double* partials, hipStream_t s) {
    const int has_demag = (ph.terms & MAGX_DEMAG) ? 1 : 0;
    MAGX_PENCIL_LAUNCH(bstage_kernel, static_cast<const cx<R>*>(Y1), static_cast<cx<R>*>(X1), make_pg(pl), ph, a, has_demag, partials);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_rhs(const Plan& pl, const Phys<R>& ph, const R* m, const R* H, R* out, hipStream_t s) {
    const long long N = pl.ncell;
    hipLaunchKernelGGL(rhs_kernel<R>, dim3((unsigned)((N + kNT - 1) / kNT), (unsigned)pl.nbatch), dim3(kNT), 0, s, m,
                       H, out, N, ph.a, ph.alpha);
    return hipGetLastError();
}

hipError_t launch_fill_zero(double* p, long long n, hipStream_t s) {
    hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)((n + kNT - 1) / kNT)), dim3(kNT), 0, s, p, n);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_reduce_partials(const double* partials, int nbatch, int blocks_per_member, int nval, R* out,
                                  int accumulate, hipStream_t s) {
    hipLaunchKernelGGL(reduce_partials_kernel<R>, dim3(nbatch), dim3(kNT), 0, s, partials, blocks_per_member, nval,
                       out, accumulate);
    return hipGetLastError();
}

hipError_t launch_energy_finish(const double* partials, int nbatch, int blocks_per_member, double pref,
                                double vku_cell, double* e_out, hipStream_t s) {
    hipLaunchKernelGGL(energy_finish_kernel, dim3(nbatch), dim3(kNT), 0, s, partials, blocks_per_member, pref,
                       vku_cell, e_out);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_copy(const R* src, R* dst, long long n, hipStream_t s) {
    hipLaunchKernelGGL(copy_kernel<R>, dim3((unsigned)((n + kNT - 1) / kNT)), dim3(kNT), 0, s, src, dst, n);
    return hipGetLastError();
}

#define MAGX_INST(R)                                                                                            \
    template hipError_t launch_xfwd<R>(const Plan&, const R*, void*, const R*, hipStream_t);                               \
    template hipError_t launch_field<R>(const Plan&, const Phys<R>&, const void*, const R*, R*, int, int, int,   \
                                        double*, hipStream_t);                                                  \
    template hipError_t launch_stage<R>(const Plan&, const Phys<R>&, const void*, void*, const StageArgs<R>&,   \
                                        hipStream_t);                                                           \
    template hipError_t launch_bstart<R>(const Plan&, const Phys<R>&, void*, const StartArgs<R>&, double*,      \
                                         hipStream_t);                                                          \
    template hipError_t launch_bstage<R>(const Plan&, const Phys<R>&, const void*, void*, const BackArgs<R>&,   \
                                         double*, hipStream_t);                                                 \
    template hipError_t launch_rhs<R>(const Plan&, const Phys<R>&, const R*, const R*, R*, hipStream_t);         \
    template hipError_t launch_reduce_partials<R>(const double*, int, int, int, R*, int, hipStream_t);          \
    template hipError_t launch_copy<R>(const R*, R*, long long, hipStream_t);

MAGX_INST(float)
MAGX_INST(double)

}  // namespace magx
