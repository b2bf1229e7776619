// Device helpers shared by the x-pass kernels and the multirate kernels:
// cell-pair accesses, the local field terms with the boundary ghost rule,
// the LLG torque and its transpose, and the x-line transforms in LDS.
//
// Boundary condition (Eq. (10) with the outward normal n): one ghost per face,
// m_ghost = m_b + h (-D/2A) (e_z x n) x m_b, shared by the exchange and DMI
// stencils; on z faces and without DMI it is plain zero-flux Neumann.
#pragma once

#include "magx_internal.hpp"

namespace magx {

// Two register budgets: BIG = false holds 16 FFT elements and 4 cell-pair
// slots per thread (np * Lh <= 1024, every grid with nx <= 1024); BIG = true
// holds 32 and 8 (nx up to 2048, float only).
template <bool BIG> constexpr int pemax() { return BIG ? 32 : 16; }
template <bool BIG> constexpr int maxslot() { return BIG ? 8 : 4; }

struct PG {
    int nx, ny, nz, Lh, lgLh, Hx, Sx, lgPx, np, npen_total;   // npen_total: pencils of one member
    // log2 of the cell-pair slots per line, max(Lh/2, 1): the cells fill the
    // lower half of a packed line (x < nx <= Px/2); the upper half is the zero
    // padding, which the forward pass never reads and nothing writes
    int lgLq;
    int bpm;                                                 // blocks per member
    int zmajor;                                              // block order: z fastest (see block_pencils)
    int stream;                                              // streaming cell-pair stores (see store_pair;
                                                             // kernels read it once, as stream_of)
    long long N;                                             // cells of one member
    FastDiv div_ny, div_hx;                                  // n / ny and n / Hx
};

// LDS bytes of a pencil block (3 np lines of Lh complex values) and its register budget
inline size_t pencil_lds(const Plan& pl) { return (size_t)3 * pl.np * pl.Lh * pl.esize * 2; }
inline bool pencil_big(const Plan& pl) { return pl.np * pl.Lh > 1024; }

// Compile-time line geometry: for a power-of-two line nx = Lh = 2^LG (so
// Px = 2 nx, Hx = Lh + 1, Sx = Lh + 16) the kernels are instantiated with the
// sizes as constants, which turns the FFT strides and row offsets into
// immediates; LG = 0 keeps them runtime values.
constexpr int kPencilLgMin = 7, kPencilLgMax = 10;

inline int pencil_lg(const Plan& pl) {
    if (pl.nx != pl.Lh || pl.lgLh < kPencilLgMin || pl.lgLh > kPencilLgMax || pl.Sx != pl.Lh + 16 ||
        pl.np * pl.Lh > 1024)
        return 0;
    return pl.lgLh;
}

template <int LG>
__device__ __forceinline__ void pg_fix(PG& g) {
    if constexpr (LG > 0) {
        g.lgLh = LG;
        g.lgLq = LG - 1;
        g.Lh = 1 << LG;
        g.lgPx = LG + 1;
        g.nx = 1 << LG;
        g.Hx = (1 << LG) + 1;
        g.Sx = (1 << LG) + 16;
    }
}

// The streaming flag of a kernel, read once into a register: the 32-element
// register budget (BIG) leaves no room for the second store path, so those
// kernels never stream.
template <bool BIG>
__device__ __forceinline__ bool stream_of(const PG& g) {
    return !BIG && g.stream != 0;
}

inline PG make_pg(const Plan& pl) {
    PG g;
    g.nx = pl.nx; g.ny = pl.ny; g.nz = pl.nz;
    g.Lh = pl.Lh; g.lgLh = pl.lgLh; g.Hx = pl.Hx; g.Sx = pl.Sx; g.lgPx = pl.lgPx;
    g.lgLq = pl.lgLh > 0 ? pl.lgLh - 1 : 0;
    g.np = pl.np; g.npen_total = pl.ny * pl.nz; g.bpm = pl.blocks_per_member; g.N = pl.ncell;
    g.div_ny = make_fastdiv(pl.ny);
    g.div_hx = make_fastdiv(pl.Hx);
    g.zmajor = pl.pencil_zmajor;
    // fields of 64 MiB and more (a batch counts whole) are far larger than the caches
    g.stream = !pencil_big(pl) && 3.0 * (double)pl.ncell * pl.nbatch * pl.esize >= 64.0 * (1 << 20) ? 1 : 0;
    return g;
}

// Pencils of block lbm of a member: np consecutive rows y of one plane z.
// With zmajor the blocks run through z fastest ((y group, z) -> lbm =
// group * nz + z), so the blocks holding a row's z neighbours run right
// before and after it on the same XCD and the stencil finds them in L2;
// otherwise pencils are numbered z * ny + y and a block takes np of them.
// Either way its pencils are consecutive in the z * ny + y numbering.
__device__ __forceinline__ void block_pencils(const PG& g, int lbm, int& pen0, int& npen) {
    if (g.zmajor) {
        const int grp = lbm / g.nz;
        const int z = lbm - grp * g.nz;
        const int y0 = grp * g.np;
        pen0 = z * g.ny + y0;
        npen = min(g.np, g.ny - y0);
    } else {
        pen0 = lbm * g.np;
        npen = min(g.np, g.npen_total - pen0);
    }
}

template <typename R>
__device__ __forceinline__ void load3(const R* __restrict__ f, long long N, long long id, R v[3]) {
    v[0] = f[id];
    v[1] = f[N + id];
    v[2] = f[2 * N + id];
}

template <typename R>
__device__ __forceinline__ void store3(R* __restrict__ f, long long N, long long id, const R v[3]) {
    f[id] = v[0];
    f[N + id] = v[1];
    f[2 * N + id] = v[2];
}

// ---- cell pairs (2n, 2n+1) along x ------------------------------------------------
// With nx even every pair is complete and 8-byte (float) / 16-byte (double)
// aligned, so a pair is one vector access per component; with nx odd the last
// pair of a row has a single cell and scalar accesses are used.  Fields that a
// pencil kernel writes are read again a whole convolution later at the
// earliest; on grids whose fields are far larger than the caches (PG::stream)
// pairs are stored with streaming stores (see st_stream), and a field read
// once (stream) is loaded the same way.  Measured at 512 x 512 x 32: the
// reverse start kernel 186 -> 178 us, the forward y pass that follows a stage
// 126 -> 122 us; at 256 x 256 x 16, whose fields stay in the caches, the same
// accesses cost 3 % of an RK4 step.
template <typename R>
__device__ __forceinline__ void load_pair(const R* __restrict__ f, long long N, long long id, bool vec, bool two,
                                          R a[3], R b[3], bool stream = false) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const R* p = f + c * N + id;
        if (vec) {
            const cx<R> v = stream ? ld_stream<R>(reinterpret_cast<const cx<R>*>(p))
                                   : *reinterpret_cast<const cx<R>*>(p);
            a[c] = v.x;
            b[c] = v.y;
        } else {
            a[c] = p[0];
            const R v1 = p[two ? 1 : 0];   // unconditional load: no wait behind a branch
            b[c] = two ? v1 : (R)0;
        }
    }
}

template <typename R>
__device__ __forceinline__ void store_pair(R* __restrict__ f, long long N, long long id, bool vec, bool two,
                                           const R a[3], const R b[3], bool stream = false) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        R* p = f + c * N + id;
        if (vec) {
            if (stream) st_stream<R>(reinterpret_cast<cx<R>*>(p), mk<R>(a[c], b[c]));
            else *reinterpret_cast<cx<R>*>(p) = mk<R>(a[c], b[c]);
        } else {
            p[0] = a[c];
            if (two) p[1] = b[c];
        }
    }
}

// Ghost values of the boundary condition (Eq. (10)) for a cell c on a face
// with outward normal -x, +x, -y, +y (kd = -D/(2A) times the cell size; on z
// faces the ghost is c itself).
template <typename R> __device__ __forceinline__ void ghost_xm(const R c[3], R kd, R o[3]) {
    o[0] = c[0] - kd * c[2]; o[1] = c[1]; o[2] = c[2] + kd * c[0];
}
template <typename R> __device__ __forceinline__ void ghost_xp(const R c[3], R kd, R o[3]) {
    o[0] = c[0] + kd * c[2]; o[1] = c[1]; o[2] = c[2] - kd * c[0];
}
template <typename R> __device__ __forceinline__ void ghost_ym(const R c[3], R kd, R o[3]) {
    o[0] = c[0]; o[1] = c[1] - kd * c[2]; o[2] = c[2] + kd * c[1];
}
template <typename R> __device__ __forceinline__ void ghost_yp(const R c[3], R kd, R o[3]) {
    o[0] = c[0]; o[1] = c[1] + kd * c[2]; o[2] = c[2] - kd * c[1];
}

template <typename R>
__device__ __forceinline__ void load_s_pair(const R* __restrict__ s, long long id, bool vec, bool two, R o[2]) {
    if (vec) {
        const cx<R> v = *reinterpret_cast<const cx<R>*>(s + id);
        o[0] = v.x;
        o[1] = v.y;
    } else {
        o[0] = s[id];
        const R v1 = s[id + (two ? 1 : 0)];
        o[1] = two ? v1 : (R)0;
    }
}

// Exchange + DMI + anisotropy of the linear field f for the pair of cells
// (x0 = 2n, x0 + 1) of row (y, z); h*[0] belongs to cell x0, h*[1] to x0 + 1.
// A neighbour outside the grid, or (with a magnetisation profile ph.msp)
// outside the magnet, is replaced by the ghost of the boundary condition built
// from the cell itself.  With a profile the local prefactors are divided by the
// cell's s = Ms(r)/Ms and cells with s = 0 get no field; sw returns s of the
// two cells (1 without a profile).
template <typename R>
__device__ __forceinline__ void local_field_pair(const R* __restrict__ f, const PG& g, int x0, int y, int z,
                                                 bool vec, bool two, const Phys<R>& ph, R m[2][3], R h[2][3],
                                                 R hex_dot[2], R hdmi_dot[2], R hani_dot[2], bool want_parts,
                                                 R sw[2]) {
    const long long N = g.N;
    const long long id = ((long long)z * g.ny + y) * g.nx + x0;
    const R* __restrict__ sp = ph.msp;
    load_pair(f, N, id, vec, two, m[0], m[1]);
    sw[0] = sw[1] = (R)1;
    if (sp) load_s_pair(sp, id, vec, two, sw);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
#pragma unroll
        for (int c = 0; c < 3; ++c) h[q][c] = (R)0;
        hex_dot[q] = hdmi_dot[q] = hani_dot[q] = (R)0;
    }
    if (ph.terms & (MAGX_EXCH | MAGX_DMI)) {
        const R kdx = ph.kap * ph.dx, kdy = ph.kap * ph.dy;
        R xl[3], xr[3], yp[2][3], ym[2][3], zp[2][3], zm[2][3];
        // Neighbour availability: in the grid and (with a profile) in the
        // magnet.  Every neighbour is loaded, at the cell itself where it lies
        // outside the grid (so the address is valid), and replaced by its ghost
        // value afterwards: no load sits behind a branch, so all of them are in
        // flight together.
        const int xr_off = two ? 2 : 1;
        const long long pz = (long long)g.nx * g.ny;
        const bool gxl = x0 > 0, gxr = x0 + xr_off < g.nx;
        const bool gyp = y + 1 < g.ny, gym = y > 0, gzp = z + 1 < g.nz, gzm = z > 0;
        const long long il = gxl ? id - 1 : id, ir = gxr ? id + xr_off : id;
        const long long iyp = gyp ? id + g.nx : id, iym = gym ? id - g.nx : id;
        const long long izp = gzp ? id + pz : id, izm = gzm ? id - pz : id;
        R xlv[3], xrv[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            xlv[c] = f[c * N + il];
            xrv[c] = f[c * N + ir];
        }
        load_pair(f, N, iyp, vec, two, yp[0], yp[1]);
        load_pair(f, N, iym, vec, two, ym[0], ym[1]);
        load_pair(f, N, izp, vec, two, zp[0], zp[1]);
        load_pair(f, N, izm, vec, two, zm[0], zm[1]);
        bool okxl = gxl, okxr = gxr;
        bool okyp[2], okym[2], okzp[2], okzm[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            okyp[q] = gyp;
            okym[q] = gym;
            okzp[q] = gzp;
            okzm[q] = gzm;
        }
        if (sp) {
            const R sl = sp[il], sr = sp[ir];
            R t0[2], t1[2], t2[2], t3[2];
            load_s_pair(sp, iyp, vec, two, t0);
            load_s_pair(sp, iym, vec, two, t1);
            load_s_pair(sp, izp, vec, two, t2);
            load_s_pair(sp, izm, vec, two, t3);
            okxl = okxl && sl > (R)0;
            okxr = okxr && sr > (R)0;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                okyp[q] = okyp[q] && t0[q] > (R)0;
                okym[q] = okym[q] && t1[q] > (R)0;
                okzp[q] = okzp[q] && t2[q] > (R)0;
                okzm[q] = okzm[q] && t3[q] > (R)0;
            }
        }
        // outer x neighbours of the pair: cell x0 - 1 and cell x0 + 2 (or x0 + 1 if alone)
        R last[3], gl[3], gr[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) last[c] = two ? m[1][c] : m[0][c];
        ghost_xm<R>(m[0], kdx, gl);
        ghost_xp<R>(last, kdx, gr);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            xl[c] = okxl ? xlv[c] : gl[c];
            xr[c] = okxr ? xrv[c] : gr[c];
        }
        // the two cells of the pair see each other unless one is outside the magnet
        const bool in0 = sw[0] > (R)0, in1 = sw[1] > (R)0;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const R* mc = m[q];
            R xp[3], xm[3], ypq[3], ymq[3], zpq[3], zmq[3];
            if (q == 0) {
#pragma unroll
                for (int c = 0; c < 3; ++c) xm[c] = xl[c];
                if (!two) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) xp[c] = xr[c];
                } else if (in1) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) xp[c] = m[1][c];
                } else {
                    ghost_xp<R>(m[0], kdx, xp);
                }
            } else {
#pragma unroll
                for (int c = 0; c < 3; ++c) xp[c] = xr[c];
                if (in0) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) xm[c] = m[0][c];
                } else {
                    ghost_xm<R>(m[1], kdx, xm);
                }
            }
            if (okyp[q]) { ypq[0] = yp[q][0]; ypq[1] = yp[q][1]; ypq[2] = yp[q][2]; }
            else ghost_yp<R>(mc, kdy, ypq);
            if (okym[q]) { ymq[0] = ym[q][0]; ymq[1] = ym[q][1]; ymq[2] = ym[q][2]; }
            else ghost_ym<R>(mc, kdy, ymq);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                zpq[c] = okzp[q] ? zp[q][c] : mc[c];
                zmq[c] = okzm[q] ? zm[q][c] : mc[c];
            }
            R hx[3] = {(R)0, (R)0, (R)0}, hd[3] = {(R)0, (R)0, (R)0};
            if (ph.terms & MAGX_EXCH) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const R m2 = (R)2 * mc[c];
                    hx[c] = ph.cex * ((xp[c] - m2 + xm[c]) * ph.idx2 + (ypq[c] - m2 + ymq[c]) * ph.idy2 +
                                      (zpq[c] - m2 + zmq[c]) * ph.idz2);
                }
            }
            if (ph.terms & MAGX_DMI) {
                hd[0] = ph.cdmi * (xp[2] - xm[2]) * ph.h2x;
                hd[1] = ph.cdmi * (ypq[2] - ymq[2]) * ph.h2y;
                hd[2] = -ph.cdmi * ((xp[0] - xm[0]) * ph.h2x + (ypq[1] - ymq[1]) * ph.h2y);
            }
            if (sp) {
                const R inv = sw[q] > (R)0 ? (R)1 / sw[q] : (R)0;
#pragma unroll
                for (int c = 0; c < 3; ++c) { hx[c] *= inv; hd[c] *= inv; }
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) h[q][c] = hx[c] + hd[c];
            if (want_parts) {
                hex_dot[q] = mc[0] * hx[0] + mc[1] * hx[1] + mc[2] * hx[2];
                hdmi_dot[q] = mc[0] * hd[0] + mc[1] * hd[1] + mc[2] * hd[2];
            }
        }
    }
    if (ph.terms & MAGX_ANIS) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const R pr = m[q][0] * ph.eK[0] + m[q][1] * ph.eK[1] + m[q][2] * ph.eK[2];
            R ca = ph.cani;
            if (sp) ca = sw[q] > (R)0 ? ca / sw[q] : (R)0;
#pragma unroll
            for (int c = 0; c < 3; ++c) h[q][c] += ca * pr * ph.eK[c];
            if (want_parts) hani_dot[q] = ca * pr * pr;
        }
    }
}

// Non-finite detection (calls made with check_finite): true if any of the
// n values is NaN or infinite; note_nonfinite sets the flag word with one
// atomic from the first lane of every wave that met such a value (called by
// all active lanes of the wave).
template <typename R, int n>
__device__ __forceinline__ bool any_nonfinite(const R* v) {
    bool bad = false;
#pragma unroll
    for (int i = 0; i < n; ++i) bad = bad || !isfinite(v[i]);
    return bad;
}

__device__ __forceinline__ void note_nonfinite(unsigned* flag, bool bad) {
    const unsigned long long b = __ballot(bad);
    if (b != 0ull && __lane_id() == (unsigned)(__ffsll((long long)b) - 1)) atomicOr(flag, 1u);
}

template <typename R>
__device__ __forceinline__ void cross3(const R a[3], const R b[3], R o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

template <typename R> __device__ __forceinline__ R dot3(const R a[3], const R b[3]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// Eq. (1) for unit m: a [m x H + alpha m x (m x H)].
template <typename R>
__device__ __forceinline__ void llg_rhs(const R m[3], const R H[3], R a, R alpha, R k[3]) {
    R mxH[3], mmH[3];
    cross3(m, H, mxH);
    cross3(m, mxH, mmH);
#pragma unroll
    for (int c = 0; c < 3; ++c) k[c] = a * (mxH[c] + alpha * mmH[c]);
}

// Cotangent of H for a cotangent kappa of R(y): a [kappa x y + alpha y x (y x kappa)].
template <typename R>
__device__ __forceinline__ void rhs_mu(const R y[3], const R kap[3], R a, R alpha, R mu[3]) {
    R kxy[3], yxk[3], yyk[3];
    cross3(kap, y, kxy);
    cross3(y, kap, yxk);
    cross3(y, yxk, yyk);
#pragma unroll
    for (int c = 0; c < 3; ++c) mu[c] = a * (kxy[c] + alpha * yyk[c]);
}

// ---- x-line transforms in LDS --------------------------------------------------
// LDS line for (pencil p, component c) starts at (3p + c) * Lh.

template <typename R>
__device__ __forceinline__ void pen_coords(const PG& g, int pen, int& y, int& z) {
    z = fdiv(pen, g.div_ny);
    y = pen - z * g.ny;
}

// Split/merge items per thread and chunk (3 np Lh/2 <= 1536 items per block
// for np Lh <= 1024).
constexpr int kXIt = 6;

// Row of X1/Y1 holding component c of pencil p (32-bit element offset: the
// spectral arrays of a whole batch stay below 2^31 elements).
__device__ __forceinline__ unsigned x_row(const PG& g, int mb, int c, int pen) {
    int y, z;
    z = fdiv(pen, g.div_ny);
    y = pen - z * g.ny;
    return (((unsigned)(mb * 3 + c) * (unsigned)g.nz + (unsigned)z) * (unsigned)g.ny + (unsigned)y) * (unsigned)g.Sx;
}

template <int V> struct IntC { static constexpr int value = V; };

// The half-length real-FFT split and merge steps pair bin k with its mirror
// Lh - k: both come from the same two values and the same twiddle
// W^k = exp(-2 pi i k / Px), since W^(Lh-k) = -conj(W^k).  Item t < Lq
// (Lq = max(Lh/2, 1)) of a line takes k = t and Lh - t; t = 0 also takes
// k = Lh/2 (its own mirror).

// Inverse x pass: Y1 rows -> real lines; afterwards the real value of cell x
// of line l is buf[l*Lh + x/2].x (x even) or .y (x odd).  Split step of the
// half-length inverse, Z[k] = (X[k] + X*[Lh-k]) + i (X[k] - X*[Lh-k]) w^-k
// (w^-k = conj(W^k)), into LDS; then the inverse FFT of every line in LDS.
template <typename R, bool BIG>
__device__ void c2r_lines(cx<R>* buf, const cx<R>* Y1, const PG& g, int mb, int pen0, int npen) {
    const int Lh = g.Lh;
    const int lgq = g.lgLh > 0 ? g.lgLh - 1 : 0;
    const int twsh = kTwLog - g.lgPx;
    auto split = [](cx<R> a, cx<R> b, cx<R> wc) {   // a = X[k], b = X[Lh-k], wc = conj(W^k)
        const cx<R> bc = cconj<R>(b);
        const cx<R> A = cadd<R>(a, bc);
        const cx<R> B = cmul<R>(csub<R>(a, bc), wc);
        return mk<R>(A.x - B.y, A.y + B.x);
    };
    tw_lds_fill<R>();   // pass twiddles, read after the barrier below
    if ((1 << lgq) >= kNT) {
        // at least one item per thread and line: thread tid takes items
        // t = tid + k kNT of every line, so its twiddles are the same for all
        // lines and each line's row address is uniform (scalar registers).
        // A chunk holds kXIt items per thread: with one item per line the six
        // lines of a two-pencil block are one chunk and their loads make one
        // round trip (measured at 512-cell lines: stage 224 -> 211 us).
        auto chunks = [&](auto ipl_c) {
            constexpr int IPL = decltype(ipl_c)::value;   // items per thread and line
            constexpr int LC = kXIt / IPL;                // lines per chunk
            cx<R> wc[IPL];
#pragma unroll
            for (int k = 0; k < IPL; ++k) wc[k] = cconj<R>(tw_fwd<R>(((int)threadIdx.x + k * kNT) << twsh));
            const int nl = npen * 3;
            for (int l0 = 0; l0 < nl; l0 += LC) {
                cx<R> A[LC][IPL], B[LC][IPL], C[LC];
#pragma unroll
                for (int i = 0; i < LC; ++i) {
                    const int l = min(l0 + i, nl - 1);
                    const int p = l / 3, c = l - 3 * p;
                    const cx<R>* row = Y1 + x_row(g, mb, c, pen0 + p);
#pragma unroll
                    for (int k = 0; k < IPL; ++k) {
                        const int t = (int)threadIdx.x + k * kNT;
                        A[i][k] = row[t];
                        B[i][k] = row[Lh - t];
                    }
                    // X[Lh/2] for item 0 of a line (loaded by the first wave only)
                    C[i] = mk<R>((R)0, (R)0);
                    if (threadIdx.x < 64) C[i] = row[threadIdx.x == 0 ? (Lh >> 1) : (int)threadIdx.x];
                }
#pragma unroll
                for (int i = 0; i < LC; ++i) {
                    const int l = l0 + i;
                    if (l >= nl) break;
                    cx<R>* out = buf + l * Lh;
#pragma unroll
                    for (int k = 0; k < IPL; ++k) {
                        const int t = (int)threadIdx.x + k * kNT;
                        if (t == 0) {
                            out[0] = split(A[i][k], B[i][k], mk<R>((R)1, (R)0));
                            out[Lh >> 1] = split(C[i], C[i], mk<R>((R)0, (R)1));   // conj(W^(Lh/2)) = i
                        } else {
                            out[t] = split(A[i][k], B[i][k], wc[k]);
                            out[Lh - t] = split(B[i][k], A[i][k], mk<R>(-wc[k].x, wc[k].y));   // conj(W^(Lh-t)) = -W^t
                        }
                    }
                }
            }
        };
        // Lh <= 2048: one, two or four items per thread and line
        if ((1 << lgq) == kNT) chunks(IntC<1>{});
        else if ((1 << lgq) == 2 * kNT) chunks(IntC<2>{});
        else chunks(IntC<4>{});
    } else {
    // items in chunks of kXIt per thread: all loads of a chunk are issued
    // before any is used (no load behind a branch or a loop-carried wait)
    const int count = (npen * 3) << lgq;
    for (int base = 0; base < count; base += kXIt * kNT) {
        cx<R> A[kXIt], B[kXIt], C[kXIt], W[kXIt];
        const int wave0 = base + ((int)threadIdx.x & ~63);
#pragma unroll
        for (int i = 0; i < kXIt; ++i) {
            const int e = min(base + (int)threadIdx.x + i * kNT, count - 1);
            const int line = e >> lgq, t = e & ((1 << lgq) - 1);
            const int p = line / 3, c = line - 3 * p;
            const cx<R>* row = Y1 + x_row(g, mb, c, pen0 + p);
            A[i] = row[t];
            B[i] = row[Lh - t];
            W[i] = tw_fwd<R>(t << twsh);
            C[i] = mk<R>((R)0, (R)0);
            // X[Lh/2] for item 0 of a line, loaded only by waves holding such an item
            if (lgq < 6 || ((wave0 + i * kNT) & ((1 << lgq) - 1)) == 0) C[i] = row[t == 0 ? (Lh >> 1) : t];
        }
#pragma unroll
        for (int i = 0; i < kXIt; ++i) {
            const int e = base + (int)threadIdx.x + i * kNT;
            if (e >= count) break;
            const int line = e >> lgq, t = e & ((1 << lgq) - 1);
            cx<R>* out = buf + line * Lh;
            if (t == 0) {
                out[0] = split(A[i], B[i], mk<R>((R)1, (R)0));
                if (Lh > 1) out[Lh >> 1] = split(C[i], C[i], mk<R>((R)0, (R)1));   // conj(W^(Lh/2)) = i
            } else {
                const cx<R> wc = cconj<R>(W[i]);
                out[t] = split(A[i], B[i], wc);
                out[Lh - t] = split(B[i], A[i], mk<R>(-wc.x, wc.y));            // conj(W^(Lh-t)) = -W^t
            }
        }
    }
    }
    __syncthreads();
    auto none_load = [&](int, int) -> cx<R> { return mk<R>(0, 0); };
    auto none_store = [&](int, int, cx<R>) {};
    fft_io<R, true, pemax<BIG>(), true, true, kLines, 1, false, true, lgmax<pemax<BIG>()>(), kNT, true>(
        buf, g.lgLh, 0, npen * 3, none_load, none_store);
}

// Forward x pass: buf holds packed lines z[n] = x[2n] + i x[2n+1]; writes the
// Hx-column half spectrum of every line to X1.  Merge step: with P = Z[k],
// Q = Z[Lh-k], E = (P + Q*)/2, O = (P - Q*)/(2i) and T = W^k O,
// X[k] = E + T and X[Lh-k] = (E - T)*.
template <typename R, bool BIG>
__device__ void r2c_lines(cx<R>* buf, cx<R>* X1, const PG& g, int mb, int pen0, int npen) {
    const int Lh = g.Lh;
    const int lgq = g.lgLh > 0 ? g.lgLh - 1 : 0;
    const int twsh = kTwLog - g.lgPx;
    auto none_load = [&](int, int) -> cx<R> { return mk<R>(0, 0); };
    auto none_store = [&](int, int, cx<R>) {};
    tw_lds_fill<R>();   // pass twiddles (same values if c2r_lines filled them)
    __syncthreads();
    fft_io<R, false, pemax<BIG>(), true, true, kLines, 1, true, false, lgmax<pemax<BIG>()>(), kNT, true>(
        buf, g.lgLh, 0, npen * 3, none_load, none_store);
    const R half = (R)0.5;
    if ((1 << lgq) >= kNT) {
        // as in the split step: fixed items t = tid + k kNT of every line,
        // uniform row addresses
        auto lines = [&](auto ipl_c) {
            constexpr int IPL = decltype(ipl_c)::value;   // items per thread and line
            cx<R> W[IPL];
#pragma unroll
            for (int k = 0; k < IPL; ++k) W[k] = tw_fwd<R>(((int)threadIdx.x + k * kNT) << twsh);
            const int nl = npen * 3;
            for (int l = 0; l < nl; ++l) {
                const int p = l / 3, c = l - 3 * p;
                cx<R>* row = X1 + x_row(g, mb, c, pen0 + p);
                const cx<R>* in = buf + l * Lh;
#pragma unroll
                for (int k = 0; k < IPL; ++k) {
                    const int t = (int)threadIdx.x + k * kNT;
                    if (t == 0) {
                        const cx<R> P = in[0];
                        row[0] = mk<R>(P.x + P.y, (R)0);
                        row[Lh] = mk<R>(P.x - P.y, (R)0);
                        row[Lh >> 1] = cconj<R>(in[Lh >> 1]);   // W^(Lh/2) = -i
                    } else {
                        const cx<R> P = in[t], Q = in[Lh - t];
                        const cx<R> E = mk<R>(half * (P.x + Q.x), half * (P.y - Q.y));
                        const cx<R> O = mk<R>(half * (P.y + Q.y), half * (Q.x - P.x));
                        const cx<R> T = cmul<R>(W[k], O);
                        row[t] = cadd<R>(E, T);
                        row[Lh - t] = mk<R>(E.x - T.x, T.y - E.y);
                    }
                }
            }
        };
        if ((1 << lgq) == kNT) lines(IntC<1>{});
        else if ((1 << lgq) == 2 * kNT) lines(IntC<2>{});
        else lines(IntC<4>{});
        return;
    }
    const int count = (npen * 3) << lgq;
    for (int base = 0; base < count; base += kXIt * kNT) {
        cx<R> W[kXIt];
#pragma unroll
        for (int i = 0; i < kXIt; ++i) {
            const int e = min(base + (int)threadIdx.x + i * kNT, count - 1);
            W[i] = tw_fwd<R>((e & ((1 << lgq) - 1)) << twsh);
        }
#pragma unroll
        for (int i = 0; i < kXIt; ++i) {
            const int e = base + (int)threadIdx.x + i * kNT;
            if (e >= count) break;
            const int line = e >> lgq, t = e & ((1 << lgq) - 1);
            const int p = line / 3, c = line - 3 * p;
            cx<R>* row = X1 + x_row(g, mb, c, pen0 + p);
            const cx<R>* in = buf + line * Lh;
            if (t == 0) {
                const cx<R> P = in[0];
                row[0] = mk<R>(P.x + P.y, (R)0);
                row[Lh] = mk<R>(P.x - P.y, (R)0);
                if (Lh > 1) row[Lh >> 1] = cconj<R>(in[Lh >> 1]);   // W^(Lh/2) = -i
            } else {
                const cx<R> P = in[t], Q = in[Lh - t];
                const cx<R> E = mk<R>(half * (P.x + Q.x), half * (P.y - Q.y));
                const cx<R> O = mk<R>(half * (P.y + Q.y), half * (Q.x - P.x));
                const cx<R> T = cmul<R>(W[i], O);
                row[t] = cadd<R>(E, T);
                row[Lh - t] = mk<R>(E.x - T.x, T.y - E.y);
            }
        }
    }
}

template <typename R>
__device__ __forceinline__ R demag_at(const cx<R>* buf, int line, int Lh, int n, int h) {
    const cx<R> v = buf[line * Lh + n];
    return h ? v.y : v.x;
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = kNT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}


}  // namespace magx
