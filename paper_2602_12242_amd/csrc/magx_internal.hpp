// Internal plan and launch interface of the magx library.
#pragma once

#include "magx_common.hpp"

namespace magx {

// Geometry and buffer layout of one grid, derived on the host.
//
// Extended grid (Section II-B): P_a = smallest power of two >= 2 n_a (the
// convolution is exact for any P_a >= 2 n_a - 1).  x is transformed real to
// complex, so spectral rows hold Hx = Px/2 + 1 columns, stored with a row
// stride Sx rounded up to 16 columns.
//
// Spectral intermediates (complex, x fastest):
//   X1 [3][nz][ny][Sx]   after the forward x pass; reused for the inverse-y output
//   X2 [3][nz][Py][Sx]   after the forward y pass; the z pass works in place
// Tensor spectrum (real), in the z pass's tile order: [Hy][ntz][6][Hz][tz],
// Hy = Py/2+1, Hz = Pz/2+1, ntz = ceil(Hx/tz) column tiles of tz values; the
// mirrored halves are read with the parity sign of each component.
struct Plan {
    magx_dtype dtype;
    int esize;                  // 4 or 8
    int nx, ny, nz;
    double dx, dy, dz;
    int Px, Py, Pz, lgPx, lgPy, lgPz;
    int Lh, lgLh;               // Px/2: length of the half-size complex FFT of the x pass
    int Hx, Hy, Hz, Sx;
    long long ncell;            // cells of one member
    int nbatch;                 // independent systems sharing the tensor spectrum
    int blocks_per_member;      // pencil blocks of one member
    int pencil_zmajor;          // pencil blocks ordered (y group, z) with z fastest
    // tensor build scratch (doubles): slab A = max(octant, y-pass output), then slab B
    long long scratch_a_elems, scratch_b_elems;
    // column tiles of the y and z passes, pencils per block of the x passes
    int ty, tz, np;
    int ntz;                    // column tiles of the z pass (and of the tensor spectrum)
    int zreg;                   // z pass held in registers (Pz = 8 ... 128 single, 16 ... 128 double precision)
    int yzfilm, yzt;            // films (nz = 1): the y and z passes fused into one kernel on yzt-column tiles
    // packed Nyquist column (single-precision register z pass with Pz = 16 ... 64,
    // Py = 32 ... 1024, Lh >= tz): X2's column Lh is stored in the padding
    // columns in groups of 16 row pairs, and the spectrum carries a copy of the
    // tensor's column Lh at element tn_off as ceil(Hy'/tz) + 1 blocks
    // [6][Hz][tz] (Hy' = Py/2) whose column c of block b holds row q = b tz + c;
    // the last block repeats block 0 with row Py/2 in column 0
    int nyqpack;
    long long tn_off;
    int pencil_blocks;
    // workspace layout (bytes): the non-finite flag word first, then X1, X2,
    // five fields and the per-block partials
    size_t off_flag, off_x1, off_x2, off_f[5], off_part, ws_bytes;
    size_t field_bytes;
    size_t tape_step_bytes, tape_extra_bytes;
    size_t spectrum_bytes, scratch_bytes;
};

int make_plan(const magx_grid* g, magx_dtype dt, int nbatch, Plan* pl);

// Physical constants prepared for the kernels (element type R).
template <typename R>
struct Phys {
    R Ms;            // demag: H = -Ms * N * m (applied in the z pass)
    R cex;           // 2A/(mu0 Ms) (Eq. (7) with M = Ms m)
    R cdmi;          // 2D/(mu0 Ms) (Eq. (9))
    R kap;           // -D/(2A): boundary condition Eq. (10), 0 without DMI
    R cani;          // 2Ku/(mu0 Ms) (Eq. (5))
    R eK[3];
    R hb[3];         // bias field (Zeeman)
    const R* hbm;    // optional per-member bias fields (nbatch x 3, device); overrides hb
    const R* msp;    // optional magnetisation profile s = Ms(r)/Ms per cell (device, shared by members)
    R a;             // mu0 gamma/(1+alpha^2) (Eq. (1))
    R alpha;
    R idx2, idy2, idz2;   // 1/d^2
    R h2x, h2y;           // 1/(2 d) for the DMI central differences
    R dx, dy;             // ghost offsets
    unsigned terms;
    int renorm;
    unsigned* nf;         // non-finite flag (device word, set to 1 by any wave that meets a
                          // non-finite output), or null when the call does not check
};

hipError_t launch_twiddle_init(hipStream_t s);
hipError_t build_tensor_spectrum(const Plan& pl, void* spectrum, void* scratch, hipStream_t s);

// FFT convolution passes (conv.hip)
template <typename R>
hipError_t launch_yfwd(const Plan& pl, const void* X1, void* X2, hipStream_t s);
template <typename R>
hipError_t launch_zconv(const Plan& pl, void* X2, const void* spec, R Ms, hipStream_t s);
template <typename R>
hipError_t launch_yinv(const Plan& pl, const void* X2, void* Y1, hipStream_t s);
// Films (plan.yzfilm): forward y pass, z pass and inverse y pass in one kernel, X1 -> Y1 in place.
template <typename R>
hipError_t launch_yzfilm(const Plan& pl, void* X1, const void* spec, R Ms, hipStream_t s);
// Diagnostic memory patterns over X2 (single precision plans): 0 copy, 1 z tiling, 2 y tiling.
hipError_t launch_memory_probe(const Plan& pl, int kind, void* X2, hipStream_t s, double* bytes);

// Pencil kernels (pencil.hip): x passes fused with the local field, LLG and RK4.
template <typename R>
struct StageArgs {
    const R* yin;      // stage input y_s (halo reads)
    const R* mn;       // state m_n at the start of the step
    R* acc;            // running sum of b_s k_s
    R* yout;           // next stage input y_{s+1} (or m_{n+1} at s = 4)
    R* yout2;          // optional extra copy of y_{s+1} (tape)
    R* tapeH;          // optional: field H_s
    R* tapeNx;         // optional: |x_{s+1}| before normalisation
    R* tapeYin;        // optional: copy of y_s
    int stage;         // 1..4, or 0 for a forward Euler step
    R dt;
    int want_next;     // 1: forward x pass of y_{s+1} into X1
};

template <typename R>
struct BackArgs {
    const R* mu;       // mu_s (halo reads) -- cotangent of H at stage s
    const R* ys;       // y_s
    const R* Hs;       // H_s
    R* kap;            // kappa_s in, kappa_{s-1} out (pointwise)
    const R* xi5;      // xi_5
    const R* nxs;      // |x_s| (s >= 2)
    const R* yprev;    // y_{s-1} (s >= 2)
    R* gm;             // lambda, accumulated
    R* muout;          // mu_{s-1}
    int stage;
    R dt;
};

template <typename R>
struct StartArgs {
    R* gm;             // in: cotangent of m_{n+1}; out: xi_5
    const R* y5;       // m_{n+1}
    const R* nx5;      // |x_5|
    const R* y4;
    R* xi5;
    R* kap;            // kappa_4
    R* muout;          // mu_4
    R dt;
};

template <typename R>
hipError_t launch_xfwd(const Plan& pl, const R* f, void* X1, const R* msp, hipStream_t s);
// mode 0: H = field of f (with bias if with_bias); mode 1: energy partials of f;
// if sum_input, per-block sums of f are added into partials (for dL/dH_bias).
template <typename R>
hipError_t launch_field(const Plan& pl, const Phys<R>& ph, const void* Y1, const R* f, R* H, int with_bias,
                        int energy, int sum_input, double* partials, hipStream_t s);
template <typename R>
hipError_t launch_stage(const Plan& pl, const Phys<R>& ph, const void* Y1, void* X1, const StageArgs<R>& a,
                        hipStream_t s);
template <typename R>
hipError_t launch_bstage(const Plan& pl, const Phys<R>& ph, const void* Y1, void* X1, const BackArgs<R>& a,
                         double* partials, hipStream_t s);
template <typename R>
hipError_t launch_bstart(const Plan& pl, const Phys<R>& ph, void* X1, const StartArgs<R>& a, double* partials,
                         hipStream_t s);
template <typename R>
hipError_t launch_rhs(const Plan& pl, const Phys<R>& ph, const R* m, const R* H, R* out, hipStream_t s);
hipError_t launch_fill_zero(double* p, long long n, hipStream_t s);
// Per member b: out[b*nval + c] (+)= sum over its blocks of partials[lb*8 + c]
// (logical block index lb, members own contiguous ranges), fixed order.
template <typename R>
hipError_t launch_reduce_partials(const double* partials, int nbatch, int blocks_per_member, int nval, R* out,
                                  int accumulate, hipStream_t s);
// vku_cell = V Ku per magnetic cell; their count is partial 5 of every block.
hipError_t launch_energy_finish(const double* partials, int nbatch, int blocks_per_member, double pref,
                                double vku_cell, double* e_out, hipStream_t s);
template <typename R>
hipError_t launch_copy(const R* src, R* dst, long long n, hipStream_t s);

// Multirate kernels (mri.hip)
template <typename R>
hipError_t launch_mri_slow(const Plan& pl, const Phys<R>& ph, const void* Y1, const R* y, int has_demag, R* S_out,
                           const R* Sa, const R* Sb, R wa, R wb, R wn, R* r_out, hipStream_t s);
template <typename R>
hipError_t launch_mri_fast(const Plan& pl, const Phys<R>& ph, const R* v, R* vout, R* q, const R* r, R Ak, R Bk,
                           R h, int first, int norm, void* X1, hipStream_t s);

}  // namespace magx
