/*
 * magx -- effective field and LLG time stepping on a uniform cell grid, on one
 * AMD Instinct MI355X (gfx950).  C ABI.
 *
 * The operations follow the paper's problem statement (Section II-A/II-B,
 * Eqs. (1)-(10)):
 *   H_eff = H_bias + H_demag + H_ani + H_exch + H_DMI                 Eq. (2)
 *   dm/dt = mu0 gamma_L [m x H_eff + alpha m x (m x H_eff)]           Eq. (1), M = Ms m
 * with the demagnetising field evaluated as a zero-padded FFT convolution
 * with a cell-averaged demag tensor (Section II-B, Eq. (3)), second-order
 * central differences for exchange and DMI with the DMI boundary condition of
 * Eq. (10), classical RK4 (Section III-C) and per-cell renormalisation of |m|
 * after every stage and step (Section II-B).  The reverse mode (gradients of a
 * scalar loss with respect to the initial m and to H_bias) is not in the
 * paper; it is the exact adjoint of the forward algorithm.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Vector fields (m, H, dm/dt, gradients) are contiguous arrays of the
 *    context's element type (float for MAGX_F32, double for MAGX_F64) laid out
 *    (3, nz, ny, nx): component-major, then z, then y, with x fastest.
 *  - A context made by magx_tensor_init_batched with nbatch = B advances B
 *    independent systems of the same grid that share one tensor spectrum
 *    (an ensemble of initial states or bias fields).  Every vector field is
 *    then (B, 3, nz, ny, nx), every per-system output (energies, gHbias)
 *    holds B consecutive records, and every size magx_sizes_batched reports
 *    covers the whole batch.  Member b's results equal those of a B = 1
 *    context run on member b alone, bit for bit.
 *  - All pointers named "device" point to memory on the context's GPU, owned
 *    by the caller.  The library never allocates or frees device memory; the
 *    sizes it needs are reported by magx_sizes().
 *  - `stream` is a hipStream_t (NULL = default stream).  Calls only enqueue
 *    work on that stream and return; they do not synchronise.
 *  - Return value: MAGX_OK (0) or a negative MAGX_E* code.  Arguments are
 *    validated before any HIP call; on an argument error nothing is enqueued.
 *    MAGX_EHIP means a HIP launch or copy reported an error; the stream's
 *    state is then undefined.
 *  - Overlapping calls on one context from several host threads are not
 *    supported (the context holds no device state other than what the caller
 *    passes in, but its evaluation counter is not atomic).
 */
#ifndef MAGX_H
#define MAGX_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes -------------------------------------------------------- */
#define MAGX_OK          0
#define MAGX_EINVAL     -1   /* null pointer, non-positive size or spacing, bad flag, DMI without exchange */
#define MAGX_ESIZE      -2   /* n > 4096 on an axis, or an extended-grid length P = next power of two
                                >= 2n exceeds the FFT passes' limits: Py <= 4096; Px <= 4096 (float)
                                or 2048 (double); Pz <= 1024 */
#define MAGX_EDTYPE     -3   /* unknown element type */
#define MAGX_EWORKSPACE -4   /* magx_step_static: the grid needs more than its fixed workspace;
                                elsewhere buffer sizes are the caller's contract (see magx_sizes) */
#define MAGX_EHIP       -5   /* a HIP call failed */
#define MAGX_ENONFINITE -6   /* magx_status: a checked call produced a NaN or infinite value */
#define MAGX_ESTATE     -7   /* reverse mode or checkpointed rollout asked for while a bias schedule is set */

/* ---- field terms (bit mask), Eq. (2) -------------------------------------- */
#define MAGX_DEMAG   1u   /* Eq. (3): demagnetising field                    */
#define MAGX_EXCH    2u   /* Eq. (7): exchange, uniform A                    */
#define MAGX_DMI     4u   /* Eq. (9) with the boundary condition Eq. (10)    */
#define MAGX_ANIS    8u   /* Eq. (5): uniaxial anisotropy                    */
#define MAGX_ZEEMAN 16u   /* uniform bias field H_bias                       */

typedef enum { MAGX_F32 = 0, MAGX_F64 = 1 } magx_dtype;

/* Cell grid (Section II-B): nx*ny*nz cells of dx*dy*dz metres, cell-centred. */
typedef struct {
    int nx, ny, nz;
    double dx, dy, dz;
} magx_grid;

/* Material and physics constants, SI units (Section II-A).
 *   Ms     saturation magnetisation, A/m (> 0)
 *   A      exchange constant, J/m (>= 0; > 0 when MAGX_DMI is set)
 *   D      interfacial DMI constant, J/m^2, used with the sign of Eq. (9)
 *   Ku     uniaxial anisotropy constant, J/m^3, easy axis eK (unit vector)
 *   Hbias  uniform bias field, A/m
 *   alpha  Gilbert damping; gamma gyromagnetic ratio (the paper's -1.759e11);
 *   mu0    vacuum permeability (4 pi 1e-7)
 *   terms  bit mask of MAGX_* field terms
 *   renorm 0: never renormalise; 1: renormalise the new state only;
 *          2: renormalise every RK stage input and the new state (default)
 *   check_finite  0 or 1.  With 1, the call clears a flag word at the start of
 *          its workspace and every kernel that writes a field, a state or a
 *          gradient sets it when one of its outputs is NaN or infinite
 *          (renormalisation keeps |m| = 1, so a non-finite value means the
 *          step size or the input was unusable); magx_status reads it.  The
 *          computation itself is unchanged.  magx_llg_rhs (no workspace)
 *          ignores the flag. */
typedef struct {
    double Ms, A, D, Ku;
    double eK[3];
    double Hbias[3];
    double alpha, gamma, mu0;
    unsigned terms;
    int renorm;
    int check_finite;
} magx_params;

/* Buffer sizes in bytes for a grid and element type. */
typedef struct {
    size_t spectrum_bytes;      /* demag tensor spectrum (persistent, magx_tensor_init) */
    size_t init_scratch_bytes;  /* scratch used only during magx_tensor_init            */
    size_t workspace_bytes;     /* workspace of every other call                          */
    size_t tape_bytes_per_step; /* per recorded RK4 step (magx_step with a tape)          */
    size_t tape_bytes_extra;    /* plus this once per tape                                */
    size_t field_bytes;         /* one vector field: 3*nx*ny*nz elements                  */
} magx_size_info;

typedef struct magx_ctx magx_ctx;

/* Sizes of every buffer for grid g and element type dt.  Host only. */
int magx_sizes(const magx_grid* g, magx_dtype dt, magx_size_info* out);
/* The same for a batch of nbatch >= 1 systems (spectrum and init scratch do
 * not grow with nbatch; fields, workspace and tape do).  MAGX_ESIZE if
 * nbatch > 65535 or the batch's fields or spectral intermediates reach 2^31
 * elements. */
int magx_sizes_batched(const magx_grid* g, magx_dtype dt, int nbatch, magx_size_info* out);

/* Creates a context and builds the demag tensor spectrum (Section II-B: the
 * real-space tensor on the extended grid of twice the problem size, then its
 * discrete Fourier transform).  The tensor is evaluated in double precision
 * (cell-averaged Newell closed forms near the source cell, Gauss-Legendre
 * quadrature of the dipole kernel against the cell-cell autocorrelation
 * elsewhere), transformed in double precision and, for MAGX_F32, rounded once
 * to float.  `spectrum` (device, spectrum_bytes, 16-byte aligned as every
 * device allocation is; MAGX_EINVAL otherwise) is kept by the context and
 * must stay valid until magx_destroy; `scratch` (device, init_scratch_bytes)
 * is free again when the stream reaches the end of this call's work.
 * On success *ctx is set; on failure *ctx is NULL. */
int magx_tensor_init(magx_ctx** ctx, const magx_grid* g, magx_dtype dt,
                     void* spectrum, void* scratch, void* stream);
/* As magx_tensor_init, for a batch of nbatch >= 1 systems of grid g. */
int magx_tensor_init_batched(magx_ctx** ctx, const magx_grid* g, magx_dtype dt, int nbatch,
                             void* spectrum, void* scratch, void* stream);

/* Per-system bias fields: hbias (device, nbatch x 3 elements of the context
 * type, A/m, owned by the caller and kept valid while in use) replaces
 * p->Hbias for member b by hbias[3b..3b+2] in every later call; NULL goes
 * back to p->Hbias for all members.  Host only; enqueues nothing. */
int magx_set_member_bias(magx_ctx* ctx, const void* hbias);
/* Number of systems of a context (host), -1 for NULL. */
int magx_ctx_batch(const magx_ctx* ctx);

/* Geometry and space-dependent saturation magnetisation: s (device, nx*ny*nz
 * elements of the context type, layout (nz, ny, nx), owned by the caller and
 * kept valid while in use, shared by all members of a batch) gives
 * Ms(r) = p->Ms * s(r) with s >= 0; s = 0 marks cells outside the magnet
 * (nanodots, patterned films).  The demagnetising field is then that of
 * M = Ms(r) m (Eq. (3)); exchange, DMI and anisotropy use each cell's own
 * Ms in their prefactors (Eqs. (5), (7), (9)); the surface of the magnet is a
 * boundary like the faces of the grid (ghost of Eq. (10) in place of a
 * neighbour outside the magnet); cells outside the magnet carry no field and
 * do not move; energies weight each cell by its Ms.  The reverse mode and the
 * checkpointed rollouts return MAGX_ESTATE while a profile is set.  NULL
 * returns to a uniform Ms.  Host only; enqueues nothing. */
int magx_set_ms_profile(magx_ctx* ctx, const void* s);

/* Effective field, Eq. (2), of the unit field m (device, read) into H (device,
 * written), in A/m.  `ws`: device workspace of workspace_bytes. */
int magx_heff(magx_ctx* ctx, const void* m, const magx_params* p, void* H,
              void* ws, void* stream);

/* Right-hand side of Eq. (1) for unit m: dmdt = mu0 gamma_L [m x H + alpha
 * m x (m x H)], gamma_L = gamma/(1+alpha^2), from m and a given field H
 * (device, read).  Pointwise; dmdt must not overlap m or H. */
int magx_llg_rhs(magx_ctx* ctx, const void* m, const void* H,
                 const magx_params* p, void* dmdt, void* stream);

/* Advances m (device, read and written in place) by nsteps classical RK4
 * steps of size dt (Section III-C: four right-hand-side evaluations per
 * step), renormalising per p->renorm.  If `tape` is not NULL (device,
 * nsteps*tape_bytes_per_step + tape_bytes_extra) every stage input, stage
 * field and pre-normalisation length is recorded for magx_step_backward.
 * On grids of at most 2^18 cells (whole batch), without a tape, a bias
 * schedule or active launch timing, the steps are replayed from HIP graphs
 * the context captures per argument signature (m, ws, p, dt, chunk of up to
 * 16 steps; at most 8 kept, released by magx_destroy); the results are the
 * same bit for bit. */
int magx_step(magx_ctx* ctx, void* m, const magx_params* p, double dt, int nsteps,
              void* tape, void* ws, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): magx_step
 * without a tape and without a caller workspace.  Its workspace is a 64 MiB
 * array in device memory that the library holds on each GPU it runs on until
 * the process ends (enough for a single-precision 256 x 256 x 8 grid or a
 * double-precision 256 x 128 x 8 one); MAGX_EWORKSPACE if the context's grid
 * and batch need more, checked before any HIP call.  Nothing is allocated:
 * no hipMalloc, hipFree or allocating library routine.  All calls on one GPU
 * share that array: calls that overlap on one GPU (concurrent streams or host
 * threads) race and must be serialised by the caller; each call writes every
 * part of it before reading it.  With check_finite the flag word is in that
 * array too, so magx_status must be called before the next call on the GPU
 * that uses it. */
int magx_step_static(magx_ctx* ctx, void* m, const magx_params* p, double dt, int nsteps, void* stream);

/* Advances m (device, in place) by nsteps forward Euler steps
 * m <- m + dt R(m) (the integrator of the paper's scaling runs, Section III-E),
 * one field evaluation per step, renormalising the new state when
 * p->renorm >= 1.  ws: workspace of workspace_bytes. */
int magx_step_euler(magx_ctx* ctx, void* m, const magx_params* p, double dt, int nsteps,
                    void* ws, void* stream);

/* Time-dependent uniform bias field.  times (host, n strictly increasing
 * values, s) and values (host, n x 3, A/m) are knots of a piecewise-linear
 * H_bias(t), held constant before the first and after the last knot; the
 * context copies them.  t0 sets the context's clock.  While a schedule is set
 * it replaces p->Hbias: magx_heff and magx_energy use H_bias(clock), every
 * stage of magx_step, magx_step_euler and magx_step_mri uses the bias at its
 * own stage time, and those calls advance the clock by nsteps*dt.  A
 * per-member bias table (magx_set_member_bias) takes precedence.  The reverse
 * mode and the checkpointed rollouts return MAGX_ESTATE while a schedule is
 * set (their gradient is with respect to a constant bias).  n = 0 removes
 * the schedule (times and values may then be NULL).  Host only. */
int magx_set_bias_schedule(magx_ctx* ctx, int n, const double* times, const double* values,
                           double t0);
/* The context's clock (s), see magx_set_bias_schedule.  Host only. */
int magx_get_time(const magx_ctx* ctx, double* t);

/* Advances m (device, in place) by nsteps explicit-explicit multirate steps
 * of size dt (Section III-C, integrator comparison): the LLG torque of the
 * exchange field is the fast partition, that of every other enabled term
 * the slow one (Eq. (1) is linear in H, so the two add up to the full
 * right-hand side).  Both scales use the three-stage third-order method of
 * Knoth and Wolke in multirate-infinitesimal-step form: three slow torque
 * evaluations (one FFT convolution each) per step, and between them the fast
 * ODE with the slow forcing, in equal substeps no longer than dt_fast (the
 * paper uses dt/10: 4 + 5 + 3 substeps of 3 stages, 36 exchange evaluations
 * per step).  Renormalisation per p->renorm: 2 renormalises every slow
 * stage value and the new state, 1 the new state only.  ws: workspace of
 * workspace_bytes.  MAGX_EINVAL if dt < 0, dt_fast <= 0 or dt/dt_fast > 2^20. */
int magx_step_mri(magx_ctx* ctx, void* m, const magx_params* p, double dt, double dt_fast,
                  int nsteps, void* ws, void* stream);

/* Reverse mode of the linear part of the field: for a cotangent gH of H_eff
 * (device, read), gm = K^T gH = K gH, where H_eff(m) = K m + H_bias (K is
 * symmetric: the demag tensor is, and the ghost-cell DMI boundary condition
 * makes exchange + DMI symmetric), and gHbias[0..2] = sum over cells of gH
 * (device, 3 elements of the context type) when MAGX_ZEEMAN is set, else 0.
 * gm and gHbias are overwritten. */
int magx_heff_backward(magx_ctx* ctx, const void* gH, const magx_params* p,
                       void* gm, void* gHbias, void* ws, void* stream);

/* Reverse of magx_step over the same nsteps, from the tape it recorded with
 * the same p and dt.  On entry gm (device) holds the cotangent of the final
 * state; on return, that of the initial state.  gHbias (device, 3 elements)
 * is incremented by the gradient with respect to H_bias. */
int magx_step_backward(magx_ctx* ctx, const void* tape, int nsteps,
                       const magx_params* p, double dt, void* gm, void* gHbias,
                       void* ws, void* stream);

/* Checkpointed rollout.  Forward: advances m by nsteps, storing the state at
 * every multiple of `ckpt` steps (the start of each segment) in ckpt_store
 * (device, ceil(nsteps/ckpt) fields).  Backward: walks the segments in
 * reverse, re-running each with a tape (device, ckpt steps of tape) and
 * reversing it; gm is the cotangent of the final state on entry and of the
 * initial state on return; gHbias (device, 3) is overwritten with dL/dH_bias.
 * `mwork` (device, one field) is scratch for the re-run segment. */
int magx_rollout_forward(magx_ctx* ctx, void* m, const magx_params* p, double dt,
                         int nsteps, int ckpt, void* ckpt_store, void* ws, void* stream);
int magx_rollout_backward(magx_ctx* ctx, const void* ckpt_store, const magx_params* p,
                          double dt, int nsteps, int ckpt, void* gm, void* gHbias,
                          void* tape, void* mwork, void* ws, void* stream);

/* Energies in joules of state m, written as 6 doubles to e_out (device):
 * demag, exchange, DMI, anisotropy, Zeeman, total.  Densities of Eqs. (4),
 * (6), (8), the DMI density whose variational derivative is Eq. (9), and
 * -mu0 Ms m.H_bias, summed over cells times the cell volume.  Eq. (4) is used
 * as -(mu0 Ms/2) m.H_demag. */
int magx_energy(magx_ctx* ctx, const void* m, const magx_params* p, void* e_out,
                void* ws, void* stream);

/* Outcome of the last call on ctx made with check_finite = 1: waits for the
 * stream of that call, then returns MAGX_ENONFINITE if one of its kernels met
 * a NaN or infinite output, MAGX_OK if none did (or if no call on ctx has
 * asked for the check yet), MAGX_EHIP if the wait or the read failed, and
 * MAGX_EINVAL for a NULL ctx.  The workspace of that call must still be
 * allocated.  A checked call clears the flag at its start, so the outcome
 * belongs to that call alone; a checkpointed rollout counts as one call.
 * Non-finite values propagate through every later step and stage, so
 * checking the last call of a sequence covers the sequence. */
int magx_status(magx_ctx* ctx);

/* Number of effective-field evaluations (FFT convolutions of a state)
 * enqueued through this context so far. */
long long magx_heff_count(const magx_ctx* ctx);

/* Grid and type of a context (host). */
int magx_ctx_info(const magx_ctx* ctx, magx_grid* g, magx_dtype* dt);

/* Diagnostics: layout of the stored tensor spectrum, dims[0..4] = (Hy, ntz,
 * 6, Hz, tz): element (c, kz, ky, kx) of the real octant of the tensor
 * spectrum (c = xx yy zz xy xz yz, already scaled by 1/(Px Py Pz)) is at
 * (((ky * ntz + kx / tz) * 6 + c) * Hz + kz) * tz + kx % tz; Hy = Py/2 + 1,
 * Hz = Pz/2 + 1, kx < Px/2 + 1 <= ntz * tz.  Host only. */
int magx_spectrum_layout(const magx_ctx* ctx, int dims[5]);

/* Diagnostics: from magx_profile_start until magx_profile_stop, every launch
 * of one kernel family enqueued through ctx is bracketed by a pair of HIP
 * events on its stream.  kind: 0 none, 1 forward x pass, 2 forward y pass,
 * 3 z pass with the spectral product, 4 inverse y pass, 5 RK4 stage (inverse
 * x pass + local field + LLG + stage update + next forward x pass), 6 field
 * output (inverse x pass + local field), 7 reverse-step start, 8 reverse RK4
 * stage.  magx_profile_stop waits for the recorded events and returns the
 * number of timed launches and their summed duration in milliseconds. */
int magx_profile_start(magx_ctx* ctx, int kind);
int magx_profile_stop(magx_ctx* ctx, long long* launches, double* total_ms);

/* Diagnostics: enqueues one pass of a plain memory pattern, with no
 * arithmetic, over the X2 region of the workspace ws (its contents are
 * overwritten): kind 0 copies its first half onto its second half as float4;
 * kind 1 reads and writes it in place with the z pass's tiling (tiles of 32
 * columns, every row z < nz of the three components, rows one plane apart);
 * kind 2 reads and writes it in place with the y pass's tiling (16 columns x
 * all Py rows of one plane).  *bytes receives the bytes read plus written.
 * The time of such a pass is the practical bandwidth of that pattern on
 * this device.  Single-precision contexts only (MAGX_EDTYPE otherwise). */
int magx_memory_probe(magx_ctx* ctx, int kind, void* ws, void* stream, double* bytes);

const char* magx_strerror(int code);
void magx_destroy(magx_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* MAGX_H */
