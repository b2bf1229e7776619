// C ABI of the magx library: argument validation, planning, buffer layout and
// launch sequencing on the caller's stream.  Every numeric step runs in the
// HIP kernels of tensor.hip, conv.hip and pencil.hip.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "magx_internal.hpp"

using namespace magx;

struct magx_ctx {
    Plan pl;
    void* spectrum;
    const void* hbias_members;   // optional per-member bias fields (device, nbatch x 3)
    const void* ms_profile;      // optional s = Ms(r)/Ms per cell (device, ncell), 0 outside the magnet
    // time-dependent uniform bias: knots (host) and the context's clock
    std::vector<double> sched_t, sched_h;
    double time;
    long long heff_count;
    int device;
    // non-finite check: flag word of the last call made with check_finite = 1
    // (in that call's workspace) and its stream; chk_hold keeps the flag of
    // a compound call (checkpointed rollout) armed across its inner calls
    unsigned* chk_flag;
    hipStream_t chk_stream;
    int chk_hold;
    // launch timing of one kernel family (diagnostics)
    int prof_kind;
    size_t prof_used;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_events;
    // RK4 step sequences of small grids replayed as HIP graphs: one
    // instantiated graph per argument signature, captured on a private stream
    struct StepGraph {
        void* m;
        void* ws;
        magx_params p;
        double dt;
        int nsteps;
        const void* hbm;
        const void* msp;
        hipGraphExec_t exec;
        hipStream_t last;        // stream of the last replay
        long long heff;          // field evaluations per replay
    };
    std::vector<StepGraph> graphs;
    hipStream_t cap_stream;
};

namespace magx {

enum ProfKind { kProfXfwd = 1, kProfYfwd, kProfZconv, kProfYinv, kProfStage, kProfField, kProfBstart, kProfBstage };

// Records a HIP event pair around one launch when its family is being timed.
struct ProfScope {
    magx_ctx* c;
    hipStream_t s;
    hipEvent_t stop = nullptr;
    ProfScope(magx_ctx* ctx, int kind, hipStream_t st) : c(ctx), s(st) {
        if (!c || c->prof_kind != kind) return;
        if (c->prof_used == c->prof_events.size()) {
            hipEvent_t a, b;
            if (hipEventCreate(&a) != hipSuccess) return;
            if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); return; }
            c->prof_events.emplace_back(a, b);
        }
        auto& ev = c->prof_events[c->prof_used++];
        (void)hipEventRecord(ev.first, s);
        stop = ev.second;
    }
    ~ProfScope() {
        if (stop) (void)hipEventRecord(stop, s);
    }
};

}  // namespace magx

namespace magx {

static int next_pow2_at_least(long long v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

static size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

static int pow2_floor(long long v) {
    int p = 1;
    while ((long long)p * 2 <= v) p <<= 1;
    return p;
}

int make_plan(const magx_grid* g, magx_dtype dt, int nbatch, Plan* pl) {
    if (!g || !pl || nbatch < 1) return MAGX_EINVAL;
    if (dt != MAGX_F32 && dt != MAGX_F64) return MAGX_EDTYPE;
    if (g->nx < 1 || g->ny < 1 || g->nz < 1) return MAGX_EINVAL;
    if (!(g->dx > 0.0) || !(g->dy > 0.0) || !(g->dz > 0.0) || !std::isfinite(g->dx) || !std::isfinite(g->dy) ||
        !std::isfinite(g->dz))
        return MAGX_EINVAL;
    Plan p{};
    p.dtype = dt;
    p.esize = dt == MAGX_F32 ? 4 : 8;
    p.nx = g->nx; p.ny = g->ny; p.nz = g->nz;
    p.dx = g->dx; p.dy = g->dy; p.dz = g->dz;
    if (g->nx > 4096 || g->ny > 4096 || g->nz > 4096) return MAGX_ESIZE;
    p.Px = next_pow2_at_least(std::max(2, 2 * g->nx));
    p.Py = next_pow2_at_least(std::max(2, 2 * g->ny));
    p.Pz = next_pow2_at_least(std::max(2, 2 * g->nz));
    // LDS budgets of the passes (64 KiB per block): x lines 3*Lh, y columns
    // Py*ty, z columns 3*Pz*tz complex values
    const int lds_cplx = dt == MAGX_F32 ? 8192 : 4096;
    if (p.Py > 4096 || 3 * (p.Px / 2) > lds_cplx || 3 * p.Pz > lds_cplx) return MAGX_ESIZE;
    p.lgPx = ilog2(p.Px); p.lgPy = ilog2(p.Py); p.lgPz = ilog2(p.Pz);
    p.Lh = p.Px / 2; p.lgLh = p.lgPx - 1;
    p.Hx = p.Lh + 1; p.Hy = p.Py / 2 + 1; p.Hz = p.Pz / 2 + 1;
    p.Sx = (p.Hx + 15) / 16 * 16;
    // 32-bit element offsets inside the spectral arrays (whole batch), 24-bit row strides
    p.nbatch = nbatch;
    if (3LL * nbatch * p.nz * p.Py * p.Sx >= (1LL << 31) || (long long)p.Py * p.Sx >= (1LL << 23) ||
        6LL * p.Hz * p.Hy * p.Sx >= (1LL << 31))
        return MAGX_ESIZE;
    p.ncell = (long long)p.nx * p.ny * p.nz;
    if (3LL * nbatch * p.ncell >= (1LL << 31) || nbatch > 65535) return MAGX_ESIZE;
    // y tile: Py*ty complex in LDS, up to 128 KiB (one block of 512 threads
    // per CU; single precision: 16 columns = whole 128-byte row segments at
    // Py = 1024; double precision: 8 columns, 128 bytes); double precision
    // with Py <= 512 keeps 64 KiB tiles (256 threads)
    const int y_cplx = dt == MAGX_F32 ? 16384 : (p.Py <= 512 ? 4096 : 8192);
    p.ty = std::min(16, pow2_floor(y_cplx / p.Py));
    // z tile: data 3*Pz*tz complex in LDS (at most 64 KiB), at most 16 FFT
    // elements per thread when possible (32 at most), and at most 4 tensor
    // items (kz <= Pz/2, column) per thread: (Pz/2+1)*tz <= 4*256
    {
        const long long per_col = (long long)p.esize * 6LL * p.Pz;
        auto fits = [&](long long t, long long emax) {
            return 3LL * p.Pz * t <= (long long)kNT * emax && per_col * t <= 65536 &&
                   (long long)(p.Pz / 2 + 1) * t <= 4LL * kNT;
        };
        int tz = 64;
        while (tz > 1 && !fits(tz, 16)) tz >>= 1;
        if (!fits(tz, 32)) return MAGX_ESIZE;
        // register-resident z passes: single precision with Pz = 8 ... 128 (Pz/8 T threads per
        // T-column tile; T = 32, 64 for Pz = 8 so a block has at least 64 threads, 16 for
        // Pz = 128), double precision with Pz = 16 ... 128 (Pz/4 threads per column,
        // T = 1024/Pz columns)
        if (dt == MAGX_F32) {
            p.zreg = (p.Pz >= 8 && p.Pz <= 128) ? 1 : 0;
            if (p.zreg) tz = p.Pz == 8 ? 64 : (p.Pz == 128 ? 16 : 32);
        } else {
            p.zreg = (p.Pz >= 16 && p.Pz <= 128) ? 1 : 0;
            if (p.zreg) tz = 1024 / p.Pz;
        }
        p.tz = tz;
        p.ntz = (p.Hx + tz - 1) / tz;
        if ((long long)p.Hy * p.ntz * 6 * p.Hz * tz >= (1LL << 31)) return MAGX_ESIZE;
    }
    // films: y and z passes fused when a tile of 3 Py ty values with ty >= 8
    // columns (8 ... 16, whole 64- to 128-byte row segments) fits in 64 KiB;
    // on small films the tiles narrow (down to 4 columns) until there are 64
    // of them, since there the kernel's latency, not its traffic, counts
    if (p.nz == 1) {
        int t = 16;
        while (t >= 8 && 3LL * p.Py * t * 2 * p.esize > 65536) t >>= 1;
        if (t >= 8) {
            while (t > 4 && (p.Hx + t - 1) / t < 64) t >>= 1;
            p.yzfilm = 1;
            p.yzt = t;
        }
    }
    // pencils per block: up to 1024/Lh (one block holds 3 np lines of Lh
    // complex values); fewer on small grids, so that a member has at least
    // 1024 blocks in single precision (four per CU, within the five resident
    // at the stage kernel's registers) and 256 in double precision (whose
    // kernels hold fewer blocks per CU) when it has enough pencils: a block's
    // chain of memory round trips, not the traffic, bounds a small grid's
    // kernels.  Independent of the batch size: a member's block partition,
    // and so the order of its block sums, is the same in a batch as alone.
    const int npen = p.ny * p.nz;
    const int min_blocks = dt == MAGX_F32 ? 1024 : 256;
    p.np = std::max(1, 1024 / p.Lh);
    if (p.np > npen) p.np = npen;
    while (p.np > 1 && (npen + p.np - 1) / p.np < min_blocks) p.np >>= 1;
    // pencil blocks never straddle two members (the last one of a member may be
    // ragged); with ny >= np and nz > 1 a block holds np rows of one plane and
    // blocks run through z fastest
    p.pencil_zmajor = (p.ny >= p.np && p.nz > 1) ? 1 : 0;
    p.blocks_per_member = p.pencil_zmajor ? p.nz * ((p.ny + p.np - 1) / p.np) : (npen + p.np - 1) / p.np;
    p.pencil_blocks = nbatch * p.blocks_per_member;
    const size_t es = (size_t)p.esize;
    const long long N = p.ncell * nbatch;
    p.field_bytes = (size_t)3 * N * es;
    size_t off = 0;
    p.off_flag = off; off = 256;
    p.off_x1 = off; off = align256(off + (size_t)3 * nbatch * p.nz * p.ny * p.Sx * 2 * es);
    p.off_x2 = off; off = align256(off + (size_t)3 * nbatch * p.nz * p.Py * p.Sx * 2 * es);
    for (int i = 0; i < 5; ++i) { p.off_f[i] = off; off = align256(off + p.field_bytes); }
    p.off_part = off; off = align256(off + (size_t)p.pencil_blocks * 8 * sizeof(double));
    p.ws_bytes = off;
    p.tape_step_bytes = (size_t)28 * N * es;
    p.tape_extra_bytes = (size_t)3 * N * es;
    // (not at Pz = 8: its one-wave blocks come two units per pair on grids of
    // that depth, too few to balance a Nyquist unit against)
    p.nyqpack = (dt == MAGX_F32 && p.zreg && p.Pz >= 16 && p.Pz <= 64 && p.Py >= 32 && p.Py <= 1024 &&
                 p.Lh >= p.tz && p.Sx == p.Lh + 16) ? 1 : 0;
    p.tn_off = (long long)p.Hy * p.ntz * 6 * p.Hz * p.tz;
    const long long tn_blocks = p.nyqpack ? (p.Py / 2 + p.tz - 1) / p.tz + 1 : 0;
    p.spectrum_bytes = (size_t)(p.tn_off + tn_blocks * 6 * p.Hz * p.tz) * es;
    const long long a1 = 6 * p.ncell, a2 = 6LL * p.Hy * p.Hx * p.nz;
    p.scratch_a_elems = std::max(a1, a2);
    p.scratch_b_elems = 6LL * p.Hx * p.nz * p.ny;
    p.scratch_bytes = (size_t)(p.scratch_a_elems + p.scratch_b_elems) * sizeof(double);
    *pl = p;
    return MAGX_OK;
}

static int check_params(const magx_params* p) {
    if (!p) return MAGX_EINVAL;
    const double v[] = {p->Ms, p->A, p->D, p->Ku, p->eK[0], p->eK[1], p->eK[2], p->Hbias[0], p->Hbias[1],
                        p->Hbias[2], p->alpha, p->gamma, p->mu0};
    for (double x : v)
        if (!std::isfinite(x)) return MAGX_EINVAL;
    if (!(p->Ms > 0.0) || !(p->mu0 > 0.0) || p->alpha < 0.0 || p->A < 0.0) return MAGX_EINVAL;
    if (p->terms & ~31u) return MAGX_EINVAL;
    if (p->renorm < 0 || p->renorm > 2) return MAGX_EINVAL;
    if (p->check_finite != 0 && p->check_finite != 1) return MAGX_EINVAL;
    if ((p->terms & MAGX_DMI) && (!(p->terms & MAGX_EXCH) || !(p->A > 0.0))) return MAGX_EINVAL;
    return MAGX_OK;
}

template <typename R>
static Phys<R> make_phys(const Plan& pl, const magx_params* p, const void* hbias_members = nullptr,
                         const void* ms_profile = nullptr) {
    Phys<R> ph{};
    ph.hbm = static_cast<const R*>(hbias_members);
    ph.msp = static_cast<const R*>(ms_profile);
    const double mu0Ms = p->mu0 * p->Ms;
    ph.Ms = (R)p->Ms;
    ph.cex = (R)(2.0 * p->A / mu0Ms);
    ph.cdmi = (R)(2.0 * p->D / mu0Ms);
    ph.kap = (p->terms & MAGX_DMI) ? (R)(-p->D / (2.0 * p->A)) : (R)0;
    ph.cani = (R)(2.0 * p->Ku / mu0Ms);
    for (int c = 0; c < 3; ++c) {
        ph.eK[c] = (R)p->eK[c];
        ph.hb[c] = (R)p->Hbias[c];
    }
    ph.a = (R)(p->mu0 * p->gamma / (1.0 + p->alpha * p->alpha));
    ph.alpha = (R)p->alpha;
    ph.idx2 = (R)(1.0 / (pl.dx * pl.dx));
    ph.idy2 = (R)(1.0 / (pl.dy * pl.dy));
    ph.idz2 = (R)(1.0 / (pl.dz * pl.dz));
    ph.h2x = (R)(0.5 / pl.dx);
    ph.h2y = (R)(0.5 / pl.dy);
    ph.dx = (R)pl.dx;
    ph.dy = (R)pl.dy;
    ph.terms = p->terms;
    ph.renorm = p->renorm;
    return ph;
}

// H_bias at time t: the schedule's piecewise-linear value (held constant
// outside its knots) if one is set, else the parameter's constant bias.
static void bias_at(const magx_ctx* c, const magx_params* p, double t, double h[3]) {
    const size_t n = c->sched_t.size();
    if (n == 0) {
        for (int k = 0; k < 3; ++k) h[k] = p->Hbias[k];
        return;
    }
    const std::vector<double>& T = c->sched_t;
    const std::vector<double>& V = c->sched_h;
    if (t <= T[0] || n == 1) {
        for (int k = 0; k < 3; ++k) h[k] = V[k];
        return;
    }
    if (t >= T[n - 1]) {
        for (int k = 0; k < 3; ++k) h[k] = V[3 * (n - 1) + k];
        return;
    }
    size_t i = std::upper_bound(T.begin(), T.end(), t) - T.begin();   // T[i-1] <= t < T[i]
    const double w = (t - T[i - 1]) / (T[i] - T[i - 1]);
    for (int k = 0; k < 3; ++k) h[k] = V[3 * (i - 1) + k] + w * (V[3 * i + k] - V[3 * (i - 1) + k]);
}

template <typename R>
static Phys<R> phys_at(const magx_ctx* c, const magx_params* p, double t) {
    Phys<R> ph = make_phys<R>(c->pl, p, c->hbias_members, c->ms_profile);
    double h[3];
    bias_at(c, p, t, h);
    for (int k = 0; k < 3; ++k) ph.hb[k] = (R)h[k];
    return ph;
}

static std::mutex g_tw_mutex;
static bool g_tw_ready[64];

static int ensure_twiddles(hipStream_t s, int* device) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MAGX_EHIP;
    *device = dev;
    if (dev < 0 || dev >= 64) return MAGX_EHIP;
    std::lock_guard<std::mutex> lk(g_tw_mutex);
    if (g_tw_ready[dev]) return MAGX_OK;
    if (launch_twiddle_init(s) != hipSuccess) return MAGX_EHIP;
    // other streams of this device may use the table right away
    if (hipStreamSynchronize(s) != hipSuccess) return MAGX_EHIP;
    g_tw_ready[dev] = true;
    return MAGX_OK;
}

static inline char* bptr(void* p, size_t off) { return static_cast<char*>(p) + off; }

// Workspace of magx_step_static: a file-scope device array (each GPU the
// library runs on holds its own copy until the process ends).  Its name is a
// host-side stand-in in host code; the device address comes from
// hipGetSymbolAddress, taken once per device with that device current (at
// context creation) and kept in g_static_ws.
constexpr size_t kStaticWsBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticWsBytes];
static std::mutex g_static_mutex;
static void* g_static_ws[64];

static int ensure_static_ws(int dev) {
    if (dev < 0 || dev >= 64) return MAGX_EHIP;
    std::lock_guard<std::mutex> lk(g_static_mutex);
    if (g_static_ws[dev]) return MAGX_OK;
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return MAGX_EHIP;
    g_static_ws[dev] = ptr;
    return MAGX_OK;
}

static void* static_ws(int dev) {
    if (dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> lk(g_static_mutex);
    return g_static_ws[dev];
}

// Non-finite check of a call made with check_finite = 1: the flag word at the
// start of its workspace is cleared on the call's stream (by a kernel) and
// handed to the kernels, which set it on a NaN or infinite output; magx_status
// reads the flag of the last such call.  Inside a compound call (chk_hold) the
// flag armed at its start is kept.
template <typename R>
static int arm_finite_check(magx_ctx* c, const magx_params* p, void* ws, hipStream_t s, Phys<R>& ph) {
    ph.nf = nullptr;
    if (!p->check_finite) return MAGX_OK;
    unsigned* flag = reinterpret_cast<unsigned*>(bptr(ws, c->pl.off_flag));
    if (!(c->chk_hold && c->chk_flag == flag)) {
        if (launch_fill_zero(reinterpret_cast<double*>(flag), 1, s) != hipSuccess) return MAGX_EHIP;
        c->chk_flag = flag;
        c->chk_stream = s;
    }
    ph.nf = flag;
    return MAGX_OK;
}

// Arms the check once for a compound call and holds it until destruction.
struct CheckHold {
    magx_ctx* c;
    int prev;
    CheckHold(magx_ctx* ctx) : c(ctx), prev(ctx->chk_hold) {}
    int arm(const magx_params* p, void* ws, hipStream_t s) {
        Phys<float> tmp{};
        const int rc = arm_finite_check<float>(c, p, ws, s, tmp);
        c->chk_hold = 1;
        return rc;
    }
    ~CheckHold() { c->chk_hold = prev; }
};

// Convolution passes on X1 (input, overwritten with Y1) using X2.
template <typename R>
static int conv_passes(magx_ctx* c, void* ws, R Ms, hipStream_t s) {
    const Plan& pl = c->pl;
    void* X1 = bptr(ws, pl.off_x1);
    void* X2 = bptr(ws, pl.off_x2);
    if (pl.yzfilm) {
        ProfScope ps(c, kProfZconv, s);
        if (launch_yzfilm<R>(pl, X1, c->spectrum, Ms, s) != hipSuccess) return MAGX_EHIP;
        c->heff_count++;
        return MAGX_OK;
    }
    {
        ProfScope ps(c, kProfYfwd, s);
        if (launch_yfwd<R>(pl, X1, X2, s) != hipSuccess) return MAGX_EHIP;
    }
    {
        ProfScope ps(c, kProfZconv, s);
        if (launch_zconv<R>(pl, X2, c->spectrum, Ms, s) != hipSuccess) return MAGX_EHIP;
    }
    {
        ProfScope ps(c, kProfYinv, s);
        if (launch_yinv<R>(pl, X2, X1, s) != hipSuccess) return MAGX_EHIP;
    }
    c->heff_count++;
    return MAGX_OK;
}

template <typename R>
static int do_heff(magx_ctx* c, const R* m, const magx_params* p, R* H, void* ws, hipStream_t s, int energy,
                   double* e_out) {
    const Plan& pl = c->pl;
    Phys<R> ph = phys_at<R>(c, p, c->time);
    int rc0 = arm_finite_check<R>(c, p, ws, s, ph);
    if (rc0) return rc0;
    void* X1 = bptr(ws, pl.off_x1);
    double* part = reinterpret_cast<double*>(bptr(ws, pl.off_part));
    if (p->terms & MAGX_DEMAG) {
        {
            ProfScope ps(c, kProfXfwd, s);
            if (launch_xfwd<R>(pl, m, X1, ph.msp, s) != hipSuccess) return MAGX_EHIP;
        }
        int rc = conv_passes<R>(c, ws, ph.Ms, s);
        if (rc) return rc;
    }
    {
        ProfScope ps(c, kProfField, s);
        if (launch_field<R>(pl, ph, X1, m, H, 1, energy, 0, part, s) != hipSuccess) return MAGX_EHIP;
    }
    if (energy) {
        const double V = pl.dx * pl.dy * pl.dz;
        const double pref = -0.5 * p->mu0 * p->Ms * V;
        const double vku = (p->terms & MAGX_ANIS) ? V * p->Ku : 0.0;     // per magnetic cell
        if (launch_energy_finish(part, pl.nbatch, pl.blocks_per_member, pref, vku, e_out, s) != hipSuccess)
            return MAGX_EHIP;
    }
    return MAGX_OK;
}

template <typename R>
struct TapeView {
    R* base;
    long long N;
    int nsteps;
    R* y(int n, int s) const {   // s = 1..5
        if (s == 5) return n + 1 < nsteps ? y(n + 1, 1) : base + (long long)nsteps * 28 * N;
        return base + (long long)n * 28 * N + (long long)(s - 1) * 3 * N;
    }
    R* H(int n, int s) const { return base + (long long)n * 28 * N + 12 * N + (long long)(s - 1) * 3 * N; }
    R* nx(int n, int s) const { return base + (long long)n * 28 * N + 24 * N + (long long)(s - 2) * N; }  // s = 2..5
};

template <typename R>
static int do_step(magx_ctx* c, R* m, const magx_params* p, double dt, int nsteps, R* tape, void* ws,
                   hipStream_t s) {
    const Plan& pl = c->pl;
    Phys<R> ph = make_phys<R>(pl, p, c->hbias_members, c->ms_profile);
    int rc0 = arm_finite_check<R>(c, p, ws, s, ph);
    if (rc0) return rc0;
    const bool timed = !c->sched_t.empty();
    static const double kC[4] = {0.0, 0.5, 0.5, 1.0};   // stage times of classical RK4
    const bool demag = (p->terms & MAGX_DEMAG) != 0;
    void* X1 = bptr(ws, pl.off_x1);
    R* acc = reinterpret_cast<R*>(bptr(ws, pl.off_f[0]));
    R* ybuf[2] = {reinterpret_cast<R*>(bptr(ws, pl.off_f[1])), reinterpret_cast<R*>(bptr(ws, pl.off_f[2]))};
    TapeView<R> tv{tape, pl.ncell * pl.nbatch, nsteps};
    if (demag) {
        ProfScope ps(c, kProfXfwd, s);
        if (launch_xfwd<R>(pl, m, X1, ph.msp, s) != hipSuccess) return MAGX_EHIP;
    }
    for (int n = 0; n < nsteps; ++n) {
        for (int st = 1; st <= 4; ++st) {
            if (demag) {
                int rc = conv_passes<R>(c, ws, ph.Ms, s);
                if (rc) return rc;
            } else {
                c->heff_count++;
            }
            StageArgs<R> a{};
            a.yin = st == 1 ? m : (tape ? tv.y(n, st) : ybuf[st % 2]);
            a.mn = m;
            a.acc = acc;
            a.yout = st < 4 ? (tape ? tv.y(n, st + 1) : ybuf[(st + 1) % 2]) : m;
            a.yout2 = (st == 4 && tape) ? tv.y(n, 5) : nullptr;
            a.tapeH = tape ? tv.H(n, st) : nullptr;
            a.tapeNx = tape ? tv.nx(n, st + 1) : nullptr;
            a.tapeYin = (st == 1 && tape) ? tv.y(n, 1) : nullptr;
            a.stage = st;
            a.dt = (R)dt;
            a.want_next = !(n == nsteps - 1 && st == 4);
            ProfScope ps(c, kProfStage, s);
            Phys<R> phs = timed ? phys_at<R>(c, p, c->time + (n + kC[st - 1]) * dt) : ph;
            phs.nf = ph.nf;
            if (launch_stage<R>(pl, phs, X1, X1, a, s) != hipSuccess) return MAGX_EHIP;
        }
    }
    if (timed) c->time += nsteps * dt;
    return MAGX_OK;
}

// ---- HIP graph replay of RK4 steps on small grids ------------------------------
// A 4096-cell grid spends most of a step launching its 17 kernels; replaying a
// captured graph of up to kGraphChunk steps removes the per-launch host cost.
// Chunks give the same results bit for bit as one long call (the forward x
// pass a chunk starts with reproduces the one the previous stage kernel would
// have fused).  Used without a tape (its layout depends on the call's step
// count), without a bias schedule (the stage biases are baked into the
// launches) and while no launch timing is active.
constexpr long long kGraphMaxCells = 1LL << 18;
constexpr int kGraphChunk = 16;
constexpr size_t kGraphCache = 8;

static bool same_params(const magx_params& a, const magx_params& b) {
    for (int k = 0; k < 3; ++k)
        if (a.eK[k] != b.eK[k] || a.Hbias[k] != b.Hbias[k]) return false;
    return a.Ms == b.Ms && a.A == b.A && a.D == b.D && a.Ku == b.Ku && a.alpha == b.alpha && a.gamma == b.gamma &&
           a.mu0 == b.mu0 && a.terms == b.terms && a.renorm == b.renorm && a.check_finite == b.check_finite;
}

static bool graph_eligible(const magx_ctx* c, const void* tape) {
    return !tape && c->sched_t.empty() && c->prof_kind == 0 && c->pl.ncell * c->pl.nbatch <= kGraphMaxCells;
}

static void drop_graph(magx_ctx::StepGraph& g) {
    if (g.last) (void)hipStreamSynchronize(g.last);
    (void)hipGraphExecDestroy(g.exec);
}

// The cached graph for these arguments, captured now if needed; nullptr if
// capture failed (the caller then launches directly).
template <typename R>
static magx_ctx::StepGraph* step_graph(magx_ctx* c, R* m, const magx_params* p, double dt, int k, void* ws) {
    for (auto& g : c->graphs)
        if (g.m == m && g.ws == ws && g.dt == dt && g.nsteps == k && g.hbm == c->hbias_members &&
            g.msp == c->ms_profile && same_params(g.p, *p))
            return &g;
    if (!c->cap_stream && hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        c->cap_stream = nullptr;
        return nullptr;
    }
    const long long h0 = c->heff_count;
    if (hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed) != hipSuccess) return nullptr;
    const int rc = do_step<R>(c, m, p, dt, k, nullptr, ws, c->cap_stream);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(c->cap_stream, &graph);
    const long long dh = c->heff_count - h0;
    c->heff_count = h0;
    hipGraphExec_t exec = nullptr;
    const bool ok = rc == MAGX_OK && ec == hipSuccess && graph &&
                    hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
    if (graph) (void)hipGraphDestroy(graph);
    if (!ok) {
        (void)hipGetLastError();
        return nullptr;
    }
    if (c->graphs.size() >= kGraphCache) {
        drop_graph(c->graphs.front());
        c->graphs.erase(c->graphs.begin());
    }
    c->graphs.push_back({m, ws, *p, dt, k, c->hbias_members, c->ms_profile, exec, nullptr, dh});
    return &c->graphs.back();
}

template <typename R>
static int do_step_graphed(magx_ctx* c, R* m, const magx_params* p, double dt, int nsteps, void* ws,
                           hipStream_t s) {
    int done = 0;
    while (done < nsteps) {
        const int k = std::min(kGraphChunk, nsteps - done);
        magx_ctx::StepGraph* g = step_graph<R>(c, m, p, dt, k, ws);
        if (!g) break;
        if (hipGraphLaunch(g->exec, s) != hipSuccess) return MAGX_EHIP;
        g->last = s;
        c->heff_count += g->heff;
        if (p->check_finite) c->chk_stream = s;
        done += k;
    }
    if (done < nsteps) return do_step<R>(c, m, p, dt, nsteps - done, nullptr, ws, s);
    return MAGX_OK;
}

// Forward Euler (stage 0 of the stage kernel), ping-pong between m and a
// workspace field.
template <typename R>
static int do_step_euler(magx_ctx* c, R* m, const magx_params* p, double dt, int nsteps, void* ws,
                         hipStream_t s) {
    const Plan& pl = c->pl;
    const bool demag = (p->terms & MAGX_DEMAG) != 0;
    const bool timed = !c->sched_t.empty();
    void* X1 = bptr(ws, pl.off_x1);
    R* acc = reinterpret_cast<R*>(bptr(ws, pl.off_f[0]));
    R* W = reinterpret_cast<R*>(bptr(ws, pl.off_f[1]));
    R* cur = m;
    R* oth = W;
    Phys<R> ph0 = make_phys<R>(pl, p, c->hbias_members, c->ms_profile);
    int rc0 = arm_finite_check<R>(c, p, ws, s, ph0);
    if (rc0) return rc0;
    if (demag) {
        ProfScope ps(c, kProfXfwd, s);
        if (launch_xfwd<R>(pl, cur, X1, static_cast<const R*>(c->ms_profile), s) != hipSuccess) return MAGX_EHIP;
    }
    for (int n = 0; n < nsteps; ++n) {
        if (demag) {
            int rc = conv_passes<R>(c, ws, (R)p->Ms, s);
            if (rc) return rc;
        } else {
            c->heff_count++;
        }
        StageArgs<R> a{};
        a.yin = cur;
        a.mn = cur;
        a.acc = acc;
        a.yout = oth;
        a.stage = 0;
        a.dt = (R)dt;
        a.want_next = n < nsteps - 1;
        Phys<R> ph = phys_at<R>(c, p, c->time + n * dt);
        ph.nf = ph0.nf;
        ProfScope ps(c, kProfStage, s);
        if (launch_stage<R>(pl, ph, X1, X1, a, s) != hipSuccess) return MAGX_EHIP;
        std::swap(cur, oth);
    }
    if (cur != m && launch_copy<R>(cur, m, 3 * pl.ncell * pl.nbatch, s) != hipSuccess) return MAGX_EHIP;
    if (timed) c->time += nsteps * dt;
    return MAGX_OK;
}

template <typename R>
static int do_step_backward(magx_ctx* c, const R* tape, int nsteps, const magx_params* p, double dt, R* gm,
                            R* gHbias, void* ws, hipStream_t s, bool fresh = true, bool finish = true) {
    const Plan& pl = c->pl;
    Phys<R> ph = make_phys<R>(pl, p, c->hbias_members, c->ms_profile);
    int rc0 = arm_finite_check<R>(c, p, ws, s, ph);
    if (rc0) return rc0;
    const bool demag = (p->terms & MAGX_DEMAG) != 0;
    void* X1 = bptr(ws, pl.off_x1);
    R* xi5 = reinterpret_cast<R*>(bptr(ws, pl.off_f[0]));
    R* kap = reinterpret_cast<R*>(bptr(ws, pl.off_f[1]));
    R* mub[2] = {reinterpret_cast<R*>(bptr(ws, pl.off_f[2])), reinterpret_cast<R*>(bptr(ws, pl.off_f[3]))};
    double* part = reinterpret_cast<double*>(bptr(ws, pl.off_part));
    TapeView<R> tv{const_cast<R*>(tape), pl.ncell * pl.nbatch, nsteps};
    // per-block double partials of dL/dH_bias; a checkpointed rollout keeps
    // them across segments so the summation order does not depend on ckpt
    if (fresh && launch_fill_zero(part, (long long)pl.pencil_blocks * 8, s) != hipSuccess) return MAGX_EHIP;
    for (int n = nsteps - 1; n >= 0; --n) {
        StartArgs<R> sa{};
        sa.gm = gm;
        sa.y5 = tv.y(n, 5);
        sa.nx5 = tv.nx(n, 5);
        sa.y4 = tv.y(n, 4);
        sa.xi5 = xi5;
        sa.kap = kap;
        sa.muout = mub[0];
        sa.dt = (R)dt;
        {
            ProfScope ps(c, kProfBstart, s);
            if (launch_bstart<R>(pl, ph, X1, sa, part, s) != hipSuccess) return MAGX_EHIP;
        }
        for (int st = 4; st >= 1; --st) {
            if (demag) {
                int rc = conv_passes<R>(c, ws, ph.Ms, s);
                if (rc) return rc;
            }
            BackArgs<R> ba{};
            ba.mu = mub[st % 2];
            ba.ys = tv.y(n, st);
            ba.Hs = tv.H(n, st);
            ba.kap = kap;
            ba.xi5 = xi5;
            ba.nxs = st >= 2 ? tv.nx(n, st) : nullptr;
            ba.yprev = st >= 2 ? tv.y(n, st - 1) : nullptr;
            ba.gm = gm;
            ba.muout = mub[(st - 1) % 2];
            ba.stage = st;
            ba.dt = (R)dt;
            ProfScope ps(c, kProfBstage, s);
            if (launch_bstage<R>(pl, ph, X1, X1, ba, part, s) != hipSuccess) return MAGX_EHIP;
        }
    }
    if (finish && (p->terms & MAGX_ZEEMAN)) {
        if (launch_reduce_partials<R>(part, pl.nbatch, pl.blocks_per_member, 3, gHbias, fresh ? 1 : 0, s) !=
            hipSuccess)
            return MAGX_EHIP;
    }
    return MAGX_OK;
}

template <typename R>
static int do_heff_backward(magx_ctx* c, const R* gH, const magx_params* p, R* gm, R* gHbias, void* ws,
                            hipStream_t s) {
    const Plan& pl = c->pl;
    Phys<R> ph = make_phys<R>(pl, p, c->hbias_members, c->ms_profile);
    int rc0 = arm_finite_check<R>(c, p, ws, s, ph);
    if (rc0) return rc0;
    void* X1 = bptr(ws, pl.off_x1);
    double* part = reinterpret_cast<double*>(bptr(ws, pl.off_part));
    if (launch_fill_zero(part, (long long)pl.pencil_blocks * 8, s) != hipSuccess) return MAGX_EHIP;
    if (p->terms & MAGX_DEMAG) {
        if (launch_xfwd<R>(pl, gH, X1, nullptr, s) != hipSuccess) return MAGX_EHIP;
        int rc = conv_passes<R>(c, ws, ph.Ms, s);
        if (rc) return rc;
    }
    const int sum_input = (p->terms & MAGX_ZEEMAN) ? 1 : 0;
    if (launch_field<R>(pl, ph, X1, gH, gm, 0, 0, sum_input, part, s) != hipSuccess) return MAGX_EHIP;
    if (launch_reduce_partials<R>(part, pl.nbatch, pl.blocks_per_member, 3, gHbias, 0, s) != hipSuccess)
        return MAGX_EHIP;
    return MAGX_OK;
}

// Knoth-Wolke method in Williamson's two-register form (A2, B2) and, expanded
// from it, the Butcher rows a (b as the fourth row), nodes c and the forcing
// weights of the three fast intervals: w[i][j] = (a[i+1][j] - a[i][j]) / (c[i+1] - c[i]).
struct KnothWolke {
    double A2[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
    double B2[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};
    double a[4][3], c[4], w[3][3];
    KnothWolke() {
        double q[3] = {0.0, 0.0, 0.0}, y[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k < 3; ++k) {
            for (int j = 0; j < 3; ++j) a[k][j] = y[j];
            for (int j = 0; j < 3; ++j) q[j] = A2[k] * q[j] + (j == k ? 1.0 : 0.0);
            for (int j = 0; j < 3; ++j) y[j] += B2[k] * q[j];
        }
        for (int j = 0; j < 3; ++j) a[3][j] = y[j];
        for (int i = 0; i < 4; ++i) c[i] = a[i][0] + a[i][1] + a[i][2];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) w[i][j] = (a[i + 1][j] - a[i][j]) / (c[i + 1] - c[i]);
    }
};

// Equal fast substeps covering dc*dt with steps no longer than dt_fast.
static long long mri_substeps(double dc, double dt, double dt_fast) {
    const double v = std::ceil(dc * dt / dt_fast * (1.0 - 1e-12));
    return v < 1.0 ? 1 : (long long)v;
}

template <typename R>
static int do_step_mri(magx_ctx* c, R* m, const magx_params* p, double dt, double dt_fast, int nsteps, void* ws,
                       hipStream_t s) {
    static const KnothWolke kw;
    const Plan& pl = c->pl;
    Phys<R> ph = make_phys<R>(pl, p, c->hbias_members, c->ms_profile);
    int rc0 = arm_finite_check<R>(c, p, ws, s, ph);
    if (rc0) return rc0;
    Phys<R> pfast = ph, pslow = ph;     // both keep the ghost rule of the full field
    pfast.terms = ph.terms & MAGX_EXCH;
    pslow.terms = ph.terms & ~MAGX_EXCH;
    const bool demag = (p->terms & MAGX_DEMAG) != 0;
    const bool timed = !c->sched_t.empty();
    void* X1 = bptr(ws, pl.off_x1);
    R* S1 = reinterpret_cast<R*>(bptr(ws, pl.off_f[0]));
    R* S2 = reinterpret_cast<R*>(bptr(ws, pl.off_f[1]));
    R* rf = reinterpret_cast<R*>(bptr(ws, pl.off_f[2]));
    R* q = reinterpret_cast<R*>(bptr(ws, pl.off_f[3]));
    R* W = reinterpret_cast<R*>(bptr(ws, pl.off_f[4]));
    long long nsub[3];
    double hsub[3];
    for (int i = 0; i < 3; ++i) {
        const double dc = kw.c[i + 1] - kw.c[i];
        nsub[i] = mri_substeps(dc, dt, dt_fast);
        hsub[i] = dc * dt / (double)nsub[i];
    }
    R* cur = m;
    R* oth = W;
    if (demag) {
        ProfScope ps(c, kProfXfwd, s);
        if (launch_xfwd<R>(pl, cur, X1, ph.msp, s) != hipSuccess) return MAGX_EHIP;
    }
    for (int n = 0; n < nsteps; ++n) {
        for (int i = 0; i < 3; ++i) {
            if (demag) {
                int rc = conv_passes<R>(c, ws, ph.Ms, s);
                if (rc) return rc;
            } else {
                c->heff_count++;
            }
            R* Sout = i == 0 ? S1 : (i == 1 ? S2 : nullptr);
            const R* Sa = i >= 1 ? S1 : nullptr;
            const R* Sb = i >= 2 ? S2 : nullptr;
            Phys<R> pslow_t = pslow;
            if (timed) {
                pslow_t = phys_at<R>(c, p, c->time + (n + kw.c[i]) * dt);
                pslow_t.terms = ph.terms & ~MAGX_EXCH;
                pslow_t.nf = ph.nf;
            }
            if (launch_mri_slow<R>(pl, pslow_t, X1, cur, demag ? 1 : 0, Sout, Sa, Sb, (R)kw.w[i][0],
                                   (R)kw.w[i][1], (R)kw.w[i][i], rf, s) != hipSuccess)
                return MAGX_EHIP;
            for (long long sub = 0; sub < nsub[i]; ++sub) {
                for (int k = 0; k < 3; ++k) {
                    const bool last = sub == nsub[i] - 1 && k == 2;
                    const int norm = last && (p->renorm == 2 || (i == 2 && p->renorm >= 1)) ? 1 : 0;
                    const bool fwd = last && demag && !(n == nsteps - 1 && i == 2);
                    if (launch_mri_fast<R>(pl, pfast, cur, oth, q, rf, (R)kw.A2[k], (R)kw.B2[k], (R)hsub[i],
                                           k == 0 ? 1 : 0, norm, fwd ? X1 : nullptr, s) != hipSuccess)
                        return MAGX_EHIP;
                    std::swap(cur, oth);
                }
            }
        }
    }
    if (cur != m && launch_copy<R>(cur, m, 3 * pl.ncell * pl.nbatch, s) != hipSuccess) return MAGX_EHIP;
    if (timed) c->time += nsteps * dt;
    return MAGX_OK;
}

}  // namespace magx

// ---------------------------------------------------------------------------------
extern "C" {

int magx_sizes_batched(const magx_grid* g, magx_dtype dt, int nbatch, magx_size_info* out) {
    if (!out) return MAGX_EINVAL;
    Plan pl;
    int rc = make_plan(g, dt, nbatch, &pl);
    if (rc) return rc;
    out->spectrum_bytes = pl.spectrum_bytes;
    out->init_scratch_bytes = pl.scratch_bytes;
    out->workspace_bytes = pl.ws_bytes;
    out->tape_bytes_per_step = pl.tape_step_bytes;
    out->tape_bytes_extra = pl.tape_extra_bytes;
    out->field_bytes = pl.field_bytes;
    return MAGX_OK;
}

int magx_sizes(const magx_grid* g, magx_dtype dt, magx_size_info* out) {
    return magx_sizes_batched(g, dt, 1, out);
}

int magx_tensor_init_batched(magx_ctx** ctx, const magx_grid* g, magx_dtype dt, int nbatch, void* spectrum,
                             void* scratch, void* stream) {
    if (!ctx) return MAGX_EINVAL;
    *ctx = nullptr;
    // the z passes copy tensor blocks in 16-byte pieces
    if (!spectrum || !scratch || (reinterpret_cast<uintptr_t>(spectrum) & 15) != 0) return MAGX_EINVAL;
    Plan pl;
    int rc = make_plan(g, dt, nbatch, &pl);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = 0;
    rc = ensure_twiddles(s, &dev);
    if (rc) return rc;
    rc = ensure_static_ws(dev);
    if (rc) return rc;
    if (build_tensor_spectrum(pl, spectrum, scratch, s) != hipSuccess) return MAGX_EHIP;
    magx_ctx* c = new (std::nothrow) magx_ctx;
    if (!c) return MAGX_EINVAL;
    c->pl = pl;
    c->spectrum = spectrum;
    c->hbias_members = nullptr;
    c->ms_profile = nullptr;
    c->time = 0.0;
    c->heff_count = 0;
    c->device = dev;
    c->prof_kind = 0;
    c->prof_used = 0;
    c->chk_flag = nullptr;
    c->chk_stream = nullptr;
    c->chk_hold = 0;
    c->cap_stream = nullptr;
    *ctx = c;
    return MAGX_OK;
}

int magx_tensor_init(magx_ctx** ctx, const magx_grid* g, magx_dtype dt, void* spectrum, void* scratch,
                     void* stream) {
    return magx_tensor_init_batched(ctx, g, dt, 1, spectrum, scratch, stream);
}

int magx_set_member_bias(magx_ctx* ctx, const void* hbias) {
    if (!ctx) return MAGX_EINVAL;
    ctx->hbias_members = hbias;
    return MAGX_OK;
}

int magx_ctx_batch(const magx_ctx* ctx) { return ctx ? ctx->pl.nbatch : -1; }

int magx_set_ms_profile(magx_ctx* ctx, const void* s) {
    if (!ctx) return MAGX_EINVAL;
    ctx->ms_profile = s;
    return MAGX_OK;
}

int magx_heff(magx_ctx* ctx, const void* m, const magx_params* p, void* H, void* ws, void* stream) {
    if (!ctx || !m || !H || !ws) return MAGX_EINVAL;
    int rc = check_params(p);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (ctx->pl.dtype == MAGX_F32)
        return do_heff<float>(ctx, static_cast<const float*>(m), p, static_cast<float*>(H), ws, s, 0, nullptr);
    return do_heff<double>(ctx, static_cast<const double*>(m), p, static_cast<double*>(H), ws, s, 0, nullptr);
}

int magx_energy(magx_ctx* ctx, const void* m, const magx_params* p, void* e_out, void* ws, void* stream) {
    if (!ctx || !m || !e_out || !ws) return MAGX_EINVAL;
    int rc = check_params(p);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* e = static_cast<double*>(e_out);
    if (ctx->pl.dtype == MAGX_F32)
        return do_heff<float>(ctx, static_cast<const float*>(m), p, nullptr, ws, s, 1, e);
    return do_heff<double>(ctx, static_cast<const double*>(m), p, nullptr, ws, s, 1, e);
}

int magx_llg_rhs(magx_ctx* ctx, const void* m, const void* H, const magx_params* p, void* dmdt, void* stream) {
    if (!ctx || !m || !H || !dmdt) return MAGX_EINVAL;
    int rc = check_params(p);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    if (ctx->pl.dtype == MAGX_F32)
        e = launch_rhs<float>(ctx->pl, make_phys<float>(ctx->pl, p), static_cast<const float*>(m),
                              static_cast<const float*>(H), static_cast<float*>(dmdt), s);
    else
        e = launch_rhs<double>(ctx->pl, make_phys<double>(ctx->pl, p), static_cast<const double*>(m),
                               static_cast<const double*>(H), static_cast<double*>(dmdt), s);
    return e == hipSuccess ? MAGX_OK : MAGX_EHIP;
}

int magx_step(magx_ctx* ctx, void* m, const magx_params* p, double dt, int nsteps, void* tape, void* ws,
              void* stream) {
    if (!ctx || !m || !ws || nsteps < 0 || !std::isfinite(dt)) return MAGX_EINVAL;
    int rc = check_params(p);
    if (rc) return rc;
    if (nsteps == 0) return MAGX_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (graph_eligible(ctx, tape)) {
        if (ctx->pl.dtype == MAGX_F32) return do_step_graphed<float>(ctx, static_cast<float*>(m), p, dt, nsteps, ws, s);
        return do_step_graphed<double>(ctx, static_cast<double*>(m), p, dt, nsteps, ws, s);
    }
    if (ctx->pl.dtype == MAGX_F32)
        return do_step<float>(ctx, static_cast<float*>(m), p, dt, nsteps, static_cast<float*>(tape), ws, s);
    return do_step<double>(ctx, static_cast<double*>(m), p, dt, nsteps, static_cast<double*>(tape), ws, s);
}

int magx_step_static(magx_ctx* ctx, void* m, const magx_params* p, double dt, int nsteps, void* stream) {
    if (!ctx || !m || nsteps < 0 || !std::isfinite(dt)) return MAGX_EINVAL;
    int rc = check_params(p);
    if (rc) return rc;
    // RK4 without a tape uses the flag word, X1, X2 and three fields: the
    // workspace prefix up to the fourth field
    if (ctx->pl.off_f[3] > kStaticWsBytes) return MAGX_EWORKSPACE;
    void* ws = static_ws(ctx->device);
    if (!ws) return MAGX_EHIP;
    if (nsteps == 0) return MAGX_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (ctx->pl.dtype == MAGX_F32)
        return do_step<float>(ctx, static_cast<float*>(m), p, dt, nsteps, nullptr, ws, s);
    return do_step<double>(ctx, static_cast<double*>(m), p, dt, nsteps, nullptr, ws, s);
}

int magx_step_euler(magx_ctx* ctx, void* m, const magx_params* p, double dt, int nsteps, void* ws, void* stream) {
    if (!ctx || !m || !ws || nsteps < 0 || !std::isfinite(dt)) return MAGX_EINVAL;
    int rc = check_params(p);
    if (rc) return rc;
    if (nsteps == 0) return MAGX_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (ctx->pl.dtype == MAGX_F32)
        return do_step_euler<float>(ctx, static_cast<float*>(m), p, dt, nsteps, ws, s);
    return do_step_euler<double>(ctx, static_cast<double*>(m), p, dt, nsteps, ws, s);
}

int magx_set_bias_schedule(magx_ctx* ctx, int n, const double* times, const double* values, double t0) {
    if (!ctx || n < 0 || !std::isfinite(t0)) return MAGX_EINVAL;
    if (n > 0 && (!times || !values)) return MAGX_EINVAL;
    for (int i = 0; i < n; ++i) {
        if (!std::isfinite(times[i]) || (i > 0 && !(times[i] > times[i - 1]))) return MAGX_EINVAL;
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(values[3 * i + k])) return MAGX_EINVAL;
    }
    ctx->sched_t.assign(times, times + n);
    ctx->sched_h.assign(values, values + 3 * (size_t)n);
    ctx->time = t0;
    return MAGX_OK;
}

int magx_get_time(const magx_ctx* ctx, double* t) {
    if (!ctx || !t) return MAGX_EINVAL;
    *t = ctx->time;
    return MAGX_OK;
}

int magx_step_mri(magx_ctx* ctx, void* m, const magx_params* p, double dt, double dt_fast, int nsteps, void* ws,
                  void* stream) {
    if (!ctx || !m || !ws || nsteps < 0 || !std::isfinite(dt) || !(dt >= 0.0) || !std::isfinite(dt_fast) ||
        !(dt_fast > 0.0))
        return MAGX_EINVAL;
    // at most 2^20 fast substeps per slow step
    if (dt / dt_fast > (double)(1 << 20)) return MAGX_EINVAL;
    int rc = check_params(p);
    if (rc) return rc;
    if (nsteps == 0) return MAGX_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (ctx->pl.dtype == MAGX_F32)
        return do_step_mri<float>(ctx, static_cast<float*>(m), p, dt, dt_fast, nsteps, ws, s);
    return do_step_mri<double>(ctx, static_cast<double*>(m), p, dt, dt_fast, nsteps, ws, s);
}

int magx_heff_backward(magx_ctx* ctx, const void* gH, const magx_params* p, void* gm, void* gHbias, void* ws,
                       void* stream) {
    if (!ctx || !gH || !gm || !gHbias || !ws) return MAGX_EINVAL;
    if (!ctx->sched_t.empty() || ctx->ms_profile) return MAGX_ESTATE;
    int rc = check_params(p);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (ctx->pl.dtype == MAGX_F32)
        return do_heff_backward<float>(ctx, static_cast<const float*>(gH), p, static_cast<float*>(gm),
                                       static_cast<float*>(gHbias), ws, s);
    return do_heff_backward<double>(ctx, static_cast<const double*>(gH), p, static_cast<double*>(gm),
                                    static_cast<double*>(gHbias), ws, s);
}

int magx_step_backward(magx_ctx* ctx, const void* tape, int nsteps, const magx_params* p, double dt, void* gm,
                       void* gHbias, void* ws, void* stream) {
    if (!ctx || !tape || !gm || !gHbias || !ws || nsteps < 0 || !std::isfinite(dt)) return MAGX_EINVAL;
    if (!ctx->sched_t.empty() || ctx->ms_profile) return MAGX_ESTATE;
    int rc = check_params(p);
    if (rc) return rc;
    if (nsteps == 0) return MAGX_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (ctx->pl.dtype == MAGX_F32)
        return do_step_backward<float>(ctx, static_cast<const float*>(tape), nsteps, p, dt,
                                       static_cast<float*>(gm), static_cast<float*>(gHbias), ws, s);
    return do_step_backward<double>(ctx, static_cast<const double*>(tape), nsteps, p, dt, static_cast<double*>(gm),
                                    static_cast<double*>(gHbias), ws, s);
}

int magx_rollout_forward(magx_ctx* ctx, void* m, const magx_params* p, double dt, int nsteps, int ckpt,
                         void* ckpt_store, void* ws, void* stream) {
    if (!ctx || !m || !ckpt_store || !ws || nsteps < 0 || ckpt < 1 || !std::isfinite(dt)) return MAGX_EINVAL;
    if (!ctx->sched_t.empty() || ctx->ms_profile) return MAGX_ESTATE;
    int rc = check_params(p);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t fb = ctx->pl.field_bytes;
    const long long n3 = 3 * ctx->pl.ncell * ctx->pl.nbatch;
    CheckHold hold(ctx);
    rc = hold.arm(p, ws, s);
    if (rc) return rc;
    for (int n0 = 0, seg = 0; n0 < nsteps; n0 += ckpt, ++seg) {
        void* slot = bptr(ckpt_store, (size_t)seg * fb);
        hipError_t e = ctx->pl.dtype == MAGX_F32
                           ? launch_copy<float>(static_cast<const float*>(m), static_cast<float*>(slot), n3, s)
                           : launch_copy<double>(static_cast<const double*>(m), static_cast<double*>(slot), n3, s);
        if (e != hipSuccess) return MAGX_EHIP;
        rc = magx_step(ctx, m, p, dt, std::min(ckpt, nsteps - n0), nullptr, ws, stream);
        if (rc) return rc;
    }
    return MAGX_OK;
}

int magx_rollout_backward(magx_ctx* ctx, const void* ckpt_store, const magx_params* p, double dt, int nsteps,
                          int ckpt, void* gm, void* gHbias, void* tape, void* mwork, void* ws, void* stream) {
    if (!ctx || !ckpt_store || !gm || !gHbias || !tape || !mwork || !ws || nsteps < 0 || ckpt < 1 ||
        !std::isfinite(dt))
        return MAGX_EINVAL;
    if (!ctx->sched_t.empty() || ctx->ms_profile) return MAGX_ESTATE;
    int rc = check_params(p);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Plan& pl = ctx->pl;
    CheckHold hold(ctx);
    rc = hold.arm(p, ws, s);
    if (rc) return rc;
    double* part = reinterpret_cast<double*>(bptr(ws, pl.off_part));
    if (launch_fill_zero(part, (long long)pl.pencil_blocks * 8, s) != hipSuccess) return MAGX_EHIP;
    hipError_t e;
    const size_t fb = pl.field_bytes;
    const long long n3 = 3 * pl.ncell * pl.nbatch;
    const int nseg = nsteps == 0 ? 0 : (nsteps + ckpt - 1) / ckpt;
    for (int seg = nseg - 1; seg >= 0; --seg) {
        const int n0 = seg * ckpt;
        const int len = std::min(ckpt, nsteps - n0);
        const void* slot = bptr(const_cast<void*>(ckpt_store), (size_t)seg * fb);
        e = pl.dtype == MAGX_F32
                ? launch_copy<float>(static_cast<const float*>(slot), static_cast<float*>(mwork), n3, s)
                : launch_copy<double>(static_cast<const double*>(slot), static_cast<double*>(mwork), n3, s);
        if (e != hipSuccess) return MAGX_EHIP;
        rc = magx_step(ctx, mwork, p, dt, len, tape, ws, stream);
        if (rc) return rc;
        rc = pl.dtype == MAGX_F32
                 ? do_step_backward<float>(ctx, static_cast<const float*>(tape), len, p, dt, static_cast<float*>(gm),
                                           static_cast<float*>(gHbias), ws, s, false, false)
                 : do_step_backward<double>(ctx, static_cast<const double*>(tape), len, p, dt,
                                            static_cast<double*>(gm), static_cast<double*>(gHbias), ws, s, false,
                                            false);
        if (rc) return rc;
    }
    // gHbias = sum over each member's blocks of the partials (0 without a Zeeman term)
    const int nb = pl.nbatch, bpm = pl.blocks_per_member;
    e = pl.dtype == MAGX_F32
            ? launch_reduce_partials<float>(part, nb, bpm, 3, static_cast<float*>(gHbias), 0, s)
            : launch_reduce_partials<double>(part, nb, bpm, 3, static_cast<double*>(gHbias), 0, s);
    return e == hipSuccess ? MAGX_OK : MAGX_EHIP;
}

long long magx_heff_count(const magx_ctx* ctx) { return ctx ? ctx->heff_count : -1; }

int magx_status(magx_ctx* ctx) {
    if (!ctx) return MAGX_EINVAL;
    if (!ctx->chk_flag) return MAGX_OK;
    if (hipStreamSynchronize(ctx->chk_stream) != hipSuccess) return MAGX_EHIP;
    unsigned v = 0;
    if (hipMemcpy(&v, ctx->chk_flag, sizeof v, hipMemcpyDeviceToHost) != hipSuccess) return MAGX_EHIP;
    return v ? MAGX_ENONFINITE : MAGX_OK;
}

int magx_spectrum_layout(const magx_ctx* ctx, int dims[5]) {
    if (!ctx || !dims) return MAGX_EINVAL;
    dims[0] = ctx->pl.Hy;
    dims[1] = ctx->pl.ntz;
    dims[2] = 6;
    dims[3] = ctx->pl.Hz;
    dims[4] = ctx->pl.tz;
    return MAGX_OK;
}

int magx_ctx_info(const magx_ctx* ctx, magx_grid* g, magx_dtype* dt) {
    if (!ctx || !g || !dt) return MAGX_EINVAL;
    g->nx = ctx->pl.nx; g->ny = ctx->pl.ny; g->nz = ctx->pl.nz;
    g->dx = ctx->pl.dx; g->dy = ctx->pl.dy; g->dz = ctx->pl.dz;
    *dt = ctx->pl.dtype;
    return MAGX_OK;
}

const char* magx_strerror(int code) {
    switch (code) {
        case MAGX_OK: return "ok";
        case MAGX_EINVAL: return "invalid argument";
        case MAGX_ESIZE: return "grid too large for the FFT passes";
        case MAGX_EDTYPE: return "unknown element type";
        case MAGX_EWORKSPACE: return "buffer too small";
        case MAGX_EHIP: return "HIP error";
        case MAGX_ENONFINITE: return "non-finite value";
        case MAGX_ESTATE: return "not available while a bias schedule or a magnetisation profile is set";
        default: return "unknown error";
    }
}

int magx_memory_probe(magx_ctx* ctx, int kind, void* ws, void* stream, double* bytes) {
    if (!ctx || !ws || !bytes || kind < 0 || kind > 2) return MAGX_EINVAL;
    if (ctx->pl.dtype != MAGX_F32) return MAGX_EDTYPE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (launch_memory_probe(ctx->pl, kind, bptr(ws, ctx->pl.off_x2), s, bytes) != hipSuccess) return MAGX_EHIP;
    return MAGX_OK;
}

int magx_profile_start(magx_ctx* ctx, int kind) {
    if (!ctx || kind < 0 || kind > kProfBstage) return MAGX_EINVAL;
    ctx->prof_kind = kind;
    ctx->prof_used = 0;
    return MAGX_OK;
}

int magx_profile_stop(magx_ctx* ctx, long long* launches, double* total_ms) {
    if (!ctx || !launches || !total_ms) return MAGX_EINVAL;
    double tot = 0.0;
    for (size_t i = 0; i < ctx->prof_used; ++i) {
        auto& ev = ctx->prof_events[i];
        if (hipEventSynchronize(ev.second) != hipSuccess) return MAGX_EHIP;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, ev.first, ev.second) != hipSuccess) return MAGX_EHIP;
        tot += ms;
    }
    *launches = (long long)ctx->prof_used;
    *total_ms = tot;
    ctx->prof_kind = 0;
    ctx->prof_used = 0;
    return MAGX_OK;
}

void magx_destroy(magx_ctx* ctx) {
    if (!ctx) return;
    for (auto& ev : ctx->prof_events) {
        (void)hipEventDestroy(ev.first);
        (void)hipEventDestroy(ev.second);
    }
    for (auto& g : ctx->graphs) drop_graph(g);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    delete ctx;
}

}  // extern "C"
