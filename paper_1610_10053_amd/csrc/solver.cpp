// Host driver and C-ABI of the implicit-step library: Newton-Raphson on the
// Crank-Nicolson system, restarted right-preconditioned GMRES with CGS2 and
// Givens rotations, Jacobian-free products, CFL time step with step halving
// (section 2 and section 2.1 of Goffrey et al. 2016).  All vectors live on
// the device; the host reads back a handful of scalars per Krylov iteration.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/jfnk.h"
#include "kernels.hpp"
#include "problem.hpp"

using namespace jfnk;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIPCHK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) return fail(-3, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

constexpr int kDsum = 512;  // device scalar area
// offsets in the device scalar area
constexpr int D_H1 = 0, D_H2 = 80, D_HN = 160, D_Y = 170, D_USQ = 250, D_EPS = 251, D_TMP = 260, D_SUSQ = 300,
              D_SEPS = 301, D_K0 = 302;  // D_K0, D_K0 + 1: finest-level coupling factor per operator

struct Buffers {
    std::vector<void*> ptrs;
    size_t bytes = 0;
    ~Buffers() {
        for (void* p : ptrs) (void)hipFree(p);
    }
};

}  // namespace

struct jfnk_problem {
    Grid G{};
    jfnk_problem_desc desc{};
    jfnk_solver_opts opts{};
    hipStream_t stream = nullptr;
    int device = 0;  // the device current at creation, which holds every buffer
    Buffers buf;
    // optional caller-provided device range that every buffer is carved from
    char* slab = nullptr;
    size_t slab_size = 0, slab_off = 0;
    // vectors of nvec doubles
    double *u = nullptr, *un = nullptr, *b = nullptr, *x = nullptr, *rhs = nullptr,
           *r = nullptr, *w = nullptr, *t = nullptr, *z = nullptr, *s1 = nullptr,
           *s2 = nullptr;
    double* Ru = nullptr;  // R at the current Newton iterate (Jacobian-free products)
    // the state at the start of the last accepted step and its dt (the
    // extrapolated first iterate); have_prev false until a step is accepted
    // and after jfnk_set_state
    double* uprev = nullptr;
    double dt_prev = 0.0;
    bool have_prev = false;
    void* V = nullptr;
    void* Zb = nullptr;  // preconditioned basis vectors M^-1 v_j of a GMRES cycle (FP64, or FP32 in the mixed form)
    Prim P{};
    Flux Fx{};
    WallFlux W{};
    double* sbal = nullptr;
    PcCoef C{};
    LevelSet<double> ac64{}, df64{};
    LevelSet<float> ac32{}, df32{};
    // device copies of the level descriptors (for the single-workgroup solve)
    LevelT<double>* dac64 = nullptr;
    LevelT<double>* ddf64 = nullptr;
    LevelT<float>* dac32 = nullptr;
    LevelT<float>* ddf32 = nullptr;
    int nlev = 1, coarse_from = 0;
    double* rEd = nullptr;
    double* lines = nullptr;
    double* part = nullptr;
    int npart = 0;
    double* dsum = nullptr;
    double* hpin = nullptr;
    bool own_hpin = false;
    double scale[5] = {1, 1, 1, 1, 1};
    double t_now = 0.0;
    double dt_ctrl = 0.0;  // the controller's bound on the next dt (0: unset)
    long nunk = 0;
    int nred = 1, ncell_blk = 1;
    // last dt limits
    double hyd = 0, adv = 0, rad = 0;
    Profiler prof;
    bool prof_on = false;
    // passive scalars: ns partial densities (ns x N), their Krylov workspace
    // and the density and mass fluxes of u^n and u^{n+1}
    int nscal = 0, renorm = 0;
    Buffers sbuf;
    double *sc = nullptr, *sc_n = nullptr, *sb = nullptr, *sG = nullptr, *sx = nullptr, *srhs = nullptr,
           *sr = nullptr, *sw = nullptr, *stmp = nullptr, *sV = nullptr;
    double *srho0 = nullptr, *srho1 = nullptr, *sfr0 = nullptr, *sfr1 = nullptr;
    int sc_newton = 0, sc_gmres = 0;
    // the multigrid solve of each operator (acoustic, conduction) replayed as
    // a HIP graph on the problem's stream (captured at its first use)
    hipGraphExec_t mg_exec[2] = {nullptr, nullptr};
    bool use_graphs = true;
    // marks the end of a GMRES step's scalar read-back, so that the host can
    // wait for it while later work already runs on the stream
    hipEvent_t rb_event = nullptr;
    // the acoustic right-hand side of the next basis vector to be
    // preconditioned was formed when that vector was stored
    bool pc_rhs_formed = false;
    // FP64 Cartesian problems: the acoustic couplings are formed directly in
    // the finest level's coupling arrays (its sigma of 1 set once), so the
    // hierarchy build needs no copy of them
    bool kap_in_level0 = false;
    ~jfnk_problem() {
        for (auto& g : mg_exec)
            if (g) (void)hipGraphExecDestroy(g);
        if (rb_event) (void)hipEventDestroy(rb_event);
        if (hpin && own_hpin) (void)hipHostFree(hpin);
    }
};

namespace {

constexpr size_t kSlabAlign = 256;
constexpr size_t kSlabSlack = 128 * kSlabAlign;  // alignment of every carved buffer

template <typename Tp>
int dalloc(jfnk_problem* p, Tp** out, size_t count) {
    void* ptr = nullptr;
    const size_t bytes = count * sizeof(Tp);
    if (p->slab) {
        const size_t off = (p->slab_off + kSlabAlign - 1) / kSlabAlign * kSlabAlign;
        if (off + bytes > p->slab_size) return fail(-2, "device range too small for the problem");
        p->slab_off = off + bytes;
        p->buf.bytes += bytes;
        *out = (Tp*)(p->slab + off);
        return 0;
    }
    hipError_t e = hipMalloc(&ptr, bytes == 0 ? 8 : bytes);
    if (e != hipSuccess) return fail(-2, std::string("hipMalloc: ") + hipGetErrorString(e));
    p->buf.ptrs.push_back(ptr);
    p->buf.bytes += bytes;
    *out = (Tp*)ptr;
    return 0;
}

#define CK(expr)              \
    do {                      \
        int rc_ = (expr);     \
        if (rc_ != 0) return rc_; \
    } while (0)

int validate(const jfnk_problem_desc* d, const jfnk_solver_opts* o) {
    if (!d || !o) return fail(-1, "null descriptor or options");
    if (d->ndim != 2 && d->ndim != 3) return fail(-1, "ndim must be 2 or 3");
    for (int a = 0; a < d->ndim; ++a) {
        if (d->n[a] < 4) return fail(-1, "every axis needs at least 4 cells");
        if (d->bc[a] != JFNK_BC_PERIODIC && d->bc[a] != JFNK_BC_WALL) return fail(-1, "unknown boundary type");
        if (d->bc[a] == JFNK_BC_PERIODIC && d->n[a] % 2) return fail(-1, "periodic axes need an even cell count");
        if (!(d->hi[a] > d->lo[a])) return fail(-1, "empty domain");
    }
    if (d->ndim == 2 && d->n[2] != 1) return fail(-1, "2D problems need n[2] = 1");
    if (!(d->gamma > 1.0)) return fail(-1, "gamma must exceed 1");
    if (d->chi0 < 0.0) return fail(-1, "chi0 must be >= 0");
    if (d->energy_form != JFNK_ENERGY_TOTAL && d->energy_form != JFNK_ENERGY_INTERNAL)
        return fail(-1, "unknown energy_form");
    if (d->geometry != JFNK_GEOM_CARTESIAN && d->geometry != JFNK_GEOM_SPHERICAL)
        return fail(-1, "unknown geometry");
    if (d->geometry == JFNK_GEOM_SPHERICAL) {
        if (d->ndim != 2) return fail(-4, "spherical geometry is two-dimensional (r, theta)");
        if (d->bc[0] != JFNK_BC_WALL || d->bc[1] != JFNK_BC_WALL)
            return fail(-4, "spherical geometry needs walls on both axes");
        if (!(d->lo[0] > 0.0)) return fail(-1, "spherical geometry needs r > 0");
        if (!(d->lo[1] > 0.0) || !(d->hi[1] < 3.141592653589793))
            return fail(-1, "spherical geometry needs 0 < theta < pi");
        if (d->g[1] != 0.0) return fail(-4, "spherical geometry takes radial gravity only (g[1] = 0)");
        if (o->pc_solver != JFNK_PCS_MULTIGRID)
            return fail(-4, "spherical geometry supports the multigrid preconditioner only");
    }
    if (o->gmres_restart < 1 || o->gmres_restart > kMaxRestart) return fail(-1, "gmres_restart out of range");
    if (o->gmres_max_cycles < 0 || o->newton_max < 0) return fail(-1, "negative iteration limits");
    if (o->pc < JFNK_PC_NONE || o->pc > JFNK_PC_ACOUSTIC_DIFFUSION) return fail(-1, "unknown preconditioner");
    if (o->pc_solver != JFNK_PCS_MULTIGRID && o->pc_solver != JFNK_PCS_ADI) return fail(-1, "unknown pc_solver");
    if (o->mg_nu1 < 1 || o->mg_nu2 < 0 || o->mg_nuc < 1 || o->mg_cycles < 1 || o->mg_light_cells < 0)
        return fail(-1, "multigrid sweeps: nu1 >= 1, nu2 >= 0, nuc >= 1, cycles >= 1, light cells >= 0");
    if (o->prec != JFNK_FP64 && o->prec != JFNK_MIXED) return fail(-1, "unknown precision");
    if (!(o->cfl_hydro > 0.0)) return fail(-1, "cfl_hydro must be positive");
    if (o->max_halvings < 0) return fail(-1, "max_halvings must be >= 0");
    if (o->newton_target < 0) return fail(-1, "newton_target must be >= 0");
    if (o->scalar_converge != 0 && o->scalar_converge != 1) return fail(-1, "scalar_converge must be 0 or 1");
    if (o->gmres_forcing != JFNK_FORCING_FIXED && o->gmres_forcing != JFNK_FORCING_EW)
        return fail(-1, "unknown gmres_forcing");
    if (o->newton_extrapolate != 0 && o->newton_extrapolate != 1) return fail(-1, "newton_extrapolate must be 0 or 1");
    if (!(o->dt_grow == o->dt_grow)) return fail(-1, "dt_grow must be a number");
    return 0;
}

void make_grid(const jfnk_problem_desc& d, Grid& G) {
    std::memset(&G, 0, sizeof(G));
    G.ndim = d.ndim;
    for (int a = 0; a < 3; ++a) {
        G.n[a] = a < d.ndim ? d.n[a] : 1;
        G.bc[a] = a < d.ndim ? d.bc[a] : PERIODIC;
        const double lo = a < d.ndim ? d.lo[a] : 0.0, hi = a < d.ndim ? d.hi[a] : 1.0;
        G.dx[a] = (hi - lo) / G.n[a];
        G.idx[a] = 1.0 / G.dx[a];
        G.g[a] = a < d.ndim ? d.g[a] : 0.0;
        if (a < d.ndim && G.bc[a] == WALL) G.has_wall = 1;
    }
    G.N = (long)G.n[0] * G.n[1] * G.n[2];
    G.nvec = (2 + G.ndim) * G.N;
    G.stride[0] = 1;
    G.stride[1] = G.n[0];
    G.stride[2] = (long)G.n[0] * G.n[1];
    G.gamma = d.gamma;
    G.gm1 = d.gamma - 1.0;
    G.chi0 = d.chi0;
    G.has_chi = d.chi0 != 0.0;
    G.heat_balance = d.heat_balance && d.chi0 != 0.0;
    G.internal = d.energy_form == JFNK_ENERGY_INTERNAL ? 1 : 0;
    G.sph = d.geometry == JFNK_GEOM_SPHERICAL ? 1 : 0;
}

// entries of the spherical metric tables (SphMet): seven of n0, two of
// n0 + 1, three of n1, one of n1 + 1
long sph_table_len(const Grid& G) { return 7L * G.n[0] + 2L * (G.n[0] + 1) + 3L * G.n[1] + (G.n[1] + 1); }

// the metric tables on the host, in the order of SphMet's members
void sph_tables(const jfnk_problem_desc& d, const Grid& G, std::vector<double>& t) {
    const int nr = G.n[0], nt = G.n[1];
    const double dr = G.dx[0], dth = G.dx[1], r0 = d.lo[0], t0 = d.lo[1];
    std::vector<double> Vr(nr), rc(nr), ith(nr), hr2(nr), Vrc(nr, 0.0), r2c(nr), hr2c(nr, 0.0), r2f(nr + 1),
        rfa(nr + 1), Vt(nt), Vtc(nt, 0.0), stc(nt), stf(nt + 1);
    for (int i = 0; i <= nr; ++i) {
        const double r = r0 + i * dr;
        rfa[i] = r;
        r2f[i] = r * r;
    }
    for (int i = 0; i < nr; ++i) {
        const double a = rfa[i], b = rfa[i + 1];
        Vr[i] = (b * b * b - a * a * a) / 3.0;
        hr2[i] = 0.5 * (b * b - a * a);
        rc[i] = r0 + (i + 0.5) * dr;
        ith[i] = 1.0 / (rc[i] * dth);
        r2c[i] = rc[i] * rc[i];
    }
    for (int i = 1; i < nr; ++i) {
        const double a = rc[i - 1], b = rc[i];
        Vrc[i] = (b * b * b - a * a * a) / 3.0;
        hr2c[i] = 0.5 * (b * b - a * a);
    }
    for (int j = 0; j <= nt; ++j) stf[j] = std::sin(t0 + j * dth);
    for (int j = 0; j < nt; ++j) {
        Vt[j] = std::cos(t0 + j * dth) - std::cos(t0 + (j + 1) * dth);
        stc[j] = std::sin(t0 + (j + 0.5) * dth);
    }
    for (int j = 1; j < nt; ++j) Vtc[j] = std::cos(t0 + (j - 0.5) * dth) - std::cos(t0 + (j + 0.5) * dth);
    t.clear();
    for (const std::vector<double>* v : {&Vr, &rc, &ith, &hr2, &Vrc, &r2c, &hr2c, &r2f, &rfa, &Vt, &Vtc, &stc, &stf})
        t.insert(t.end(), v->begin(), v->end());
}

// point G.M into a device copy of the tables at dev (sph_table_len entries)
void sph_bind(Grid& G, const double* dev) {
    const long n0 = G.n[0], n1 = G.n[1];
    const double* q = dev;
    auto take = [&](long n) {
        const double* r = q;
        q += n;
        return r;
    };
    G.M.Vr = take(n0);
    G.M.rc = take(n0);
    G.M.ith = take(n0);
    G.M.hr2 = take(n0);
    G.M.Vrc = take(n0);
    G.M.r2c = take(n0);
    G.M.hr2c = take(n0);
    G.M.r2f = take(n0 + 1);
    G.M.rfa = take(n0 + 1);
    G.M.Vt = take(n1);
    G.M.Vtc = take(n1);
    G.M.stc = take(n1);
    G.M.stf = take(n1 + 1);
}

// multigrid depth: halve every active axis while all are even and >= 4
// multigrid levels: every active axis halves while all are even and >= 4
// (so only the coarsest level can have an odd axis)
int count_levels(const Grid& G, int n_out[][3]) {
    int n[3] = {G.n[0], G.n[1], G.n[2]}, L = 0;
    for (;;) {
        for (int a = 0; a < 3; ++a) n_out[L][a] = n[a];
        L++;
        bool ok = true;
        for (int a = 0; a < G.ndim; ++a)
            if (n[a] % 2 || n[a] < 4) ok = false;
        if (!ok || L >= kMaxLevels) break;
        for (int a = 0; a < G.ndim; ++a) n[a] /= 2;
    }
    return L;
}


// entries of a level's x, b and x2 arrays: room for the colour-split order
// (x-pairs merged, one slot per colour), which holds every natural index too
long level_xb_len(const int n[3]) { return 2L * ((n[0] + 1) / 2) * n[1] * n[2]; }
// a level's arrays: sig, a[0..2], D (N each), x and b (and x2 on the coarsest)
constexpr int kLevelCoefArrays = 5;
size_t level_bytes(const int n[3], bool coarsest, size_t rsize) {
    const long N = (long)n[0] * n[1] * n[2];
    return ((size_t)kLevelCoefArrays * N + (size_t)(coarsest ? 3 : 2) * level_xb_len(n)) * rsize;
}

// split: store x, b and x2 of the multi-block levels in colour-split order
template <typename R>
int alloc_levels(jfnk_problem* p, LevelSet<R>& S, LevelT<R>** dS, int nl[][3], bool unit_sig, bool split) {
    for (int l = 0; l < p->nlev; ++l) {
        LevelT<R>& L = S.L[l];
        L.unit_sig = unit_sig ? 1 : 0;
        for (int a = 0; a < 3; ++a) L.n[a] = nl[l][a];
        L.N = (long)L.n[0] * L.n[1] * L.n[2];
        // the single-workgroup coarse kernel takes its levels in natural order
        L.split = split && l < p->coarse_from ? 1 : 0;
        L.hn0 = (L.n[0] + 1) / 2;
        L.H = L.hn0 * L.n[1] * L.n[2];
        const bool coarsest = l == p->nlev - 1;
        const long xb = level_xb_len(L.n);
        R* blk = nullptr;
        CK(dalloc(p, &blk, level_bytes(L.n, coarsest, sizeof(R)) / sizeof(R)));
        L.sig = blk;
        L.a[0] = blk + L.N;
        L.a[1] = blk + 2 * L.N;
        L.a[2] = blk + 3 * L.N;
        L.D = blk + 4 * L.N;
        L.x = blk + kLevelCoefArrays * L.N;
        L.b = L.x + xb;
        L.x2 = coarsest ? L.b + xb : nullptr;
    }
    CK(dalloc(p, dS, (size_t)kMaxLevels));
    HIPCHK(hipMemcpyAsync(*dS, S.L, sizeof(LevelT<R>) * kMaxLevels, hipMemcpyHostToDevice, p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
    return 0;
}

// ---------------------------------------------------------------- reductions with read-back
int read_scalars(jfnk_problem* p, int off, int count, double* out) {
    HIPCHK(hipMemcpyAsync(p->hpin, p->dsum + off, sizeof(double) * count, hipMemcpyDeviceToHost, p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
    std::memcpy(out, p->hpin, sizeof(double) * count);
    if (g_prof) g_prof->drain();
    return 0;
}

// On short vectors the last reduction of a GMRES step also writes the
// step's scalars into the pinned area's second half (the mirror, at the same
// offsets as in dsum; its own result and the earlier ones copied from dsum),
// so that the read-back, whose latency is then most of the step, needs no
// copy launch: an event after the reduction, a wait for it, and the values
// are in host memory.  (The residual and time-step read-backs measured no
// better that way and keep the copy.)
double* mirror(jfnk_problem* p, int off) { return p->hpin + kDsum + off; }
int read_mirror(jfnk_problem* p, int off, int count, double* out) {
    HIPCHK(hipEventRecord(p->rb_event, p->stream));
    HIPCHK(hipEventSynchronize(p->rb_event));
    std::memcpy(out, mirror(p, off), sizeof(double) * count);
    if (g_prof) g_prof->drain();
    return 0;
}

// read-back of scalars with more work queued behind it: the copy, an event,
// then `after` (launches), and a wait for the event only, so that the device
// runs the queued work while the host takes the scalars
// vectors at least this long store the next basis vector during the read-back
constexpr long kOverlapStoreMin = 65536;
constexpr long kStoreRhsMaxCells = 1L << 18;
template <class After>
int read_scalars_then(jfnk_problem* p, int off, int count, double* out, After after) {
    HIPCHK(hipMemcpyAsync(p->hpin, p->dsum + off, sizeof(double) * count, hipMemcpyDeviceToHost, p->stream));
    HIPCHK(hipEventRecord(p->rb_event, p->stream));
    after();
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventSynchronize(p->rb_event));
    std::memcpy(out, p->hpin, sizeof(double) * count);
    return 0;
}

// installs the problem's profiler for the duration of an API call
struct ProfGuard {
    jfnk_problem* p;
    explicit ProfGuard(jfnk_problem* pp) : p(pp) { g_prof = (pp && pp->prof_on) ? &pp->prof : nullptr; }
    ~ProfGuard() {
        if (g_prof && p) {
            (void)hipStreamSynchronize(p->stream);
            g_prof->drain();
        }
        g_prof = nullptr;
    }
};

StateView view(jfnk_problem* p, const double* u, const double* v, const float* vf = nullptr) {
    StateView s;
    s.u = u;
    s.v = v;
    s.vf = vf;
    s.eps = p->dsum + D_EPS;
    for (int f = 0; f < 5; ++f) s.scale[f] = p->scale[f];
    s.N = p->G.N;
    return s;
}

// rout: R written there too (the Newton iterate's R for the products)
OutSpec outspec(jfnk_problem* p, int mode, double dt, double* out, double* out2, const double* b,
                const double* Ru, bool want_norm, double* rout = nullptr) {
    OutSpec o;
    o.mode = mode;
    o.h = 0.5 * dt;
    o.out = out;
    o.out2 = out2;
    o.b = b;
    o.Ru = Ru;
    o.rout = rout;
    o.neg_scaled = 0;
    for (int f = 0; f < 5; ++f) o.scale[f] = p->scale[f];
    o.partial = want_norm ? p->part : nullptr;
    for (int f = 0; f < 5; ++f) o.inv_scale[f] = 1.0 / p->scale[f];
    o.partial_u = nullptr;
    o.dotk = 0;
    o.dotv = nullptr;
    o.dotvf = nullptr;
    o.dot_part = nullptr;
    return o;
}

// residual evaluation at a Newton iterate: the norm partials, R kept for the
// products, the Newton right-hand side -S^-1 F written in place of F, and the
// partials of |S^-1 u|^2 for the products' difference step (summed into the
// device scalar by usq_from_residual)
OutSpec newton_spec(jfnk_problem* p, int mode, double dt, double* out, double* out2, const double* b) {
    OutSpec o = outspec(p, mode, dt, out, out2, b, nullptr, true, p->Ru);
    o.neg_scaled = 1;
    o.partial_u = p->part + p->ncell_blk;
    return o;
}
void usq_from_residual(jfnk_problem* p) {
    launch_final_sum(p->part + p->ncell_blk, p->ncell_blk, 1, p->dsum + D_USQ, p->stream);
}

// dt and limits of eqs. (5)-(7) for state u; sets the variable scales
int time_step(jfnk_problem* p, const double* u, double* dt_out) {
    const Grid& G = p->G;
    StateView s = view(p, u, nullptr);
    launch_prim(G, s, p->P, p->stream);
    launch_dt_partial(G, p->P, u, p->part, p->stream);
    launch_final_max(p->part, p->ncell_blk, 6, p->dsum + D_TMP, p->stream);
    HIPCHK(hipGetLastError());
    double m[6];
    CK(read_scalars(p, D_TMP, 6, m));
    const double hyd = m[0], adv = m[1], rad = m[2];
    const jfnk_solver_opts& o = p->opts;
    double dt = o.cfl_hydro / hyd;
    if (o.cfl_adv_max > 0.0 && adv > 0.0 && o.cfl_adv_max / adv < dt) dt = o.cfl_adv_max / adv;
    if (o.cfl_rad_max > 0.0 && rad > 0.0 && o.cfl_rad_max / rad < dt) dt = o.cfl_rad_max / rad;
    if (o.dt_max > 0.0 && o.dt_max < dt) dt = o.dt_max;
    p->scale[0] = m[3];
    p->scale[1] = m[4];
    for (int d = 0; d < G.ndim; ++d) p->scale[2 + d] = m[3] * m[5];
    for (int d = G.ndim; d < 3; ++d) p->scale[2 + d] = 1.0;
    p->hyd = hyd;
    p->adv = adv;
    p->rad = rad;
    if (dt_out) *dt_out = dt;
    return 0;
}

// sum of squares of F/S from the fused partials of the output sweep
int residual_norm(jfnk_problem* p, double* f) {
    launch_final_sum(p->part, p->ncell_blk, 1, p->dsum + D_TMP, p->stream);
    double s;
    CK(read_scalars(p, D_TMP, 1, &s));
    *f = std::sqrt(s);
    return 0;
}

// ---------------------------------------------------------------- preconditioner
template <typename R>
LevelSet<R>& levels(jfnk_problem* p, int which);
template <>
LevelSet<double>& levels<double>(jfnk_problem* p, int which) {
    return which == 0 ? p->ac64 : p->df64;
}
template <>
LevelSet<float>& levels<float>(jfnk_problem* p, int which) {
    return which == 0 ? p->ac32 : p->df32;
}

template <typename R>
void build_hierarchy(jfnk_problem* p, int which) {
    const Grid& G = p->G;
    LevelSet<R>& S = levels<R>(p, which);
    // the finest level of a Cartesian operator forms its couplings from one
    // cell field (enthalpy, or conductivity) in the sweeps; the stored arrays
    // serve the coarsening
    LevelT<R>& L0 = S.L[0];
    L0.qf = nullptr;
    if (!G.sph && (which == 0 || G.has_chi)) {
        const double tau = p->C.tau;
        L0.qf = which == 0 ? p->C.H : p->C.chi;
        launch_put_scalar(p->dsum + D_K0 + which, which == 0 ? (tau * tau) * G.gm1 : tau, p->stream);
        L0.K0 = p->dsum + D_K0 + which;
        for (int d = 0; d < 3; ++d) L0.i2[d] = d < G.ndim ? G.idx[d] * G.idx[d] : 0.0;
    }
    // D is built only without unit sigma: with sigma == 1 the sweeps form it
    // from the couplings
    const bool diag = !S.L[0].unit_sig;
    if (!(which == 0 && p->kap_in_level0)) launch_level0<R>(G, p->C, which, S.L[0], p->stream);
    if (diag) launch_level_diag<R>(G, S.L[0], p->stream);
    for (int l = 1; l < p->nlev; ++l) {
        launch_coarsen<R>(G, S.L[l - 1], S.L[l], p->stream);
        if (diag) launch_level_diag<R>(G, S.L[l], p->stream);
    }
}

// frozen coefficients at state u; prim_valid: the primitives in P are
// already those of u (the Newton loop has just evaluated the residual there)
int pc_build(jfnk_problem* p, const double* u, double dt, bool prim_valid) {
    const Grid& G = p->G;
    p->C.tau = 0.5 * dt;
    p->pc_rhs_formed = false;
    if (p->opts.pc == JFNK_PC_NONE) return 0;
    if (!prim_valid) launch_prim(G, view(p, u, nullptr), p->P, p->stream);
    launch_pc_coef(G, u, p->P, p->C, dt, p->opts.pc == JFNK_PC_ACOUSTIC_DIFFUSION, p->stream);
    if (p->opts.pc_solver == JFNK_PCS_MULTIGRID) {
        const bool diff = p->opts.pc == JFNK_PC_ACOUSTIC_DIFFUSION;
        if (p->opts.prec == JFNK_MIXED) {
            build_hierarchy<float>(p, 0);
            if (diff) build_hierarchy<float>(p, 1);
        } else {
            build_hierarchy<double>(p, 0);
            if (diff) build_hierarchy<double>(p, 1);
        }
    }
    HIPCHK(hipGetLastError());
    return 0;
}

template <typename R>
const LevelT<R>* dlevels(jfnk_problem* p, int which);
template <>
const LevelT<double>* dlevels<double>(jfnk_problem* p, int which) {
    return which == 0 ? p->dac64 : p->ddf64;
}
template <>
const LevelT<float>* dlevels<float>(jfnk_problem* p, int which) {
    return which == 0 ? p->dac32 : p->ddf32;
}

// the acoustic right-hand side kernels also form the first colour-0
// half-sweep of the finest level (multigrid on a Cartesian grid, whose
// finest level forms its couplings from the enthalpy, is a multi-block level
// and not the coarsest), and the first V-cycle skips that half-sweep
bool x0_with_rhs(const jfnk_problem* p) {
    return p->opts.pc_solver == JFNK_PCS_MULTIGRID && !p->G.sph && p->coarse_from > 0 && p->nlev > 1;
}

template <typename R>
void mg_launches(jfnk_problem* p, int which) {
    const LevelSet<R>& S = levels<R>(p, which);
    for (int c = 0; c < p->opts.mg_cycles; ++c)
        mg_vcycle<R>(p->G, S, dlevels<R>(p, which), p->nlev, p->coarse_from, p->opts.mg_nu1, p->opts.mg_nu2,
                     p->opts.mg_nuc, p->opts.mg_light_cells, c == 0, c == 0 && which == 0 && x0_with_rhs(p),
                     p->stream);
}

// The V-cycles' launches depend only on the problem (level arrays, sweep
// counts), never on values, so on a stream of its own the sequence is
// captured once into a graph and replayed; with kernel timing on, or on the
// legacy default stream (which cannot be captured), the launches are issued
// one by one.
template <typename R>
void mg_solve(jfnk_problem* p, int which) {
    const bool timed = g_prof && g_prof->mask;
    if (!p->stream || timed || !p->use_graphs) {
        mg_launches<R>(p, which);
        return;
    }
    hipGraphExec_t& ge = p->mg_exec[which];
    if (!ge) {
        hipGraph_t g = nullptr;
        if (hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            (void)hipGetLastError();
            mg_launches<R>(p, which);
            return;
        }
        mg_launches<R>(p, which);
        if (hipStreamEndCapture(p->stream, &g) != hipSuccess || !g) {
            (void)hipGetLastError();
            p->use_graphs = false;
            mg_launches<R>(p, which);
            return;
        }
        const hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            ge = nullptr;
            p->use_graphs = false;
            mg_launches<R>(p, which);
            return;
        }
    }
    if (hipGraphLaunch(ge, p->stream) != hipSuccess) {
        // nothing was queued: the launches go one by one from now on
        (void)hipGetLastError();
        (void)hipGraphExecDestroy(ge);
        ge = nullptr;
        p->use_graphs = false;
        mg_launches<R>(p, which);
    }
}

// z = S^-1 P^-1 S v, and the Jacobian-free step for the next product along z;
// v and z are vectors of the preconditioner's precision R
template <typename R>
void pc_apply_t(jfnk_problem* p, const R* v, R* z) {
    const Grid& G = p->G;
    Scales5 sc;
    for (int f = 0; f < 5; ++f) sc.v[f] = p->scale[f];
    const double* rE = nullptr;
    const bool mg = p->opts.pc_solver == JFNK_PCS_MULTIGRID;
    if (p->opts.pc == JFNK_PC_ACOUSTIC_DIFFUSION) {
        if (mg) {
            LevelSet<R>& S = levels<R>(p, 1);
            launch_field_to_level<R>(G, v + G.N, sc.v[1], S.L[0], p->stream);
            mg_solve<R>(p, 1);
            launch_pc_diff_back<R>(G, p->C, v, S.L[0], sc, p->rEd, p->stream);
        } else {
            // the conduction lines run in FP64 on an FP64 copy of r_E in both forms
            launch_field_scaled<R>(v + G.N, sc.v[1], p->rEd, G.N, p->stream);
            for (int d = 0; d < G.ndim; ++d) launch_line_solve<double>(G, p->C, d, 1, p->rEd, p->lines, p->stream);
        }
        rE = p->rEd;
    }
    LevelSet<R>& A = levels<R>(p, 0);
    if (!p->pc_rhs_formed) launch_pc_rhs<R>(G, p->C, v, rE, sc, A.L[0], x0_with_rhs(p), p->stream);
    p->pc_rhs_formed = false;
    const R* dp;
    if (mg) {
        mg_solve<R>(p, 0);
        dp = A.L[0].x;
    } else {
        for (int d = 0; d < G.ndim; ++d) launch_line_solve<R>(G, p->C, d, 0, A.L[0].b, p->lines, p->stream);
        dp = A.L[0].b;
    }
    launch_pc_back<R>(G, p->C, v, rE, dp, A.L[0], sc, z, p->part, p->ncell_blk, p->stream);
}

// T: double (FP64 form) or float (mixed form, whose Krylov basis and
// preconditioned basis are FP32)
template <typename T>
void pc_apply(jfnk_problem* p, const T* v, T* z) {
    int nb;
    if (p->opts.pc == JFNK_PC_NONE) {
        nb = p->nred;
        launch_copy_sumsq<T>(v, z, p->G.nvec, p->part, nb, p->stream);
    } else {
        nb = p->ncell_blk;
        pc_apply_t<T>(p, v, z);
    }
    launch_jv_eps(p->dsum + D_USQ, p->part, nb, (double)p->nunk, p->dsum + D_EPS, p->stream);
}

// Jacobian-free product along v (eps already on the device), Ru = R(u)
// With Vb (k <= kJvDotsMax basis vectors of the product's precision) the
// output sweep also forms the first orthogonalisation pass's per-block sums
// (V_i . w, then w . w) into p->part; returns their block count, else 0.
int jv(jfnk_problem* p, const double* u, const double* Ru, double dt, const double* v, double* w,
       const double* Vb = nullptr, int k = 0) {
    OutSpec o = outspec(p, OUT_JV, dt, w, nullptr, nullptr, Ru, false);
    if (Vb && k >= 1 && k <= kJvDotsMax) {
        o.dotk = k;
        o.dotv = Vb;
        o.dot_part = p->part;
    }
    launch_residual(p->G, view(p, u, v), p->P, p->Fx, p->W, p->sbal, o, p->stream);
    return o.dotk ? p->ncell_blk : 0;
}
int jv(jfnk_problem* p, const double* u, const double* Ru, double dt, const float* v, double* w,
       const float* Vb = nullptr, int k = 0) {
    OutSpec o = outspec(p, OUT_JV, dt, w, nullptr, nullptr, Ru, false);
    if (Vb && k >= 1 && k <= kJvDotsMax) {
        o.dotk = k;
        o.dotvf = Vb;
        o.dot_part = p->part;
    }
    launch_residual(p->G, view(p, u, nullptr, v), p->P, p->Fx, p->W, p->sbal, o, p->stream);
    return o.dotk ? p->ncell_blk : 0;
}

// eps for a product along x from |x|
void eps_for(jfnk_problem* p, const double* x) {
    launch_scaled_sumsq(x, p->G, nullptr, p->part, p->nred, p->stream);
    launch_jv_eps(p->dsum + D_USQ, p->part, p->nred, (double)p->nunk, p->dsum + D_EPS, p->stream);
}

// sum of (S^-1 u)^2 into the device scalar used by eps
void set_usq(jfnk_problem* p, const double* u) {
    double inv[5];
    for (int f = 0; f < 5; ++f) inv[f] = 1.0 / p->scale[f];
    launch_scaled_sumsq(u, p->G, inv, p->part, p->nred, p->stream);
    launch_final_sum(p->part, p->nred, 1, p->dsum + D_USQ, p->stream);
}

// |v|^2 (plain) read back
int plain_norm(jfnk_problem* p, const double* v, double* out) {
    launch_scaled_sumsq(v, p->G, nullptr, p->part, p->nred, p->stream);
    launch_final_sum(p->part, p->nred, 1, p->dsum + D_TMP, p->stream);
    double s;
    CK(read_scalars(p, D_TMP, 1, &s));
    *out = std::sqrt(s);
    return 0;
}

struct GmresInfo {
    int its = 0, cycles = 0, converged = 0;
    int finished = 0;  // the converged correction went to fin instead of x
    double res = 0.0, beta0 = 0.0;
};

// ---------------------------------------------------------------- GMRES(m), right preconditioned, CGS2
// Restarted GMRES on vectors of n doubles: basis V (T), classical
// Gram-Schmidt applied twice on the device, Givens rotations and the
// triangular solve on the host (one read-back per iteration, during which
// the device already stores the next basis vector).
//   norm(v, &out): the 2-norm of v (synchronises);
//   pc(j, v, z):   z_j = M^-1 v_j into Zb column j (not called when Zb is null:
//                  no preconditioner, the basis vectors themselves are used);
//                  v and z in the basis precision T;
//   op(z, w, V, k): w = A z for a preconditioned basis vector (precision T);
//                  may also form the first CGS2 pass against V_0..V_{k-1}
//                  (returns its partial-block count, or 0 when it did not);
//   opx(x, t):     t = A x for the restart residual.
// x += M^-1 V y is formed from the kept preconditioned vectors.
// rhs_norm >= 0: |rhs| as the caller already has it (no reduction and no
// read-back before the first basis vector); < 0: formed here.
//   fin(Z, k, acc): given the correction of a converged solve (Z, y on the
//                  device, acc: add to x), either consumes it in place of x
//                  and returns true (info->finished) or returns false;
//   store(w, v, hn, hnsq): the basis vector v = w / hn (hn given, or, with
//                  hnsq, sqrt of the sum there on the device).
// eta: the relative tolerance of this solve.
template <typename T, class Norm, class Pc, class Op, class OpX, class Fin, class Store>
int gmres_core(jfnk_problem* p, long n, T* V, T* Zb, const double* rhs, double* x, double* r, double* w,
               double* t, Norm norm, Pc pc, Op op, OpX opx, Fin fin, Store store, GmresInfo* info, double eta,
               double rhs_norm = -1.0) {
    const int m = p->opts.gmres_restart;
    std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m, 0.0), sn(m, 0.0), g(m + 1, 0.0), y(m, 0.0);
    // x starts at 0: the first cycle's correction is written, later ones added;
    // the residual of the first cycle is the right-hand side itself
    double beta0 = rhs_norm;
    if (!(beta0 >= 0.0)) CK(norm(rhs, &beta0));
    info->its = 0;
    info->cycles = 0;
    info->converged = 0;
    info->finished = 0;
    info->res = beta0;
    info->beta0 = beta0;
    if (beta0 == 0.0) {
        info->converged = 1;
        HIPCHK(hipMemsetAsync(x, 0, sizeof(double) * n, p->stream));
        return 0;
    }
    std::vector<double> hb(D_HN + 1);
    for (int cyc = 0; cyc < p->opts.gmres_max_cycles; ++cyc) {
        double beta = beta0;
        if (cyc > 0) CK(norm(r, &beta));
        info->res = beta;
        if (beta <= eta * beta0) {
            info->converged = 1;
            break;
        }
        info->cycles++;
        store(cyc == 0 ? rhs : r, V, beta, nullptr);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int kdim = 0;
        bool conv = false;
        // |g_j| and |g_{j-1}| of the least-squares residual before step j
        double res_j = beta, res_jm1 = 0.0;
        for (int j = 0; j < m; ++j) {
            const T* vj = V + (long)j * n;
            const T* zj = vj;
            if (Zb) {
                pc(j, vj, Zb + (long)j * n);
                zj = Zb + (long)j * n;
            }
            int nb = op(zj, w, V, j + 1);
            if (nb == 0) nb = launch_mdot<T>(V, n, j + 1, w, n, p->part, p->stream);
            launch_final_sum(p->part, nb, j + 2, p->dsum + D_H1, p->stream);
            nb = launch_update_mdot<T>(V, n, j + 1, p->dsum + D_H1, w, n, p->part, true, p->stream);
            launch_final_sum(p->part, nb, j + 1, p->dsum + D_H2, p->stream);
            nb = launch_update_mdot<T>(V, n, j + 1, p->dsum + D_H2, w, n, p->part, false, p->stream);
            T* vnext = V + (long)(j + 1) * n;
            const bool overlap = n >= kOverlapStoreMin;
            // short vectors: the scalars come back through the mirror (the
            // read-back's latency is the iteration's); long ones: copied
            // behind the reductions while the next basis vector is stored
            if (overlap)
                launch_final_sum(p->part, nb, 1, p->dsum + D_HN, p->stream);
            else
                launch_final_sum(p->part, nb, 1, p->dsum + D_HN, p->stream, mirror(p, D_HN), p->dsum + D_H1,
                                 mirror(p, D_H1), D_HN - D_H1);
            HIPCHK(hipGetLastError());
            // on long vectors the next basis vector is stored (from |w|^2 on
            // the device, the same bits as the host's division) while the
            // host takes the scalars, unless this step ends the cycle or is
            // expected to end the solve (the residual's last reduction
            // ratio, applied once more, reaches the tolerance): a vector
            // stored by a step that ends either is never read.  Otherwise,
            // and on short vectors (where the store is too brief to hide the
            // wait), the store follows the read-back when it is needed.
            const bool last = j == m - 1;
            bool spec = false;
            if (overlap) {
                const bool expect_end = res_jm1 > 0.0 && res_j * (res_j / res_jm1) <= eta * beta0;
                spec = !last && !expect_end;
                if (spec)
                    CK(read_scalars_then(p, 0, D_HN + 1, hb.data(), [&] { store(w, vnext, 0.0, p->dsum + D_HN); }));
                else
                    CK(read_scalars(p, 0, D_HN + 1, hb.data()));
            } else {
                CK(read_mirror(p, 0, D_HN + 1, hb.data()));
            }
            const double w0 = std::sqrt(hb[D_H1 + j + 1]);
            const double hn = std::sqrt(hb[D_HN]);
            for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hb[D_H1 + i] + hb[D_H2 + i];
            H[(size_t)(j + 1) * m + j] = hn;
            for (int i = 0; i < j; ++i) {
                const double a = H[(size_t)i * m + j], bb = H[(size_t)(i + 1) * m + j];
                H[(size_t)i * m + j] = cs[i] * a + sn[i] * bb;
                H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * bb;
            }
            const double a = H[(size_t)j * m + j], bb = H[(size_t)(j + 1) * m + j];
            const double den = std::sqrt(a * a + bb * bb);
            cs[j] = a / den;
            sn[j] = bb / den;
            H[(size_t)j * m + j] = den;
            H[(size_t)(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            info->its++;
            kdim = j + 1;
            info->res = std::fabs(g[j + 1]);
            if (hn <= 1e-14 * w0) {
                conv = true;
                break;
            }
            if (info->res <= eta * beta0) {
                conv = true;
                break;
            }
            if (!spec && !last) store(w, vnext, hn, nullptr);
            res_jm1 = res_j;
            res_j = info->res;
        }
        for (int i = kdim - 1; i >= 0; --i) {
            double s = g[i];
            for (int l = i + 1; l < kdim; ++l) s -= H[(size_t)i * m + l] * y[l];
            y[i] = s / H[(size_t)i * m + i];
        }
        std::memcpy(p->hpin, y.data(), sizeof(double) * kdim);
        HIPCHK(hipMemcpyAsync(p->dsum + D_Y, p->hpin, sizeof(double) * kdim, hipMemcpyHostToDevice, p->stream));
        // x += M^-1 V y, formed from the preconditioned vectors already at hand
        const T* Zs = Zb ? Zb : V;
        if (conv && fin(Zs, kdim, cyc > 0)) {
            info->finished = 1;
            info->converged = 1;
            break;
        }
        launch_combine<T>(Zs, n, kdim, p->dsum + D_Y, x, n, cyc > 0, p->stream);
        // no wait here: the Newton update queues behind the correction, and
        // the pinned slot that holds y is written again only after a later
        // read-back has drained the stream
        if (conv) {
            info->converged = 1;
            break;
        }
        opx(x, t);
        launch_sub(rhs, t, r, n, p->stream);
        CK(norm(r, &info->res));
    }
    HIPCHK(hipGetLastError());
    return 0;
}

// the flow's linear system in scaled variables, with the physics-based preconditioner
template <typename T>
int gmres(jfnk_problem* p, const double* u, double dt, GmresInfo* info, double eta, double rhs_norm) {
    const long n = p->G.nvec;
    auto norm = [&](const double* v, double* out) { return plain_norm(p, v, out); };
    auto pc = [&](int, const T* v, T* z) { pc_apply<T>(p, v, z); };
    auto op = [&](const T* z, double* w, const T* Vb, int k) { return jv(p, u, p->Ru, dt, z, w, Vb, k); };
    auto opx = [&](const double* x, double* t) {
        eps_for(p, x);
        jv(p, u, p->Ru, dt, x, t);
    };
    // a converged solve's correction goes straight into the Newton update
    // u += S x (and its max |S x / u| partials) without storing x
    auto fin = [&](const T* Z, int k, bool acc) {
        launch_combine_update<T>(Z, n, k, p->dsum + D_Y, p->x, acc, p->u, p->G, p->scale, p->part, p->nred,
                                 p->stream);
        return true;
    };
    // with the acoustic preconditioner alone each stored basis vector's
    // right-hand side for it is formed in the same pass, in the mixed form
    // and on FP64 grids of up to kStoreRhsMaxCells cells (on larger FP64
    // grids the fused pass, which divides each neighbour's entries by |w|
    // again, measured slower than the two launches)
    const bool rhs_with_store =
        p->opts.pc == JFNK_PC_ACOUSTIC && (sizeof(T) == sizeof(float) || p->G.N <= kStoreRhsMaxCells);
    auto store = [&](const double* src, T* dst, double hn, const double* hnsq) {
        if (rhs_with_store) {
            Scales5 sc;
            for (int f = 0; f < 5; ++f) sc.v[f] = p->scale[f];
            launch_store_pc_rhs<T>(p->G, p->C, src, dst, hn, hnsq, sc, levels<T>(p, 0).L[0], x0_with_rhs(p),
                                   p->stream);
            p->pc_rhs_formed = true;
        } else if (hnsq) {
            launch_store_scaled_dev<T>(src, dst, hnsq, n, p->stream);
        } else {
            launch_store_scaled<T>(src, dst, hn, n, p->stream);
        }
    };
    const int rc = gmres_core<T>(p, n, (T*)p->V, (T*)p->Zb, p->rhs, p->x, p->r, p->w, p->t, norm, pc, op, opx, fin,
                                 store, info, eta, rhs_norm);
    // a vector stored by a step that ended the solve is never preconditioned:
    // later applications form their own right-hand side
    p->pc_rhs_formed = false;
    return rc;
}

// Linear tolerance of Newton iteration k >= 1 under JFNK_FORCING_EW:
// Eisenstat and Walker's choice 2 (gamma 0.9, exponent 2) with Kelley's
// safeguards, from the residual norms f = |S^-1 F(u_k)| and f_prev of the
// last two iterates, the previous tolerance, the cap eta_max (gmres_eta)
// and the Newton tolerance tol.
double ew_forcing(double f, double f_prev, double eta_prev, double eta_max, double tol) {
    const double gamma = 0.9;
    const double ratio = f / f_prev;
    double eta = gamma * (ratio * ratio);
    const double keep = gamma * (eta_prev * eta_prev);  // no sudden drop of the tolerance
    if (keep > 0.1 && keep > eta) eta = keep;
    if (eta > eta_max) eta = eta_max;
    const double end = 0.5 * tol / f;  // no oversolving near the end
    if (end > eta) eta = end;
    if (eta > eta_max) eta = eta_max;
    return eta;
}

// Newton-Raphson from u^n at dt; on failure the state is restored.
// fresh: the caller has just evaluated the time step at u^n (the scales and
// the primitives in P are those of u^n)
int newton(jfnk_problem* p, double dt, jfnk_step_stats* st, bool fresh) {
    const Grid& G = p->G;
    const long n = G.nvec;
    const jfnk_solver_opts& o = p->opts;
    launch_copy(p->un, p->u, n, p->stream);
    if (!fresh) CK(time_step(p, p->u, nullptr));  // scales (and the primitives in P) from u^n
    launch_residual(G, view(p, p->u, nullptr), p->P, p->Fx, p->W, p->sbal,
                    newton_spec(p, OUT_CN_OLD, dt, p->b, p->rhs, nullptr), p->stream, true);
    usq_from_residual(p);
    HIPCHK(hipGetLastError());
    double f0;
    CK(residual_norm(p, &f0));
    double f = f0;
    double tol = o.newton_rtol * f0;
    const double floor_ = o.newton_atol * std::sqrt((double)p->nunk);
    if (floor_ > tol) tol = floor_;
    int status = 0, its = 0, gits = 0;
    double max_corr = 0.0;
    // optional extrapolated first iterate, kept when its residual is below
    // F(u^n)'s (the stopping test stays relative to F(u^n)); the residual's
    // outputs (right-hand side, R for the products, primitives, |S^-1 u|)
    // are those of the iterate Newton starts from
    int extrapolated = 0;
    double f_extrap = -1.0;
    if (o.newton_extrapolate && p->have_prev && std::isfinite(f0)) {
        launch_extrapolate(p->r, p->u, p->uprev, dt / p->dt_prev, n, p->stream);
        launch_residual(G, view(p, p->r, nullptr), p->P, p->Fx, p->W, p->sbal,
                        newton_spec(p, OUT_RESIDUAL, dt, p->rhs, nullptr, p->b), p->stream);
        usq_from_residual(p);
        CK(residual_norm(p, &f_extrap));
        if (f_extrap < f0) {
            launch_copy(p->u, p->r, n, p->stream);
            f = f_extrap;
            extrapolated = 1;
        } else {
            launch_residual(G, view(p, p->u, nullptr), p->P, p->Fx, p->W, p->sbal,
                            newton_spec(p, OUT_RESIDUAL, dt, p->rhs, nullptr, p->b), p->stream);
            usq_from_residual(p);
        }
    }
    double eta = o.gmres_eta, f_prev = f;
    if (!std::isfinite(f0)) status = 3;
    while (status == 0 && f > tol) {
        if (its >= o.newton_max) {
            status = 1;
            break;
        }
        if (o.gmres_forcing == JFNK_FORCING_EW && its > 0) eta = ew_forcing(f, f_prev, eta, o.gmres_eta, tol);
        // P holds the primitives of u from the residual just evaluated, and
        // the device scalar |S^-1 u|^2 was summed from the same sweep
        CK(pc_build(p, p->u, dt, true));
        GmresInfo gi;
        // the right-hand side -S^-1 F is the residual just measured: its norm
        // is f (the same squares, summed by the residual sweep's blocks)
        int rc = o.prec == JFNK_MIXED ? gmres<float>(p, p->u, dt, &gi, eta, f) : gmres<double>(p, p->u, dt, &gi, eta, f);
        if (rc) return rc;
        gits += gi.its;
        if (!gi.converged && gi.res >= 0.999 * gi.beta0) {
            status = 2;
            break;
        }
        if (!gi.finished) launch_update_state(p->u, p->x, G, p->scale, p->part, p->nred, p->stream);
        launch_final_max(p->part, p->nred, 1, p->dsum + D_TMP + 1, p->stream);
        launch_residual(G, view(p, p->u, nullptr), p->P, p->Fx, p->W, p->sbal,
                        newton_spec(p, OUT_RESIDUAL, dt, p->rhs, nullptr, p->b), p->stream);
        launch_final_sum(p->part, p->ncell_blk, 1, p->dsum + D_TMP, p->stream);
        usq_from_residual(p);
        HIPCHK(hipGetLastError());
        double rb[2];
        CK(read_scalars(p, D_TMP, 2, rb));
        f_prev = f;
        f = std::sqrt(rb[0]);
        max_corr = rb[1];
        its++;
        if (!std::isfinite(f)) {
            status = 3;
            break;
        }
        if (max_corr <= o.newton_corr_tol) break;
    }
    if (st) {
        st->newton_its = its;
        st->gmres_its = gits;
        st->f0 = f0;
        st->f = f;
        st->rel_res = f0 > 0.0 ? f / f0 : 0.0;
        st->max_rel_corr = max_corr;
        st->dt = dt;
        st->status = status;
        st->newton_exit = status != 0 ? -1 : (f > tol ? 1 : 0);
        st->extrapolated = extrapolated;
        st->f_extrap = f_extrap;
    }
    if (status != 0) launch_copy(p->u, p->un, n, p->stream);
    HIPCHK(hipGetLastError());
    return status;
}

// ---------------------------------------------------------------- passive scalars (section 2.2)
// After a converged step of the flow the scalars take a Crank-Nicolson step
// with the mass fluxes of u^n and u^{n+1}, solved by Jacobian-free
// Newton-Krylov without a preconditioner (the same tolerances as the flow),
// then are re-normalised so that the concentrations sum to one per cell.
ScalarArgs scalar_args(jfnk_problem* p, int mode, const double* rho, const double* fr, const double* s,
                       double* out, double h) {
    ScalarArgs A;
    A.ns = p->nscal;
    A.rho = rho;
    for (int d = 0; d < 3; ++d) A.fr[d] = d < p->G.ndim ? fr + (long)d * p->G.N : nullptr;
    A.s = s;
    A.v = nullptr;
    A.eps = p->dsum + D_SEPS;
    A.b = p->sb;
    A.Gs = p->sG;
    A.h = h;
    A.mode = mode;
    A.out = out;
    A.partial = mode == OUT_RESIDUAL ? p->part : nullptr;
    return A;
}

// 2-norm of a vector of n doubles
int vec_norm(jfnk_problem* p, const double* v, long n, double* out) {
    const int nb = launch_mdot<double>(v, n, 1, v, n, p->part, p->stream);
    launch_final_sum(p->part, nb, 1, p->dsum + D_TMP, p->stream);
    double s2;
    CK(read_scalars(p, D_TMP, 1, &s2));
    *out = std::sqrt(s2);
    return 0;
}

// flow_its: the Newton iterations of the flow's solve of this step (the
// scalars' count when they do not converge on their own)
int scalar_step(jfnk_problem* p, double dt, int flow_its) {
    const Grid& G = p->G;
    const long N = G.N, n = (long)p->nscal * N;
    const jfnk_solver_opts& o = p->opts;
    // density and mass fluxes of u^n and u^{n+1}
    launch_prim_flux(G, view(p, p->un, nullptr), p->P, p->Fx, p->W, p->stream);
    HIPCHK(hipMemcpyAsync(p->srho0, p->P.rho, sizeof(double) * N, hipMemcpyDeviceToDevice, p->stream));
    for (int d = 0; d < G.ndim; ++d)
        HIPCHK(hipMemcpyAsync(p->sfr0 + (long)d * N, p->Fx.fr[d], sizeof(double) * N, hipMemcpyDeviceToDevice,
                              p->stream));
    launch_prim_flux(G, view(p, p->u, nullptr), p->P, p->Fx, p->W, p->stream);
    HIPCHK(hipMemcpyAsync(p->srho1, p->P.rho, sizeof(double) * N, hipMemcpyDeviceToDevice, p->stream));
    for (int d = 0; d < G.ndim; ++d)
        HIPCHK(hipMemcpyAsync(p->sfr1 + (long)d * N, p->Fx.fr[d], sizeof(double) * N, hipMemcpyDeviceToDevice,
                              p->stream));
    launch_copy(p->sc_n, p->sc, n, p->stream);
    const double h = 0.5 * dt;
    launch_scalar_out(G, scalar_args(p, OUT_CN_OLD, p->srho0, p->sfr0, p->sc, p->sb, h), p->stream);
    auto residual = [&](double* g) {
        launch_scalar_out(G, scalar_args(p, OUT_RESIDUAL, p->srho1, p->sfr1, p->sc, p->sG, h), p->stream);
        launch_final_sum(p->part, p->ncell_blk, 1, p->dsum + D_TMP, p->stream);
        double g2;
        CK(read_scalars(p, D_TMP, 1, &g2));
        *g = std::sqrt(g2);
        return 0;
    };
    double g0;
    CK(residual(&g0));
    double g = g0, tol = o.newton_rtol * g0;
    const double floor_ = o.newton_atol * std::sqrt((double)n);
    if (floor_ > tol) tol = floor_;
    int status = 0, its = 0, gits = 0;
    if (!std::isfinite(g0)) status = 3;
    auto norm = [&](const double* v, double* out) { return vec_norm(p, v, n, out); };
    auto pc = [&](int, const double*, double*) {};
    // w = (G(s + eps v) - G(s)) / eps, eps = sqrt(2^-52)(1 + rms(s))/rms(v)
    auto op = [&](const double* v, double* w) {
        const int nb = launch_mdot<double>(v, n, 1, v, n, p->part, p->stream);
        launch_jv_eps(p->dsum + D_SUSQ, p->part, nb, (double)n, p->dsum + D_SEPS, p->stream);
        ScalarArgs A = scalar_args(p, OUT_JV, p->srho1, p->sfr1, p->sc, w, h);
        A.v = v;
        launch_scalar_out(G, A, p->stream);
    };
    const int nfix = flow_its > 1 ? flow_its : 1;
    while (status == 0 && (o.scalar_converge ? g > tol : (its < nfix && g > floor_))) {
        if (its >= o.newton_max) {
            status = 1;
            break;
        }
        const int nb = launch_mdot<double>(p->sc, n, 1, p->sc, n, p->part, p->stream);
        launch_final_sum(p->part, nb, 1, p->dsum + D_SUSQ, p->stream);
        launch_negate(p->sG, p->srhs, n, p->stream);
        GmresInfo gi;
        auto keep_x = [](const double*, int, bool) { return false; };
        auto store = [&](const double* src, double* dst, double hn, const double* hnsq) {
            if (hnsq) launch_store_scaled_dev<double>(src, dst, hnsq, n, p->stream);
            else launch_store_scaled<double>(src, dst, hn, n, p->stream);
        };
        auto op_dots = [&](const double* v, double* w, const double*, int) {
            op(v, w);
            return 0;
        };
        CK(gmres_core<double>(p, n, p->sV, nullptr, p->srhs, p->sx, p->sr, p->sw, p->stmp, norm, pc, op_dots, op,
                              keep_x, store, &gi, p->opts.gmres_eta));
        gits += gi.its;
        if (!gi.converged && gi.res >= 0.999 * gi.beta0) {
            status = 2;
            break;
        }
        launch_add(p->sc, p->sx, n, p->stream);
        CK(residual(&g));
        its++;
        if (!std::isfinite(g)) {
            status = 3;
            break;
        }
    }
    if (status == 0 && p->renorm && p->nscal > 1) launch_scalar_renorm(p->sc, p->srho1, p->nscal, N, p->stream);
    if (status != 0) launch_copy(p->sc, p->sc_n, n, p->stream);
    p->sc_newton = its;
    p->sc_gmres = gits;
    HIPCHK(hipGetLastError());
    return status;
}

// a step of the flow and then of the scalars at dt; on failure both are at u^n
int step_at(jfnk_problem* p, double dt, jfnk_step_stats* st, bool fresh = false) {
    int rc = newton(p, dt, st, fresh);
    p->sc_newton = p->sc_gmres = 0;
    if (rc == 0 && p->nscal > 0) {
        rc = scalar_step(p, dt, st ? st->newton_its : 1);
        if (rc != 0) launch_copy(p->u, p->un, p->G.nvec, p->stream);
        if (rc > 0 && st) st->status = rc;
    }
    if (rc == 0) {
        // an accepted step: u^n and its dt are the next extrapolation's past
        launch_copy(p->uprev, p->un, p->G.nvec, p->stream);
        p->dt_prev = dt;
        p->have_prev = true;
    }
    if (st) {
        st->scalar_newton_its = p->sc_newton;
        st->scalar_gmres_its = p->sc_gmres;
    }
    return rc;
}

// sums of rho and E (drift report), two-stage device reduction
int field_sums(jfnk_problem* p, const double* u, double* m, double* e) {
    const long N = p->G.N;
    launch_sum(u, N, p->part, p->nred, p->stream);
    launch_final_sum(p->part, p->nred, 1, p->dsum + D_TMP + 4, p->stream);
    launch_sum(u + N, N, p->part, p->nred, p->stream);
    launch_final_sum(p->part, p->nred, 1, p->dsum + D_TMP + 5, p->stream);
    HIPCHK(hipGetLastError());
    double r[2];
    CK(read_scalars(p, D_TMP + 4, 2, r));
    *m = r[0];
    *e = r[1];
    return 0;
}

int copy_in(jfnk_problem* p, double* dst, const double* src, int on_device) {
    HIPCHK(hipMemcpyAsync(dst, src, sizeof(double) * p->G.nvec,
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, p->stream));
    if (!on_device) HIPCHK(hipStreamSynchronize(p->stream));
    return 0;
}
int copy_out(jfnk_problem* p, double* dst, const double* src, int on_device) {
    HIPCHK(hipMemcpyAsync(dst, src, sizeof(double) * p->G.nvec,
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
    return 0;
}

// frozen wall conductive fluxes and heat-balance source from the creation state
int freeze_sources(jfnk_problem* p);

}  // namespace

// ---------------------------------------------------------------- sources (device kernels in this file)
namespace jfnk {
__global__ void k_wall_flux(Grid G, Prim P, int d, double* lo, double* hi) {
    const int r1 = (d + 1) % 3, r2 = (d + 2) % 3;
    const long nt = (long)G.n[r1] * G.n[r2];
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    Ijk q;
    q.v[r1] = (int)(t % G.n[r1]);
    q.v[r2] = (int)(t / G.n[r1]);
    const double hg = 0.5 * G.g[d] * G.dx[d];
    (void)hg;
    // bottom: ghost T = 2 T0 - T1 and chi of the ghost
    q.v[d] = 0;
    const long c0 = flat(G, q.v[0], q.v[1], q.v[2]);
    q.v[d] = 1;
    const long c1 = flat(G, q.v[0], q.v[1], q.v[2]);
    double Tg = 2.0 * P.T[c0] - P.T[c1];
    double chig = G.chi0 * (Tg * Tg * Tg);
    lo[t] = ((-0.5 * (chig + P.chi[c0])) * (P.T[c0] - Tg)) * face_ids(G, d, q.v[0]);
    q.v[d] = G.n[d] - 1;
    const long cn = flat(G, q.v[0], q.v[1], q.v[2]);
    q.v[d] = G.n[d] - 2;
    const long cm = flat(G, q.v[0], q.v[1], q.v[2]);
    Tg = 2.0 * P.T[cn] - P.T[cm];
    chig = G.chi0 * (Tg * Tg * Tg);
    hi[t] = ((-0.5 * (P.chi[cn] + chig)) * (Tg - P.T[cn])) * face_ids(G, d, q.v[0]);
}

// heat-balance source: + the divergence of the conductive flux, sum_d
// (f_T(up) - f_T(lo)) / dx (spherical: area-weighted over the cell volume)
__global__ void k_sbal(Grid G, Prim P, WallFlux W, double* sbal) {
    Ijk q;
    long c;
    if (!cell_from_launch(G, q, c)) return;
    double acc = 0.0;
    for (int d = 0; d < G.ndim; ++d) {
        double flo, fhi;
        if (G.bc[d] == WALL && q.v[d] == 0) {
            flo = W.lo[d] ? W.lo[d][transverse(G, q, d)] : 0.0;
        } else {
            const long l = shifted(G, q, d, -1);
            flo = ((-0.5 * (P.chi[l] + P.chi[c])) * (P.T[c] - P.T[l])) * face_ids(G, d, q.v[0]);
        }
        if (G.bc[d] == WALL && q.v[d] == G.n[d] - 1) {
            fhi = W.hi[d] ? W.hi[d][transverse(G, q, d)] : 0.0;
        } else {
            const long up = shifted(G, q, d, 1);
            fhi = ((-0.5 * (P.chi[c] + P.chi[up])) * (P.T[up] - P.T[c])) * face_ids(G, d, q.v[0]);
        }
        if (G.sph) {
            const int i = q.v[0], j = q.v[1];
            const double Alo = sph_area(G, d, i, j), Ahi = sph_area(G, d, d == 0 ? i + 1 : i, d == 1 ? j + 1 : j);
            acc = acc + (Ahi * fhi - Alo * flo) / sph_vol(G, i, j);
        } else {
            acc = acc + (fhi - flo) * G.idx[d];
        }
    }
    sbal[c] = acc;
}
}  // namespace jfnk

namespace {
int freeze_sources(jfnk_problem* p) {
    const Grid& G = p->G;
    launch_prim(G, view(p, p->u, nullptr), p->P, p->stream);
    for (int d = 0; d < G.ndim; ++d) {
        if (!p->W.lo[d]) continue;
        const int r1 = (d + 1) % 3, r2 = (d + 2) % 3;
        const long nt = (long)G.n[r1] * G.n[r2];
        {
            JFNK_PROF(KC_OTHER, p->stream);
            JFNK_KLAUNCH(k_wall_flux, dim3(grid_blocks(nt)), dim3(kBlock), 0, p->stream, G, p->P, d,
                               (double*)p->W.lo[d], (double*)p->W.hi[d]);
        }
    }
    {
        JFNK_PROF(KC_OTHER, p->stream);
        if (p->sbal) JFNK_KLAUNCH(k_sbal, cell_grid3(G.n), dim3(kBx, kBy), 0, p->stream, G, p->P, p->W, p->sbal);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(p->stream));
    return 0;
}

// device bytes create_problem requests (buffer for buffer)
size_t footprint(const Grid& G, const jfnk_solver_opts& o, int nlev, int nl[][3]) {
    const size_t nv = (size_t)G.nvec, N = (size_t)G.N;
    size_t b = 13 * nv * 8;                                                       // vectors
    b += (size_t)(o.gmres_restart + 1) * nv * (o.prec == JFNK_MIXED ? 4 : 8);    // basis
    b += (size_t)o.gmres_restart * nv * (o.prec == JFNK_MIXED ? 4 : 8);          // preconditioned basis
    b += 9 * N * 8 + (size_t)(2 * G.ndim + G.ndim * G.ndim) * N * 8;             // primitives, fluxes
    for (int d = 0; d < G.ndim; ++d)                                              // frozen wall fluxes
        if (G.bc[d] == WALL && G.has_chi) b += 2 * (size_t)G.n[(d + 1) % 3] * G.n[(d + 2) % 3] * 8;
    if (G.heat_balance) b += N * 8;                                               // heat-balance source
    if (G.sph) b += (size_t)sph_table_len(G) * 8;                                 // spherical metric
    b += 9 * N * 8 + N * 8 + 4 * N * 8;                                           // pc coefficients, rE, lines
    const size_t rs = o.prec == JFNK_MIXED ? 4 : 8;
    for (int l = 0; l < nlev; ++l) b += 2 * level_bytes(nl[l], l == nlev - 1, rs);  // two operators
    b += 2 * kMaxLevels * (o.prec == JFNK_MIXED ? sizeof(LevelT<float>) : sizeof(LevelT<double>));
    const size_t npart = (size_t)std::max(cell_blocks(G.n), kRedBlocks) * (kMaxRestart + 2);
    b += npart * 8 + kDsum * 8;
    return b;
}

}  // namespace

// ---------------------------------------------------------------- C-ABI
extern "C" {

void jfnk_default_opts(jfnk_solver_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->newton_rtol = 1e-8;
    o->newton_atol = 1e-14;
    o->newton_corr_tol = 1e-12;
    o->newton_max = 20;
    o->newton_target = 0;
    o->dt_grow = 0.0;
    o->scalar_converge = 1;
    o->gmres_restart = 30;
    o->gmres_max_cycles = 10;
    o->gmres_eta = 1e-2;
    o->pc = JFNK_PC_ACOUSTIC;
    o->pc_solver = JFNK_PCS_MULTIGRID;
    o->mg_nu1 = 2;
    o->mg_nu2 = 2;
    o->mg_nuc = 4;
    o->mg_cycles = 1;
    o->prec = JFNK_FP64;
    o->cfl_hydro = 1.0;
    o->max_halvings = 5;
}

const char* jfnk_last_error(void) { return g_err.c_str(); }

int jfnk_footprint_bytes(const jfnk_problem_desc* desc, const jfnk_solver_opts* opts, size_t* out) {
    int rc = validate(desc, opts);
    if (rc) return rc;
    if (!out) return fail(-1, "null output");
    Grid G;
    make_grid(*desc, G);
    int nl[kMaxLevels][3];
    const int nlev = count_levels(G, nl);
    *out = footprint(G, *opts, nlev, nl);
    return 0;
}

int jfnk_create_problem(const jfnk_problem_desc* desc, const jfnk_solver_opts* opts, const double* u0,
                        int on_device, void* hip_stream, jfnk_problem** out) {
    return jfnk::create_problem_in(desc, opts, u0, on_device, hip_stream, nullptr, 0, nullptr, out);
}
}  // extern "C"

namespace jfnk {
size_t problem_range_bytes(const jfnk_problem_desc* desc, const jfnk_solver_opts* opts) {
    size_t b = 0;
    if (jfnk_footprint_bytes(desc, opts, &b) != 0) return 0;
    return b + kSlabSlack;
}

int create_problem_in(const jfnk_problem_desc* desc, const jfnk_solver_opts* opts, const double* u0,
                      int on_device, void* hip_stream, void* range, size_t range_bytes, void* pinned_host,
                      jfnk_problem** out) {
    g_err.clear();
    int rc = validate(desc, opts);
    if (rc) return rc;
    if (!u0 || !out) return fail(-1, "null state or output pointer");
    jfnk_problem* p = new (std::nothrow) jfnk_problem();
    if (!p) return fail(-2, "host allocation failed");
    p->slab = (char*)range;
    p->slab_size = range ? range_bytes : 0;
    p->desc = *desc;
    p->opts = *opts;
    p->stream = (hipStream_t)hip_stream;
    make_grid(*desc, p->G);
    Grid& G = p->G;
    p->nunk = G.nvec;
    for (int d = 0; d < G.ndim; ++d)
        if (G.bc[d] == WALL) p->nunk -= G.N / G.n[d];
    if (G.nvec >= (1L << 31) / 2) {
        delete p;
        return fail(-4, "grid too large for 32-bit cell indexing");
    }
    if (hipGetDevice(&p->device) != hipSuccess) {
        delete p;
        return fail(-3, "hipGetDevice");
    }
    int nl[kMaxLevels][3];
    p->nlev = count_levels(G, nl);
    // the coarse kernel takes the deepest levels whose cells fit in its LDS
    // (none if the coarsest level alone does not: that level is then smoothed
    // by multi-block sweeps), and above them one level of more than
    // kCoarseMaxLevelCells and at most kCoarseBigCells cells, every axis
    // shorter than 1024 (not the coarsest, so every axis it has is even); the
    // kernel tells that level from the LDS levels by its size
    p->coarse_from = p->nlev;
    {
        long tail = 0;
        for (int l = p->nlev - 1; l >= 0; --l) {
            tail += (long)nl[l][0] * nl[l][1] * nl[l][2];
            if (tail > kCoarseLdsCells || (long)nl[l][0] * nl[l][1] * nl[l][2] > kCoarseMaxLevelCells) break;
            p->coarse_from = l;
        }
        const int l = p->coarse_from - 1;
        const long nc = l >= 0 ? (long)nl[l][0] * nl[l][1] * nl[l][2] : 0;
        if (p->coarse_from < p->nlev && l >= 0 && nc > kCoarseMaxLevelCells && nc <= kCoarseBigCells &&
            nl[l][0] < 1024 && nl[l][1] < 1024 && nl[l][2] < 1024)
            p->coarse_from = l;
    }
    p->ncell_blk = cell_blocks(G.n);
    p->nred = std::min(kRedBlocks, grid_blocks(G.nvec));
    p->npart = std::max(p->ncell_blk, kRedBlocks) * (kMaxRestart + 2);
    const long n = G.nvec, N = G.N;
    auto cleanup = [&](int code) {
        delete p;
        return code;
    };
#define AL(ptr, cnt)                     \
    do {                                 \
        int r_ = dalloc(p, &(ptr), (cnt)); \
        if (r_) return cleanup(r_);      \
    } while (0)
    AL(p->u, n); AL(p->un, n); AL(p->b, n); AL(p->x, n); AL(p->rhs, n); AL(p->r, n); AL(p->Ru, n);
    AL(p->w, n); AL(p->t, n); AL(p->z, n); AL(p->s1, n); AL(p->s2, n); AL(p->uprev, n);
    if (opts->prec == JFNK_MIXED) {
        float* V = nullptr;
        AL(V, (size_t)(opts->gmres_restart + 1) * n);
        p->V = V;
    } else {
        double* V = nullptr;
        AL(V, (size_t)(opts->gmres_restart + 1) * n);
        p->V = V;
    }
    if (opts->prec == JFNK_MIXED) {
        float* Z = nullptr;
        AL(Z, (size_t)opts->gmres_restart * n);
        p->Zb = Z;
    } else {
        double* Z = nullptr;
        AL(Z, (size_t)opts->gmres_restart * n);
        p->Zb = Z;
    }
    double* prim = nullptr;
    AL(prim, (size_t)9 * N);
    p->P.rho = prim;
    for (int d = 0; d < 3; ++d) p->P.uf[d] = prim + (1 + d) * N;
    p->P.p = prim + 4 * N;
    p->P.eps = prim + 5 * N;
    p->P.T = prim + 6 * N;
    p->P.chi = prim + 7 * N;
    p->P.q = prim + 8 * N;
    double* flux = nullptr;
    const int nphi = G.ndim * G.ndim;
    AL(flux, (size_t)(2 * G.ndim + nphi) * N);
    for (int d = 0; d < G.ndim; ++d) {
        p->Fx.fr[d] = flux + d * N;
        p->Fx.fe[d] = flux + (G.ndim + d) * N;
    }
    {
        double* ph = flux + 2 * G.ndim * N;
        for (int d = 0; d < G.ndim; ++d) {
            p->Fx.phic[d] = ph;
            ph += N;
            for (int e = 0; e < G.ndim; ++e) {
                if (e == d) continue;
                p->Fx.phie[d][e] = ph;
                ph += N;
            }
        }
    }
    for (int d = 0; d < G.ndim; ++d) {
        if (G.bc[d] == WALL && G.has_chi) {
            const int r1 = (d + 1) % 3, r2 = (d + 2) % 3;
            const long nt = (long)G.n[r1] * G.n[r2];
            double* wl = nullptr;
            AL(wl, (size_t)2 * nt);
            p->W.lo[d] = wl;
            p->W.hi[d] = wl + nt;
        }
    }
    if (G.heat_balance) AL(p->sbal, N);
    if (G.sph) {
        double* met = nullptr;
        AL(met, (size_t)sph_table_len(G));
        std::vector<double> tab;
        sph_tables(*desc, G, tab);
        if (hipMemcpyAsync(met, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice, p->stream) !=
                hipSuccess ||
            hipStreamSynchronize(p->stream) != hipSuccess)
            return cleanup(fail(-3, "copy of the spherical metric"));
        sph_bind(p->G, met);
    }
    double* pcb = nullptr;
    AL(pcb, (size_t)9 * N);
    for (int d = 0; d < 3; ++d) {
        p->C.kap[d] = pcb + d * N;
        p->C.beta[d] = pcb + (3 + d) * N;
    }
    p->C.W = pcb + 6 * N;
    p->C.H = pcb + 7 * N;
    p->C.chi = pcb + 8 * N;
    AL(p->rEd, N);
    AL(p->lines, (size_t)4 * N);
    const bool split = opts->pc_solver == JFNK_PCS_MULTIGRID;
    if (opts->prec == JFNK_MIXED) {
        if ((rc = alloc_levels<float>(p, p->ac32, &p->dac32, nl, !G.sph, split))) return cleanup(rc);
        if ((rc = alloc_levels<float>(p, p->df32, &p->ddf32, nl, false, split))) return cleanup(rc);
    } else {
        if ((rc = alloc_levels<double>(p, p->ac64, &p->dac64, nl, !G.sph, split))) return cleanup(rc);
        if ((rc = alloc_levels<double>(p, p->df64, &p->ddf64, nl, false, split))) return cleanup(rc);
        if (!G.sph) {
            // the finest acoustic level's couplings are C.kap itself; its
            // sigma (1) is written once here, from zeroed couplings
            LevelT<double>& L0 = p->ac64.L[0];
            for (int d = 0; d < G.ndim; ++d) p->C.kap[d] = L0.a[d];
            p->kap_in_level0 = true;
            for (int d = 0; d < G.ndim; ++d)
                if (hipMemsetAsync(L0.a[d], 0, sizeof(double) * N, p->stream) != hipSuccess)
                    return cleanup(fail(-3, "memset"));
            launch_level0<double>(G, p->C, 0, L0, p->stream);
        }
    }
    AL(p->part, (size_t)p->npart);
    AL(p->dsum, (size_t)kDsum);
#undef AL
    static_assert(kPinnedBytes == 2 * sizeof(double) * kDsum, "read-back area size: staging and mirror");
    if (pinned_host) {
        p->hpin = (double*)pinned_host;
    } else {
        hipError_t e = hipHostMalloc((void**)&p->hpin, kPinnedBytes, hipHostMallocDefault);
        if (e != hipSuccess) return cleanup(fail(-2, "hipHostMalloc failed"));
        p->own_hpin = true;
    }
    if (hipEventCreateWithFlags(&p->rb_event, hipEventDisableTiming) != hipSuccess)
        return cleanup(fail(-3, "hipEventCreateWithFlags"));
    if (hipMemsetAsync(p->dsum, 0, sizeof(double) * kDsum, p->stream) != hipSuccess) return cleanup(fail(-3, "memset"));
    if ((rc = copy_in(p, p->u, u0, on_device))) return cleanup(rc);
    launch_zero_walls(p->u, G, p->stream);
    if ((rc = freeze_sources(p))) return cleanup(rc);
    *out = p;
    return 0;
}
int set_error(int code, const char* msg) { return fail(code, msg ? msg : ""); }
}  // namespace jfnk

extern "C" {

int jfnk_destroy_problem(jfnk_problem* p) {
    if (!p) return 0;
    (void)hipStreamSynchronize(p->stream);
    p->prof.release();
    delete p;
    return 0;
}

int jfnk_set_state(jfnk_problem* p, const double* u, int on_device) {
    if (!p || !u) return fail(-1, "null argument");
    int rc = copy_in(p, p->u, u, on_device);
    if (rc) return rc;
    launch_zero_walls(p->u, p->G, p->stream);
    HIPCHK(hipStreamSynchronize(p->stream));
    p->have_prev = false;
    return 0;
}

int jfnk_get_state(jfnk_problem* p, double* u, int on_device) {
    if (!p || !u) return fail(-1, "null argument");
    return copy_out(p, u, p->u, on_device);
}

int jfnk_set_scalars(jfnk_problem* p, int nscal, int renormalize, const double* s, int on_device) {
    if (!p || nscal < 0 || (nscal > 0 && !s)) return fail(-1, "bad scalar arguments");
    if (p->slab) return fail(-4, "passive scalars need their own device memory (not a caller-provided range)");
    if (p->G.sph && nscal > 0) return fail(-4, "passive scalars are for Cartesian grids");
    HIPCHK(hipStreamSynchronize(p->stream));
    for (void* q : p->sbuf.ptrs) (void)hipFree(q);
    p->sbuf.ptrs.clear();
    p->sbuf.bytes = 0;
    p->nscal = 0;
    if (nscal == 0) return 0;
    const long N = p->G.N, n = (long)nscal * N;
    const int m = p->opts.gmres_restart;
    auto al = [&](double** out, size_t count) {
        void* q = nullptr;
        if (hipMalloc(&q, count * sizeof(double)) != hipSuccess) return fail(-2, "hipMalloc (scalars)");
        p->sbuf.ptrs.push_back(q);
        p->sbuf.bytes += count * sizeof(double);
        *out = (double*)q;
        return 0;
    };
    double** vecs[] = {&p->sc, &p->sc_n, &p->sb, &p->sG, &p->sx, &p->srhs, &p->sr, &p->sw, &p->stmp};
    for (double** v : vecs) CK(al(v, (size_t)n));
    CK(al(&p->sV, (size_t)(m + 1) * n));
    CK(al(&p->srho0, (size_t)N));
    CK(al(&p->srho1, (size_t)N));
    CK(al(&p->sfr0, (size_t)3 * N));
    CK(al(&p->sfr1, (size_t)3 * N));
    HIPCHK(hipMemcpyAsync(p->sc, s, sizeof(double) * n, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                          p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
    p->nscal = nscal;
    p->renorm = renormalize ? 1 : 0;
    return 0;
}

int jfnk_get_scalars(jfnk_problem* p, double* s, int on_device) {
    if (!p || !s) return fail(-1, "null argument");
    if (p->nscal == 0) return 0;
    HIPCHK(hipMemcpyAsync(s, p->sc, sizeof(double) * (long)p->nscal * p->G.N,
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
    return 0;
}

int jfnk_set_time(jfnk_problem* p, double t) {
    if (!p) return fail(-1, "null problem");
    p->t_now = t;
    return 0;
}

int jfnk_set_opts(jfnk_problem* p, const jfnk_solver_opts* opts) {
    if (!p) return fail(-1, "null problem");
    int rc = validate(&p->desc, opts);
    if (rc) return rc;
    if (opts->prec != p->opts.prec || opts->gmres_restart > p->opts.gmres_restart)
        return fail(-1, "precision and a larger restart need a new problem");
    p->opts = *opts;
    p->dt_ctrl = 0.0;
    // the captured multigrid sequence depends on the sweep options
    (void)hipStreamSynchronize(p->stream);
    for (auto& g : p->mg_exec) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
    return 0;
}

int jfnk_newton_solve(jfnk_problem* p, double dt, jfnk_step_stats* out) {
    if (!p) return fail(-1, "null problem");
    ProfGuard guard(p);
    if (!(dt > 0.0)) return fail(-1, "dt must be positive");
    auto t0 = std::chrono::steady_clock::now();
    jfnk_step_stats st;
    std::memset(&st, 0, sizeof(st));
    double m0, e0;
    int rc = field_sums(p, p->u, &m0, &e0);
    if (rc) return rc;
    rc = step_at(p, dt, &st);
    if (rc < 0) return rc;
    if (rc == 0) {
        p->t_now += dt;
        double m1, e1;
        int r2 = field_sums(p, p->u, &m1, &e1);
        if (r2) return r2;
        st.mass_drift = (m1 - m0) / m0;
        st.energy_drift = (e1 - e0) / e0;
    }
    st.cfl_hydro = dt * p->hyd;
    st.cfl_adv = dt * p->adv;
    st.cfl_rad = dt * p->rad;
    st.t = p->t_now;
    st.status = rc;
    st.wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (out) *out = st;
    return rc;
}

int jfnk_implicit_step(jfnk_problem* p, jfnk_step_stats* out) {
    if (!p) return fail(-1, "null problem");
    ProfGuard guard(p);
    auto t0 = std::chrono::steady_clock::now();
    jfnk_step_stats st;
    std::memset(&st, 0, sizeof(st));
    double dt;
    int rc = time_step(p, p->u, &dt);
    if (rc) return rc;
    const double hyd = p->hyd, adv = p->adv, rad = p->rad;
    const bool ctrl = p->opts.dt_grow > 1.0;
    // the controller's bound on dt (section 2.1: dt adjusted for efficiency
    // within the user's CFL limits, the most restrictive applying)
    if (ctrl && p->dt_ctrl > 0.0 && p->dt_ctrl < dt) dt = p->dt_ctrl;
    int rej = 0;
    for (;;) {
        // the first attempt starts from the time step just evaluated at u^n;
        // a retry re-evaluates it (the failed attempt overwrote P)
        rc = step_at(p, dt, &st, rej == 0);
        if (rc < 0) return rc;
        if (rc == 0 || rej >= p->opts.max_halvings) break;
        rej++;
        dt = 0.5 * dt;
    }
    if (ctrl) {
        if (rc == 0) {
            double f = p->opts.dt_grow;
            if (p->opts.newton_target > 0 && st.newton_its > 0) {
                const double r = (double)p->opts.newton_target / (double)st.newton_its;
                f = r < 0.5 ? 0.5 : (r > p->opts.dt_grow ? p->opts.dt_grow : r);
            }
            p->dt_ctrl = dt * f;
        } else {
            p->dt_ctrl = dt;
        }
    }
    if (rc == 0) p->t_now += dt;
    st.rejections = rej;
    st.dt = dt;
    st.cfl_hydro = dt * hyd;
    st.cfl_adv = dt * adv;
    st.cfl_rad = dt * rad;
    st.t = p->t_now;
    st.status = rc;
    HIPCHK(hipStreamSynchronize(p->stream));
    st.wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (out) *out = st;
    return rc;
}

int jfnk_eval_rhs(jfnk_problem* p, const double* u, double* R, int on_device) {
    if (!p || !u || !R) return fail(-1, "null argument");
    ProfGuard guard(p);
    int rc = copy_in(p, p->s1, u, on_device);
    if (rc) return rc;
    launch_residual(p->G, view(p, p->s1, nullptr), p->P, p->Fx, p->W, p->sbal,
                    outspec(p, OUT_RHS, 0.0, p->s2, nullptr, nullptr, nullptr, false), p->stream);
    HIPCHK(hipGetLastError());
    return copy_out(p, R, p->s2, on_device);
}

int jfnk_eval_cn_old(jfnk_problem* p, const double* un, double dt, double* b, int on_device) {
    if (!p || !un || !b) return fail(-1, "null argument");
    ProfGuard guard(p);
    int rc = copy_in(p, p->s1, un, on_device);
    if (rc) return rc;
    launch_residual(p->G, view(p, p->s1, nullptr), p->P, p->Fx, p->W, p->sbal,
                    outspec(p, OUT_CN_OLD, dt, p->s2, p->t, nullptr, nullptr, false), p->stream);
    HIPCHK(hipGetLastError());
    return copy_out(p, b, p->s2, on_device);
}

int jfnk_eval_residual(jfnk_problem* p, const double* u, const double* b, double dt, double* F, int on_device) {
    if (!p || !u || !b || !F) return fail(-1, "null argument");
    ProfGuard guard(p);
    int rc = copy_in(p, p->s1, u, on_device);
    if (rc) return rc;
    rc = copy_in(p, p->s2, b, on_device);
    if (rc) return rc;
    launch_residual(p->G, view(p, p->s1, nullptr), p->P, p->Fx, p->W, p->sbal,
                    outspec(p, OUT_RESIDUAL, dt, p->t, nullptr, p->s2, nullptr, false), p->stream);
    HIPCHK(hipGetLastError());
    return copy_out(p, F, p->t, on_device);
}

int jfnk_eval_time_step(jfnk_problem* p, const double* u, double* out9, int on_device) {
    if (!p || !u || !out9) return fail(-1, "null argument");
    ProfGuard guard(p);
    int rc = copy_in(p, p->s1, u, on_device);
    if (rc) return rc;
    double dt;
    rc = time_step(p, p->s1, &dt);
    if (rc) return rc;
    out9[0] = dt;
    out9[1] = p->hyd;
    out9[2] = p->adv;
    out9[3] = p->rad;
    for (int f = 0; f < 5; ++f) out9[4 + f] = p->scale[f];
    return 0;
}

int jfnk_eval_diagnostics(jfnk_problem* p, const double* u, int on_device, double rho_light, double rho_heavy,
                          int mix_axis, jfnk_diagnostics* out) {
    if (!p || !out) return fail(-1, "null argument");
    const Grid& G = p->G;
    if (G.sph) return fail(-4, "diagnostics are for Cartesian grids");
    if (mix_axis >= G.ndim || mix_axis < -1) return fail(-1, "mix_axis must be -1 or a grid axis");
    if (mix_axis >= 0 && !(rho_heavy != rho_light)) return fail(-1, "rho_heavy must differ from rho_light");
    if (mix_axis >= 0 && 4L * p->ncell_blk + G.n[mix_axis] > (long)p->npart)
        return fail(-4, "too many layers for the reduction buffer");
    ProfGuard guard(p);
    const double* src = p->u;
    if (u) {
        int rc = copy_in(p, p->s1, u, on_device);
        if (rc) return rc;
        src = p->s1;
    }
    launch_prim(G, view(p, src, nullptr), p->P, p->stream);
    const double* scal = (!u && p->nscal >= 2) ? p->sc : nullptr;  // the scalars belong to the problem's state
    launch_diagnostics(G, p->P, src, mix_axis, rho_light, rho_heavy, scal, p->part, p->dsum + D_TMP, p->stream);
    HIPCHK(hipGetLastError());
    double m[6] = {0, 0, 0, 0, 0, 0};
    CK(read_scalars(p, D_TMP, mix_axis < 0 ? 4 : (scal ? 6 : 5), m));
    double dv = 1.0;
    for (int d = 0; d < G.ndim; ++d) dv *= G.dx[d];
    out->kinetic = m[0] * dv;
    out->mass = m[1] * dv;
    out->energy = m[2] * dv;
    out->max_mach = m[3];
    out->mix_width = mix_axis >= 0 ? m[4] * G.dx[mix_axis] : 0.0;
    out->mix_width_scalars = (mix_axis >= 0 && scal) ? m[5] * G.dx[mix_axis] : 0.0;
    return 0;
}

int jfnk_velocity_error(jfnk_problem* p, const double* u_low, const double* u_high, int on_device, int ratio,
                        int axis, double* out) {
    if (!p || !u_high || !out) return fail(-1, "null argument");
    const Grid& G = p->G;
    if (G.sph) return fail(-4, "the eq. (17) error is for Cartesian grids");
    if (ratio < 1 || ratio > 1024) return fail(-1, "ratio must lie in 1..1024");
    if (axis < 0 || axis >= G.ndim) return fail(-1, "axis must be a grid axis");
    Grid Gh = G;
    Gh.N = 1;
    for (int d = 0; d < 3; ++d) {
        if (d < G.ndim) Gh.n[d] = G.n[d] * ratio;
        Gh.N *= Gh.n[d];
    }
    Gh.nvec = (long)(2 + G.ndim) * Gh.N;
    if (Gh.nvec >= (1L << 31)) return fail(-4, "high-resolution grid too large for 32-bit cell indexing");
    ProfGuard guard(p);
    const double* lo = p->u;
    if (u_low) {
        int rc = copy_in(p, p->s1, u_low, on_device);
        if (rc) return rc;
        lo = p->s1;
    }
    const double* hi = u_high;
    double* tmp = nullptr;
    if (!on_device) {
        if (hipMalloc(&tmp, sizeof(double) * Gh.nvec) != hipSuccess) return fail(-2, "hipMalloc (high-resolution state)");
        if (hipMemcpyAsync(tmp, u_high, sizeof(double) * Gh.nvec, hipMemcpyHostToDevice, p->stream) != hipSuccess) {
            (void)hipFree(tmp);
            return fail(-3, "copy of the high-resolution state");
        }
        hi = tmp;
    }
    launch_vel_error(G, Gh, lo, hi, ratio, axis, p->part, p->dsum + D_TMP, p->stream);
    double r[2] = {0.0, 0.0};
    int rc = hipGetLastError() == hipSuccess ? read_scalars(p, D_TMP, 2, r) : fail(-3, "vel_error launch");
    if (tmp) (void)hipFree(tmp);
    if (rc) return rc;
    *out = r[1] > 0.0 ? r[0] / r[1] : 0.0;
    return 0;
}

int jfnk_velocity_error_noalloc(jfnk_problem* p, const double* u_low, const double* u_high, int ratio, int axis,
                                double* out) {
    if (!p || !u_high || !out) return fail(-1, "null argument");
    const Grid& G = p->G;
    if (G.sph) return fail(-4, "the eq. (17) error is for Cartesian grids");
    if (ratio < 1 || ratio > 1024) return fail(-1, "ratio must lie in 1..1024");
    if (axis < 0 || axis >= G.ndim) return fail(-1, "axis must be a grid axis");
    Grid Gh = G;
    Gh.N = 1;
    for (int d = 0; d < 3; ++d) {
        if (d < G.ndim) Gh.n[d] = G.n[d] * ratio;
        Gh.N *= Gh.n[d];
    }
    Gh.nvec = (long)(2 + G.ndim) * Gh.N;
    if (Gh.nvec >= (1L << 31)) return fail(-4, "high-resolution grid too large for 32-bit cell indexing");
    const long need = noalloc_vel_error_doubles(G);
    if (need > kNoallocScratchDoubles)
        return fail(-4, "grid too large for the allocation-free scratch (" + std::to_string(need) +
                            " doubles needed, at most " + std::to_string(kNoallocScratchDoubles) + ")");
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != p->device)
        return fail(-1, "the problem's device must be the current device");
    ProfGuard guard(p);
    // one call at a time per process: the scratch is shared by every call on
    // a device, and the lock is held until the result has been read back
    std::lock_guard<std::mutex> lk(noalloc_scratch_lock());
    double* scr = nullptr;
    int rc = noalloc_scratch(p->device, &scr);
    if (rc) return fail(rc, "hipGetSymbolAddress (allocation-free scratch)");
    const double* lo = u_low ? u_low : p->u;
    launch_vel_error_scratch(G, Gh, lo, u_high, ratio, axis, scr, p->stream);
    HIPCHK(hipGetLastError());
    // the pinned read-back slot of the problem is free: its last use was synchronised
    HIPCHK(hipStreamSynchronize(p->stream));
    HIPCHK(hipMemcpyAsync(p->hpin, scr + (need - 2), 2 * sizeof(double), hipMemcpyDeviceToHost, p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
    const double e = p->hpin[0], a = p->hpin[1];
    *out = a > 0.0 ? e / a : 0.0;
    return 0;
}

int jfnk_set_scales(jfnk_problem* p, const double* s5) {
    if (!p || !s5) return fail(-1, "null argument");
    for (int f = 0; f < 5; ++f) {
        if (!(s5[f] > 0.0)) return fail(-1, "scales must be positive");
        p->scale[f] = s5[f];
    }
    return 0;
}

int jfnk_apply_jv(jfnk_problem* p, const double* u, const double* b, double dt, const double* v, double* w,
                  int on_device) {
    if (!p || !u || !b || !v || !w) return fail(-1, "null argument");
    ProfGuard guard(p);
    int rc;
    if ((rc = copy_in(p, p->s1, u, on_device))) return rc;
    if ((rc = copy_in(p, p->s2, b, on_device))) return rc;
    if ((rc = copy_in(p, p->z, v, on_device))) return rc;
    launch_residual(p->G, view(p, p->s1, nullptr), p->P, p->Fx, p->W, p->sbal,
                    outspec(p, OUT_RESIDUAL, dt, p->w, nullptr, p->s2, nullptr, false, p->Ru), p->stream);
    set_usq(p, p->s1);
    eps_for(p, p->z);
    jv(p, p->s1, p->Ru, dt, p->z, p->w);
    HIPCHK(hipGetLastError());
    return copy_out(p, w, p->w, on_device);
}

int jfnk_apply_jv_eps(jfnk_problem* p, const double* u, const double* b, double dt, const double* v, double eps,
                      double* w, int on_device) {
    if (!p || !u || !b || !v || !w) return fail(-1, "null argument");
    if (!(eps > 0.0) || !std::isfinite(eps)) return fail(-1, "eps must be positive and finite");
    ProfGuard guard(p);
    int rc;
    if ((rc = copy_in(p, p->s1, u, on_device))) return rc;
    if ((rc = copy_in(p, p->s2, b, on_device))) return rc;
    if ((rc = copy_in(p, p->z, v, on_device))) return rc;
    launch_residual(p->G, view(p, p->s1, nullptr), p->P, p->Fx, p->W, p->sbal,
                    outspec(p, OUT_RESIDUAL, dt, p->w, nullptr, p->s2, nullptr, false, p->Ru), p->stream);
    // the pinned staging slot is free: every earlier read-back has completed
    HIPCHK(hipStreamSynchronize(p->stream));
    p->hpin[0] = eps;
    HIPCHK(hipMemcpyAsync(p->dsum + D_EPS, p->hpin, sizeof(double), hipMemcpyHostToDevice, p->stream));
    jv(p, p->s1, p->Ru, dt, p->z, p->w);
    HIPCHK(hipGetLastError());
    return copy_out(p, w, p->w, on_device);
}

int jfnk_apply_precond(jfnk_problem* p, const double* u, double dt, const double* v, double* z, int on_device) {
    if (!p || !u || !v || !z) return fail(-1, "null argument");
    ProfGuard guard(p);
    if (!(dt > 0.0)) return fail(-1, "dt must be positive");
    int rc;
    if ((rc = copy_in(p, p->s1, u, on_device))) return rc;
    if ((rc = copy_in(p, p->s2, v, on_device))) return rc;
    if ((rc = pc_build(p, p->s1, dt, false))) return rc;
    HIPCHK(hipMemsetAsync(p->dsum + D_USQ, 0, sizeof(double), p->stream));
    if (p->opts.prec == JFNK_MIXED) {
        // the mixed form's preconditioner maps FP32 vectors: v rounded into
        // basis column 0, z from column 1 (the basis is idle between solves)
        float* V = (float*)p->V;
        const long n = p->G.nvec;
        launch_store_scaled<float>(p->s2, V, 1.0, n, p->stream);
        pc_apply<float>(p, V, V + n);
        launch_widen<float>(V + n, p->w, n, p->stream);
    } else {
        pc_apply<double>(p, p->s2, p->w);
    }
    HIPCHK(hipGetLastError());
    return copy_out(p, z, p->w, on_device);
}

static const char* kClassNames[KC_COUNT] = {
    "residual_prim", "residual_flux", "residual_mflux", "residual_out", "cgs2_dot", "cgs2_update_dot", "cgs2_update_norm",
    "basis_store", "basis_combine", "mg_smooth", "mg_restrict", "mg_prolong", "mg_coarse", "pc_rhs",
    "pc_back", "pc_build", "reduce", "adi_lines", "other"};

int jfnk_profile_enable(jfnk_problem* p, unsigned class_mask) {
    if (!p) return fail(-1, "null problem");
    p->prof.mask = class_mask;
    p->prof_on = class_mask != 0;
    for (int c = 0; c < KC_COUNT; ++c) {
        p->prof.ms[c] = 0.0;
        p->prof.count[c] = 0;
        p->prof.bytes[c] = 0.0;
        p->prof.seen[c] = 0;
    }
    p->prof.left = 0;
    p->prof.lcg = 0;
    return 0;
}

int jfnk_profile_sample(jfnk_problem* p, int period, int burst) {
    if (!p) return fail(-1, "null problem");
    if (period < 1 || burst < 1 || burst > period) return fail(-1, "need 1 <= burst <= period");
    p->prof.period = (unsigned)period;
    p->prof.burst = (unsigned)burst;
    p->prof.left = 0;
    p->prof.lcg = 0;
    return 0;
}

int jfnk_profile_read(jfnk_problem* p, double* ms, long long* count, double* bytes, int nclass) {
    if (!p || !ms || !count || !bytes) return fail(-1, "null argument");
    HIPCHK(hipStreamSynchronize(p->stream));
    p->prof.drain();
    for (int c = 0; c < nclass; ++c) {
        ms[c] = c < KC_COUNT ? p->prof.ms[c] : 0.0;
        count[c] = c < KC_COUNT ? p->prof.count[c] : 0;
        bytes[c] = c < KC_COUNT ? p->prof.bytes[c] : 0.0;
        if (c < KC_COUNT) {
            p->prof.ms[c] = 0.0;
            p->prof.count[c] = 0;
            p->prof.bytes[c] = 0.0;
        }
    }
    return KC_COUNT;
}

const char* jfnk_profile_class_name(int cls) {
    return cls >= 0 && cls < KC_COUNT ? kClassNames[cls] : "";
}

}  // extern "C"
