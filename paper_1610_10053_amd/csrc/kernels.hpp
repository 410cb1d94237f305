// Kernel-side data views and the host launchers of every kernel of the
// implicit-step library.
#pragma once

#include <mutex>

#include "jfnk_internal.hpp"

namespace jfnk {

struct Scales5 {
    double v[5];
};

// A state, optionally perturbed along v: u + (eps * scale[f]) * v, with the
// step eps read from device memory (v may be null).
struct StateView {
    const double* u;
    const double* v;    // FP64 direction, or
    const float* vf;    // FP32 direction (the mixed form's preconditioned basis); at most one is set
    const double* eps;
    double scale[5];
    long N;
};

// Cell primitives and face velocities of one state.
struct Prim {
    double* rho;
    double* uf[3];
    double* p;
    double* eps;
    double* T;
    double* chi;
    double* q;
};

// Mass and total-energy fluxes on the lower face of each cell, per axis, and
// the momentum transport fluxes: phic[d] cell-centred flux of m_d along d,
// phie[d][e] (e != d) flux of m_d along e at the lower e-edge of the d-face.
struct Flux {
    double* fr[3];
    double* fe[3];
    double* phic[3];
    double* phie[3][3];
};

// Frozen conductive fluxes through the lower/upper wall of each wall axis,
// indexed by the transverse position (null when absent).
struct WallFlux {
    const double* lo[3];
    const double* hi[3];
};

enum OutMode : int { OUT_RHS = 0, OUT_CN_OLD = 1, OUT_RESIDUAL = 2, OUT_JV = 3 };

struct OutSpec {
    int mode;
    double h;            // dt / 2
    double* out;         // R, b, F or w
    double* out2;        // F (OUT_CN_OLD)
    const double* b;     // Crank-Nicolson old-time term
    const double* Ru;    // R(u) for OUT_JV
    double* rout;        // R written here as well (any mode), or null
    int neg_scaled;      // the F output holds -F/S (the Newton right-hand side) instead of F
    double scale[5];     // variable scales for the fused norm
    double* partial;     // per-block sum of (F/S)^2, or null
    double inv_scale[5]; // 1/S for the state's own norm
    double* partial_u;   // per-block sum of (u/S)^2 (OUT_CN_OLD, OUT_RESIDUAL), or null
    // OUT_JV: the first pass of the orthogonalisation against the dotk
    // (<= kJvDotsMax) basis vectors at dotv (FP64) or dotvf (FP32), leading
    // dimension the vector length: per-block sums of V_i . w (columns i) and
    // w . w (column dotk) into dot_part, column-major over the blocks
    int dotk;
    const double* dotv;
    const float* dotvf;
    double* dot_part;
};
constexpr int kJvDotsMax = 4;

// residual.hip
// prim_valid: P already holds the primitives of the (unperturbed) state
void launch_residual(const Grid& G, const StateView& s, const Prim& P, const Flux& Fx, const WallFlux& W,
                     const double* sbal, const OutSpec& o, hipStream_t stream, bool prim_valid = false);
void launch_prim(const Grid& G, const StateView& s, const Prim& P, hipStream_t stream);
void launch_dt_partial(const Grid& G, const Prim& P, const double* u, double* part, hipStream_t stream);
// passive scalars: residual consumers of s_k = c_k rho under the mass fluxes
// fr and density rho of a flow state (modes OUT_CN_OLD, OUT_RESIDUAL, OUT_JV)
struct ScalarArgs {
    int ns;
    const double* rho;
    const double* fr[3];
    const double* s;
    const double* v;    // direction (OUT_JV) or null
    const double* eps;  // device scalar (OUT_JV)
    const double* b;    // old-time term (OUT_RESIDUAL, OUT_JV)
    const double* Gs;   // G(s) (OUT_JV)
    double h;
    int mode;
    double* out;
    double* partial;    // block sums of out^2 (OUT_RESIDUAL) or null
};
void launch_scalar_out(const Grid& G, const ScalarArgs& A, hipStream_t stream);
void launch_scalar_renorm(double* s, const double* rho, int ns, long N, hipStream_t stream);
void launch_negate(const double* in, double* out, long n, hipStream_t stream);
// primitives and lower-face fluxes of a state (the first two residual sweeps)
void launch_prim_flux(const Grid& G, const StateView& s, const Prim& P, const Flux& Fx, const WallFlux& W,
                      hipStream_t stream);

// diagnostics of the state whose primitives P hold: out5 = sum kin, sum rho,
// sum E (per unit volume), max Mach, sum of the layers' X_M along axis (or
// untouched when axis < 0), and with two passive scalars scal (or null) the
// sum of their layers' 2 min(<c1>, <c2>); part needs 4 cell_blocks + n[axis]
// doubles
int launch_diagnostics(const Grid& G, const Prim& P, const double* u, int axis, double rho_l, double rho_h,
                       const double* scal, double* part, double* out5, hipStream_t stream);
// eq. (17) sums for velocity component axis: out2 = sum |v_low - <v_high>|,
// sum |<v_high>| over the cells of Gl; Gh is r times finer on every active
// axis; part needs 2 cell_blocks(Gl.n) doubles
void launch_vel_error(const Grid& Gl, const Grid& Gh, const double* ul, const double* uh, int r, int axis,
                      double* part, double* out2, hipStream_t stream);
// allocation-free form: partial sums and the two final sums (at
// scr + 2 * blocks) in the caller-given scratch of noalloc_vel_error_doubles(Gl)
constexpr long kNoallocScratchDoubles = 32768;
constexpr int kNoallocMaxDevices = 64;
int noalloc_scratch(int device, double** ptr);
std::mutex& noalloc_scratch_lock();
long noalloc_vel_error_doubles(const Grid& Gl);
void launch_vel_error_scratch(const Grid& Gl, const Grid& Gh, const double* ul, const double* uh, int r, int axis,
                              double* scr, hipStream_t stream);

// krylov.hip: deterministic two-stage reductions and Krylov vector kernels
// partial layout: part[col * nblk + block]
// dst[0] = v, ordered on the stream
void launch_put_scalar(double* dst, double v, hipStream_t stream);
// host (or null): pinned host memory that receives a copy of the ncol
// results; xsrc[0, xn) (earlier device results) is copied to xhost as well
void launch_final_sum(const double* part, int nblk, int ncol, double* out, hipStream_t stream,
                      double* host = nullptr, const double* xsrc = nullptr, double* xhost = nullptr, int xn = 0);
void launch_final_max(const double* part, int nblk, int ncol, double* out, hipStream_t stream);
void launch_scaled_sumsq(const double* x, const Grid& G, const double* inv_scale5, double* part, int nblk,
                         hipStream_t stream);
// the multi-dot launchers return the number of blocks (partials per column)
template <typename T>
int launch_mdot(const T* V, long ld, int k, const double* w, long n, double* part, hipStream_t stream);
template <typename T>
int launch_update_mdot(const T* V, long ld, int k, const double* h, double* w, long n, double* part,
                       bool want_dots, hipStream_t stream);
template <typename T>
void launch_store_scaled(const double* w, T* v, double hn, long n, hipStream_t stream);
// v = w / sqrt(hnsq[0]), hnsq in device memory
template <typename T>
void launch_store_scaled_dev(const double* w, T* v, const double* hnsq, long n, hipStream_t stream);
template <typename T>
void launch_combine(const T* V, long ld, int k, const double* y, double* t, long n, bool acc, hipStream_t stream);
void launch_add(double* x, const double* z, long n, hipStream_t stream);
void launch_sub(const double* a, const double* b, double* r, long n, hipStream_t stream);
template <typename T>
void launch_combine_update(const T* V, long ld, int k, const double* y, const double* x, bool acc, double* u,
                           const Grid& G, const double* scale5, double* part, int nblk, hipStream_t stream);
// out = a + r (a - b)
void launch_extrapolate(double* out, const double* a, const double* b, double r, long n, hipStream_t stream);
void launch_update_state(double* u, const double* x, const Grid& G, const double* scale5, double* part,
                         int nblk, hipStream_t stream);
void launch_copy(double* dst, const double* src, long n, hipStream_t stream);
void launch_zero_walls(double* u, const Grid& G, hipStream_t stream);
void launch_sum(const double* x, long n, double* part, int nblk, hipStream_t stream);
template <typename T>
void launch_widen(const T* v, double* out, long n, hipStream_t stream);

// precond.hip
// One level of the geometric multigrid hierarchy of an operator
//   (M x)_c = sig_c x_c + sum over faces f of c of a_f (x_c - x_neighbour(f))
// in precision R (FP64, or FP32 in the mixed form).
constexpr int kMaxLevels = 16;
// x and b of the levels solved by the single-workgroup coarse kernel live in
// LDS: at most this many cells over those levels, and at most
// kCoarseMaxLevelCells (one per thread) in each
constexpr int kCoarseLdsCells = 1408;
constexpr int kCoarseMaxLevelCells = 1024;
// above those levels the coarse kernel may take one more level of at most
// this many cells (its x in LDS, its coefficients in registers)
constexpr int kCoarseBigCells = 4096;
template <typename R>
struct LevelT {
    int n[3];
    long N;
    R* sig;   // diagonal mass term
    R* a[3];  // face couplings on the lower face of each cell (0 on walls)
    R* D;     // sig + sum of the cell's couplings
    R* x;
    R* b;
    R* x2;         // second iterate buffer (coarsest level only, else null)
    int unit_sig;  // sig == 1 on every cell (acoustic operator): D is formed from the couplings
    // x, b and x2 of a multi-block level are stored split by colour: the cells
    // of colour (i+j+k)&1 together, x-pairs merged (H entries per colour,
    // hn0 per row), so that a half-sweep reads and writes them contiguously
    int split, hn0, H;
    // finest level of a Cartesian operator: the couplings are formed on the
    // fly from one cell field, a_d = (K0 ((qf_lo + qf_c) / 2)) i2_d on the
    // lower face (bitwise the stored a), so a sweep reads one array instead
    // of ndim; null on other levels.  K0 (which changes with dt) is read from
    // device memory, so that a captured launch sequence stays valid
    const double* qf;
    const double* K0;
    double i2[3];
};
// coupling on the face between cells lo and c of a level with qf set
template <typename R>
__device__ __forceinline__ R qf_coupling(const LevelT<R>& L, int d, int lo, int c) {
    return (R)((L.K0[0] * (0.5 * (L.qf[lo] + L.qf[c]))) * L.i2[d]);
}
// index of cell (i, j, k) in a level's x, b and x2 arrays (levels hold fewer
// than 2^30 cells)
template <typename R>
__device__ __forceinline__ int xbi(const LevelT<R>& L, int i, int j, int k) {
    const int row = j + L.n[1] * k;
    if (!L.split) return i + L.n[0] * row;
    return ((i + j + k) & 1) * L.H + (i >> 1) + L.hn0 * row;
}
template <typename R>
struct LevelSet {
    LevelT<R> L[kMaxLevels];
};

struct PcCoef {
    double* H;        // cell enthalpy (E + p) / rho; the face value is the mean of the two cells'
    double* chi;      // cell conductivity (with a conduction operator)
    double* kap[3];   // acoustic couplings tau^2 (gamma-1) h_f / dx^2
    double* beta[3];  // conduction couplings tau chi_f / dx^2
    double* W;        // (gamma-1)/rho
    double tau;
};

// diff: the conduction block's beta and W are formed too
void launch_pc_coef(const Grid& G, const double* u, const Prim& P, const PcCoef& C, double dt, bool diff,
                    hipStream_t stream);
// which = 0: acoustic operator (sig = 1, a = kap); 1: conduction (sig = 1/W, a = beta)
template <typename R>
void launch_level0(const Grid& G, const PcCoef& C, int which, const LevelT<R>& L0, hipStream_t stream);
template <typename R>
void launch_coarsen(const Grid& G, const LevelT<R>& F, const LevelT<R>& C, hipStream_t stream);
template <typename R>
void launch_level_diag(const Grid& G, const LevelT<R>& L, hipStream_t stream);
// V-cycles on b of level 0; levels >= coarse_from run in one single-block
// kernel; levels (not the coarsest) of at most `light` cells take V(1,1)
template <typename R>
// x0: the finest level's first colour-0 half-sweep values are already in x
// (formed with the right-hand side); the first cycle skips that half-sweep
void mg_vcycle(const Grid& G, const LevelSet<R>& S, const LevelT<R>* Ld, int nlev, int coarse_from, int nu1, int nu2,
               int nuc, int light, bool first, bool x0, hipStream_t stream);

// The preconditioner's input v and output z are vectors of the
// preconditioner's precision R (FP64; the mixed form's FP32 Krylov basis and
// preconditioned basis); its arithmetic outside the elliptic solves is FP64.
// r_p = (gamma-1)(r_E - tau D(h_f r_m)) with r = S v; r_E from rE if given
template <typename R>
void launch_store_pc_rhs(const Grid& G, const PcCoef& C, const double* w, R* v, double hn, const double* hnsq,
                         Scales5 sc, const LevelT<R>& L0, bool x0, hipStream_t stream);
// x0: also the first multigrid half-sweep's colour-0 values from x = 0 (the
// finest level's couplings formed from its cell field, unit sigma)
template <typename R>
void launch_pc_rhs(const Grid& G, const PcCoef& C, const R* v, const double* rE, Scales5 sc,
                   const LevelT<R>& L0, bool x0, hipStream_t stream);
// conduction block: rE = S_E v_E + tau D(chi_f G s)
template <typename R>
void launch_pc_diff_back(const Grid& G, const PcCoef& C, const R* v, const LevelT<R>& L0, Scales5 sc,
                         double* rE, hipStream_t stream);
// dm = r_m - tau G dp, drho = r_rho - tau D dm, dE = r_E - tau D(h_f dm),
// z = S^-1 delta (stored in precision R) and per-block |z|^2 of the stored values
template <typename R>
void launch_pc_back(const Grid& G, const PcCoef& C, const R* v, const double* rE, const R* dp,
                    const LevelT<R>& L0, Scales5 sc, R* z, double* part, int nblk, hipStream_t stream);
// out = s * v for a cell field v of the preconditioner's vector precision R
template <typename R>
void launch_field_scaled(const R* v, double s, double* out, long N, hipStream_t stream);
// L0.b = s * v (a cell field) in precision R, in the level's x/b order
template <typename R>
void launch_field_to_level(const Grid& G, const R* v, double s, const LevelT<R>& L0, hipStream_t stream);
// z = v and per-block |z|^2 (no preconditioner)
template <typename T>
void launch_copy_sumsq(const T* v, T* z, long n, double* part, int nblk, hipStream_t stream);
// eps of the Jacobian-free product from sum (S^-1 u)^2 and sum v^2
void launch_jv_eps(const double* usumsq, const double* part_v, int nblk, double nunk, double* eps,
                   hipStream_t stream);

// ADI: solve every line along axis d of the acoustic (kind 0) or conduction
// (kind 1) operator in place; scratch4 holds 4 N doubles
template <typename R>
void launch_line_solve(const Grid& G, const PcCoef& C, int d, int kind, R* x, double* scratch4,
                       hipStream_t stream);

}  // namespace jfnk
