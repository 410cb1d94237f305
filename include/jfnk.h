/*
 * jfnk.h -- C-ABI of the MI355X implicit-step library.
 *
 * One Crank-Nicolson implicit time step of the compressible Euler equations
 * with gravity and thermal (radiative) conduction, solved by Jacobian-free
 * Newton-Krylov with a physics-based preconditioner, after Goffrey et al.,
 * "Benchmarking the Multi-dimensional Stellar Implicit Code MUSIC"
 * (arXiv:1610.10053), section 2:
 *   - equations (1)-(3), discretised in total-energy conservative form or,
 *     on request, with the internal-energy variable of eq. (2) as written;
 *     ideal-gas closure, conductivity chi = chi0 T^3 (stand-in for eq. 4);
 *   - staggered grid: rho and E at cell centres, momentum on cell faces;
 *     upstream linear reconstruction limited by van Leer;
 *   - ghost-cell boundaries: periodic, or reflecting/stress-free walls with
 *     linearly extrapolated temperature and hydrostatic ghost density
 *     (section 3.1) and a constant-luminosity wall energy flux (section 6);
 *   - Crank-Nicolson in time, Newton-Raphson, restarted GMRES, Jacobian-free
 *     matrix-vector products, a semi-implicit physics-based preconditioner
 *     that treats sound waves (and optionally thermal diffusion) implicitly;
 *   - time step from the CFL numbers of eqs. (5)-(7), the most restrictive
 *     constraint applying (section 2.1).
 *
 * Conventions
 *   - Every function returns int: 0 success; > 0 solver outcome
 *     (1 Newton did not converge, 2 GMRES stagnated, 3 non-finite residual);
 *     < 0 usage or system error (-1 bad argument, -2 out of device memory,
 *     -3 HIP runtime error, -4 unsupported configuration).  jfnk_last_error()
 *     returns a thread-local message describing the last failure.
 *   - State layout: one array of (2 + ndim) * N doubles, N = n[0]*n[1]*n[2]:
 *     rho, E (or rho e), m_x, m_y (, m_z) one after another, each in C order with x
 *     fastest (index i + n0*(j + n1*k)).  m_d at index c is the momentum on
 *     the lower face of cell c along d.  Along a wall direction the face with
 *     i_d = 0 is the wall: its entry must be 0, stays 0 and is not an unknown.
 *   - Pointers flagged on_device = 1 are device (HIP) pointers on the
 *     problem's device; on_device = 0 means host memory.  The library copies
 *     in and out; callers keep ownership of their buffers.
 *   - All device work is enqueued on the HIP stream given at creation
 *     (NULL = the default stream).  Calls that return host values
 *     synchronise that stream.  A problem may be used by one host thread at
 *     a time.
 */
#ifndef JFNK_H
#define JFNK_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { JFNK_BC_PERIODIC = 0, JFNK_BC_WALL = 1 };
enum { JFNK_PC_NONE = 0, JFNK_PC_ACOUSTIC = 1, JFNK_PC_ACOUSTIC_DIFFUSION = 2 };
enum { JFNK_PCS_MULTIGRID = 0, JFNK_PCS_ADI = 1 };
enum { JFNK_FP64 = 0, JFNK_MIXED = 1 };
enum { JFNK_ENERGY_TOTAL = 0, JFNK_ENERGY_INTERNAL = 1 };
enum { JFNK_GEOM_CARTESIAN = 0, JFNK_GEOM_SPHERICAL = 1 };

/* Problem: grid, boundaries, gas and forces (section 2). */
typedef struct {
    int ndim;          /* 2 or 3 */
    int n[3];          /* cells per axis (n[2] = 1 in 2D); periodic axes need even n >= 4 */
    double lo[3], hi[3];
    int bc[3];         /* JFNK_BC_PERIODIC or JFNK_BC_WALL (both ends of an axis) */
    double gamma;      /* ideal-gas ratio of specific heats, p = rho T */
    double g[3];       /* constant gravitational acceleration (body force) */
    double chi0;       /* conductivity chi = chi0 T^3 (0: no conduction) */
    int heat_balance;  /* 1: add the time-independent source that cancels the
                          conductive divergence of the creation state */
    int energy_form;   /* JFNK_ENERGY_TOTAL: energy variable E, total-energy
                          conservative form; JFNK_ENERGY_INTERNAL: rho e,
                          eq. (2) as written (flux rho e u, -p div u at cell
                          centres, no gravitational work) */
    int geometry;      /* JFNK_GEOM_CARTESIAN, or JFNK_GEOM_SPHERICAL: 2D
                          (r, theta) with azimuthal symmetry (section 6):
                          axis 0 the radius, axis 1 the colatitude (radians),
                          walls on both axes, 0 < lo[0], 0 < theta < pi,
                          radial gravity g[0] only, multigrid preconditioner
                          only; volumes and areas per radian of azimuth.
                          Passive scalars, the diagnostics and the eq. (17)
                          error are Cartesian only (-4) */
} jfnk_problem_desc;

/* Solver options.  Defaults (jfnk_default_opts): rtol 1e-8, atol 1e-14,
 * corr_tol 1e-12, newton_max 20, GMRES(30) x 10 cycles, eta 1e-2, acoustic
 * preconditioner with one multigrid V(2,2) cycle (4 sweeps on the coarsest
 * level), FP64. */
typedef struct {
    double newton_rtol;     /* stop when |S^-1 F| <= max(rtol |S^-1 F0|, atol sqrt(N_unknowns)) */
    double newton_atol;
    double newton_corr_tol; /* ... or when max |d rho / rho| of a Newton correction <= corr_tol */
    int newton_max;
    int gmres_restart;      /* Krylov basis size m (<= 32) */
    int gmres_max_cycles;
    double gmres_eta;       /* relative linear tolerance */
    int pc;                 /* JFNK_PC_* */
    int pc_solver;          /* JFNK_PCS_*: elliptic solves by multigrid or by ADI tridiagonal
                               (cyclic on periodic lines) line solves, each line solved by the
                               Thomas algorithm in one thread, consecutive threads on lines
                               adjacent in x where the lines run along y or z; in the mixed
                               form the acoustic lines hold FP32 values (FP64 arithmetic) */
    int mg_nu1, mg_nu2, mg_nuc, mg_cycles;
    int prec;               /* JFNK_FP64, or JFNK_MIXED: FP32 preconditioner and Krylov basis */
    double cfl_hydro;       /* eq. (5) target */
    double cfl_adv_max;     /* eq. (6) cap, 0 = off */
    double cfl_rad_max;     /* eq. (7) cap with D = chi/(rho c_P), 0 = off */
    double dt_max;          /* 0 = off */
    int max_halvings;       /* step retries at dt/2 after a failed Newton solve */
    int mg_light_cells;     /* multigrid levels of at most this many cells (not the coarsest) take one
                               pre- and one post-smoothing sweep; 0: every level takes mg_nu1/mg_nu2 */
    int newton_target;      /* time-step controller (on when dt_grow > 1): Newton iterations a step
                               should take; 0: grow by dt_grow after every accepted step */
    double dt_grow;         /* section 2.1: dt is adjusted for efficiency within the CFL limits above.
                               > 1 turns the controller on: a step's dt is the CFL dt of its state, but
                               at most dt_ctrl, which after an accepted step at dt with k Newton
                               iterations becomes dt * f, f = newton_target / k clamped to
                               [0.5, dt_grow] (f = dt_grow when newton_target is 0), and after a
                               failed step the last (halved) dt tried.  dt_ctrl starts unset at
                               creation and after jfnk_set_opts; it survives jfnk_set_state.
                               <= 1: off, every step at its CFL dt */
    int scalar_converge;    /* passive scalars (section 2.2): 1 (default) their Newton iterations run
                               until their own residual meets the flow's tolerances (the option
                               section 3.3 compares, in which the scalars' corrections must converge
                               as far as the primary variables');
                               0 they take as many Newton iterations as the flow's solve of the
                               step did (at least one), relying on the convergence of the flow
                               alone, with no test of their own (the paper's default) */
    int gmres_forcing;      /* JFNK_FORCING_*: the linear tolerance of each Newton iteration's GMRES
                               solve.  FIXED (default): gmres_eta throughout.  EW: Eisenstat and
                               Walker's choice 2 (SIAM J. Sci. Comput. 17, 1996) with gamma = 0.9,
                               alpha = 2 and the safeguards of Kelley's inexact Newton (Iterative
                               Methods for Linear and Nonlinear Equations, SIAM 1995, section 6.3):
                               eta_0 = gmres_eta; then eta_k = 0.9 (f_k / f_{k-1})^2, raised to
                               0.9 eta_{k-1}^2 when that exceeds 0.1, capped at gmres_eta, raised
                               to 0.5 tol / f_k (tol the Newton tolerance, f_k = |S^-1 F(u_k)|)
                               and capped at gmres_eta again (the flow's solve; the passive
                               scalars' solve keeps gmres_eta). */
    int newton_extrapolate; /* section 2.1 asks for efficiency within the limits; 1: the first
                               Newton iterate of a step is u^n + (dt / dt_prev)(u^n - u^{n-1}),
                               the linear extrapolation in time from the last two accepted
                               states of this problem (none before its first accepted step, or
                               after jfnk_set_state), used when its residual norm is below
                               |S^-1 F(u^n)|; the stopping test stays relative to F(u^n).
                               0 (default): the first iterate is u^n */
} jfnk_solver_opts;
#define JFNK_FORCING_FIXED 0
#define JFNK_FORCING_EW 1

/* Statistics of the last step. */
typedef struct {
    double t, dt, cfl_hydro, cfl_adv, cfl_rad;
    double rel_res;       /* final |S^-1 F| / |S^-1 F0| */
    double max_rel_corr;  /* max |d rho / rho| of the last Newton correction */
    double mass_drift, energy_drift;  /* relative change of sum rho, sum E */
    double f0, f;         /* initial and final |S^-1 F| */
    int newton_its, gmres_its, rejections, status;
    double wall_ms;       /* host wall time of the call */
    int scalar_newton_its, scalar_gmres_its;  /* passive-scalar solve of the accepted attempt */
    int newton_exit;      /* how Newton stopped: 0 the residual test (|S^-1 F| within its
                             tolerance, also when F0 already was), 1 the density-correction
                             test (max |d rho / rho| <= corr_tol) with |S^-1 F| still above
                             its tolerance, -1 failure */
    int extrapolated;     /* newton_extrapolate: 1 when the accepted attempt started from the
                             extrapolated iterate */
    double f_extrap;      /* its |S^-1 F| (-1 when none was tried) */
} jfnk_step_stats;

typedef struct jfnk_problem jfnk_problem;

/* Fill opts with the defaults listed above. */
void jfnk_default_opts(jfnk_solver_opts* opts);

/* Device bytes a problem would allocate (admission control). */
int jfnk_footprint_bytes(const jfnk_problem_desc* desc, const jfnk_solver_opts* opts, size_t* out);

/* Create a problem with initial state u0 (layout above): eqs. (1)-(3) of
 * section 2 on the staggered grid of section 2 (rho, E at cell centres,
 * momenta on faces), with the ghost-cell boundaries of section 3.1 (walls)
 * and section 6 (constant-luminosity walls).  The frozen wall conductive
 * fluxes and the heat-balance source are computed from u0.  Allocates the
 * state, the Krylov workspaces and the preconditioner hierarchy on the
 * current device (-2 if device memory runs out; nothing is left allocated).
 * hip_stream: a hipStream_t (NULL for the default stream); on a stream of
 * its own the multigrid solves are replayed as HIP graphs. */
int jfnk_create_problem(const jfnk_problem_desc* desc, const jfnk_solver_opts* opts,
                        const double* u0, int on_device, void* hip_stream, jfnk_problem** out);
int jfnk_destroy_problem(jfnk_problem* p);

/* Copy the state in or out; t is carried separately (jfnk_set_time). */
int jfnk_set_state(jfnk_problem* p, const double* u, int on_device);
int jfnk_get_state(jfnk_problem* p, double* u, int on_device);
int jfnk_set_time(jfnk_problem* p, double t);
int jfnk_set_opts(jfnk_problem* p, const jfnk_solver_opts* opts);

/* One adaptive implicit step (section 2.1 for dt, section 2 for the step):
 * dt from the CFL limits of eqs. (5)-(7) of the current state, the most
 * restrictive applying (and the efficiency controller's bound when
 * dt_grow > 1); a Crank-Nicolson step F(u) = u - u^n - dt/2 (R(u) + R(u^n))
 * = 0 solved by Newton-Raphson with right-preconditioned restarted GMRES
 * and Jacobian-free products; on failure the state is restored and dt
 * halved up to max_halvings times.  On a final failure the state is u^n
 * and the status code is returned.  Synchronises the problem's stream. */
int jfnk_implicit_step(jfnk_problem* p, jfnk_step_stats* out);

/* One Crank-Nicolson step (section 2) at the given dt > 0 with no retry
 * and no time-step controller: Newton-Raphson on F(u) = 0 from u^n, the
 * linear systems by GMRES with the physics-based preconditioner (section
 * 2, last paragraph).  On failure (status > 0) the state is restored to
 * u^n.  Synchronises the problem's stream. */
int jfnk_newton_solve(jfnk_problem* p, double dt, jfnk_step_stats* out);

/* ---- passive scalars (section 2.2) ----
 * nscal scalars given as partial densities s_k = c_k rho (nscal * N doubles,
 * scalar k at [k*N, (k+1)*N), cell order as rho), advanced by every later
 * step: after the flow's Newton solve has converged they take a
 * Crank-Nicolson step of d s_k/dt = -div(c_k rho u) with the mass fluxes of
 * u^n and u^{n+1} (face concentration reconstructed upstream with the van
 * Leer limiter, mirror image beyond walls), solved by Jacobian-free
 * Newton-Krylov without a preconditioner to the flow's tolerances; with
 * renormalize = 1 (and nscal > 1) the concentrations are then scaled to sum
 * to one in every cell.  A failed scalar solve fails the step like a failed
 * flow solve (state and scalars restored, dt halved).  nscal = 0 detaches
 * them.  Not available for problems created inside a caller-provided device
 * range (-4). */
int jfnk_set_scalars(jfnk_problem* p, int nscal, int renormalize, const double* s, int on_device);
int jfnk_get_scalars(jfnk_problem* p, double* s, int on_device);

/* ---- component entry points (operate on caller buffers of nvec doubles) ---- */

/* R(u): right-hand side of eqs. (1)-(3) on the staggered grid. */
int jfnk_eval_rhs(jfnk_problem* p, const double* u, double* R, int on_device);
/* b = u^n + dt/2 R(u^n) */
int jfnk_eval_cn_old(jfnk_problem* p, const double* un, double dt, double* b, int on_device);
/* F(u) = (u - b) - dt/2 R(u) */
int jfnk_eval_residual(jfnk_problem* p, const double* u, const double* b, double dt, double* F,
                       int on_device);
/* dt and limits for state u: out[0..8] = dt, max (|u|+c)/dx, max |u|/dx,
 * max D/dx^2, scales rho_ref, E_ref, m_ref (x3).  Also sets the problem's
 * variable scales S used by jv and precond. */
int jfnk_eval_time_step(jfnk_problem* p, const double* u, double* out9, int on_device);
/* Override the variable scales S (5 values: rho, E, m_x, m_y, m_z). */
int jfnk_set_scales(jfnk_problem* p, const double* s5);
/* Jacobian-free product in scaled variables (section 2, JFNK):
 * w = S^-1 (F(u + eps S v) - F(u)) / eps, eps = sqrt(2^-52)(1 + rms(S^-1 u))/rms(v),
 * evaluated as v - (dt/2) S^-1 (R(u + eps S v) - R(u)) / eps: the part u - b of
 * F is linear, so only R is differenced.  Wall faces of w are 0; v = 0 gives
 * eps = 0 and w = 0. */
int jfnk_apply_jv(jfnk_problem* p, const double* u, const double* b, double dt, const double* v,
                  double* w, int on_device);
/* The product of jfnk_apply_jv with a given difference step eps (> 0,
 * finite; -1 otherwise) in place of the automatic one: the same formula,
 * w = v - (dt/2) S^-1 (R(u + eps S v) - R(u)) / eps, wall faces 0.  Two
 * implementations that take the same eps difference the residual at the
 * same perturbed state, so their products can be compared element by
 * element (the automatic eps comes from two norms whose summation order is
 * implementation-defined).  Synchronises the problem's stream. */
int jfnk_apply_jv_eps(jfnk_problem* p, const double* u, const double* b, double dt, const double* v, double eps,
                      double* w, int on_device);
/* Preconditioner with coefficients frozen at u: z = S^-1 P^-1 (S v). */
int jfnk_apply_precond(jfnk_problem* p, const double* u, double dt, const double* v, double* z,
                       int on_device);

/* ---- diagnostics (reductions over a state on the device) ----
 * kinetic: sum over cells of (1/2) rho |v|^2 dV, |v|^2 of a cell being the
 *   mean over each axis of the squared velocities of its two faces (the
 *   kinetic energy of the Taylor-Green study, section 5.3; its rate of change
 *   is the difference of successive values over dt);
 * mass, energy: sum of rho dV and of E dV;
 * max_mach: max over cells of |v| / c_s, c_s^2 = gamma p / rho;
 * mix_width: mixing-region width of eqs. (12)-(14) along grid axis mix_axis,
 *   X_H = (rho - rho_light)/(rho_heavy - rho_light), mean per layer normal to
 *   the axis, X_M = 2 min(<X_H>, 1 - <X_H>), summed over layers times the
 *   layer thickness; 0 when mix_axis < 0;
 * mix_width_scalars: the same width from the first two passive scalars,
 *   eq. (16): X_M = 2 min(<c1>, <c2>) of the layer means of c_k = s_k / rho
 *   (0 unless the problem's own state is evaluated, it carries two or more
 *   scalars and mix_axis >= 0). */
typedef struct {
    double kinetic, mass, energy, max_mach, mix_width, mix_width_scalars;
} jfnk_diagnostics;

/* u: a state in the layout above (host or device per on_device), or NULL for
 * the problem's current state.  Errors: -1 bad axis or rho_heavy == rho_light
 * with mix_axis >= 0. */
int jfnk_eval_diagnostics(jfnk_problem* p, const double* u, int on_device, double rho_light, double rho_heavy,
                          int mix_axis, jfnk_diagnostics* out);

/* Relative error of eq. (17) (section 4.3) of velocity component `axis`
 * between a solution and a higher-resolution one of the same problem:
 * eps = sum |v_low - <v_high>| / sum |<v_high>| over the cells of this
 * problem's grid, where the velocity of a cell is the mean of the velocities
 * m / rho_f on its two faces along the axis and <v_high> is the volume
 * average of the high-resolution cell velocities over the ratio^ndim cells
 * that make up the cell.  u_low: a state of this problem's grid, or NULL
 * for the problem's current state; u_high: a state on the grid ratio times
 * finer on every active axis (same domain and boundaries), host or device
 * per on_device (a host u_high is staged through a temporary device buffer).
 * *out = 0 when the averaged field is zero.  Errors: -1 bad ratio or axis,
 * -2 no device memory for staging, -4 high-resolution grid too large. */
int jfnk_velocity_error(jfnk_problem* p, const double* u_low, const double* u_high, int on_device, int ratio,
                        int axis, double* out);

/* Allocation-free form of jfnk_velocity_error, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The same eq. (17) error with the same
 * kernels and summation order (bit for bit the result of jfnk_velocity_error
 * on the same inputs), but u_low (NULL: the problem's current state) and
 * u_high are device pointers on the problem's device, which must be the
 * current device (-1 otherwise), and the per-block partial sums live in a
 * scratch array of 32768 doubles (256 KiB) that the library keeps in every
 * GPU's memory for the life of the process; no call allocates.  The scratch
 * holds 2 doubles per block of the low-resolution grid plus 2, i.e. grids of
 * up to about 4.19 million cells (16383 blocks of 64 x 4 cells); larger
 * grids are refused with -4 before anything is launched.  Every call on a
 * GPU shares its scratch: the library serialises its own calls in a process
 * (a lock held until the result is read back), so concurrent calls from
 * several threads of one process are safe but wait for each other.  Other
 * errors as jfnk_velocity_error. */
int jfnk_velocity_error_noalloc(jfnk_problem* p, const double* u_low, const double* u_high, int ratio, int axis,
                                double* out);

/* ---- kernel-class timing ----
 * Time the launches of the kernel classes in class_mask (bit c = class c;
 * 0 disables) during later calls on p, with a HIP event pair attached to the
 * kernel dispatch itself (start and end of its execution).  Events are read
 * at the host synchronisation points the solver already has.
 * jfnk_profile_sample(p, period, burst) keeps the host cost of timing small:
 * with burst = 1 one launch in every `period` of each selected class is timed
 * (default period 1: all); with burst > 1 windows of `burst` consecutive
 * launches of any class carry events, a window opening at a launch with
 * probability 1/period (a fixed pseudo-random sequence, which does not alias
 * with the solver's periodic launch pattern), and only the selected classes'
 * launches after the first of a window are counted,
 * so every counted kernel follows one that also carried events (an event
 * pair on a kernel that follows one without events can open before that
 * kernel has drained and read long).
 * jfnk_profile_read copies the accumulated milliseconds, timed-launch counts
 * and compulsory bytes (every array a launch reads or writes counted once) of
 * the first nclass classes, resets them, and returns the number of classes.
 * jfnk_profile_class_name names class c ("residual_out", "cgs2_update_dot", ...). */
int jfnk_profile_enable(jfnk_problem* p, unsigned class_mask);
int jfnk_profile_sample(jfnk_problem* p, int period, int burst);
int jfnk_profile_read(jfnk_problem* p, double* ms, long long* count, double* bytes, int nclass);
const char* jfnk_profile_class_name(int cls);

/* ---- serving: continuous batching of independent simulations ----
 * A server owns one device arena of hbm_bytes and max_active worker threads,
 * each with its own non-blocking HIP stream.  Submitted requests (a problem,
 * its initial state and a number of implicit steps) wait in arrival order; a
 * free worker admits the oldest waiting request whose footprint
 * (jfnk_footprint_bytes plus alignment) fits a free range of the arena, so
 * requests arriving while others run are admitted as workers and memory free
 * up.  An admitted request keeps its state and Krylov workspaces resident in
 * its arena range until its last step; the work of concurrent requests
 * overlaps on the device through their streams.  Each request runs exactly
 * the kernels and host decisions it would run alone, so its result does not
 * depend on the mix.  Times are host milliseconds since server creation. */
typedef struct jfnk_server jfnk_server;

typedef struct {
    int status;            /* 0 ok; > 0 solver status of the step that failed; < 0 error */
    int steps_done;        /* accepted implicit steps */
    int newton_its, gmres_its, rejections;
    int pad;
    double cells;          /* cells of the grid */
    double t_submit_ms, t_admit_ms, t_done_ms;
    double sim_time;       /* simulated time reached */
    double footprint_bytes;
} jfnk_request_stats;

/* hbm_bytes: arena size (> 0); max_active: concurrent requests (1..64). */
int jfnk_server_create(size_t hbm_bytes, int max_active, jfnk_server** out);
/* Queue a request.  u0 is host memory in the state layout above; the server
 * copies it.  Fails with -1 if the request can never fit the arena. */
int jfnk_server_submit(jfnk_server* s, const jfnk_problem_desc* desc, const jfnk_solver_opts* opts,
                       const double* u0, int nsteps, long long* id);
/* 0 waiting, 1 running, 2 finished; -1 unknown id. */
int jfnk_server_poll(jfnk_server* s, long long id);
/* Block until the request has finished; copy its final state (host, may be
 * NULL) and statistics, and the wall time of each step (host milliseconds,
 * up to cap values, count in *nsteps_out).  The request is then released. */
int jfnk_server_wait(jfnk_server* s, long long id, double* u_out, jfnk_request_stats* st, double* step_ms,
                     int cap, int* nsteps_out);
/* Finish every admitted and queued request, stop the workers and free the arena. */
int jfnk_server_destroy(jfnk_server* s);

/* Thread-local description of the last error (empty string if none). */
const char* jfnk_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* JFNK_H */
