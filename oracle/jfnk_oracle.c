/*
 * Oracle: plain, slow, double-precision CPU implementation of one implicit
 * Crank-Nicolson step solved by Jacobian-free Newton-Krylov, written from
 * Goffrey et al., "Benchmarking the Multi-dimensional Stellar Implicit Code
 * MUSIC" (arXiv:1610.10053).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code with
 * the GPU path.
 *
 * Passages followed:
 *   - governing equations: section 2, eqs. (1)-(3), discretised by default in
 *     the total-energy conservative form (a reading: eq. 2 is written for
 *     internal energy, but the conservation checks need a flux form for E),
 *     or, as an option, with the energy variable rho e of eq. (2) as written:
 *     advective flux of rho e, the -p div u term at cell centres, no
 *     gravitational work;
 *   - ideal-gas closure and conductivity: section 2 (eq. 4 replaced by the
 *     synthetic chi = chi0 T^3);
 *   - staggered grid, upstream linear reconstruction with the van Leer
 *     limiter, ghost-cell boundaries: section 2 and section 3.1 (walls);
 *   - Crank-Nicolson, Newton-Raphson, GMRES, Jacobian-free products: section 2;
 *   - physics-based preconditioner (sound waves and optionally thermal
 *     diffusion implicit): section 2, last paragraph, and section 6;
 *   - time-step choice from CFL numbers: section 2.1, eqs. (5)-(7);
 *   - optionally, the linear tolerance of each Newton iteration from
 *     Eisenstat and Walker's choice 2 with Kelley's safeguards (the paper
 *     leaves it open; or_ew_forcing);
 *   - two-dimensional spherical geometry (r, theta) with azimuthal symmetry
 *     and radial gravity (section 2: constant or radial gravity as a body
 *     force; section 6: the radiative envelope in 2D spherical geometry):
 *     finite volumes with the cell volumes and face areas of the sphere, the
 *     momentum equations with their geometric terms.
 * Every detail the paper leaves open is a documented reading; the readings
 * are listed with the design notes of the repository.
 *
 * Parity pins for every function here live in the CPU test-suite.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define BC_PERIODIC 0
#define BC_WALL 1
#define PC_NONE 0
#define PC_ACOUSTIC 1
#define PC_ACOUSTIC_DIFFUSION 2
#define PCS_MULTIGRID 0
#define PCS_ADI 1
#define GH 3 /* ghost layers kept around every padded array */
#define MAXLEV 16

/* one level of a geometric multigrid hierarchy for the operator
 * (M x)_c = sigma_c x_c + sum over faces f of c of a_f (x_c - x_neighbour(f)) */
typedef struct {
    int n[3];
    long N;
    double *sig, *a[3], *D, *x, *b, *r, *t;
} Level;

typedef struct {
    /* problem */
    int ndim, n[3], bc[3], heat_balance;
    int internal; /* energy variable rho e (eq. 2) instead of total energy E */
    int sph;      /* 2D spherical: axis 0 = r, axis 1 = colatitude theta */
    double lo[3], hi[3], dx[3], idx[3], gamma, g[3], chi0;
    /* solver */
    double rtol, atol, eta, cfl_hydro, cfl_adv_max, cfl_rad_max, dt_max;
    int newton_max, restart, max_cycles, pc, max_halvings;
    int pc_solver, mg_nu1, mg_nu2, mg_nuc, mg_cycles;
    int mg_light; /* levels of at most this many cells: one pre- and one post-sweep (0: off) */
    double corr_tol;
    /* time-step controller (section 2.1: dt adjusted for efficiency within
     * the user's limits): on when dt_grow > 1 */
    double dt_grow, dt_ctrl;
    int newton_target;
    /* passive scalars (section 2.2): 1 their Newton iterations converge on
     * their own residual; 0 they take the flow's Newton count of the step */
    int scalar_converge;
    /* linear tolerance of the flow's Newton iterations: 0 eta throughout,
     * 1 Eisenstat-Walker choice 2 (or_ew_forcing) */
    int forcing;
    /* the last Newton solve: |S^-1 F(u_k)| for k = 0..hist_n-1 and the
     * linear tolerance and the GMRES solve's final relative residual of
     * iteration k (k < hist_n - 1) */
    double hist_f[64], hist_eta[64], hist_lin[64];
    int hist_n;
    /* optional first Newton iterate extrapolated in time: u^n + (dt /
     * dt_prev)(u^n - u^{n-1}) from the last two accepted states, used when
     * its residual norm is below that of u^n */
    int extrap, have_prev;
    double *uprev, *ux, *Fx, dt_prev;
    double st_fx;  /* residual norm of the extrapolated iterate (-1: none tried) */
    int st_extrap; /* 1 when the last solve started from it */
    /* spherical metric, per radial index i and colatitude index j:
     *   Vr[i] = (r_{i+1/2}^3 - r_{i-1/2}^3)/3, Vt[j] = cos th_{j-1/2} - cos th_{j+1/2}
     *   (cell volume Vr Vt per radian of azimuth); r2f[i] = r_{i-1/2}^2 and
     *   hr2[i] = (r_{i+1/2}^2 - r_{i-1/2}^2)/2 (face areas r2f Vt and hr2 stf);
     *   stf[j] = sin th_{j-1/2}; rc[i] cell-centre radius; ith[i] = 1/(rc dth);
     *   momentum control volumes: Vrc[i] = (rc_i^3 - rc_{i-1}^3)/3,
     *   r2c[i] = rc_i^2, hr2c[i] = (rc_i^2 - rc_{i-1}^2)/2,
     *   Vtc[j] = cos thc_{j-1} - cos thc_j, stc[j] = sin thc_j */
    double *Vr, *Vt, *r2f, *hr2, *stf, *rfa, *rc, *ith, *Vrc, *r2c, *hr2c, *Vtc, *stc;
    /* sizes */
    int gh[3], pn[3];  /* ghost layers per axis, padded extents */
    long N, P, nvar, nvec, nunk;
    /* state */
    double *u, *un;
    double t;
    /* frozen sources */
    double *sbal;         /* N cells, heat-balance source */
    double *qwall[3][2];  /* per wall direction: lower/upper wall diffusive flux per transverse cell */
    int sources_frozen;
    /* padded scratch (P entries each) */
    double *rho, *eps, *p, *T, *chi, *q, *uf[3], *m[3], *fr[3], *fe[3], *phic[3][3];
    /* residual / Krylov workspace (nvec entries) */
    double *b, *F, *w1, *w2, *R1;
    double *Ru; /* R at the current Newton iterate (Jacobian-free products) */
    /* scaling */
    double scale[5];
    /* preconditioner coefficients (cells N, faces per direction N) */
    double *pc_hf[3], *pc_kap[3], *pc_beta[3], *pc_W, tau;
    Level mg_ac[MAXLEV], mg_df[MAXLEV];
    int nlev;
    /* line solver scratch */
    double *la, *lb, *lc, *ld, *lx, *lt1, *lt2;
    /* statistics of the last solve */
    double st_dt, st_cfl_h, st_cfl_a, st_cfl_r, st_rel_res, st_max_rel_corr, st_mass_drift,
        st_energy_drift, st_f0, st_f;
    int st_newton, st_gmres, st_rejections, st_status, st_gmres_fail, st_exit;
    /* passive scalars (section 2.2): nscal partial densities s_k = c_k rho */
    int nscal, renorm;
    double *sc, *sc_n;
    int st_sc_newton, st_sc_gmres;
} Or;

/* ------------------------------------------------------------------ indexing */

static long pidx(const Or *o, int i, int j, int k) {
    return (long)(i + o->gh[0]) + (long)o->pn[0] * ((long)(j + o->gh[1]) + (long)o->pn[1] * (long)(k + o->gh[2]));
}
static long cidx(const Or *o, int i, int j, int k) {
    return (long)i + (long)o->n[0] * ((long)j + (long)o->n[1] * (long)k);
}
/* offset of one step along axis d in the padded layout */
static long pstride(const Or *o, int d) {
    if (d == 0) return 1;
    if (d == 1) return o->pn[0];
    return (long)o->pn[0] * o->pn[1];
}

#define FOR_CELLS(o) \
    for (int k = 0; k < (o)->n[2]; ++k) for (int j = 0; j < (o)->n[1]; ++j) for (int i = 0; i < (o)->n[0]; ++i)
/* Every loop marked PARC (cells) or PAR1 (flat vectors) computes each cell's
 * or entry's outputs from inputs the loop does not write.  Built with
 * -fopenmp (the all-cores CPU timing) these loops run on several threads
 * with unchanged arithmetic; the reductions (norms, dot products, maxima)
 * stay serial, so results are bit for bit those of the serial build. */
#ifdef _OPENMP
#include <omp.h>
#define PARC _Pragma("omp parallel for collapse(2) schedule(static)")
#define PAR1 _Pragma("omp parallel for schedule(static)")
#else
#define PARC
#define PAR1
#endif


static int coord(int d, int i, int j, int k) { return d == 0 ? i : (d == 1 ? j : k); }

/* periodic wrap of a padded array along every periodic axis (all ghost depths) */
static void wrap(const Or *o, double *a) {
    for (int d = 0; d < o->ndim; ++d) {
        if (o->bc[d] != BC_PERIODIC) continue;
        int n = o->n[d], g = o->gh[d];
        int lo1 = -o->gh[(d + 1) % 3], hi1 = o->n[(d + 1) % 3] + o->gh[(d + 1) % 3];
        int lo2 = -o->gh[(d + 2) % 3], hi2 = o->n[(d + 2) % 3] + o->gh[(d + 2) % 3];
        PAR1 for (int b = lo2; b < hi2; ++b)
            for (int a1 = lo1; a1 < hi1; ++a1)
                for (int s = 1; s <= g; ++s) {
                    int c[3];
                    c[d] = -s; c[(d + 1) % 3] = a1; c[(d + 2) % 3] = b;
                    long dst = pidx(o, c[0], c[1], c[2]);
                    c[d] = n - s;
                    long src = pidx(o, c[0], c[1], c[2]);
                    a[dst] = a[src];
                    c[d] = n - 1 + s;
                    dst = pidx(o, c[0], c[1], c[2]);
                    c[d] = s - 1;
                    src = pidx(o, c[0], c[1], c[2]);
                    a[dst] = a[src];
                }
    }
}

static void fill_nan(const Or *o, double *a) {
    for (long x = 0; x < o->P; ++x) a[x] = NAN;
}

/* ------------------------------------------------------------------ limiter */

/* van Leer's harmonic limiter of two one-sided differences (section 2). */
static double vanleer(double a, double b) {
    double ab = a * b;
    if (ab > 0.0) return (ab + ab) / (a + b);
    return 0.0;
}

/* Upstream linear extrapolation to a face between cells/faces with values
 * ql (slope sl) and qr (slope sr): take the upwind side, shift half a cell. */
static double upstream(double vel, double ql, double sl, double qr, double sr) {
    double qu, su;
    if (vel >= 0.0) { qu = ql; su = 0.5 * sl; }
    else { qu = qr; su = -0.5 * sr; }
    return qu + su;
}

/* ------------------------------------------------------------------ state -> primitives */

static double *field(const Or *o, const double *u, int f) { return (double *)u + (long)f * o->N; }

/* ---- spherical metric (section 6 geometry) ---- */
static void sph_tables(Or *o) {
    int nr = o->n[0], nt = o->n[1];
    double dr = o->dx[0], dth = o->dx[1];
    o->Vr = calloc(nr, sizeof(double)); o->rc = calloc(nr, sizeof(double)); o->ith = calloc(nr, sizeof(double));
    o->r2f = calloc(nr + 1, sizeof(double)); o->rfa = calloc(nr + 1, sizeof(double));
    o->hr2 = calloc(nr, sizeof(double));
    o->Vrc = calloc(nr, sizeof(double)); o->r2c = calloc(nr, sizeof(double)); o->hr2c = calloc(nr, sizeof(double));
    o->Vt = calloc(nt, sizeof(double)); o->stf = calloc(nt + 1, sizeof(double));
    o->Vtc = calloc(nt, sizeof(double)); o->stc = calloc(nt, sizeof(double));
    for (int i = 0; i <= nr; ++i) {
        double r = o->lo[0] + i * dr;
        o->rfa[i] = r;
        o->r2f[i] = r * r;
    }
    for (int i = 0; i < nr; ++i) {
        double a = o->rfa[i], b = o->rfa[i + 1];
        o->Vr[i] = (b * b * b - a * a * a) / 3.0;
        o->hr2[i] = 0.5 * (b * b - a * a);
        o->rc[i] = o->lo[0] + (i + 0.5) * dr;
        o->ith[i] = 1.0 / (o->rc[i] * dth);
        o->r2c[i] = o->rc[i] * o->rc[i];
    }
    for (int i = 1; i < nr; ++i) {
        double a = o->rc[i - 1], b = o->rc[i];
        o->Vrc[i] = (b * b * b - a * a * a) / 3.0;
        o->hr2c[i] = 0.5 * (b * b - a * a);
    }
    for (int j = 0; j <= nt; ++j) o->stf[j] = sin(o->lo[1] + j * dth);
    for (int j = 0; j < nt; ++j) {
        o->Vt[j] = cos(o->lo[1] + j * dth) - cos(o->lo[1] + (j + 1) * dth);
        o->stc[j] = sin(o->lo[1] + (j + 0.5) * dth);
    }
    for (int j = 1; j < nt; ++j)
        o->Vtc[j] = cos(o->lo[1] + (j - 0.5) * dth) - cos(o->lo[1] + (j + 0.5) * dth);
}
static double sph_vol(const Or *o, int i, int j) { return o->Vr[i] * o->Vt[j]; }
/* area of the lower face of cell (i, j) along d (i may be n0, j may be n1) */
static double sph_area(const Or *o, int d, int i, int j) {
    return d == 0 ? o->r2f[i] * o->Vt[j] : o->hr2[i] * o->stf[j];
}
/* inverse distance between the two cells of a face along d in row i */
static double face_ids(const Or *o, int d, int i) {
    return (o->sph && d == 1) ? o->ith[i] : o->idx[d];
}

/* Velocities on faces, pressure, specific energy of the energy variable
 * (total E/rho, or internal e), temperature, conductivity, with ghosts.
 * Section 2: scalars at cell centres, velocity components on faces; ideal gas
 * p = (gamma-1) rho e, with p = rho T. */
static void primitives(Or *o, const double *u) {
    const double *rho_c = field(o, u, 0), *E_c = field(o, u, 1);
    fill_nan(o, o->rho);
    PARC FOR_CELLS(o) o->rho[pidx(o, i, j, k)] = rho_c[cidx(o, i, j, k)];
    wrap(o, o->rho);
    for (int d = 0; d < o->ndim; ++d) {
        const double *m_c = field(o, u, 2 + d);
        double *uf = o->uf[d], *mm = o->m[d];
        long sd = pstride(o, d);
        fill_nan(o, uf);
        fill_nan(o, mm);
        PARC FOR_CELLS(o) {
            long pc = pidx(o, i, j, k);
            double mv = m_c[cidx(o, i, j, k)];
            if (o->bc[d] == BC_WALL && coord(d, i, j, k) == 0) {
                uf[pc] = 0.0;
                mm[pc] = 0.0;
            } else {
                double rf = 0.5 * (o->rho[pc - sd] + o->rho[pc]);
                uf[pc] = mv / rf;
                mm[pc] = mv;
            }
        }
        wrap(o, uf);
        wrap(o, mm);
    }
    /* ghost velocities beyond walls: normal component antisymmetric, tangential mirrored */
    for (int d = 0; d < o->ndim; ++d) {
        if (o->bc[d] != BC_WALL) continue;
        int n = o->n[d];
        for (int c = 0; c < o->ndim; ++c) {
            double *uf = o->uf[c], *mm = o->m[c];
            int r1 = (d + 1) % 3, r2 = (d + 2) % 3;
            for (int b = -o->gh[r2]; b < o->n[r2] + o->gh[r2]; ++b)
                for (int a1 = -o->gh[r1]; a1 < o->n[r1] + o->gh[r1]; ++a1) {
                    int x[3];
                    x[r1] = a1; x[r2] = b;
                    for (int s = 0; s <= GH; ++s) {
                        if (c == d) {
                            /* faces sit at lo + idx*dx: wall at 0 and n */
                            if (s == 0) {
                                x[d] = n; uf[pidx(o, x[0], x[1], x[2])] = 0.0; mm[pidx(o, x[0], x[1], x[2])] = 0.0;
                                continue;
                            }
                            if (s > GH - 1) continue;
                            x[d] = s; double lo_in = uf[pidx(o, x[0], x[1], x[2])];
                            x[d] = -s; uf[pidx(o, x[0], x[1], x[2])] = -lo_in;
                            x[d] = n - s; double hi_in = uf[pidx(o, x[0], x[1], x[2])];
                            x[d] = n + s; uf[pidx(o, x[0], x[1], x[2])] = -hi_in;
                        } else {
                            if (s == 0 || s > GH) continue;
                            x[d] = s - 1; double lo_in = uf[pidx(o, x[0], x[1], x[2])];
                            x[d] = -s; uf[pidx(o, x[0], x[1], x[2])] = lo_in;
                            x[d] = n - s; double hi_in = uf[pidx(o, x[0], x[1], x[2])];
                            x[d] = n - 1 + s; uf[pidx(o, x[0], x[1], x[2])] = hi_in;
                        }
                    }
                }
        }
    }
    /* cell thermodynamics */
    fill_nan(o, o->p); fill_nan(o, o->eps); fill_nan(o, o->T); fill_nan(o, o->chi); fill_nan(o, o->q);
    PARC FOR_CELLS(o) {
        long pc = pidx(o, i, j, k);
        double q = 0.0;
        for (int d = 0; d < o->ndim; ++d) {
            double a = o->uf[d][pc], b = o->uf[d][pc + pstride(o, d)];
            q = q + 0.5 * (a * a + b * b);
        }
        double r = o->rho[pc], E = E_c[cidx(o, i, j, k)];
        double kin = 0.5 * r * q;
        /* E holds rho e in the internal-energy form */
        double p = o->internal ? (o->gamma - 1.0) * E : (o->gamma - 1.0) * (E - kin);
        double T = p / r;
        o->q[pc] = q;
        o->p[pc] = p;
        o->eps[pc] = E / r;
        o->T[pc] = T;
        o->chi[pc] = o->chi0 * (T * T * T);
    }
    wrap(o, o->p); wrap(o, o->eps); wrap(o, o->T); wrap(o, o->chi); wrap(o, o->q);
    /* wall ghost cells, one layer: T extrapolated linearly, rho from the
     * discrete hydrostatic balance across the wall face (section 3.1) */
    for (int d = 0; d < o->ndim; ++d) {
        if (o->bc[d] != BC_WALL) continue;
        int n = o->n[d];
        double hg = 0.5 * o->g[d] * o->dx[d];
        int r1 = (d + 1) % 3, r2 = (d + 2) % 3;
        for (int b = 0; b < o->n[r2]; ++b)
            for (int a1 = 0; a1 < o->n[r1]; ++a1) {
                int x[3];
                x[r1] = a1; x[r2] = b;
                x[d] = 0; long c0 = pidx(o, x[0], x[1], x[2]);
                x[d] = 1; long c1 = pidx(o, x[0], x[1], x[2]);
                x[d] = -1; long cg = pidx(o, x[0], x[1], x[2]);
                double Tg = 2.0 * o->T[c0] - o->T[c1];
                double rg = o->rho[c0] * (o->T[c0] - hg) / (Tg + hg);
                o->T[cg] = Tg; o->rho[cg] = rg;
                o->eps[cg] = o->internal ? Tg / (o->gamma - 1.0) : Tg / (o->gamma - 1.0) + 0.5 * o->q[c0];
                o->chi[cg] = o->chi0 * (Tg * Tg * Tg);
                x[d] = n - 1; c0 = pidx(o, x[0], x[1], x[2]);
                x[d] = n - 2; c1 = pidx(o, x[0], x[1], x[2]);
                x[d] = n; cg = pidx(o, x[0], x[1], x[2]);
                Tg = 2.0 * o->T[c0] - o->T[c1];
                rg = o->rho[c0] * (o->T[c0] + hg) / (Tg - hg);
                o->T[cg] = Tg; o->rho[cg] = rg;
                o->eps[cg] = o->internal ? Tg / (o->gamma - 1.0) : Tg / (o->gamma - 1.0) + 0.5 * o->q[c0];
                o->chi[cg] = o->chi0 * (Tg * Tg * Tg);
            }
    }
}

/* diffusive flux -chi_f dT/ds on the face between padded cells l and r,
 * ids the inverse distance of their centres */
static double diff_flux(const Or *o, long l, long r, double ids) {
    return ((-0.5 * (o->chi[l] + o->chi[r])) * (o->T[r] - o->T[l])) * ids;
}

/* Mass and energy fluxes on every lower face (section 2: upstream linear
 * extrapolation of rho and of the specific energy, limited by van Leer): the
 * total-energy flux carries the pressure work p u, the internal-energy flux
 * of eq. (2) only rho e u. */
static void fluxes(Or *o) {
    for (int d = 0; d < o->ndim; ++d) {
        double *fr = o->fr[d], *fe = o->fe[d];
        long s = pstride(o, d);
        fill_nan(o, fr);
        fill_nan(o, fe);
        PARC FOR_CELLS(o) {
            long c = pidx(o, i, j, k);
            int id = coord(d, i, j, k);
            if (o->bc[d] == BC_WALL && id == 0) continue;
            double v = o->uf[d][c];
            long L = c - s, LL = c - 2 * s, R = c + s;
            double sl = vanleer(o->rho[c] - o->rho[L], o->rho[L] - o->rho[LL]);
            double sr = vanleer(o->rho[R] - o->rho[c], o->rho[c] - o->rho[L]);
            double rf = upstream(v, o->rho[L], sl, o->rho[c], sr);
            double el = vanleer(o->eps[c] - o->eps[L], o->eps[L] - o->eps[LL]);
            double er = vanleer(o->eps[R] - o->eps[c], o->eps[c] - o->eps[L]);
            double ef = upstream(v, o->eps[L], el, o->eps[c], er);
            double f_rho = v * rf;
            double f_e = o->internal ? f_rho * ef : f_rho * ef + v * (0.5 * (o->p[L] + o->p[c]));
            if (o->chi0 != 0.0) f_e = f_e + diff_flux(o, L, c, face_ids(o, d, i));
            fr[c] = f_rho;
            fe[c] = f_e;
        }
        if (o->bc[d] == BC_PERIODIC) {
            wrap(o, fr);
            wrap(o, fe);
        } else {
            /* walls: no advective flux, frozen diffusive flux */
            int n = o->n[d], r1 = (d + 1) % 3, r2 = (d + 2) % 3;
            for (int b = 0; b < o->n[r2]; ++b)
                for (int a1 = 0; a1 < o->n[r1]; ++a1) {
                    int x[3];
                    x[r1] = a1; x[r2] = b;
                    long t = (long)a1 + (long)o->n[r1] * b;
                    x[d] = 0;
                    fr[pidx(o, x[0], x[1], x[2])] = 0.0;
                    fe[pidx(o, x[0], x[1], x[2])] = o->qwall[d][0] ? o->qwall[d][0][t] : 0.0;
                    x[d] = n;
                    fr[pidx(o, x[0], x[1], x[2])] = 0.0;
                    fe[pidx(o, x[0], x[1], x[2])] = o->qwall[d][1] ? o->qwall[d][1][t] : 0.0;
                }
            /* periodic wrap along the other axes */
            wrap(o, fr);
            wrap(o, fe);
        }
    }
}

/* Momentum transport fluxes on the staggered control volumes: for component c
 * along direction d, phic[c][d] holds the flux through the control-volume side
 * that is crossed by direction d (cell centre if d == c, edge otherwise) at the
 * lower position of each face; velocity components are extrapolated upstream
 * and limited like the scalars (section 2). */
static void momentum_fluxes(Or *o) {
    for (int c = 0; c < o->ndim; ++c)
        for (int d = 0; d < o->ndim; ++d) {
            double *ph = o->phic[c][d];
            const double *uc = o->uf[c];
            long sc = pstride(o, c), sd = pstride(o, d);
            fill_nan(o, ph);
            if (c == d) {
                PARC FOR_CELLS(o) {
                    long x = pidx(o, i, j, k);
                    /* cell-centre flux for component c at cell x */
                    double Fb = 0.5 * (o->fr[c][x] + o->fr[c][x + sc]);
                    double a = uc[x - sc], b = uc[x], cc = uc[x + sc], dd = uc[x + 2 * sc];
                    double sl = vanleer(cc - b, b - a);
                    double sr = vanleer(dd - cc, cc - b);
                    double ur = upstream(Fb, b, sl, cc, sr);
                    ph[x] = Fb * ur;
                }
                wrap(o, ph);
            } else {
                /* positions along d from 0 to n_d inclusive, other axes interior */
                int ext[3] = {o->n[0], o->n[1], o->n[2]};
                ext[d] = o->n[d] + 1;
                PARC for (int k = 0; k < ext[2]; ++k)
                    for (int j = 0; j < ext[1]; ++j)
                        for (int i = 0; i < ext[0]; ++i) {
                            int id = coord(d, i, j, k);
                            if (o->bc[d] == BC_PERIODIC && id == o->n[d]) continue;
                            long x = pidx(o, i, j, k);
                            /* edge at the lower d-side of the c-face x: mass flux through
                             * d-faces of the two cells sharing face x */
                            double G;
                            if (o->bc[d] == BC_WALL && (id == 0 || id == o->n[d])) G = 0.0;
                            else G = 0.5 * (o->fr[d][x - sc] + o->fr[d][x]);
                            double a = uc[x - 2 * sd], b = uc[x - sd], cc = uc[x], dd = uc[x + sd];
                            double sl = vanleer(cc - b, b - a);
                            double sr = vanleer(dd - cc, cc - b);
                            double ur = upstream(G, b, sl, cc, sr);
                            ph[x] = G * ur;
                        }
                wrap(o, ph);
            }
        }
}

/* Momentum right-hand side in 2D spherical geometry on the staggered control
 * volume of the lower d-face of cell (i, j): transport fluxes through the
 * volume's sides times their areas over its volume, the pressure gradient
 * across the face, gravity (radial), and the geometric terms of the
 * spherical momentum equations, +rho u_th^2/r for the radial and
 * -rho u_r u_th/r for the polar component (u_phi = 0), with the face density
 * and the mean of the other component over the four faces around the face. */
static double sph_momentum(const Or *o, int d, int i, int j, long x) {
    long s0 = pstride(o, 0), s1 = pstride(o, 1);
    double a = 0.0;
    if (d == 0) {
        double rf = 0.5 * (o->rho[x - s0] + o->rho[x]);
        double V = o->Vrc[i] * o->Vt[j];
        double Ahi = o->r2c[i] * o->Vt[j], Alo = o->r2c[i - 1] * o->Vt[j];
        a = a - (Ahi * o->phic[0][0][x] - Alo * o->phic[0][0][x - s0]) / V;
        double Bhi = o->hr2c[i] * o->stf[j + 1], Blo = o->hr2c[i] * o->stf[j];
        a = a - (Bhi * o->phic[0][1][x + s1] - Blo * o->phic[0][1][x]) / V;
        a = a - (o->p[x] - o->p[x - s0]) * o->idx[0];
        if (o->g[0] != 0.0) a = a + rf * o->g[0];
        double u1 = o->uf[1][x - s0], u2 = o->uf[1][x - s0 + s1], u3 = o->uf[1][x], u4 = o->uf[1][x + s1];
        double ut2 = 0.25 * (((u1 * u1 + u2 * u2) + u3 * u3) + u4 * u4);
        a = a + rf * ut2 / o->rfa[i];
    } else {
        double rf = 0.5 * (o->rho[x - s1] + o->rho[x]);
        double V = o->Vr[i] * o->Vtc[j];
        double Ahi = o->r2f[i + 1] * o->Vtc[j], Alo = o->r2f[i] * o->Vtc[j];
        a = a - (Ahi * o->phic[1][0][x + s0] - Alo * o->phic[1][0][x]) / V;
        double Bhi = o->hr2[i] * o->stc[j], Blo = o->hr2[i] * o->stc[j - 1];
        a = a - (Bhi * o->phic[1][1][x] - Blo * o->phic[1][1][x - s1]) / V;
        a = a - (o->p[x] - o->p[x - s1]) * o->ith[i];
        double ur = 0.25 * (((o->uf[0][x - s1] + o->uf[0][x - s1 + s0]) + o->uf[0][x]) + o->uf[0][x + s0]);
        a = a - rf * ur * o->uf[1][x] / o->rc[i];
    }
    return a;
}

/* R(u): the right-hand side of eqs. (1)-(3) with gravity as a body force and
 * the heat-balance source, on the staggered grid.  Total-energy form: the
 * energy equation gains the work of gravity, rho u . g; internal-energy form
 * (eq. 2): it gains -p div u, with p at the cell centre and div u from the
 * cell's face velocities. */
static void rhs(Or *o, const double *u, double *R) {
    primitives(o, u);
    fluxes(o);
    momentum_fluxes(o);
    double *Rr = R, *RE = R + o->N;
    PARC FOR_CELLS(o) {
        long x = pidx(o, i, j, k), c = cidx(o, i, j, k);
        double ar = 0.0, ae = 0.0;
        for (int d = 0; d < o->ndim; ++d) {
            long s = pstride(o, d);
            if (o->sph) {
                /* (1/V) sum of area-weighted face fluxes */
                double V = sph_vol(o, i, j);
                double Alo = sph_area(o, d, i, j), Ahi = sph_area(o, d, d == 0 ? i + 1 : i, d == 1 ? j + 1 : j);
                ar = ar - (Ahi * o->fr[d][x + s] - Alo * o->fr[d][x]) / V;
                ae = ae - (Ahi * o->fe[d][x + s] - Alo * o->fe[d][x]) / V;
                continue;
            }
            ar = ar - (o->fr[d][x + s] - o->fr[d][x]) * o->idx[d];
            ae = ae - (o->fe[d][x + s] - o->fe[d][x]) * o->idx[d];
        }
        for (int d = 0; d < o->ndim; ++d) {
            long s = pstride(o, d);
            if (o->internal) {
                if (o->sph) {
                    double V = sph_vol(o, i, j);
                    double Alo = sph_area(o, d, i, j), Ahi = sph_area(o, d, d == 0 ? i + 1 : i, d == 1 ? j + 1 : j);
                    ae = ae - o->p[x] * ((Ahi * o->uf[d][x + s] - Alo * o->uf[d][x]) / V);
                    continue;
                }
                ae = ae - o->p[x] * ((o->uf[d][x + s] - o->uf[d][x]) * o->idx[d]);
                continue;
            }
            if (o->g[d] == 0.0) continue;
            ae = ae + o->g[d] * (0.5 * (o->m[d][x] + o->m[d][x + s]));
        }
        if (o->heat_balance && o->sources_frozen) ae = ae + o->sbal[c];
        Rr[c] = ar;
        RE[c] = ae;
    }
    for (int d = 0; d < o->ndim; ++d) {
        double *Rm = R + (long)(2 + d) * o->N;
        long sd = pstride(o, d);
        PARC FOR_CELLS(o) {
            long x = pidx(o, i, j, k), c = cidx(o, i, j, k);
            if (o->bc[d] == BC_WALL && coord(d, i, j, k) == 0) { Rm[c] = 0.0; continue; }
            if (o->sph) { Rm[c] = sph_momentum(o, d, i, j, x); continue; }
            double a = 0.0;
            for (int e = 0; e < o->ndim; ++e) {
                long se = pstride(o, e);
                if (e == d) a = a - (o->phic[d][d][x] - o->phic[d][d][x - sd]) * o->idx[d];
                else a = a - (o->phic[d][e][x + se] - o->phic[d][e][x]) * o->idx[e];
            }
            a = a - (o->p[x] - o->p[x - sd]) * o->idx[d];
            if (o->g[d] != 0.0) a = a + (0.5 * (o->rho[x - sd] + o->rho[x])) * o->g[d];
            Rm[c] = a;
        }
    }
}

/* Frozen sources from a reference state: wall diffusive fluxes from the
 * linearly extrapolated ghost temperature (constant luminosity, section 6) and
 * the heat-balance source that cancels the diffusive divergence there. */
static void freeze_sources(Or *o, const double *u) {
    o->sources_frozen = 0;
    for (int d = 0; d < o->ndim; ++d) {
        for (int s = 0; s < 2; ++s) { free(o->qwall[d][s]); o->qwall[d][s] = NULL; }
        if (o->bc[d] != BC_WALL || o->chi0 == 0.0) continue;
        int r1 = (d + 1) % 3, r2 = (d + 2) % 3;
        long nt = (long)o->n[r1] * o->n[r2];
        o->qwall[d][0] = calloc(nt, sizeof(double));
        o->qwall[d][1] = calloc(nt, sizeof(double));
    }
    primitives(o, u);
    for (int d = 0; d < o->ndim; ++d) {
        if (!o->qwall[d][0]) continue;
        int n = o->n[d], r1 = (d + 1) % 3, r2 = (d + 2) % 3;
        long s = pstride(o, d);
        for (int b = 0; b < o->n[r2]; ++b)
            for (int a1 = 0; a1 < o->n[r1]; ++a1) {
                int x[3];
                x[r1] = a1; x[r2] = b;
                long t = (long)a1 + (long)o->n[r1] * b;
                x[d] = 0; long c = pidx(o, x[0], x[1], x[2]);
                o->qwall[d][0][t] = diff_flux(o, c - s, c, face_ids(o, d, x[0]));
                x[d] = n; c = pidx(o, x[0], x[1], x[2]);
                o->qwall[d][1][t] = diff_flux(o, c - s, c, face_ids(o, d, x[0]));
            }
    }
    memset(o->sbal, 0, sizeof(double) * o->N);
    if (o->heat_balance && o->chi0 != 0.0) {
        /* diffusive fluxes only, including the frozen wall values */
        for (int d = 0; d < o->ndim; ++d) {
            double *f = o->fe[d];
            long s = pstride(o, d);
            fill_nan(o, f);
            PARC FOR_CELLS(o) {
                long c = pidx(o, i, j, k);
                if (o->bc[d] == BC_WALL && coord(d, i, j, k) == 0) continue;
                f[c] = diff_flux(o, c - s, c, face_ids(o, d, i));
            }
            if (o->bc[d] == BC_WALL) {
                int n = o->n[d], r1 = (d + 1) % 3, r2 = (d + 2) % 3;
                for (int b = 0; b < o->n[r2]; ++b)
                    for (int a1 = 0; a1 < o->n[r1]; ++a1) {
                        int x[3];
                        x[r1] = a1; x[r2] = b;
                        long t = (long)a1 + (long)o->n[r1] * b;
                        x[d] = 0; f[pidx(o, x[0], x[1], x[2])] = o->qwall[d][0][t];
                        x[d] = n; f[pidx(o, x[0], x[1], x[2])] = o->qwall[d][1][t];
                    }
            }
            wrap(o, f);
        }
        PARC FOR_CELLS(o) {
            long x = pidx(o, i, j, k);
            double acc = 0.0;
            for (int d = 0; d < o->ndim; ++d) {
                long s = pstride(o, d);
                if (o->sph) {
                    int ih = d == 0 ? i + 1 : i, jh = d == 1 ? j + 1 : j;
                    acc = acc + (sph_area(o, d, ih, jh) * o->fe[d][x + s] - sph_area(o, d, i, j) * o->fe[d][x]) /
                                    sph_vol(o, i, j);
                } else {
                    acc = acc + (o->fe[d][x + s] - o->fe[d][x]) * o->idx[d];
                }
            }
            o->sbal[cidx(o, i, j, k)] = acc;
        }
    }
    o->sources_frozen = 1;
}

/* ------------------------------------------------------------------ Crank-Nicolson residual */

/* b = u^n + dt/2 R(u^n): the old-time half of the Crank-Nicolson system */
static void cn_old(Or *o, const double *un, double dt, double *b) {
    rhs(o, un, o->R1);
    double h = 0.5 * dt;
    PAR1 for (long x = 0; x < o->nvec; ++x) b[x] = un[x] + h * o->R1[x];
}

/* F(u) = u - u^n - dt/2 (R(u) + R(u^n)) = (u - b) - dt/2 R(u) */
static void cn_residual(Or *o, const double *u, const double *b, double dt, double *F) {
    rhs(o, u, o->R1);
    double h = 0.5 * dt;
    PAR1 for (long x = 0; x < o->nvec; ++x) F[x] = (u[x] - b[x]) - h * o->R1[x];
    /* stored wall faces are not unknowns */
    for (int d = 0; d < o->ndim; ++d) {
        if (o->bc[d] != BC_WALL) continue;
        double *Fm = F + (long)(2 + d) * o->N;
        PARC FOR_CELLS(o) if (coord(d, i, j, k) == 0) Fm[cidx(o, i, j, k)] = 0.0;
    }
}

static double scale_of(const Or *o, long x) { return o->scale[x / o->N]; }

static double snorm2(const Or *o, const double *v) {
    double s = 0.0;
    for (long x = 0; x < o->nvec; ++x) {
        double t = v[x] / scale_of(o, x);
        s += t * t;
    }
    return sqrt(s);
}

static double norm2(long n, const double *v) {
    double s = 0.0;
    for (long x = 0; x < n; ++x) s += v[x] * v[x];
    return sqrt(s);
}

static double dot(long n, const double *a, const double *b) {
    double s = 0.0;
    for (long x = 0; x < n; ++x) s += a[x] * b[x];
    return s;
}

/* ------------------------------------------------------------------ time step (section 2.1) */

/* eqs. (5)-(7): the most restrictive constraint sets dt.  Also the variable
 * scales used to non-dimensionalise the Newton and Krylov vectors. */
static double time_step(Or *o, const double *u, double *hyd_out, double *adv_out, double *rad_out) {
    primitives(o, u);
    double hyd = 0.0, adv = 0.0, rad = 0.0, rmax = 0.0, emax = 0.0, cmax = 0.0;
    double cp = o->gamma / (o->gamma - 1.0);
    FOR_CELLS(o) {
        long x = pidx(o, i, j, k);
        double r = o->rho[x];
        double cs = sqrt(o->gamma * o->p[x] / r);
        for (int d = 0; d < o->ndim; ++d) {
            double a = fabs(o->uf[d][x]), b = fabs(o->uf[d][x + pstride(o, d)]);
            double ud = a > b ? a : b;
            double ids = face_ids(o, d, i);
            double h = (ud + cs) * ids;
            double v = ud * ids;
            if (h > hyd) hyd = h;
            if (v > adv) adv = v;
            if (o->chi0 != 0.0) {
                double D = o->chi[x] / (r * cp);
                double z = D * (ids * ids);
                if (z > rad) rad = z;
            }
        }
        if (r > rmax) rmax = r;
        double E = u[o->N + cidx(o, i, j, k)];
        if (E > emax) emax = E;
        if (cs > cmax) cmax = cs;
    }
    double dt = o->cfl_hydro / hyd;
    if (o->cfl_adv_max > 0.0 && adv > 0.0 && o->cfl_adv_max / adv < dt) dt = o->cfl_adv_max / adv;
    if (o->cfl_rad_max > 0.0 && rad > 0.0 && o->cfl_rad_max / rad < dt) dt = o->cfl_rad_max / rad;
    if (o->dt_max > 0.0 && o->dt_max < dt) dt = o->dt_max;
    o->scale[0] = rmax;
    o->scale[1] = emax;
    for (int d = 0; d < o->ndim; ++d) o->scale[2 + d] = rmax * cmax;
    if (hyd_out) *hyd_out = hyd;
    if (adv_out) *adv_out = adv;
    if (rad_out) *rad_out = rad;
    return dt;
}

/* ------------------------------------------------------------------ Jacobian-free product */

/* J v ~ (F(u + eps S v) - F(u)) / eps in scaled variables (section 2: the
 * matrix-vector products GMRES needs are approximated from residuals). */
/* Jacobian-free product (section 2) in scaled variables.  F(u) = (u - b) -
 * h R(u) is linear in u apart from R, so the difference quotient
 * (F(u + e S v) - F(u)) / (e S) equals v - h (R(u + e S v) - R(u)) / (e S):
 * only R is differenced, the identity part is applied exactly (reading R27).
 * Ru = R(u); wall faces, which are not unknowns, give 0. */
static void jv_at(Or *o, const double *u, const double *Ru, double dt, double e, const double *v, double *w);

static void jv(Or *o, const double *u, const double *Ru, double dt, double urms, const double *v, double *w) {
    double vn = norm2(o->nvec, v) / sqrt((double)o->nunk);
    if (vn == 0.0) { memset(w, 0, sizeof(double) * o->nvec); return; }
    double e = sqrt(2.220446049250313e-16) * (1.0 + urms) / vn;
    jv_at(o, u, Ru, dt, e, v, w);
}

/* the product at a given difference step e > 0 */
static void jv_at(Or *o, const double *u, const double *Ru, double dt, double e, const double *v, double *w) {
    PAR1 for (long x = 0; x < o->nvec; ++x) o->w2[x] = u[x] + (e * scale_of(o, x)) * v[x];
    rhs(o, o->w2, o->R1);
    double h = 0.5 * dt;
    PAR1 for (long x = 0; x < o->nvec; ++x) w[x] = v[x] - (h * (o->R1[x] - Ru[x])) / (e * scale_of(o, x));
    for (int d = 0; d < o->ndim; ++d) {
        if (o->bc[d] != BC_WALL) continue;
        double *wm = w + (long)(2 + d) * o->N;
        PARC FOR_CELLS(o) if (coord(d, i, j, k) == 0) wm[cidx(o, i, j, k)] = 0.0;
    }
}

/* ------------------------------------------------------------------ tridiagonal lines */

/* Thomas algorithm for a[i] x[i-1] + b[i] x[i] + c[i] x[i+1] = d[i]. */
static void thomas(int n, const double *a, const double *b, const double *c, const double *d,
                   double *x, double *cp, double *dp) {
    cp[0] = c[0] / b[0];
    dp[0] = d[0] / b[0];
    for (int i = 1; i < n; ++i) {
        double den = b[i] - a[i] * cp[i - 1];
        cp[i] = c[i] / den;
        dp[i] = (d[i] - a[i] * dp[i - 1]) / den;
    }
    x[n - 1] = dp[n - 1];
    for (int i = n - 2; i >= 0; --i) x[i] = dp[i] - cp[i] * x[i + 1];
}

/* Periodic (cyclic) system: a[0] couples to x[n-1], c[n-1] to x[0].
 * Solved with the Sherman-Morrison correction of a modified Thomas system. */
static void cyclic(int n, const double *a, const double *b, const double *c, const double *d,
                   double *x, double *tmp /* 5n */) {
    if (n == 1) { x[0] = d[0] / (b[0] + a[0] + c[0]); return; }
    double *bb = tmp, *u = tmp + n, *z = tmp + 2 * n, *cp = tmp + 3 * n, *dp = tmp + 4 * n;
    double gam = -b[0];
    double alpha = a[0], beta = c[n - 1];
    for (int i = 0; i < n; ++i) bb[i] = b[i];
    bb[0] = b[0] - gam;
    bb[n - 1] = b[n - 1] - beta * alpha / gam;
    /* a[0] and c[n-1] are ignored by Thomas */
    thomas(n, a, bb, c, d, x, cp, dp);
    for (int i = 0; i < n; ++i) u[i] = 0.0;
    u[0] = gam;
    u[n - 1] = beta;
    thomas(n, a, bb, c, u, z, cp, dp);
    double fact = (x[0] + alpha * x[n - 1] / gam) / (1.0 + z[0] + alpha * z[n - 1] / gam);
    for (int i = 0; i < n; ++i) x[i] = x[i] - fact * z[i];
}


/* ------------------------------------------------------------------ geometric multigrid */

static long lidx(const Level *L, int i, int j, int k) {
    return (long)i + (long)L->n[0] * ((long)j + (long)L->n[1] * (long)k);
}

/* neighbour on a level along d (periodic wrap), -1 beyond a wall */
static long lnb(const Or *o, const Level *L, int i, int j, int k, int d, int s) {
    int c[3] = {i, j, k};
    c[d] += s;
    if (c[d] < 0 || c[d] >= L->n[d]) {
        if (o->bc[d] == BC_WALL) return -1;
        c[d] = (c[d] + L->n[d]) % L->n[d];
    }
    return lidx(L, c[0], c[1], c[2]);
}

#define FOR_LEVEL(L) \
    for (int k = 0; k < (L)->n[2]; ++k) for (int j = 0; j < (L)->n[1]; ++j) for (int i = 0; i < (L)->n[0]; ++i)

static void level_free(Level *L) {
    free(L->sig); free(L->D); free(L->x); free(L->b); free(L->r); free(L->t);
    for (int d = 0; d < 3; ++d) free(L->a[d]);
    memset(L, 0, sizeof(*L));
}

static void level_alloc(Level *L, const int n[3]) {
    for (int d = 0; d < 3; ++d) L->n[d] = n[d];
    L->N = (long)n[0] * n[1] * n[2];
    L->sig = calloc(L->N, sizeof(double)); L->D = calloc(L->N, sizeof(double));
    L->x = calloc(L->N, sizeof(double)); L->b = calloc(L->N, sizeof(double));
    L->r = calloc(L->N, sizeof(double));
    L->t = calloc(L->N, sizeof(double));
    for (int d = 0; d < 3; ++d) L->a[d] = calloc(L->N, sizeof(double));
}

/* number of levels: halve every active axis while all are even and >= 4 */
static int count_levels(const Or *o) {
    int n[3] = {o->n[0], o->n[1], o->n[2]}, L = 1;
    for (;;) {
        int ok = 1;
        for (int d = 0; d < o->ndim; ++d) if (n[d] % 2 || n[d] < 4) ok = 0;
        if (!ok || L >= MAXLEV) break;
        for (int d = 0; d < o->ndim; ++d) n[d] /= 2;
        L++;
    }
    return L;
}

/* diagonal D = sigma + sum of the face couplings of each cell */
static void level_diag(const Or *o, Level *L) {
    PARC FOR_LEVEL(L) {
        long c = lidx(L, i, j, k);
        double den = L->sig[c];
        for (int d = 0; d < o->ndim; ++d) {
            long up = lnb(o, L, i, j, k, d, 1);
            double alo = L->a[d][c], ahi = up >= 0 ? L->a[d][up] : 0.0;
            den = den + alo;
            den = den + ahi;
        }
        L->D[c] = den;
    }
}

/* Hierarchy by re-discretisation: sigma averaged over the 2^ndim children,
 * face couplings averaged over the fine faces of a coarse face and divided by
 * 4 (the coupling scales as 1/dx^2). */
static void mg_build(Or *o, Level *lev, const double *sig, double *const *a) {
    for (int l = 0; l < MAXLEV; ++l) level_free(&lev[l]);
    level_alloc(&lev[0], o->n);
    memcpy(lev[0].sig, sig, sizeof(double) * o->N);
    for (int d = 0; d < o->ndim; ++d) memcpy(lev[0].a[d], a[d], sizeof(double) * o->N);
    level_diag(o, &lev[0]);
    int nch = 1 << o->ndim;
    double inv_ch = 1.0 / nch, inv_face = 1.0 / ((nch / 2) * 4);
    for (int l = 1; l < o->nlev; ++l) {
        Level *F = &lev[l - 1], *C = &lev[l];
        int n[3];
        for (int d = 0; d < 3; ++d) n[d] = d < o->ndim ? F->n[d] / 2 : 1;
        level_alloc(C, n);
        PARC FOR_LEVEL(C) {
            long c = lidx(C, i, j, k);
            int kk = o->ndim > 2 ? 2 : 1, jj = 2, ii = 2;
            double s = 0.0;
            for (int dk = 0; dk < kk; ++dk)
                for (int dj = 0; dj < jj; ++dj)
                    for (int di = 0; di < ii; ++di)
                        s = s + F->sig[lidx(F, 2 * i + di, 2 * j + dj, o->ndim > 2 ? 2 * k + dk : k)];
            C->sig[c] = s * inv_ch;
            for (int d = 0; d < o->ndim; ++d) {
                /* fine faces on the lower coarse face along d: fine index 2*I along d */
                double t = 0.0;
                for (int dk = 0; dk < kk; ++dk)
                    for (int dj = 0; dj < jj; ++dj)
                        for (int di = 0; di < ii; ++di) {
                            int off[3] = {di, dj, dk};
                            if (off[d] != 0) continue;
                            t = t + F->a[d][lidx(F, 2 * i + di, 2 * j + dj, o->ndim > 2 ? 2 * k + dk : k)];
                        }
                C->a[d][c] = t * inv_face;
            }
        }
        level_diag(o, C);
    }
}

/* red-black Gauss-Seidel: red cells (i+j+k even) first, then black.  The
 * cells of one colour are updated together from the values before their
 * half-sweep.  While every periodic axis has even length no two cells of one
 * colour are neighbours and this is the classical red-black sweep; on a
 * coarsest level with an odd periodic axis the two cells facing each other
 * across the wrap share a colour and see each other's previous values. */
static void mg_smooth(const Or *o, Level *L, int sweeps) {
    for (int s = 0; s < sweeps; ++s)
        for (int color = 0; color < 2; ++color) {
            PARC FOR_LEVEL(L) {
                if (((i + j + k) & 1) != color) continue;
                long c = lidx(L, i, j, k);
                double num = L->b[c];
                for (int d = 0; d < o->ndim; ++d) {
                    long up = lnb(o, L, i, j, k, d, 1), dn = lnb(o, L, i, j, k, d, -1);
                    if (dn >= 0) num = num + L->a[d][c] * L->x[dn];
                    if (up >= 0) num = num + L->a[d][up] * L->x[up];
                }
                L->t[c] = num / L->D[c];
            }
            PARC FOR_LEVEL(L) {
                if (((i + j + k) & 1) != color) continue;
                long c = lidx(L, i, j, k);
                L->x[c] = L->t[c];
            }
        }
}

static void mg_residual(const Or *o, Level *L) {
    PARC FOR_LEVEL(L) {
        long c = lidx(L, i, j, k);
        double xc = L->x[c];
        double acc = L->sig[c] * xc;
        for (int d = 0; d < o->ndim; ++d) {
            long up = lnb(o, L, i, j, k, d, 1), dn = lnb(o, L, i, j, k, d, -1);
            if (dn >= 0) acc = acc + L->a[d][c] * (xc - L->x[dn]);
            if (up >= 0) acc = acc + L->a[d][up] * (xc - L->x[up]);
        }
        L->r[c] = L->b[c] - acc;
    }
}

static void mg_vcycle(Or *o, Level *lev, int l) {
    Level *L = &lev[l];
    if (l == o->nlev - 1) { mg_smooth(o, L, o->mg_nuc); return; }
    int light = o->mg_light > 0 && L->N <= o->mg_light;
    mg_smooth(o, L, light ? 1 : o->mg_nu1);
    mg_residual(o, L);
    Level *C = &lev[l + 1];
    int nch = 1 << o->ndim;
    double inv_ch = 1.0 / nch;
    int kk = o->ndim > 2 ? 2 : 1;
    /* restriction: mean of the children */
    PARC FOR_LEVEL(C) {
        double s = 0.0;
        for (int dk = 0; dk < kk; ++dk)
            for (int dj = 0; dj < 2; ++dj)
                for (int di = 0; di < 2; ++di)
                    s = s + L->r[lidx(L, 2 * i + di, 2 * j + dj, o->ndim > 2 ? 2 * k + dk : k)];
        C->b[lidx(C, i, j, k)] = s * inv_ch;
        C->x[lidx(C, i, j, k)] = 0.0;
    }
    mg_vcycle(o, lev, l + 1);
    /* prolongation: cell-centred (bi/tri)linear interpolation, weights 3/4 and
     * 1/4 per axis; beyond a wall the parent value is used */
    PARC FOR_LEVEL(L) {
        int f[3] = {i, j, k}, P[3] = {i / 2, j / 2, o->ndim > 2 ? k / 2 : k};
        double e = 0.0;
        for (int m = 0; m < (1 << o->ndim); ++m) {
            int q[3] = {P[0], P[1], P[2]};
            double w = 1.0;
            for (int d = 0; d < o->ndim; ++d) {
                if (m & (1 << d)) {
                    int off = (f[d] % 2 == 0) ? -1 : 1;
                    w = w * 0.25;
                    q[d] += off;
                    if (q[d] < 0 || q[d] >= C->n[d]) {
                        if (o->bc[d] == BC_WALL) q[d] -= off;
                        else q[d] = (q[d] + C->n[d]) % C->n[d];
                    }
                } else {
                    w = w * 0.75;
                }
            }
            e = e + w * C->x[lidx(C, q[0], q[1], q[2])];
        }
        L->x[lidx(L, i, j, k)] = L->x[lidx(L, i, j, k)] + e;
    }
    mg_smooth(o, L, light ? 1 : o->mg_nu2);
}

/* approximate solve of M x = b by V-cycles from x = 0 (a fixed linear map) */
static void mg_solve(Or *o, Level *lev, double *v) {
    Level *L = &lev[0];
    memcpy(L->b, v, sizeof(double) * L->N);
    memset(L->x, 0, sizeof(double) * L->N);
    for (int c = 0; c < o->mg_cycles; ++c) mg_vcycle(o, lev, 0);
    memcpy(v, L->x, sizeof(double) * L->N);
}

/* ------------------------------------------------------------------ physics-based preconditioner */

/* Coefficients frozen at the current Newton iterate: face enthalpy h_f,
 * acoustic line coupling kappa_f = tau^2 (gamma-1) h_f / dx^2, diffusion
 * coupling beta_f = tau chi_f / dx^2 and W = (gamma-1)/rho. */
static void pc_build(Or *o, const double *u, double dt) {
    primitives(o, u);
    o->tau = 0.5 * dt;
    double tau = o->tau, gm1 = o->gamma - 1.0;
    const double *Ec = field(o, u, 1);
    for (int d = 0; d < o->ndim; ++d) {
        long s = pstride(o, d);
        PARC FOR_CELLS(o) {
            long x = pidx(o, i, j, k), c = cidx(o, i, j, k);
            double hf, chif;
            if (o->bc[d] == BC_WALL && coord(d, i, j, k) == 0) {
                hf = 0.0; chif = 0.0;
            } else {
                /* neighbour below along d (periodic wrap via padded arrays) */
                long xl = x - s;
                long cl;
                int ii = i, jj = j, kk = k;
                if (d == 0) ii = (i + o->n[0] - 1) % o->n[0];
                if (d == 1) jj = (j + o->n[1] - 1) % o->n[1];
                if (d == 2) kk = (k + o->n[2] - 1) % o->n[2];
                cl = cidx(o, ii, jj, kk);
                /* (E + p)/rho of the energy variable: in the internal-energy
                 * form the enthalpy, i.e. the p div u term is linearised in dm
                 * as the divergence of (p/rho)_f dm */
                double hl = (Ec[cl] + o->p[xl]) / o->rho[xl];
                double hr = (Ec[c] + o->p[x]) / o->rho[x];
                hf = 0.5 * (hl + hr);
                chif = 0.5 * (o->chi[xl] + o->chi[x]);
            }
            o->pc_hf[d][c] = hf;
            /* couplings per unit volume, or, in spherical geometry, of the
             * volume-weighted system: area over centre distance */
            double w = o->sph ? sph_area(o, d, i, j) * face_ids(o, d, i) : o->idx[d] * o->idx[d];
            o->pc_kap[d][c] = ((tau * tau) * gm1) * hf * w;
            o->pc_beta[d][c] = (tau * chif) * w;
        }
    }
    PARC FOR_CELLS(o) o->pc_W[cidx(o, i, j, k)] = gm1 / o->rho[pidx(o, i, j, k)];
    if (o->pc_solver == PCS_MULTIGRID && o->pc != PC_NONE) {
        double *sig = calloc(o->N, sizeof(double));
        PARC FOR_CELLS(o) sig[cidx(o, i, j, k)] = o->sph ? sph_vol(o, i, j) : 1.0;
        mg_build(o, o->mg_ac, sig, o->pc_kap);
        if (o->pc == PC_ACOUSTIC_DIFFUSION) {
            PARC FOR_CELLS(o) {
                long c = cidx(o, i, j, k);
                sig[c] = o->sph ? sph_vol(o, i, j) / o->pc_W[c] : 1.0 / o->pc_W[c];
            }
            mg_build(o, o->mg_df, sig, o->pc_beta);
        }
        free(sig);
    }
}

/* neighbour cell index along d with periodic wrap; -1 when outside a wall */
static long nb(const Or *o, int i, int j, int k, int d, int s) {
    int c[3] = {i, j, k};
    c[d] += s;
    if (c[d] < 0 || c[d] >= o->n[d]) {
        if (o->bc[d] == BC_WALL) return -1;
        c[d] = (c[d] + o->n[d]) % o->n[d];
    }
    return cidx(o, c[0], c[1], c[2]);
}

/* Solve every line along d of the system with per-cell rows built by rowfn.
 * kind 0: acoustic I - tau^2 D (gamma-1) h_f G; kind 1: diffusion I - tau D chi_f G W. */
static void line_solve(Or *o, int d, int kind, double *v) {
    int n = o->n[d];
    int r1 = (d + 1) % 3, r2 = (d + 2) % 3;
    for (int b2 = 0; b2 < o->n[r2]; ++b2)
        for (int b1 = 0; b1 < o->n[r1]; ++b1) {
            for (int t = 0; t < n; ++t) {
                int x[3];
                x[d] = t; x[r1] = b1; x[r2] = b2;
                long c = cidx(o, x[0], x[1], x[2]);
                long up = nb(o, x[0], x[1], x[2], d, 1);
                long dn = nb(o, x[0], x[1], x[2], d, -1);
                /* face below cell c is stored at c; face above at the upper neighbour,
                 * or is the top wall (coefficient 0) */
                double klo, khi;
                if (kind == 0) {
                    klo = o->pc_kap[d][c];
                    khi = up >= 0 ? o->pc_kap[d][up] : 0.0;
                    o->la[t] = -klo;
                    o->lc[t] = -khi;
                    o->lb[t] = 1.0 + (klo + khi);
                } else {
                    klo = o->pc_beta[d][c];
                    khi = up >= 0 ? o->pc_beta[d][up] : 0.0;
                    double wl = dn >= 0 ? o->pc_W[dn] : 0.0;
                    double wr = up >= 0 ? o->pc_W[up] : 0.0;
                    o->la[t] = -klo * wl;
                    o->lc[t] = -khi * wr;
                    o->lb[t] = 1.0 + (klo + khi) * o->pc_W[c];
                }
                o->ld[t] = v[c];
            }
            if (o->bc[d] == BC_PERIODIC) {
                cyclic(n, o->la, o->lb, o->lc, o->ld, o->lx, o->lt1);
            } else {
                thomas(n, o->la, o->lb, o->lc, o->ld, o->lx, o->lt1, o->lt2);
            }
            for (int t = 0; t < n; ++t) {
                int x[3];
                x[d] = t; x[r1] = b1; x[r2] = b2;
                v[cidx(o, x[0], x[1], x[2])] = o->lx[t];
            }
        }
}

/* discrete divergence of face values (optionally weighted by h_f) into a cell vector */
static void div_faces(Or *o, const double *const *mf, int weighted, double *out) {
    PARC FOR_CELLS(o) {
        long c = cidx(o, i, j, k);
        double acc = 0.0;
        for (int d = 0; d < o->ndim; ++d) {
            long up = nb(o, i, j, k, d, 1);
            double flo = mf[d][c], fhi = up >= 0 ? mf[d][up] : 0.0;
            if (weighted) {
                flo = o->pc_hf[d][c] * flo;
                fhi = up >= 0 ? o->pc_hf[d][up] * fhi : 0.0;
            }
            if (o->sph) {
                double Alo = sph_area(o, d, i, j), Ahi = sph_area(o, d, d == 0 ? i + 1 : i, d == 1 ? j + 1 : j);
                acc = acc + (Ahi * fhi - Alo * flo) / sph_vol(o, i, j);
                continue;
            }
            acc = acc + (fhi - flo) * o->idx[d];
        }
        out[c] = acc;
    }
}

/* z = P^{-1} v in scaled variables.  The semi-implicit approximate solve of
 * section 2 (sound waves and, optionally, thermal diffusion implicit;
 * advection and gravity left to the Krylov iteration):
 * (diffusion) implicit heat conduction on E;
 * (acoustic) Schur complement for the pressure correction,
 * (I - tau^2 D (gamma-1) h_f G) dp = (gamma-1)(r_E - tau D(h_f r_m)),
 * then dm = r_m - tau G dp, drho = r_rho - tau D dm, dE = r_E - tau D(h_f dm).
 * The elliptic solves use one multigrid V-cycle (default) or
 * alternating-direction tridiagonal line solves. */
static void pc_apply(Or *o, const double *v, double *z) {
    long N = o->N;
    double tau = o->tau, gm1 = o->gamma - 1.0;
    double *r = o->w1; /* scratch: unscaled rhs */
    PAR1 for (long x = 0; x < o->nvec; ++x) r[x] = scale_of(o, x) * v[x];
    if (o->pc == PC_NONE) {
        PAR1 for (long x = 0; x < o->nvec; ++x) z[x] = v[x];
        return;
    }
    double *rr = r, *rE = r + N;
    const double *rm[3] = {r + 2 * N, o->ndim > 1 ? r + 3 * N : NULL, o->ndim > 2 ? r + 4 * N : NULL};
    if (o->pc == PC_ACOUSTIC_DIFFUSION) {
        if (o->pc_solver == PCS_ADI) {
            for (int d = 0; d < o->ndim; ++d) line_solve(o, d, 1, rE);
        } else {
            /* with s = W dE the block is the symmetric system
             * (1/W - tau D chi_f G) s = r_E; solve it approximately, then form
             * dE = r_E + tau D(chi_f G s), which keeps sum(dE) = sum(r_E) */
            double *sv = o->w2;
            memcpy(sv, rE, sizeof(double) * N);
            if (o->sph) {PARC FOR_CELLS(o) sv[cidx(o, i, j, k)] *= sph_vol(o, i, j); } /* volume-weighted system */
            mg_solve(o, o->mg_df, sv);
            double *y = o->w2 + N;
            PARC FOR_CELLS(o) {
                long c = cidx(o, i, j, k);
                double acc = o->sph ? 0.0 : rE[c];
                for (int d = 0; d < o->ndim; ++d) {
                    long up = nb(o, i, j, k, d, 1), dn = nb(o, i, j, k, d, -1);
                    double thi = up >= 0 ? o->pc_beta[d][up] * (sv[up] - sv[c]) : 0.0;
                    double tlo = dn >= 0 ? o->pc_beta[d][c] * (sv[c] - sv[dn]) : 0.0;
                    acc = acc + (thi - tlo);
                }
                y[c] = o->sph ? rE[c] + acc / sph_vol(o, i, j) : acc;
            }
            memcpy(rE, y, sizeof(double) * N);
        }
    }
    double *dp = o->w2;
    div_faces(o, rm, 1, dp);
    PAR1 for (long c = 0; c < N; ++c) dp[c] = gm1 * (rE[c] - tau * dp[c]);
    if (o->sph) {PARC FOR_CELLS(o) dp[cidx(o, i, j, k)] *= sph_vol(o, i, j); } /* volume-weighted system */
    if (o->pc_solver == PCS_ADI) {
        for (int d = 0; d < o->ndim; ++d) line_solve(o, d, 0, dp);
    } else {
        mg_solve(o, o->mg_ac, dp);
    }
    double *dm[3] = {z + 2 * N, o->ndim > 1 ? z + 3 * N : NULL, o->ndim > 2 ? z + 4 * N : NULL};
    for (int d = 0; d < o->ndim; ++d) {
        PARC FOR_CELLS(o) {
            long c = cidx(o, i, j, k);
            if (o->bc[d] == BC_WALL && coord(d, i, j, k) == 0) { dm[d][c] = 0.0; continue; }
            long lo = nb(o, i, j, k, d, -1);
            dm[d][c] = rm[d][c] - tau * ((dp[c] - dp[lo]) * face_ids(o, d, i));
        }
    }
    double *tmp = dp; /* dp no longer needed */
    div_faces(o, (const double *const *)dm, 0, tmp);
    PAR1 for (long c = 0; c < N; ++c) z[c] = rr[c] - tau * tmp[c];
    div_faces(o, (const double *const *)dm, 1, tmp);
    PAR1 for (long c = 0; c < N; ++c) z[N + c] = rE[c] - tau * tmp[c];
    PAR1 for (long x = 0; x < o->nvec; ++x) z[x] = z[x] / scale_of(o, x);
}

/* ------------------------------------------------------------------ GMRES (Saad & Schultz) */

typedef void (*opfn)(void *ctx, const double *x, double *y);

typedef struct {
    int its, cycles, converged;
    double res; /* final estimated residual norm */
    double beta0;
} GmresInfo;

/* Right-preconditioned restarted GMRES(m), zero initial guess, classical
 * Gram-Schmidt applied twice, Givens rotations on the Hessenberg matrix. */
static void gmres(long n, opfn A, opfn Minv, void *ctx, const double *rhs, double *x,
                  int m, int max_cycles, double eta, GmresInfo *info) {
    double *V = calloc((size_t)(m + 1) * n, sizeof(double));
    double *Z = calloc((size_t)m * n, sizeof(double)); /* M^-1 v_j */
    double *H = calloc((size_t)(m + 1) * m, sizeof(double));
    double *cs = calloc(m, sizeof(double)), *sn = calloc(m, sizeof(double));
    double *gv = calloc(m + 1, sizeof(double)), *y = calloc(m, sizeof(double));
    double *h1 = calloc(m + 1, sizeof(double)), *h2 = calloc(m + 1, sizeof(double));
    double *r = calloc(n, sizeof(double)), *zt = calloc(n, sizeof(double)), *t = calloc(n, sizeof(double));
    memset(x, 0, sizeof(double) * n);
    memcpy(r, rhs, sizeof(double) * n);
    double beta0 = norm2(n, r);
    info->its = 0; info->cycles = 0; info->converged = 0; info->res = beta0; info->beta0 = beta0;
    if (beta0 == 0.0) { info->converged = 1; goto done; }
    for (int cyc = 0; cyc < max_cycles; ++cyc) {
        double beta = norm2(n, r);
        info->res = beta;
        if (beta <= eta * beta0) { info->converged = 1; break; }
        info->cycles++;
        PAR1 for (long i = 0; i < n; ++i) V[i] = r[i] / beta;
        for (int i = 0; i <= m; ++i) gv[i] = 0.0;
        gv[0] = beta;
        int kdim = 0, conv = 0;
        for (int j = 0; j < m; ++j) {
            double *vj = V + (long)j * n, *w = V + (long)(j + 1) * n, *zj = Z + (long)j * n;
            Minv(ctx, vj, zj);
            A(ctx, zj, w);
            double w0 = norm2(n, w);
            for (int i = 0; i <= j; ++i) h1[i] = dot(n, V + (long)i * n, w);
            for (int i = 0; i <= j; ++i) {
                const double *vi = V + (long)i * n;
                PAR1 for (long q = 0; q < n; ++q) w[q] -= h1[i] * vi[q];
            }
            for (int i = 0; i <= j; ++i) h2[i] = dot(n, V + (long)i * n, w);
            for (int i = 0; i <= j; ++i) {
                const double *vi = V + (long)i * n;
                PAR1 for (long q = 0; q < n; ++q) w[q] -= h2[i] * vi[q];
            }
            double hn = norm2(n, w);
            for (int i = 0; i <= j; ++i) H[(long)i * m + j] = h1[i] + h2[i];
            H[(long)(j + 1) * m + j] = hn;
            for (int i = 0; i < j; ++i) {
                double a = H[(long)i * m + j], b = H[(long)(i + 1) * m + j];
                H[(long)i * m + j] = cs[i] * a + sn[i] * b;
                H[(long)(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
            }
            double a = H[(long)j * m + j], b = H[(long)(j + 1) * m + j];
            double den = sqrt(a * a + b * b);
            cs[j] = a / den;
            sn[j] = b / den;
            H[(long)j * m + j] = den;
            H[(long)(j + 1) * m + j] = 0.0;
            gv[j + 1] = -sn[j] * gv[j];
            gv[j] = cs[j] * gv[j];
            info->its++;
            kdim = j + 1;
            info->res = fabs(gv[j + 1]);
            if (hn <= 1e-14 * w0) { conv = 1; break; } /* happy breakdown */
            PAR1 for (long q = 0; q < n; ++q) w[q] = w[q] / hn;
            if (info->res <= eta * beta0) { conv = 1; break; }
        }
        /* back substitution R y = g */
        for (int i = kdim - 1; i >= 0; --i) {
            double s = gv[i];
            for (int l = i + 1; l < kdim; ++l) s -= H[(long)i * m + l] * y[l];
            y[i] = s / H[(long)i * m + i];
        }
        /* x += M^-1 V y = sum_i y_i M^-1 v_i (M^-1 is a fixed linear map), from
         * the preconditioned vectors the Arnoldi process formed */
        PAR1 for (long q = 0; q < n; ++q) t[q] = 0.0;
        for (int i = 0; i < kdim; ++i) {
            const double *zi = Z + (long)i * n;
            PAR1 for (long q = 0; q < n; ++q) t[q] += y[i] * zi[q];
        }
        PAR1 for (long q = 0; q < n; ++q) x[q] += t[q];
        if (conv) { info->converged = 1; break; }
        /* true residual for the restart */
        A(ctx, x, t);
        PAR1 for (long q = 0; q < n; ++q) r[q] = rhs[q] - t[q];
        info->res = norm2(n, r);
    }
done:
    free(V); free(Z); free(H); free(cs); free(sn); free(gv); free(y); free(h1); free(h2);
    free(r); free(zt); free(t);
}

/* ------------------------------------------------------------------ Newton */

typedef struct { Or *o; const double *u, *Ru; double dt, urms; } JCtx;

static void op_jv(void *ctx, const double *x, double *y) {
    JCtx *c = ctx;
    jv(c->o, c->u, c->Ru, c->dt, c->urms, x, y);
}
static void op_pc(void *ctx, const double *x, double *y) {
    JCtx *c = ctx;
    pc_apply(c->o, x, y);
}

static int all_finite(long n, const double *a) {
    for (long x = 0; x < n; ++x) if (!isfinite(a[x])) return 0;
    return 1;
}

static double field_sum(const Or *o, const double *u, int f) {
    /* compensated sum so that drift reports are not dominated by summation error */
    double s = 0.0, c = 0.0;
    const double *a = u + (long)f * o->N;
    for (long x = 0; x < o->N; ++x) {
        double y = a[x] - c;
        double t = s + y;
        c = (t - s) - y;
        s = t;
    }
    return s;
}

/* Forcing term of inexact Newton iteration k >= 1 (the section 2 solver
 * leaves the linear tolerance open; this is an option, not the default):
 * Eisenstat and Walker's choice 2 (SIAM J. Sci. Comput. 17, 1996) with
 * gamma = 0.9 and exponent 2, safeguarded as in Kelley, Iterative Methods
 * for Linear and Nonlinear Equations (SIAM 1995), section 6.3: the ratio of
 * the last two nonlinear residual norms squared times gamma; kept at least
 * gamma eta_prev^2 when that exceeds 0.1 (no sudden drop of the tolerance);
 * at most eta_max; at least half the nonlinear tolerance over the current
 * residual (no oversolving of the last iteration); at most eta_max. */
double or_ew_forcing(double f, double f_prev, double eta_prev, double eta_max, double tol) {
    const double gamma = 0.9;
    const double ratio = f / f_prev;
    double eta = gamma * (ratio * ratio);
    const double keep = gamma * (eta_prev * eta_prev);
    if (keep > 0.1 && keep > eta) eta = keep;
    if (eta > eta_max) eta = eta_max;
    const double end = 0.5 * tol / f;
    if (end > eta) eta = end;
    if (eta > eta_max) eta = eta_max;
    return eta;
}

/* Newton-Raphson on F(u) = 0 from u = u^n at a given dt; state updated in
 * place on success, restored on failure.  Returns 0 or a failure code. */
static int newton(Or *o, double dt) {
    long nv = o->nvec;
    double *u = o->u, *b = o->b, *F = o->F;
    double *x = calloc(nv, sizeof(double)), *rhsv = calloc(nv, sizeof(double));
    memcpy(o->un, u, sizeof(double) * nv);
    double m0 = field_sum(o, u, 0), e0 = field_sum(o, u, 1);
    time_step(o, u, NULL, NULL, NULL); /* scales from u^n */
    cn_old(o, u, dt, b);
    cn_residual(o, u, b, dt, F);
    memcpy(o->Ru, o->R1, sizeof(double) * nv);
    double f0 = snorm2(o, F), f = f0;
    double tol = o->rtol * f0;
    double floor_ = o->atol * sqrt((double)o->nunk);
    if (floor_ > tol) tol = floor_;
    int status = 0, its = 0, gits = 0;
    double max_corr = 0.0;
    /* optional extrapolated first iterate: kept when its residual is below
     * F(u^n)'s; the stopping test stays relative to F(u^n) */
    o->st_fx = -1.0;
    o->st_extrap = 0;
    if (o->extrap && o->have_prev && isfinite(f0)) {
        const double r = dt / o->dt_prev;
        for (long q = 0; q < nv; ++q) o->ux[q] = u[q] + r * (u[q] - o->uprev[q]);
        cn_residual(o, o->ux, b, dt, o->Fx);
        const double fx = snorm2(o, o->Fx);
        o->st_fx = fx;
        if (fx < f0) {
            memcpy(u, o->ux, sizeof(double) * nv);
            memcpy(F, o->Fx, sizeof(double) * nv);
            memcpy(o->Ru, o->R1, sizeof(double) * nv);
            f = fx;
            o->st_extrap = 1;
        }
    }
    double eta = o->eta, f_prev = f;
    o->hist_f[0] = f;
    o->hist_n = 1;
    o->st_gmres_fail = 0;
    if (!isfinite(f0)) status = 3;
    while (status == 0 && f > tol) {
        if (its >= o->newton_max) { status = 1; break; }
        if (o->forcing == 1 && its > 0) eta = or_ew_forcing(f, f_prev, eta, o->eta, tol);
        if (its < 64) o->hist_eta[its] = eta;
        pc_build(o, u, dt);
        double urms = snorm2(o, u) / sqrt((double)o->nunk);
        PAR1 for (long q = 0; q < nv; ++q) rhsv[q] = -F[q] / scale_of(o, q);
        JCtx ctx = {o, u, o->Ru, dt, urms};
        GmresInfo gi;
        gmres(nv, op_jv, op_pc, &ctx, rhsv, x, o->restart, o->max_cycles, eta, &gi);
        if (its < 64) o->hist_lin[its] = gi.beta0 > 0.0 ? gi.res / gi.beta0 : 0.0;
        gits += gi.its;
        if (!gi.converged && gi.res >= 0.999 * gi.beta0) { status = 2; o->st_gmres_fail = 1; break; }
        max_corr = 0.0;
        PAR1 for (long q = 0; q < nv; ++q) u[q] = u[q] + scale_of(o, q) * x[q];
        for (long c = 0; c < o->N; ++c) {
            double rc = fabs(scale_of(o, c) * x[c] / u[c]);
            if (rc > max_corr) max_corr = rc;
        }
        cn_residual(o, u, b, dt, F);
        memcpy(o->Ru, o->R1, sizeof(double) * nv);
        f_prev = f;
        f = snorm2(o, F);
        its++;
        if (its < 64) { o->hist_f[its] = f; o->hist_n = its + 1; }
        if (!isfinite(f) || !all_finite(nv, u)) { status = 3; break; }
        /* density corrections converged to roundoff: the iteration has
         * reached its floor (the paper's stopping test is on density) */
        if (max_corr <= o->corr_tol) break;
    }
    o->st_newton = its;
    o->st_gmres = gits;
    /* how Newton stopped: 0 residual test, 1 density-correction test with the
     * residual still above its tolerance, -1 failure */
    o->st_exit = status != 0 ? -1 : (f > tol ? 1 : 0);
    o->st_f0 = f0;
    o->st_f = f;
    o->st_rel_res = f0 > 0.0 ? f / f0 : 0.0;
    o->st_max_rel_corr = max_corr;
    o->st_dt = dt;
    if (status != 0) {
        memcpy(u, o->un, sizeof(double) * nv);
    } else {
        o->st_mass_drift = (field_sum(o, u, 0) - m0) / m0;
        o->st_energy_drift = (field_sum(o, u, 1) - e0) / e0;
    }
    free(x); free(rhsv);
    o->st_status = status;
    return status;
}

/* ------------------------------------------------------------------ passive scalars (section 2.2)
 * Each scalar is a concentration c_k carried by the flow, advanced in its
 * conservative form d(c_k rho)/dt = -div(c_k rho u): the face flux is the
 * face mass flux of the hydrodynamic solution times the concentration
 * reconstructed on the face like the other cell quantities (upstream linear
 * extrapolation with the van Leer limiter; beyond a wall the mirror-image
 * cell).  After a converged hydrodynamic step the scalars take their own
 * Crank-Nicolson step with the mass fluxes of u^n and u^{n+1}, solved by
 * Jacobian-free Newton-Krylov without a preconditioner, and are
 * re-normalised so that the concentrations sum to one in every cell. */

/* density and lower-face mass fluxes of state u, cell-indexed (0 on walls) */
static void mass_flux_cells(Or *o, const double *u, double *rho, double *fr) {
    primitives(o, u);
    fluxes(o);
    FOR_CELLS(o) {
        long c = cidx(o, i, j, k), pc = pidx(o, i, j, k);
        rho[c] = o->rho[pc];
        for (int d = 0; d < o->ndim; ++d) fr[(long)d * o->N + c] = o->fr[d][pc];
    }
}

/* concentration of the cell at offset a along d from (i, j, k) */
static double conc(const Or *o, const double *s, const double *rho, int i, int j, int k, int d, int a) {
    int x[3] = {i, j, k};
    int n = o->n[d], v = x[d] + a;
    if (v < 0 || v >= n) {
        if (o->bc[d] == BC_WALL) v = v < 0 ? -1 - v : 2 * n - 1 - v;
        else v = (v % n + n) % n;
    }
    x[d] = v;
    long c = cidx(o, x[0], x[1], x[2]);
    return s[c] / rho[c];
}

/* scalar flux through the lower face of cell (i, j, k) along d */
static double scalar_flux(const Or *o, const double *s, const double *rho, const double *fr, int i, int j, int k,
                          int d) {
    int id = coord(d, i, j, k);
    if (o->bc[d] == BC_WALL && id == 0) return 0.0;
    double f = fr[(long)d * o->N + cidx(o, i, j, k)];
    double cLL = conc(o, s, rho, i, j, k, d, -2), cL = conc(o, s, rho, i, j, k, d, -1);
    double cc = conc(o, s, rho, i, j, k, d, 0), cR = conc(o, s, rho, i, j, k, d, 1);
    double sl = vanleer(cc - cL, cL - cLL);
    double sr = vanleer(cR - cc, cc - cL);
    return f * upstream(f, cL, sl, cc, sr);
}

/* R_k = -div(c_k rho u) for every scalar */
static void scalar_rhs(const Or *o, const double *s, const double *rho, const double *fr, double *R) {
    for (int q = 0; q < o->nscal; ++q) {
        const double *sq = s + (long)q * o->N;
        FOR_CELLS(o) {
            double r = 0.0;
            for (int d = 0; d < o->ndim; ++d) {
                int x[3] = {i, j, k};
                double lo = scalar_flux(o, sq, rho, fr, i, j, k, d), hi = 0.0;
                if (!(o->bc[d] == BC_WALL && x[d] == o->n[d] - 1)) {
                    x[d] = (x[d] + 1) % o->n[d];
                    hi = scalar_flux(o, sq, rho, fr, x[0], x[1], x[2], d);
                }
                r = r - (hi - lo) * o->idx[d];
            }
            R[(long)q * o->N + cidx(o, i, j, k)] = r;
        }
    }
}

typedef struct { Or *o; const double *s, *Gs, *b, *rho, *fr; double h, srms; double *sp, *R; } SCtx;

/* G(s) = (s - b) - h R(s) */
static void scalar_residual(SCtx *c, const double *s, double *G) {
    long n = (long)c->o->nscal * c->o->N;
    scalar_rhs(c->o, s, c->rho, c->fr, c->R);
    for (long q = 0; q < n; ++q) G[q] = (s[q] - c->b[q]) - c->h * c->R[q];
}
static void op_sjv(void *ctx, const double *v, double *w) {
    SCtx *c = ctx;
    long n = (long)c->o->nscal * c->o->N;
    double vrms = norm2(n, v) / sqrt((double)n);
    if (vrms == 0.0) { memset(w, 0, sizeof(double) * n); return; }
    double eps = sqrt(2.220446049250313e-16) * (1.0 + c->srms) / vrms;
    for (long q = 0; q < n; ++q) c->sp[q] = c->s[q] + eps * v[q];
    scalar_residual(c, c->sp, w);
    for (long q = 0; q < n; ++q) w[q] = (w[q] - c->Gs[q]) / eps;
}
static void op_copy(void *ctx, const double *x, double *y) {
    SCtx *c = ctx;
    memcpy(y, x, sizeof(double) * (long)c->o->nscal * c->o->N);
}

/* Crank-Nicolson step of the scalars from u^n (o->un) to u^{n+1} (o->u) */
static int scalar_step(Or *o, double dt) {
    long N = o->N, n = (long)o->nscal * N;
    double *rho0 = calloc(N, sizeof(double)), *rho1 = calloc(N, sizeof(double));
    double *fr0 = calloc(3 * N, sizeof(double)), *fr1 = calloc(3 * N, sizeof(double));
    double *b = calloc(n, sizeof(double)), *G = calloc(n, sizeof(double)), *R = calloc(n, sizeof(double));
    double *x = calloc(n, sizeof(double)), *rhs = calloc(n, sizeof(double)), *sp = calloc(n, sizeof(double));
    mass_flux_cells(o, o->un, rho0, fr0);
    mass_flux_cells(o, o->u, rho1, fr1);
    double *s = o->sc;
    memcpy(o->sc_n, s, sizeof(double) * n);
    double h = 0.5 * dt;
    scalar_rhs(o, s, rho0, fr0, R);
    for (long q = 0; q < n; ++q) b[q] = s[q] + h * R[q];
    SCtx ctx = {o, s, G, b, rho1, fr1, h, 0.0, sp, R};
    scalar_residual(&ctx, s, G);
    double g0 = norm2(n, G), g = g0;
    double tol = o->rtol * g0, floor_ = o->atol * sqrt((double)n);
    if (floor_ > tol) tol = floor_;
    int status = 0, its = 0, gits = 0;
    if (!isfinite(g0)) status = 3;
    int nfix = o->st_newton > 1 ? o->st_newton : 1; /* the flow's Newton count of this step */
    while (status == 0 && (o->scalar_converge ? g > tol : (its < nfix && g > floor_))) {
        if (its >= o->newton_max) { status = 1; break; }
        ctx.srms = norm2(n, s) / sqrt((double)n);
        for (long q = 0; q < n; ++q) rhs[q] = -G[q];
        GmresInfo gi;
        gmres(n, op_sjv, op_copy, &ctx, rhs, x, o->restart, o->max_cycles, o->eta, &gi);
        gits += gi.its;
        if (!gi.converged && gi.res >= 0.999 * gi.beta0) { status = 2; break; }
        for (long q = 0; q < n; ++q) s[q] = s[q] + x[q];
        scalar_residual(&ctx, s, G);
        g = norm2(n, G);
        its++;
        if (!isfinite(g)) { status = 3; break; }
    }
    if (status == 0 && o->renorm && o->nscal > 1) {
        for (long c = 0; c < N; ++c) {
            double tot = 0.0;
            for (int q = 0; q < o->nscal; ++q) tot = tot + s[(long)q * N + c];
            if (tot > 0.0)
                for (int q = 0; q < o->nscal; ++q) s[(long)q * N + c] = s[(long)q * N + c] * (rho1[c] / tot);
        }
    }
    if (status != 0) memcpy(s, o->sc_n, sizeof(double) * n);
    o->st_sc_newton = its;
    o->st_sc_gmres = gits;
    free(rho0); free(rho1); free(fr0); free(fr1); free(b); free(G); free(R); free(x); free(rhs); free(sp);
    return status;
}

/* one Crank-Nicolson step of the flow and then of the scalars; on failure
 * the state (and the scalars) are those of u^n */
static int step_at(Or *o, double dt) {
    int s = newton(o, dt);
    if (s == 0 && o->nscal > 0) {
        s = scalar_step(o, dt);
        if (s != 0) memcpy(o->u, o->un, sizeof(double) * o->nvec);
    }
    if (s == 0) {
        /* an accepted step: u^n and its dt are the next extrapolation's past */
        memcpy(o->uprev, o->un, sizeof(double) * o->nvec);
        o->dt_prev = dt;
        o->have_prev = 1;
    }
    return s;
}

/* ------------------------------------------------------------------ public entry points */

static void or_free(Or *o) {
    if (!o) return;
    double **ptrs[] = {&o->u, &o->un, &o->sbal, &o->Vr, &o->Vt, &o->r2f, &o->hr2, &o->stf, &o->rfa, &o->rc,
                       &o->ith, &o->Vrc, &o->r2c, &o->hr2c, &o->Vtc, &o->stc, &o->rho, &o->eps, &o->p, &o->T, &o->chi, &o->q,
                       &o->b, &o->F, &o->w1, &o->w2, &o->R1, &o->Ru, &o->pc_W, &o->la, &o->lb, &o->lc,
                       &o->ld, &o->lx, &o->lt1, &o->lt2, &o->uprev, &o->ux, &o->Fx};
    for (size_t i = 0; i < sizeof(ptrs) / sizeof(ptrs[0]); ++i) free(*ptrs[i]);
    for (int d = 0; d < 3; ++d) {
        free(o->uf[d]); free(o->m[d]); free(o->fr[d]); free(o->fe[d]);
        free(o->pc_hf[d]); free(o->pc_kap[d]); free(o->pc_beta[d]);
        free(o->qwall[d][0]); free(o->qwall[d][1]);
        for (int e = 0; e < 3; ++e) free(o->phic[d][e]);
    }
    for (int l = 0; l < MAXLEV; ++l) { level_free(&o->mg_ac[l]); level_free(&o->mg_df[l]); }
    free(o->sc); free(o->sc_n);
    free(o);
}

/* ip: ndim, n0, n1, n2, bc0, bc1, bc2, heat_balance, newton_max, restart,
 *     max_cycles, pc, max_halvings, pc_solver, mg_nu1, mg_nu2, mg_nuc, mg_cycles,
 *     energy form (0 total, 1 internal), geometry (0 Cartesian, 1 2D spherical),
 *     mg_light (levels of at most this many cells take V(1,1), 0 = off),
 *     newton_target, scalar_converge, forcing (0 eta, 1 Eisenstat-Walker),
 *     extrapolate (1: extrapolated first Newton iterate)
 * dp: lo0..2, hi0..2, gamma, g0..2, chi0, rtol, atol, eta, cfl_hydro,
 *     cfl_adv_max, cfl_rad_max, dt_max, corr_tol, dt_grow */
void *or_create(const int *ip, const double *dp, const double *u0) {
    Or *o = calloc(1, sizeof(Or));
    o->ndim = ip[0];
    for (int d = 0; d < 3; ++d) { o->n[d] = ip[1 + d]; o->bc[d] = ip[4 + d]; }
    o->heat_balance = ip[7]; o->newton_max = ip[8]; o->restart = ip[9]; o->max_cycles = ip[10];
    o->pc = ip[11]; o->max_halvings = ip[12];
    o->pc_solver = ip[13]; o->mg_nu1 = ip[14]; o->mg_nu2 = ip[15]; o->mg_nuc = ip[16]; o->mg_cycles = ip[17];
    o->internal = ip[18];
    o->sph = ip[19];
    o->mg_light = ip[20];
    o->corr_tol = dp[18];
    o->dt_grow = dp[19];
    o->newton_target = ip[21];
    o->scalar_converge = ip[22];
    o->forcing = ip[23];
    o->extrap = ip[24];
    o->dt_ctrl = 0.0;
    for (int d = 0; d < 3; ++d) { o->lo[d] = dp[d]; o->hi[d] = dp[3 + d]; o->g[d] = dp[7 + d]; }
    o->gamma = dp[6]; o->chi0 = dp[10]; o->rtol = dp[11]; o->atol = dp[12]; o->eta = dp[13];
    o->cfl_hydro = dp[14]; o->cfl_adv_max = dp[15]; o->cfl_rad_max = dp[16]; o->dt_max = dp[17];
    if (o->ndim == 2) { o->n[2] = 1; o->bc[2] = BC_PERIODIC; o->g[2] = 0.0; }
    for (int d = 0; d < 3; ++d) {
        o->dx[d] = (o->hi[d] - o->lo[d]) / o->n[d];
        o->idx[d] = 1.0 / o->dx[d];
        o->gh[d] = d < o->ndim ? GH : 0;
        o->pn[d] = o->n[d] + 2 * o->gh[d];
    }
    o->N = (long)o->n[0] * o->n[1] * o->n[2];
    if (o->sph) sph_tables(o);
    o->nlev = count_levels(o);
    o->P = (long)o->pn[0] * o->pn[1] * o->pn[2];
    o->nvar = 2 + o->ndim;
    o->nvec = o->nvar * o->N;
    o->nunk = o->nvec;
    for (int d = 0; d < o->ndim; ++d) if (o->bc[d] == BC_WALL) o->nunk -= o->N / o->n[d];
    o->u = calloc(o->nvec, sizeof(double));
    o->un = calloc(o->nvec, sizeof(double));
    o->uprev = calloc(o->nvec, sizeof(double));
    o->ux = calloc(o->nvec, sizeof(double));
    o->Fx = calloc(o->nvec, sizeof(double));
    o->b = calloc(o->nvec, sizeof(double));
    o->F = calloc(o->nvec, sizeof(double));
    o->w1 = calloc(o->nvec, sizeof(double));
    o->w2 = calloc(o->nvec, sizeof(double));
    o->R1 = calloc(o->nvec, sizeof(double));
    o->Ru = calloc(o->nvec, sizeof(double));
    o->sbal = calloc(o->N, sizeof(double));
    o->pc_W = calloc(o->N, sizeof(double));
    double **pp[] = {&o->rho, &o->eps, &o->p, &o->T, &o->chi, &o->q};
    for (size_t i = 0; i < 6; ++i) *pp[i] = calloc(o->P, sizeof(double));
    for (int d = 0; d < 3; ++d) {
        o->uf[d] = calloc(o->P, sizeof(double));
        o->m[d] = calloc(o->P, sizeof(double));
        o->fr[d] = calloc(o->P, sizeof(double));
        o->fe[d] = calloc(o->P, sizeof(double));
        for (int e = 0; e < 3; ++e) o->phic[d][e] = calloc(o->P, sizeof(double));
        o->pc_hf[d] = calloc(o->N, sizeof(double));
        o->pc_kap[d] = calloc(o->N, sizeof(double));
        o->pc_beta[d] = calloc(o->N, sizeof(double));
    }
    int nmax = o->n[0];
    if (o->n[1] > nmax) nmax = o->n[1];
    if (o->n[2] > nmax) nmax = o->n[2];
    o->la = calloc(nmax, sizeof(double)); o->lb = calloc(nmax, sizeof(double));
    o->lc = calloc(nmax, sizeof(double)); o->ld = calloc(nmax, sizeof(double));
    o->lx = calloc(nmax, sizeof(double)); o->lt1 = calloc(5 * nmax, sizeof(double));
    o->lt2 = calloc(nmax, sizeof(double));
    memcpy(o->u, u0, sizeof(double) * o->nvec);
    for (int f = 0; f < 5; ++f) o->scale[f] = 1.0;
    freeze_sources(o, o->u);
    return o;
}

void or_destroy(void *h) { or_free((Or *)h); }

void or_set_state(void *h, const double *u) {
    Or *o = h;
    memcpy(o->u, u, sizeof(double) * o->nvec);
    o->have_prev = 0;
}
/* the last solve's extrapolated first iterate: out[0] its residual norm
 * (-1 when none was tried), out[1] 1 when the solve started from it */
void or_extrap_info(void *h, double *out) {
    Or *o = h;
    out[0] = o->st_fx;
    out[1] = o->st_extrap;
}
void or_get_state(void *h, double *u) { Or *o = h; memcpy(u, o->u, sizeof(double) * o->nvec); }

/* R(u) */
void or_rhs(void *h, const double *u, double *R) { rhs((Or *)h, u, R); }

/* b = u^n + dt/2 R(u^n) */
void or_cn_old(void *h, const double *un, double dt, double *b) { cn_old((Or *)h, un, dt, b); }

/* F(u) */
void or_residual(void *h, const double *u, const double *b, double dt, double *F) {
    cn_residual((Or *)h, u, b, dt, F);
}

/* dt and scales from a state; out: dt, hyd, adv, rad, scale[0..4] */
void or_time_step(void *h, const double *u, double *out) {
    Or *o = h;
    double hy, ad, ra;
    out[0] = time_step(o, u, &hy, &ad, &ra);
    out[1] = hy; out[2] = ad; out[3] = ra;
    for (int f = 0; f < 5; ++f) out[4 + f] = o->scale[f];
}

/* set the scales explicitly (5 values) */
void or_set_scales(void *h, const double *s) { Or *o = h; for (int f = 0; f < 5; ++f) o->scale[f] = s[f]; }

/* Jv with F(u) recomputed from (u, b, dt) */
void or_jv(void *h, const double *u, const double *b, double dt, const double *v, double *w) {
    Or *o = h;
    double *Ru = calloc(o->nvec, sizeof(double));
    (void)b; /* the product does not depend on the old-time term */
    rhs(o, u, Ru);
    double urms = snorm2(o, u) / sqrt((double)o->nunk);
    jv(o, u, Ru, dt, urms, v, w);
    free(Ru);
}

/* threads the parallel loops run on (1 in the serial build) */
int or_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Jv at a given difference step eps > 0 (F(u) recomputed from u) */
void or_jv_eps(void *h, const double *u, const double *b, double dt, const double *v, double eps, double *w) {
    Or *o = h;
    double *Ru = calloc(o->nvec, sizeof(double));
    (void)b;
    rhs(o, u, Ru);
    jv_at(o, u, Ru, dt, eps, v, w);
    free(Ru);
}

/* z = P^{-1} v with coefficients frozen at u */
void or_precond(void *h, const double *u, double dt, const double *v, double *z) {
    Or *o = h;
    pc_build(o, u, dt);
    pc_apply(o, v, z);
}

static void fill_stats(Or *o, double *st) {
    st[0] = o->t; st[1] = o->st_dt; st[2] = o->st_cfl_h; st[3] = o->st_cfl_a; st[4] = o->st_cfl_r;
    st[5] = o->st_rel_res; st[6] = o->st_max_rel_corr; st[7] = o->st_mass_drift;
    st[8] = o->st_energy_drift; st[9] = o->st_newton; st[10] = o->st_gmres;
    st[11] = o->st_rejections; st[12] = o->st_status; st[13] = o->st_f0; st[14] = o->st_f;
    st[15] = o->st_exit;
}

/* the last Newton solve's history (see Or.hist_*): returns the number of
 * residual norms written to f; eta and lin receive one fewer entries */
int or_newton_history(void *h, double *f, double *eta, double *lin, int max) {
    Or *o = h;
    int n = o->hist_n < max ? o->hist_n : max;
    for (int k = 0; k < n; ++k) {
        f[k] = o->hist_f[k];
        if (k + 1 < n) { eta[k] = o->hist_eta[k]; lin[k] = o->hist_lin[k]; }
    }
    return n;
}

/* one Crank-Nicolson step at the given dt (no retry) */
int or_newton_solve(void *h, double dt, double *stats) {
    Or *o = h;
    o->st_rejections = 0;
    int s = step_at(o, dt);
    if (s == 0) o->t += dt;
    double hy, ad, ra;
    time_step(o, o->un, &hy, &ad, &ra);
    o->st_cfl_h = dt * hy; o->st_cfl_a = dt * ad; o->st_cfl_r = dt * ra;
    fill_stats(o, stats);
    return s;
}

/* one adaptive step: dt from the CFL limits, halved on failure */
int or_implicit_step(void *h, double *stats) {
    Or *o = h;
    double hy, ad, ra;
    double dt = time_step(o, o->u, &hy, &ad, &ra);
    /* the controller bounds dt by the previous accepted dt times a factor
     * set by that step's Newton count; the CFL limits still apply */
    int ctrl = o->dt_grow > 1.0;
    if (ctrl && o->dt_ctrl > 0.0 && o->dt_ctrl < dt) dt = o->dt_ctrl;
    int rej = 0, s = 0;
    for (;;) {
        s = step_at(o, dt);
        if (s == 0 || rej >= o->max_halvings) break;
        rej++;
        dt = 0.5 * dt;
    }
    if (ctrl) {
        if (s == 0) {
            double f = o->dt_grow;
            if (o->newton_target > 0 && o->st_newton > 0) {
                double r = (double)o->newton_target / (double)o->st_newton;
                f = r < 0.5 ? 0.5 : (r > o->dt_grow ? o->dt_grow : r);
            }
            o->dt_ctrl = dt * f;
        } else {
            o->dt_ctrl = dt;
        }
    }
    if (s == 0) o->t += dt;
    o->st_rejections = rej;
    o->st_cfl_h = dt * hy; o->st_cfl_a = dt * ad; o->st_cfl_r = dt * ra;
    fill_stats(o, stats);
    return s;
}

/* passive scalars: nscal partial densities s_k = c_k rho (nscal * N values) */
void or_set_scalars(void *h, int nscal, int renorm, const double *s) {
    Or *o = h;
    free(o->sc); free(o->sc_n);
    o->nscal = nscal;
    o->renorm = renorm;
    o->sc = calloc((long)nscal * o->N + 1, sizeof(double));
    o->sc_n = calloc((long)nscal * o->N + 1, sizeof(double));
    memcpy(o->sc, s, sizeof(double) * (long)nscal * o->N);
}
void or_get_scalars(void *h, double *s) { Or *o = h; memcpy(s, o->sc, sizeof(double) * (long)o->nscal * o->N); }
void or_scalar_rhs(void *h, const double *u, const double *s, double *R) {
    Or *o = h;
    double *rho = calloc(o->N, sizeof(double)), *fr = calloc(3 * o->N, sizeof(double));
    mass_flux_cells(o, u, rho, fr);
    scalar_rhs(o, s, rho, fr, R);
    free(rho); free(fr);
}
int or_scalar_its(void *h, int *out) { Or *o = h; out[0] = o->st_sc_newton; out[1] = o->st_sc_gmres; return 0; }

/* frozen wall fluxes and heat-balance source: for tests */
void or_get_sources(void *h, double *sbal) { Or *o = h; memcpy(sbal, o->sbal, sizeof(double) * o->N); }

/* dense helpers for the Krylov pins */
void or_tridiag(int n, const double *a, const double *b, const double *c, const double *d,
                double *x, int periodic) {
    double *t = calloc(5 * (size_t)n, sizeof(double)), *t2 = calloc(n, sizeof(double));
    if (periodic) cyclic(n, a, b, c, d, x, t);
    else thomas(n, a, b, c, d, x, t, t2);
    free(t); free(t2);
}

typedef struct { long n; const double *A, *M; } DCtx;
static void dmat(void *ctx, const double *x, double *y) {
    DCtx *c = ctx;
    for (long i = 0; i < c->n; ++i) {
        double s = 0.0;
        for (long j = 0; j < c->n; ++j) s += c->A[i * c->n + j] * x[j];
        y[i] = s;
    }
}
static void dpre(void *ctx, const double *x, double *y) {
    DCtx *c = ctx;
    if (!c->M) { memcpy(y, x, sizeof(double) * c->n); return; }
    for (long i = 0; i < c->n; ++i) {
        double s = 0.0;
        for (long j = 0; j < c->n; ++j) s += c->M[i * c->n + j] * x[j];
        y[i] = s;
    }
}

/* GMRES on an explicit matrix with an optional explicit right preconditioner
 * M (approximate inverse).  info: its, cycles, converged, res, beta0 */
void or_gmres_dense(long n, const double *A, const double *M, const double *b, double *x,
                    int m, int max_cycles, double eta, double *info) {
    DCtx c = {n, A, M};
    GmresInfo gi;
    gmres(n, dmat, dpre, &c, b, x, m, max_cycles, eta, &gi);
    info[0] = gi.its; info[1] = gi.cycles; info[2] = gi.converged; info[3] = gi.res; info[4] = gi.beta0;
}
