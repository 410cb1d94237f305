// Residual of the Crank-Nicolson system on the staggered grid (section 2 of
// Goffrey et al. 2016): R(u) of eqs. (1)-(3) in total-energy form (or with the
// internal-energy variable of eq. 2: flux rho e u, -p div u at cell centres,
// no gravitational work) with gravity as a body force and conduction
// chi = chi0 T^3, upstream linear extrapolation with the van Leer limiter, and
// the three consumers
//   b = u + dt/2 R(u)                 (old-time half of Crank-Nicolson)
//   F = (u - b) - dt/2 R(u)           (residual; at a Newton iterate it is
//                                      written as -S^-1 F, the right-hand side)
//   w = v - dt/2 (R(u + eps S v) - R(u)) / (eps S)   (Jacobian-free product:
//       the difference quotient of F, whose part u - b is linear, with only
//       R differenced)
// Four sweeps: cell primitives, face fluxes of mass and energy, momentum
// transport fluxes, then the cell and face outputs.
#include "kernels.hpp"

namespace jfnk {

// PERT: 0 the state itself; 1 perturbed along the FP64 direction v; 2 along
// the FP32 direction vf (the mixed form's preconditioned basis vectors)
template <int PERT>
__device__ __forceinline__ double dir_t(const StateView& s, long x) {
    return PERT == 2 ? (double)s.vf[x] : s.v[x];
}
// value of state field f at cell c, perturbed along the direction when PERT
template <int PERT>
__device__ __forceinline__ double st_t(const StateView& s, int f, long c) {
    const long x = (long)f * s.N + c;
    double a = s.u[x];
    if (PERT) a = a + (s.eps[0] * s.scale[f]) * dir_t<PERT>(s, x);
    return a;
}

// ---------------------------------------------------------------- sweep 1: primitives per cell
// PERT (state perturbed along a direction) is compile-time so that the
// state loads form one straight-line block
template <int ND, int PERT>
__global__ void __launch_bounds__(kBlock) k_prim(Grid G, StateView s, Prim P) {
    Ijk q;
    long c;
    if (!cell_from_launch(G, q, c)) return;
    const auto st = [&](int f, long cc) { return st_t<PERT>(s, f, cc); };
    const double rho = st(0, c), E = st(1, c);
    double qk = 0.0;
    for (int d = 0; d < ND; ++d) {
        const bool wall = G.bc[d] == WALL;
        // both neighbours are loaded on walls too (the periodic wrap keeps
        // them in bounds) and the wall faces' values replaced by 0
        const long cu = shifted(G, q, d, 1);
        const double rl = st(0, shifted(G, q, d, -1)), ru = st(0, cu);
        const double ml = st(2 + d, c), mu = st(2 + d, cu);
        const double a0 = ml / (0.5 * (rl + rho)), b0 = mu / (0.5 * (rho + ru));
        const double a = (wall && q.v[d] == 0) ? 0.0 : a0;
        const double b = (wall && q.v[d] == G.n[d] - 1) ? 0.0 : b0;
        qk = qk + 0.5 * (a * a + b * b);
        P.uf[d][c] = a;
    }
    const double kin = 0.5 * rho * qk;
    const double p = G.internal ? G.gm1 * E : G.gm1 * (E - kin);  // E holds rho e in the internal form
    P.rho[c] = rho;
    P.p[c] = p;
    P.eps[c] = E / rho;
    if (G.has_wall || G.has_chi) {
        const double T = p / rho;
        P.T[c] = T;
        if (G.has_chi) P.chi[c] = G.chi0 * (T * T * T);
    }
    if (G.has_wall) P.q[c] = qk;
}

// The same sweep on a 3D grid without walls, with the workgroup's in-plane
// tile (kBx x kBy cells and 1 on every in-plane side) of the density and of
// the momenta along x and y, each formed once (perturbed when PERT), staged
// in LDS: per cell the loads of the neighbours one plane away along z and of
// the cell's own energy and z momentum stay in memory.  Every axis has at
// least 4 cells, so one periodic wrap brings each halo entry into the grid;
// entries still outside it (a tile wider than the grid) are left unset and
// never read.  The values and the order of the arithmetic are those of k_prim.
constexpr int kPhx = kBx + 2, kPhy = kBy + 2;
template <int PERT>
__global__ void __launch_bounds__(kBlock) k_prim_tile3(Grid G, StateView s, Prim P) {
    __shared__ double srho[kPhy][kPhx], sm0[kPhy][kPhx], sm1[kPhy][kPhx];
    const auto st = [&](int f, long cc) { return st_t<PERT>(s, f, cc); };
    const Tile tl = xcd_tile();
    const int i0 = (int)tl.x * kBx, j0 = (int)tl.y * kBy, k = (int)tl.z;
    const int tid = (int)(threadIdx.x + kBx * threadIdx.y);
    for (int e = tid; e < kPhx * kPhy; e += kBlock) {
        const int hx = e % kPhx, hy = e / kPhx;
        int i = i0 - 1 + hx, j = j0 - 1 + hy;
        if (i < 0) i += G.n[0];
        else if (i >= G.n[0]) i -= G.n[0];
        if (j < 0) j += G.n[1];
        else if (j >= G.n[1]) j -= G.n[1];
        if (i >= G.n[0] || j >= G.n[1]) continue;  // tile wider than the grid
        const long c = flat(G, i, j, k);
        srho[hy][hx] = st(0, c);
        // m_x is read at the cell and its upper x neighbour, m_y at the cell
        // and its upper y neighbour
        if (hy >= 1 && hy <= kBy && hx >= 1) sm0[hy][hx] = st(2, c);
        if (hx >= 1 && hx <= kBx && hy >= 1) sm1[hy][hx] = st(3, c);
    }
    __syncthreads();
    Ijk q;
    long c;
    if (!cell_from_launch(G, q, c)) return;
    const int tx = (int)threadIdx.x + 1, ty = (int)threadIdx.y + 1;
    const double rho = srho[ty][tx], E = st(1, c);
    double qk = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double rl, ru, ml, mu;
        if (d == 0) {
            rl = srho[ty][tx - 1];
            ru = srho[ty][tx + 1];
            ml = sm0[ty][tx];
            mu = sm0[ty][tx + 1];
        } else if (d == 1) {
            rl = srho[ty - 1][tx];
            ru = srho[ty + 1][tx];
            ml = sm1[ty][tx];
            mu = sm1[ty + 1][tx];
        } else {
            const long cu = shifted(G, q, 2, 1);
            rl = st(0, shifted(G, q, 2, -1));
            ru = st(0, cu);
            ml = st(4, c);
            mu = st(4, cu);
        }
        const double a = ml / (0.5 * (rl + rho)), b = mu / (0.5 * (rho + ru));
        qk = qk + 0.5 * (a * a + b * b);
        P.uf[d][c] = a;
    }
    const double kin = 0.5 * rho * qk;
    const double p = G.internal ? G.gm1 * E : G.gm1 * (E - kin);  // E holds rho e in the internal form
    P.rho[c] = rho;
    P.p[c] = p;
    P.eps[c] = E / rho;
    if (G.has_chi) {
        const double T = p / rho;
        P.T[c] = T;
        P.chi[c] = G.chi0 * (T * T * T);
    }
}

// ---------------------------------------------------------------- sweep 2: fluxes on lower faces

// Ghost-cell values one layer beyond a wall: temperature extrapolated
// linearly, density from the discrete hydrostatic balance across the wall
// face, specific energy from the ghost temperature (plus the mirrored kinetic
// energy in the total-energy form) (section 3.1).  c0 is the wall cell, c1
// its inner neighbour.
struct Ghost {
    double rho, eps;
};
__device__ __forceinline__ Ghost wall_ghost(const Grid& G, const Prim& P, long c0, long c1, int d,
                                            bool top) {
    const double hg = 0.5 * G.g[d] * G.dx[d];
    const double T0 = P.T[c0], T1 = P.T[c1];
    const double Tg = 2.0 * T0 - T1;
    Ghost gh;
    gh.rho = top ? P.rho[c0] * (T0 + hg) / (Tg - hg) : P.rho[c0] * (T0 - hg) / (Tg + hg);
    gh.eps = G.internal ? Tg / G.gm1 : Tg / G.gm1 + 0.5 * P.q[c0];
    return gh;
}

// In-plane tile of the flux sweep in LDS: the workgroup's kBx x kBy cells
// with the halo the reconstruction reads along x and y (2 below, 1 above);
// out-of-domain entries beyond a wall are never read.
constexpr int kFhx = kBx + 3, kFhy = kBy + 3;
struct FluxTile {
    double rho[kFhy][kFhx], eps[kFhy][kFhx], p[kFhy][kFhx], T[kFhy][kFhx], chi[kFhy][kFhx];
};

template <int ND>
__global__ void __launch_bounds__(kBlock) k_flux(Grid G, Prim P, Flux Fx, WallFlux W) {
    __shared__ FluxTile sm;
    const Tile tl = xcd_tile();
    const int i0 = (int)tl.x * kBx, j0 = (int)tl.y * kBy, k = (int)tl.z;
    const int tid = (int)(threadIdx.x + kBx * threadIdx.y);
    for (int e = tid; e < kFhx * kFhy; e += kBlock) {
        const int hx = e % kFhx, hy = e / kFhx;
        int i = i0 - 2 + hx, j = j0 - 2 + hy;
        if (i < 0 || i >= G.n[0]) {
            if (G.bc[0] == WALL) continue;
            i = i < 0 ? i + G.n[0] : i - G.n[0];
        }
        if (j < 0 || j >= G.n[1]) {
            if (G.bc[1] == WALL) continue;
            j = j < 0 ? j + G.n[1] : j - G.n[1];
        }
        if (i < 0 || i >= G.n[0] || j < 0 || j >= G.n[1]) continue;  // tile wider than the grid
        const long c = flat(G, i, j, k);
        sm.rho[hy][hx] = P.rho[c];
        sm.eps[hy][hx] = P.eps[c];
        sm.p[hy][hx] = P.p[c];
        if (G.has_chi) {
            sm.T[hy][hx] = P.T[c];
            sm.chi[hy][hx] = P.chi[c];
        }
    }
    __syncthreads();
    Ijk q;
    long c;
    if (!cell_from_launch(G, q, c)) return;
    const int tx = (int)threadIdx.x + 2, ty = (int)threadIdx.y + 2;
    for (int d = 0; d < ND; ++d) {
        const bool wall = G.bc[d] == WALL;
        const int id = q.v[d];
        if (wall && id == 0) {
            Fx.fr[d][c] = 0.0;
            Fx.fe[d][c] = W.lo[d] ? W.lo[d][transverse(G, q, d)] : 0.0;
            continue;
        }
        // neighbour s along d: LDS for the in-plane axes, memory along z
        const int ox = d == 0 ? 1 : 0, oy = d == 1 ? 1 : 0;
        auto rho_at = [&](int s) { return d < 2 ? sm.rho[ty + s * oy][tx + s * ox] : P.rho[shifted(G, q, d, s)]; };
        auto eps_at = [&](int s) { return d < 2 ? sm.eps[ty + s * oy][tx + s * ox] : P.eps[shifted(G, q, d, s)]; };
        const long L = shifted(G, q, d, -1);
        const double v = P.uf[d][c];
        const double rc = rho_at(0), rL = rho_at(-1), ec = eps_at(0), eL = eps_at(-1);
        // second neighbours loaded everywhere (in bounds by the wrap; beyond
        // a wall in the LDS tile the entry is unset and replaced) and
        // replaced by the ghost values next to a wall
        double rLL = rho_at(-2), eLL = eps_at(-2), rR = rho_at(1), eR = eps_at(1);
        if (wall && id == 1) {
            const Ghost gh = wall_ghost(G, P, L, c, d, false);
            rLL = gh.rho;
            eLL = gh.eps;
        }
        if (wall && id == G.n[d] - 1) {
            const Ghost gh = wall_ghost(G, P, c, L, d, true);
            rR = gh.rho;
            eR = gh.eps;
        }
        const double sl = van_leer(rc - rL, rL - rLL);
        const double sr = van_leer(rR - rc, rc - rL);
        const double rf = upstream(v, rL, sl, rc, sr);
        const double el = van_leer(ec - eL, eL - eLL);
        const double er = van_leer(eR - ec, ec - eL);
        const double ef = upstream(v, eL, el, ec, er);
        const double f_rho = v * rf;
        const double pL = d < 2 ? sm.p[ty - oy][tx - ox] : P.p[L], pc = d < 2 ? sm.p[ty][tx] : P.p[c];
        double f_e = G.internal ? f_rho * ef : f_rho * ef + v * (0.5 * (pL + pc));
        if (G.has_chi) {
            const double chiL = d < 2 ? sm.chi[ty - oy][tx - ox] : P.chi[L], chic = d < 2 ? sm.chi[ty][tx] : P.chi[c];
            const double TL = d < 2 ? sm.T[ty - oy][tx - ox] : P.T[L], Tc = d < 2 ? sm.T[ty][tx] : P.T[c];
            f_e = f_e + ((-0.5 * (chiL + chic)) * (Tc - TL)) * face_ids(G, d, q.v[0]);
        }
        Fx.fr[d][c] = f_rho;
        Fx.fe[d][c] = f_e;
    }
}

// ---------------------------------------------------------------- sweep 3: outputs

// Velocity component d on the d-face with index a along d (row of the
// other coordinates of q), across walls: the wall faces carry 0 and faces
// beyond a wall are the negated mirror images (reflecting wall).
// WALLS: the grid has a wall on some axis (compile-time; without walls every
// axis wraps and the sweep has no wall branches)
template <bool WALLS>
__device__ __forceinline__ double uf_normal(const Grid& G, const Prim& P, const Ijk& q, int d, int a) {
    const int n = G.n[d];
    if (WALLS && G.bc[d] == WALL) {
        double sgn = 1.0;
        if (a < 0) { a = -a; sgn = -1.0; }
        else if (a > n) { a = 2 * n - a; sgn = -1.0; }
        if (a == n) return 0.0;
        return sgn * P.uf[d][flat(G, d == 0 ? a : q.v[0], d == 1 ? a : q.v[1], d == 2 ? a : q.v[2])];
    }
    if (a < 0) a += n;
    else if (a >= n) a -= n;
    return P.uf[d][flat(G, d == 0 ? a : q.v[0], d == 1 ? a : q.v[1], d == 2 ? a : q.v[2])];
}

// Velocity component c on its face at row a along another axis e, across
// walls of e: stress-free mirror images.
template <bool WALLS>
__device__ __forceinline__ double uf_tangential(const Grid& G, const Prim& P, const Ijk& q, int c, int e,
                                                int a) {
    const int n = G.n[e];
    if (WALLS && G.bc[e] == WALL) {
        if (a < 0) a = -1 - a;
        else if (a >= n) a = 2 * n - 1 - a;
    } else {
        if (a < 0) a += n;
        else if (a >= n) a -= n;
    }
    return P.uf[c][flat(G, e == 0 ? a : q.v[0], e == 1 ? a : q.v[1], e == 2 ? a : q.v[2])];
}

// Momentum transported by the mass flux F through a side of a staggered
// control volume: F times the velocity extrapolated upstream to the side
// from the four values ua, ub | uc, ud around it (van Leer slopes).
__device__ __forceinline__ double transported(double F, double ua, double ub, double uc, double ud) {
    const double sl = van_leer(uc - ub, ub - ua);
    const double sr = van_leer(ud - uc, uc - ub);
    return F * upstream(F, ub, sl, uc, sr);
}

// Cell-centred momentum flux of component d along d at the cell with
// coordinates x (x on or inside the domain along d).
template <bool WALLS>
__device__ __forceinline__ double phi_cell(const Grid& G, const Prim& P, const Flux& Fx, const Ijk& x,
                                           int d) {
    const long c = flat(G, x.v[0], x.v[1], x.v[2]);
    const bool top = WALLS && G.bc[d] == WALL && x.v[d] == G.n[d] - 1;
    const double fhi = top ? 0.0 : Fx.fr[d][shifted(G, x, d, 1)];
    const double Fb = 0.5 * (Fx.fr[d][c] + fhi);
    const int a0 = x.v[d];
    const double ua = uf_normal<WALLS>(G, P, x, d, a0 - 1), ub = uf_normal<WALLS>(G, P, x, d, a0);
    const double uc = uf_normal<WALLS>(G, P, x, d, a0 + 1), ud = uf_normal<WALLS>(G, P, x, d, a0 + 2);
    return transported(Fb, ua, ub, uc, ud);
}

// Edge momentum flux of component d along e != d at the lower e-side of the
// d-face whose cell has coordinates x; x.v[e] may equal n_e (upper edge).
template <bool WALLS>
__device__ __forceinline__ double phi_edge(const Grid& G, const Prim& P, const Flux& Fx, Ijk x, int d,
                                           int e) {
    const int ne = G.n[e];
    double Gm;
    const int a0 = x.v[e];
    if (WALLS && G.bc[e] == WALL && (a0 == 0 || a0 == ne)) {
        Gm = 0.0;
    } else {
        Ijk xw = x;
        if (xw.v[e] >= ne) xw.v[e] -= ne;  // periodic wrap of the upper edge
        const long cx = flat(G, xw.v[0], xw.v[1], xw.v[2]);
        const long cl = shifted(G, xw, d, -1);
        Gm = 0.5 * (Fx.fr[e][cl] + Fx.fr[e][cx]);
    }
    const double ua = uf_tangential<WALLS>(G, P, x, d, e, a0 - 2), ub = uf_tangential<WALLS>(G, P, x, d, e, a0 - 1);
    const double uc = uf_tangential<WALLS>(G, P, x, d, e, a0), ud = uf_tangential<WALLS>(G, P, x, d, e, a0 + 1);
    return transported(Gm, ua, ub, uc, ud);
}

// Momentum transport fluxes of the staggered control volumes, one per
// (component, direction) and cell: cell-centred for d == e, at the lower
// e-edge of the d-face otherwise (wall faces, which are not unknowns, get 0).
// Each flux is stored as soon as it is formed (forming all before storing
// any measured slower: 114 VGPRs, occupancy 4).
template <int ND, bool WALLS>
__global__ void __launch_bounds__(kBlock) k_mflux(Grid G, Prim P, Flux Fx) {
    Ijk q;
    long c;
    if (!cell_from_launch(G, q, c)) return;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        Fx.phic[d][c] = phi_cell<WALLS>(G, P, Fx, q, d);
        const bool wallface = WALLS && G.bc[d] == WALL && q.v[d] == 0;
#pragma unroll
        for (int e = 0; e < ND; ++e) {
            if (e == d) continue;
            Fx.phie[d][e][c] = wallface ? 0.0 : phi_edge<WALLS>(G, P, Fx, q, d, e);
        }
    }
}

// The same fluxes on a 3D grid without walls, with the workgroup's in-plane
// tile of face velocities and mass fluxes (kBx x kBy cells and 2 on every
// in-plane side) staged in LDS: per cell 12 of the 54 loads above stay in
// memory, those one or two planes away along z.  Every axis has at least 4
// cells, so one periodic wrap brings each halo entry a cell of the tile reads
// into the grid; entries still outside it (a tile wider than the grid) are
// left unset and never read.
constexpr int kMhx = kBx + 4, kMhy = kBy + 4;
struct MfluxTile {
    double uf[3][kMhy][kMhx], fr[3][kMhy][kMhx];
};

__global__ void __launch_bounds__(kBlock) k_mflux_tile3(Grid G, Prim P, Flux Fx) {
    __shared__ MfluxTile sm;
    const Tile tl = xcd_tile();
    const int i0 = (int)tl.x * kBx, j0 = (int)tl.y * kBy, k = (int)tl.z;
    const int tid = (int)(threadIdx.x + kBx * threadIdx.y);
    for (int e = tid; e < kMhx * kMhy; e += kBlock) {
        const int hx = e % kMhx, hy = e / kMhx;
        int i = i0 - 2 + hx, j = j0 - 2 + hy;
        if (i < 0) i += G.n[0];
        else if (i >= G.n[0]) i -= G.n[0];
        if (j < 0) j += G.n[1];
        else if (j >= G.n[1]) j -= G.n[1];
        if (i >= G.n[0] || j >= G.n[1]) continue;  // tile wider than the grid
        const long c = flat(G, i, j, k);
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            sm.uf[f][hy][hx] = P.uf[f][c];
            sm.fr[f][hy][hx] = Fx.fr[f][c];
        }
    }
    __syncthreads();
    Ijk q;
    long c;
    if (!cell_from_launch(G, q, c)) return;
    const int tx = (int)threadIdx.x + 2, ty = (int)threadIdx.y + 2;
    // value of array a (component f) at s cells along axis ax from q
    const auto at = [&](const double* const* a, const double (*t)[kMhy][kMhx], int f, int ax, int s) {
        return ax == 2 && s != 0 ? a[f][shifted(G, q, 2, s)] : t[f][ty + (ax == 1 ? s : 0)][tx + (ax == 0 ? s : 0)];
    };
    const auto U = [&](int f, int ax, int s) { return at(P.uf, sm.uf, f, ax, s); };
    const auto FR = [&](int f, int ax, int s) { return at(Fx.fr, sm.fr, f, ax, s); };
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double Fb = 0.5 * (FR(d, d, 0) + FR(d, d, 1));
        Fx.phic[d][c] = transported(Fb, U(d, d, -1), U(d, d, 0), U(d, d, 1), U(d, d, 2));
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            if (e == d) continue;
            const double Gm = 0.5 * (FR(e, d, -1) + FR(e, d, 0));
            Fx.phie[d][e][c] = transported(Gm, U(d, e, -2), U(d, e, -1), U(d, e, 0), U(d, e, 1));
        }
    }
}

// Momentum right-hand side on a 2D spherical grid, on the staggered control
// volume of the lower d-face of cell q (not a wall face): transport fluxes
// through the volume's sides times their areas over its volume, the pressure
// gradient across the face, radial gravity, and the geometric terms
// +rho u_th^2 / r (radial) and -rho u_r u_th / r (polar) with the face
// density and the other component's mean over the four faces around.
__device__ __forceinline__ double sph_momentum(const Grid& G, const Prim& P, const Flux& Fx, const Ijk& q, long c,
                                               int d) {
    const SphMet& M = G.M;
    const int i = q.v[0], j = q.v[1];
    const long n0 = G.n[0];
    double a = 0.0;
    if (d == 0) {
        const long cl = c - 1;  // i - 1 (i >= 1: the wall face is excluded)
        const bool topj = j == G.n[1] - 1;
        const double rf = 0.5 * (P.rho[cl] + P.rho[c]);
        const double V = M.Vrc[i] * M.Vt[j];
        const double Ahi = M.r2c[i] * M.Vt[j], Alo = M.r2c[i - 1] * M.Vt[j];
        a = a - (Ahi * Fx.phic[0][c] - Alo * Fx.phic[0][cl]) / V;
        const double Bhi = M.hr2c[i] * M.stf[j + 1], Blo = M.hr2c[i] * M.stf[j];
        const double ehi = topj ? 0.0 : Fx.phie[0][1][c + n0];
        a = a - (Bhi * ehi - Blo * Fx.phie[0][1][c]) / V;
        a = a - (P.p[c] - P.p[cl]) * G.idx[0];
        if (G.g[0] != 0.0) a = a + rf * G.g[0];
        const double u1 = P.uf[1][cl], u2 = topj ? 0.0 : P.uf[1][cl + n0];
        const double u3 = P.uf[1][c], u4 = topj ? 0.0 : P.uf[1][c + n0];
        const double ut2 = 0.25 * (((u1 * u1 + u2 * u2) + u3 * u3) + u4 * u4);
        a = a + rf * ut2 / M.rfa[i];
    } else {
        const long cl = c - n0;  // j - 1 (j >= 1)
        const bool topi = i == G.n[0] - 1;
        const double rf = 0.5 * (P.rho[cl] + P.rho[c]);
        const double V = M.Vr[i] * M.Vtc[j];
        const double Ahi = M.r2f[i + 1] * M.Vtc[j], Alo = M.r2f[i] * M.Vtc[j];
        const double ehi = topi ? 0.0 : Fx.phie[1][0][c + 1];
        a = a - (Ahi * ehi - Alo * Fx.phie[1][0][c]) / V;
        const double Bhi = M.hr2[i] * M.stc[j], Blo = M.hr2[i] * M.stc[j - 1];
        a = a - (Bhi * Fx.phic[1][c] - Blo * Fx.phic[1][cl]) / V;
        a = a - (P.p[c] - P.p[cl]) * M.ith[i];
        const double ua = P.uf[0][cl], ub = topi ? 0.0 : P.uf[0][cl + 1];
        const double uc = P.uf[0][c], ud = topi ? 0.0 : P.uf[0][c + 1];
        const double ur = 0.25 * (((ua + ub) + uc) + ud);
        a = a - rf * ur * P.uf[1][c] / M.rc[i];
    }
    return a;
}

// MODE and PERT (state perturbed along v) are compile-time so that each
// instance's loads form straight-line blocks
// The outputs come as their own __restrict__ parameters (they never alias
// an input), so that the loads of a later field need not wait for the stores
// of an earlier one.
// KD (OUT_JV only): the number of basis vectors whose dots with the product
// are formed as its entries are (0: none)
template <int ND, int MODE, int PERT, int KD>
__global__ void __launch_bounds__(kBlock) k_out(Grid G, StateView s, Prim P, Flux Fx, WallFlux W,
                                                const double* __restrict__ sbal, OutSpec o,
                                                double* __restrict__ out, double* __restrict__ out2,
                                                double* __restrict__ rout, double* __restrict__ partial) {
    Ijk q;
    long c = 0;
    double part = 0.0, part_u = 0.0;
    double dacc[KD + 1];
#pragma unroll
    for (int i = 0; i <= KD; ++i) dacc[i] = 0.0;
    if (cell_from_launch(G, q, c)) {
        // consumer of field f's right-hand side Rf, called field by field in
        // order (each value is written as soon as it is formed)
        auto emit = [&](int f, double Rf) {
            const long x = (long)f * G.N + c;
            const bool wallface = f >= 2 && G.bc[f - 2] == WALL && q.v[f - 2] == 0;
            if (rout) rout[x] = Rf;
            if (MODE == OUT_RHS) {
                out[x] = Rf;
            } else if (MODE == OUT_CN_OLD) {
                const double u0 = s.u[x];
                const double b = u0 + o.h * Rf;
                out[x] = b;
                const double F = wallface ? 0.0 : (u0 - b) - o.h * Rf;
                out2[x] = o.neg_scaled ? -F / o.scale[f] : F;
                const double t = F / o.scale[f];
                part += t * t;
                const double tu = u0 * o.inv_scale[f];
                part_u += tu * tu;
            } else if (MODE == OUT_RESIDUAL) {
                const double uf = st_t<PERT>(s, f, c);
                const double F0 = (uf - o.b[x]) - o.h * Rf;  // loaded on wall faces too
                const double F = wallface ? 0.0 : F0;
                out[x] = o.neg_scaled ? -F / o.scale[f] : F;
                const double t = F / o.scale[f];
                part += t * t;
                const double tu = uf * o.inv_scale[f];
                part_u += tu * tu;
            } else {  // OUT_JV
                const double e = s.eps[0];
                const double w0 = dir_t<PERT>(s, x) - (o.h * (Rf - o.Ru[x])) / (e * s.scale[f]);  // loaded everywhere
                const double wv = (!wallface && e != 0.0) ? w0 : 0.0;
                out[x] = wv;
                if (KD > 0) {
                    const long ld = (long)(2 + ND) * G.N;
#pragma unroll
                    for (int i = 0; i < KD; ++i) {
                        const double vi = PERT == 2 ? (double)o.dotvf[(long)i * ld + x] : o.dotv[(long)i * ld + x];
                        dacc[i] += vi * wv;
                    }
                    dacc[KD] += wv * wv;
                }
            }
        };
        // mass and energy in the cell
        double ar = 0.0, ae = 0.0;
        for (int d = 0; d < ND; ++d) {
            const bool top = G.bc[d] == WALL && q.v[d] == G.n[d] - 1;
            // the upper neighbour's fluxes are loaded at a top wall too (the
            // wrap keeps them in bounds) and replaced by the wall's
            const long cu = shifted(G, q, d, 1);
            double frh = Fx.fr[d][cu], feh = Fx.fe[d][cu];
            if (top) {
                frh = 0.0;
                feh = W.hi[d] ? W.hi[d][transverse(G, q, d)] : 0.0;
            }
            if (G.sph) {
                // (1/V) sum of area-weighted face fluxes
                const int i = q.v[0], j = q.v[1];
                const double V = sph_vol(G, i, j);
                const double Alo = sph_area(G, d, i, j), Ahi = sph_area(G, d, d == 0 ? i + 1 : i, d == 1 ? j + 1 : j);
                ar = ar - (Ahi * frh - Alo * Fx.fr[d][c]) / V;
                ae = ae - (Ahi * feh - Alo * Fx.fe[d][c]) / V;
                continue;
            }
            ar = ar - (frh - Fx.fr[d][c]) * G.idx[d];
            ae = ae - (feh - Fx.fe[d][c]) * G.idx[d];
        }
        if (G.internal) {
            // -p div u with the cell's face velocities
            const double pc = P.p[c];
            for (int d = 0; d < ND; ++d) {
                const bool top = G.bc[d] == WALL && q.v[d] == G.n[d] - 1;
                const double ulo = P.uf[d][c];
                const double uu = P.uf[d][shifted(G, q, d, 1)];  // wrapped at a top wall, replaced by 0
                const double uhi = top ? 0.0 : uu;
                if (G.sph) {
                    const int i = q.v[0], j = q.v[1];
                    const double V = sph_vol(G, i, j);
                    const double Alo = sph_area(G, d, i, j), Ahi = sph_area(G, d, d == 0 ? i + 1 : i, d == 1 ? j + 1 : j);
                    ae = ae - pc * ((Ahi * uhi - Alo * ulo) / V);
                    continue;
                }
                ae = ae - pc * ((uhi - ulo) * G.idx[d]);
            }
        } else {
            for (int d = 0; d < ND; ++d) {
                if (G.g[d] == 0.0) continue;
                const bool top = G.bc[d] == WALL && q.v[d] == G.n[d] - 1;
                const double mlo = st_t<PERT>(s, 2 + d, c);
                const double mu = st_t<PERT>(s, 2 + d, shifted(G, q, d, 1));  // wrapped at a top wall, replaced by 0
                const double mhi = top ? 0.0 : mu;
                ae = ae + G.g[d] * (0.5 * (mlo + mhi));
            }
        }
        if (G.heat_balance && sbal) ae = ae + sbal[c];
        emit(0, ar);
        emit(1, ae);
        // momentum on the lower faces
        for (int d = 0; d < ND; ++d) {
            const bool wallface = G.bc[d] == WALL && q.v[d] == 0;
            if (G.sph) {
                emit(2 + d, wallface ? 0.0 : sph_momentum(G, P, Fx, q, c, d));
                continue;
            }
            // formed on a wall face too (the wrapped lower neighbour is in
            // bounds) and replaced by 0 there
            double a = 0.0;
            const long cl = shifted(G, q, d, -1);
#pragma unroll
            for (int e = 0; e < ND; ++e) {
                if (e == d) {
                    a = a - (Fx.phic[d][c] - Fx.phic[d][cl]) * G.idx[d];
                } else {
                    // the edge above along e; on a wall of e it carries no flux
                    const double pu = Fx.phie[d][e][shifted(G, q, e, 1)];
                    const double up = (G.bc[e] == WALL && q.v[e] == G.n[e] - 1) ? 0.0 : pu;
                    a = a - (up - Fx.phie[d][e][c]) * G.idx[e];
                }
            }
            a = a - (P.p[c] - P.p[cl]) * G.idx[d];
            if (G.g[d] != 0.0) a = a + (0.5 * (P.rho[cl] + P.rho[c])) * G.g[d];
            emit(2 + d, wallface ? 0.0 : a);
        }
    }
    if (partial) {
        __shared__ double sh[kBlock / 64];
        const double t = block_sum(part, sh);
        if (lin_thread() == 0) partial[lin_block()] = t;
    }
    if (KD > 0)
        block_sum_cols<KD + 1>(dacc, o.dot_part, lin_thread(), (long)lin_block(),
                               (long)gridDim.x * gridDim.y * gridDim.z);
    if (MODE != OUT_JV && o.partial_u) {
        __shared__ double shu[kBlock / 64];
        const double t = block_sum(part_u, shu);
        if (lin_thread() == 0) o.partial_u[lin_block()] = t;
    }
}

// ---------------------------------------------------------------- time step and scales (eqs. 5-7)
template <int ND>
__global__ void __launch_bounds__(kBlock) k_dt_partial(Grid G, Prim P, const double* __restrict__ u,
                                                        double* __restrict__ part) {
    Ijk q;
    long c = 0;
    double hyd = 0.0, adv = 0.0, rad = 0.0, rmax = 0.0, emax = 0.0, cmax = 0.0;
    if (cell_from_launch(G, q, c)) {
        const double r = P.rho[c];
        const double cs = sqrt(G.gamma * P.p[c] / r);
        const double cp = G.gamma / G.gm1;
        for (int d = 0; d < ND; ++d) {
            const bool top = G.bc[d] == WALL && q.v[d] == G.n[d] - 1;
            const double a = fabs(P.uf[d][c]);
            const double b = top ? 0.0 : fabs(P.uf[d][shifted(G, q, d, 1)]);
            const double ud = a > b ? a : b;
            const double ids = face_ids(G, d, q.v[0]);
            hyd = fmax(hyd, (ud + cs) * ids);
            adv = fmax(adv, ud * ids);
            if (G.has_chi) {
                const double D = P.chi[c] / (r * cp);
                rad = fmax(rad, D * (ids * ids));
            }
        }
        rmax = r;
        emax = u[G.N + c];
        cmax = cs;
    }
    __shared__ double sh[kBlock / 64];
    double vals[6] = {hyd, adv, rad, rmax, emax, cmax};
    for (int k = 0; k < 6; ++k) {
        const double m = block_max(vals[k], sh);
        if (lin_thread() == 0) part[(long)k * (gridDim.x * gridDim.y * gridDim.z) + lin_block()] = m;
        __syncthreads();
    }
}

// ---------------------------------------------------------------- host launchers

// the output sweep's instance for the mode, the perturbation flag and (for
// products) the number of basis vectors dotted
template <int ND, int MODE, int PERT>
static void launch_out_k(const Grid& G, const StateView& s, const Prim& P, const Flux& Fx, const WallFlux& W,
                         const double* sbal, const OutSpec& o, hipStream_t stream) {
    const dim3 g = cell_grid3(G.n), bl(kBx, kBy);
#define OUTK(KD) \
    JFNK_KLAUNCH((k_out<ND, MODE, PERT, KD>), g, bl, 0, stream, G, s, P, Fx, W, sbal, o, o.out, o.out2, o.rout, o.partial)
    if (MODE == OUT_JV && PERT != 0) {
        static_assert(kJvDotsMax == 4, "instances below");
        switch (o.dotk) {
            case 1: OUTK(1); return;
            case 2: OUTK(2); return;
            case 3: OUTK(3); return;
            case 4: OUTK(4); return;
            default: break;
        }
    }
    OUTK(0);
#undef OUTK
}
template <int ND, int MODE>
static void launch_out_m(const Grid& G, const StateView& s, const Prim& P, const Flux& Fx, const WallFlux& W,
                         const double* sbal, const OutSpec& o, hipStream_t stream) {
    if (s.v) launch_out_k<ND, MODE, 1>(G, s, P, Fx, W, sbal, o, stream);
    else if (MODE == OUT_JV && s.vf) launch_out_k<ND, MODE == OUT_JV ? MODE : OUT_JV, 2>(G, s, P, Fx, W, sbal, o, stream);
    else launch_out_k<ND, MODE, 0>(G, s, P, Fx, W, sbal, o, stream);
}
template <int ND>
static void launch_out_nd(const Grid& G, const StateView& s, const Prim& P, const Flux& Fx, const WallFlux& W,
                          const double* sbal, const OutSpec& o, hipStream_t stream) {
    switch (o.mode) {
        case OUT_RHS: launch_out_m<ND, OUT_RHS>(G, s, P, Fx, W, sbal, o, stream); break;
        case OUT_CN_OLD: launch_out_m<ND, OUT_CN_OLD>(G, s, P, Fx, W, sbal, o, stream); break;
        case OUT_RESIDUAL: launch_out_m<ND, OUT_RESIDUAL>(G, s, P, Fx, W, sbal, o, stream); break;
        default: launch_out_m<ND, OUT_JV>(G, s, P, Fx, W, sbal, o, stream); break;
    }
}

static void launch_prim_kernel(const Grid& G, const StateView& s, const Prim& P, hipStream_t stream) {
    const dim3 g = cell_grid3(G.n), bl(kBx, kBy);
    if (G.ndim == 3) {
        if (G.has_wall) {
            if (s.v) JFNK_KLAUNCH((k_prim<3, 1>), g, bl, 0, stream, G, s, P);
            else if (s.vf) JFNK_KLAUNCH((k_prim<3, 2>), g, bl, 0, stream, G, s, P);
            else JFNK_KLAUNCH((k_prim<3, 0>), g, bl, 0, stream, G, s, P);
        } else {
            if (s.v) JFNK_KLAUNCH((k_prim_tile3<1>), g, bl, 0, stream, G, s, P);
            else if (s.vf) JFNK_KLAUNCH((k_prim_tile3<2>), g, bl, 0, stream, G, s, P);
            else JFNK_KLAUNCH((k_prim_tile3<0>), g, bl, 0, stream, G, s, P);
        }
    } else {
        if (s.v) JFNK_KLAUNCH((k_prim<2, 1>), g, bl, 0, stream, G, s, P);
        else if (s.vf) JFNK_KLAUNCH((k_prim<2, 2>), g, bl, 0, stream, G, s, P);
        else JFNK_KLAUNCH((k_prim<2, 0>), g, bl, 0, stream, G, s, P);
    }
}

// compulsory bytes of the sweeps (each array read or written once)
static double prim_writes(const Grid& G) {
    return 8.0 * G.N * (3 + G.ndim + ((G.has_wall || G.has_chi) ? 1 : 0) + (G.has_chi ? 1 : 0) + (G.has_wall ? 1 : 0));
}

void launch_residual(const Grid& G, const StateView& s, const Prim& P, const Flux& Fx, const WallFlux& W,
                     const double* sbal, const OutSpec& o, hipStream_t stream, bool prim_valid) {
    const double vec = 8.0 * G.nvec;
    const double dirb = s.v ? vec : (s.vf ? 0.5 * vec : 0.0);  // the direction's bytes
    const double b_prim = vec + dirb + prim_writes(G);
    const double b_flux = prim_writes(G) + 8.0 * G.N * 2 * G.ndim;
    // fluxes, momentum fluxes, p, rho (with gravity), the face velocities
    // (internal-energy form), the heat-balance source, the state, the output
    bool gravity = false;
    for (int d = 0; d < G.ndim; ++d) gravity = gravity || G.g[d] != 0.0;
    double b_out = 8.0 * G.N *
                       (2 * G.ndim + G.ndim * G.ndim + 1 + (gravity ? 1 : 0) + (G.internal ? G.ndim : 0) +
                        (sbal ? 1 : 0)) +
                   vec;  // the output
    if (o.mode == OUT_CN_OLD) b_out += 2.0 * vec;  // u read, F written
    if (o.mode == OUT_RESIDUAL) b_out += 2.0 * vec;  // u and b read
    if (o.mode == OUT_JV) b_out += dirb + vec + (gravity ? 2.0 * 8.0 * G.N * G.ndim : 0.0);  // v, R(u) [, m]
    if (o.mode == OUT_JV && o.dotk > 0) b_out += o.dotk * (o.dotvf ? 0.5 : 1.0) * vec;      // the basis dotted
    if (o.rout) b_out += vec;
    if (!prim_valid) {
        JFNK_PROFB(KC_PRIM, stream, b_prim);
        launch_prim_kernel(G, s, P, stream);
    }
    {
        JFNK_PROFB(KC_FLUX, stream, b_flux);
        JFNK_LAUNCH_ND(G.ndim, k_flux, cell_grid3(G.n), dim3(kBx, kBy), 0, stream, G, P, Fx, W);
    }
    {
        JFNK_PROFB(KC_MFLUX, stream, 8.0 * G.N * (2 * G.ndim + G.ndim * G.ndim));
        const dim3 g = cell_grid3(G.n), bl(kBx, kBy);
        if (G.ndim == 3) {
            if (G.has_wall) JFNK_KLAUNCH((k_mflux<3, true>), g, bl, 0, stream, G, P, Fx);
            else JFNK_KLAUNCH(k_mflux_tile3, g, bl, 0, stream, G, P, Fx);
        } else {
            if (G.has_wall) JFNK_KLAUNCH((k_mflux<2, true>), g, bl, 0, stream, G, P, Fx);
            else JFNK_KLAUNCH((k_mflux<2, false>), g, bl, 0, stream, G, P, Fx);
        }
    }
    {
        JFNK_PROFB(KC_OUT, stream, b_out);
        if (G.ndim == 3) launch_out_nd<3>(G, s, P, Fx, W, sbal, o, stream);
        else launch_out_nd<2>(G, s, P, Fx, W, sbal, o, stream);
    }
}

void launch_prim_flux(const Grid& G, const StateView& s, const Prim& P, const Flux& Fx, const WallFlux& W,
                      hipStream_t stream) {
    launch_prim(G, s, P, stream);
    {
        JFNK_PROFB(KC_FLUX, stream, prim_writes(G) + 8.0 * G.N * 2 * G.ndim);
        JFNK_LAUNCH_ND(G.ndim, k_flux, cell_grid3(G.n), dim3(kBx, kBy), 0, stream, G, P, Fx, W);
    }
}

void launch_prim(const Grid& G, const StateView& s, const Prim& P, hipStream_t stream) {
    {
        JFNK_PROFB(KC_PRIM, stream, (s.v ? 2.0 : (s.vf ? 1.5 : 1.0)) * 8.0 * G.nvec + prim_writes(G));
        launch_prim_kernel(G, s, P, stream);
    }
}

void launch_dt_partial(const Grid& G, const Prim& P, const double* u, double* part, hipStream_t stream) {
    {
        JFNK_PROF(KC_OTHER, stream);
        JFNK_LAUNCH_ND(G.ndim, k_dt_partial, cell_grid3(G.n), dim3(kBx, kBy), 0, stream, G, P, u, part);
    }
}

}  // namespace jfnk
