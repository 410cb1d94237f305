// Physics-based preconditioner (section 2 of Goffrey et al. 2016): a
// semi-implicit approximate solve in which sound waves, and optionally
// thermal diffusion, are implicit while advection and gravity are left to
// the Krylov iteration.  Coefficients are frozen at the Newton iterate.
//   conduction (optional):  (1/W - tau D chi_f G) s = r_E,
//                           r_E <- r_E + tau D(chi_f G s)
//   acoustic:               (I - tau^2 D (gamma-1) h_f G) dp
//                               = (gamma-1)(r_E - tau D(h_f r_m))
//                           dm = r_m - tau G dp, drho = r_rho - tau D dm,
//                           dE = r_E - tau D(h_f dm)
// The elliptic solves use geometric multigrid V-cycles with red-black
// Gauss-Seidel smoothing (default) or alternating-direction line solves.
// Divergence-form back-substitution keeps the sums of rho, E and m.
#include "kernels.hpp"

namespace jfnk {

// ---------------------------------------------------------------- coefficients
// DIFF: the conduction block is on (its couplings beta and the cells' W are
// formed only then)
template <int ND, bool DIFF>
__global__ void __launch_bounds__(kBlock) k_pc_coef(Grid G, const double* __restrict__ u, Prim P, PcCoef C,
                                                    double tau) {
    Ijk q;
    long c;
    if (!cell_from_launch(G, q, c)) return;
    const double* E = u + G.N;
    for (int d = 0; d < ND; ++d) {
        // the lower neighbour is loaded on a wall too (wrapped, in bounds)
        // and the wall face's values replaced by 0
        const bool wall = G.bc[d] == WALL && q.v[d] == 0;
        const long xl = shifted(G, q, d, -1);
        const double hl = (E[xl] + P.p[xl]) / P.rho[xl];
        const double hr = (E[c] + P.p[c]) / P.rho[c];
        const double hf = wall ? 0.0 : 0.5 * (hl + hr);
        const double chif = (wall || !G.has_chi) ? 0.0 : 0.5 * (P.chi[xl] + P.chi[c]);
        // couplings per unit volume, or, on spherical grids, of the
        // volume-weighted system: face area over centre distance
        const double i2 = G.sph ? sph_area(G, d, q.v[0], q.v[1]) * face_ids(G, d, q.v[0]) : G.idx[d] * G.idx[d];
        C.kap[d][c] = ((tau * tau) * G.gm1) * hf * i2;
        if (DIFF) C.beta[d][c] = (tau * chif) * i2;
    }
    if (DIFF) C.W[c] = G.gm1 / P.rho[c];
    C.H[c] = (E[c] + P.p[c]) / P.rho[c];
    if (G.has_chi) C.chi[c] = P.chi[c];
}

void launch_pc_coef(const Grid& G, const double* u, const Prim& P, const PcCoef& C, double dt, bool diff,
                    hipStream_t stream) {
    {
        JFNK_PROF(KC_PC_BUILD, stream);
        const dim3 g = cell_grid3(G.n), bl(kBx, kBy);
        if (G.ndim == 3) {
            if (diff) JFNK_KLAUNCH((k_pc_coef<3, true>), g, bl, 0, stream, G, u, P, C, 0.5 * dt);
            else JFNK_KLAUNCH((k_pc_coef<3, false>), g, bl, 0, stream, G, u, P, C, 0.5 * dt);
        } else {
            if (diff) JFNK_KLAUNCH((k_pc_coef<2, true>), g, bl, 0, stream, G, u, P, C, 0.5 * dt);
            else JFNK_KLAUNCH((k_pc_coef<2, false>), g, bl, 0, stream, G, u, P, C, 0.5 * dt);
        }
    }
}

// ---------------------------------------------------------------- multigrid level helpers
struct LIjk {
    int v[3];
};
// a / b (and the remainder) for 0 <= a < 2^20 and b >= 1: a float estimate
// (off by at most one at these sizes) corrected once, in a few instructions
// instead of an integer division's few dozen
__device__ __forceinline__ int small_div(int a, int b, int& rem) {
    int q = (int)((float)a * __builtin_amdgcn_rcpf((float)b));
    int r = a - q * b;
    if (r < 0) {
        --q;
        r += b;
    } else if (r >= b) {
        ++q;
        r -= b;
    }
    rem = r;
    return q;
}
// coordinates of cell c of a level (the single-workgroup solve's levels, far
// below 2^20 cells)
template <typename R>
__device__ __forceinline__ LIjk lcoords(const LevelT<R>& L, int c) {
    LIjk r;
    const int t = small_div(c, L.n[0], r.v[0]);
    r.v[2] = small_div(t, L.n[1], r.v[1]);
    return r;
}
template <typename R>
__device__ __forceinline__ int lflat(const LevelT<R>& L, int i, int j, int k) {
    return i + L.n[0] * (j + L.n[1] * k);
}
// coordinates of the neighbour along d on a level: periodic wrap, false
// beyond a wall
template <typename R>
__device__ __forceinline__ bool lnbq(const Grid& G, const LevelT<R>& L, LIjk& q, int d, int s) {
    int a = q.v[d] + s;
    if (a < 0 || a >= L.n[d]) {
        if (G.bc[d] == WALL) return false;
        a = a < 0 ? a + L.n[d] : a - L.n[d];
    }
    q.v[d] = a;
    return true;
}
// neighbour along d on a level (coefficient index): -1 beyond a wall
template <typename R>
__device__ __forceinline__ int lnb(const Grid& G, const LevelT<R>& L, LIjk q, int d, int s) {
    if (!lnbq(G, L, q, d, s)) return -1;
    return lflat(L, q.v[0], q.v[1], q.v[2]);
}
// index of a cell in the level's x, b and x2 arrays
template <typename R>
__device__ __forceinline__ int xbq(const LevelT<R>& L, const LIjk& q) {
    return xbi(L, q.v[0], q.v[1], q.v[2]);
}
// cell of a 3D launch over a level
template <typename R>
__device__ __forceinline__ bool lcell(const LevelT<R>& L, LIjk& q, int& c) {
    const Tile tl = xcd_tile();
    q.v[0] = (int)(tl.x * kBx + threadIdx.x);
    q.v[1] = (int)(tl.y * kBy + threadIdx.y);
    q.v[2] = (int)tl.z;
    if (q.v[0] >= L.n[0] || q.v[1] >= L.n[1]) return false;
    c = lflat(L, q.v[0], q.v[1], q.v[2]);
    return true;
}
// cell of one colour (i + j + k parity) of a launch over half the x extent
template <typename R>
__device__ __forceinline__ bool lcell_color(const LevelT<R>& L, int color, LIjk& q, int& c) {
    const Tile tl = xcd_tile();
    const int t = (int)(tl.x * kBx + threadIdx.x);
    q.v[1] = (int)(tl.y * kBy + threadIdx.y);
    q.v[2] = (int)tl.z;
    q.v[0] = 2 * t + ((q.v[1] + q.v[2] + color) & 1);
    if (q.v[0] >= L.n[0] || q.v[1] >= L.n[1]) return false;
    c = lflat(L, q.v[0], q.v[1], q.v[2]);
    return true;
}
inline dim3 color_grid3(const int n[3]) {
    const int half = (n[0] + 1) / 2;
    return dim3((half + kBx - 1) / kBx, (n[1] + kBy - 1) / kBy, n[2]);
}

template <typename R, int ND>
__global__ void __launch_bounds__(kBlock) k_level0(Grid G, PcCoef C, int which, LevelT<R> L) {
    LIjk q;
    int c;
    if (!lcell(L, q, c)) return;
    if (G.sph) {  // volume-weighted system: sigma = V (acoustic) or V / W (conduction)
        const double V = sph_vol(G, q.v[0], q.v[1]);
        L.sig[c] = which == 0 ? (R)V : (R)(V / C.W[c]);
    } else {
        L.sig[c] = which == 0 ? (R)1.0 : (R)(1.0 / C.W[c]);
    }
    for (int d = 0; d < ND; ++d) L.a[d][c] = which == 0 ? (R)C.kap[d][c] : (R)C.beta[d][c];
}

template <typename R, int ND>
__global__ void __launch_bounds__(kBlock) k_level_diag(Grid G, LevelT<R> L) {
    LIjk q;
    int c;
    if (!lcell(L, q, c)) return;
    R den = L.sig[c];
    for (int d = 0; d < ND; ++d) {
        const int up = lnb(G, L, q, d, 1);
        const R alo = L.a[d][c], ahi = up >= 0 ? L.a[d][up] : (R)0.0;
        den = den + alo;
        den = den + ahi;
    }
    L.D[c] = den;
}

// coarse coefficients by re-discretisation: sig averaged over the children,
// face couplings averaged over the fine faces of a coarse face and divided by
// 4 (couplings scale as 1/dx^2)
template <typename R, int ND>
__global__ void __launch_bounds__(kBlock) k_coarsen(Grid G, LevelT<R> F, LevelT<R> Cl) {
    LIjk q;
    int c;
    if (!lcell(Cl, q, c)) return;
    const int nch = 1 << ND;
    const R inv_ch = (R)(1.0 / nch), inv_face = (R)(1.0 / ((nch / 2) * 4));
    const int kk = ND > 2 ? 2 : 1;
    R s = 0.0;
    for (int dk = 0; dk < kk; ++dk)
        for (int dj = 0; dj < 2; ++dj)
            for (int di = 0; di < 2; ++di)
                s = s + F.sig[lflat(F, 2 * q.v[0] + di, 2 * q.v[1] + dj, ND > 2 ? 2 * q.v[2] + dk : q.v[2])];
    Cl.sig[c] = s * inv_ch;
    for (int d = 0; d < ND; ++d) {
        R t = 0.0;
        for (int dk = 0; dk < kk; ++dk)
            for (int dj = 0; dj < 2; ++dj)
                for (int di = 0; di < 2; ++di) {
                    const int off[3] = {di, dj, dk};
                    if (off[d] != 0) continue;
                    t = t + F.a[d][lflat(F, 2 * q.v[0] + di, 2 * q.v[1] + dj, ND > 2 ? 2 * q.v[2] + dk : q.v[2])];
                }
        Cl.a[d][c] = t * inv_face;
    }
}

template <typename R>
void launch_level0(const Grid& G, const PcCoef& C, int which, const LevelT<R>& L0, hipStream_t stream) {
    JFNK_PROF(KC_PC_BUILD, stream);
    JFNK_LAUNCH_RND(G.ndim, k_level0, R, cell_grid3(L0.n), dim3(kBx, kBy), 0, stream, G, C, which, L0);
}
template <typename R>
void launch_coarsen(const Grid& G, const LevelT<R>& F, const LevelT<R>& C, hipStream_t stream) {
    JFNK_PROF(KC_PC_BUILD, stream);
    JFNK_LAUNCH_RND(G.ndim, k_coarsen, R, cell_grid3(C.n), dim3(kBx, kBy), 0, stream, G, F, C);
}
template <typename R>
void launch_level_diag(const Grid& G, const LevelT<R>& L, hipStream_t stream) {
    JFNK_PROF(KC_PC_BUILD, stream);
    JFNK_LAUNCH_RND(G.ndim, k_level_diag, R, cell_grid3(L.n), dim3(kBx, kBy), 0, stream, G, L);
}

// ---------------------------------------------------------------- multigrid cell operations
// x and b are read and written through pointers so that the single-workgroup
// coarse solver can keep them in LDS.  c is the cell's index in the
// coefficient arrays (natural order); x and b are indexed by xbq.

// Gauss-Seidel value of one cell from its neighbours in x (first: neighbours
// taken as 0)
// FIRST, QF (couplings from the level's cell field) and UNIT (sigma == 1)
// are compile-time so that a sweep's loads form one straight-line block
// XNB(n, d, side): the value of x at neighbour n, the lower (side 0) or
// upper (side 1) one along d
template <typename R, int ND, bool FIRST, bool QF, bool UNIT, class XNB>
__device__ __forceinline__ R gs_value_bv(const Grid& G, const LevelT<R>& L, R bq, XNB xnb, LIjk q, int c) {
    R num = bq;
    R den = (R)1.0;  // sig + the couplings in the order of k_level_diag (when sig == 1)
    for (int d = 0; d < ND; ++d) {
        // a neighbour beyond a wall stays at q: its loads are issued (in
        // bounds) like every other and their values discarded
        LIjk qu = q, qd = q;
        const bool hu = lnbq(G, L, qu, d, 1), hd = lnbq(G, L, qd, d, -1);
        const int lo = lflat(L, qd.v[0], qd.v[1], qd.v[2]), up = lflat(L, qu.v[0], qu.v[1], qu.v[2]);
        R alo, ahi;
        if (QF) {
            alo = qf_coupling(L, d, lo, c);
            ahi = qf_coupling(L, d, c, up);
        } else {
            alo = L.a[d][c];
            ahi = L.a[d][up];
        }
        alo = hd ? alo : (R)0.0;
        ahi = hu ? ahi : (R)0.0;
        const R xlo = FIRST ? (R)0.0 : xnb(qd, d, 0), xhi = FIRST ? (R)0.0 : xnb(qu, d, 1);
        num = hd ? num + alo * xlo : num;
        num = hu ? num + ahi * xhi : num;
        den = den + alo;
        den = den + ahi;
    }
    return num / (UNIT ? den : L.D[c]);
}
template <typename R, int ND, bool FIRST, bool QF, bool UNIT, class XNB>
__device__ __forceinline__ R gs_value_nb(const Grid& G, const LevelT<R>& L, const R* b, XNB xnb, LIjk q, int c) {
    return gs_value_bv<R, ND, FIRST, QF, UNIT>(G, L, b[xbq(L, q)], xnb, q, c);
}
template <typename R, int ND, bool FIRST, bool QF, bool UNIT>
__device__ __forceinline__ R gs_value_t(const Grid& G, const LevelT<R>& L, const R* b, const R* x, LIjk q, int c) {
    return gs_value_nb<R, ND, FIRST, QF, UNIT>(G, L, b, [&](const LIjk& n, int, int) { return x[xbq(L, n)]; }, q,
                                               c);
}
template <typename R, int ND, bool FIRST>
__device__ __forceinline__ R gs_value_f(const Grid& G, const LevelT<R>& L, const R* b, const R* x, LIjk q, int c) {
    if (L.qf) {
        if (L.unit_sig) return gs_value_t<R, ND, FIRST, true, true>(G, L, b, x, q, c);
        return gs_value_t<R, ND, FIRST, true, false>(G, L, b, x, q, c);
    }
    if (L.unit_sig) return gs_value_t<R, ND, FIRST, false, true>(G, L, b, x, q, c);
    return gs_value_t<R, ND, FIRST, false, false>(G, L, b, x, q, c);
}
template <typename R, int ND>
__device__ __forceinline__ R gs_value(const Grid& G, const LevelT<R>& L, const R* b, const R* x, LIjk q, int c,
                                      bool first) {
    return first ? gs_value_f<R, ND, true>(G, L, b, x, q, c) : gs_value_f<R, ND, false>(G, L, b, x, q, c);
}
// a periodic axis of odd length (possible on the coarsest level only): the
// two cells facing each other across the wrap share a colour, so a colour's
// cells are updated together from the values before their half-sweep
template <typename R, int ND>
__device__ __forceinline__ bool odd_periodic(const Grid& G, const LevelT<R>& L) {
    bool odd = false;
#pragma unroll
    for (int d = 0; d < ND; ++d) odd = odd || (G.bc[d] == PERIODIC && (L.n[d] & 1));
    return odd;
}

// residual of one fine cell, from the stored couplings (forming them from the
// cell field, as the sweeps do on the finest level, measured slower here)
template <typename R, int ND, bool UNIT>
__device__ __forceinline__ R resid_cell_t(const Grid& G, const LevelT<R>& L, const R* b, const R* x, LIjk q,
                                          int c) {
    const R xc = x[xbq(L, q)];
    R acc = UNIT ? xc : L.sig[c] * xc;
    for (int d = 0; d < ND; ++d) {
        LIjk qu = q, qd = q;  // beyond a wall a neighbour stays at q (loads issued, values discarded)
        const bool hu = lnbq(G, L, qu, d, 1), hd = lnbq(G, L, qd, d, -1);
        const int up = lflat(L, qu.v[0], qu.v[1], qu.v[2]);
        const R alo = L.a[d][c], ahi = L.a[d][up];
        const R xlo = x[xbq(L, qd)], xhi = x[xbq(L, qu)];
        acc = hd ? acc + alo * (xc - xlo) : acc;
        acc = hu ? acc + ahi * (xc - xhi) : acc;
    }
    return b[xbq(L, q)] - acc;
}

// cell-centred (bi/tri)linear prolongation of the coarse correction, weights
// 3/4 and 1/4 per axis; beyond a wall the parent value is reused.  The two
// parent indices of each axis are found once, with selects, and the corners
// are summed in the order m = 0..2^ND-1 (bit d of m: the neighbour along d).
template <typename R, int ND>
__device__ __forceinline__ R prolong_cell(const Grid& G, const LevelT<R>& Cl, const R* cx, LIjk f) {
    int p0[3], p1[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int P = d < ND ? f.v[d] / 2 : f.v[d];
        p0[d] = P;
        p1[d] = P;
        if (d < ND) {
            const int n = Cl.n[d];
            const int a = P + ((f.v[d] % 2 == 0) ? -1 : 1);
            const int w = a < 0 ? a + n : (a >= n ? a - n : a);
            p1[d] = (a < 0 || a >= n) ? (G.bc[d] == WALL ? P : w) : a;
        }
    }
    R e = 0.0;
#pragma unroll
    for (int m = 0; m < (1 << ND); ++m) {
        R w = 1.0;
        int qq[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const bool nb = d < ND && (m & (1 << d));
            if (d < ND) w = w * (nb ? (R)0.25 : (R)0.75);
            qq[d] = nb ? p1[d] : p0[d];
        }
        e = e + w * cx[xbi(Cl, qq[0], qq[1], qq[2])];
    }
    return e;
}

// ---------------------------------------------------------------- multigrid kernels (multi-block levels)
template <typename R, int ND, bool FIRST, bool QF, bool UNIT>
__global__ void __launch_bounds__(kBlock) k_gs(Grid G, LevelT<R> L, int color) {
    LIjk q;
    int c;
    if (!lcell_color(L, color, q, c)) return;
    L.x[xbq(L, q)] = gs_value_t<R, ND, FIRST, QF, UNIT>(G, L, L.b, L.x, q, c);
}
// one half-sweep of a multi-block level
template <typename R, int ND, bool FIRST, bool QF>
void launch_gs_u(const Grid& G, const LevelT<R>& L, int color, hipStream_t stream) {
    const dim3 g = color_grid3(L.n), bl(kBx, kBy);
    if (L.unit_sig) JFNK_KLAUNCH((k_gs<R, ND, FIRST, QF, true>), g, bl, 0, stream, G, L, color);
    else JFNK_KLAUNCH((k_gs<R, ND, FIRST, QF, false>), g, bl, 0, stream, G, L, color);
}
template <typename R, int ND>
void launch_gs_nd(const Grid& G, const LevelT<R>& L, int color, bool first, hipStream_t stream) {
    if (L.qf) {
        if (first) launch_gs_u<R, ND, true, true>(G, L, color, stream);
        else launch_gs_u<R, ND, false, true>(G, L, color, stream);
    } else {
        if (first) launch_gs_u<R, ND, true, false>(G, L, color, stream);
        else launch_gs_u<R, ND, false, false>(G, L, color, stream);
    }
}
template <typename R>
void launch_gs(const Grid& G, const LevelT<R>& L, int color, bool first, hipStream_t stream) {
    if (G.ndim == 3) launch_gs_nd<R, 3>(G, L, color, first, stream);
    else launch_gs_nd<R, 2>(G, L, color, first, stream);
}
// half-sweep of one colour from xin into xout (the other colour copied, or
// zeroed on a first sweep): the update for levels with an odd periodic axis
template <typename R, int ND>
__global__ void __launch_bounds__(kBlock) k_gs_pp(Grid G, LevelT<R> L, int color, int first,
                                                  const R* __restrict__ xin, R* __restrict__ xout) {
    LIjk q;
    int c;
    if (!lcell(L, q, c)) return;
    const int e = xbq(L, q);
    if (((q.v[0] + q.v[1] + q.v[2]) & 1) != color) {
        xout[e] = first ? (R)0.0 : xin[e];
        return;
    }
    xout[e] = gs_value<R, ND>(G, L, L.b, xin, q, c, first != 0);
}
// Restriction of a multi-block level: the coarse right-hand side is the mean
// of the children's residuals.  One thread per fine cell computes its
// residual, and the 2^ND children of each coarse cell (all in one workgroup)
// are summed in LDS in a fixed order (k, then j, then i of the child, each
// from the lower one), then times 1/2^ND.  Workgroups are
// kRx x kRy x kRz fine cells (kRz = 2 in 3D, 1 in 2D).
constexpr int kRx = 32, kRy = 4;
template <int ND>
inline dim3 restrict_block() { return ND > 2 ? dim3(kRx, kRy, 2) : dim3(2 * kRx, kRy, 1); }
template <int ND>
inline dim3 restrict_grid(const int n[3]) {
    const dim3 b = restrict_block<ND>();
    return dim3((n[0] + b.x - 1) / b.x, (n[1] + b.y - 1) / b.y, ND > 2 ? (n[2] + 1) / 2 : n[2]);
}
template <typename R, int ND, bool UNIT>
__global__ void __launch_bounds__(kBlock) k_restrict(Grid G, LevelT<R> F, LevelT<R> Cl) {
    constexpr int BX = ND > 2 ? kRx : 2 * kRx, BZ = ND > 2 ? 2 : 1;
    __shared__ R rs[BZ][kRy][BX];
    const Tile t = xcd_tile();
    LIjk f;
    f.v[0] = (int)(t.x * BX + threadIdx.x);
    f.v[1] = (int)(t.y * kRy + threadIdx.y);
    f.v[2] = (int)(t.z * BZ + threadIdx.z);
    R r = (R)0.0;
    if (f.v[0] < F.n[0] && f.v[1] < F.n[1] && f.v[2] < F.n[2])
        r = resid_cell_t<R, ND, UNIT>(G, F, F.b, F.x, f, lflat(F, f.v[0], f.v[1], f.v[2]));
    rs[threadIdx.z][threadIdx.y][threadIdx.x] = r;
    __syncthreads();
    // coarse cells of the tile: (BX/2) x (kRy/2) x 1
    const int lt = (int)(threadIdx.x + BX * (threadIdx.y + kRy * threadIdx.z));
    constexpr int CX = BX / 2, CY = kRy / 2;
    if (lt >= CX * CY) return;
    const int ci = lt % CX, cj = lt / CX;
    LIjk q;
    q.v[0] = (int)(t.x * CX) + ci;
    q.v[1] = (int)(t.y * CY) + cj;
    q.v[2] = (int)t.z;
    if (q.v[0] >= Cl.n[0] || q.v[1] >= Cl.n[1] || q.v[2] >= Cl.n[2]) return;
    const R inv_ch = (R)(1.0 / (1 << ND));
    R s = 0.0;
    for (int dk = 0; dk < BZ; ++dk)
        for (int dj = 0; dj < 2; ++dj)
            for (int di = 0; di < 2; ++di) s = s + rs[dk][2 * cj + dj][2 * ci + di];
    Cl.b[xbq(Cl, q)] = s * inv_ch;
}
// Prolongation of the coarse correction onto the cells of one colour (color
// 0 or 1), or onto every cell (color < 0).  When post-smoothing follows, only
// colour 1 needs it: the colour-0 half-sweep that comes next overwrites every
// colour-0 value without reading it, so the result is the same as correcting
// every cell.
template <typename R, int ND>
__global__ void __launch_bounds__(kBlock) k_prolong(Grid G, LevelT<R> F, LevelT<R> Cl, int color) {
    LIjk q;
    int c;
    if (color < 0 ? !lcell(F, q, c) : !lcell_color(F, color, q, c)) return;
    const int e = xbq(F, q);
    F.x[e] = F.x[e] + prolong_cell<R, ND>(G, Cl, Cl.x, q);
}
// The same correction of the colour-1 cells, one thread per coarse cell
// for its 2^(ND-1) colour-1 children (the children of a coarse cell at
// offsets o with an odd offset sum): the parent rows one below and one above
// along each axis are found once for all of them, each child then sums its
// corners as prolong_cell does, in its corner order (bit d of the corner
// picks the row on the child's side of the parent along d).
template <typename R, int ND>
__global__ void __launch_bounds__(kBlock) k_prolong_c1(Grid G, LevelT<R> F, LevelT<R> Cl) {
    LIjk Q;
    int cc;
    if (!lcell(Cl, Q, cc)) return;
    int P[3], side[3][2];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        P[d] = Q.v[d];
        side[d][0] = side[d][1] = P[d];
        if (d < ND) {
            const int n = Cl.n[d];
            const bool wall = G.bc[d] == WALL;
            const int lo = P[d] - 1, hi = P[d] + 1;
            side[d][0] = lo < 0 ? (wall ? P[d] : lo + n) : lo;   // even child coordinate
            side[d][1] = hi >= n ? (wall ? P[d] : hi - n) : hi;  // odd child coordinate
        }
    }
#pragma unroll
    for (int o = 0; o < (1 << ND); ++o) {
        int par = 0;
#pragma unroll
        for (int d = 0; d < ND; ++d) par += (o >> d) & 1;
        if ((par & 1) == 0) continue;
        R e = 0.0;
#pragma unroll
        for (int m = 0; m < (1 << ND); ++m) {
            R w = 1.0;
            int qq[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const bool nb = d < ND && (m & (1 << d));
                if (d < ND) w = w * (nb ? (R)0.25 : (R)0.75);
                qq[d] = nb ? side[d][(o >> d) & 1] : P[d];
            }
            e = e + w * Cl.x[xbi(Cl, qq[0], qq[1], qq[2])];
        }
        const int f0 = 2 * P[0] + (o & 1), f1 = 2 * P[1] + ((o >> 1) & 1),
                  f2 = ND > 2 ? 2 * P[2] + ((o >> 2) & 1) : P[2];
        const int fe = xbi(F, f0, f1, f2);
        F.x[fe] = F.x[fe] + e;
    }
}

constexpr long kGsProlongMaxCells = 1L << 18;
// Prolongation and the first post-smoothing half-sweep (colour 0) in one
// launch: each colour-0 cell takes its neighbours' corrected values
// x + prolong_cell (the sums k_prolong would store) as it goes.  The
// half-sweep overwrites colour 0 without reading it, and nothing else reads
// the corrected colour-1 values (the colour-1 half-sweep that follows
// overwrites them without reading them), so no corrected value is stored and
// the result is that of correcting every cell and sweeping.
//
// The six neighbours' prolongations share their coarse values.  Along each
// axis the parents of the cell and of its two neighbours lie among three
// coarse rows, h - 1, h and h + 1 (h = the cell's coordinate / 2; wrapped on
// a periodic axis, and on a wall the parent h where prolong_cell reuses the
// parent): the cell's own pair is (h, o) with o = h - 1 for an even
// coordinate and h + 1 for an odd one, and t is the third row.  Of the two
// neighbours along an axis one has the pair (o, h) and the other (h, t).  So
// the values of the cell's own 2^ND parents (cube) and, per axis, of the
// 2^(ND-1) cells one row further (row t, the other axes as in the cube) are
// loaded once, and each neighbour's correction is summed from them with
// prolong_cell's weights in its corner order.
template <typename R, int ND, bool QF, bool UNIT>
__global__ void __launch_bounds__(kBlock) k_gs_prolong(Grid G, LevelT<R> F, LevelT<R> Cl) {
    LIjk q;
    int c;
    if (!lcell_color(F, 0, q, c)) return;
    int P[3], o[3], t[3];
    bool even[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        even[d] = true;
        P[d] = o[d] = t[d] = q.v[d];
        if (d < ND) {
            const int h = q.v[d] >> 1, n = Cl.n[d];
            const bool wall = G.bc[d] == WALL;
            int lo = h - 1, hi = h + 1;
            lo = lo < 0 ? (wall ? h : lo + n) : lo;
            hi = hi >= n ? (wall ? h : hi - n) : hi;
            even[d] = (q.v[d] & 1) == 0;
            P[d] = h;
            o[d] = even[d] ? lo : hi;
            t[d] = even[d] ? hi : lo;
        }
    }
    constexpr int NC = 1 << ND, NE = 1 << (ND - 1);
    R cube[NC], ext[ND][NE], w[NC];
#pragma unroll
    for (int m = 0; m < NC; ++m) {
        int qq[3];
        R wm = 1.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const bool nb = d < ND && (m & (1 << d));
            if (d < ND) wm = wm * (nb ? (R)0.25 : (R)0.75);
            qq[d] = nb ? o[d] : P[d];
        }
        w[m] = wm;
        cube[m] = Cl.x[xbi(Cl, qq[0], qq[1], qq[2])];
    }
#pragma unroll
    for (int d = 0; d < ND; ++d)
#pragma unroll
        for (int k = 0; k < NE; ++k) {
            int qq[3] = {P[0], P[1], P[2]};
            int j = 0;
#pragma unroll
            for (int e = 0; e < ND; ++e) {
                if (e == d) continue;
                qq[e] = (k & (1 << j)) ? o[e] : P[e];
                ++j;
            }
            qq[d] = t[d];
            ext[d][k] = Cl.x[xbi(Cl, qq[0], qq[1], qq[2])];
        }
    // corrections of the neighbours along d: pair (o, h) reads the cube with
    // bit d flipped, pair (h, t) reads row t where bit d is set
    const auto xnb = [&](const LIjk& n, int d, int side) {
        R ea = 0.0, eb = 0.0;
#pragma unroll
        for (int m = 0; m < NC; ++m) {
            const int sq = ((m >> (d + 1)) << d) | (m & ((1 << d) - 1));
            ea = ea + w[m] * cube[m ^ (1 << d)];
            eb = eb + w[m] * ((m & (1 << d)) ? ext[d][sq] : cube[m]);
        }
        const bool pair_oh = even[d] == (side == 0);
        return F.x[xbq(F, n)] + (pair_oh ? ea : eb);
    };
    F.x[xbq(F, q)] = gs_value_nb<R, ND, false, QF, UNIT>(G, F, F.b, xnb, q, c);
}
template <typename R, int ND, bool QF>
void launch_gs_prolong_u(const Grid& G, const LevelT<R>& F, const LevelT<R>& Cl, hipStream_t stream) {
    const dim3 g = color_grid3(F.n), bl(kBx, kBy);
    if (F.unit_sig) JFNK_KLAUNCH((k_gs_prolong<R, ND, QF, true>), g, bl, 0, stream, G, F, Cl);
    else JFNK_KLAUNCH((k_gs_prolong<R, ND, QF, false>), g, bl, 0, stream, G, F, Cl);
}
template <typename R>
void launch_gs_prolong(const Grid& G, const LevelT<R>& F, const LevelT<R>& Cl, hipStream_t stream) {
    if (G.ndim == 3) {
        if (F.qf) launch_gs_prolong_u<R, 3, true>(G, F, Cl, stream);
        else launch_gs_prolong_u<R, 3, false>(G, F, Cl, stream);
    } else {
        if (F.qf) launch_gs_prolong_u<R, 2, true>(G, F, Cl, stream);
        else launch_gs_prolong_u<R, 2, false>(G, F, Cl, stream);
    }
}

// The rest of the V-cycle, levels from..nlev-1, in one workgroup.  Every
// level of at most kCoarseMaxLevelCells cells (at most kCoarseLdsCells cells
// over those levels) keeps its arrays in LDS.  The first level may instead be
// a larger one of at most kCoarseBigCells cells (never the coarsest): its x
// and residuals live in LDS, and each thread holds its cells' couplings,
// right-hand side and divisor in registers.  Level descriptors come from
// device memory (Ld) so that the level loop may index them at run time.
constexpr int kCoarseThreads = 1024;
constexpr int kCoarseBigPer = kCoarseBigCells / kCoarseThreads;  // cells per thread on the larger first level

// A cell of a level in the single-workgroup solve: its colour, neighbour
// indices (-1 beyond a wall), couplings, right-hand side and divisor, found
// once per call.  The update is gs_value's, operation for operation.
template <typename R, int ND>
struct CoarseCell {
    int up[ND], dn[ND], colour;
    R alo[ND], ahi[ND], bc, dv;
};
template <typename R, int ND, bool UNIT>
__device__ __forceinline__ CoarseCell<R, ND> coarse_cell(const Grid& G, const LevelT<R>& L, const R* b, int c,
                                                        const LIjk& q) {
    CoarseCell<R, ND> k;
    k.colour = (q.v[0] + q.v[1] + q.v[2]) & 1;
    R den = (R)1.0;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        k.up[d] = lnb(G, L, q, d, 1);
        k.dn[d] = lnb(G, L, q, d, -1);
        k.alo[d] = L.a[d][c];
        k.ahi[d] = k.up[d] >= 0 ? L.a[d][k.up[d]] : (R)0.0;
        den = den + k.alo[d];
        den = den + k.ahi[d];
    }
    k.bc = b[c];
    k.dv = UNIT ? den : L.D[c];
    return k;
}
template <typename R, int ND, bool UNIT>
__device__ __forceinline__ CoarseCell<R, ND> coarse_cell(const Grid& G, const LevelT<R>& L, const R* b, int c) {
    return coarse_cell<R, ND, UNIT>(G, L, b, c, lcoords(L, c));
}
// Gauss-Seidel value of the cell from x (f: first sweep, x taken as 0)
template <typename R, int ND>
__device__ __forceinline__ R coarse_update(const CoarseCell<R, ND>& k, const R* x, bool f) {
    R num = k.bc;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        if (k.dn[d] >= 0) num = num + k.alo[d] * (f ? (R)0.0 : x[k.dn[d]]);
        if (k.up[d] >= 0) num = num + k.ahi[d] * (f ? (R)0.0 : x[k.up[d]]);
    }
    return num / k.dv;
}
// Sweeps of a level held in LDS: every cell has its own thread (levels of at
// most kCoarseMaxLevelCells <= kCoarseThreads cells)
template <typename R, int ND, bool UNIT>
__device__ __forceinline__ void lds_smooth(const Grid& G, const LevelT<R>& L, int sweeps, bool first) {
    const bool together = odd_periodic<R, ND>(G, L);
    const int c = (int)threadIdx.x;
    const bool mine = c < L.N;
    CoarseCell<R, ND> k;
    k.colour = -1;
    if (mine) k = coarse_cell<R, ND, UNIT>(G, L, L.b, c);
    for (int s = 0; s < sweeps; ++s)
        for (int color = 0; color < 2; ++color) {
            const bool f = first && s == 0 && color == 0;
            R val = (R)0.0;
            if (k.colour == color) val = coarse_update<R, ND>(k, L.x, f);
            if (!together) {
                if (k.colour == color) L.x[c] = val;
            } else {
                __syncthreads();
                if (k.colour == color) L.x[c] = val;
                else if (f && mine) L.x[c] = (R)0.0;
            }
            __syncthreads();
        }
}
// A cell of the larger first level, in registers: couplings, right-hand
// side and (without unit sigma) divisor, its index (-1: no cell) and its
// coordinates packed as i | j << 10 | k << 20 (every axis of that level is
// shorter than 1024).  To keep the registers few, the neighbours are found
// again from the coordinates at each use, the unit-sigma divisor is summed
// again from the couplings in coarse_cell's order, and sigma is read again
// where the residual needs it.  Thread t holds, for each colour, that
// colour's cells t, t + 1024, ... in row order, so that every lane has work
// in every half-sweep.
template <typename R, int ND>
struct BigCell {
    R alo[ND], ahi[ND], bc, dv;
    int c, pq;
};
__device__ __forceinline__ LIjk unpack_ijk(int pq) {
    LIjk q;
    q.v[0] = pq & 1023;
    q.v[1] = (pq >> 10) & 1023;
    q.v[2] = pq >> 20;
    return q;
}
// the e-th cell of colour col on a level with even axes: its coordinates
__device__ __forceinline__ LIjk colour_cell(const int n[3], int col, int e) {
    int h;
    const int row = small_div(e, n[0] / 2, h);
    LIjk q;
    q.v[2] = small_div(row, n[1], q.v[1]);
    q.v[0] = 2 * h + ((q.v[1] + q.v[2] + col) & 1);
    return q;
}
template <typename R, int ND, bool UNIT>
__device__ __forceinline__ BigCell<R, ND> big_cell(const Grid& G, const LevelT<R>& L, const LIjk& q) {
    const int c = lflat(L, q.v[0], q.v[1], q.v[2]);
    const CoarseCell<R, ND> k = coarse_cell<R, ND, UNIT>(G, L, L.b, c, q);
    BigCell<R, ND> b;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        b.alo[d] = k.alo[d];
        b.ahi[d] = k.ahi[d];
    }
    b.bc = k.bc;
    b.dv = k.dv;
    b.c = c;
    b.pq = q.v[0] | (q.v[1] << 10) | (q.v[2] << 20);
    return b;
}
// index of the neighbour along d (s = -1 or 1) of the cell, -1 beyond a wall:
// lnb's result, from the cell's index and coordinates
template <typename R>
__device__ __forceinline__ int big_nb(const Grid& G, const LevelT<R>& L, int c, int pq, int d, int s) {
    const int a = (pq >> (10 * d)) & 1023, n = L.n[d];
    const int stride = d == 0 ? 1 : (d == 1 ? L.n[0] : L.n[0] * L.n[1]);
    const bool edge = s < 0 ? a == 0 : a == n - 1;
    if (!edge) return c + s * stride;
    if (G.bc[d] == WALL) return -1;
    return c - s * (n - 1) * stride;
}
// coarse_update and the residual of resid_cell_t, operation for operation
template <typename R, int ND, bool UNIT>
__device__ __forceinline__ R big_update(const Grid& G, const LevelT<R>& L, const BigCell<R, ND>& k, const R* x,
                                        bool f) {
    R den = (R)1.0;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        den = den + k.alo[d];
        den = den + k.ahi[d];
    }
    R num = k.bc;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        const int dn = big_nb(G, L, k.c, k.pq, d, -1), up = big_nb(G, L, k.c, k.pq, d, 1);
        if (dn >= 0) num = num + k.alo[d] * (f ? (R)0.0 : x[dn]);
        if (up >= 0) num = num + k.ahi[d] * (f ? (R)0.0 : x[up]);
    }
    return num / (UNIT ? den : k.dv);
}
template <typename R, int ND, bool UNIT>
__device__ __forceinline__ R big_resid(const Grid& G, const LevelT<R>& L, const BigCell<R, ND>& k, const R* x) {
    const R xc = x[k.c];
    R acc = UNIT ? xc : L.sig[k.c] * xc;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        const int dn = big_nb(G, L, k.c, k.pq, d, -1), up = big_nb(G, L, k.c, k.pq, d, 1);
        acc = dn >= 0 ? acc + k.alo[d] * (xc - x[dn]) : acc;
        acc = up >= 0 ? acc + k.ahi[d] * (xc - x[up]) : acc;
    }
    return k.bc - acc;
}
// Sweeps of the larger first level (no odd periodic axis: the level is not
// the coarsest); k[col][m] is the thread's m-th cell of colour col
template <typename R, int ND, bool UNIT>
__device__ __forceinline__ void big_smooth(const Grid& G, const LevelT<R>& L, R* x,
                                           const BigCell<R, ND> (*k)[kCoarseBigPer / 2], int sweeps, bool first) {
    for (int s = 0; s < sweeps; ++s)
#pragma unroll
        for (int color = 0; color < 2; ++color) {
            const bool f = first && s == 0 && color == 0;
            R val[kCoarseBigPer / 2];
#pragma unroll
            for (int m = 0; m < kCoarseBigPer / 2; ++m)
                val[m] = k[color][m].c >= 0 ? big_update<R, ND, UNIT>(G, L, k[color][m], x, f) : (R)0.0;
#pragma unroll
            for (int m = 0; m < kCoarseBigPer / 2; ++m)
                if (k[color][m].c >= 0) x[k[color][m].c] = val[m];
            __syncthreads();
        }
}
// LDS view of level l: its arrays at sm + base (sig, a[0..ND-1], D, x, b),
// built in registers so that every access is a direct LDS access, from the
// dimensions kept in LDS (ldim: n[0..2], N of each level) read as
// wavefront-uniform values, so that after the kernel's first load no level
// loop waits on a descriptor in device memory.  Only the fields the
// single-workgroup solve uses are set (its levels are in natural order).
template <typename R, int ND>
__device__ __forceinline__ LevelT<R> lds_view(const int (*ldim)[4], int l, R* sm, int base) {
    LevelT<R> L{};
    for (int a = 0; a < 3; ++a) L.n[a] = __builtin_amdgcn_readfirstlane(ldim[l][a]);
    const int n = __builtin_amdgcn_readfirstlane(ldim[l][3]);
    L.N = n;
    base = __builtin_amdgcn_readfirstlane(base);
    L.sig = sm + base;
    for (int d = 0; d < 3; ++d) L.a[d] = d < ND ? sm + base + (1 + d) * n : nullptr;
    L.D = sm + base + (1 + ND) * n;
    L.x = sm + base + (2 + ND) * n;
    L.b = sm + base + (3 + ND) * n;
    return L;
}
// residuals of level L's cells t, t + step, ... into rb
template <typename R, int ND, bool UNIT>
__device__ __forceinline__ void lds_resid(const Grid& G, const LevelT<R>& L, R* rb, int t, int step) {
    for (int c = t; c < L.N; c += step) rb[c] = resid_cell_t<R, ND, UNIT>(G, L, L.b, L.x, lcoords(L, c), c);
}
// coarse right-hand sides from the fine residuals rb (natural order of the
// fine level F): the children's sums in the order of the multi-block
// restriction
template <typename R, int ND>
__device__ __forceinline__ void lds_restrict_sum(const LevelT<R>& F, const LevelT<R>& C, const R* rb) {
    for (int c = (int)threadIdx.x; c < C.N; c += kCoarseThreads) {
        const LIjk q = lcoords(C, c);
        const int kk = ND > 2 ? 2 : 1;
        R sum = 0.0;
        for (int dk = 0; dk < kk; ++dk)
            for (int dj = 0; dj < 2; ++dj)
                for (int di = 0; di < 2; ++di)
                    sum = sum + rb[lflat(F, 2 * q.v[0] + di, 2 * q.v[1] + dj, ND > 2 ? 2 * q.v[2] + dk : q.v[2])];
        C.b[c] = sum * (R)(1.0 / (1 << ND));
    }
}
template <typename R, int ND, bool UNIT>
__global__ void __launch_bounds__(kCoarseThreads) k_coarse_vcycle(Grid G, const LevelT<R>* __restrict__ Ld,
                                                                   int from, int nlev, int nu1, int nu2, int nuc,
                                                                   int first_top, int light) {
    __shared__ R sm[(4 + ND) * kCoarseLdsCells];
    __shared__ R bigx[kCoarseBigCells];  // x of the larger first level
    __shared__ R rbuf[kCoarseBigCells];  // residuals of the level being restricted
    __shared__ int base[kMaxLevels];
    // the load into LDS: the arrays each LDS level needs (sigma and D only
    // without unit sigma, x and b of the first level only), every element of
    // them one entry of a single index space, so that a thread's loads do
    // not wait for one another level by level
    __shared__ int lN[kMaxLevels], nload[kMaxLevels], first_el[kMaxLevels + 1];
    __shared__ const R* lsrc[kMaxLevels][4 + ND];
    __shared__ int lslot[kMaxLevels][4 + ND];
    __shared__ int ldim[kMaxLevels][4];
    const int tid = (int)threadIdx.x;
    const bool top_first = first_top != 0;
    const LevelT<R> gB = Ld[from];
    const bool big = gB.N > kCoarseMaxLevelCells;
    const int lf = big ? from + 1 : from;  // first level held in LDS
    if (tid < nlev - lf) {
        const int l = lf + tid;
        const LevelT<R> gL = Ld[l];
        int k = 0;
        auto add = [&](const R* p, int slot) {
            lsrc[l][k] = p;
            lslot[l][k] = slot;
            ++k;
        };
        if (!UNIT) add(gL.sig, 0);
        for (int d = 0; d < ND; ++d) add(gL.a[d], 1 + d);
        if (!UNIT) add(gL.D, 1 + ND);  // built only without unit sigma
        if (l == from) {
            if (!top_first) add(gL.x, 2 + ND);
            add(gL.b, 3 + ND);
        }
        nload[l] = k;
        lN[l] = (int)gL.N;
        for (int a = 0; a < 3; ++a) ldim[l][a] = gL.n[a];
        ldim[l][3] = (int)gL.N;
    }
    // the larger first level: couplings, b and divisor of each thread's cells
    BigCell<R, ND> bk[2][kCoarseBigPer / 2];
    if (big) {
#pragma unroll
        for (int col = 0; col < 2; ++col)
#pragma unroll
            for (int m = 0; m < kCoarseBigPer / 2; ++m) {
                const int e = tid + kCoarseThreads * m;
                bk[col][m].c = -1;
                if (e < gB.N / 2) {
                    bk[col][m] = big_cell<R, ND, UNIT>(G, gB, colour_cell(gB.n, col, e));
                    const int c = bk[col][m].c;
                    bigx[c] = top_first ? (R)0.0 : gB.x[c];
                }
            }
    }
    __syncthreads();
    if (tid == 0) {
        int off = 0, el = 0;
        for (int l = lf; l < nlev; ++l) {
            base[l] = off;
            off += (4 + ND) * lN[l];
            first_el[l] = el;
            el += nload[l] * lN[l];
        }
        first_el[nlev] = el;
    }
    __syncthreads();
    {
        constexpr int U = 4;  // loads in flight per thread
        const int total = first_el[nlev];
        for (int e0 = tid; e0 < total; e0 += U * kCoarseThreads) {
            R v[U];
            int dst[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = e0 + u * kCoarseThreads;
                dst[u] = -1;
                v[u] = (R)0.0;
                if (e < total) {
                    int l = lf;
                    while (e >= first_el[l + 1]) ++l;
                    const int n = lN[l], r = e - first_el[l], k = r / n, c = r - k * n;
                    v[u] = lsrc[l][k][c];
                    dst[u] = base[l] + lslot[l][k] * n + c;
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (dst[u] >= 0) sm[dst[u]] = v[u];
        }
    }
    __syncthreads();
    if (big) {
        // pre-smoothing, residual and restriction onto the first LDS level
        big_smooth<R, ND, UNIT>(G, gB, bigx, bk, (light > 0 && gB.N <= light) ? 1 : nu1, top_first);
#pragma unroll
        for (int col = 0; col < 2; ++col)
#pragma unroll
            for (int m = 0; m < kCoarseBigPer / 2; ++m)
                if (bk[col][m].c >= 0) rbuf[bk[col][m].c] = big_resid<R, ND, UNIT>(G, gB, bk[col][m], bigx);
        __syncthreads();
        lds_restrict_sum<R, ND>(gB, lds_view<R, ND>(ldim, lf, sm, base[lf]), rbuf);
        __syncthreads();
    }
    // the LDS levels: x of the first one starts at 0 below a larger level
    const bool lds_first = big ? true : top_first;
    for (int l = lf; l < nlev - 1; ++l) {
        const bool first = l == lf ? lds_first : true;
        const LevelT<R> L = lds_view<R, ND>(ldim, l, sm, base[l]);
        const LevelT<R> C = lds_view<R, ND>(ldim, l + 1, sm, base[l + 1]);
        lds_smooth<R, ND, UNIT>(G, L, (light > 0 && L.N <= light) ? 1 : nu1, first);
        lds_resid<R, ND, UNIT>(G, L, rbuf, tid, kCoarseThreads);
        __syncthreads();
        lds_restrict_sum<R, ND>(L, C, rbuf);
        __syncthreads();
    }
    {
        const LevelT<R> L = lds_view<R, ND>(ldim, nlev - 1, sm, base[nlev - 1]);
        lds_smooth<R, ND, UNIT>(G, L, nuc, nlev - 1 == lf ? lds_first : true);
    }
    for (int l = nlev - 2; l >= lf; --l) {
        const LevelT<R> L = lds_view<R, ND>(ldim, l, sm, base[l]);
        const LevelT<R> C = lds_view<R, ND>(ldim, l + 1, sm, base[l + 1]);
        for (int c = tid; c < L.N; c += kCoarseThreads) L.x[c] = L.x[c] + prolong_cell<R, ND>(G, C, C.x, lcoords(L, c));
        __syncthreads();
        lds_smooth<R, ND, UNIT>(G, L, (light > 0 && L.N <= light) ? 1 : nu2, false);
    }
    if (big) {
        const LevelT<R> C = lds_view<R, ND>(ldim, lf, sm, base[lf]);
#pragma unroll
        for (int col = 0; col < 2; ++col)
#pragma unroll
            for (int m = 0; m < kCoarseBigPer / 2; ++m) {
                const int c = bk[col][m].c;
                if (c >= 0) bigx[c] = bigx[c] + prolong_cell<R, ND>(G, C, C.x, unpack_ijk(bk[col][m].pq));
            }
        __syncthreads();
        big_smooth<R, ND, UNIT>(G, gB, bigx, bk, (light > 0 && gB.N <= light) ? 1 : nu2, false);
        for (int c = tid; c < gB.N; c += kCoarseThreads) gB.x[c] = bigx[c];
    } else {
        const LevelT<R> T = lds_view<R, ND>(ldim, from, sm, base[from]);
        for (int c = tid; c < T.N; c += kCoarseThreads) gB.x[c] = T.x[c];
    }
}

// light: levels (not the coarsest) of at most this many cells take one pre-
// and one post-smoothing sweep (0: none); x0: the first half-sweep's colour-0
// values of this (multi-block, not the coarsest) level are already in x
// (formed with its right-hand side), so that half-sweep is skipped
template <typename R>
static void vcycle_level(const Grid& G, const LevelSet<R>& S, const LevelT<R>* Ld, int l, int nlev,
                         int coarse_from, int nu1, int nu2, int nuc, int light, bool first, bool x0,
                         hipStream_t stream) {
    if (l >= coarse_from) {
        JFNK_PROF(KC_MG_COARSE, stream);
        const int ft = first ? 1 : 0;
        const dim3 g(1), bl(kCoarseThreads);
        if (G.ndim == 3) {
            if (S.L[l].unit_sig)
                JFNK_KLAUNCH((k_coarse_vcycle<R, 3, true>), g, bl, 0, stream, G, Ld, l, nlev, nu1, nu2, nuc, ft, light);
            else
                JFNK_KLAUNCH((k_coarse_vcycle<R, 3, false>), g, bl, 0, stream, G, Ld, l, nlev, nu1, nu2, nuc, ft, light);
        } else {
            if (S.L[l].unit_sig)
                JFNK_KLAUNCH((k_coarse_vcycle<R, 2, true>), g, bl, 0, stream, G, Ld, l, nlev, nu1, nu2, nuc, ft, light);
            else
                JFNK_KLAUNCH((k_coarse_vcycle<R, 2, false>), g, bl, 0, stream, G, Ld, l, nlev, nu1, nu2, nuc, ft, light);
        }
        return;
    }
    const LevelT<R>& L = S.L[l];
    if (light > 0 && L.N <= light) nu1 = nu2 = 1;
    const dim3 bl(kBx, kBy);
    // compulsory bytes of a half-sweep: the couplings of every face (ndim per
    // cell, or the one cell field they are formed from), b (and D without
    // unit sigma) and the other colour's x for half the cells, this colour's
    // x written; the two-buffer sweep of an odd periodic coarsest level also
    // writes the other colour's copy
    const double bs = (double)L.N * sizeof(R) * ((L.qf ? 0 : G.ndim) + 1.5 + (L.unit_sig ? 0.0 : 0.5)) +
                      (L.qf ? (double)L.N * sizeof(double) : 0.0);
    const double bs_pp = bs + 0.5 * (double)L.N * sizeof(R);
    if (l == nlev - 1) {
        // coarsest level too large for the single-workgroup solve: the same
        // nuc red-black sweeps as multi-block launches
        bool odd = false;
        for (int d = 0; d < G.ndim; ++d) odd = odd || (G.bc[d] == PERIODIC && (L.n[d] & 1));
        if (odd) {
            const dim3 fg = cell_grid3(L.n);
            for (int s = 0; s < nuc; ++s) {
                {
                    JFNK_PROFB(KC_MG_SMOOTH, stream, bs_pp);
                    JFNK_LAUNCH_RND(G.ndim, k_gs_pp, R, fg, bl, 0, stream, G, L, 0, (first && s == 0) ? 1 : 0,
                                    (const R*)L.x, L.x2);
                }
                {
                    JFNK_PROFB(KC_MG_SMOOTH, stream, bs_pp);
                    JFNK_LAUNCH_RND(G.ndim, k_gs_pp, R, fg, bl, 0, stream, G, L, 1, 0, (const R*)L.x2, L.x);
                }
            }
            return;
        }
        for (int s = 0; s < nuc; ++s) {
            {
                JFNK_PROFB(KC_MG_SMOOTH, stream, bs);
                launch_gs<R>(G, L, 0, (first && s == 0) ? 1 : 0, stream);
            }
            {
                JFNK_PROFB(KC_MG_SMOOTH, stream, bs);
                launch_gs<R>(G, L, 1, 0, stream);
            }
        }
        return;
    }
    for (int s = 0; s < nu1; ++s) {
        if (!(first && x0 && s == 0)) {
            JFNK_PROFB(KC_MG_SMOOTH, stream, bs);
            launch_gs<R>(G, L, 0, (first && s == 0) ? 1 : 0, stream);
        }
        {
            JFNK_PROFB(KC_MG_SMOOTH, stream, bs);
            launch_gs<R>(G, L, 1, 0, stream);
        }
    }
    {
        // fine x, b, couplings (and sigma) read once, coarse b written
        JFNK_PROFB(KC_MG_RESTRICT, stream,
                   (double)L.N * sizeof(R) * (2 + G.ndim + (L.unit_sig ? 0 : 1)) + (double)S.L[l + 1].N * sizeof(R));
        if (G.ndim == 3) {
            if (L.unit_sig)
                JFNK_KLAUNCH((k_restrict<R, 3, true>), restrict_grid<3>(L.n), restrict_block<3>(), 0, stream, G, L, S.L[l + 1]);
            else
                JFNK_KLAUNCH((k_restrict<R, 3, false>), restrict_grid<3>(L.n), restrict_block<3>(), 0, stream, G, L, S.L[l + 1]);
        } else {
            if (L.unit_sig)
                JFNK_KLAUNCH((k_restrict<R, 2, true>), restrict_grid<2>(L.n), restrict_block<2>(), 0, stream, G, L, S.L[l + 1]);
            else
                JFNK_KLAUNCH((k_restrict<R, 2, false>), restrict_grid<2>(L.n), restrict_block<2>(), 0, stream, G, L, S.L[l + 1]);
        }
    }
    vcycle_level(G, S, Ld, l + 1, nlev, coarse_from, nu1, nu2, nuc, light, true, false, stream);
    // the prolongation goes into the first post-smoothing half-sweep on
    // levels of at most kGsProlongMaxCells cells; on larger ones the fused
    // sweep (about 80 VGPRs in FP64, 5 waves per SIMD) measured slower than
    // the prolongation and the half-sweep as two launches
    const bool fuse = nu2 > 0 && L.N <= kGsProlongMaxCells;
    if (nu2 == 0) {
        JFNK_PROFB(KC_MG_PROLONG, stream, (double)L.N * sizeof(R) * 2 + (double)S.L[l + 1].N * sizeof(R));
        JFNK_LAUNCH_RND(G.ndim, k_prolong, R, cell_grid3(L.n), bl, 0, stream, G, L, S.L[l + 1], -1);
    } else if (!fuse) {
        JFNK_PROFB(KC_MG_PROLONG, stream, (double)L.N * sizeof(R) + (double)S.L[l + 1].N * sizeof(R));
        JFNK_LAUNCH_RND(G.ndim, k_prolong_c1, R, cell_grid3(S.L[l + 1].n), bl, 0, stream, G, L, S.L[l + 1]);
    }
    for (int s = 0; s < nu2; ++s) {
        if (s == 0 && fuse) {
            // the correction read with the half-sweep: the coarse x once more
            JFNK_PROFB(KC_MG_SMOOTH, stream, bs + (double)S.L[l + 1].N * sizeof(R));
            launch_gs_prolong<R>(G, L, S.L[l + 1], stream);
        } else {
            JFNK_PROFB(KC_MG_SMOOTH, stream, bs);
            launch_gs<R>(G, L, 0, 0, stream);
        }
        {
            JFNK_PROFB(KC_MG_SMOOTH, stream, bs);
            launch_gs<R>(G, L, 1, 0, stream);
        }
    }
}

template <typename R>
void mg_vcycle(const Grid& G, const LevelSet<R>& S, const LevelT<R>* Ld, int nlev, int coarse_from, int nu1, int nu2,
               int nuc, int light, bool first, bool x0, hipStream_t stream) {
    vcycle_level(G, S, Ld, 0, nlev, coarse_from, nu1, nu2, nuc, light, first, x0, stream);
}

// ---------------------------------------------------------------- right-hand sides and back-substitution
// x/b index on the finest level of the cell one step along d from q (periodic
// wrap; the caller excludes steps through a wall)
template <typename R>
__device__ __forceinline__ int xb_shifted(const LevelT<R>& L, const Ijk& q, int d, int s) {
    int v[3] = {q.v[0], q.v[1], q.v[2]};
    int a = v[d] + s;
    if (a < 0) a += L.n[d];
    else if (a >= L.n[d]) a -= L.n[d];
    v[d] = a;
    return xbi(L, v[0], v[1], v[2]);
}
// enthalpy on the lower face of cell c along d: the mean of the two cells'
// values, 0 on a wall
__device__ __forceinline__ double face_h(const Grid& G, const PcCoef& C, const Ijk& q, long c, int d) {
    const bool wall = G.bc[d] == WALL && q.v[d] == 0;
    const double h = 0.5 * (C.H[wall ? c : shifted(G, q, d, -1)] + C.H[c]);  // load issued on walls too
    return wall ? 0.0 : h;
}
// RE: the energy right-hand side comes from the conduction solve (rE), else
// from v (compile-time, so that the loads form one block)
// Right-hand side of the Schur complement at cell q from the energy
// right-hand side re and the momentum entries of v, read through VM(d, x):
// the value of v's component d at cell x.  FACES(d, lower_open, h_lower,
// upper_open, h_upper) receives the face enthalpies along d as formed here.
template <int ND, class VM, class FACES>
__device__ __forceinline__ double pc_rhs_value(const Grid& G, const PcCoef& C, const Ijk& q, long c, double re,
                                               Scales5 sc, VM vm, FACES faces) {
    double acc = 0.0;
    for (int d = 0; d < ND; ++d) {
        const double s = sc.v[2 + d];
        const double hlo = face_h(G, C, q, c, d);
        const double flo = hlo * (s * vm(d, c));
        const bool top = G.bc[d] == WALL && q.v[d] == G.n[d] - 1;
        const long up = top ? c : shifted(G, q, d, 1);  // loads issued at a top wall too, value discarded
        const double hhi = 0.5 * (C.H[c] + C.H[up]);
        const double fu = hhi * (s * vm(d, up));
        faces(d, !(G.bc[d] == WALL && q.v[d] == 0), hlo, !top, hhi);
        const double fhi = top ? 0.0 : fu;
        if (G.sph) {
            const int i = q.v[0], j = q.v[1];
            const double Alo = sph_area(G, d, i, j), Ahi = sph_area(G, d, d == 0 ? i + 1 : i, d == 1 ? j + 1 : j);
            acc = acc + (Ahi * fhi - Alo * flo) / sph_vol(G, i, j);
        } else {
            acc = acc + (fhi - flo) * G.idx[d];
        }
    }
    double rp = G.gm1 * (re - C.tau * acc);
    if (G.sph) rp = rp * sph_vol(G, q.v[0], q.v[1]);  // volume-weighted system
    return rp;
}
// The level's right-hand side at cell q and, with X0 (the finest level's
// couplings formed from the enthalpy, unit sigma), the first multigrid
// half-sweep's colour-0 value from x = 0 as well, so the V-cycle skips that
// half-sweep.  The couplings come from the face enthalpies the right-hand
// side has just formed (the sums qf_coupling forms from the same cells), and
// the value is formed as gs_value forms a first-sweep value, operation for
// operation.
template <typename R, int ND>
struct FirstSweep {
    R alo[ND], ahi[ND];
    bool hd[ND], hu[ND];
};
template <typename R, int ND, bool X0, class VM>
__device__ __forceinline__ void put_level_rhs(const Grid& G, const PcCoef& C, const LevelT<R>& L0, const Ijk& q,
                                              long c, double re, Scales5 sc, VM vm) {
    FirstSweep<R, ND> f;
    const bool red = ((q.v[0] + q.v[1] + q.v[2]) & 1) == 0;
    const auto faces = [&](int d, bool lo_open, double hlo, bool hi_open, double hhi) {
        if (!X0) return;
        const double k0 = L0.K0[0];
        f.hd[d] = lo_open;
        f.hu[d] = hi_open;
        f.alo[d] = lo_open ? (R)((k0 * hlo) * L0.i2[d]) : (R)0.0;
        f.ahi[d] = hi_open ? (R)((k0 * hhi) * L0.i2[d]) : (R)0.0;
    };
    const double rp = pc_rhs_value<ND>(G, C, q, c, re, sc, vm, faces);
    const int e = xbi(L0, q.v[0], q.v[1], q.v[2]);
    const R bq = (R)rp;
    L0.b[e] = bq;
    if (X0 && red) {
        R num = bq, den = (R)1.0;
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            num = f.hd[d] ? num + f.alo[d] * (R)0.0 : num;
            num = f.hu[d] ? num + f.ahi[d] * (R)0.0 : num;
            den = den + f.alo[d];
            den = den + f.ahi[d];
        }
        L0.x[e] = num / den;
    }
}
template <typename R, int ND, bool RE, bool X0>
__global__ void __launch_bounds__(kBlock) k_pc_rhs(Grid G, PcCoef C, const R* __restrict__ v,
                                                   const double* __restrict__ rE, Scales5 sc, LevelT<R> L0) {
    Ijk q;
    long c;
    if (!cell_from_launch(G, q, c)) return;
    const double re = RE ? rE[c] : sc.v[1] * (double)v[G.N + c];
    const auto vm = [&](int d, long x) { return (double)v[(long)(2 + d) * G.N + x]; };
    put_level_rhs<R, ND, X0>(G, C, L0, q, c, re, sc, vm);
}
// A Krylov basis vector v = w / hn stored (the cell's 2 + ND entries) together
// with the acoustic right-hand side k_pc_rhs forms from it: the neighbours'
// entries of v are formed again from w (the same bits as the stored ones),
// so the next preconditioner application need not read v for it.  hn is
// given, or (DEV) formed on the device as sqrt of the sum in hnsq.
template <typename R, int ND, bool DEV, bool X0>
__global__ void __launch_bounds__(kBlock) k_store_pc_rhs(Grid G, PcCoef C, const double* __restrict__ w,
                                                         R* __restrict__ v, double hn_given,
                                                         const double* __restrict__ hnsq, Scales5 sc,
                                                         LevelT<R> L0) {
    Ijk q;
    long c;
    if (!cell_from_launch(G, q, c)) return;
    const double hn = DEV ? sqrt(hnsq[0]) : hn_given;
#pragma unroll
    for (int f = 0; f < 2 + ND; ++f) v[(long)f * G.N + c] = (R)(w[(long)f * G.N + c] / hn);
    const double re = sc.v[1] * (double)(R)(w[G.N + c] / hn);
    const auto vm = [&](int d, long x) { return (double)(R)(w[(long)(2 + d) * G.N + x] / hn); };
    put_level_rhs<R, ND, X0>(G, C, L0, q, c, re, sc, vm);
}

template <typename R, int ND>
__global__ void __launch_bounds__(kBlock) k_pc_diff_back(Grid G, PcCoef C, const R* __restrict__ v,
                                                         LevelT<R> L0, Scales5 sc, double* __restrict__ rE) {
    Ijk q;
    long c;
    if (!cell_from_launch(G, q, c)) return;
    const R* __restrict__ s = L0.x;
    double acc = G.sph ? 0.0 : sc.v[1] * (double)v[G.N + c];
    const double sc0 = (double)s[xbi(L0, q.v[0], q.v[1], q.v[2])];
    for (int d = 0; d < ND; ++d) {
        const bool top = G.bc[d] == WALL && q.v[d] == G.n[d] - 1;
        const bool bot = G.bc[d] == WALL && q.v[d] == 0;
        double thi = 0.0, tlo = 0.0;
        if (!top) {
            const long up = shifted(G, q, d, 1);
            thi = C.beta[d][up] * ((double)s[xb_shifted(L0, q, d, 1)] - sc0);
        }
        if (!bot) tlo = C.beta[d][c] * (sc0 - (double)s[xb_shifted(L0, q, d, -1)]);
        acc = acc + (thi - tlo);
    }
    rE[c] = G.sph ? sc.v[1] * (double)v[G.N + c] + acc / sph_vol(G, q.v[0], q.v[1]) : acc;
}

template <typename R, int ND, bool RE>
__global__ void __launch_bounds__(kBlock) k_pc_back(Grid G, PcCoef C, const R* __restrict__ v,
                                                    const double* __restrict__ rE, const R* __restrict__ dp,
                                                    LevelT<R> L0, Scales5 sc, R* __restrict__ z,
                                                    double* __restrict__ part) {
    Ijk q;
    long c = 0;
    double ss = 0.0;
    if (cell_from_launch(G, q, c)) {
        const double re = RE ? rE[c] : sc.v[1] * (double)v[G.N + c];
        const double dpc = (double)dp[xbi(L0, q.v[0], q.v[1], q.v[2])];
        double dmlo[3], dmhi[3];
        bool top[3];
        long upi[3];
        for (int d = 0; d < ND; ++d) {
            const R* vm = v + (long)(2 + d) * G.N;
            const double s = sc.v[2 + d];
            // both neighbours are loaded on walls too (the wrap keeps them in
            // bounds) and the wall faces' values replaced by 0
            const long up = shifted(G, q, d, 1);
            const double lo = s * (double)vm[c] - C.tau * ((dpc - (double)dp[xb_shifted(L0, q, d, -1)]) * face_ids(G, d, q.v[0]));
            const double hi = s * (double)vm[up] - C.tau * (((double)dp[xb_shifted(L0, q, d, 1)] - dpc) * face_ids(G, d, q.v[0]));
            top[d] = G.bc[d] == WALL && q.v[d] == G.n[d] - 1;
            dmlo[d] = (G.bc[d] == WALL && q.v[d] == 0) ? 0.0 : lo;
            dmhi[d] = top[d] ? 0.0 : hi;
            upi[d] = up;
        }
        // divergence of face values: (hi - lo)/dx, or on spherical grids
        // (A_hi hi - A_lo lo)/V
        auto divterm = [&](int d, double hi, double lo) {
            if (!G.sph) return (hi - lo) * G.idx[d];
            const int i = q.v[0], j = q.v[1];
            const double Alo = sph_area(G, d, i, j), Ahi = sph_area(G, d, d == 0 ? i + 1 : i, d == 1 ? j + 1 : j);
            return (Ahi * hi - Alo * lo) / sph_vol(G, i, j);
        };
        double acc = 0.0;
        for (int d = 0; d < ND; ++d) acc = acc + divterm(d, dmhi[d], dmlo[d]);
        const double drho = sc.v[0] * (double)v[c] - C.tau * acc;
        acc = 0.0;
        for (int d = 0; d < ND; ++d) {
            const double flo = face_h(G, C, q, c, d) * dmlo[d];
            const double fhi = top[d] ? 0.0 : (0.5 * (C.H[c] + C.H[upi[d]])) * dmhi[d];
            acc = acc + divterm(d, fhi, flo);
        }
        const double dE = re - C.tau * acc;
        // the norm is that of the stored values (the product's direction)
        double t = (double)(R)(drho / sc.v[0]);
        z[c] = (R)t;
        ss += t * t;
        t = (double)(R)(dE / sc.v[1]);
        z[G.N + c] = (R)t;
        ss += t * t;
        for (int d = 0; d < ND; ++d) {
            t = (double)(R)(dmlo[d] / sc.v[2 + d]);
            z[(long)(2 + d) * G.N + c] = (R)t;
            ss += t * t;
        }
    }
    __shared__ double sh[kBlock / 64];
    const double t = block_sum(ss, sh);
    if (lin_thread() == 0) part[lin_block()] = t;
}

template <typename R>
__global__ void __launch_bounds__(kBlock) k_field_scaled(const R* __restrict__ v, double s,
                                                         double* __restrict__ out, long N) {
    const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < N) out[c] = s * (double)v[c];
}

template <typename R, int ND>
__global__ void __launch_bounds__(kBlock) k_field_to_level(Grid G, const R* __restrict__ v, double s,
                                                           LevelT<R> L0) {
    Ijk q;
    long c;
    if (!cell_from_launch(G, q, c)) return;
    double b = s * (double)v[c];
    if (G.sph) b = b * sph_vol(G, q.v[0], q.v[1]);  // volume-weighted system
    L0.b[xbi(L0, q.v[0], q.v[1], q.v[2])] = (R)b;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_copy_sumsq(const T* __restrict__ v, T* __restrict__ z,
                                                       long n, double* __restrict__ part) {
    double ss = 0.0;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        const T t = v[e];
        z[e] = t;
        ss += (double)t * (double)t;
    }
    __shared__ double sh[kBlock / 64];
    const double t = block_sum(ss, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void __launch_bounds__(kFinalThreads) k_jv_eps(const double* __restrict__ usumsq,
                                                          const double* __restrict__ part, int nblk, double nunk,
                                                          double* __restrict__ eps) {
    __shared__ double sh[kFinalThreads / 64];
    double s = 0.0;
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) s += part[i];
    const double vs = block_sum(s, sh);
    if (threadIdx.x == 0) {
        const double urms = sqrt(usumsq[0]) / sqrt(nunk);
        const double vn = sqrt(vs) / sqrt(nunk);
        eps[0] = vn == 0.0 ? 0.0 : sqrt(2.220446049250313e-16) * (1.0 + urms) / vn;
    }
}

template <typename R>
void launch_pc_rhs(const Grid& G, const PcCoef& C, const R* v, const double* rE, Scales5 sc,
                   const LevelT<R>& L0, bool x0, hipStream_t stream) {
    {
        // v (sizeof(R)), enthalpy, rE; the level's right-hand side
        JFNK_PROFB(KC_PC_RHS, stream,
                   (double)sizeof(R) * G.N * (G.ndim + (rE ? 0 : 1)) + 8.0 * G.N * (1 + (rE ? 1 : 0)) +
                       (double)sizeof(R) * G.N);
        const dim3 g = cell_grid3(G.n), bl(kBx, kBy);
#define RHS(ND, RE, X0) JFNK_KLAUNCH((k_pc_rhs<R, ND, RE, X0>), g, bl, 0, stream, G, C, v, rE, sc, L0)
        if (G.ndim == 3) {
            if (rE) { if (x0) RHS(3, true, true); else RHS(3, true, false); }
            else { if (x0) RHS(3, false, true); else RHS(3, false, false); }
        } else {
            if (rE) { if (x0) RHS(2, true, true); else RHS(2, true, false); }
            else { if (x0) RHS(2, false, true); else RHS(2, false, false); }
        }
#undef RHS
    }
}
template <typename R>
void launch_store_pc_rhs(const Grid& G, const PcCoef& C, const double* w, R* v, double hn, const double* hnsq,
                         Scales5 sc, const LevelT<R>& L0, bool x0, hipStream_t stream) {
    // w read, v and the level's right-hand side written, the enthalpy read
    JFNK_PROFB(KC_STORE, stream, (double)G.nvec * (8 + sizeof(R)) + (double)G.N * (8 + sizeof(R)));
    const dim3 g = cell_grid3(G.n), bl(kBx, kBy);
#define ST(ND, DEV, X0) \
    JFNK_KLAUNCH((k_store_pc_rhs<R, ND, DEV, X0>), g, bl, 0, stream, G, C, w, v, hn, hnsq, sc, L0)
    if (G.ndim == 3) {
        if (hnsq) { if (x0) ST(3, true, true); else ST(3, true, false); }
        else { if (x0) ST(3, false, true); else ST(3, false, false); }
    } else {
        if (hnsq) { if (x0) ST(2, true, true); else ST(2, true, false); }
        else { if (x0) ST(2, false, true); else ST(2, false, false); }
    }
#undef ST
}
template <typename R>
void launch_pc_diff_back(const Grid& G, const PcCoef& C, const R* v, const LevelT<R>& L0, Scales5 sc,
                         double* rE, hipStream_t stream) {
    {
        JFNK_PROF(KC_PC_RHS, stream);
        JFNK_LAUNCH_RND(G.ndim, k_pc_diff_back, R, cell_grid3(G.n), dim3(kBx, kBy), 0, stream, G, C, v, L0, sc, rE);
    }
}
template <typename R>
void launch_pc_back(const Grid& G, const PcCoef& C, const R* v, const double* rE, const R* dp,
                    const LevelT<R>& L0, Scales5 sc, R* z, double* part, int nblk, hipStream_t stream) {
    (void)nblk;
    {
        // v read and z written (sizeof(R)), enthalpy, rE, dp
        JFNK_PROFB(KC_PC_BACK, stream,
                   (double)sizeof(R) * G.nvec * 2 + 8.0 * G.N * (1 + (rE ? 1 : 0)) + (double)sizeof(R) * G.N);
        const dim3 g = cell_grid3(G.n), bl(kBx, kBy);
        if (G.ndim == 3) {
            if (rE) JFNK_KLAUNCH((k_pc_back<R, 3, true>), g, bl, 0, stream, G, C, v, rE, dp, L0, sc, z, part);
            else JFNK_KLAUNCH((k_pc_back<R, 3, false>), g, bl, 0, stream, G, C, v, rE, dp, L0, sc, z, part);
        } else {
            if (rE) JFNK_KLAUNCH((k_pc_back<R, 2, true>), g, bl, 0, stream, G, C, v, rE, dp, L0, sc, z, part);
            else JFNK_KLAUNCH((k_pc_back<R, 2, false>), g, bl, 0, stream, G, C, v, rE, dp, L0, sc, z, part);
        }
    }
}
template <typename R>
void launch_field_scaled(const R* v, double s, double* out, long N, hipStream_t stream) {
    {
        JFNK_PROF(KC_PC_RHS, stream);
        JFNK_KLAUNCH((k_field_scaled<R>), dim3(grid_blocks(N)), dim3(kBlock), 0, stream, v, s, out, N);
    }
}
template <typename R>
void launch_field_to_level(const Grid& G, const R* v, double s, const LevelT<R>& L0, hipStream_t stream) {
    {
        JFNK_PROF(KC_PC_RHS, stream);
        JFNK_LAUNCH_RND(G.ndim, k_field_to_level, R, cell_grid3(G.n), dim3(kBx, kBy), 0, stream, G, v, s, L0);
    }
}
template <typename T>
void launch_copy_sumsq(const T* v, T* z, long n, double* part, int nblk, hipStream_t stream) {
    {
        JFNK_PROF(KC_OTHER, stream);
        JFNK_KLAUNCH((k_copy_sumsq<T>), dim3(nblk), dim3(kBlock), 0, stream, v, z, n, part);
    }
}
template void launch_copy_sumsq<double>(const double*, double*, long, double*, int, hipStream_t);
template void launch_copy_sumsq<float>(const float*, float*, long, double*, int, hipStream_t);
void launch_jv_eps(const double* usumsq, const double* part_v, int nblk, double nunk, double* eps,
                   hipStream_t stream) {
    {
        JFNK_PROF(KC_REDUCE, stream);
        JFNK_KLAUNCH(k_jv_eps, dim3(1), dim3(kFinalThreads), 0, stream, usumsq, part_v, nblk, nunk, eps);
    }
}

// ---------------------------------------------------------------- alternating-direction line solves
// One thread per line along axis d; Thomas algorithm, and for periodic lines
// the Sherman-Morrison correction of a modified Thomas system.  Scratch per
// line lives in the cell-indexed arrays cp, dp, bb, zz.
template <typename R>
__device__ __forceinline__ void line_row(const Grid& G, const PcCoef& C, int d, int kind, const Ijk& q0, int t,
                                         double& a, double& b, double& cc) {
    Ijk q = q0;
    q.v[d] = t;
    const long c = flat(G, q.v[0], q.v[1], q.v[2]);
    const int n = G.n[d];
    const bool wall = G.bc[d] == WALL;
    const bool has_up = !(wall && t == n - 1), has_dn = !(wall && t == 0);
    const long up = has_up ? shifted(G, q, d, 1) : -1;
    const long dn = has_dn ? shifted(G, q, d, -1) : -1;
    if (kind == 0) {
        const double klo = C.kap[d][c], khi = has_up ? C.kap[d][up] : 0.0;
        a = -klo;
        cc = -khi;
        b = 1.0 + (klo + khi);
    } else {
        const double klo = C.beta[d][c], khi = has_up ? C.beta[d][up] : 0.0;
        const double wl = has_dn ? C.W[dn] : 0.0, wr = has_up ? C.W[up] : 0.0;
        a = -klo * wl;
        cc = -khi * wr;
        b = 1.0 + (klo + khi) * C.W[c];
    }
}

template <typename R>
__global__ void __launch_bounds__(kBlock) k_line(Grid G, PcCoef C, int d, int kind, R* __restrict__ x,
                                                 double* __restrict__ cp, double* __restrict__ dpv,
                                                 double* __restrict__ x1, double* __restrict__ zz) {
    // consecutive threads take lines adjacent along the lowest other axis:
    // for y- and z-lines that is x, so a wave's loads and stores at one
    // position along the line are contiguous
    const int r1 = d == 0 ? 1 : 0, r2 = d == 2 ? 1 : 2;
    const long nl = (long)G.n[r1] * G.n[r2];
    const long line = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (line >= nl) return;
    Ijk q0;
    q0.v[d] = 0;
    q0.v[r1] = (int)(line % G.n[r1]);
    q0.v[r2] = (int)(line / G.n[r1]);
    const int n = G.n[d];
    const long sd = G.stride[d];
    const long base = flat(G, q0.v[0], q0.v[1], q0.v[2]);
    const bool periodic = G.bc[d] == PERIODIC;
    double a0, b0, c0, an, bn, cn;
    line_row<R>(G, C, d, kind, q0, 0, a0, b0, c0);
    line_row<R>(G, C, d, kind, q0, n - 1, an, bn, cn);
    const double gam = -b0, alpha = a0, beta = cn;
    // pass 1: Thomas on (a, bb, c, x)
    for (int rhs = 0; rhs < (periodic ? 2 : 1); ++rhs) {
        double cprev = 0.0, dprev = 0.0;
        for (int t = 0; t < n; ++t) {
            double a, b, cc;
            line_row<R>(G, C, d, kind, q0, t, a, b, cc);
            if (periodic) {
                if (t == 0) b = b0 - gam;
                if (t == n - 1) b = bn - beta * alpha / gam;
            }
            double dv;
            if (rhs == 0) dv = (double)x[base + t * sd];
            else dv = t == 0 ? gam : (t == n - 1 ? beta : 0.0);
            double cpt, dpt;
            if (t == 0) {
                cpt = cc / b;
                dpt = dv / b;
            } else {
                const double den = b - a * cprev;
                cpt = cc / den;
                dpt = (dv - a * dprev) / den;
            }
            cp[base + t * sd] = cpt;
            dpv[base + t * sd] = dpt;
            cprev = cpt;
            dprev = dpt;
        }
        double xn = dpv[base + (long)(n - 1) * sd];
        double* out = rhs == 0 ? x1 : zz;
        out[base + (long)(n - 1) * sd] = xn;
        for (int t = n - 2; t >= 0; --t) {
            xn = dpv[base + t * sd] - cp[base + t * sd] * xn;
            out[base + t * sd] = xn;
        }
    }
    if (periodic) {
        const double x0 = x1[base], xl = x1[base + (long)(n - 1) * sd];
        const double z0 = zz[base], zl = zz[base + (long)(n - 1) * sd];
        const double fact = (x0 + alpha * xl / gam) / (1.0 + z0 + alpha * zl / gam);
        for (int t = 0; t < n; ++t) x[base + t * sd] = (R)(x1[base + t * sd] - fact * zz[base + t * sd]);
    } else {
        for (int t = 0; t < n; ++t) x[base + t * sd] = (R)x1[base + t * sd];
    }
}

template <typename R>
void launch_line_solve(const Grid& G, const PcCoef& C, int d, int kind, R* x, double* scratch4,
                       hipStream_t stream) {
    const int r1 = (d + 1) % 3, r2 = (d + 2) % 3;
    const long nl = (long)G.n[r1] * G.n[r2];
    {
        JFNK_PROF(KC_LINES, stream);
        JFNK_KLAUNCH((k_line<R>), dim3(grid_blocks(nl)), dim3(kBlock), 0, stream, G, C, d, kind, x, scratch4,
                           scratch4 + G.N, scratch4 + 2 * G.N, scratch4 + 3 * G.N);
    }
}

// ---------------------------------------------------------------- instantiations
#define INST(R)                                                                                              \
    template void launch_level0<R>(const Grid&, const PcCoef&, int, const LevelT<R>&, hipStream_t);          \
    template void launch_coarsen<R>(const Grid&, const LevelT<R>&, const LevelT<R>&, hipStream_t);           \
    template void launch_level_diag<R>(const Grid&, const LevelT<R>&, hipStream_t);                          \
    template void mg_vcycle<R>(const Grid&, const LevelSet<R>&, const LevelT<R>*, int, int, int, int, int,     \
                               int, bool, bool, hipStream_t);                                                \
    template void launch_pc_rhs<R>(const Grid&, const PcCoef&, const R*, const double*, Scales5,        \
                                   const LevelT<R>&, bool, hipStream_t);                                     \
    template void launch_store_pc_rhs<R>(const Grid&, const PcCoef&, const double*, R*, double,          \
                                         const double*, Scales5, const LevelT<R>&, bool, hipStream_t);        \
    template void launch_pc_diff_back<R>(const Grid&, const PcCoef&, const R*, const LevelT<R>&,        \
                                         Scales5, double*, hipStream_t);                                     \
    template void launch_pc_back<R>(const Grid&, const PcCoef&, const R*, const double*, const R*,      \
                                    const LevelT<R>&, Scales5, R*, double*, int, hipStream_t);               \
    template void launch_field_scaled<R>(const R*, double, double*, long, hipStream_t);                      \
    template void launch_field_to_level<R>(const Grid&, const R*, double, const LevelT<R>&, hipStream_t);     \
    template void launch_line_solve<R>(const Grid&, const PcCoef&, int, int, R*, double*, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace jfnk
