// Passive scalars (section 2.2 of Goffrey et al. 2016): partial densities
// s_k = c_k rho carried by the flow, d s_k/dt = -div(c_k rho u).  The face
// flux is the face mass flux of the flow times the concentration c = s/rho
// reconstructed on the face (upstream linear extrapolation with the van Leer
// limiter, upwind side by the sign of the mass flux; beyond a wall the
// mirror-image cell).  Residual consumers as for the flow:
//   b = s + h R(s) (old time), G = (s - b) - h R(s) with partial sums of G^2,
//   w = (G(s + eps v) - G(s)) / eps.
#include "kernels.hpp"

namespace jfnk {

// concentration of the cell at offset a along d from q (mirror beyond walls)
__device__ __forceinline__ double sconc(const Grid& G, const ScalarArgs& A, const double* sq, const double* vq,
                                        double e, Ijk q, int d, int a) {
    const int n = G.n[d];
    int x = q.v[d] + a;
    if (x < 0 || x >= n) {
        if (G.bc[d] == WALL) x = x < 0 ? -1 - x : 2 * n - 1 - x;
        else x = x < 0 ? x + n : x - n;
    }
    q.v[d] = x;
    const long c = flat(G, q.v[0], q.v[1], q.v[2]);
    double sv = sq[c];
    if (vq) sv = sv + e * vq[c];
    return sv / A.rho[c];
}

// scalar flux through the lower face of cell q along d
__device__ __forceinline__ double sflux(const Grid& G, const ScalarArgs& A, const double* sq, const double* vq,
                                        double e, const Ijk& q, int d) {
    if (G.bc[d] == WALL && q.v[d] == 0) return 0.0;
    const double f = A.fr[d][flat(G, q.v[0], q.v[1], q.v[2])];
    const double cLL = sconc(G, A, sq, vq, e, q, d, -2), cL = sconc(G, A, sq, vq, e, q, d, -1);
    const double cc = sconc(G, A, sq, vq, e, q, d, 0), cR = sconc(G, A, sq, vq, e, q, d, 1);
    const double sl = van_leer(cc - cL, cL - cLL);
    const double sr = van_leer(cR - cc, cc - cL);
    return f * upstream(f, cL, sl, cc, sr);
}

template <int ND>
__global__ void __launch_bounds__(kBlock) k_scalar_out(Grid G, ScalarArgs A) {
    Ijk q;
    long c = 0;
    double part = 0.0;
    if (cell_from_launch(G, q, c)) {
        const double e = A.mode == OUT_JV ? A.eps[0] : 0.0;
        for (int k = 0; k < A.ns; ++k) {
            const long off = (long)k * G.N;
            const double* sq = A.s + off;
            const double* vq = A.mode == OUT_JV ? A.v + off : nullptr;
            double r = 0.0;
#pragma unroll
            for (int d = 0; d < ND; ++d) {
                const double lo = sflux(G, A, sq, vq, e, q, d);
                double hi = 0.0;
                if (!(G.bc[d] == WALL && q.v[d] == G.n[d] - 1)) {
                    Ijk qu = q;
                    qu.v[d] = q.v[d] + 1 < G.n[d] ? q.v[d] + 1 : 0;
                    hi = sflux(G, A, sq, vq, e, qu, d);
                }
                r = r - (hi - lo) * G.idx[d];
            }
            const long x = off + c;
            if (A.mode == OUT_CN_OLD) {
                A.out[x] = sq[c] + A.h * r;
            } else if (A.mode == OUT_RESIDUAL) {
                const double g = (sq[c] - A.b[x]) - A.h * r;
                A.out[x] = g;
                part += g * g;
            } else {
                double w = 0.0;
                if (e != 0.0) {
                    const double sp = sq[c] + e * vq[c];
                    const double gp = (sp - A.b[x]) - A.h * r;
                    w = (gp - A.Gs[x]) / e;
                }
                A.out[x] = w;
            }
        }
    }
    if (A.partial) {
        __shared__ double sh[kBlock / 64];
        const double t = block_sum(part, sh);
        if (lin_thread() == 0) A.partial[lin_block()] = t;
    }
}

// concentrations re-normalised to sum to one: s_k <- s_k rho / sum_j s_j
__global__ void __launch_bounds__(kBlock) k_scalar_renorm(double* __restrict__ s, const double* __restrict__ rho,
                                                          int ns, long N) {
    for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (long)gridDim.x * blockDim.x) {
        double tot = 0.0;
        for (int k = 0; k < ns; ++k) tot = tot + s[(long)k * N + c];
        if (tot > 0.0)
            for (int k = 0; k < ns; ++k) s[(long)k * N + c] = s[(long)k * N + c] * (rho[c] / tot);
    }
}

// out = -in
__global__ void __launch_bounds__(kBlock) k_negate(const double* __restrict__ in, double* __restrict__ out, long n) {
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
        out[e] = -in[e];
}

void launch_scalar_out(const Grid& G, const ScalarArgs& A, hipStream_t stream) {
    JFNK_PROF(KC_OTHER, stream);
    JFNK_LAUNCH_ND(G.ndim, k_scalar_out, cell_grid3(G.n), dim3(kBx, kBy), 0, stream, G, A);
}
void launch_scalar_renorm(double* s, const double* rho, int ns, long N, hipStream_t stream) {
    JFNK_PROF(KC_OTHER, stream);
    JFNK_KLAUNCH(k_scalar_renorm, dim3(grid_blocks(N, kBlock * 4)), dim3(kBlock), 0, stream, s, rho, ns, N);
}
void launch_negate(const double* in, double* out, long n, hipStream_t stream) {
    JFNK_PROF(KC_OTHER, stream);
    JFNK_KLAUNCH(k_negate, dim3(grid_blocks(n, kBlock * 4)), dim3(kBlock), 0, stream, in, out, n);
}

}  // namespace jfnk
