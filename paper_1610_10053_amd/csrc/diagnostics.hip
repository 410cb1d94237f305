// Diagnostics of a state (reductions on the device): kinetic energy
// sum (1/2) rho |v|^2 dV with |v|^2 of a cell the mean over each axis of the
// squared velocities of its two faces (the Taylor-Green kinetic energy of
// section 5.3), mass and total energy, the maximum Mach number (section 3.1),
// the mixing-region width of eqs. (12)-(14) along a vertical axis, and the
// relative velocity error of eq. (17) against a higher-resolution solution.
#include <mutex>

#include "kernels.hpp"

namespace jfnk {

// per-block partials: sum kin dV-free, sum rho, sum E, max Mach
template <int ND>
__global__ void __launch_bounds__(kBlock) k_diag_cells(Grid G, Prim P, const double* __restrict__ u,
                                                       double* __restrict__ part) {
    Ijk q;
    long c = 0;
    double kin = 0.0, mass = 0.0, en = 0.0, mach = 0.0;
    if (cell_from_launch(G, q, c)) {
        double qk = 0.0;
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            const bool top = G.bc[d] == WALL && q.v[d] == G.n[d] - 1;
            const double a = P.uf[d][c];
            const double b = top ? 0.0 : P.uf[d][shifted(G, q, d, 1)];
            qk = qk + 0.5 * (a * a + b * b);
        }
        const double rho = P.rho[c];
        kin = 0.5 * rho * qk;
        mass = rho;
        en = u[G.N + c];
        mach = sqrt(qk) / sqrt(G.gamma * P.p[c] / rho);
    }
    __shared__ double sh[kBlock / 64];
    const long nb = (long)gridDim.x * gridDim.y * gridDim.z;
    const int b = lin_block();
    double t = block_sum(kin, sh);
    if (lin_thread() == 0) part[b] = t;
    __syncthreads();
    t = block_sum(mass, sh);
    if (lin_thread() == 0) part[nb + b] = t;
    __syncthreads();
    t = block_sum(en, sh);
    if (lin_thread() == 0) part[2 * nb + b] = t;
    __syncthreads();
    t = block_max(mach, sh);
    if (lin_thread() == 0) part[3 * nb + b] = t;
}

// one workgroup per layer normal to `axis`: X_M of the layer's mean X_H
__global__ void __launch_bounds__(kBlock) k_diag_layers(Grid G, Prim P, int axis, double rho_l, double rho_h,
                                                        double* __restrict__ xm) {
    const int j = (int)blockIdx.x;
    const int a1 = axis == 0 ? 1 : 0, a2 = axis == 2 ? 1 : 2;
    const long n1 = G.n[a1], n2 = G.n[a2], nl = n1 * n2;
    double s = 0.0;
    for (long e = threadIdx.x; e < nl; e += blockDim.x) {
        int v[3];
        v[axis] = j;
        v[a1] = (int)(e % n1);
        v[a2] = (int)(e / n1);
        const long c = flat(G, v[0], v[1], v[2]);
        s += (P.rho[c] - rho_l) / (rho_h - rho_l);
    }
    __shared__ double sh[kBlock / 64];
    const double t = block_sum(s, sh);
    if (threadIdx.x == 0) {
        const double mean = t / (double)nl;
        xm[j] = mean <= 0.5 ? 2.0 * mean : 2.0 * (1.0 - mean);
    }
}

// one workgroup per layer normal to `axis`: 2 min(<c1>, <c2>) of the layer
// means of the concentrations of two passive scalars
__global__ void __launch_bounds__(kBlock) k_diag_layers_scalars(Grid G, Prim P, const double* __restrict__ s,
                                                                int axis, double* __restrict__ xm) {
    const int j = (int)blockIdx.x;
    const int a1 = axis == 0 ? 1 : 0, a2 = axis == 2 ? 1 : 2;
    const long n1 = G.n[a1], n2 = G.n[a2], nl = n1 * n2;
    double s1 = 0.0, s2 = 0.0;
    for (long e = threadIdx.x; e < nl; e += blockDim.x) {
        int v[3];
        v[axis] = j;
        v[a1] = (int)(e % n1);
        v[a2] = (int)(e / n1);
        const long c = flat(G, v[0], v[1], v[2]);
        s1 += s[c] / P.rho[c];
        s2 += s[G.N + c] / P.rho[c];
    }
    __shared__ double sh[kBlock / 64];
    const double t1 = block_sum(s1, sh);
    __syncthreads();
    const double t2 = block_sum(s2, sh);
    if (threadIdx.x == 0) {
        const double m1 = t1 / (double)nl, m2 = t2 / (double)nl;
        xm[j] = 2.0 * (m1 < m2 ? m1 : m2);
    }
}

// Velocity component `axis` of cell q of state u on grid G: the mean of the
// velocities m / rho_f of its two faces along the axis (rho_f the mean of the
// two cells of a face; 0 on wall faces).
__device__ __forceinline__ double cell_velocity(const Grid& G, const double* __restrict__ u, const Ijk& q, long c,
                                                int axis) {
    const double* m = u + (long)(2 + axis) * G.N;
    const bool wall = G.bc[axis] == WALL;
    double a = 0.0, b = 0.0;
    if (!(wall && q.v[axis] == 0)) a = m[c] / (0.5 * (u[shifted(G, q, axis, -1)] + u[c]));
    if (!(wall && q.v[axis] == G.n[axis] - 1)) {
        const long cu = shifted(G, q, axis, 1);
        b = m[cu] / (0.5 * (u[c] + u[cu]));
    }
    return 0.5 * (a + b);
}

// eq. (17): per block, sum over low-resolution cells of |v_low - <v_high>|
// and of |<v_high>|, <.> the mean over the r^ND cells of the high-resolution
// grid Gh that make up the low cell (equal volumes: the volume average)
template <int ND>
__global__ void __launch_bounds__(kBlock) k_vel_error(Grid Gl, Grid Gh, const double* __restrict__ ul,
                                                      const double* __restrict__ uh, int r, int axis,
                                                      double* __restrict__ part) {
    Ijk q;
    long c = 0;
    double e = 0.0, a = 0.0;
    if (cell_from_launch(Gl, q, c)) {
        const double vl = cell_velocity(Gl, ul, q, c, axis);
        const int rz = ND > 2 ? r : 1;
        double s = 0.0;
        for (int dk = 0; dk < rz; ++dk)
            for (int dj = 0; dj < r; ++dj)
                for (int di = 0; di < r; ++di) {
                    Ijk f;
                    f.v[0] = q.v[0] * r + di;
                    f.v[1] = q.v[1] * r + dj;
                    f.v[2] = ND > 2 ? q.v[2] * r + dk : 0;
                    s += cell_velocity(Gh, uh, f, flat(Gh, f.v[0], f.v[1], f.v[2]), axis);
                }
        const double avg = s / (double)(r * r * rz);
        e = fabs(vl - avg);
        a = fabs(avg);
    }
    __shared__ double sh[kBlock / 64];
    const long nb = (long)gridDim.x * gridDim.y * gridDim.z;
    const int b = lin_block();
    double t = block_sum(e, sh);
    if (lin_thread() == 0) part[b] = t;
    __syncthreads();
    t = block_sum(a, sh);
    if (lin_thread() == 0) part[nb + b] = t;
}

void launch_vel_error(const Grid& Gl, const Grid& Gh, const double* ul, const double* uh, int r, int axis,
                      double* part, double* out2, hipStream_t stream) {
    const int nb = cell_blocks(Gl.n);
    {
        JFNK_PROF(KC_OTHER, stream);
        JFNK_LAUNCH_ND(Gl.ndim, k_vel_error, cell_grid3(Gl.n), dim3(kBx, kBy), 0, stream, Gl, Gh, ul, uh, r, axis,
                       part);
    }
    launch_final_sum(part, nb, 2, out2, stream);
}

// ---------------------------------------------------------------- allocation-free velocity error
// Workspace of jfnk_velocity_error_noalloc: the per-block partial sums of
// eq. (17) and the two final sums, in a file-scope device array of
// kNoallocScratchDoubles doubles (256 KiB).  Each GPU the library runs on
// holds its own copy until the process ends.  Host code never passes the
// array's name to a kernel or a copy: it looks up the array's address on
// each device once (hipGetSymbolAddress, with that device current) and uses
// that pointer.
static __device__ __align__(256) double scratch[kNoallocScratchDoubles];

namespace {
std::mutex g_scratch_mu;
double* g_scratch_dev[kNoallocMaxDevices] = {};
}  // namespace

std::mutex& noalloc_scratch_lock() { return g_scratch_mu; }

int noalloc_scratch(int device, double** ptr) {
    if (device < 0 || device >= kNoallocMaxDevices) return -1;
    if (!g_scratch_dev[device]) {
        void* a = nullptr;
        if (hipGetSymbolAddress(&a, HIP_SYMBOL(scratch)) != hipSuccess || !a) return -3;
        g_scratch_dev[device] = (double*)a;
    }
    *ptr = g_scratch_dev[device];
    return 0;
}

long noalloc_vel_error_doubles(const Grid& Gl) { return 2L * cell_blocks(Gl.n) + 2; }

void launch_vel_error_scratch(const Grid& Gl, const Grid& Gh, const double* ul, const double* uh, int r, int axis,
                              double* scr, hipStream_t stream) {
    const int nb = cell_blocks(Gl.n);
    launch_vel_error(Gl, Gh, ul, uh, r, axis, scr, scr + 2L * nb, stream);
}

int launch_diagnostics(const Grid& G, const Prim& P, const double* u, int axis, double rho_l, double rho_h,
                       const double* scal, double* part, double* out5, hipStream_t stream) {
    const int nb = cell_blocks(G.n);
    {
        JFNK_PROF(KC_OTHER, stream);
        JFNK_LAUNCH_ND(G.ndim, k_diag_cells, cell_grid3(G.n), dim3(kBx, kBy), 0, stream, G, P, u, part);
    }
    launch_final_sum(part, nb, 3, out5, stream);
    launch_final_max(part + 3L * nb, nb, 1, out5 + 3, stream);
    if (axis >= 0) {
        double* xm = part + 4L * nb;
        {
            JFNK_PROF(KC_OTHER, stream);
            JFNK_KLAUNCH(k_diag_layers, dim3(G.n[axis]), dim3(kBlock), 0, stream, G, P, axis, rho_l, rho_h, xm);
        }
        launch_final_sum(xm, G.n[axis], 1, out5 + 4, stream);
        if (scal) {
            {
                JFNK_PROF(KC_OTHER, stream);
                JFNK_KLAUNCH(k_diag_layers_scalars, dim3(G.n[axis]), dim3(kBlock), 0, stream, G, P, scal, axis, xm);
            }
            launch_final_sum(xm, G.n[axis], 1, out5 + 5, stream);
        }
    }
    return 0;
}

}  // namespace jfnk
