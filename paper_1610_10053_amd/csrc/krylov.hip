// Krylov vector kernels: deterministic two-stage reductions, the fused
// multi-dot / update passes of classical Gram-Schmidt applied twice (CGS2),
// basis combination and Newton update.  The basis may be stored in FP64 or
// FP32; every dot product and update is accumulated in FP64.
#include "kernels.hpp"

namespace jfnk {

// ---------------------------------------------------------------- final reductions (single block, fixed order)
__global__ void __launch_bounds__(kBlock) k_final_sum(const double* __restrict__ part, int nblk, int ncol,
                                                      double* __restrict__ out) {
    __shared__ double sh[kBlock / 64];
    for (int col = 0; col < ncol; ++col) {
        double s = 0.0;
        for (int i = threadIdx.x; i < nblk; i += blockDim.x) s += part[(long)col * nblk + i];
        const double t = block_sum(s, sh);
        if (threadIdx.x == 0) out[col] = t;
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kBlock) k_final_max(const double* __restrict__ part, int nblk, int ncol,
                                                      double* __restrict__ out) {
    __shared__ double sh[kBlock / 64];
    for (int col = 0; col < ncol; ++col) {
        double s = 0.0;
        for (int i = threadIdx.x; i < nblk; i += blockDim.x) s = fmax(s, part[(long)col * nblk + i]);
        const double t = block_max(s, sh);
        if (threadIdx.x == 0) out[col] = t;
        __syncthreads();
    }
}

void launch_final_sum(const double* part, int nblk, int ncol, double* out, hipStream_t stream) {
    {
        JFNK_PROF(KC_REDUCE, stream);
        hipLaunchKernelGGL(k_final_sum, dim3(1), dim3(kBlock), 0, stream, part, nblk, ncol, out);
    }
}
void launch_final_max(const double* part, int nblk, int ncol, double* out, hipStream_t stream) {
    {
        JFNK_PROF(KC_REDUCE, stream);
        hipLaunchKernelGGL(k_final_max, dim3(1), dim3(kBlock), 0, stream, part, nblk, ncol, out);
    }
}

// ---------------------------------------------------------------- sum of (x/S)^2 over a state-shaped vector
__global__ void __launch_bounds__(kBlock) k_scaled_sumsq(const double* __restrict__ x, long N, int nv,
                                                         Scales5 inv, double* __restrict__ part) {
    double s = 0.0;
    const long n = N * nv;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        const double t = x[e] * inv.v[e / N];
        s += t * t;
    }
    __shared__ double sh[kBlock / 64];
    const double t = block_sum(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

void launch_scaled_sumsq(const double* x, const Grid& G, const double* inv_scale5, double* part, int nblk,
                         hipStream_t stream) {
    Scales5 inv;
    for (int f = 0; f < 5; ++f) inv.v[f] = inv_scale5 ? inv_scale5[f] : 1.0;
    {
        JFNK_PROF(KC_REDUCE, stream);
        hipLaunchKernelGGL(k_scaled_sumsq, dim3(nblk), dim3(kBlock), 0, stream, x, G.N, 2 + G.ndim, inv, part);
    }
}

// ---------------------------------------------------------------- CGS2 passes
// pass 1: h_i = V_i . w (i < k) and w . w in column k
template <typename T, int KMAX>
__global__ void __launch_bounds__(kBlock) k_mdot(const T* __restrict__ V, long ld, int k,
                                                 const double* __restrict__ w, long n,
                                                 double* __restrict__ part) {
    double acc[KMAX + 1];
#pragma unroll
    for (int i = 0; i <= KMAX; ++i) acc[i] = 0.0;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        const double we = w[e];
#pragma unroll
        for (int i = 0; i < KMAX; ++i)
            if (i < k) acc[i] += (double)V[(long)i * ld + e] * we;
        acc[KMAX] += we * we;
    }
    __shared__ double sh[kBlock / 64];
#pragma unroll
    for (int i = 0; i <= KMAX; ++i) {
        if (i < k || i == KMAX) {
            const double t = block_sum(acc[i], sh);
            const int col = i == KMAX ? k : i;
            if (threadIdx.x == 0) part[(long)col * gridDim.x + blockIdx.x] = t;
        }
    }
}

// passes 2 and 3: w -= sum_i h_i V_i (in order of i), then either the new
// dots V_i . w (column i) or |w|^2 (column 0)
template <typename T, int KMAX>
__global__ void __launch_bounds__(kBlock) k_update_mdot(const T* __restrict__ V, long ld, int k,
                                                        const double* __restrict__ h,
                                                        double* __restrict__ w, long n,
                                                        double* __restrict__ part, int want_dots) {
    double acc[KMAX];
    double hh[KMAX];
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
        acc[i] = 0.0;
        hh[i] = i < k ? h[i] : 0.0;
    }
    double nrm = 0.0;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        double vv[KMAX];
        double we = w[e];
#pragma unroll
        for (int i = 0; i < KMAX; ++i) {
            if (i < k) {
                vv[i] = (double)V[(long)i * ld + e];
                we -= hh[i] * vv[i];
            }
        }
        w[e] = we;
        if (want_dots) {
#pragma unroll
            for (int i = 0; i < KMAX; ++i)
                if (i < k) acc[i] += vv[i] * we;
        } else {
            nrm += we * we;
        }
    }
    __shared__ double sh[kBlock / 64];
    if (want_dots) {
#pragma unroll
        for (int i = 0; i < KMAX; ++i) {
            if (i < k) {
                const double t = block_sum(acc[i], sh);
                if (threadIdx.x == 0) part[(long)i * gridDim.x + blockIdx.x] = t;
            }
        }
    } else {
        const double t = block_sum(nrm, sh);
        if (threadIdx.x == 0) part[blockIdx.x] = t;
    }
}

template <typename T>
void launch_mdot(const T* V, long ld, int k, const double* w, long n, double* part, int nblk,
                 hipStream_t stream) {
    JFNK_PROFB(KC_MDOT, stream, (double)n * (k * sizeof(T) + 8));
    if (k <= 8)
        hipLaunchKernelGGL((k_mdot<T, 8>), dim3(nblk), dim3(kBlock), 0, stream, V, ld, k, w, n, part);
    else if (k <= 16)
        hipLaunchKernelGGL((k_mdot<T, 16>), dim3(nblk), dim3(kBlock), 0, stream, V, ld, k, w, n, part);
    else if (k <= 32)
        hipLaunchKernelGGL((k_mdot<T, 32>), dim3(nblk), dim3(kBlock), 0, stream, V, ld, k, w, n, part);
    else
        hipLaunchKernelGGL((k_mdot<T, 64>), dim3(nblk), dim3(kBlock), 0, stream, V, ld, k, w, n, part);
}

template <typename T>
void launch_update_mdot(const T* V, long ld, int k, const double* h, double* w, long n, double* part,
                        int nblk, bool want_dots, hipStream_t stream) {
    const int wd = want_dots ? 1 : 0;
    JFNK_PROFB((wd ? KC_UPDATE_DOT : KC_UPDATE_NORM), stream, (double)n * (k * sizeof(T) + 16));
    if (k <= 8)
        hipLaunchKernelGGL((k_update_mdot<T, 8>), dim3(nblk), dim3(kBlock), 0, stream, V, ld, k, h, w, n, part, wd);
    else if (k <= 16)
        hipLaunchKernelGGL((k_update_mdot<T, 16>), dim3(nblk), dim3(kBlock), 0, stream, V, ld, k, h, w, n, part, wd);
    else if (k <= 32)
        hipLaunchKernelGGL((k_update_mdot<T, 32>), dim3(nblk), dim3(kBlock), 0, stream, V, ld, k, h, w, n, part, wd);
    else
        hipLaunchKernelGGL((k_update_mdot<T, 64>), dim3(nblk), dim3(kBlock), 0, stream, V, ld, k, h, w, n, part, wd);
}

// v = w / hn (rounded to the basis type)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_store_scaled(const double* __restrict__ w, T* __restrict__ v,
                                                         double hn, long n) {
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
        v[e] = (T)(w[e] / hn);
}

template <typename T>
void launch_store_scaled(const double* w, T* v, double hn, long n, hipStream_t stream) {
    {
        JFNK_PROFB(KC_STORE, stream, (double)n * (8 + sizeof(T)));
        hipLaunchKernelGGL((k_store_scaled<T>), dim3(grid_blocks(n, kBlock * 4)), dim3(kBlock), 0, stream, w, v, hn, n);
    }
}

// t = sum_i y_i V_i, accumulated in order of i
template <typename T, int KMAX>
__global__ void __launch_bounds__(kBlock) k_combine(const T* __restrict__ V, long ld, int k,
                                                    const double* __restrict__ y, double* __restrict__ t,
                                                    long n) {
    double yy[KMAX];
#pragma unroll
    for (int i = 0; i < KMAX; ++i) yy[i] = i < k ? y[i] : 0.0;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < KMAX; ++i)
            if (i < k) s += yy[i] * (double)V[(long)i * ld + e];
        t[e] = s;
    }
}

template <typename T>
void launch_combine(const T* V, long ld, int k, const double* y, double* t, long n, hipStream_t stream) {
    const int nb = grid_blocks(n, kBlock * 4);
    JFNK_PROFB(KC_COMBINE, stream, (double)n * (k * sizeof(T) + 8));
    if (k <= 8)
        hipLaunchKernelGGL((k_combine<T, 8>), dim3(nb), dim3(kBlock), 0, stream, V, ld, k, y, t, n);
    else if (k <= 16)
        hipLaunchKernelGGL((k_combine<T, 16>), dim3(nb), dim3(kBlock), 0, stream, V, ld, k, y, t, n);
    else if (k <= 32)
        hipLaunchKernelGGL((k_combine<T, 32>), dim3(nb), dim3(kBlock), 0, stream, V, ld, k, y, t, n);
    else
        hipLaunchKernelGGL((k_combine<T, 64>), dim3(nb), dim3(kBlock), 0, stream, V, ld, k, y, t, n);
}

// ---------------------------------------------------------------- small vector kernels
__global__ void __launch_bounds__(kBlock) k_add(double* __restrict__ x, const double* __restrict__ z, long n) {
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
        x[e] += z[e];
}
void launch_add(double* x, const double* z, long n, hipStream_t stream) {
    {
        JFNK_PROF(KC_OTHER, stream);
        hipLaunchKernelGGL(k_add, dim3(grid_blocks(n, kBlock * 4)), dim3(kBlock), 0, stream, x, z, n);
    }
}

__global__ void __launch_bounds__(kBlock) k_neg_scaled(const double* __restrict__ F, double* __restrict__ r,
                                                       long N, long n, Scales5 s) {
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
        r[e] = -F[e] / s.v[e / N];
}
void launch_neg_scaled(const double* F, double* r, const Grid& G, const double* scale5, hipStream_t stream) {
    Scales5 s;
    for (int f = 0; f < 5; ++f) s.v[f] = scale5[f];
    {
        JFNK_PROF(KC_OTHER, stream);
        hipLaunchKernelGGL(k_neg_scaled, dim3(grid_blocks(G.nvec, kBlock * 4)), dim3(kBlock), 0, stream, F, r, G.N,
                           G.nvec, s);
    }
}

__global__ void __launch_bounds__(kBlock) k_sub(const double* __restrict__ a, const double* __restrict__ b,
                                                double* __restrict__ r, long n) {
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
        r[e] = a[e] - b[e];
}
void launch_sub(const double* a, const double* b, double* r, long n, hipStream_t stream) {
    {
        JFNK_PROF(KC_OTHER, stream);
        hipLaunchKernelGGL(k_sub, dim3(grid_blocks(n, kBlock * 4)), dim3(kBlock), 0, stream, a, b, r, n);
    }
}

__global__ void __launch_bounds__(kBlock) k_copy(double* __restrict__ d, const double* __restrict__ s, long n) {
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
        d[e] = s[e];
}
void launch_copy(double* dst, const double* src, long n, hipStream_t stream) {
    {
        JFNK_PROF(KC_OTHER, stream);
        hipLaunchKernelGGL(k_copy, dim3(grid_blocks(n, kBlock * 4)), dim3(kBlock), 0, stream, dst, src, n);
    }
}

// u += S x, with the largest relative density correction |S_rho x / u_new|
__global__ void __launch_bounds__(kBlock) k_update_state(double* __restrict__ u, const double* __restrict__ x,
                                                         long N, long n, Scales5 s, double* __restrict__ part) {
    double m = 0.0;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        const double sc = s.v[e / N];
        const double un = u[e] + sc * x[e];
        u[e] = un;
        if (e < N) m = fmax(m, fabs(sc * x[e] / un));
    }
    __shared__ double sh[kBlock / 64];
    const double t = block_max(m, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}
void launch_update_state(double* u, const double* x, const Grid& G, const double* scale5, double* part,
                         int nblk, hipStream_t stream) {
    Scales5 s;
    for (int f = 0; f < 5; ++f) s.v[f] = scale5[f];
    {
        JFNK_PROF(KC_OTHER, stream);
        hipLaunchKernelGGL(k_update_state, dim3(nblk), dim3(kBlock), 0, stream, u, x, G.N, G.nvec, s, part);
    }
}

// stored wall faces are not unknowns: force them to zero
__global__ void __launch_bounds__(kBlock) k_zero_walls(double* __restrict__ u, Grid G) {
    Ijk q;
    long c;
    if (!cell_from_launch(G, q, c)) return;
    for (int d = 0; d < G.ndim; ++d)
        if (G.bc[d] == WALL && q.v[d] == 0) u[(long)(2 + d) * G.N + c] = 0.0;
}
void launch_zero_walls(double* u, const Grid& G, hipStream_t stream) {
    if (!G.has_wall) return;
    {
        JFNK_PROF(KC_OTHER, stream);
        hipLaunchKernelGGL(k_zero_walls, cell_grid3(G.n), dim3(kBx, kBy), 0, stream, u, G);
    }
}

// plain sum of a vector (per-block partials)
__global__ void __launch_bounds__(kBlock) k_sum(const double* __restrict__ x, long n, double* __restrict__ part) {
    double s = 0.0;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) s += x[e];
    __shared__ double sh[kBlock / 64];
    const double t = block_sum(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}
void launch_sum(const double* x, long n, double* part, int nblk, hipStream_t stream) {
    {
        JFNK_PROF(KC_REDUCE, stream);
        hipLaunchKernelGGL(k_sum, dim3(nblk), dim3(kBlock), 0, stream, x, n, part);
    }
}

// basis vector to FP64
template <typename T>
__global__ void __launch_bounds__(kBlock) k_widen(const T* __restrict__ v, double* __restrict__ out, long n) {
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
        out[e] = (double)v[e];
}
template <typename T>
void launch_widen(const T* v, double* out, long n, hipStream_t stream) {
    {
        JFNK_PROF(KC_OTHER, stream);
        hipLaunchKernelGGL((k_widen<T>), dim3(grid_blocks(n, kBlock * 4)), dim3(kBlock), 0, stream, v, out, n);
    }
}

// explicit instantiations
template void launch_widen<double>(const double*, double*, long, hipStream_t);
template void launch_widen<float>(const float*, double*, long, hipStream_t);
template void launch_mdot<double>(const double*, long, int, const double*, long, double*, int, hipStream_t);
template void launch_mdot<float>(const float*, long, int, const double*, long, double*, int, hipStream_t);
template void launch_update_mdot<double>(const double*, long, int, const double*, double*, long, double*, int,
                                         bool, hipStream_t);
template void launch_update_mdot<float>(const float*, long, int, const double*, double*, long, double*, int,
                                        bool, hipStream_t);
template void launch_store_scaled<double>(const double*, double*, double, long, hipStream_t);
template void launch_store_scaled<float>(const double*, float*, double, long, hipStream_t);
template void launch_combine<double>(const double*, long, int, const double*, double*, long, hipStream_t);
template void launch_combine<float>(const float*, long, int, const double*, double*, long, hipStream_t);

}  // namespace jfnk
