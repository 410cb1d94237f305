// Krylov vector kernels: deterministic two-stage reductions, the fused
// multi-dot / update passes of classical Gram-Schmidt applied twice (CGS2),
// basis combination and Newton update.  The basis may be stored in FP64 or
// FP32; every dot product and update is accumulated in FP64.
#include <algorithm>
#include <atomic>

#include "kernels.hpp"

namespace jfnk {

// ---------------------------------------------------------------- final reductions (one block per column, fixed order)
// host (or null): pinned host memory that receives a copy of each result, so
// that the host can read it once the kernel is done, with no copy launch;
// block 0 also copies xn earlier device results xsrc to xhost, so that one
// kernel's host stores carry a whole read-back
__global__ void __launch_bounds__(kFinalThreads) k_final_sum(const double* __restrict__ part, int nblk,
                                                             double* __restrict__ out, double* __restrict__ host,
                                                             const double* __restrict__ xsrc,
                                                             double* __restrict__ xhost, int xn) {
    __shared__ double sh[kFinalThreads / 64];
    const int col = blockIdx.x;
    double s = 0.0;
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) s += part[(long)col * nblk + i];
    const double t = block_sum(s, sh);
    if (threadIdx.x == 0) {
        out[col] = t;
        if (host) host[col] = t;
    }
    if (col == 0)
        for (int i = threadIdx.x; i < xn; i += blockDim.x) xhost[i] = xsrc[i];
}

__global__ void __launch_bounds__(kFinalThreads) k_final_max(const double* __restrict__ part, int nblk,
                                                             double* __restrict__ out) {
    __shared__ double sh[kFinalThreads / 64];
    const int col = blockIdx.x;
    double s = 0.0;
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) s = fmax(s, part[(long)col * nblk + i]);
    const double t = block_max(s, sh);
    if (threadIdx.x == 0) out[col] = t;
}

__global__ void k_put_scalar(double* __restrict__ dst, double v) {
    if (threadIdx.x == 0) dst[0] = v;
}
void launch_put_scalar(double* dst, double v, hipStream_t stream) {
    JFNK_PROF(KC_OTHER, stream);
    JFNK_KLAUNCH(k_put_scalar, dim3(1), dim3(64), 0, stream, dst, v);
}

void launch_final_sum(const double* part, int nblk, int ncol, double* out, hipStream_t stream, double* host,
                      const double* xsrc, double* xhost, int xn) {
    JFNK_PROF(KC_REDUCE, stream);
    JFNK_KLAUNCH(k_final_sum, dim3(ncol), dim3(kFinalThreads), 0, stream, part, nblk, out, host, xsrc, xhost,
                 xhost ? xn : 0);
}
void launch_final_max(const double* part, int nblk, int ncol, double* out, hipStream_t stream) {
    JFNK_PROF(KC_REDUCE, stream);
    JFNK_KLAUNCH(k_final_max, dim3(ncol), dim3(kFinalThreads), 0, stream, part, nblk, out);
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
        JFNK_KLAUNCH(k_scaled_sumsq, dim3(nblk), dim3(kBlock), 0, stream, x, G.N, 2 + G.ndim, inv, part);
    }
}

// ---------------------------------------------------------------- CGS2 passes
// Every kernel is instantiated for the exact number K of basis vectors, so
// the K loads of an element are issued together and all loops unroll.

// pass 1: h_i = V_i . w (i < K) and w . w in column K
template <typename T, int K>
__global__ void __launch_bounds__(kBlock) k_mdot(const T* __restrict__ V, long ld, const double* __restrict__ w,
                                                 long n, double* __restrict__ part) {
    double acc[K + 1];
#pragma unroll
    for (int i = 0; i <= K; ++i) acc[i] = 0.0;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        double vv[K];
#pragma unroll
        for (int i = 0; i < K; ++i) vv[i] = (double)V[(long)i * ld + e];
        const double we = w[e];
#pragma unroll
        for (int i = 0; i < K; ++i) acc[i] += vv[i] * we;
        acc[K] += we * we;
    }
    block_sum_cols<K + 1>(acc, part, (int)threadIdx.x, (long)blockIdx.x, (long)gridDim.x);
}

// passes 2 and 3: w -= sum_i h_i V_i (in order of i), then the new dots
// V_i . w (DOTS) or |w|^2 in column 0
template <typename T, int K, bool DOTS>
__global__ void __launch_bounds__(kBlock) k_update(const T* __restrict__ V, long ld, const double* __restrict__ h,
                                                   double* __restrict__ w, long n, double* __restrict__ part) {
    constexpr int NC = DOTS ? K : 1;
    double acc[NC];
    double hh[K];
#pragma unroll
    for (int i = 0; i < NC; ++i) acc[i] = 0.0;
#pragma unroll
    for (int i = 0; i < K; ++i) hh[i] = h[i];
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        double vv[K];
#pragma unroll
        for (int i = 0; i < K; ++i) vv[i] = (double)V[(long)i * ld + e];
        double we = w[e];
#pragma unroll
        for (int i = 0; i < K; ++i) we -= hh[i] * vv[i];
        w[e] = we;
        if (DOTS) {
#pragma unroll
            for (int i = 0; i < NC; ++i) acc[i] += vv[i] * we;
        } else {
            acc[0] += we * we;
        }
    }
    block_sum_cols<NC>(acc, part, (int)threadIdx.x, (long)blockIdx.x, (long)gridDim.x);
}

// t = sum_i y_i V_i, accumulated in order of i (then added to t when acc)
template <typename T, int K>
__global__ void __launch_bounds__(kBlock) k_combine(const T* __restrict__ V, long ld, const double* __restrict__ y,
                                                    double* __restrict__ t, long n, int acc) {
    double yy[K];
#pragma unroll
    for (int i = 0; i < K; ++i) yy[i] = y[i];
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        double vv[K];
#pragma unroll
        for (int i = 0; i < K; ++i) vv[i] = (double)V[(long)i * ld + e];
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < K; ++i) s += yy[i] * vv[i];
        t[e] = acc ? t[e] + s : s;
    }
}

// The final correction of a converged GMRES solve and the Newton update in
// one pass: x = sum_i y_i V_i (plus the x of earlier cycles when acc),
// u += S x and the block maxima of |S x / u| over the density entries,
// each value formed as k_combine and k_update_state form it; x itself is
// not stored (nothing reads it after the update).
template <typename T, int K>
__global__ void __launch_bounds__(kBlock) k_combine_update(const T* __restrict__ V, long ld,
                                                           const double* __restrict__ y,
                                                           const double* __restrict__ x, int acc,
                                                           double* __restrict__ u, long N, long n, Scales5 sc,
                                                           double* __restrict__ part) {
    double yy[K];
#pragma unroll
    for (int i = 0; i < K; ++i) yy[i] = y[i];
    double m = 0.0;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        double vv[K];
#pragma unroll
        for (int i = 0; i < K; ++i) vv[i] = (double)V[(long)i * ld + e];
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < K; ++i) s += yy[i] * vv[i];
        const double xe = acc ? x[e] + s : s;
        const double f = sc.v[e / N];
        const double un = u[e] + f * xe;
        u[e] = un;
        if (e < N) m = fmax(m, fabs(f * xe / un));
    }
    __shared__ double sh[kBlock / 64];
    const double t = block_max(m, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// blocks that fill the device once for a kernel (grid-stride loops take the
// rest), capped by the partial-sum capacity
template <typename Kern>
static int resident_blocks(Kern kern) {
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, kBlock, 0) != hipSuccess || per <= 0) per = 1;
    const int nb = cus * per;
    return nb > kRedBlocks ? kRedBlocks : nb;
}
// resident_blocks computed once per kernel (the library drives one device
// type; concurrent first calls compute the same value)
template <typename Kern>
static int cached_blocks(std::atomic<int>& slot, Kern kern) {
    int v = slot.load(std::memory_order_relaxed);
    if (!v) {
        v = resident_blocks(kern);
        slot.store(v, std::memory_order_relaxed);
    }
    return v;
}

#define JFNK_K_CASES(X)                                                                                    \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17) X(18) X(19) \
        X(20) X(21) X(22) X(23) X(24) X(25) X(26) X(27) X(28) X(29) X(30) X(31) X(32)

template <typename T>
int launch_mdot(const T* V, long ld, int k, const double* w, long n, double* part, hipStream_t stream) {
    JFNK_PROFB(KC_MDOT, stream, (double)n * (k * sizeof(T) + 8));
    int nblk = 1;
    switch (k) {
#define C(K)                                                                                           \
    case K: {                                                                                          \
        static std::atomic<int> nb{0};                                                                 \
        nblk = std::min(cached_blocks(nb, k_mdot<T, K>), grid_blocks(n));                              \
        JFNK_KLAUNCH((k_mdot<T, K>), dim3(nblk), dim3(kBlock), 0, stream, V, ld, w, n, part); \
        break;                                                                                         \
    }
        JFNK_K_CASES(C)
#undef C
        default:
            break;
    }
    return nblk;
}

template <typename T>
int launch_update_mdot(const T* V, long ld, int k, const double* h, double* w, long n, double* part,
                       bool want_dots, hipStream_t stream) {
    JFNK_PROFB((want_dots ? KC_UPDATE_DOT : KC_UPDATE_NORM), stream, (double)n * (k * sizeof(T) + 16));
    int nblk = 1;
    switch (k) {
#define C(K)                                                                                                      \
    case K: {                                                                                                     \
        static std::atomic<int> nbd{0}, nbn{0};                                                                   \
        if (want_dots) {                                                                                          \
            nblk = std::min(cached_blocks(nbd, k_update<T, K, true>), grid_blocks(n));                            \
            JFNK_KLAUNCH((k_update<T, K, true>), dim3(nblk), dim3(kBlock), 0, stream, V, ld, h, w, n, part); \
        } else {                                                                                                  \
            nblk = std::min(cached_blocks(nbn, k_update<T, K, false>), grid_blocks(n));                           \
            JFNK_KLAUNCH((k_update<T, K, false>), dim3(nblk), dim3(kBlock), 0, stream, V, ld, h, w, n, part); \
        }                                                                                                         \
        break;                                                                                                    \
    }
        JFNK_K_CASES(C)
#undef C
        default:
            break;
    }
    return nblk;
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
    JFNK_PROFB(KC_STORE, stream, (double)n * (8 + sizeof(T)));
    JFNK_KLAUNCH((k_store_scaled<T>), dim3(grid_blocks(n, kBlock * 4)), dim3(kBlock), 0, stream, w, v, hn, n);
}

// the same store with hn = sqrt(|w|^2) formed on the device from the sum
// the last CGS2 pass left there (the value the host forms from it)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_store_scaled_dev(const double* __restrict__ w, T* __restrict__ v,
                                                             const double* __restrict__ hnsq, long n) {
    const double hn = sqrt(hnsq[0]);
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
        v[e] = (T)(w[e] / hn);
}
template <typename T>
void launch_store_scaled_dev(const double* w, T* v, const double* hnsq, long n, hipStream_t stream) {
    JFNK_PROFB(KC_STORE, stream, (double)n * (8 + sizeof(T)));
    JFNK_KLAUNCH((k_store_scaled_dev<T>), dim3(grid_blocks(n, kBlock * 4)), dim3(kBlock), 0, stream, w, v, hnsq,
                 n);
}

template <typename T>
void launch_combine(const T* V, long ld, int k, const double* y, double* t, long n, bool acc, hipStream_t stream) {
    const int nb = grid_blocks(n, kBlock * 4);
    JFNK_PROFB(KC_COMBINE, stream, (double)n * (k * sizeof(T) + (acc ? 16 : 8)));
    switch (k) {
#define C(K)                                                                                        \
    case K:                                                                                         \
        JFNK_KLAUNCH((k_combine<T, K>), dim3(nb), dim3(kBlock), 0, stream, V, ld, y, t, n, acc ? 1 : 0); \
        break;
        JFNK_K_CASES(C)
#undef C
        default:
            break;
    }
}

template <typename T>
void launch_combine_update(const T* V, long ld, int k, const double* y, const double* x, bool acc, double* u,
                           const Grid& G, const double* scale5, double* part, int nblk, hipStream_t stream) {
    Scales5 s;
    for (int f = 0; f < 5; ++f) s.v[f] = scale5[f];
    const long n = G.nvec;
    JFNK_PROFB(KC_COMBINE, stream, (double)n * (k * sizeof(T) + (acc ? 24 : 16)));
    switch (k) {
#define C(K)                                                                                                    \
    case K:                                                                                                     \
        JFNK_KLAUNCH((k_combine_update<T, K>), dim3(nblk), dim3(kBlock), 0, stream, V, ld, y, x, acc ? 1 : 0, u, \
                     G.N, n, s, part);                                                                          \
        break;
        JFNK_K_CASES(C)
#undef C
        default:
            break;
    }
}

// ---------------------------------------------------------------- small vector kernels
// out = a + r (a - b): the state extrapolated in time from a (now) and b (one
// step back), r the ratio of the step to the previous one
__global__ void __launch_bounds__(kBlock) k_extrapolate(double* __restrict__ out, const double* __restrict__ a,
                                                        const double* __restrict__ b, double r, long n) {
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
        out[e] = a[e] + r * (a[e] - b[e]);
}
void launch_extrapolate(double* out, const double* a, const double* b, double r, long n, hipStream_t stream) {
    JFNK_PROF(KC_OTHER, stream);
    JFNK_KLAUNCH(k_extrapolate, dim3(grid_blocks(n, kBlock * 4)), dim3(kBlock), 0, stream, out, a, b, r, n);
}

__global__ void __launch_bounds__(kBlock) k_add(double* __restrict__ x, const double* __restrict__ z, long n) {
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
        x[e] += z[e];
}
void launch_add(double* x, const double* z, long n, hipStream_t stream) {
    {
        JFNK_PROF(KC_OTHER, stream);
        JFNK_KLAUNCH(k_add, dim3(grid_blocks(n, kBlock * 4)), dim3(kBlock), 0, stream, x, z, n);
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
        JFNK_KLAUNCH(k_sub, dim3(grid_blocks(n, kBlock * 4)), dim3(kBlock), 0, stream, a, b, r, n);
    }
}

__global__ void __launch_bounds__(kBlock) k_copy(double* __restrict__ d, const double* __restrict__ s, long n) {
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
        d[e] = s[e];
}
void launch_copy(double* dst, const double* src, long n, hipStream_t stream) {
    {
        JFNK_PROF(KC_OTHER, stream);
        JFNK_KLAUNCH(k_copy, dim3(grid_blocks(n, kBlock * 4)), dim3(kBlock), 0, stream, dst, src, n);
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
        JFNK_KLAUNCH(k_update_state, dim3(nblk), dim3(kBlock), 0, stream, u, x, G.N, G.nvec, s, part);
    }
}

// stored wall faces are not unknowns: force them to zero
template <int ND>
__global__ void __launch_bounds__(kBlock) k_zero_walls(double* __restrict__ u, Grid G) {
    Ijk q;
    long c;
    if (!cell_from_launch(G, q, c)) return;
    for (int d = 0; d < ND; ++d)
        if (G.bc[d] == WALL && q.v[d] == 0) u[(long)(2 + d) * G.N + c] = 0.0;
}
void launch_zero_walls(double* u, const Grid& G, hipStream_t stream) {
    if (!G.has_wall) return;
    {
        JFNK_PROF(KC_OTHER, stream);
        JFNK_LAUNCH_ND(G.ndim, k_zero_walls, cell_grid3(G.n), dim3(kBx, kBy), 0, stream, u, G);
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
        JFNK_KLAUNCH(k_sum, dim3(nblk), dim3(kBlock), 0, stream, x, n, part);
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
        JFNK_KLAUNCH((k_widen<T>), dim3(grid_blocks(n, kBlock * 4)), dim3(kBlock), 0, stream, v, out, n);
    }
}

// explicit instantiations
template void launch_widen<double>(const double*, double*, long, hipStream_t);
template void launch_widen<float>(const float*, double*, long, hipStream_t);
template int launch_mdot<double>(const double*, long, int, const double*, long, double*, hipStream_t);
template int launch_mdot<float>(const float*, long, int, const double*, long, double*, hipStream_t);
template int launch_update_mdot<double>(const double*, long, int, const double*, double*, long, double*, bool,
                                        hipStream_t);
template int launch_update_mdot<float>(const float*, long, int, const double*, double*, long, double*, bool,
                                       hipStream_t);
template void launch_store_scaled<double>(const double*, double*, double, long, hipStream_t);
template void launch_store_scaled<float>(const double*, float*, double, long, hipStream_t);
template void launch_store_scaled_dev<double>(const double*, double*, const double*, long, hipStream_t);
template void launch_store_scaled_dev<float>(const double*, float*, const double*, long, hipStream_t);
template void launch_combine<double>(const double*, long, int, const double*, double*, long, bool, hipStream_t);
template void launch_combine<float>(const float*, long, int, const double*, double*, long, bool, hipStream_t);
template void launch_combine_update<double>(const double*, long, int, const double*, const double*, bool, double*,
                                            const Grid&, const double*, double*, int, hipStream_t);
template void launch_combine_update<float>(const float*, long, int, const double*, const double*, bool, double*,
                                           const Grid&, const double*, double*, int, hipStream_t);

}  // namespace jfnk
