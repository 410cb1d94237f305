// Internal definitions shared by the HIP kernels and the host driver of the
// implicit-step library.  Grid geometry, boundary handling and the small
// device helpers (limiter, upstream extrapolation, reductions).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cstddef>
#include <cstdint>

namespace jfnk {

constexpr int kBlock = 256;        // threads per block of the sweep kernels
constexpr int kMaxRestart = 32;    // largest Krylov basis
constexpr int kRedBlocks = 2048;   // most blocks of a multi-dot reduction

enum Bc : int { PERIODIC = 0, WALL = 1 };

// Metric tables of a 2D spherical grid (axis 0 = radius r, axis 1 =
// colatitude theta, azimuthal symmetry), in device memory, per radial index i
// and colatitude index j, per radian of azimuth:
//   Vr[i] = (r_{i+1/2}^3 - r_{i-1/2}^3)/3, Vt[j] = cos th_{j-1/2} - cos th_{j+1/2}
//     (cell volume Vr Vt);
//   r2f[i] = r_{i-1/2}^2 (lower r-face area r2f Vt), rfa[i] = r_{i-1/2};
//   hr2[i] = (r_{i+1/2}^2 - r_{i-1/2}^2)/2, stf[j] = sin th_{j-1/2}
//     (lower theta-face area hr2 stf);
//   rc[i] cell-centre radius, ith[i] = 1/(rc[i] dth);
//   momentum control volumes: Vrc[i] = (rc_i^3 - rc_{i-1}^3)/3,
//   r2c[i] = rc_i^2, hr2c[i] = (rc_i^2 - rc_{i-1}^2)/2,
//   Vtc[j] = cos thc_{j-1} - cos thc_j, stc[j] = sin thc_j.
struct SphMet {
    const double *Vr, *rc, *ith, *hr2, *Vrc, *r2c, *hr2c, *r2f, *rfa;
    const double *Vt, *Vtc, *stc, *stf;
};

// Geometry and physics constants passed by value to every kernel.
struct Grid {
    int ndim;
    int n[3];
    int bc[3];
    long N;          // cells
    long nvec;       // (2 + ndim) * N
    long stride[3];  // 1, n0, n0*n1
    double dx[3], idx[3];
    double gamma, gm1, g[3], chi0;
    int heat_balance;
    int has_wall, has_chi;
    int internal;  // energy variable rho e (eq. 2 as written) instead of E
    int sph;       // 2D spherical geometry (metric tables M)
    SphMet M;
};

// inverse distance between the centres of the two cells of a lower face
// along d in radial row i (r dtheta along theta on spherical grids)
__device__ __forceinline__ double face_ids(const Grid& G, int d, int i) {
    return (G.sph && d == 1) ? G.M.ith[i] : G.idx[d];
}
// spherical cell volume and lower-face area along d of cell (i, j) (i may
// be n0 and j n1 for the upper wall faces)
__device__ __forceinline__ double sph_vol(const Grid& G, int i, int j) { return G.M.Vr[i] * G.M.Vt[j]; }
__device__ __forceinline__ double sph_area(const Grid& G, int d, int i, int j) {
    return d == 0 ? G.M.r2f[i] * G.M.Vt[j] : G.M.hr2[i] * G.M.stf[j];
}

// Cell coordinates from a flat index.
struct Ijk {
    int v[3];
};

__device__ __forceinline__ Ijk cell_coords(const Grid& G, long c) {
    Ijk r;
    r.v[0] = (int)(c % G.n[0]);
    long t = c / G.n[0];
    r.v[1] = (int)(t % G.n[1]);
    r.v[2] = (int)(t / G.n[1]);
    return r;
}

// cell indices fit in 32 bits (checked at creation)
__device__ __forceinline__ long flat(const Grid& G, int i, int j, int k) {
    return (long)(i + G.n[0] * (j + G.n[1] * k));
}

// 3D launches of the cell sweeps: blocks of kBx x kBy threads (one wave per
// row of kBx), grid (ceil(n0/kBx), ceil(n1/kBy), n2)
constexpr int kBx = 64, kBy = 4;
// threads of the single-workgroup final reductions (one workgroup per column)
constexpr int kFinalThreads = 1024;
inline dim3 cell_grid3(const int n[3]) { return dim3((n[0] + kBx - 1) / kBx, (n[1] + kBy - 1) / kBy, n[2]); }
inline int cell_blocks(const int n[3]) {
    const dim3 g = cell_grid3(n);
    return (int)(g.x * g.y * g.z);
}
// XCD-aware tile order.  The device hands the workgroups of a launch to its
// 8 XCDs round-robin by flattened id, and each XCD has its own L2.  The
// logical tile of a workgroup is chosen so that XCD x walks one contiguous
// range of tiles (a slab of whole rows and planes): the halo rows and planes
// a stencil reads are mostly tiles of the same XCD, found in its L2.
constexpr unsigned kXcds = 8;
struct Tile {
    unsigned x, y, z, id;
};
__device__ __forceinline__ Tile xcd_tile() {
    const unsigned gx = gridDim.x, gy = gridDim.y;
    const unsigned total = gx * gy * gridDim.z;
    const unsigned hw = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const unsigned q = total / kXcds, r = total % kXcds;
    const unsigned xcd = hw % kXcds, slot = hw / kXcds;
    Tile t;
    t.id = xcd * q + (xcd < r ? xcd : r) + slot;
    t.x = t.id % gx;
    const unsigned rest = t.id / gx;
    t.y = rest % gy;
    t.z = rest / gy;
    return t;
}
__device__ __forceinline__ bool cell_from_launch(const Grid& G, Ijk& q, long& c) {
    const Tile t = xcd_tile();
    q.v[0] = (int)(t.x * kBx + threadIdx.x);
    q.v[1] = (int)(t.y * kBy + threadIdx.y);
    q.v[2] = (int)t.z;
    if (q.v[0] >= G.n[0] || q.v[1] >= G.n[1]) return false;
    c = flat(G, q.v[0], q.v[1], q.v[2]);
    return true;
}
// per-block sums of K columns with one barrier: wave shuffles, then one
// thread per column adds the waves' values in a fixed order; t is the
// thread's linear index in its block (waves are 64 consecutive t), and the
// sums go to part[col * nblk + blk]
template <int K>
__device__ __forceinline__ void block_sum_cols(double (&acc)[K], double* __restrict__ part, int t, long blk,
                                               long nblk) {
    __shared__ double sh[(kBlock / 64) * K];
#pragma unroll
    for (int i = 0; i < K; ++i)
        for (int o = 32; o > 0; o >>= 1) acc[i] += __shfl_down(acc[i], o, 64);
    const int lane = t & 63, wv = t >> 6;
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < K; ++i) sh[wv * K + i] = acc[i];
    }
    __syncthreads();
    if (t < K) {
        double s = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) s += sh[w * K + t];
        part[(long)t * nblk + blk] = s;
    }
}
// index of a workgroup's partial result (its logical tile)
__device__ __forceinline__ int lin_block() { return (int)xcd_tile().id; }
__device__ __forceinline__ int lin_thread() { return (int)(threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z)); }

// Flat index of the cell shifted by s along axis d, with periodic wrap.
// The caller guarantees the shift stays inside along a wall axis.
__device__ __forceinline__ long shifted(const Grid& G, const Ijk& q, int d, int s) {
    int a = q.v[d] + s;
    const int n = G.n[d];
    if (a < 0) a += n;
    else if (a >= n) a -= n;
    return flat(G, d == 0 ? a : q.v[0], d == 1 ? a : q.v[1], d == 2 ? a : q.v[2]);
}

// Index of the transverse position of a wall-normal axis d (for the frozen
// wall-flux arrays): r1 = (d+1)%3 fastest.
__device__ __forceinline__ long transverse(const Grid& G, const Ijk& q, int d) {
    const int r1 = (d + 1) % 3, r2 = (d + 2) % 3;
    return (long)q.v[r1] + (long)G.n[r1] * (long)q.v[r2];
}

// van Leer's harmonic limiter of two one-sided differences.
__device__ __forceinline__ double van_leer(double a, double b) {
    const double ab = a * b;
    return ab > 0.0 ? (ab + ab) / (a + b) : 0.0;
}

// Upstream linear extrapolation: operands are selected first and then one
// shared expression is evaluated, so that mirror-image faces give
// mirror-image values bit for bit.
__device__ __forceinline__ double upstream(double vel, double ql, double sl, double qr, double sr) {
    const bool left = vel >= 0.0;
    const double qu = left ? ql : qr;
    const double su = left ? 0.5 * sl : -0.5 * sr;
    return qu + su;
}

// Block-wide sum of one double per thread (kBlock threads, wave64).
// Fixed reduction order, so results are reproducible run to run.
__device__ __forceinline__ double block_sum(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int t = lin_thread();
    const int lane = t & 63, wv = t >> 6;
    const int nw = (int)(blockDim.x * blockDim.y * blockDim.z) >> 6;
    __syncthreads();
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    double s = 0.0;
    if (t == 0) {
        for (int w = 0; w < nw; ++w) s += sh[w];
    }
    return s;  // valid in thread 0
}

__device__ __forceinline__ double block_max(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    const int t = lin_thread();
    const int lane = t & 63, wv = t >> 6;
    const int nw = (int)(blockDim.x * blockDim.y * blockDim.z) >> 6;
    __syncthreads();
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    double s = 0.0;
    if (t == 0) {
        s = sh[0];
        for (int w = 1; w < nw; ++w) s = fmax(s, sh[w]);
    }
    return s;
}

// launch a kernel templated on the number of dimensions (2 or 3), so that
// every loop over axes unrolls and all axis indices are compile-time
#define JFNK_LAUNCH_ND(ndim, kern, ...)                                   \
    do {                                                                  \
        if ((ndim) == 3) JFNK_KLAUNCH((kern<3>), __VA_ARGS__);           \
        else JFNK_KLAUNCH((kern<2>), __VA_ARGS__);                        \
    } while (0)
#define JFNK_LAUNCH_RND(ndim, kern, R, ...)                               \
    do {                                                                  \
        if ((ndim) == 3) JFNK_KLAUNCH((kern<R, 3>), __VA_ARGS__);        \
        else JFNK_KLAUNCH((kern<R, 2>), __VA_ARGS__);                     \
    } while (0)

inline int grid_blocks(long n, int block = kBlock) {
    long b = (n + block - 1) / block;
    return (int)(b < 1 ? 1 : b);
}

}  // namespace jfnk

// ---------------------------------------------------------------- kernel-class timing with HIP events
// When a problem has profiling enabled, its API calls install a profiler;
// launchers record an event pair around each launch of a selected class on
// the launch stream.  Completed pairs are drained at the host's existing
// synchronisation points, so profiling adds no synchronisation.
#include <vector>
namespace jfnk {
enum KClass : int {
    KC_PRIM = 0, KC_FLUX, KC_MFLUX, KC_OUT, KC_MDOT, KC_UPDATE_DOT, KC_UPDATE_NORM, KC_STORE, KC_COMBINE,
    KC_MG_SMOOTH, KC_MG_RESTRICT, KC_MG_PROLONG, KC_MG_COARSE, KC_PC_RHS, KC_PC_BACK, KC_PC_BUILD,
    KC_REDUCE, KC_LINES, KC_OTHER, KC_COUNT
};
struct Profiler {
    unsigned mask = 0;
    // sampling: with burst == 1, one launch in every `period` of each selected
    // class is timed; with burst > 1, windows of `burst` consecutive launches
    // (of any class) carry events, and the selected classes' launches in a
    // window after its first one are counted, so each counted kernel follows
    // a kernel that carried events too.  Outside a window each launch opens
    // one with probability 1/period, drawn from a fixed 64-bit linear
    // congruential sequence, so the windows do not alias with the periodic
    // launch pattern of the solver.
    unsigned period = 1, burst = 1;
    long long seen[KC_COUNT] = {};   // launches of each selected class so far
    unsigned left = 0;               // launches left in the open window
    unsigned long long lcg = 0;      // state of the window draw
    std::vector<hipEvent_t> pool;
    std::vector<int> cls;  // class of each recorded pair
    size_t used = 0;       // events in use (2 per pair)
    double ms[KC_COUNT] = {};
    long long count[KC_COUNT] = {};
    double bytes[KC_COUNT] = {};  // compulsory bytes of the timed launches
    std::vector<double> pend;     // bytes of each recorded pair
    // arm an event pair for the next launch of class c (b: its bytes)
    void begin(int c, double b);
    void withdraw();  // drop the most recent pair
    void drain();  // caller has synchronised the stream
    void release();
};
extern thread_local Profiler* g_prof;
// Event pair armed for the next kernel launch on this thread: the launch
// macros attach it to the dispatch itself (hipExtLaunchKernelGGL), so it
// brackets exactly the kernel's execution.
extern thread_local hipEvent_t g_ev_start, g_ev_stop;

struct ProfScope {
    bool armed = false;
    explicit ProfScope(int c, double b = 0.0) {
        if (!g_prof || !g_prof->mask) return;
        const bool sel = (g_prof->mask >> c & 1u) != 0;
        if (g_prof->burst <= 1) {
            if (sel && (g_prof->seen[c]++ % g_prof->period) == 0) {
                g_prof->begin(c, b);
                armed = g_ev_start != nullptr;
            }
            return;
        }
        if (g_prof->left == 0) {
            g_prof->lcg = g_prof->lcg * 6364136223846793005ULL + 1442695040888963407ULL;
            if ((g_prof->lcg >> 33) % g_prof->period == 0) g_prof->left = g_prof->burst;
        }
        if (g_prof->left > 0) {
            const bool opening = g_prof->left == g_prof->burst;
            g_prof->left--;
            g_prof->begin(sel && !opening ? c : -1, b);  // -1: events only, not counted
            armed = g_ev_start != nullptr;
        }
    }
    ~ProfScope() {
        // a pair no launch consumed is withdrawn (its events were never recorded)
        if (armed && g_ev_start && g_prof) g_prof->withdraw();
        g_ev_start = g_ev_stop = nullptr;
    }
};
}  // namespace jfnk
#define JFNK_CAT2(a, b) a##b
#define JFNK_CAT(a, b) JFNK_CAT2(a, b)
#define JFNK_PROF(cls, stream) ::jfnk::ProfScope JFNK_CAT(prof_scope_, __LINE__)((cls))
#define JFNK_PROFB(cls, stream, b) ::jfnk::ProfScope JFNK_CAT(prof_scope_, __LINE__)((cls), (double)(b))
// kernel launch carrying the armed event pair, if any (then disarmed)
// A launch that carries timing events goes through hipExtLaunchKernelGGL
// (events on the dispatch itself); every other launch is a plain one, which
// stream capture records into a graph.
#define JFNK_KLAUNCH(kern, grid, block, shm, stream, ...)                                              \
    do {                                                                                              \
        hipEvent_t jfnk_es_ = ::jfnk::g_ev_start, jfnk_ee_ = ::jfnk::g_ev_stop;                       \
        ::jfnk::g_ev_start = ::jfnk::g_ev_stop = nullptr;                                             \
        if (jfnk_es_ || jfnk_ee_)                                                                     \
            hipExtLaunchKernelGGL(kern, grid, block, shm, stream, jfnk_es_, jfnk_ee_, 0u, __VA_ARGS__); \
        else                                                                                          \
            hipLaunchKernelGGL(kern, grid, block, shm, stream, __VA_ARGS__);                         \
    } while (0)
