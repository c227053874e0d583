// NFFT fast summation of a Gaussian kernel (Algorithm 1, Sec. 4):
//   W~ v ~= A diag(b^) A* v,  A = (exp(2 pi i l.x_j)), l in {-N/2..N/2}^d.
//
// Plan (once per layer):
//   torus scaling   x -> s (x - c) with ||s (x - c)|| <= 1/4 - eps_B/2, so every
//                   pair distance stays where the regularised kernel equals K;
//                   sigma -> s sigma (Alg. 1 input domain).
//   grid coords     u = (x_scaled + 1/2) * 2N lies in (N/2, 3N/2): a window of
//                   support w with bin + w/2 <= N/2 never wraps around the grid.
//   bin sort        points sorted by the grid cell of u, grouped in bins of
//                   B^d cells (rocPRIM radix sort); each bin's points are cut
//                   into tasks of at most 256 points.
//   coefficients    b^_l = N^-d sum_{k in I_N} K_R(k/N) exp(-2 pi i l.k/N)
//                   (the kernel's Fourier coefficients, computed by sampling
//                   the regularised kernel and a d-dimensional DFT), FP64.
//   multipliers     M_l = b^_l / prod_t psi^(l_t/2N)^2 for |l_t| <= N/2, 0
//                   elsewhere, with weight 1/2 per coordinate at |l_t| = N/2
//                   (the real part of the sum over I_N).  psi^ is the window's
//                   Fourier transform by Gauss-Legendre quadrature.
//
// Apply (per block of vectors z, stride bs, in node order; the kernels walk
// the points in bin order through the permutation; no atomics):
//   spread   one wavefront per task: the bin's patch (the union of its
//            points' window footprints) accumulates psi(u_p - k) z_p over the
//            task's points (matrix cores for FP32 blocks of 16, registers
//            otherwise);
//   reduce   bins cut into several tasks: task patches summed in task order;
//   gather   one thread per grid cell: sum over the bins whose patch covers
//            the cell (bin order), via a dense bin table and a coarse
//            occupancy map that skips empty neighbourhoods;
//   FFT      forward complex FFT (two real vectors per complex lane), times M,
//            inverse FFT (Alg. 1 steps 1-3; deconvolution folded into M);
//   interp   one thread per point: f_p = sum over its window footprint of
//            psi(u_p - k) h_k.
#include <cmath>
#include <cstring>
#include <type_traits>

#include <numeric>
#include <queue>

#include "internal.h"

#include <rocprim/rocprim.hpp>

namespace mlg {

constexpr int kMaxP = 20;          // patch edge limit (B + w - 1)
constexpr int kWaves = 4;
constexpr int kGL = 256;           // quadrature nodes for the window transform

// ------------------------------------------------------------------------------
// device helpers
// ------------------------------------------------------------------------------
template <class T>
__device__ inline T dexp(T a);
template <>
__device__ inline float dexp<float>(float a) { return __expf(a); }
template <>
__device__ inline double dexp<double>(double a) { return exp(a); }

// Exponential-of-semicircle window in grid units, support |t| <= w/2:
// psi(t) = exp(beta (sqrt(1 - (2t/w)^2) - 1)).  The FP32 form uses the
// hardware square root and base-2 exponential (about 1 ulp each): the
// relative error of a weight stays near 1e-7, far below the FP32 gate.
template <class T>
__device__ inline T es_psi(T t, T two_over_w, T beta) {
    T z = t * two_over_w;
    T s = T(1) - z * z;
    s = s > T(0) ? s : T(0);
    return dexp<T>(beta * (sqrt(s) - T(1)));
}
template <>
__device__ inline float es_psi<float>(float t, float two_over_w, float beta) {
    const float z = t * two_over_w;
    const float s = fmaxf(fmaf(-z, z, 1.0f), 0.0f);
    const float bl = beta * 1.44269504088896341f;   // beta log2(e)
    return __builtin_amdgcn_exp2f(fmaf(bl, __builtin_amdgcn_sqrtf(s), -bl));
}

struct KRParams {
    double sigma2;   // sigma_s^2
    double r0;       // 1/2 - eps_B
    double epsB;
    double kend;     // value for r >= 1/2
    int ncoef;
    double coef[24]; // polynomial in t = (r - r0)/eps_B on [0,1]
};

// Regularised kernel K_R(r): K for r <= r0, a two-point Taylor (Hermite)
// polynomial on (r0, 1/2) that meets K smoothly at r0 and is flat at 1/2,
// constant beyond.
__device__ inline double kernel_reg(double r, const KRParams &kr) {
    if (r <= kr.r0) return exp(-r * r / kr.sigma2);
    if (r >= 0.5) return kr.kend;
    double t = (r - kr.r0) / kr.epsB;
    double acc = kr.coef[kr.ncoef - 1];
    for (int i = kr.ncoef - 2; i >= 0; --i) acc = acc * t + kr.coef[i];
    return acc;
}

// ------------------------------------------------------------------------------
// plan kernels
// ------------------------------------------------------------------------------
// Per-block min and max of each coordinate.
__global__ void k_minmax(int64_t n, int d, const double *__restrict__ pts, double *part) {
    __shared__ double smin[256 * 3], smax[256 * 3];
    const int tid = threadIdx.x;
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = (int64_t)blockIdx.x * 256 + tid; i < n; i += (int64_t)gridDim.x * 256)
        for (int t = 0; t < d; ++t) {
            double v = pts[i * d + t];
            mn[t] = fmin(mn[t], v);
            mx[t] = fmax(mx[t], v);
        }
    for (int t = 0; t < 3; ++t) { smin[t * 256 + tid] = mn[t]; smax[t * 256 + tid] = mx[t]; }
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (tid < off)
            for (int t = 0; t < 3; ++t) {
                smin[t * 256 + tid] = fmin(smin[t * 256 + tid], smin[t * 256 + tid + off]);
                smax[t * 256 + tid] = fmax(smax[t * 256 + tid], smax[t * 256 + tid + off]);
            }
        __syncthreads();
    }
    if (tid == 0)
        for (int t = 0; t < 3; ++t) {
            part[blockIdx.x * 6 + t] = smin[t * 256];
            part[blockIdx.x * 6 + 3 + t] = smax[t * 256];
        }
}

// flag := 1 if some coordinate is not finite.
__global__ void k_check_finite(int64_t cnt, const double *__restrict__ pts, int *flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt && !isfinite(pts[i])) flag[0] = 1;
}

// Per-block max of ||x - c||^2.
__global__ void k_maxrad(int64_t n, int d, const double *__restrict__ pts, double c0, double c1,
                         double c2, double *part) {
    __shared__ double s[256];
    const int tid = threadIdx.x;
    const double c[3] = {c0, c1, c2};
    double mx = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + tid; i < n; i += (int64_t)gridDim.x * 256) {
        double r2 = 0.0;
        for (int t = 0; t < d; ++t) {
            double dl = pts[i * d + t] - c[t];
            r2 += dl * dl;
        }
        mx = fmax(mx, r2);
    }
    s[tid] = mx;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (tid < off) s[tid] = fmax(s[tid], s[tid + off]);
        __syncthreads();
    }
    if (tid == 0) part[blockIdx.x] = s[0];
}

// Grid coordinates u (SoA) and bin keys; idx = i.
__global__ void k_coords_keys(int64_t n, int d, const double *__restrict__ pts, double c0,
                              double c1, double c2, double scale, int nos, int B, int nb,
                              double *__restrict__ u, unsigned *__restrict__ keys,
                              int *__restrict__ idx) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double c[3] = {c0, c1, c2};
    unsigned key = 0, mul = 1;
    for (int t = 0; t < d; ++t) {
        double ut = (scale * (pts[i * d + t] - c[t]) + 0.5) * (double)nos;
        u[(int64_t)t * n + i] = ut;
        // valid input keeps u inside (nos/4, 3nos/4); the clamp keeps every
        // patch inside the grid even for inputs that are not
        int cell = ut > 0.0 ? (int)floor(ut) : 0;
        const int lo = nos / 4 - 1, hi = 3 * nos / 4;
        cell = cell < lo ? lo : (cell > hi ? hi : cell);
        key += (unsigned)(cell / B) * mul;
        mul *= (unsigned)nb;
    }
    keys[i] = key;
    idx[i] = (int)i;
}

// Sorted coordinates: FP64 u, and for FP32 kernels the integer cell plus the
// fractional offset (so the FP32 cell always equals the bin-key cell).
__global__ void k_gather_coords(int64_t n, int d, int nos, const double *__restrict__ u,
                                const int *__restrict__ perm, double *__restrict__ u64,
                                int *__restrict__ c32, float *__restrict__ f32) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int64_t i = perm[p];
    for (int t = 0; t < d; ++t) {
        double v = u[(int64_t)t * n + i];
        u64[(int64_t)t * n + p] = v;
        int cell = v > 0.0 ? (int)floor(v) : 0;
        const int lo = nos / 4 - 1, hi = 3 * nos / 4;
        cell = cell < lo ? lo : (cell > hi ? hi : cell);
        double fr = v - (double)cell;
        float ff = (float)fr;
        ff = ff < 0.0f ? 0.0f : (ff >= 1.0f ? 0x1.fffffep-1f : ff);
        c32[(int64_t)t * n + p] = cell;
        f32[(int64_t)t * n + p] = ff;
    }
}

__global__ void k_task_counts(int runs, const unsigned *__restrict__ counts, int ch,
                              unsigned *__restrict__ ntask) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < runs) ntask[r] = (counts[r] + ch - 1) / ch;
}

// Tasks of each run (bin) of sorted points; a run cut into several tasks
// accumulates into scratch patch slots that a reduction sums afterwards.
__global__ void k_fill_tasks(int runs, const unsigned *__restrict__ ukeys,
                             const unsigned *__restrict__ counts,
                             const unsigned *__restrict__ run_start,
                             const unsigned *__restrict__ task_first,
                             const unsigned *__restrict__ scr_first,
                             const unsigned *__restrict__ multi_idx, int ch,
                             int4 *__restrict__ tasks, int *__restrict__ bin_run,
                             int4 *__restrict__ multi) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= runs) return;
    const unsigned cnt = counts[r], st = run_start[r], tf = task_first[r];
    const unsigned nt = (cnt + ch - 1) / ch;
    for (unsigned j = 0; j < nt; ++j) {
        unsigned first = st + j * ch;
        unsigned c = cnt - j * ch < (unsigned)ch ? cnt - j * ch : (unsigned)ch;
        int dest = nt == 1 ? r : runs + (int)(scr_first[r] + j);
        tasks[tf + j] = make_int4((int)ukeys[r], (int)first, (int)c, dest);
    }
    bin_run[ukeys[r]] = r;
    if (nt > 1) multi[multi_idx[r]] = make_int4(r, runs + (int)scr_first[r], (int)nt, 0);
}

__global__ void k_scr_counts(int runs, const unsigned *__restrict__ ntask,
                             unsigned *__restrict__ scr, unsigned *__restrict__ ism) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r > runs) return;
    const unsigned nt = r < runs ? ntask[r] : 0u;
    scr[r] = nt > 1 ? nt : 0u;
    ism[r] = nt > 1 ? 1u : 0u;
}

// Coarse occupancy: superbin (SB^d bins) holding at least one point.
__global__ void k_superbins(int runs, const unsigned *__restrict__ ukeys, int d, int nb, int SB,
                            int nsb, unsigned char *__restrict__ occ) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= runs) return;
    unsigned key = ukeys[r];
    int idx = 0, mul = 1;
    for (int t = 0; t < d; ++t) {
        int b = (int)(key % (unsigned)nb);
        key /= (unsigned)nb;
        idx += (b / SB) * mul;
        mul *= nsb;
    }
    occ[idx] = 1;
}

// Samples S[k] = K_R(k~/N), k in [0,N)^d with k~ = k or k - N (the set I_N).
__global__ void k_sample_kr(int d, int N, KRParams kr, double *__restrict__ S) {
    int64_t cnt = 1;
    for (int t = 0; t < d; ++t) cnt *= N;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= cnt) return;
    int64_t rem = e;
    double r2 = 0.0;
    for (int t = 0; t < d; ++t) {
        int k = (int)(rem % N);
        rem /= N;
        int kk = k < N / 2 ? k : k - N;
        double y = (double)kk / (double)N;
        r2 += y * y;
    }
    S[e] = kernel_reg(sqrt(r2), kr);
}

// One separable pass of the real-even DFT along dimension `axis`:
// out[.., l, ..] = sum_k in[.., k, ..] cos(2 pi l k / N) * scale.
__global__ void k_cos_dft(int d, int N, int axis, const double *__restrict__ in,
                          double *__restrict__ out, double scale) {
    int64_t cnt = 1;
    for (int t = 0; t < d; ++t) cnt *= N;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= cnt) return;
    int64_t stride = 1;
    for (int t = 0; t < axis; ++t) stride *= N;
    const int l = (int)((e / stride) % N);
    const int64_t base = e - (int64_t)l * stride;
    double acc = 0.0;
    for (int k = 0; k < N; ++k) {
        int ph = (int)(((int64_t)l * k) % N);
        acc += in[base + (int64_t)k * stride] * cospi(2.0 * (double)ph / (double)N);
    }
    out[e] = acc * scale;
}

// psi^(l / nos) for l = 0..N/2 by Gauss-Legendre quadrature on [0, w/2]:
// psi^(xi) = 2 int_0^{w/2} psi(t) cos(2 pi xi t) dt.
__global__ void k_window_hat(int N, int nos, int w, double beta, const double *__restrict__ gx,
                             const double *__restrict__ gw, int q, double *__restrict__ ph) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l > N / 2) return;
    const double half = 0.5 * w;
    const double xi = (double)l / (double)nos;
    double acc = 0.0;
    for (int j = 0; j < q; ++j) {
        double t = (gx[j] + 1.0) * 0.5 * half;
        double z = t / half;
        double s = 1.0 - z * z;
        s = s > 0.0 ? s : 0.0;
        double psi = exp(beta * (sqrt(s) - 1.0));
        acc += gw[j] * 0.5 * half * psi * cospi(2.0 * xi * t);
    }
    ph[l] = 2.0 * acc;
}

// Multipliers on the full 2N grid (FFT index k <-> frequency k or k - nos).
template <class T>
__global__ void k_make_M(int d, int N, int nos, const double *__restrict__ bhat,
                         const double *__restrict__ ph, T *__restrict__ M) {
    int64_t cnt = 1;
    for (int t = 0; t < d; ++t) cnt *= nos;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= cnt) return;
    int64_t rem = e, bidx = 0, bmul = 1;
    double fac = 1.0;
    bool inband = true;
    for (int t = 0; t < d; ++t) {
        int k = (int)(rem % nos);
        rem /= nos;
        int l = k < nos / 2 ? k : k - nos;
        int al = l < 0 ? -l : l;
        if (al > N / 2) { inband = false; break; }
        double p = ph[al];
        fac *= (al == N / 2 ? 0.5 : 1.0) / (p * p);
        int lm = ((l % N) + N) % N;
        bidx += (int64_t)lm * bmul;
        bmul *= N;
    }
    M[e] = inband ? (T)(bhat[bidx] * fac) : T(0);
}

__global__ void k_twiddles(int L, float2 *__restrict__ t32, double2 *__restrict__ t64) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= L / 2) return;
    double a = 2.0 * (double)j / (double)L;
    double c = cospi(a), s = -sinpi(a);
    t64[j] = make_double2(c, s);
    t32[j] = make_float2((float)c, (float)s);
}

// ------------------------------------------------------------------------------
// apply kernels
// ------------------------------------------------------------------------------
struct Geom {
    int d, nos, B, nb, w, P, PD, bs;
    int64_t n;
    // sorted position -> original index: the vector blocks Zs / Fs are kept
    // in the caller's node order, points in bin order
    const int *perm;
    // optional per-point factor (bin order) applied to each z row as it is
    // read: the matrix-core spreading of a layer that reads the shared FP32
    // slice of x multiplies by its D^-1/2 (rounded to FP32) there
    const float *zsc;
};



// One layer of a batched launch (several layers' tasks in one grid): the
// matrix-core kernels take the layer of task k from tlayer[k] and its
// geometry and arrays from here instead of their own arguments.
struct LayerArgs {
    Geom g;
    const int *c32;
    const float *f32;
    const float *Zs;     // spreading input slice
    float *Fs;           // interpolation output slice
    const float *grid;   // interpolation input grid
    float beta;
};

// The arrays the matrix-core kernels read come either from their arguments or
// from a LayerArgs entry in device memory; a pointer loaded from memory has no
// known address space, and its loads compile to flat instructions.  Flat loads
// count against the LDS wait counter too, so every LDS wait in the matrix loop
// would also wait for the next chunk's prefetched rows.  Every such pointer
// addresses global memory; typing it so gives global loads and stores.
#define MLG_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ MLG_GLOBAL T *to_global(T *p) {
    return (MLG_GLOBAL T *)p;
}

// (cell, fractional offset) of point p along dimension t.
template <class T>
__device__ inline void point_coord(const double *u64, const int *c32, const float *f32,
                                   int64_t idx, int &cell, T &frac);
template <>
__device__ inline void point_coord<float>(const double *, const int *c32, const float *f32,
                                          int64_t idx, int &cell, float &frac) {
    cell = c32[idx];
    frac = f32[idx];
}
template <>
__device__ inline void point_coord<double>(const double *u64, const int *, const float *,
                                           int64_t idx, int &cell, double &frac) {
    const double u = u64[idx];
    cell = (int)floor(u);
    frac = u - (double)cell;
}

__device__ inline int floor_div(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

template <class T, int V>
__device__ inline void load_vec(const T *__restrict__ p, T (&out)[V]) {
    if constexpr (sizeof(T) == 4 && V % 4 == 0) {
#pragma unroll
        for (int i = 0; i < V; i += 4) {
            float4 q = *reinterpret_cast<const float4 *>(p + i);
            out[i] = q.x; out[i + 1] = q.y; out[i + 2] = q.z; out[i + 3] = q.w;
        }
    } else if constexpr (sizeof(T) == 8 && V % 2 == 0) {
#pragma unroll
        for (int i = 0; i < V; i += 2) {
            double2 q = *reinterpret_cast<const double2 *>(p + i);
            out[i] = q.x; out[i + 1] = q.y;
        }
    } else {
#pragma unroll
        for (int i = 0; i < V; ++i) out[i] = p[i];
    }
}

template <class T, int V>
__device__ inline void store_vec(T *__restrict__ p, const T (&v)[V]) {
    if constexpr (sizeof(T) == 4 && V % 4 == 0) {
#pragma unroll
        for (int i = 0; i < V; i += 4)
            *reinterpret_cast<float4 *>(p + i) = make_float4(v[i], v[i + 1], v[i + 2], v[i + 3]);
    } else if constexpr (sizeof(T) == 8 && V % 2 == 0) {
#pragma unroll
        for (int i = 0; i < V; i += 2)
            *reinterpret_cast<double2 *>(p + i) = make_double2(v[i], v[i + 1]);
    } else {
#pragma unroll
        for (int i = 0; i < V; ++i) p[i] = v[i];
    }
}

// Grid layout: bg/2 complex planes of G cells each (plane-major); vector v
// of cell c is component (v & 1) of complex entry (v >> 1) * G + c.  Every
// plane is a contiguous nos^d array, so each FFT pass streams whole lines.
template <class T>
__device__ inline int64_t grid_index(int64_t G, int64_t cell, int v) {
    return ((int64_t)(v >> 1) * G + cell) * 2 + (v & 1);
}

template <class T, int V>
__device__ inline void grid_store(T *__restrict__ grid, int64_t G, int64_t cell, int v0, const T (&v)[V]) {
    if constexpr (V == 1) {
        grid[grid_index<T>(G, cell, v0)] = v[0];
    } else {
        using C2 = typename std::conditional<sizeof(T) == 4, float2, double2>::type;
#pragma unroll
        for (int i = 0; i < V; i += 2) {
            C2 c;
            c.x = v[i];
            c.y = v[i + 1];
            *reinterpret_cast<C2 *>(grid + grid_index<T>(G, cell, v0 + i)) = c;
        }
    }
}

template <class T, int V>
__device__ inline void grid_load(const T *__restrict__ grid, int64_t G, int64_t cell, int v0, T (&out)[V]) {
    if constexpr (V == 1) {
        out[0] = grid[grid_index<T>(G, cell, v0)];
    } else {
        using C2 = typename std::conditional<sizeof(T) == 4, float2, double2>::type;
#pragma unroll
        for (int i = 0; i < V; i += 2) {
            const C2 c = *reinterpret_cast<const C2 *>(grid + grid_index<T>(G, cell, v0 + i));
            out[i] = c.x;
            out[i + 1] = c.y;
        }
    }
}

// Spread: one 64-lane workgroup per (task, vector group).  Lane l owns patch
// cells l, l+64, ... and VPL vectors of each; points are staged 64 at a time
// (their 1D window weights at the P patch positions per dimension, and their
// values) and accumulated in the task's point order.
template <class T, int D, int VPL, int CMAX>
__global__ __launch_bounds__(64) void k_spread(Geom g, const int4 *__restrict__ tasks,
                                               const double *__restrict__ u64,
                                               const int *__restrict__ c32,
                                               const float *__restrict__ f32,
                                               const T *__restrict__ Zs, T beta,
                                               T *__restrict__ patch) {
    extern __shared__ unsigned char smem_raw[];
    const int P = g.P, PD = g.PD, bs = g.bs;
    T *wts = reinterpret_cast<T *>(smem_raw);       // [64][D][P]
    T *zv = wts + 64 * D * P;                        // [64][VPL]
    const int lane = threadIdx.x;
    const int4 tk = tasks[blockIdx.x];
    const int v0 = blockIdx.y * VPL;
    int org[3] = {0, 0, 0};
    {
        unsigned key = (unsigned)tk.x;
        for (int t = 0; t < D; ++t) {
            org[t] = (int)(key % (unsigned)g.nb) * g.B - g.w / 2 + 1;
            key /= (unsigned)g.nb;
        }
    }
    int qoff[CMAX];
    T acc[CMAX][VPL];
#pragma unroll
    for (int j = 0; j < CMAX; ++j) {
        const int c = lane + 64 * j;
        const int qx = c % P, qy = (c / P) % P, qz = c / (P * P);
        qoff[j] = c < PD ? (qx | ((P + qy) << 8) | ((2 * P + qz) << 16)) : -1;
#pragma unroll
        for (int v = 0; v < VPL; ++v) acc[j][v] = T(0);
    }
    const T two_over_w = T(2) / (T)g.w;
    const int cpl = (PD + 63) / 64;
    for (int c0 = 0; c0 < tk.z; c0 += 64) {
        const int cnt = (tk.z - c0) < 64 ? (tk.z - c0) : 64;
        const int64_t first = (int64_t)tk.y + c0;
        __syncthreads();
        if (lane < cnt) {
            const int64_t p = first + lane;
            for (int t = 0; t < D; ++t) {
                int cell;
                T frac;
                point_coord<T>(u64, c32, f32, (int64_t)t * g.n + p, cell, frac);
                const int s0 = cell - g.w / 2 + 1;
                for (int q = 0; q < P; ++q) {
                    const int k = org[t] + q;
                    T val = T(0);
                    if (k >= s0 && k < s0 + g.w) val = es_psi<T>((T)(cell - k) + frac, two_over_w, beta);
                    wts[(lane * D + t) * P + q] = val;
                }
            }
            T zz[VPL];
            load_vec<T, VPL>(Zs + (int64_t)g.perm[p] * bs + v0, zz);
#pragma unroll
            for (int v = 0; v < VPL; ++v) zv[lane * VPL + v] = zz[v];
        }
        __syncthreads();
        for (int pt = 0; pt < cnt; ++pt) {
            const T *wp = wts + pt * D * P;
            T zz[VPL];
#pragma unroll
            for (int v = 0; v < VPL; ++v) zz[v] = zv[pt * VPL + v];
#pragma unroll
            for (int j = 0; j < CMAX; ++j) {
                if (j < cpl && qoff[j] >= 0) {   // j < cpl is uniform
                    T wgt = wp[qoff[j] & 0xff];
                    if (D > 1) wgt *= wp[(qoff[j] >> 8) & 0xff];
                    if (D > 2) wgt *= wp[(qoff[j] >> 16) & 0xff];
#pragma unroll
                    for (int v = 0; v < VPL; ++v) acc[j][v] += wgt * zz[v];
                }
            }
        }
    }
    T *out = patch + (int64_t)tk.w * PD * bs + v0;
#pragma unroll
    for (int j = 0; j < CMAX; ++j)
        if (qoff[j] >= 0) store_vec<T, VPL>(out + (int64_t)(lane + 64 * j) * bs, acc[j]);
}

// Bins cut into several tasks: their task patches are summed in a fixed
// two-level order.  Level 1: each group of up to 32 consecutive task patches
// (int4: first slot, count, destination slot, 0) is summed in task order
// into its destination: the run's own patch slot when the run has a single
// group, else the group's first slot.
template <class T>
__global__ void k_reduce1(int64_t elems, const int4 *__restrict__ grp, T *__restrict__ patch) {
    const int64_t e = (int64_t)blockIdx.y * blockDim.x + threadIdx.x;
    if (e >= elems) return;
    const int4 gr = grp[blockIdx.x];
    const T *src = patch + (int64_t)gr.x * elems + e;
    // loads in batches of 8 (all in flight together), sums in task order
    T s = src[0];
    for (int j0 = 1; j0 < gr.y; j0 += 8) {
        T h[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) h[u] = j0 + u < gr.y ? src[(int64_t)(j0 + u) * elems] : T(0);
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (j0 + u < gr.y) s += h[u];
    }
    patch[(int64_t)gr.z * elems + e] = s;
}

// Level 2 (int4: run, first scratch slot, groups, 0), runs of more than one
// group only: the group sums, in group order, into the run's own patch slot.
template <class T>
__global__ void k_reduce2(int64_t elems, const int4 *__restrict__ runs, T *__restrict__ patch) {
    const int64_t e = (int64_t)blockIdx.y * blockDim.x + threadIdx.x;
    if (e >= elems) return;
    const int4 r = runs[blockIdx.x];
    const T *src = patch + (int64_t)r.y * elems + e;
    T s = src[0];
    for (int j0 = 1; j0 < r.z; j0 += 8) {
        T h[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) h[u] = j0 + u < r.z ? src[(int64_t)(j0 + u) * 32 * elems] : T(0);
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (j0 + u < r.z) s += h[u];
    }
    patch[(int64_t)r.x * elems + e] = s;
}

// Patch entry e = run * PD + o covers grid cell key[e].
__global__ void k_csr_keys(int64_t total, int d, int PD, int P, int nos, int B, int nb, int w,
                           const unsigned *__restrict__ run_key, unsigned *__restrict__ keys,
                           int *__restrict__ vals) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const int64_t u = e / PD;
    int o = (int)(e - u * PD);
    unsigned key = run_key[u];
    int64_t cell = 0, mul = 1;
    for (int t = 0; t < d; ++t) {
        const int b = (int)(key % (unsigned)nb);
        key /= (unsigned)nb;
        const int q = o % P;
        o /= P;
        cell += (int64_t)(b * B - w / 2 + 1 + q) * mul;
        mul *= nos;
    }
    keys[e] = (unsigned)cell;
    vals[e] = (int)e;
}

__global__ void k_scatter_counts(int nu, const unsigned *__restrict__ ucell,
                                 const unsigned *__restrict__ cnt, int *__restrict__ dense) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nu) dense[ucell[i]] = (int)cnt[i];
}

template <class T, int VPL>
constexpr int csr_batch() {
    constexpr int w = 64 / (VPL * (int)(sizeof(T) / 4));
    return w < 4 ? 4 : (w > 16 ? 16 : w);
}

// Gather through the cell table: sum of the cell's patch entries in entry
// order (entries of one cell are sorted by run), NB entries in flight per
// batch (NB x VPL values of at most 64 registers).  Workgroup w takes cells
// 256 (w div ng) on and vector group w mod ng (ng = bs / VPL): the groups of
// one cell range run side by side, so each patch row and table entry comes
// from HBM once and is shared through L2.
// Batched form: the cells of nl layers in one flat index; layer t owns flat
// cells [coff[t], coff[t+1]) and its grid starts goff[t] elements after
// gridb; ptr / ent are the layers' tables concatenated (entries of patch
// slots in the batch's shared patch buffer).
template <class T, int VPL, int NB = csr_batch<T, VPL>()>
__global__ __launch_bounds__(256) void k_gather_csr(int64_t G, int bs, int bg,
                                                    const int *__restrict__ ptr,
                                                    const int *__restrict__ ent,
                                                    const T *__restrict__ patch,
                                                    T *__restrict__ grid_, int nl,
                                                    const int64_t *__restrict__ coff,
                                                    const int64_t *__restrict__ goff) {
    const int ng = bs / VPL, vg = (int)(blockIdx.x % (unsigned)ng);
    const int64_t flat = (int64_t)(blockIdx.x / (unsigned)ng) * blockDim.x + threadIdx.x;
    int64_t cell = flat;
    T *__restrict__ grid = grid_;
    if (nl > 0) {
        if (flat >= coff[nl]) return;
        int lo = 0, hi = nl - 1;   // the layer: largest t with coff[t] <= flat
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (coff[mid] <= flat) lo = mid;
            else hi = mid - 1;
        }
        G = coff[lo + 1] - coff[lo];
        cell = flat - coff[lo];
        grid = grid_ + goff[lo];
    } else if (cell >= G) {
        return;
    }
    const int v0 = vg * VPL;
    T acc[VPL];
#pragma unroll
    for (int v = 0; v < VPL; ++v) acc[v] = T(0);
    const int e1 = ptr[flat + 1];
    // entries in batches of NB: indices, then rows, all in flight; summed in
    // entry order
    for (int e0 = ptr[flat]; e0 < e1; e0 += NB) {
        int idx[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) idx[u] = e0 + u < e1 ? ent[e0 + u] : -1;
        T h[NB][VPL];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            if (idx[u] >= 0) load_vec<T, VPL>(patch + (int64_t)idx[u] * bs + v0, h[u]);
            else
#pragma unroll
                for (int v = 0; v < VPL; ++v) h[u][v] = T(0);
        }
#pragma unroll
        for (int u = 0; u < NB; ++u)
            if (idx[u] >= 0)
#pragma unroll
                for (int v = 0; v < VPL; ++v) acc[v] += h[u][v];
    }
    grid_store<T, VPL>(grid, G, cell, v0, acc);
    if (bg > bs && vg == 0)
        for (int v = bs; v < bg; ++v) grid[grid_index<T>(G, cell, v)] = T(0);
}

// Gather: one thread per (grid cell, vector group): sum over the bins whose
// patch covers the cell, in bin order.  The grid has stride bg >= bs per cell
// (extra components written as zero).
template <class T, int D, int VPL>
__global__ __launch_bounds__(256) void k_gather(Geom g, int SB, int nsb,
                                                const unsigned char *__restrict__ occ,
                                                const int *__restrict__ bin_run,
                                                const T *__restrict__ patch, int bg,
                                                T *__restrict__ grid, int64_t G) {
    const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= G) return;
    const int v0 = blockIdx.y * VPL;
    const int P = g.P, bs = g.bs;
    int c[3] = {0, 0, 0}, blo[3] = {0, 0, 0}, bhi[3] = {0, 0, 0};
    {
        int64_t rem = cell;
        for (int t = 0; t < D; ++t) {
            c[t] = (int)(rem % g.nos);
            rem /= g.nos;
            int lo = floor_div(c[t] + g.w / 2 - P + g.B - 1, g.B);   // ceil((c+w/2-P)/B)
            int hi = floor_div(c[t] + g.w / 2 - 1, g.B);
            blo[t] = lo < 0 ? 0 : lo;
            bhi[t] = hi > g.nb - 1 ? g.nb - 1 : hi;
        }
    }
    T acc[VPL];
#pragma unroll
    for (int v = 0; v < VPL; ++v) acc[v] = T(0);
    bool any = true;
    for (int t = 0; t < D; ++t)
        if (bhi[t] < blo[t]) any = false;
    if (any) {
        any = false;
        const int s2lo = D > 2 ? blo[2] / SB : 0, s2hi = D > 2 ? bhi[2] / SB : 0;
        const int s1lo = D > 1 ? blo[1] / SB : 0, s1hi = D > 1 ? bhi[1] / SB : 0;
        for (int s2 = s2lo; s2 <= s2hi; ++s2)
            for (int s1 = s1lo; s1 <= s1hi; ++s1)
                for (int s0 = blo[0] / SB; s0 <= bhi[0] / SB; ++s0)
                    any |= occ[s0 + nsb * (s1 + nsb * s2)] != 0;
    }
    if (any) {
        const int PD = g.PD;
        for (int b2 = blo[2]; b2 <= bhi[2]; ++b2) {
            const int o2 = D > 2 ? (c[2] - (b2 * g.B - g.w / 2 + 1)) * P * P : 0;
            for (int b1 = blo[1]; b1 <= bhi[1]; ++b1) {
                const int o1 = D > 1 ? (c[1] - (b1 * g.B - g.w / 2 + 1)) * P : 0;
                const int64_t rowkey = (int64_t)g.nb * (b1 + (int64_t)g.nb * b2);
                for (int b0 = blo[0]; b0 <= bhi[0]; ++b0) {
                    const int r = bin_run[rowkey + b0];
                    if (r < 0) continue;
                    const int o = o2 + o1 + (c[0] - (b0 * g.B - g.w / 2 + 1));
                    T h[VPL];
                    load_vec<T, VPL>(patch + ((int64_t)r * PD + o) * bs + v0, h);
#pragma unroll
                    for (int v = 0; v < VPL; ++v) acc[v] += h[v];
                }
            }
        }
    }
    grid_store<T, VPL>(grid, G, cell, v0, acc);
    if (bg > bs && blockIdx.y == 0)
        for (int v = bs; v < bg; ++v) grid[grid_index<T>(G, cell, v)] = T(0);
}

// ------------------------------------------------------------------------------
// FP32 matrix-core variants (16 vectors per workgroup).  Within one task the
// spreading is the dense product  patch (PD x 16) = Wt (PD x pts) Z (pts x 16)
// and the interpolation  F (pts x 16) = Wt^T (pts x PD) H (PD x 16), with
// Wt[c][p] the window weight of point p at patch cell c: both run on
// v_mfma_f32_16x16x4_f32 (FP32 inputs, FP32 accumulation).
// Operand layout of that instruction (one wavefront): A[i][k] in lane i+16k,
// B[k][j] in lane j+16k, D[i][j] in register i%4 of lane j+16*(i/4).
//
// A task is processed in chunks of 64 points.  Each lane owns one point of a
// chunk: it evaluates the point's D x P one-dimensional window values (and,
// for D = 3, the P x P products of the y and z factors) into an LDS record,
// while the cell/offset coordinates (and for spreading the 16 vector values)
// of the next chunk are already being fetched into registers.  The patch
// edge P is a compile-time constant, so the staging is branch-free and every
// LDS address in the MFMA loops is a per-lane base plus an immediate.
// ------------------------------------------------------------------------------
typedef float floatx4 __attribute__((ext_vector_type(4)));

// Four consecutive floats (16-byte aligned) of global memory.
__device__ __forceinline__ float4 load_row4(const MLG_GLOBAL float *p) {
    const floatx4 v = *reinterpret_cast<const MLG_GLOBAL floatx4 *>(p);
    return make_float4(v[0], v[1], v[2], v[3]);
}

template <int D, int P>
struct MfShape {
    static constexpr int PD = D == 3 ? P * P * P : (D == 2 ? P * P : P);
    static constexpr int NT = (PD + 15) / 16;                    // 16-cell tiles
    static constexpr int OB = D == 3 ? 3 * P : P;                 // second factor: wyz (D=3) or wy
    static constexpr int ZS = D == 3 ? 3 * P + P * P : D * P;     // zero slot
    // record stride (floats): a multiple of 4 (float4 stores) with an odd
    // quotient, so that the 16 records one read instruction touches start in
    // 16 different 4-bank groups
    static constexpr int WSP4 = (ZS + 1 + 3) / 4 * 4;
    static constexpr int WSP = (WSP4 / 4) % 2 == 1 ? WSP4 : WSP4 + 4;
    static constexpr int gcd(int a, int b) { return b == 0 ? a : gcd(b, a % b); }
    static constexpr int S16 = P / gcd(P, 16);   // period in tiles of (16t + li) mod P
    static constexpr int S4 = P / gcd(P, 4);     // period in steps of (4s + lk) mod P
};

// Coordinates of one point: grid cell and FP32 offset inside it, per dimension.
template <int D>
struct PtIn {
    int cell[D];
    float frac[D];
};

template <int D, class IP, class FP>
__device__ inline void fetch_point(IP c32, FP f32, int64_t n, int64_t p, bool ok, PtIn<D> &pi) {
#pragma unroll
    for (int t = 0; t < D; ++t) {
        pi.cell[t] = ok ? c32[(int64_t)t * n + p] : 0;
        pi.frac[t] = ok ? f32[(int64_t)t * n + p] : 0.0f;
    }
}

// Window values of one point along one dimension at the patch cells
// org + q, q = 0..P-1 (zero outside the point's w support cells, and for an
// absent point).
template <int P>
__device__ inline void window_row(int cell, float frac, int org, int w, float two_over_w, float beta,
                                  bool ok, float (&out)[P]) {
    const int lo = cell - w / 2 + 1 - org;   // first support cell, relative to org
    const float bi = (float)(cell - org);    // exact small integer
#pragma unroll
    for (int q = 0; q < P; ++q) {
        // (cell - (org + q)) + frac: exact integer part, one rounding
        const float v = es_psi<float>((bi - (float)q) + frac, two_over_w, beta);
        out[q] = (ok && q >= lo && q < lo + w) ? v : 0.0f;
    }
}

// The record of one point: wx[P] | wy[P] | wz[P] | wyz[P*P] (D = 3), wx | wy
// (D = 2) or wx (D = 1), then zeros; weights outside the point's footprint
// (and all weights of an absent point) are zero.
template <int D, int P>
__device__ inline void put_record(const PtIn<D> &pi, bool ok, const int org[3], int w,
                                  float two_over_w, float beta, float *__restrict__ wp) {
    using S = MfShape<D, P>;
    float wv[D][P];
#pragma unroll
    for (int t = 0; t < D; ++t) window_row<P>(pi.cell[t], pi.frac[t], org[t], w, two_over_w, beta, ok, wv[t]);
    float rec[S::WSP];
#pragma unroll
    for (int t = 0; t < D; ++t)
#pragma unroll
        for (int q = 0; q < P; ++q) rec[t * P + q] = wv[t][q];
    if constexpr (D == 3) {
#pragma unroll
        for (int qz = 0; qz < P; ++qz)
#pragma unroll
            for (int qy = 0; qy < P; ++qy) rec[3 * P + qy + P * qz] = wv[1][qy] * wv[2][qz];
    }
#pragma unroll
    for (int e = S::ZS; e < S::WSP; ++e) rec[e] = 0.0f;
#pragma unroll
    for (int e = 0; e < S::WSP; e += 4)
        *reinterpret_cast<float4 *>(wp + e) = make_float4(rec[e], rec[e + 1], rec[e + 2], rec[e + 3]);
}

template <int D>
__device__ inline void task_origin(const Geom &g, unsigned key, int org[3]) {
    org[0] = org[1] = org[2] = 0;
#pragma unroll
    for (int t = 0; t < D; ++t) {
        org[t] = (int)(key % (unsigned)g.nb) * g.B - g.w / 2 + 1;
        key /= (unsigned)g.nb;
    }
}

template <int D, int P>
__global__ __launch_bounds__(64) void k_spread_mfma(Geom g_, const int4 *__restrict__ tasks,
                                                    const int *__restrict__ c32_,
                                                    const float *__restrict__ f32_,
                                                    const float *__restrict__ Zs_, float beta_,
                                                    float *__restrict__ patch,
                                                    const LayerArgs *__restrict__ lay,
                                                    const int *__restrict__ tlayer) {
    const LayerArgs *lp = lay ? lay + tlayer[blockIdx.x] : nullptr;
    const Geom g = lp ? lp->g : g_;
    const MLG_GLOBAL int *__restrict__ c32 = to_global(lp ? lp->c32 : c32_);
    const MLG_GLOBAL float *__restrict__ f32 = to_global(lp ? lp->f32 : f32_);
    const MLG_GLOBAL float *__restrict__ Zs = to_global(lp ? lp->Zs : Zs_);
    const MLG_GLOBAL int *__restrict__ perm = to_global(g.perm);
    const MLG_GLOBAL float *__restrict__ zsc = to_global(g.zsc);
    const float beta = lp ? lp->beta : beta_;
    using S = MfShape<D, P>;
    constexpr int NT = S::NT, WSP = S::WSP;
    __shared__ __attribute__((aligned(16))) float wts[64 * WSP];
    __shared__ __attribute__((aligned(16))) float zv[64 * 16];
    const int bs = g.bs;
    const int lane = threadIdx.x, li = lane & 15, lk = lane >> 4;
    const int4 tk = tasks[blockIdx.x];
    const int v0 = blockIdx.y * 16;
    int org[3];
    task_origin<D>(g, (unsigned)tk.x, org);
    const float two_over_w = 2.0f / (float)g.w;

    // LDS offsets (floats) of the two factors of tile t's cell 16t + li for the
    // lane's k slot; periodic in t with period S16, the remainder folded into
    // immediates.  Cells past the patch (last tile only) read the zero slot.
    int ra[S::S16], rb[S::S16];
#pragma unroll
    for (int tm = 0; tm < S::S16; ++tm) {
        const int c = 16 * tm + li;
        ra[tm] = lk * WSP + c % P;
        rb[tm] = lk * WSP + S::OB + c / P;
    }
    int la, lb;
    {
        const int c = 16 * (NT - 1) + li;
        la = c < S::PD ? lk * WSP + c % P : lk * WSP + S::ZS;
        lb = c < S::PD ? lk * WSP + S::OB + c / P : lk * WSP + S::ZS;
    }
    floatx4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};

    PtIn<D> pin;
    float4 zin[4];
    float zf = 1.0f;   // the row's factor, applied when the row is staged
    // node rows of the points run one chunk ahead of their coordinates, so
    // no load waits on another inside the loop
    int rown;
    {
        const bool ok = lane < tk.z;
        const int64_t p = (int64_t)tk.y + lane;
        fetch_point<D>(c32, f32, g.n, p, ok, pin);
        const int row = ok ? perm[p] : 0;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            zin[j] = ok ? load_row4(Zs + (int64_t)row * bs + v0 + 4 * j) : make_float4(0.f, 0.f, 0.f, 0.f);
        zf = (ok && zsc) ? zsc[p] : 1.0f;
        rown = lane + 64 < tk.z ? perm[(int64_t)tk.y + 64 + lane] : 0;
    }
    for (int c0 = 0; c0 < tk.z; c0 += 64) {
        const int cnt = (tk.z - c0) < 64 ? (tk.z - c0) : 64;
        __syncthreads();
        put_record<D, P>(pin, lane < cnt, org, g.w, two_over_w, beta, wts + lane * WSP);
#pragma unroll
        for (int j = 0; j < 4; ++j)
            *reinterpret_cast<float4 *>(zv + lane * 16 + 4 * j) =
                make_float4(zin[j].x * zf, zin[j].y * zf, zin[j].z * zf, zin[j].w * zf);
        __syncthreads();
        const int c1 = c0 + 64;
        if (c1 < tk.z) {   // prefetch the next chunk while this one is multiplied
            const bool ok = lane < tk.z - c1;
            const int64_t p = (int64_t)tk.y + c1 + lane;
            fetch_point<D>(c32, f32, g.n, p, ok, pin);
            const int row = rown;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                zin[j] = ok ? load_row4(Zs + (int64_t)row * bs + v0 + 4 * j) : make_float4(0.f, 0.f, 0.f, 0.f);
            zf = (ok && zsc) ? zsc[p] : 1.0f;
            rown = lane + 64 < tk.z - c1 ? perm[(int64_t)tk.y + c1 + 64 + lane] : 0;
        }
#pragma unroll
        for (int gi = 0; gi < 16; ++gi) {
            {
                const float b = zv[(4 * gi + lk) * 16 + li];
                float a[NT];
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const int tm = t % S::S16, tq = t / S::S16;
                    const int oa = (t == NT - 1 ? la : ra[tm]) + 4 * gi * WSP;
                    const int ob = (t == NT - 1 ? lb : rb[tm] + tq * (16 * S::S16 / P)) + 4 * gi * WSP;
                    a[t] = D > 1 ? wts[oa] * wts[ob] : wts[oa];
                }
#pragma unroll
                for (int t = 0; t < NT; ++t) acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t], b, acc[t], 0, 0, 0);
            }
        }
    }
    float *out = patch + (int64_t)tk.w * S::PD * bs + v0 + li;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int c = 16 * t + 4 * lk + r;
            if (c < S::PD) out[(int64_t)c * bs] = acc[t][r];
        }
    }
}

// Chunk body of the interpolation for NQ groups of 16 points: KSV steps of 4
// patch cells; the four point groups give four independent accumulators.
template <int D, int P, int NQ>
__device__ inline void interp_chunk(const float *__restrict__ wts, const int (&qa)[MfShape<D, P>::S4],
                                    const int (&qb)[MfShape<D, P>::S4], int li, int lk,
                                    const float *hb, int cnt, const int *wperm, int bs, int v0,
                                    MLG_GLOBAL float *__restrict__ Fs) {
    using S = MfShape<D, P>;
    constexpr int WSP = S::WSP;
    constexpr int KSV = (S::PD + 3) / 4;
    floatx4 acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < KSV; ++s) {
        const int sm = s % S::S4, sq = s / S::S4;
        int oa = qa[sm], ob = qb[sm] + sq * (4 * S::S4 / P);
        if (4 * s + 3 >= S::PD) {      // partial last step: cells past the patch
            const bool in = 4 * s + lk < S::PD;
            oa = in ? oa : li * WSP + S::ZS;
            ob = in ? ob : li * WSP + S::ZS;
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const float a = D > 1 ? wts[oa + 16 * q * WSP] * wts[ob + 16 * q * WSP] : wts[oa + 16 * q * WSP];
            acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, hb[s], acc[q], 0, 0, 0);
        }
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int pt = 16 * q + 4 * lk + r;
            if (pt < cnt) Fs[(int64_t)wperm[pt] * bs + v0 + li] = acc[q][r];
        }
}

template <int D, int P>
__global__ __launch_bounds__(64) void k_interp_mfma(Geom g_, const int4 *__restrict__ tasks,
                                                    const int *__restrict__ c32_,
                                                    const float *__restrict__ f32_,
                                                    const float *__restrict__ grid_, int bg,
                                                    float beta_, float *__restrict__ Fs_,
                                                    const LayerArgs *__restrict__ lay,
                                                    const int *__restrict__ tlayer) {
    const LayerArgs *lp = lay ? lay + tlayer[blockIdx.x] : nullptr;
    const Geom g = lp ? lp->g : g_;
    const MLG_GLOBAL int *__restrict__ c32 = to_global(lp ? lp->c32 : c32_);
    const MLG_GLOBAL float *__restrict__ f32 = to_global(lp ? lp->f32 : f32_);
    const MLG_GLOBAL float *__restrict__ grid = to_global(lp ? lp->grid : grid_);
    const MLG_GLOBAL int *__restrict__ perm = to_global(g.perm);
    const float beta = lp ? lp->beta : beta_;
    MLG_GLOBAL float *__restrict__ Fs = to_global(lp ? lp->Fs : Fs_);
    using S = MfShape<D, P>;
    constexpr int WSP = S::WSP;
    constexpr int KSV = (S::PD + 3) / 4;
    __shared__ __attribute__((aligned(16))) float wts[64 * WSP];
    int64_t G = g.nos;
    if (D > 1) G *= g.nos;
    if (D > 2) G *= g.nos;
    const int bs = g.bs;
    const int lane = threadIdx.x, li = lane & 15, lk = lane >> 4;
    const int4 tk = tasks[blockIdx.x];
    const int v0 = blockIdx.y * 16;
    int org[3];
    task_origin<D>(g, (unsigned)tk.x, org);
    const float two_over_w = 2.0f / (float)g.w;

    __shared__ int wperm[64];
    PtIn<D> pin;
    fetch_point<D>(c32, f32, g.n, (int64_t)tk.y + lane, lane < tk.z, pin);
    int prow = lane < tk.z ? perm[(int64_t)tk.y + lane] : 0;
    // B fragments: the task's patch of the grid, cell 4s + lk, vector li
    float hb[KSV];
#pragma unroll
    for (int s = 0; s < KSV; ++s) {
        const int c = 4 * s + lk;
        float h = 0.0f;
        if (c < S::PD) {
            const int qx = c % P, qy = (c / P) % P, qz = c / (P * P);
            int64_t cell = org[0] + qx;
            if (D > 1) cell += (int64_t)(org[1] + qy) * g.nos;
            if (D > 2) cell += (int64_t)(org[2] + qz) * g.nos * g.nos;
            h = grid[grid_index<float>(G, cell, v0 + li)];
        }
        hb[s] = h;
    }
    // LDS offsets of the factors of cell 4s + lk for point 16q + li: periodic
    // in s with period S4; q and the remainder of s are immediates.
    int qa[S::S4], qb[S::S4];
#pragma unroll
    for (int sm = 0; sm < S::S4; ++sm) {
        const int c = 4 * sm + lk;
        qa[sm] = li * WSP + c % P;
        qb[sm] = li * WSP + S::OB + c / P;
    }
    for (int c0 = 0; c0 < tk.z; c0 += 64) {
        const int cnt = (tk.z - c0) < 64 ? (tk.z - c0) : 64;
        __syncthreads();
        put_record<D, P>(pin, lane < cnt, org, g.w, two_over_w, beta, wts + lane * WSP);
        wperm[lane] = prow;
        __syncthreads();
        const int c1 = c0 + 64;
        if (c1 < tk.z) {
            fetch_point<D>(c32, f32, g.n, (int64_t)tk.y + c1 + lane, lane < tk.z - c1, pin);
            prow = lane < tk.z - c1 ? perm[(int64_t)tk.y + c1 + lane] : 0;
        }
        interp_chunk<D, P, 4>(wts, qa, qb, li, lk, hb, cnt, wperm, bs, v0, Fs);
    }
}

// ------------------------------------------------------------------------------
// d = 3 matrix-core variants built on the tensor structure of the window:
// the weight of a point at patch cell (cx, cy, cz) is wxy[cx + P cy] wz[cz].
//   spreading:      patch[(cx,cy), cz] = sum_p wxy_p[(cx,cy)] (wz_p[cz] z_p)
//     one A fragment (16 (cx,cy) rows x 4 points) serves all P values of cz,
//     B = wz_p[cz] z_p (one multiply per lane per cz);
//   interpolation:  f_p = sum_cz wz_p[cz] sum_(cx,cy) wxy_p[(cx,cy)] H[(cx,cy), cz]
//     one A fragment (16 points x 4 (cx,cy) cells) serves all P values of cz;
//     the P partial sums are combined per point on the vector ALUs.
// Per matrix instruction this needs a fraction of an LDS read instead of two
// reads and a multiply.
// ------------------------------------------------------------------------------
template <int P>
struct MfShape3 {
    static constexpr int C2 = P * P;                 // (cx, cy) cells
    static constexpr int T2 = (C2 + 15) / 16;        // 16-row tiles of (cx, cy)
    // spreading record stride, = 16 mod 32 so that the four k slots of a
    // wavefront read disjoint LDS banks
    static constexpr int RS = (T2 % 2 == 1) ? 16 * T2 : 16 * T2 + 16;
    static constexpr int KS2 = (C2 + 3) / 4;         // 4-cell steps of (cx, cy)
    static constexpr int NE = 4 * KS2 + P;           // interpolation entries per point
    static constexpr int ES = 80;                    // entry stride (64 points + 16)
};

// Window factors of one point: wx, wy, wz over the patch (zero outside the
// footprint and for an absent point).
template <int P>
__device__ inline void window_factors(const PtIn<3> &pi, bool ok, const int org[3], int w,
                                      float two_over_w, float beta, float (&wv)[3][P]) {
#pragma unroll
    for (int t = 0; t < 3; ++t) window_row<P>(pi.cell[t], pi.frac[t], org[t], w, two_over_w, beta, ok, wv[t]);
}

// Spreading tiles: TF full tiles of 16 (cx, cy) rows serve every cz with
// B = wz[cz] z; the RR = C2 mod 16 remaining (cx, cy) cells are packed with
// cz into TR mixed tiles, rows (r, cz) -> A = wxy[16 TF + r] wz[cz], B = z.
// Record layout: up to P = 6 a point's record holds its C2 products at
// stride RS (16 mod 32), mixed-tile cells included.  At P = 7 (TF = 3, one
// remaining cell) the record holds the 48 full-tile products at stride 48
// and the remaining product sits in an array of its own, so the stride stays
// 16 mod 32 without growing to 80 floats (LDS for two wavefronts per SIMD);
// its mixed tile has rows cz = 0..15, of which those >= P are zeroed.
template <int P>
struct SpreadTiles3 {
    static constexpr int C2 = P * P;
    static constexpr int TF = C2 / 16;
    static constexpr int RR = C2 % 16;
    static constexpr int TR = (RR * P + 15) / 16;
    static constexpr bool TAIL = P == 7;
    static constexpr int RS = TAIL ? 16 * TF : MfShape3<P>::RS;
    static constexpr int RW = TAIL ? 16 * TF : (C2 + 3) / 4 * 4;   // record entries written
};

// One task (points of one bin) of the d = 3 matrix-core spreading, written to
// its patch slot tk.w.  LDS: wxy (64 RS), wzs (64 x 8), zv (64 x 16), and
// for P = 7 wxt (64).
template <int P>
__device__ __forceinline__ void spread3_task(const Geom g, const int4 tk,
                                             const MLG_GLOBAL int *__restrict__ c32,
                                             const MLG_GLOBAL float *__restrict__ f32,
                                             const MLG_GLOBAL float *__restrict__ Zs, float beta,
                                             float *__restrict__ patch, float *wxy, float *wzs,
                                             float *zv, float *wxt) {
    using U = SpreadTiles3<P>;
    const MLG_GLOBAL int *__restrict__ perm = to_global(g.perm);
    const MLG_GLOBAL float *__restrict__ zsc = to_global(g.zsc);
    constexpr int RS = U::RS, RW = U::RW, C2 = U::C2, TF = U::TF, RR = U::RR, TR = U::TR;
    constexpr bool TAIL = U::TAIL;
    const int bs = g.bs;
    const int lane = threadIdx.x, li = lane & 15, lk = lane >> 4;
    const int v0 = blockIdx.y * 16;
    int org[3];
    task_origin<3>(g, (unsigned)tk.x, org);
    const float two_over_w = 2.0f / (float)g.w;
    floatx4 acc[TF > 0 ? TF : 1][P];
    floatx4 accr[TR > 0 ? TR : 1];
#pragma unroll
    for (int t = 0; t < TF; ++t)
#pragma unroll
        for (int cz = 0; cz < P; ++cz) acc[t][cz] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int u = 0; u < TR; ++u) accr[u] = floatx4{0.f, 0.f, 0.f, 0.f};
    // mixed-tile row of this lane: (cx, cy) cell 16 TF + r, z slice cz
    // (cz < 8 for every P <= 6; slots cz >= P select a zero factor; at P = 7
    // rows cz >= 8 are zeroed when the operand is formed)
    static_assert(TAIL || TR == 0 || (16 * TR - 1) / (RR > 0 ? RR : 1) < 8,
                  "mixed tile rows exceed the z slots");
    static_assert(!TAIL || (RR == 1 && TR == 1), "separate tail holds one cell");
    int rr_cell[TR > 0 ? TR : 1], rr_cz[TR > 0 ? TR : 1];
#pragma unroll
    for (int u = 0; u < TR; ++u) {
        const int flat = 16 * u + li;
        rr_cell[u] = 16 * TF + flat % (RR > 0 ? RR : 1);
        rr_cz[u] = flat / (RR > 0 ? RR : 1);
    }

    PtIn<3> pin;
    float4 zin[4];
    float zf = 1.0f;   // the row's factor, applied when the row is staged
    // node rows of the points run one chunk ahead of their coordinates, so
    // no load waits on another inside the loop
    int rown;
    {
        const bool ok = lane < tk.z;
        const int64_t p = (int64_t)tk.y + lane;
        fetch_point<3>(c32, f32, g.n, p, ok, pin);
        const int row = ok ? perm[p] : 0;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            zin[j] = ok ? load_row4(Zs + (int64_t)row * bs + v0 + 4 * j) : make_float4(0.f, 0.f, 0.f, 0.f);
        zf = (ok && zsc) ? zsc[p] : 1.0f;
        rown = lane + 64 < tk.z ? perm[(int64_t)tk.y + 64 + lane] : 0;
    }
    for (int c0 = 0; c0 < tk.z; c0 += 64) {
        const int cnt = (tk.z - c0) < 64 ? (tk.z - c0) : 64;
        __syncthreads();
        {
            float wv[3][P];
            window_factors<P>(pin, lane < cnt, org, g.w, two_over_w, beta, wv);
            float rec[RW];
#pragma unroll
            for (int e = 0; e < RW; ++e) rec[e] = e < C2 ? wv[0][e % P] * wv[1][e / P] : 0.0f;
            float *wp = wxy + lane * RS;
#pragma unroll
            for (int e = 0; e < RW; e += 4)
                *reinterpret_cast<float4 *>(wp + e) = make_float4(rec[e], rec[e + 1], rec[e + 2], rec[e + 3]);
            if constexpr (TAIL) wxt[lane] = wv[0][(C2 - 1) % P] * wv[1][(C2 - 1) / P];
            float zr[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) zr[e] = e < P ? wv[2][e] : 0.0f;
            *reinterpret_cast<float4 *>(wzs + lane * 8) = make_float4(zr[0], zr[1], zr[2], zr[3]);
            *reinterpret_cast<float4 *>(wzs + lane * 8 + 4) = make_float4(zr[4], zr[5], zr[6], zr[7]);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
            *reinterpret_cast<float4 *>(zv + lane * 16 + 4 * j) =
                make_float4(zin[j].x * zf, zin[j].y * zf, zin[j].z * zf, zin[j].w * zf);
        __syncthreads();
        const int c1 = c0 + 64;
        if (c1 < tk.z) {   // prefetch the next chunk while this one is multiplied
            const bool ok = lane < tk.z - c1;
            const int64_t p = (int64_t)tk.y + c1 + lane;
            fetch_point<3>(c32, f32, g.n, p, ok, pin);
            const int row = rown;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                zin[j] = ok ? load_row4(Zs + (int64_t)row * bs + v0 + 4 * j) : make_float4(0.f, 0.f, 0.f, 0.f);
            zf = (ok && zsc) ? zsc[p] : 1.0f;
            rown = lane + 64 < tk.z - c1 ? perm[(int64_t)tk.y + c1 + 64 + lane] : 0;
        }
        // all 16 groups in one straight-line block (absent points carry zero
        // records); the operands of group gi + 1 are read from LDS before the
        // matrix instructions of group gi are issued
        struct Ops {
            float z, a[TF > 0 ? TF : 1], rx[TR > 0 ? TR : 1], rz[TR > 0 ? TR : 1], wz[8];
        };
        auto read_ops = [&](int gi, Ops &o) {
            const int pp = 4 * gi + lk;
            o.z = zv[pp * 16 + li];
#pragma unroll
            for (int t = 0; t < TF; ++t) o.a[t] = wxy[pp * RS + 16 * t + li];
            // mixed-tile factors; z slots >= P of a record hold zero
#pragma unroll
            for (int u = 0; u < TR; ++u) {
                if constexpr (TAIL) {
                    o.rx[u] = wxt[pp];
                    o.rz[u] = wzs[pp * 8 + (rr_cz[u] & 7)];
                } else {
                    o.rx[u] = wxy[pp * RS + rr_cell[u]];
                    o.rz[u] = wzs[pp * 8 + rr_cz[u]];
                }
            }
            const float4 wz0 = *reinterpret_cast<const float4 *>(wzs + pp * 8);
            const float4 wz1 = *reinterpret_cast<const float4 *>(wzs + pp * 8 + 4);
            o.wz[0] = wz0.x; o.wz[1] = wz0.y; o.wz[2] = wz0.z; o.wz[3] = wz0.w;
            o.wz[4] = wz1.x; o.wz[5] = wz1.y; o.wz[6] = wz1.z; o.wz[7] = wz1.w;
        };
        Ops nxt;
        read_ops(0, nxt);
#pragma unroll
        for (int gi = 0; gi < 16; ++gi) {
            const Ops cur = nxt;
            if (gi + 1 < 16) read_ops(gi + 1, nxt);
            // keep the reads above the matrix instructions that hide them
            __builtin_amdgcn_sched_barrier(0);
            // every B operand of the group in its own register before the
            // first matrix instruction: the products do not rewrite a
            // register that an issued matrix instruction still reads
            float bb[P], rb[TR > 0 ? TR : 1];
#pragma unroll
            for (int cz = 0; cz < P; ++cz) bb[cz] = cur.z * cur.wz[cz];
#pragma unroll
            for (int u = 0; u < TR; ++u) {
                rb[u] = cur.rx[u] * cur.rz[u];
                if constexpr (TAIL) rb[u] = rr_cz[u] < P ? rb[u] : 0.0f;
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int cz = 0; cz < P; ++cz) {
#pragma unroll
                for (int t = 0; t < TF; ++t)
                    acc[t][cz] = __builtin_amdgcn_mfma_f32_16x16x4f32(cur.a[t], bb[cz], acc[t][cz], 0, 0, 0);
            }
#pragma unroll
            for (int u = 0; u < TR; ++u)
                accr[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(rb[u], cur.z, accr[u], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    float *out = patch + (int64_t)tk.w * (C2 * P) * bs + v0 + li;
#pragma unroll
    for (int t = 0; t < TF; ++t)
#pragma unroll
        for (int cz = 0; cz < P; ++cz)
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int cxy = 16 * t + 4 * lk + m;
                out[(int64_t)(cxy + C2 * cz) * bs] = acc[t][cz][m];
            }
#pragma unroll
    for (int u = 0; u < TR; ++u)
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int flat = 16 * u + 4 * lk + m;
            const int cz = flat / (RR > 0 ? RR : 1);
            if (cz < P) out[(int64_t)(16 * TF + flat % (RR > 0 ? RR : 1) + C2 * cz) * bs] = accr[u][m];
        }
}

// Two wavefronts per SIMD keep one wave's matrix work running while the
// other stages its records; the register budget is capped to allow that.
// Workgroup w runs task w (of the plan's task list or of its spreading
// schedule).
template <int P>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_spread_mfma3(Geom g, const int4 *__restrict__ tasks,
                                                     const int *__restrict__ c32,
                                                     const float *__restrict__ f32,
                                                     const float *__restrict__ Zs, float beta,
                                                     float *__restrict__ patch,
                                                     const LayerArgs *__restrict__ lay,
                                                     const int *__restrict__ tlayer) {
    using U = SpreadTiles3<P>;
    __shared__ __attribute__((aligned(16))) float wxy[64 * U::RS];
    __shared__ __attribute__((aligned(16))) float wzs[64 * 8];
    __shared__ __attribute__((aligned(16))) float zv[64 * 16];
    __shared__ float wxt[U::TAIL ? 64 : 1];
    const LayerArgs *lp = lay ? lay + tlayer[blockIdx.x] : nullptr;
    const Geom gl = lp ? lp->g : g;
    spread3_task<P>(gl, tasks[blockIdx.x], to_global(lp ? lp->c32 : c32),
                    to_global(lp ? lp->f32 : f32), to_global(lp ? lp->Zs : Zs),
                    lp ? lp->beta : beta, patch, wxy, wzs, zv, wxt);
}

template <int P>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(P <= 6 ? 3 : 2))) void k_interp_mfma3(Geom g_, const int4 *__restrict__ tasks,
                                                     const int *__restrict__ c32_,
                                                     const float *__restrict__ f32_,
                                                     const float *__restrict__ grid_, int bg,
                                                     float beta_, float *__restrict__ Fs_, int split,
                                                     int per, const LayerArgs *__restrict__ lay,
                                                     const int *__restrict__ tlayer) {
    const LayerArgs *lp = lay ? lay + tlayer[blockIdx.x / split] : nullptr;
    const Geom g = lp ? lp->g : g_;
    const MLG_GLOBAL int *__restrict__ c32 = to_global(lp ? lp->c32 : c32_);
    const MLG_GLOBAL float *__restrict__ f32 = to_global(lp ? lp->f32 : f32_);
    const MLG_GLOBAL float *__restrict__ grid = to_global(lp ? lp->grid : grid_);
    const MLG_GLOBAL int *__restrict__ perm = to_global(g.perm);
    const float beta = lp ? lp->beta : beta_;
    MLG_GLOBAL float *__restrict__ Fs = to_global(lp ? lp->Fs : Fs_);
    using S = MfShape3<P>;
    constexpr int KS2 = S::KS2, ES = S::ES, NE = S::NE, C2 = S::C2;
    // entry-major weights: entry e of point p at wt[e * ES + p]; entries
    // 0..4 KS2-1: wxy (zero past C2), then wz[0..P-1]
    __shared__ __attribute__((aligned(16))) float wt[NE * ES];
    const int64_t G = (int64_t)g.nos * g.nos * g.nos;
    const int bs = g.bs;
    const int lane = threadIdx.x, li = lane & 15, lk = lane >> 4;
    // workgroup = part (blockIdx.x mod split) of task blockIdx.x / split:
    // its points [part * per, part * per + per); a workgroup past the end of
    // a short task has nothing to do (one wavefront: it leaves before any
    // barrier)
    int4 tk = tasks[blockIdx.x / split];
    {
        const int lo = (blockIdx.x % split) * per;
        if (lo >= tk.z) return;
        tk.y += lo;
        tk.z = (tk.z - lo) < per ? (tk.z - lo) : per;
    }
    const int v0 = blockIdx.y * 16;
    int org[3];
    task_origin<3>(g, (unsigned)tk.x, org);
    const float two_over_w = 2.0f / (float)g.w;

    __shared__ int wperm[64];
    PtIn<3> pin;
    fetch_point<3>(c32, f32, g.n, (int64_t)tk.y + lane, lane < tk.z, pin);
    int prow = lane < tk.z ? perm[(int64_t)tk.y + lane] : 0;
    // B fragments: grid at (cx, cy) = 4s + lk, cz, vector li.  Addresses:
    // the lane's vector plane (grid_index layout) plus twice the cell index,
    // cell = task origin + cx + cy nos + cz nos^2 with (cx, cy) stepped
    // along s instead of divided out per load.
    float hb[P][KS2];
    {
        const int64_t nos = g.nos, nos2 = nos * nos;
        const int v = v0 + li;
        const MLG_GLOBAL float *gl = grid + 2 * ((int64_t)(v >> 1) * G) + (v & 1) +
                          2 * ((int64_t)org[0] + org[1] * nos + org[2] * nos2);
        int cx = lk, cy = 0;
#pragma unroll
        for (int s = 0; s < KS2; ++s) {
            const bool ok = 4 * s + lk < C2;
            const MLG_GLOBAL float *ps = gl + 2 * ((int64_t)cx + cy * nos);
#pragma unroll
            for (int cz = 0; cz < P; ++cz) hb[cz][s] = ok ? ps[2 * cz * nos2] : 0.0f;
            cx += 4;
            while (cx >= P) {
                cx -= P;
                ++cy;
            }
        }
    }
    for (int c0 = 0; c0 < tk.z; c0 += 64) {
        const int cnt = (tk.z - c0) < 64 ? (tk.z - c0) : 64;
        __syncthreads();
        {
            float wv[3][P];
            window_factors<P>(pin, lane < cnt, org, g.w, two_over_w, beta, wv);
#pragma unroll
            for (int e = 0; e < 4 * KS2; ++e) {
                const float v = e < C2 ? wv[0][e % P] * wv[1][e / P] : 0.0f;
                wt[e * ES + lane] = v;
            }
#pragma unroll
            for (int cz = 0; cz < P; ++cz) wt[(4 * KS2 + cz) * ES + lane] = wv[2][cz];
        }
        wperm[lane] = prow;
        __syncthreads();
        const int c1 = c0 + 64;
        if (c1 < tk.z) {
            fetch_point<3>(c32, f32, g.n, (int64_t)tk.y + c1 + lane, lane < tk.z - c1, pin);
            prow = lane < tk.z - c1 ? perm[(int64_t)tk.y + c1 + lane] : 0;
        }
        // four point groups of 16 in one straight-line block (absent points
        // carry zero weights and are not stored)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            floatx4 gz[P];
#pragma unroll
            for (int cz = 0; cz < P; ++cz) gz[cz] = floatx4{0.f, 0.f, 0.f, 0.f};
            // the A operand of step s + 1 is read before the matrix
            // instructions of step s are issued
            float an = wt[lk * ES + 16 * q + li];
#pragma unroll
            for (int s = 0; s < KS2; ++s) {
                const float a = an;
                if (s + 1 < KS2) an = wt[(4 * (s + 1) + lk) * ES + 16 * q + li];
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int cz = 0; cz < P; ++cz)
                    gz[cz] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, hb[cz][s], gz[cz], 0, 0, 0);
                __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int pt = 16 * q + 4 * lk + r;
                float f = 0.0f;
#pragma unroll
                for (int cz = 0; cz < P; ++cz) f += wt[(4 * KS2 + cz) * ES + pt] * gz[cz][r];
                if (pt < cnt) Fs[(int64_t)wperm[pt] * bs + v0 + li] = f;
            }
        }
    }
}

// Patch edges with a compiled matrix-core variant, per dimension.
// Mean points per occupied bin below which an automatic bin edge doubles
// (four 64-point matrix-core chunks).
constexpr int64_t kAutoBinPoints = 256;

static bool mfma_patch_ok(int D, int P) {
    if (P < 2) return false;
    if (D == 3) return P <= 7;
    if (D == 2) return P <= 12;
    return P <= 16;
}

#define MLG_P_SWITCH(D, p, CALL)                                                   \
    switch (p) {                                                                   \
        case 2: CALL(D, 2); break;                                                 \
        case 3: CALL(D, 3); break;                                                 \
        case 4: CALL(D, 4); break;                                                 \
        case 5: CALL(D, 5); break;                                                 \
        case 6: CALL(D, 6); break;                                                 \
        case 7: CALL(D, 7); break;                                                 \
        default:                                                                   \
            if constexpr (D < 3) {                                                 \
                switch (p) {                                                       \
                    case 8: CALL(D, 8); break;                                     \
                    case 9: CALL(D, 9); break;                                     \
                    case 10: CALL(D, 10); break;                                   \
                    case 11: CALL(D, 11); break;                                   \
                    case 12: CALL(D, 12); break;                                   \
                    default:                                                       \
                        if constexpr (D < 2) {                                     \
                            switch (p) {                                           \
                                case 13: CALL(D, 13); break;                       \
                                case 14: CALL(D, 14); break;                       \
                                case 15: CALL(D, 15); break;                       \
                                case 16: CALL(D, 16); break;                       \
                                default: throw Error(MLG_ERR_ARG, "unsupported patch edge"); \
                            }                                                      \
                        } else {                                                   \
                            throw Error(MLG_ERR_ARG, "unsupported patch edge");    \
                        }                                                          \
                }                                                                  \
            } else {                                                               \
                throw Error(MLG_ERR_ARG, "unsupported patch edge");                \
            }                                                                      \
    }

template <class T>
struct Cplx;
template <>
struct Cplx<float> { using type = float2; };
template <>
struct Cplx<double> { using type = double2; };

// Batched FFT of length L = 2^LOGL along one axis of each complex
// plane of the grid (plane-major layout: plane q = blockIdx.y, qstr complex
// entries apart; inside a plane the cells are [z][y][x], x contiguous).  A
// line is addressed as  off(o) + k S + coff(a),  k = 0..L-1 along the axis:
//   a in [0, A): the columns below the axis (contiguous), or the band
//                columns of the x axis (abnd = 1);
//   o in [0, O): the lines above the axis (stride ostr), or the band rows of
//                the y axis (obnd = 1).
// Band mapping: index i of the N + 1 band frequencies -> grid index i
// (i <= N/2) or L - (N + 1) + i.  Only frequency lines that can reach the
// band |l_t| <= N/2 are touched, which prunes the later axes.
// mode 0: forward, only the band entries along the axis are stored (the
// others are never read again); mode 1: inverse, entries whose k is outside
// the band read as zero (they were never multiplied); mode 2: forward, times
// the multiplier M (indexed by the in-plane cell), inverse: the last axis of
// Algorithm 1 in one pass.
// A workgroup takes OB consecutive o and C consecutive a (OB * C = LINES
// lines); loads and stores walk memory order (a fastest, then k, then o).
// The LDS buffer holds buf[k][line] with a padded row (LINES + 1) so that
// both the load pattern and the butterflies are free of bank conflicts.
__device__ inline int band_index(int i, int N, int nos) { return i <= N / 2 ? i : nos - (N + 1) + i; }

__device__ inline bool in_band(int k, int N, int nos) { return k <= N / 2 || k >= nos - N / 2; }

struct FftPass {
    int64_t O, A;        // lines: O outer x A columns
    int64_t S;           // element stride along the axis
    int64_t ostr;        // element stride of o (before band mapping)
    int64_t qstr;        // complex entries per plane
    int obnd, abnd;      // band-mapped o / a
    int N;               // bandwidth
    int mode;
    int logC, logOB;     // workgroup tile: C = 2^logC columns, OB = 2^logOB outers
    int64_t nachunk;     // ceil(A / C)
    int flat;            // lines numbered o * A + a, LINES consecutive ones per workgroup
    // batched layers: plane q = blockIdx.y belongs to layer q / lq, whose
    // multipliers start at M + (q / lq) mstr (mstr = 0: one set for all)
    int lq;
    int64_t mstr;
};

// 8-point DFT in registers (radix-2 decimation in frequency), natural order
// in and out: a[k] <- sum_n a[n] exp(-+2 pi i n k / 8) (+ for the inverse).
template <class C2>
__device__ inline void dft8(C2 (&a)[8], bool inverse) {
    using T = decltype(a[0].x);
    const T h = T(0.70710678118654752440);
    const T sg = inverse ? T(1) : T(-1);
    auto add = [](C2 u, C2 v) { C2 r; r.x = u.x + v.x; r.y = u.y + v.y; return r; };
    auto sub = [](C2 u, C2 v) { C2 r; r.x = u.x - v.x; r.y = u.y - v.y; return r; };
    // multiply by sg * i
    auto mul_i = [sg](C2 u) { C2 r; r.x = -sg * u.y; r.y = sg * u.x; return r; };
    // multiply by (h, sg h) resp. (-h, sg h)
    auto mul_w1 = [h, sg](C2 u) { C2 r; r.x = h * (u.x - sg * u.y); r.y = h * (u.y + sg * u.x); return r; };
    auto mul_w3 = [h, sg](C2 u) { C2 r; r.x = -h * (u.x + sg * u.y); r.y = h * (sg * u.x - u.y); return r; };
    const C2 b0 = add(a[0], a[4]), b4 = sub(a[0], a[4]);
    const C2 b1 = add(a[1], a[5]), b5 = mul_w1(sub(a[1], a[5]));
    const C2 b2 = add(a[2], a[6]), b6 = mul_i(sub(a[2], a[6]));
    const C2 b3 = add(a[3], a[7]), b7 = mul_w3(sub(a[3], a[7]));
    const C2 c0 = add(b0, b2), c2 = sub(b0, b2), c1 = add(b1, b3), c3 = mul_i(sub(b1, b3));
    const C2 c4 = add(b4, b6), c6 = sub(b4, b6), c5 = add(b5, b7), c7 = mul_i(sub(b5, b7));
    a[0] = add(c0, c1);
    a[4] = sub(c0, c1);
    a[2] = add(c2, c3);
    a[6] = sub(c2, c3);
    a[1] = add(c4, c5);
    a[5] = sub(c4, c5);
    a[3] = add(c6, c7);
    a[7] = sub(c6, c7);
}

// 4- and 2-point DFTs in registers, natural order (same sign convention).
template <class C2>
__device__ inline void dft4(C2 (&a)[4], bool inverse) {
    using T = decltype(a[0].x);
    const T sg = inverse ? T(1) : T(-1);
    C2 b0, b1, b2, b3;
    b0.x = a[0].x + a[2].x; b0.y = a[0].y + a[2].y;
    b1.x = a[0].x - a[2].x; b1.y = a[0].y - a[2].y;
    b2.x = a[1].x + a[3].x; b2.y = a[1].y + a[3].y;
    // (a1 - a3) times sg i
    b3.x = -sg * (a[1].y - a[3].y);
    b3.y = sg * (a[1].x - a[3].x);
    a[0].x = b0.x + b2.x; a[0].y = b0.y + b2.y;
    a[2].x = b0.x - b2.x; a[2].y = b0.y - b2.y;
    a[1].x = b1.x + b3.x; a[1].y = b1.y + b3.y;
    a[3].x = b1.x - b3.x; a[3].y = b1.y - b3.y;
}

template <class C2>
__device__ inline void dft2(C2 (&a)[2], bool) {
    const C2 u = a[0], v = a[1];
    a[0].x = u.x + v.x; a[0].y = u.y + v.y;
    a[1].x = u.x - v.x; a[1].y = u.y - v.y;
}

// Mixed-radix Stockham FFT of the LINES = 2^LOGLINES lines held in buf
// (element k of a line at buf[k * LDL + line]; natural order in and out):
// radix-8 stages, the last one of radix 4 or 2 when log2 L is not a
// multiple of 3.  A stage of radix R after sub-transforms of length Ns (the
// product of the earlier radices) takes, for butterfly j < L / R of a line,
// the inputs x[j + r L / R] (r < R), multiplies input r by
// W_{Ns R}^{(j mod Ns) r}, does an R-point DFT and writes output r to
// (j div Ns) Ns R + (j mod Ns) + r Ns.  All reads of a stage come before a
// barrier, all writes after it, so the stage runs in place.  tw[q] =
// exp(-2 pi i q / L), q < L / 2; 256 threads, each reaching every barrier.
template <class C2, int LOGL, int LDL, int LOGLINES, int LOGNS = 0>
__device__ inline void fft_stockham(C2 *buf, const C2 *tw, bool inverse) {
    constexpr int L = 1 << LOGL, LINES = 1 << LOGLINES;
    constexpr int LOGR = (LOGL - LOGNS) >= 3 ? 3 : (LOGL - LOGNS);
    if constexpr (LOGR > 0) {
        constexpr int R = 1 << LOGR, NS = 1 << LOGNS;
        constexpr int NB = (L / R) * LINES;   // butterflies of the stage
        constexpr int BPT = (NB + 255) / 256;
        C2 v[BPT][R];
#pragma unroll
        for (int i = 0; i < BPT; ++i) {
            const int b = threadIdx.x + 256 * i;
            if (NB % 256 != 0 && b >= NB) continue;
            const int ln = b & (LINES - 1), j = b >> LOGLINES, k = j & (NS - 1);
#pragma unroll
            for (int r = 0; r < R; ++r) v[i][r] = buf[(j + r * (L / R)) * LDL + ln];
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const int q = (k * r) << (LOGL - LOGNS - LOGR);
                C2 w = tw[q & (L / 2 - 1)];
                if (q & (L / 2)) {
                    w.x = -w.x;
                    w.y = -w.y;
                }
                if (inverse) w.y = -w.y;
                const C2 u = v[i][r];
                v[i][r].x = u.x * w.x - u.y * w.y;
                v[i][r].y = u.x * w.y + u.y * w.x;
            }
            if constexpr (R == 8) dft8(v[i], inverse);
            else if constexpr (R == 4) dft4(v[i], inverse);
            else dft2(v[i], inverse);
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < BPT; ++i) {
            const int b = threadIdx.x + 256 * i;
            if (NB % 256 != 0 && b >= NB) continue;
            const int ln = b & (LINES - 1), j = b >> LOGLINES, k = j & (NS - 1);
            const int dst = ((j >> LOGNS) << (LOGNS + LOGR)) + k;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[(dst + r * NS) * LDL + ln] = v[i][r];
        }
        __syncthreads();
        fft_stockham<C2, LOGL, LDL, LOGLINES, LOGNS + LOGR>(buf, tw, inverse);
    }
}

// 64-point FFTs of the 32 lines in buf (buf[k * LDL + line], natural order
// in and out) as 8 x 8 Cooley-Tukey: thread (line, j) takes x[8 m + j],
// m = 0..7, does an 8-point DFT, multiplies by exp(-+2 pi i j k1 / 64), and
// after one transpose through LDS does the 8-point DFT over j for k1 = its
// own index:  X[k1 + 8 k2] = sum_j W64^(j k1) W8^(j k2) sum_m x[8 m + j] W8^(m k1).
// tw[q] = exp(-2 pi i q / 64), q < 32.  Lines are the fastest thread index
// (line = t mod 32, j = t / 32), so every LDS access of a half-wavefront
// touches 16 consecutive lines of one row (no bank conflicts) and the
// twiddle reads are broadcasts.  The first write-back goes to the slots the
// thread itself read, so it needs no barrier.
template <class C2, int LDL>
__device__ inline void fft64_r8(C2 *buf, const C2 *tw, bool inverse) {
    const int ln = threadIdx.x & 31, j = threadIdx.x >> 5;
    C2 v[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) v[m] = buf[(8 * m + j) * LDL + ln];
    dft8(v, inverse);
#pragma unroll
    for (int k1 = 1; k1 < 8; ++k1) {
        const int q = j * k1;
        C2 w = tw[q & 31];
        if (q & 32) {
            w.x = -w.x;
            w.y = -w.y;
        }
        if (inverse) w.y = -w.y;
        const C2 u = v[k1];
        v[k1].x = u.x * w.x - u.y * w.y;
        v[k1].y = u.x * w.y + u.y * w.x;
    }
#pragma unroll
    for (int k1 = 0; k1 < 8; ++k1) buf[(8 * k1 + j) * LDL + ln] = v[k1];
    __syncthreads();
#pragma unroll
    for (int n2 = 0; n2 < 8; ++n2) v[n2] = buf[(8 * j + n2) * LDL + ln];
    dft8(v, inverse);
    __syncthreads();
#pragma unroll
    for (int k2 = 0; k2 < 8; ++k2) buf[(j + 8 * k2) * LDL + ln] = v[k2];
    __syncthreads();
}

// 64-point FFTs (the 8 x 8 split of fft64_r8) of two lines per thread in
// an LDS array with element k of a line at buf[off + k * KS]: slot s is the
// thread's line of index 32 s + (t mod 32), j = t / 32; act[s] says whether
// that line exists.  Every thread reaches every barrier.
template <class C2, int KS>
__device__ inline void fft64_r8_two(C2 *buf, const C2 *tw, bool inverse, const int (&off)[2],
                                    const bool (&act)[2]) {
    const int j = threadIdx.x >> 5;
    C2 v[2][8];
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
        if (!act[sl]) continue;
#pragma unroll
        for (int m = 0; m < 8; ++m) v[sl][m] = buf[off[sl] + (8 * m + j) * KS];
    }
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
        if (!act[sl]) continue;
        dft8(v[sl], inverse);
#pragma unroll
        for (int k1 = 1; k1 < 8; ++k1) {
            const int q = j * k1;
            C2 w = tw[q & 31];
            if (q & 32) {
                w.x = -w.x;
                w.y = -w.y;
            }
            if (inverse) w.y = -w.y;
            const C2 u = v[sl][k1];
            v[sl][k1].x = u.x * w.x - u.y * w.y;
            v[sl][k1].y = u.x * w.y + u.y * w.x;
        }
        // the slots this thread read: no other thread touches them
#pragma unroll
        for (int k1 = 0; k1 < 8; ++k1) buf[off[sl] + (8 * k1 + j) * KS] = v[sl][k1];
    }
    __syncthreads();
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
        if (!act[sl]) continue;
#pragma unroll
        for (int n2 = 0; n2 < 8; ++n2) v[sl][n2] = buf[off[sl] + (8 * j + n2) * KS];
        dft8(v[sl], inverse);
    }
    __syncthreads();
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
        if (!act[sl]) continue;
#pragma unroll
        for (int k2 = 0; k2 < 8; ++k2) buf[off[sl] + (j + 8 * k2) * KS] = v[sl][k2];
    }
    __syncthreads();
}

// The x and y passes of one 64 x 64 plane (one workgroup per plane and
// complex vector pair), held in LDS as buf[y * 65 + x]:
//   MODE 0 (d = 3): x forward on all 64 rows, y forward on the N + 1 band x
//            columns; stores the entries with x and y both in the band (the
//            only ones the z pass and its inverse read);
//   MODE 1 (d = 3): reads those entries (zero elsewhere), y inverse on the
//            band x columns, x inverse on all rows; stores the whole plane;
//   MODE 2 (d = 2, the plane is the grid): x forward, y forward on the band
//            columns, every entry times M (zero outside the band, so the
//            untransformed out-of-band columns become zero), y inverse on
//            the band columns, x inverse; stores the whole plane.
// The same transforms as the separate line passes, without the round trips
// of the partly transformed plane through memory.
template <class C2, int MODE>
__global__ __launch_bounds__(256) void k_fft_xy64(C2 *__restrict__ data, int N, int64_t qstr,
                                                  const C2 *__restrict__ twg,
                                                  const decltype(C2::x) *__restrict__ M, int lq,
                                                  int64_t mstr) {
    constexpr int INV = MODE == 1;
    constexpr int L = 64, LD = 65, PER = L * L / 256;
    __shared__ C2 buf[L * LD];
    __shared__ C2 tw[L / 2];
    const int t = threadIdx.x;
    if (t < L / 2) tw[t] = twg[t];
    data += (int64_t)blockIdx.y * qstr + (int64_t)blockIdx.x * (L * L);
    // batched layers: vector pair blockIdx.y belongs to layer blockIdx.y / lq
    if (MODE == 2 && mstr) M += (int64_t)(blockIdx.y / lq) * mstr;
    C2 val[PER];
#pragma unroll
    for (int it = 0; it < PER; ++it) {
        const int e = t + 256 * it;
        const int y = e >> 6, x = e & (L - 1);
        val[it].x = 0;
        val[it].y = 0;
        if (!INV || (in_band(x, N, L) && in_band(y, N, L))) val[it] = data[e];
    }
#pragma unroll
    for (int it = 0; it < PER; ++it) {
        const int e = t + 256 * it;
        buf[(e >> 6) * LD + (e & (L - 1))] = val[it];
    }
    __syncthreads();
    const int l = t & 31;
    const int rows[2] = {l * LD, (l + 32) * LD};
    const bool all[2] = {true, true};
    const int cols[2] = {band_index(l, N, L), l + 32 <= N ? band_index(l + 32, N, L) : 0};
    const bool band[2] = {l <= N, l + 32 <= N};
    if (MODE == 0 || MODE == 2) {
        fft64_r8_two<C2, 1>(buf, tw, false, rows, all);
        fft64_r8_two<C2, LD>(buf, tw, false, cols, band);
    }
    if (MODE == 2) {
        decltype(C2::x) m[PER];
#pragma unroll
        for (int it = 0; it < PER; ++it) m[it] = M[t + 256 * it];
#pragma unroll
        for (int it = 0; it < PER; ++it) {
            const int e = t + 256 * it;
            C2 &v = buf[(e >> 6) * LD + (e & (L - 1))];
            v.x *= m[it];
            v.y *= m[it];
        }
        __syncthreads();
    }
    if (MODE == 1 || MODE == 2) {
        fft64_r8_two<C2, LD>(buf, tw, true, cols, band);
        fft64_r8_two<C2, 1>(buf, tw, true, rows, all);
    }
#pragma unroll
    for (int it = 0; it < PER; ++it) {
        const int e = t + 256 * it;
        const int y = e >> 6, x = e & (L - 1);
        if (MODE != 0 || (in_band(x, N, L) && in_band(y, N, L))) data[e] = buf[y * LD + x];
    }
}

template <class T, int LOGL, int LOGLINES>
__global__ __launch_bounds__(256) void k_fft(typename Cplx<T>::type *__restrict__ data, FftPass p,
                                             const typename Cplx<T>::type *__restrict__ twg,
                                             const T *__restrict__ M) {
    using C2 = typename Cplx<T>::type;
    constexpr int L = 1 << LOGL, LINES = 1 << LOGLINES, LDL = LINES + 1;
    // 64-point lines, 32 per workgroup: 8 x 8 in registers (fft64_r8);
    // other lengths: Stockham stages of radix 8 (natural order throughout)
    constexpr bool R8 = LOGL == 6 && LOGLINES == 5;
    __shared__ C2 buf[L * LDL];
    __shared__ C2 tw[L / 2];
    for (int j = threadIdx.x; j < L / 2; j += blockDim.x) tw[j] = twg[j];
    data += (int64_t)blockIdx.y * p.qstr;
    if (p.mstr) M += (int64_t)(blockIdx.y / p.lq) * p.mstr;
    int C = 1 << p.logC;
    int64_t a0 = ((int64_t)blockIdx.x % p.nachunk) << p.logC;
    int64_t o0 = ((int64_t)blockIdx.x / p.nachunk) << p.logOB;
    if (p.flat) {
        // C = LINES and one outer per tile: the thread's line is fixed
        // (t mod LINES); number it o * A + a across the whole pass, so that
        // no workgroup holds a partial chunk of columns
        const int64_t lam = (int64_t)blockIdx.x * LINES + (threadIdx.x & (LINES - 1));
        o0 = lam / p.A;
        a0 = lam - o0 * p.A - (threadIdx.x & (LINES - 1));
    }
    // in-plane offset of column a / outer o
    auto coff = [&](int64_t a) -> int64_t { return p.abnd ? (int64_t)band_index((int)a, p.N, L) : a; };
    auto ooff = [&](int64_t o) -> int64_t {
        return (p.obnd ? (int64_t)band_index((int)o, p.N, L) : o) * p.ostr;
    };
    // all loads of the thread in flight before the first LDS write
    constexpr int PER = L * LINES / 256;
    C2 val[PER];
#pragma unroll
    for (int it = 0; it < PER; ++it) {
        const int e = threadIdx.x + 256 * it;
        const int cc = e & (C - 1);
        const int k = (e >> p.logC) & (L - 1);
        const int oo = e >> (p.logC + LOGL);
        const int64_t a = a0 + cc, o = o0 + oo;
        val[it].x = T(0);
        val[it].y = T(0);
        if (a < p.A && o < p.O && (p.mode != 1 || in_band(k, p.N, L)))
            val[it] = data[ooff(o) + (int64_t)k * p.S + coff(a)];
    }
#pragma unroll
    for (int it = 0; it < PER; ++it) {
        const int e = threadIdx.x + 256 * it;
        const int cc = e & (C - 1);
        const int k = (e >> p.logC) & (L - 1);
        const int oo = e >> (p.logC + LOGL);
        buf[k * LDL + (oo << p.logC) + cc] = val[it];
    }
    __syncthreads();
    if constexpr (R8) fft64_r8<C2, LDL>(buf, tw, p.mode == 1);
    else fft_stockham<C2, LOGL, LDL, LOGLINES>(buf, tw, p.mode == 1);
    if (p.mode == 2) {
        T m[PER];
#pragma unroll
        for (int it = 0; it < PER; ++it) {
            const int e = threadIdx.x + 256 * it;
            const int cc = e & (C - 1);
            const int k = (e >> p.logC) & (L - 1);
            const int oo = e >> (p.logC + LOGL);
            const int64_t a = a0 + cc, o = o0 + oo;
            m[it] = T(0);
            if (a < p.A && o < p.O) m[it] = M[ooff(o) + (int64_t)k * p.S + coff(a)];
        }
#pragma unroll
        for (int it = 0; it < PER; ++it) {
            const int e = threadIdx.x + 256 * it;
            const int cc = e & (C - 1);
            const int k = (e >> p.logC) & (L - 1);
            const int oo = e >> (p.logC + LOGL);
            const int i = k * LDL + (oo << p.logC) + cc;
            C2 v = buf[i];
            v.x *= m[it];
            v.y *= m[it];
            buf[i] = v;
        }
        __syncthreads();
        if constexpr (R8) fft64_r8<C2, LDL>(buf, tw, true);
        else fft_stockham<C2, LOGL, LDL, LOGLINES>(buf, tw, true);
    }
#pragma unroll
    for (int it = 0; it < PER; ++it) {
        const int e = threadIdx.x + 256 * it;
        const int cc = e & (C - 1);
        const int k = (e >> p.logC) & (L - 1);
        const int oo = e >> (p.logC + LOGL);
        const int64_t a = a0 + cc, o = o0 + oo;
        if (a < p.A && o < p.O && (p.mode != 0 || in_band(k, p.N, L)))
            data[ooff(o) + (int64_t)k * p.S + coff(a)] = buf[k * LDL + (oo << p.logC) + cc];
    }
}

// The first FFT pass fused with the cell-table gather, for blocks of 16
// vectors on grids of side L >= 128: workgroup o takes x line o (cells
// o L .. o L + L - 1) of all eight complex planes.  Each cell's patch entries
// are summed in entry order (the sums k_gather_csr writes to the grid) into
// LDS as buf[x][plane]; the eight x lines are transformed (the x pass of
// mode 0) and only their band entries are stored, so the gathered grid is
// never written to HBM nor read back.
template <class T, int LOGL>
__global__ __launch_bounds__(256) void k_gather_fftx(typename Cplx<T>::type *__restrict__ data,
                                                     int64_t G, int N, const int *__restrict__ ptr,
                                                     const int *__restrict__ ent,
                                                     const T *__restrict__ patch,
                                                     const typename Cplx<T>::type *__restrict__ twg) {
    using C2 = typename Cplx<T>::type;
    constexpr int L = 1 << LOGL, LOGLINES = 3, LINES = 8, LDL = LINES + 1;
    constexpr int BS = 16, VPL = 4, NG = BS / VPL, NB = csr_batch<T, VPL>();
    constexpr int ITEMS = L * NG / 256;   // (cell, vector group) items per thread
    __shared__ C2 buf[L * LDL];
    __shared__ C2 tw[L / 2];
    for (int j = threadIdx.x; j < L / 2; j += 256) tw[j] = twg[j];
    const int64_t c0 = (int64_t)blockIdx.x * L;
    int e0[ITEMS], e1[ITEMS];
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
        const int x = (threadIdx.x + 256 * it) / NG;
        e0[it] = ptr[c0 + x];
        e1[it] = ptr[c0 + x + 1];
    }
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
        const int i = threadIdx.x + 256 * it, x = i / NG, vg = i % NG;
        T acc[VPL];
#pragma unroll
        for (int v = 0; v < VPL; ++v) acc[v] = T(0);
        for (int e = e0[it]; e < e1[it]; e += NB) {
            int idx[NB];
#pragma unroll
            for (int u = 0; u < NB; ++u) idx[u] = e + u < e1[it] ? ent[e + u] : -1;
            T h[NB][VPL];
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                if (idx[u] >= 0) load_vec<T, VPL>(patch + (int64_t)idx[u] * BS + vg * VPL, h[u]);
                else
#pragma unroll
                    for (int v = 0; v < VPL; ++v) h[u][v] = T(0);
            }
#pragma unroll
            for (int u = 0; u < NB; ++u)
                if (idx[u] >= 0)
#pragma unroll
                    for (int v = 0; v < VPL; ++v) acc[v] += h[u][v];
        }
        // vectors 4 vg .. 4 vg + 3: planes 2 vg and 2 vg + 1 (re, im)
        C2 a, b;
        a.x = acc[0];
        a.y = acc[1];
        b.x = acc[2];
        b.y = acc[3];
        buf[x * LDL + 2 * vg] = a;
        buf[x * LDL + 2 * vg + 1] = b;
    }
    __syncthreads();
    fft_stockham<C2, LOGL, LDL, LOGLINES>(buf, tw, false);
#pragma unroll
    for (int it = 0; it < L * LINES / 256; ++it) {
        const int e = threadIdx.x + 256 * it;
        const int q = e >> LOGL, k = e & (L - 1);
        if (in_band(k, N, L)) data[(int64_t)q * G + c0 + k] = buf[k * LDL + q];
    }
}

// Interpolation: one thread per (point, vector group); window weights in
// registers, the footprint read from the grid.
template <class T, int D, int VPL>
__global__ __launch_bounds__(256) void k_interp(Geom g, const double *__restrict__ u64,
                                                const int *__restrict__ c32,
                                                const float *__restrict__ f32,
                                                const T *__restrict__ grid, int bg, T beta,
                                                T *__restrict__ Fs) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= g.n) return;
    const int v0 = blockIdx.y * VPL;
    const int w = g.w;
    const T two_over_w = T(2) / (T)w;
    int64_t G = g.nos;
    if (D > 1) G *= g.nos;
    if (D > 2) G *= g.nos;
    // innermost dimension's weights in registers (compile-time indices);
    // the outer dimensions' weights are evaluated in their loops
    T phi0[16];
    int s0[3] = {0, 0, 0};
    T fr[3] = {T(0), T(0), T(0)};
    for (int t = 0; t < D; ++t) {
        int cell;
        point_coord<T>(u64, c32, f32, (int64_t)t * g.n + p, cell, fr[t]);
        s0[t] = cell - w / 2 + 1;
    }
#pragma unroll
    for (int k = 0; k < 16; ++k)
        phi0[k] = k < w ? es_psi<T>((T)(w / 2 - 1 - k) + fr[0], two_over_w, beta) : T(0);
    T acc[VPL];
#pragma unroll
    for (int v = 0; v < VPL; ++v) acc[v] = T(0);
    const int n2 = D > 2 ? w : 1, n1 = D > 1 ? w : 1;
    for (int k2 = 0; k2 < n2; ++k2) {
        const T w2 = D > 2 ? es_psi<T>((T)(w / 2 - 1 - k2) + fr[2], two_over_w, beta) : T(1);
        for (int k1 = 0; k1 < n1; ++k1) {
            T wyz = w2;
            int64_t base = s0[0];
            if (D > 1) {
                wyz *= es_psi<T>((T)(w / 2 - 1 - k1) + fr[1], two_over_w, beta);
                base += (int64_t)g.nos * (s0[1] + k1);
            }
            if (D > 2) base += (int64_t)g.nos * g.nos * (s0[2] + k2);
#pragma unroll
            for (int k0 = 0; k0 < 16; ++k0) {
                if (k0 < w) {
                    const T wgt = wyz * phi0[k0];
                    T h[VPL];
                    grid_load<T, VPL>(grid, G, base + k0, v0, h);
#pragma unroll
                    for (int v = 0; v < VPL; ++v) acc[v] += wgt * h[v];
                }
            }
        }
    }
    store_vec<T, VPL>(Fs + (int64_t)g.perm[p] * g.bs + v0, acc);
}

// ------------------------------------------------------------------------------
// host side
// ------------------------------------------------------------------------------
static void gauss_legendre(int q, std::vector<double> &x, std::vector<double> &w) {
    x.resize(q);
    w.resize(q);
    for (int i = 0; i < q; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (q + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= q; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            double dp = q * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= q; ++k) {
            double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        double dp = q * (z * p1 - p0) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// Two-point Taylor polynomial on t in [0,1] (t = (r - r0)/eps_B), degree
// 2p-1: derivatives 0..p-1 equal eps_B^j K^(j)(r0) at t=0; value K(1/2) and
// zero derivatives 1..p-1 at t=1.  K(r) = exp(-r^2/s^2) has derivatives
// K^(j)(r) = (-1/s)^j H_j(r/s) K(r) with physicists' Hermite H_j.
static KRParams make_kr(double sigma_s, double eps_B, int p) {
    KRParams kr{};
    kr.sigma2 = sigma_s * sigma_s;
    kr.r0 = 0.5 - eps_B;
    kr.epsB = eps_B;
    kr.kend = std::exp(-0.25 / kr.sigma2);
    const int n2 = 2 * p;
    kr.ncoef = n2;
    double uu = kr.r0 / sigma_s;
    double K0 = std::exp(-uu * uu);
    std::vector<double> H(p + 1);
    H[0] = 1.0;
    if (p >= 1) H[1] = 2.0 * uu;
    for (int j = 1; j < p; ++j) H[j + 1] = 2.0 * uu * H[j] - 2.0 * j * H[j - 1];
    std::vector<double> A(n2 * n2, 0.0), rhs(n2, 0.0);
    auto fact = [](int j) { double f = 1; for (int i = 2; i <= j; ++i) f *= i; return f; };
    // t = 0 conditions: coef[j] * j! = eps^j K^(j)(r0)
    for (int j = 0; j < p; ++j) {
        A[j * n2 + j] = fact(j);
        rhs[j] = std::pow(eps_B, j) * std::pow(-1.0 / sigma_s, j) * H[j] * K0;
    }
    // t = 1: value kend, derivatives 1..p-1 zero
    for (int j = 0; j < p; ++j) {
        int row = p + j;
        for (int i = j; i < n2; ++i) {
            double c = 1.0;  // i!/(i-j)!
            for (int m = 0; m < j; ++m) c *= (i - m);
            A[row * n2 + i] = c;
        }
        rhs[row] = (j == 0) ? kr.kend : 0.0;
    }
    // Gaussian elimination with partial pivoting
    for (int c = 0; c < n2; ++c) {
        int piv = c;
        for (int r = c + 1; r < n2; ++r)
            if (std::fabs(A[r * n2 + c]) > std::fabs(A[piv * n2 + c])) piv = r;
        if (piv != c) {
            for (int k = 0; k < n2; ++k) std::swap(A[c * n2 + k], A[piv * n2 + k]);
            std::swap(rhs[c], rhs[piv]);
        }
        for (int r = c + 1; r < n2; ++r) {
            double f = A[r * n2 + c] / A[c * n2 + c];
            for (int k = c; k < n2; ++k) A[r * n2 + k] -= f * A[c * n2 + k];
            rhs[r] -= f * rhs[c];
        }
    }
    for (int r = n2 - 1; r >= 0; --r) {
        double acc = rhs[r];
        for (int k = r + 1; k < n2; ++k) acc -= A[r * n2 + k] * kr.coef[k];
        kr.coef[r] = acc / A[r * n2 + r];
    }
    return kr;
}

// Smallest power-of-two bandwidth (16..256) whose dropped Gaussian Fourier
// tail, about 2 d sqrt(pi) sigma exp(-pi^2 sigma^2 N^2 / 4), is below a
// precision-dependent bound.
int nfft_auto_bandwidth(double sigma_s, int d, int prec) {
    const double tol = prec == 64 ? 1e-13 : 1e-8;
    int N = 16;
    while (N < 256) {
        double x = M_PI * sigma_s * N / 2.0;
        if (2.0 * d * std::sqrt(M_PI) * sigma_s * std::exp(-x * x) <= tol) break;
        N *= 2;
    }
    return N;
}

// Two-level fixed-order reduction lists for runs whose patch is the sum of
// several scratch slots: multi = (run, first scratch slot, slot count).
// Level 1 sums groups of <= 32 slots (straight into the run's slot when one
// group covers it); level 2 sums a run's group results.
static void reduction_lists(const std::vector<int4> &multi, std::vector<int4> &g1,
                            std::vector<int4> &g2) {
    for (const int4 &m : multi) {
        const int ng = (m.z + 31) / 32;
        for (int q = 0; q < ng; ++q)
            g1.push_back(make_int4(m.y + 32 * q, std::min(32, m.z - 32 * q),
                                   ng == 1 ? m.x : m.y + 32 * q, 0));
        if (ng > 1) g2.push_back(make_int4(m.x, m.y, ng, 0));
    }
}

// Chunks per task (2..16) for which the runs' tasks, dispatched in order of
// decreasing size onto `slots` equal slots, finish earliest; `over` is a
// task's fixed cost in chunks (set-up, patch load or store).
static int best_task_chunks(const std::vector<int> &nch, int slots, double over) {
    int best_c = 4;
    double best = INFINITY;
    for (int c = 2; c <= 16; ++c) {
        std::vector<int> sizes;
        for (int k : nch)
            for (int j = 0; j < k; j += c) sizes.push_back(std::min(c, k - j));
        std::stable_sort(sizes.begin(), sizes.end(), std::greater<int>());
        std::priority_queue<double, std::vector<double>, std::greater<double>> q;
        for (int i = 0; i < slots; ++i) q.push(0.0);
        double end = 0.0;
        for (int z : sizes) {
            const double t = q.top() + z + over;
            q.pop();
            q.push(t);
            end = std::max(end, t);
        }
        if (end < best * 0.999) {
            best = end;
            best_c = c;
        }
    }
    return best_c;
}

// The runs cut into tasks of at most c chunks of 64 points, larger tasks
// first (stable: ties keep run order).  With `slots_base` >= 0, a run cut
// into several tasks gets consecutive scratch patch slots from slots_base on
// (in task order) and a multi entry (run, first slot, tasks); a run of one
// task writes its own slot.
static std::vector<int4> cut_runs(const std::vector<unsigned> &key,
                                  const std::vector<unsigned> &start,
                                  const std::vector<unsigned> &count, int c, int slots_base,
                                  std::vector<int4> &multi, int &scr) {
    const int runs = (int)key.size();
    std::vector<int4> seg;
    std::vector<int> size;
    scr = 0;
    for (int r = 0; r < runs; ++r) {
        const int nch = (int)((count[r] + 63) / 64);
        const int nt = (nch + c - 1) / c;
        const int base = slots_base + scr;
        for (int k = 0; k < nt; ++k) {
            const int64_t p0 = (int64_t)k * c * 64;
            const int64_t cnt = std::min<int64_t>((int64_t)count[r] - p0, (int64_t)c * 64);
            seg.push_back(make_int4((int)key[r], (int)(start[r] + p0), (int)cnt,
                                    nt == 1 ? r : base + k));
            size.push_back((int)((cnt + 63) / 64));
        }
        if (nt > 1 && slots_base >= 0) {
            multi.push_back(make_int4(r, base, nt, 0));
            scr += nt;
        }
    }
    std::vector<int> ord(seg.size());
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return size[x] > size[y]; });
    std::vector<int4> sorted(seg.size());
    for (size_t i = 0; i < ord.size(); ++i) sorted[i] = seg[ord[i]];
    return sorted;
}

// Matrix-core schedules of a d = 3 plan (see NfftPlan::seg and ::iseg):
// spreading on two wavefronts per SIMD (task overhead: its patch store,
// about half a chunk), interpolation on three (overhead: its patch load,
// about one chunk).  Scratch slots of the spreading start at
// runs + nscratch, after the task list's own.
static void build_mfma_schedules(NfftPlan &P, const std::vector<unsigned> &key,
                                 const std::vector<unsigned> &start,
                                 const std::vector<unsigned> &count, hipStream_t s) {
    const int runs = (int)key.size();
    int dev = 0, cus = 0;
    MLG_HIP(hipGetDevice(&dev));
    MLG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int simds = std::max(1, cus) * 4;
    std::vector<int> nch(runs);
    for (int r = 0; r < runs; ++r) nch[r] = (int)((count[r] + 63) / 64);
    std::vector<int4> multi, unused;
    int scr = 0, iscr = 0;
    const int cs = best_task_chunks(nch, 2 * simds, 0.5);
    std::vector<int4> seg = cut_runs(key, start, count, cs, runs + P.nscratch, multi, scr);
    const int ci = best_task_chunks(nch, 3 * simds, 1.0);
    std::vector<int4> iseg = cut_runs(key, start, count, ci, -1, unused, iscr);
    std::vector<int4> g1, g2;
    reduction_lists(multi, g1, g2);
    P.nseg = (int)seg.size();
    P.seg_chunks = cs;
    P.nsscr = scr;
    P.nsred1 = (int)g1.size();
    P.nsred2 = (int)g2.size();
    upload(P.seg, seg.data(), seg.size(), false, s);
    upload(P.sred1, g1.data(), g1.size(), false, s);
    upload(P.sred2, g2.data(), g2.size(), false, s);
    P.niseg = (int)iseg.size();
    P.iseg_chunks = ci;
    upload(P.iseg, iseg.data(), iseg.size(), false, s);
}

template <class F>
static void with_temp(DevBuf<char> &tmp, size_t bytes, F f) {
    tmp.ensure(bytes ? bytes : 1);
    f(tmp.p);
}

void nfft_plan_layer(Layer &L, const double *pts, hipStream_t s) {
    NfftPlan &P = L.nf;
    const int d = L.d;
    const int64_t n = L.n;
    MLG_REQUIRE(d >= 1 && d <= 3, MLG_ERR_RANGE, "NFFT layers need d in 1..3");
    MLG_REQUIRE(L.kp.N == 0 || (is_pow2(L.kp.N) && L.kp.N >= 8 && L.kp.N <= 256), MLG_ERR_RANGE,
                "NFFT bandwidth N must be 0 (automatic) or a power of two in 8..256");
    MLG_REQUIRE(L.kp.eps_B > 0.0 && L.kp.eps_B < 0.25, MLG_ERR_RANGE, "eps_B must be in (0, 1/4)");
    MLG_REQUIRE(L.kp.p_reg >= 1 && L.kp.p_reg <= 12, MLG_ERR_RANGE, "p_reg must be in 1..12");
    MLG_REQUIRE(n < (int64_t)1 << 31, MLG_ERR_RANGE, "NFFT layers need n < 2^31");
    P.d = d;
    P.n = n;
    MLG_REQUIRE(L.kp.bin == 0 || L.kp.bin == 1 || L.kp.bin == 2 || L.kp.bin == 4, MLG_ERR_RANGE,
                "bin must be 0 (automatic), 1, 2 or 4");
    P.B = L.kp.bin > 0 ? L.kp.bin : 1;
    P.eps_B = L.kp.eps_B;
    P.p_reg = L.kp.p_reg;

    // --- input check, torus scaling (bounding-box centre, radius, scale) ---
    {
        DevBuf<int> flag(1);
        MLG_HIP(hipMemsetAsync(flag.p, 0, 4, s));
        hipLaunchKernelGGL(k_check_finite, dim3(ceil_div(n * d, 256)), dim3(256), 0, s, n * d, pts,
                           flag.p);
        MLG_LAUNCH_CHECK();
        int hf = 0;
        MLG_HIP(hipMemcpyAsync(&hf, flag.p, 4, hipMemcpyDeviceToHost, s));
        MLG_HIP(hipStreamSynchronize(s));
        MLG_REQUIRE(hf == 0, MLG_ERR_ARG, "point coordinates must be finite");
    }
    const int nblk = std::min(1024, ceil_div(n, 256));
    DevBuf<double> part((size_t)nblk * 6);
    hipLaunchKernelGGL(k_minmax, dim3(nblk), dim3(256), 0, s, n, d, pts, part.p);
    MLG_LAUNCH_CHECK();
    std::vector<double> hp((size_t)nblk * 6);
    MLG_HIP(hipMemcpyAsync(hp.data(), part.p, hp.size() * 8, hipMemcpyDeviceToHost, s));
    MLG_HIP(hipStreamSynchronize(s));
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int b = 0; b < nblk; ++b)
        for (int t = 0; t < d; ++t) {
            mn[t] = std::fmin(mn[t], hp[b * 6 + t]);
            mx[t] = std::fmax(mx[t], hp[b * 6 + 3 + t]);
        }
    for (int t = 0; t < 3; ++t) P.center[t] = t < d ? 0.5 * (mn[t] + mx[t]) : 0.0;
    for (int t = 0; t < d; ++t)
        MLG_REQUIRE(std::isfinite(mn[t]) && std::isfinite(mx[t]), MLG_ERR_ARG,
                    "point coordinates must be finite");
    hipLaunchKernelGGL(k_maxrad, dim3(nblk), dim3(256), 0, s, n, d, pts, P.center[0], P.center[1],
                       P.center[2], part.p);
    MLG_LAUNCH_CHECK();
    MLG_HIP(hipMemcpyAsync(hp.data(), part.p, (size_t)nblk * 8, hipMemcpyDeviceToHost, s));
    MLG_HIP(hipStreamSynchronize(s));
    double r2 = 0.0;
    for (int b = 0; b < nblk; ++b) r2 = std::fmax(r2, hp[b]);
    const double R = std::sqrt(r2);
    const double rho = 0.25 - 0.5 * P.eps_B;
    P.scale = R > 0 ? rho / R : 1.0;
    P.sigma_s = P.scale * L.sigma;
    P.N = L.kp.N > 0 ? L.kp.N : nfft_auto_bandwidth(P.sigma_s, d, L.kp.precision);
    P.nos = 2 * P.N;

    // --- grid coordinates, keys, sort, runs of equal bins (for bin edge P.B) ---
    DevBuf<double> uun((size_t)d * n);
    DevBuf<unsigned> keys(n), skeys(n);
    DevBuf<int> idx(n);
    P.perm.alloc(n);
    P.u64.alloc((size_t)d * n);
    P.c32.alloc((size_t)d * n);
    P.f32.alloc((size_t)d * n);
    DevBuf<unsigned> ukeys(n), counts(n), runs_dev(1);
    DevBuf<char> tmp;
    auto sort_bins = [&]() -> unsigned {
        P.nb = P.nos / P.B;
        P.nbins = 1;
        for (int t = 0; t < d; ++t) P.nbins *= P.nb;
        hipLaunchKernelGGL(k_coords_keys, dim3(ceil_div(n, 256)), dim3(256), 0, s, n, d, pts,
                           P.center[0], P.center[1], P.center[2], P.scale, P.nos, P.B, P.nb, uun.p,
                           keys.p, idx.p);
        MLG_LAUNCH_CHECK();
        unsigned endbit = 1;
        while (((int64_t)1 << endbit) < P.nbins) ++endbit;
        size_t tbytes = 0;
        MLG_HIP(rocprim::radix_sort_pairs(nullptr, tbytes, keys.p, skeys.p, idx.p, P.perm.p,
                                          (unsigned)n, 0u, endbit, s));
        tmp.ensure(tbytes + 1);
        MLG_HIP(rocprim::radix_sort_pairs(tmp.p, tbytes, keys.p, skeys.p, idx.p, P.perm.p,
                                          (unsigned)n, 0u, endbit, s));
        hipLaunchKernelGGL(k_gather_coords, dim3(ceil_div(n, 256)), dim3(256), 0, s, n, d, P.nos,
                           uun.p, P.perm.p, P.u64.p, P.c32.p, P.f32.p);
        MLG_LAUNCH_CHECK();
        tbytes = 0;
        MLG_HIP(rocprim::run_length_encode(nullptr, tbytes, skeys.p, (unsigned)n, ukeys.p, counts.p,
                                           runs_dev.p, s));
        tmp.ensure(tbytes + 1);
        MLG_HIP(rocprim::run_length_encode(tmp.p, tbytes, skeys.p, (unsigned)n, ukeys.p, counts.p,
                                           runs_dev.p, s));
        unsigned r = 0;
        MLG_HIP(hipMemcpyAsync(&r, runs_dev.p, 4, hipMemcpyDeviceToHost, s));
        MLG_HIP(hipStreamSynchronize(s));
        return r;
    };
    unsigned runs = sort_bins();
    // Automatic bin edge (FP32): every occupied bin costs a patch and at
    // least one 64-point chunk of matrix-core work, so the edge doubles
    // while the occupied bins hold fewer than kAutoBinPoints points on
    // average and the larger patch still fits the matrix-core kernels and
    // the bandwidth (bin + w/2 <= N/2).  Only the grouping of points
    // changes, not what is summed.
    if (L.kp.bin == 0 && L.kp.precision == 32) {
        const int w = L.kp.window > 0 ? L.kp.window : 6;
        while (P.B < 4 && (int64_t)n < kAutoBinPoints * (int64_t)runs) {
            const int B2 = 2 * P.B;
            if (B2 + w / 2 > P.N / 2 || !mfma_patch_ok(d, B2 + w - 1)) break;
            P.B = B2;
            runs = sort_bins();
        }
    }

    DevBuf<unsigned> run_start(runs + 1), ntask(runs + 1), task_first(runs + 1), scr(runs + 1),
        scr_first(runs + 1), ism(runs + 1), multi_idx(runs + 1);
    auto xscan = [&](const unsigned *in, unsigned *out, size_t cnt) {
        size_t tb = 0;
        MLG_HIP(rocprim::exclusive_scan(nullptr, tb, in, out, 0u, cnt, rocprim::plus<unsigned>(), s));
        tmp.ensure(tb + 1);
        MLG_HIP(rocprim::exclusive_scan(tmp.p, tb, in, out, 0u, cnt, rocprim::plus<unsigned>(), s));
    };
    xscan(counts.p, run_start.p, runs);
    hipLaunchKernelGGL(k_task_counts, dim3(ceil_div(runs, 256)), dim3(256), 0, s, (int)runs,
                       counts.p, kMaxTaskPoints, ntask.p);
    MLG_LAUNCH_CHECK();
    // ntask[runs] = 0 so that the scans give totals at index runs
    MLG_HIP(hipMemsetAsync(ntask.p + runs, 0, 4, s));
    xscan(ntask.p, task_first.p, (size_t)runs + 1);
    hipLaunchKernelGGL(k_scr_counts, dim3(ceil_div(runs + 1, 256)), dim3(256), 0, s, (int)runs,
                       ntask.p, scr.p, ism.p);
    MLG_LAUNCH_CHECK();
    xscan(scr.p, scr_first.p, (size_t)runs + 1);
    xscan(ism.p, multi_idx.p, (size_t)runs + 1);
    unsigned tot[3] = {0, 0, 0};
    MLG_HIP(hipMemcpyAsync(&tot[0], task_first.p + runs, 4, hipMemcpyDeviceToHost, s));
    MLG_HIP(hipMemcpyAsync(&tot[1], scr_first.p + runs, 4, hipMemcpyDeviceToHost, s));
    MLG_HIP(hipMemcpyAsync(&tot[2], multi_idx.p + runs, 4, hipMemcpyDeviceToHost, s));
    MLG_HIP(hipStreamSynchronize(s));
    P.nruns = (int)runs;
    P.run_key.alloc(runs > 0 ? runs : 1);
    MLG_HIP(hipMemcpyAsync(P.run_key.p, ukeys.p, sizeof(unsigned) * runs, hipMemcpyDeviceToDevice, s));
    P.ntasks = (int)tot[0];
    P.nscratch = (int)tot[1];
    P.nmulti = (int)tot[2];
    P.tasks.alloc(P.ntasks);
    P.multi.alloc(P.nmulti > 0 ? P.nmulti : 1);
    P.bin_run.alloc(P.nbins);
    MLG_HIP(hipMemsetAsync(P.bin_run.p, 0xff, sizeof(int) * P.nbins, s));   // -1: empty bin
    hipLaunchKernelGGL(k_fill_tasks, dim3(ceil_div(runs, 256)), dim3(256), 0, s, (int)runs, ukeys.p,
                       counts.p, run_start.p, task_first.p, scr_first.p, multi_idx.p, kMaxTaskPoints,
                       P.tasks.p, P.bin_run.p, P.multi.p);
    MLG_LAUNCH_CHECK();
    // fixed two-level reduction order for runs cut into several tasks
    if (P.nmulti > 0) {
        std::vector<int4> hm(P.nmulti);
        MLG_HIP(hipMemcpyAsync(hm.data(), P.multi.p, sizeof(int4) * P.nmulti, hipMemcpyDeviceToHost, s));
        MLG_HIP(hipStreamSynchronize(s));
        std::vector<int4> g1;
        std::vector<int4> g2;
        reduction_lists(hm, g1, g2);
        P.nred1 = (int)g1.size();
        P.nred2 = (int)g2.size();
        upload(P.red1, g1.data(), g1.size(), false, s);
        upload(P.red2, g2.data(), g2.size(), false, s);
    }
    // balanced spreading schedule for d = 3 plans whose runs hold a full
    // chunk of points on average (the matrix-core spreading's work unit)
    if (d == 3 && runs > 0 && (int64_t)n >= 64 * (int64_t)runs) {
        std::vector<unsigned> hkey(runs), hst(runs), hcnt(runs);
        MLG_HIP(hipMemcpyAsync(hkey.data(), ukeys.p, 4 * (size_t)runs, hipMemcpyDeviceToHost, s));
        MLG_HIP(hipMemcpyAsync(hst.data(), run_start.p, 4 * (size_t)runs, hipMemcpyDeviceToHost, s));
        MLG_HIP(hipMemcpyAsync(hcnt.data(), counts.p, 4 * (size_t)runs, hipMemcpyDeviceToHost, s));
        MLG_HIP(hipStreamSynchronize(s));
        build_mfma_schedules(P, hkey, hst, hcnt, s);
    }
    P.SB = std::min(8, P.nb);
    P.nsb = (P.nb + P.SB - 1) / P.SB;
    int64_t nsbd = 1;
    for (int t = 0; t < d; ++t) nsbd *= P.nsb;
    P.occ.alloc(nsbd);
    MLG_HIP(hipMemsetAsync(P.occ.p, 0, nsbd, s));
    hipLaunchKernelGGL(k_superbins, dim3(ceil_div(runs, 256)), dim3(256), 0, s, (int)runs, ukeys.p, d,
                       P.nb, P.SB, P.nsb, P.occ.p);
    MLG_LAUNCH_CHECK();

    // --- kernel Fourier coefficients b^ (FP64) ---
    const KRParams kr = make_kr(P.sigma_s, P.eps_B, P.p_reg);
    int64_t Nd = 1;
    for (int t = 0; t < d; ++t) Nd *= P.N;
    DevBuf<double> S(Nd), S2(Nd);
    hipLaunchKernelGGL(k_sample_kr, dim3(ceil_div(Nd, 256)), dim3(256), 0, s, d, P.N, kr, S.p);
    MLG_LAUNCH_CHECK();
    double *src = S.p, *dst = S2.p;
    for (int t = 0; t < d; ++t) {
        double sc = (t == d - 1) ? std::pow((double)P.N, -d) : 1.0;
        hipLaunchKernelGGL(k_cos_dft, dim3(ceil_div(Nd, 256)), dim3(256), 0, s, d, P.N, t, src, dst,
                           sc);
        MLG_LAUNCH_CHECK();
        std::swap(src, dst);
    }
    P.bhat = (src == S.p) ? std::move(S) : std::move(S2);

    // --- FFT twiddles ---
    P.tw32.alloc(P.nos / 2);
    P.tw64.alloc(P.nos / 2);
    hipLaunchKernelGGL(k_twiddles, dim3(ceil_div(P.nos / 2, 256)), dim3(256), 0, s, P.nos, P.tw32.p,
                       P.tw64.p);
    MLG_LAUNCH_CHECK();
    MLG_HIP(hipStreamSynchronize(s));
}

void nfft_make_window(const Layer &L, NfftWindow &W, int w, int prec, int bs, hipStream_t s) {
    const NfftPlan &P = L.nf;
    MLG_REQUIRE(w >= 2 && w <= 16 && w % 2 == 0, MLG_ERR_RANGE, "window must be even, 2..16");
    MLG_REQUIRE(P.B + w / 2 <= P.N / 2, MLG_ERR_RANGE,
                "window too wide for the bandwidth: need bin + w/2 <= N/2");
    MLG_REQUIRE(P.B + w - 1 <= kMaxP, MLG_ERR_RANGE, "bin + window - 1 exceeds 20");
    W.w = w;
    W.beta = 2.30 * w;
    W.prec = prec;
    std::vector<double> gx, gw;
    gauss_legendre(kGL, gx, gw);
    DevBuf<double> dgx(kGL), dgw(kGL), ph(P.N / 2 + 1);
    MLG_HIP(hipMemcpyAsync(dgx.p, gx.data(), kGL * 8, hipMemcpyHostToDevice, s));
    MLG_HIP(hipMemcpyAsync(dgw.p, gw.data(), kGL * 8, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_window_hat, dim3(1), dim3(256), 0, s, P.N, P.nos, w, W.beta, dgx.p, dgw.p,
                       kGL, ph.p);
    MLG_LAUNCH_CHECK();
    int64_t G = 1;
    for (int t = 0; t < P.d; ++t) G *= P.nos;
    if (prec == 64) {
        W.M64.alloc(G);
        hipLaunchKernelGGL(k_make_M<double>, dim3(ceil_div(G, 256)), dim3(256), 0, s, P.d, P.N,
                           P.nos, P.bhat.p, ph.p, W.M64.p);
    } else {
        W.M32.alloc(G);
        hipLaunchKernelGGL(k_make_M<float>, dim3(ceil_div(G, 256)), dim3(256), 0, s, P.d, P.N, P.nos,
                           P.bhat.p, ph.p, W.M32.p);
    }
    MLG_LAUNCH_CHECK();
    // grid cell -> patch entry table
    W.csr = false;
    const int Pside = P.B + w - 1;
    int64_t PDw = 1;
    for (int t = 0; t < P.d; ++t) PDw *= Pside;
    const int64_t total = (int64_t)P.nruns * PDw;
    if (total > 0 && total <= ((int64_t)1 << 28) && G < ((int64_t)1 << 31)) {
        DevBuf<unsigned> keys(total), skeys(total);
        DevBuf<int> vals(total);
        W.cell_ent.alloc(total);
        hipLaunchKernelGGL(k_csr_keys, dim3(ceil_div(total, 256)), dim3(256), 0, s, total, P.d, (int)PDw,
                           Pside, P.nos, P.B, P.nb, w, P.run_key.p, keys.p, vals.p);
        MLG_LAUNCH_CHECK();
        unsigned endbit = 1;
        while (((int64_t)1 << endbit) < G) ++endbit;
        DevBuf<char> tmp;
        size_t tb = 0;
        MLG_HIP(rocprim::radix_sort_pairs(nullptr, tb, keys.p, skeys.p, vals.p, W.cell_ent.p,
                                          (unsigned)total, 0u, endbit, s));
        tmp.ensure(tb + 1);
        MLG_HIP(rocprim::radix_sort_pairs(tmp.p, tb, keys.p, skeys.p, vals.p, W.cell_ent.p,
                                          (unsigned)total, 0u, endbit, s));
        DevBuf<unsigned> ucell(total), ucnt(total), nu_d(1);
        tb = 0;
        MLG_HIP(rocprim::run_length_encode(nullptr, tb, skeys.p, (unsigned)total, ucell.p, ucnt.p,
                                           nu_d.p, s));
        tmp.ensure(tb + 1);
        MLG_HIP(rocprim::run_length_encode(tmp.p, tb, skeys.p, (unsigned)total, ucell.p, ucnt.p,
                                           nu_d.p, s));
        unsigned nu = 0;
        MLG_HIP(hipMemcpyAsync(&nu, nu_d.p, 4, hipMemcpyDeviceToHost, s));
        MLG_HIP(hipStreamSynchronize(s));
        DevBuf<int> dense(G + 1);
        MLG_HIP(hipMemsetAsync(dense.p, 0, sizeof(int) * (G + 1), s));
        hipLaunchKernelGGL(k_scatter_counts, dim3(ceil_div(nu, 256)), dim3(256), 0, s, (int)nu, ucell.p,
                           ucnt.p, dense.p);
        MLG_LAUNCH_CHECK();
        W.cell_ptr.alloc(G + 1);
        tb = 0;
        MLG_HIP(rocprim::exclusive_scan(nullptr, tb, dense.p, W.cell_ptr.p, 0, (size_t)G + 1,
                                        rocprim::plus<int>(), s));
        tmp.ensure(tb + 1);
        MLG_HIP(rocprim::exclusive_scan(tmp.p, tb, dense.p, W.cell_ptr.p, 0, (size_t)G + 1,
                                        rocprim::plus<int>(), s));
        W.csr = true;
    }
    MLG_HIP(hipStreamSynchronize(s));
}

static int patch_side(const NfftPlan &P, const NfftWindow &W) { return P.B + W.w - 1; }

static int patch_cells(const NfftPlan &P, const NfftWindow &W) {
    int pd = 1;
    for (int t = 0; t < P.d; ++t) pd *= patch_side(P, W);
    return pd;
}

// The d = 3 matrix-core spreading (FP32, blocks of 16 vectors, patches of
// at most 7^3 cells) runs the balanced schedule when the plan has one.
static bool uses_spread_schedule(const NfftPlan &P, const NfftWindow &W, int bs) {
    return P.nseg > 0 && P.d == 3 && W.prec == 32 && bs % 16 == 0 &&
           mfma_patch_ok(3, patch_side(P, W));
}

size_t nfft_patch_elems(const NfftPlan &P, const NfftWindow &W, int bs) {
    const size_t slots = (size_t)P.nruns + P.nscratch + (uses_spread_schedule(P, W, bs) ? P.nsscr : 0);
    return (size_t)patch_cells(P, W) * bs * slots;
}

size_t nfft_grid_elems(const NfftPlan &P, int bs) {
    size_t g = 1;
    for (int t = 0; t < P.d; ++t) g *= (size_t)P.nos;
    return g * (size_t)(bs < 2 ? 2 : bs);
}

template <class T>
static const T *mult_of(const NfftWindow &W);
template <>
const float *mult_of<float>(const NfftWindow &W) { return W.M32.p; }
template <>
const double *mult_of<double>(const NfftWindow &W) { return W.M64.p; }
template <class T>
static const typename Cplx<T>::type *tw_of(const NfftPlan &P);
template <>
const float2 *tw_of<float>(const NfftPlan &P) { return P.tw32.p; }
template <>
const double2 *tw_of<double>(const NfftPlan &P) { return P.tw64.p; }

static int ilog2(int64_t v) {
    int l = 0;
    while (((int64_t)1 << l) < v) ++l;
    return l;
}

// Lines per workgroup: 2^LOGLINES with L * LINES = 2048 complex values (at
// most 64 lines).
template <class T, int LOGL>
static void fft_launch(FftPass p, int nq, typename Cplx<T>::type *grid,
                       const typename Cplx<T>::type *tw, const T *M, hipStream_t s) {
    constexpr int LOGLINES = 11 - LOGL > 6 ? 6 : 11 - LOGL;
    const int logA = ilog2(p.A);
    p.logC = std::min(logA, LOGLINES);
    p.logOB = LOGLINES - p.logC;
    p.nachunk = (p.A + ((int64_t)1 << p.logC) - 1) >> p.logC;
    const int64_t nob = (p.O + ((int64_t)1 << p.logOB) - 1) >> p.logOB;
    // a full-width tile (one outer, LINES columns) numbers its lines across
    // the outers instead of padding the last column chunk of every outer
    p.flat = p.logC == LOGLINES && p.A > 1;
    const int64_t nblk = p.flat ? (p.O * p.A + (1 << LOGLINES) - 1) >> LOGLINES : p.nachunk * nob;
    MLG_REQUIRE(nblk < ((int64_t)1 << 31) && nq <= 65535, MLG_ERR_RANGE, "FFT grid too large");
    hipLaunchKernelGGL((k_fft<T, LOGL, LOGLINES>), dim3((unsigned)nblk, nq), dim3(256), 0, s, grid, p, tw, M);
    MLG_LAUNCH_CHECK();
}

template <class T>
static void fft_dispatch(const NfftPlan &P, const FftPass &p, int nq, typename Cplx<T>::type *grid,
                         const T *M, hipStream_t s) {
    const auto *tw = tw_of<T>(P);
    switch (ilog2(P.nos)) {
        case 4: fft_launch<T, 4>(p, nq, grid, tw, M, s); break;
        case 5: fft_launch<T, 5>(p, nq, grid, tw, M, s); break;
        case 6: fft_launch<T, 6>(p, nq, grid, tw, M, s); break;
        case 7: fft_launch<T, 7>(p, nq, grid, tw, M, s); break;
        case 8: fft_launch<T, 8>(p, nq, grid, tw, M, s); break;
        case 9: fft_launch<T, 9>(p, nq, grid, tw, M, s); break;
        default: throw Error(MLG_ERR_RANGE, "FFT length must be 16..512");
    }
}

// One FFT pass along axis `ax` of every plane of the grid.
//   x (ax = 0): lines of L contiguous entries, every line of the plane;
//   y (ax = 1): the band x columns of every z slab;
//   z (ax = 2): the band x columns of the band y rows.
template <class T>
static void fft_pass(const NfftPlan &P, int bg, typename Cplx<T>::type *grid, int ax, int mode,
                     const T *M, hipStream_t s, int nl = 1, int64_t mstr = 0) {
    const int64_t L = P.nos;
    FftPass p{};
    p.N = P.N;
    p.mode = mode;
    p.lq = bg / 2;
    p.mstr = M ? mstr : 0;
    p.qstr = 1;
    for (int t = 0; t < P.d; ++t) p.qstr *= L;
    if (ax == 0) {
        p.S = 1;
        p.A = 1;
        p.abnd = 0;
        p.O = p.qstr / L;
        p.ostr = L;
        p.obnd = 0;
    } else if (ax == 1) {
        p.S = L;
        p.A = P.N + 1;
        p.abnd = 1;
        p.O = p.qstr / (L * L);
        p.ostr = L * L;
        p.obnd = 0;
    } else {
        p.S = L * L;
        p.A = P.N + 1;
        p.abnd = 1;
        p.O = P.N + 1;
        p.ostr = L;
        p.obnd = 1;
    }
    fft_dispatch<T>(P, p, bg / 2 * nl, grid, M, s);
}

// Forward FFT, multiplication by M and inverse FFT with band pruning, plane
// by plane:
//   d = 1: x: forward * M * inverse.
//   d = 2: x forward (all rows); y forward * M * inverse on the band x
//          columns; x inverse (all rows, out-of-band x read as zero).
//   d = 3: x forward (all); y forward on band x columns (all z); z forward *
//          M * inverse on band x columns of band y rows; y inverse on band
//          x columns; x inverse (all, out-of-band read as zero).
// FP32 grids of side 64 do the x and y passes of each plane in one kernel
// (d = 2: the whole convolution).
// Only entries with every frequency inside the band are ever multiplied;
// the out-of-band ones are never read again.
// With nl > 1 the grid holds nl layers of the same N one after another
// (bg / 2 planes each) and their multipliers sit mstr apart from M on.
// Whether the first FFT pass of a plan takes the gather with it
// (k_gather_fftx): one layer, blocks of 16, d >= 2, sides 128..512 (FP64:
// up to 256, for its LDS tile), and a cell table.
template <class T>
static bool fused_gather_fft(const NfftPlan &P, const NfftWindow &W, int bs) {
    const int maxL = sizeof(T) == 4 ? 512 : 256;
    return W.csr && bs == 16 && P.d >= 2 && P.nos >= 128 && P.nos <= maxL;
}

template <class T>
static void launch_gather_fftx(const NfftPlan &P, const NfftWindow &W, typename Cplx<T>::type *grid,
                               const T *patch, hipStream_t s) {
    int64_t G = 1;
    for (int t = 0; t < P.d; ++t) G *= P.nos;
    const int64_t lines = G / P.nos;
    MLG_REQUIRE(lines < ((int64_t)1 << 31), MLG_ERR_RANGE, "FFT grid too large");
#define GFX_CALL(LG)                                                                              \
    hipLaunchKernelGGL((k_gather_fftx<T, LG>), dim3((unsigned)lines), dim3(256), 0, s, grid, G, P.N, \
                       W.cell_ptr.p, W.cell_ent.p, patch, tw_of<T>(P))
    switch (ilog2(P.nos)) {
        case 7: GFX_CALL(7); break;
        case 8: GFX_CALL(8); break;
        case 9:
            if constexpr (sizeof(T) == 4) {
                GFX_CALL(9);
                break;
            }
            [[fallthrough]];
        default: throw Error(MLG_ERR_ARG, "fused gather: unsupported grid side");
    }
#undef GFX_CALL
    MLG_LAUNCH_CHECK();
}

// With first_done the x pass of mode 0 has already run (k_gather_fftx).
template <class T>
static void fft_convolve(const NfftPlan &P, int bg, typename Cplx<T>::type *grid, const T *M,
                         hipStream_t s, int nl = 1, int64_t mstr = 0, bool first_done = false) {
    const int d = P.d;
    const int nq = bg / 2 * nl;
    if (d == 1) {
        fft_pass<T>(P, bg, grid, 0, 2, M, s, nl, mstr);
    } else if (d == 2) {
        if constexpr (std::is_same<T, float>::value) {
            if (P.nos == 64) {
                MLG_REQUIRE(nq <= 65535, MLG_ERR_RANGE, "FFT grid too large");
                hipLaunchKernelGGL((k_fft_xy64<float2, 2>), dim3(1, nq), dim3(256), 0, s, grid, P.N,
                                   (int64_t)64 * 64, tw_of<T>(P), M, bg / 2, mstr);
                MLG_LAUNCH_CHECK();
                return;
            }
        }
        if (!first_done) fft_pass<T>(P, bg, grid, 0, 0, nullptr, s, nl);
        fft_pass<T>(P, bg, grid, 1, 2, M, s, nl, mstr);
        fft_pass<T>(P, bg, grid, 0, 1, nullptr, s, nl);
    } else {
        if constexpr (std::is_same<T, float>::value) {
            if (P.nos == 64) {
                const int64_t qstr = (int64_t)64 * 64 * 64;
                MLG_REQUIRE(nq <= 65535, MLG_ERR_RANGE, "FFT grid too large");
                hipLaunchKernelGGL((k_fft_xy64<float2, 0>), dim3(64, nq), dim3(256), 0, s, grid,
                                   P.N, qstr, tw_of<T>(P), nullptr, bg / 2, (int64_t)0);
                MLG_LAUNCH_CHECK();
                fft_pass<T>(P, bg, grid, 2, 2, M, s, nl, mstr);
                hipLaunchKernelGGL((k_fft_xy64<float2, 1>), dim3(64, nq), dim3(256), 0, s, grid,
                                   P.N, qstr, tw_of<T>(P), nullptr, bg / 2, (int64_t)0);
                MLG_LAUNCH_CHECK();
                return;
            }
        }
        if (!first_done) fft_pass<T>(P, bg, grid, 0, 0, nullptr, s, nl);
        fft_pass<T>(P, bg, grid, 1, 0, nullptr, s, nl);
        fft_pass<T>(P, bg, grid, 2, 2, M, s, nl, mstr);
        fft_pass<T>(P, bg, grid, 1, 1, nullptr, s, nl);
        fft_pass<T>(P, bg, grid, 0, 1, nullptr, s, nl);
    }
}

// Widest vector group (power of two <= min(bs, 16)) whose patch slots fit the
// spreading lanes' registers: ceil(PD/64) cells x VPL vectors <= 64.
static int spread_vpl(int PD, int bs) {
    int v = std::min(bs, 16);
    while (v > 1 && ceil_div(PD, 64) * v > 64) v >>= 1;
    return v;
}

// Cell slots per lane: the smallest compiled count covering the patch.
template <class T, int D, int VPL>
static void launch_spread(const Geom &g, const NfftPlan &P, const T *Zs, T beta, T *patch,
                          hipStream_t s) {
    const size_t lds = (size_t)64 * (D * g.P + VPL) * sizeof(T);
    const int cpl = ceil_div(g.PD, 64);
    constexpr int CFULL = 64 / VPL;
    dim3 grd(P.ntasks, g.bs / VPL);
    if (cpl <= 4 && CFULL >= 4)
        hipLaunchKernelGGL((k_spread<T, D, VPL, (CFULL < 4 ? CFULL : 4)>), grd, dim3(64), lds, s, g,
                           P.tasks.p, P.u64.p, P.c32.p, P.f32.p, Zs, beta, patch);
    else if (cpl <= 16 && CFULL >= 16)
        hipLaunchKernelGGL((k_spread<T, D, VPL, (CFULL < 16 ? CFULL : 16)>), grd, dim3(64), lds, s, g,
                           P.tasks.p, P.u64.p, P.c32.p, P.f32.p, Zs, beta, patch);
    else
        hipLaunchKernelGGL((k_spread<T, D, VPL, CFULL>), grd, dim3(64), lds, s, g, P.tasks.p, P.u64.p,
                           P.c32.p, P.f32.p, Zs, beta, patch);
    MLG_LAUNCH_CHECK();
}

template <class T, int D, int VPL>
static void launch_gather(const Geom &g, const NfftPlan &P, const T *patch, int bg, T *grid,
                          int64_t G, hipStream_t s) {
    hipLaunchKernelGGL((k_gather<T, D, VPL>), dim3(ceil_div(G, 256), g.bs / VPL), dim3(256), 0, s, g,
                       P.SB, P.nsb, P.occ.p, P.bin_run.p, patch, bg, grid, G);
    MLG_LAUNCH_CHECK();
}

template <class T, int D, int VPL>
static void launch_interp(const Geom &g, const NfftPlan &P, const T *grid, int bg, T beta, T *Fs,
                          hipStream_t s) {
    hipLaunchKernelGGL((k_interp<T, D, VPL>), dim3(ceil_div(g.n, 256), g.bs / VPL), dim3(256), 0, s,
                       g, P.u64.p, P.c32.p, P.f32.p, grid, bg, beta, Fs);
    MLG_LAUNCH_CHECK();
}

#define MLG_VPL_SWITCH(vpl, CALL)                                                   \
    switch (vpl) {                                                                  \
        case 1: CALL(1); break;                                                     \
        case 2: CALL(2); break;                                                     \
        case 4: CALL(4); break;                                                     \
        case 8: CALL(8); break;                                                     \
        case 16: CALL(16); break;                                                   \
        default: throw Error(MLG_ERR_ARG, "unsupported vector group");              \
    }

template <class T, int D>
static void apply_d(const NfftPlan &P, const NfftWindow &W, int bs, const T *Zs, T *Fs, T *patch,
                    T *grid, hipStream_t s, hipEvent_t *ev, const float *zsc) {
    Geom g;
    g.zsc = zsc;
    g.d = D;
    g.nos = P.nos;
    g.B = P.B;
    g.nb = P.nb;
    g.w = W.w;
    g.P = patch_side(P, W);
    g.PD = patch_cells(P, W);
    g.bs = bs;
    g.n = P.n;
    g.perm = P.perm.p;
    MLG_REQUIRE(bs >= 1 && bs <= 64 && is_pow2(bs), MLG_ERR_ARG, "block stride must be a power of two <= 64");
    const int vs = spread_vpl(g.PD, bs);
    MLG_REQUIRE(ceil_div(g.PD, 64) * vs <= 64, MLG_ERR_RANGE,
                "patch too large for one task (reduce window or bin)");
    const int bg = bs < 2 ? 2 : bs;
    const T beta = (T)W.beta;
    // FP32 blocks of 16 vectors with patches of <= 256 cells use the matrix
    // cores; everything else the vector-ALU kernels.
    const bool mf = std::is_same<T, float>::value && bs % 16 == 0 && mfma_patch_ok(D, g.P);
    const bool sched = mf && uses_spread_schedule(P, W, bs);
    if (P.ntasks > 0) {
        if constexpr (std::is_same<T, float>::value) {
            if (mf) {
#define SPREADM_CALL(DD, PP)                                                                      \
    if constexpr (DD == 3)                                                                        \
        hipLaunchKernelGGL((k_spread_mfma3<PP>), dim3(sched ? P.nseg : P.ntasks, bs / 16), dim3(64), 0, s, \
                           g, sched ? P.seg.p : P.tasks.p, P.c32.p, P.f32.p, Zs, beta, patch,    \
                           nullptr, nullptr);                                                     \
    else                                                                                          \
        hipLaunchKernelGGL((k_spread_mfma<DD, PP>), dim3(P.ntasks, bs / 16), dim3(64), 0, s, g, P.tasks.p, \
                           P.c32.p, P.f32.p, Zs, beta, patch, nullptr, nullptr)
                MLG_P_SWITCH(D, g.P, SPREADM_CALL)
#undef SPREADM_CALL
                MLG_LAUNCH_CHECK();
            }
        }
        if (!mf) {
#define SPREAD_CALL(V) launch_spread<T, D, V>(g, P, Zs, beta, patch, s)
            MLG_VPL_SWITCH(vs, SPREAD_CALL)
#undef SPREAD_CALL
        }
    }
    if (ev) MLG_HIP(hipEventRecord(ev[1], s));   // spreading kernel alone
    if (P.ntasks > 0) {
        const int nr1 = sched ? P.nsred1 : P.nred1, nr2 = sched ? P.nsred2 : P.nred2;
        const int4 *r1 = sched ? P.sred1.p : P.red1.p, *r2 = sched ? P.sred2.p : P.red2.p;
        if (nr1 > 0) {
            const int64_t elems = (int64_t)g.PD * bs;
            hipLaunchKernelGGL(k_reduce1<T>, dim3(nr1, ceil_div(elems, 256)), dim3(256), 0, s, elems,
                               r1, patch);
            MLG_LAUNCH_CHECK();
            if (nr2 > 0) {
                hipLaunchKernelGGL(k_reduce2<T>, dim3(nr2, ceil_div(elems, 256)), dim3(256), 0, s,
                                   elems, r2, patch);
                MLG_LAUNCH_CHECK();
            }
        }
    }
    int64_t G = 1;
    for (int t = 0; t < D; ++t) G *= P.nos;
    // four vectors per thread and sixteen entries per batch: the gather is
    // bound by the latency of each cell's chain of entry loads, so many
    // short chains beat few wide ones (measured: 16 -> 4 vectors per thread
    // takes the d = 3 gathers of the image graph from 94 to 60 us)
    const int vgat = std::min(bs, 4);
    const bool fused = fused_gather_fft<T>(P, W, bs);
    if (fused) {
        // the gather runs inside the first FFT pass
    } else if (W.csr) {
#define GATHERC_CALL(V)                                                                           \
    hipLaunchKernelGGL((k_gather_csr<T, V>), dim3(ceil_div(G, 256) * (bs / V)), dim3(256), 0, s, G, bs, bg, \
                       W.cell_ptr.p, W.cell_ent.p, patch, grid, 0, nullptr, nullptr)
        MLG_VPL_SWITCH(vgat, GATHERC_CALL)
#undef GATHERC_CALL
        MLG_LAUNCH_CHECK();
    } else {
#define GATHER_CALL(V) launch_gather<T, D, V>(g, P, patch, bg, grid, G, s)
        MLG_VPL_SWITCH(vgat, GATHER_CALL)
#undef GATHER_CALL
    }
    if (ev) MLG_HIP(hipEventRecord(ev[2], s));
    using C2 = typename Cplx<T>::type;
    if (fused) launch_gather_fftx<T>(P, W, reinterpret_cast<C2 *>(grid), patch, s);
    fft_convolve<T>(P, bg, reinterpret_cast<C2 *>(grid), mult_of<T>(W), s, 1, 0, fused);
    if (ev) MLG_HIP(hipEventRecord(ev[3], s));
    if constexpr (std::is_same<T, float>::value) {
        if (mf && P.ntasks > 0) {
            // d = 3: each task's points are interpolated by two workgroups
            // (128 points each); the task's grid patch is fetched twice, but
            // twice as many shorter wavefronts fill the chip better (image
            // graph, b = 16: 65.8 -> 69 TFLOP/s; four parts: 57).  The
            // d <= 2 kernel measured no gain from it.
            // With the plan's interpolation schedule (tasks of a few chunks
            // sized for three wavefronts per SIMD) one workgroup runs a whole
            // task and loads its grid patch once.
            const bool isch = P.niseg > 0 && sched;
            const int isplit = isch ? 1 : 2;
            const int iper = isch ? (1 << 30) : kMaxTaskPoints / isplit;
            const int ntk = isch ? P.niseg : P.ntasks;
            const int4 *itk = isch ? P.iseg.p : P.tasks.p;
#define INTERPM_CALL(DD, PP)                                                                      \
    if constexpr (DD == 3)                                                                        \
        hipLaunchKernelGGL((k_interp_mfma3<PP>), dim3(ntk * isplit, bs / 16), dim3(64), 0, s, g,  \
                           itk, P.c32.p, P.f32.p, grid, bg, beta, Fs, isplit, iper, nullptr, nullptr); \
    else                                                                                          \
        hipLaunchKernelGGL((k_interp_mfma<DD, PP>), dim3(P.ntasks, bs / 16), dim3(64), 0, s, g, P.tasks.p, \
                           P.c32.p, P.f32.p, grid, bg, beta, Fs, nullptr, nullptr)
            MLG_P_SWITCH(D, g.P, INTERPM_CALL)
#undef INTERPM_CALL
            MLG_LAUNCH_CHECK();
        }
    }
    if (!mf) {
        const int vint = std::min(bs, 16);
#define INTERP_CALL(V) launch_interp<T, D, V>(g, P, grid, bg, beta, Fs, s)
        MLG_VPL_SWITCH(vint, INTERP_CALL)
#undef INTERP_CALL
    }
    if (ev) MLG_HIP(hipEventRecord(ev[4], s));
}

template <class T>
void nfft_apply(const NfftPlan &P, const NfftWindow &W, int bs, const T *Zs, T *Fs, T *patch,
                T *grid, hipStream_t s, hipEvent_t *ev, const float *zsc) {
    MLG_REQUIRE(!zsc || (std::is_same<T, float>::value && nfft_scaled_input_ok(P, W, bs)),
                MLG_ERR_ARG, "scaled summation input needs the matrix-core spreading");
    switch (P.d) {
        case 1: apply_d<T, 1>(P, W, bs, Zs, Fs, patch, grid, s, ev, zsc); break;
        case 2: apply_d<T, 2>(P, W, bs, Zs, Fs, patch, grid, s, ev, zsc); break;
        case 3: apply_d<T, 3>(P, W, bs, Zs, Fs, patch, grid, s, ev, zsc); break;
        default: throw Error(MLG_ERR_RANGE, "NFFT layers need d in 1..3");
    }
}

bool nfft_scaled_input_ok(const NfftPlan &P, const NfftWindow &W, int bs) {
    return W.prec == 32 && bs % 16 == 0 && mfma_patch_ok(P.d, patch_side(P, W)) && P.ntasks > 0;
}

// ------------------------------------------------------------------------------
// batched layers (see NfftBatch)
// ------------------------------------------------------------------------------
__global__ void k_offset_copy(int64_t cnt, const int *__restrict__ src, int add, int *__restrict__ dst) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < cnt) dst[e] = src[e] + add;
}

static Geom layer_geom(const Layer &L, int bs) {
    Geom g;
    g.d = L.d;
    g.nos = L.nf.nos;
    g.B = L.nf.B;
    g.nb = L.nf.nb;
    g.w = L.win.w;
    g.P = patch_side(L.nf, L.win);
    g.PD = patch_cells(L.nf, L.win);
    g.bs = bs;
    g.n = L.nf.n;
    g.perm = L.nf.perm.p;
    g.zsc = nullptr;
    return g;
}

bool nfft_batchable(const Layer &L, int bs, int *key) {
    if (L.kp.method != MLG_METHOD_NFFT || L.kp.precision != 32 || L.win.prec != 32) return false;
    if (bs % 16 != 0 || !L.win.csr || L.nf.ntasks <= 0) return false;
    const int side = patch_side(L.nf, L.win);
    if (!mfma_patch_ok(L.d, side)) return false;
    // one interpolation task form per batch
    const bool isch = L.nf.niseg > 0 && uses_spread_schedule(L.nf, L.win, bs);
    *key = (L.d * 64 + side) * 2 + (isch ? 1 : 0);
    return true;
}

template <class V>
static std::vector<V> to_host(const DevBuf<V> &b, size_t cnt, hipStream_t s) {
    std::vector<V> h(cnt);
    if (cnt) MLG_HIP(hipMemcpyAsync(h.data(), b.p, sizeof(V) * cnt, hipMemcpyDeviceToHost, s));
    return h;
}

void nfft_batch_build(NfftBatch &B, const std::vector<const Layer *> &layers,
                      const std::vector<int> &ids, const float *X32,
                      const std::vector<float *> &Fs, int bs, hipStream_t s) {
    const int nl = (int)layers.size();
    MLG_REQUIRE(nl >= 1, MLG_ERR_ARG, "empty batch");
    // batch order: by N (equal N adjacent for the batched FFT), then layer id
    std::vector<int> ord(nl);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(),
                     [&](int a, int b) { return layers[a]->nf.N < layers[b]->nf.N; });
    B = NfftBatch();
    B.nl = nl;
    B.bs = bs;
    B.bg = bs < 2 ? 2 : bs;
    B.D = layers[0]->d;
    B.Pside = patch_side(layers[0]->nf, layers[0]->win);
    const int PD = patch_cells(layers[0]->nf, layers[0]->win);
    std::vector<LayerArgs> la(nl);
    std::vector<int4> st, it, r1, r2;
    std::vector<int> sl, il;
    std::vector<int64_t> coff(nl + 1, 0), goff(nl, 0);
    std::vector<int64_t> eoff(nl + 1, 0);   // entry offsets of the concatenated cell tables
    int64_t slot_off = 0;
    std::vector<int64_t> slots(nl);
    bool any_isched = false, any_plain = false;
    for (int i = 0; i < nl; ++i) {
        const Layer &L = *layers[ord[i]];
        const NfftPlan &P = L.nf;
        MLG_REQUIRE(L.d == B.D && patch_side(P, L.win) == B.Pside, MLG_ERR_ARG, "mixed batch");
        B.layers.push_back(ids[ord[i]]);
        LayerArgs &a = la[i];
        a.g = layer_geom(L, bs);
        a.c32 = P.c32.p;
        a.f32 = P.f32.p;
        a.Zs = X32;
        a.g.zsc = L.zsc.p;
        a.Fs = Fs[ord[i]];
        int64_t G = 1;
        for (int t = 0; t < L.d; ++t) G *= P.nos;
        a.beta = (float)L.win.beta;
        const bool sched = uses_spread_schedule(P, L.win, bs);
        const bool isch = P.niseg > 0 && sched;
        any_isched |= isch;
        any_plain |= !isch;
        slots[i] = (int64_t)P.nruns + P.nscratch + (sched ? P.nsscr : 0);
        MLG_REQUIRE(slot_off + slots[i] < ((int64_t)1 << 31) / std::max(PD, 1), MLG_ERR_RANGE,
                    "batched patch slots exceed the index range");
        const int so = (int)slot_off;
        // spreading tasks and reduction lists, slots shifted
        {
            const int n = sched ? P.nseg : P.ntasks;
            std::vector<int4> tk = to_host(sched ? P.seg : P.tasks, (size_t)n, s);
            std::vector<int4> g1 = to_host(sched ? P.sred1 : P.red1, (size_t)(sched ? P.nsred1 : P.nred1), s);
            std::vector<int4> g2 = to_host(sched ? P.sred2 : P.red2, (size_t)(sched ? P.nsred2 : P.nred2), s);
            std::vector<int4> ik = to_host(isch ? P.iseg : P.tasks, (size_t)(isch ? P.niseg : P.ntasks), s);
            MLG_HIP(hipStreamSynchronize(s));
            for (int4 t : tk) {
                t.w += so;
                st.push_back(t);
                sl.push_back(i);
            }
            for (int4 t : g1) {
                t.x += so;
                t.z += so;
                r1.push_back(t);
            }
            for (int4 t : g2) {
                t.x += so;
                t.y += so;
                r2.push_back(t);
            }
            for (const int4 &t : ik) {
                it.push_back(t);
                il.push_back(i);
            }
        }
        slot_off += slots[i];
        coff[i + 1] = coff[i] + G;
        if (i + 1 < nl) goff[i + 1] = goff[i] + (int64_t)B.bg * G;
        eoff[i + 1] = eoff[i] + (int64_t)L.win.cell_ent.n;
    }
    // the interpolation of a batch runs one task per workgroup when every
    // layer has its own interpolation schedule, else 256-point tasks in two
    // halves (the per-layer path's choice for each layer)
    MLG_REQUIRE(!(any_isched && any_plain), MLG_ERR_ARG, "batch mixes interpolation task forms");
    B.isplit = any_isched ? 1 : (B.D == 3 ? 2 : 1);
    B.iper = any_isched ? (1 << 30) : kMaxTaskPoints / B.isplit;
    MLG_REQUIRE(eoff[nl] < ((int64_t)1 << 31), MLG_ERR_RANGE, "batched cell tables too large");
    B.nst = (int)st.size();
    B.nit = (int)it.size();
    B.nred1 = (int)r1.size();
    B.nred2 = (int)r2.size();
    B.ncell = coff[nl];
    upload(B.stasks, st.data(), st.size(), false, s);
    upload(B.slayer, sl.data(), sl.size(), false, s);
    upload(B.itasks, it.data(), it.size(), false, s);
    upload(B.ilayer, il.data(), il.size(), false, s);
    upload(B.red1, r1.data(), r1.size(), false, s);
    upload(B.red2, r2.data(), r2.size(), false, s);
    upload(B.coff, coff.data(), coff.size(), false, s);
    upload(B.goff, goff.data(), goff.size(), false, s);
    B.goff_h = goff;
    // concatenated cell tables: pointers shifted by the entries before the
    // layer, entries by its first patch slot
    B.cptr.alloc((size_t)B.ncell + 1);
    B.cent.alloc((size_t)std::max<int64_t>(eoff[nl], 1));
    slot_off = 0;
    for (int i = 0; i < nl; ++i) {
        const Layer &L = *layers[ord[i]];
        const int64_t G = coff[i + 1] - coff[i];
        const int64_t cnt = i + 1 < nl ? G : G + 1;   // the last layer's end pointer too
        hipLaunchKernelGGL(k_offset_copy, dim3(ceil_div(cnt, 256)), dim3(256), 0, s, cnt,
                           L.win.cell_ptr.p, (int)eoff[i], B.cptr.p + coff[i]);
        MLG_LAUNCH_CHECK();
        const int64_t ne = (int64_t)L.win.cell_ent.n;
        if (ne > 0) {
            hipLaunchKernelGGL(k_offset_copy, dim3(ceil_div(ne, 256)), dim3(256), 0, s, ne,
                               L.win.cell_ent.p, (int)(slot_off * PD), B.cent.p + eoff[i]);
            MLG_LAUNCH_CHECK();
        }
        slot_off += slots[i];
    }
    // groups of equal N for the FFT, their multipliers one after another
    for (int i = 0; i < nl;) {
        int j = i + 1;
        while (j < nl && layers[ord[j]]->nf.N == layers[ord[i]]->nf.N) ++j;
        NfftBatch::Sub sb;
        sb.first = i;
        sb.count = j - i;
        sb.plan = &layers[ord[i]]->nf;
        const int64_t G = coff[i + 1] - coff[i];
        sb.mstr = G;
        sb.M.alloc((size_t)G * sb.count);
        for (int k = i; k < j; ++k)
            MLG_HIP(hipMemcpyAsync(sb.M.p + (size_t)(k - i) * G, layers[ord[k]]->win.M32.p,
                                   sizeof(float) * G, hipMemcpyDeviceToDevice, s));
        B.subs.push_back(std::move(sb));
        i = j;
    }
    B.patch_elems = (size_t)slot_off * PD * bs;
    B.grid_elems = (size_t)B.bg * coff[nl];
    B.patch.alloc(B.patch_elems);
    B.grid.alloc(B.grid_elems);
    for (int i = 0; i < nl; ++i) la[i].grid = B.grid.p + goff[i];   // the interpolation's input
    B.args.alloc(sizeof(LayerArgs) * nl);
    MLG_HIP(hipMemcpyAsync(B.args.p, la.data(), sizeof(LayerArgs) * nl, hipMemcpyHostToDevice, s));
    // products without D^-1/2 (the weight matrix itself): no factor
    for (int i = 0; i < nl; ++i) la[i].g.zsc = nullptr;
    B.args_n.alloc(sizeof(LayerArgs) * nl);
    MLG_HIP(hipMemcpyAsync(B.args_n.p, la.data(), sizeof(LayerArgs) * nl, hipMemcpyHostToDevice, s));
    MLG_HIP(hipStreamSynchronize(s));
    // the argument table is read by every batched launch; nothing above is
    // needed on the host afterwards
}

void nfft_batch_apply(const NfftBatch &B, int use_dinv, hipStream_t s) {
    const int bs = B.bs, bg = B.bg, D = B.D;
    const LayerArgs *la = reinterpret_cast<const LayerArgs *>(use_dinv ? B.args.p : B.args_n.p);
    const int PD = [&] {
        int pd = 1;
        for (int t = 0; t < D; ++t) pd *= B.Pside;
        return pd;
    }();
    Geom g0{};
    g0.bs = bs;
    float *patch = B.patch.p, *grid = B.grid.p;
    // spreading
    if (B.nst > 0) {
#define SPREADB_CALL(DD, PP)                                                                      \
    if constexpr (DD == 3)                                                                        \
        hipLaunchKernelGGL((k_spread_mfma3<PP>), dim3(B.nst, bs / 16), dim3(64), 0, s, g0, B.stasks.p, \
                           nullptr, nullptr, nullptr, 0.0f, patch, la, B.slayer.p);              \
    else                                                                                          \
        hipLaunchKernelGGL((k_spread_mfma<DD, PP>), dim3(B.nst, bs / 16), dim3(64), 0, s, g0, B.stasks.p, \
                           nullptr, nullptr, nullptr, 0.0f, patch, la, B.slayer.p)
        switch (D) {
            case 1: MLG_P_SWITCH(1, B.Pside, SPREADB_CALL); break;
            case 2: MLG_P_SWITCH(2, B.Pside, SPREADB_CALL); break;
            case 3: MLG_P_SWITCH(3, B.Pside, SPREADB_CALL); break;
            default: throw Error(MLG_ERR_ARG, "bad batch dimension");
        }
#undef SPREADB_CALL
        MLG_LAUNCH_CHECK();
    }
    // split-bin reductions
    const int64_t elems = (int64_t)PD * bs;
    if (B.nred1 > 0) {
        hipLaunchKernelGGL(k_reduce1<float>, dim3(B.nred1, ceil_div(elems, 256)), dim3(256), 0, s, elems,
                           B.red1.p, patch);
        MLG_LAUNCH_CHECK();
    }
    if (B.nred2 > 0) {
        hipLaunchKernelGGL(k_reduce2<float>, dim3(B.nred2, ceil_div(elems, 256)), dim3(256), 0, s, elems,
                           B.red2.p, patch);
        MLG_LAUNCH_CHECK();
    }
    // cell-table gather over every layer's grid
    const int vgat = std::min(bs, 4);
#define GATHERB_CALL(V)                                                                           \
    hipLaunchKernelGGL((k_gather_csr<float, V>), dim3(ceil_div(B.ncell, 256) * (bs / V)), dim3(256), 0, s, \
                       (int64_t)0, bs, bg, B.cptr.p, B.cent.p, patch, grid, B.nl, B.coff.p, B.goff.p)
    MLG_VPL_SWITCH(vgat, GATHERB_CALL)
#undef GATHERB_CALL
    MLG_LAUNCH_CHECK();
    // FFT, multiply, inverse FFT: one call per group of equal N (their grids
    // are adjacent, bg / 2 planes each)
    for (const NfftBatch::Sub &sb : B.subs)
        fft_convolve<float>(*sb.plan, bg, reinterpret_cast<float2 *>(grid + B.goff_h[sb.first]), sb.M.p, s,
                            sb.count, sb.mstr);
    // interpolation
    if (B.nit > 0) {
#define INTERPB_CALL(DD, PP)                                                                      \
    if constexpr (DD == 3)                                                                        \
        hipLaunchKernelGGL((k_interp_mfma3<PP>), dim3(B.nit * B.isplit, bs / 16), dim3(64), 0, s, g0, \
                           B.itasks.p, nullptr, nullptr, nullptr, bg, 0.0f, nullptr, B.isplit, B.iper, \
                           la, B.ilayer.p);                                                       \
    else                                                                                          \
        hipLaunchKernelGGL((k_interp_mfma<DD, PP>), dim3(B.nit, bs / 16), dim3(64), 0, s, g0, B.itasks.p, \
                           nullptr, nullptr, nullptr, bg, 0.0f, nullptr, la, B.ilayer.p)
        switch (D) {
            case 1: MLG_P_SWITCH(1, B.Pside, INTERPB_CALL); break;
            case 2: MLG_P_SWITCH(2, B.Pside, INTERPB_CALL); break;
            case 3: MLG_P_SWITCH(3, B.Pside, INTERPB_CALL); break;
            default: throw Error(MLG_ERR_ARG, "bad batch dimension");
        }
#undef INTERPB_CALL
        MLG_LAUNCH_CHECK();
    }
}

template void nfft_apply<float>(const NfftPlan &, const NfftWindow &, int, const float *, float *,
                                float *, float *, hipStream_t, hipEvent_t *, const float *);
template void nfft_apply<double>(const NfftPlan &, const NfftWindow &, int, const double *,
                                 double *, double *, double *, hipStream_t, hipEvent_t *,
                                 const float *);

}  // namespace mlg
