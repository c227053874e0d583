// NFFT fast summation of a Gaussian kernel (Algorithm 1, Sec. 4):
//   W~ v ~= A diag(b^) A* v,  A = (exp(2 pi i l.x_j)), l in {-N/2..N/2}^d.
//
// Plan (once per layer):
//   torus scaling   x -> s (x - c) with ||s (x - c)|| <= 1/4 - eps_B/2, so every
//                   pair distance stays where the regularised kernel equals K;
//                   sigma -> s sigma (Alg. 1 input domain).
//   grid coords     u = (x_scaled + 1/2) * 2N lies in [N/2, 3N/2]: a window of
//                   support w < N never wraps around the 2N grid.
//   bin sort        points sorted by the grid cell of u grouped in bins of
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
// Apply (per block of vectors z, stride bs, sorted order):
//   spread   per task: patch[o][v] = sum_p psi(u_p - o) z_p[v] over the task's
//            points, accumulated in registers (no atomics);
//   gather   per tile of the grid: sum of the patches covering it, one LDS
//            copy per wavefront, copies added in a fixed order (no atomics);
//   FFT      forward complex FFT (two real vectors per complex lane), times M,
//            inverse FFT (Alg. 1 steps 1-3 with deconvolution folded into M);
//   interp   per task: f_p[v] = sum_o psi(u_p - o) h[o][v], partial sums
//            reduced across lanes by butterfly shuffles, then across the
//            four wavefronts in a fixed order.
#include <cmath>
#include <cstring>

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
// psi(t) = exp(beta (sqrt(1 - (2t/w)^2) - 1)).
template <class T>
__device__ inline T es_psi(T t, T two_over_w, T beta) {
    T z = t * two_over_w;
    T s = T(1) - z * z;
    s = s > T(0) ? s : T(0);
    return dexp<T>(beta * (sqrt(s) - T(1)));
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

__global__ void k_gather_coords(int64_t n, int d, const double *__restrict__ u,
                                const int *__restrict__ perm, double *__restrict__ u64,
                                float *__restrict__ u32) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int64_t i = perm[p];
    for (int t = 0; t < d; ++t) {
        double v = u[(int64_t)t * n + i];
        u64[(int64_t)t * n + p] = v;
        u32[(int64_t)t * n + p] = (float)v;
    }
}

__global__ void k_task_counts(int runs, const unsigned *__restrict__ counts, int ch,
                              unsigned *__restrict__ ntask) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < runs) ntask[r] = (counts[r] + ch - 1) / ch;
}

__global__ void k_fill_tasks(int runs, const unsigned *__restrict__ ukeys,
                             const unsigned *__restrict__ counts,
                             const unsigned *__restrict__ run_start,
                             const unsigned *__restrict__ task_first, int ch,
                             int4 *__restrict__ tasks, int2 *__restrict__ bin_tasks) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= runs) return;
    const unsigned cnt = counts[r], st = run_start[r], tf = task_first[r];
    const unsigned nt = (cnt + ch - 1) / ch;
    for (unsigned j = 0; j < nt; ++j) {
        unsigned first = st + j * ch;
        unsigned c = cnt - j * ch < (unsigned)ch ? cnt - j * ch : (unsigned)ch;
        tasks[tf + j] = make_int4((int)ukeys[r], (int)first, (int)c, 0);
    }
    bin_tasks[ukeys[r]] = make_int2((int)tf, (int)nt);
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
struct TaskGeom {
    int d, nos, B, nb, w, P, bs;
    int64_t n;
};

__device__ inline void decode_bin(unsigned key, int nb, int d, int b[3]) {
    b[0] = b[1] = b[2] = 0;
    for (int t = 0; t < d; ++t) {
        b[t] = (int)(key % (unsigned)nb);
        key /= (unsigned)nb;
    }
}

// Stage `cnt` points starting at `first`: 1D window weights at the P patch
// positions of each dimension (zero outside the point's footprint).
template <class T, int D>
__device__ inline void stage_weights(const TaskGeom &g, const T *__restrict__ u, int64_t first,
                                     int cnt, const int org[3], T beta, T *__restrict__ wts) {
    const T two_over_w = T(2) / (T)g.w;
    for (int e = threadIdx.x; e < cnt * D * g.P; e += blockDim.x) {
        int pt = e / (D * g.P);
        int r = e - pt * D * g.P;
        int t = r / g.P, q = r - t * g.P;
        T ut = u[(int64_t)t * g.n + first + pt];
        int cell = (int)floor((double)ut);
        int s0 = cell - g.w / 2 + 1;          // first footprint cell
        int k = org[t] + q;                   // grid cell of this patch position
        T val = T(0);
        if (k >= s0 && k < s0 + g.w) val = es_psi<T>(ut - (T)k, two_over_w, beta);
        wts[e] = val;
    }
}

template <class T, int D>
__global__ __launch_bounds__(256) void k_spread(TaskGeom g, const int4 *__restrict__ tasks,
                                                const T *__restrict__ u, const T *__restrict__ Zs,
                                                T beta, int chs, int vg, T *__restrict__ patch) {
    extern __shared__ unsigned char smem_raw[];
    T *wts = reinterpret_cast<T *>(smem_raw);
    T *zv = wts + (size_t)chs * D * g.P;
    const int4 tk = tasks[blockIdx.x];
    int bb[3];
    decode_bin((unsigned)tk.x, g.nb, D, bb);
    int org[3] = {0, 0, 0};
    for (int t = 0; t < D; ++t) org[t] = bb[t] * g.B - g.w / 2 + 1;
    const int tid = threadIdx.x;
    const int P = g.P;
    int PD = P;
    for (int t = 1; t < D; ++t) PD *= P;
    const int bs = g.bs;
    // this workgroup handles vectors [blockIdx.y*vg, +vg) of the block
    const int v = blockIdx.y * vg + tid % vg;
    const int ostep = 256 / vg;
    const int o0 = tid / vg;
    int qoff[kMaxSlots];
    T acc[kMaxSlots];
#pragma unroll
    for (int j = 0; j < kMaxSlots; ++j) {
        int o = o0 + j * ostep;
        int qx = o % P, qy = (o / P) % P, qz = o / (P * P);
        qoff[j] = (o < PD) ? (qx | (qy << 8) | (qz << 16)) : -1;
        acc[j] = T(0);
    }
    for (int c0 = 0; c0 < tk.z; c0 += chs) {
        const int cnt = (tk.z - c0) < chs ? (tk.z - c0) : chs;
        const int64_t first = (int64_t)tk.y + c0;
        __syncthreads();
        stage_weights<T, D>(g, u, first, cnt, org, beta, wts);
        for (int e = tid; e < cnt * bs; e += 256) zv[e] = Zs[first * bs + e];
        __syncthreads();
        for (int pt = 0; pt < cnt; ++pt) {
            const T *wp = wts + pt * D * P;
            const T z = zv[pt * bs + v];
#pragma unroll
            for (int j = 0; j < kMaxSlots; ++j) {
                if (qoff[j] >= 0) {
                    T wgt = wp[qoff[j] & 0xff];
                    if (D > 1) wgt *= wp[P + ((qoff[j] >> 8) & 0xff)];
                    if (D > 2) wgt *= wp[2 * P + ((qoff[j] >> 16) & 0xff)];
                    acc[j] += wgt * z;
                }
            }
        }
    }
    T *out = patch + (int64_t)blockIdx.x * PD * bs;
#pragma unroll
    for (int j = 0; j < kMaxSlots; ++j)
        if (qoff[j] >= 0) out[(o0 + j * ostep) * bs + v] = acc[j];
}

// Sum of the patches that cover one TS^D tile; the grid has stride bg >= bs
// (extra components written as zero).
template <class T, int D>
__global__ __launch_bounds__(256) void k_gather(TaskGeom g, int TS, int ntd,
                                                const int4 *__restrict__ tasks,
                                                const int2 *__restrict__ bin_tasks,
                                                const T *__restrict__ patch, int bg,
                                                T *__restrict__ grid) {
    extern __shared__ unsigned char smem_raw[];
    T *cp = reinterpret_cast<T *>(smem_raw);
    const int bs = g.bs, P = g.P;
    int TC = TS;
    for (int t = 1; t < D; ++t) TC *= TS;
    const int csz = TC * bs;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    T *my = cp + (size_t)wv * csz;
    for (int e = lane; e < csz; e += 64) my[e] = T(0);
    int tix[3] = {0, 0, 0};
    {
        int rem = blockIdx.x;
        for (int t = 0; t < D; ++t) { tix[t] = rem % ntd; rem /= ntd; }
    }
    int T0[3] = {0, 0, 0}, blo[3] = {0, 0, 0}, bhi[3] = {0, 0, 0};
    int PD = P;
    for (int t = 1; t < D; ++t) PD *= P;
    for (int t = 0; t < D; ++t) {
        T0[t] = tix[t] * TS;
        int a = T0[t] - g.B - g.w / 2 + 1;                 // ceil(a / B)
        int lo = a >= 0 ? (a + g.B - 1) / g.B : -((-a) / g.B);
        int hb = T0[t] + TS - 2 + g.w / 2;                 // floor(hb / B), hb >= 0
        int hi = hb / g.B;
        blo[t] = lo < 0 ? 0 : lo;
        bhi[t] = hi > g.nb - 1 ? g.nb - 1 : hi;
    }
    int ext[3] = {1, 1, 1};
    int ncand = 1;
    for (int t = 0; t < D; ++t) {
        ext[t] = bhi[t] >= blo[t] ? bhi[t] - blo[t] + 1 : 0;
        ncand *= ext[t];
    }
    __syncthreads();
    for (int c = wv; c < ncand; c += kWaves) {
        int rem = c, b3[3] = {0, 0, 0};
        for (int t = 0; t < D; ++t) { b3[t] = blo[t] + rem % ext[t]; rem /= ext[t]; }
        unsigned key = 0, mul = 1;
        for (int t = 0; t < D; ++t) { key += (unsigned)b3[t] * mul; mul *= (unsigned)g.nb; }
        const int2 bt = bin_tasks[key];
        if (bt.y == 0) continue;
        // intersection of this bin's patch with the tile
        int lo[3] = {0, 0, 0}, ex[3] = {1, 1, 1}, po[3] = {0, 0, 0};
        int tot = bs;
        for (int t = 0; t < D; ++t) {
            po[t] = b3[t] * g.B - g.w / 2 + 1;
            int a = po[t] > T0[t] ? po[t] : T0[t];
            int e2 = (po[t] + P) < (T0[t] + TS) ? (po[t] + P) : (T0[t] + TS);
            lo[t] = a;
            ex[t] = e2 - a;
            tot *= ex[t];
        }
        if (tot <= 0) continue;
        for (int tsk = bt.x; tsk < bt.x + bt.y; ++tsk) {
            const T *src = patch + (int64_t)tsk * PD * bs;
            for (int e = lane; e < tot; e += 64) {
                int vv = e % bs;
                int r = e / bs;
                int cx = r % ex[0];
                r /= ex[0];
                int cy = D > 1 ? r % ex[1] : 0;
                int cz = D > 2 ? r / ex[1] : 0;
                int gx = lo[0] + cx, gy = lo[1] + cy, gz = lo[2] + cz;
                int pidx = gx - po[0];
                int tidx = gx - T0[0];
                if (D > 1) { pidx += (gy - po[1]) * P; tidx += (gy - T0[1]) * TS; }
                if (D > 2) { pidx += (gz - po[2]) * P * P; tidx += (gz - T0[2]) * TS * TS; }
                my[tidx * bs + vv] += src[pidx * bs + vv];
            }
        }
    }
    __syncthreads();
    for (int e = tid; e < TC * bg; e += 256) {
        int vv = e % bg, cell = e / bg;
        T s = T(0);
        if (vv < bs) {
            s = cp[cell * bs + vv];
            for (int c = 1; c < kWaves; ++c) s += cp[(size_t)c * csz + cell * bs + vv];
        }
        int cx = cell % TS, cy = D > 1 ? (cell / TS) % TS : 0, cz = D > 2 ? cell / (TS * TS) : 0;
        int64_t gidx = T0[0] + cx;
        if (D > 1) gidx += (int64_t)(T0[1] + cy) * g.nos;
        if (D > 2) gidx += (int64_t)(T0[2] + cz) * g.nos * g.nos;
        grid[gidx * bg + vv] = s;
    }
}

template <class T>
struct Cplx;
template <>
struct Cplx<float> { using type = float2; };
template <>
struct Cplx<double> { using type = double2; };

// Batched radix-2 FFT of length L along lines of a [outer][L][inner] complex
// array.  A workgroup handles LB outers x IC inner columns.
template <class T>
__global__ __launch_bounds__(256) void k_fft(typename Cplx<T>::type *__restrict__ data, int L,
                                             int logL, int64_t outer_cnt, int64_t inner, int IC,
                                             int LB, int sign,
                                             const typename Cplx<T>::type *__restrict__ tw) {
    using C2 = typename Cplx<T>::type;
    extern __shared__ unsigned char smem_raw[];
    C2 *buf = reinterpret_cast<C2 *>(smem_raw);
    const int tid = threadIdx.x;
    const int64_t c0 = (int64_t)blockIdx.x * IC;
    const int64_t o0 = (int64_t)blockIdx.y * LB;
    const int lines = IC * LB;
    for (int e = tid; e < L * lines; e += 256) {
        int ln = e % lines, k = e / lines;
        int oo = ln / IC, cc = ln - oo * IC;
        int64_t o = o0 + oo;
        C2 val;
        val.x = T(0);
        val.y = T(0);
        if (o < outer_cnt) val = data[(o * L + k) * inner + c0 + cc];
        int rk = __brev((unsigned)k) >> (32 - logL);
        buf[rk * lines + ln] = val;
    }
    __syncthreads();
    for (int s = 0; s < logL; ++s) {
        const int half = 1 << s;
        const int tstride = L >> (s + 1);
        for (int e = tid; e < (L / 2) * lines; e += 256) {
            int ln = e % lines, bf = e / lines;
            int grp = bf >> s, pos = bf & (half - 1);
            int i0 = (grp << (s + 1)) + pos, i1 = i0 + half;
            C2 w = tw[pos * tstride];
            if (sign > 0) w.y = -w.y;
            C2 a = buf[i0 * lines + ln], b = buf[i1 * lines + ln];
            C2 bw;
            bw.x = b.x * w.x - b.y * w.y;
            bw.y = b.x * w.y + b.y * w.x;
            C2 r0, r1;
            r0.x = a.x + bw.x;
            r0.y = a.y + bw.y;
            r1.x = a.x - bw.x;
            r1.y = a.y - bw.y;
            buf[i0 * lines + ln] = r0;
            buf[i1 * lines + ln] = r1;
        }
        __syncthreads();
    }
    for (int e = tid; e < L * lines; e += 256) {
        int ln = e % lines, k = e / lines;
        int oo = ln / IC, cc = ln - oo * IC;
        int64_t o = o0 + oo;
        if (o < outer_cnt) data[(o * L + k) * inner + c0 + cc] = buf[k * lines + ln];
    }
}

template <class T>
__global__ void k_mul(typename Cplx<T>::type *__restrict__ grid, const T *__restrict__ M,
                      int64_t cells, int nq) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= cells * nq) return;
    const T m = M[e / nq];
    auto g = grid[e];
    g.x *= m;
    g.y *= m;
    grid[e] = g;
}

template <class T, int D>
__global__ __launch_bounds__(256) void k_interp(TaskGeom g, const int4 *__restrict__ tasks,
                                                const T *__restrict__ u,
                                                const T *__restrict__ grid, int bg, T beta,
                                                int chs, int vg, T *__restrict__ Fs) {
    extern __shared__ unsigned char smem_raw[];
    T *wts = reinterpret_cast<T *>(smem_raw);
    T *red = wts + (size_t)chs * D * g.P;
    const int4 tk = tasks[blockIdx.x];
    int bb[3];
    decode_bin((unsigned)tk.x, g.nb, D, bb);
    int org[3] = {0, 0, 0};
    for (int t = 0; t < D; ++t) org[t] = bb[t] * g.B - g.w / 2 + 1;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int P = g.P;
    int PD = P;
    for (int t = 1; t < D; ++t) PD *= P;
    const int bs = g.bs;
    const int v0 = blockIdx.y * vg;
    const int v = v0 + tid % vg;
    const int ostep = 256 / vg;
    const int o0 = tid / vg;
    int qoff[kMaxSlots];
    T h[kMaxSlots];
#pragma unroll
    for (int j = 0; j < kMaxSlots; ++j) {
        int o = o0 + j * ostep;
        int qx = o % P, qy = (o / P) % P, qz = o / (P * P);
        bool ok = o < PD;
        qoff[j] = ok ? (qx | (qy << 8) | (qz << 16)) : -1;
        T val = T(0);
        if (ok) {
            int64_t cell = org[0] + qx;
            if (D > 1) cell += (int64_t)(org[1] + qy) * g.nos;
            if (D > 2) cell += (int64_t)(org[2] + qz) * g.nos * g.nos;
            val = grid[cell * bg + v];
        }
        h[j] = val;
    }
    for (int c0 = 0; c0 < tk.z; c0 += chs) {
        const int cnt = (tk.z - c0) < chs ? (tk.z - c0) : chs;
        const int64_t first = (int64_t)tk.y + c0;
        __syncthreads();
        stage_weights<T, D>(g, u, first, cnt, org, beta, wts);
        __syncthreads();
        for (int pt = 0; pt < cnt; ++pt) {
            const T *wp = wts + pt * D * P;
            T part = T(0);
#pragma unroll
            for (int j = 0; j < kMaxSlots; ++j) {
                if (qoff[j] >= 0) {
                    T wgt = wp[qoff[j] & 0xff];
                    if (D > 1) wgt *= wp[P + ((qoff[j] >> 8) & 0xff)];
                    if (D > 2) wgt *= wp[2 * P + ((qoff[j] >> 16) & 0xff)];
                    part += wgt * h[j];
                }
            }
            for (int off = vg; off < 64; off <<= 1) part += __shfl_xor(part, off, 64);
            if (lane < vg) red[((size_t)wv * chs + pt) * vg + lane] = part;
        }
        __syncthreads();
        for (int e = tid; e < cnt * vg; e += 256) {
            T s = red[e];
            for (int c = 1; c < kWaves; ++c) s += red[(size_t)c * chs * vg + e];
            const int pt = e / vg, vv = e - pt * vg;
            Fs[(first + pt) * bs + v0 + vv] = s;
        }
    }
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
static int auto_bandwidth(double sigma_s, int d, int prec) {
    const double tol = prec == 64 ? 1e-13 : 1e-8;
    int N = 16;
    while (N < 256) {
        double x = M_PI * sigma_s * N / 2.0;
        if (2.0 * d * std::sqrt(M_PI) * sigma_s * std::exp(-x * x) <= tol) break;
        N *= 2;
    }
    return N;
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
    P.B = L.kp.bin > 0 ? L.kp.bin : 1;
    MLG_REQUIRE(P.B == 1 || P.B == 2 || P.B == 4, MLG_ERR_RANGE, "bin must be 1, 2 or 4");
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
    P.N = L.kp.N > 0 ? L.kp.N : auto_bandwidth(P.sigma_s, d, L.kp.precision);
    P.nos = 2 * P.N;
    P.nb = P.nos / P.B;
    P.nbins = 1;
    for (int t = 0; t < d; ++t) P.nbins *= P.nb;

    // --- grid coordinates, keys, sort ---
    DevBuf<double> uun((size_t)d * n);
    DevBuf<unsigned> keys(n), skeys(n);
    DevBuf<int> idx(n);
    P.perm.alloc(n);
    hipLaunchKernelGGL(k_coords_keys, dim3(ceil_div(n, 256)), dim3(256), 0, s, n, d, pts,
                       P.center[0], P.center[1], P.center[2], P.scale, P.nos, P.B, P.nb, uun.p,
                       keys.p, idx.p);
    MLG_LAUNCH_CHECK();
    unsigned endbit = 1;
    while (((int64_t)1 << endbit) < P.nbins) ++endbit;
    DevBuf<char> tmp;
    size_t tbytes = 0;
    MLG_HIP(rocprim::radix_sort_pairs(nullptr, tbytes, keys.p, skeys.p, idx.p, P.perm.p,
                                      (unsigned)n, 0u, endbit, s));
    tmp.ensure(tbytes + 1);
    MLG_HIP(rocprim::radix_sort_pairs(tmp.p, tbytes, keys.p, skeys.p, idx.p, P.perm.p,
                                      (unsigned)n, 0u, endbit, s));
    P.u64.alloc((size_t)d * n);
    P.u32.alloc((size_t)d * n);
    hipLaunchKernelGGL(k_gather_coords, dim3(ceil_div(n, 256)), dim3(256), 0, s, n, d, uun.p,
                       P.perm.p, P.u64.p, P.u32.p);
    MLG_LAUNCH_CHECK();

    // --- runs of equal bins -> tasks ---
    DevBuf<unsigned> ukeys(n), counts(n), runs_dev(1);
    tbytes = 0;
    MLG_HIP(rocprim::run_length_encode(nullptr, tbytes, skeys.p, (unsigned)n, ukeys.p, counts.p,
                                       runs_dev.p, s));
    tmp.ensure(tbytes + 1);
    MLG_HIP(rocprim::run_length_encode(tmp.p, tbytes, skeys.p, (unsigned)n, ukeys.p, counts.p,
                                       runs_dev.p, s));
    unsigned runs = 0;
    MLG_HIP(hipMemcpyAsync(&runs, runs_dev.p, 4, hipMemcpyDeviceToHost, s));
    MLG_HIP(hipStreamSynchronize(s));
    DevBuf<unsigned> run_start(runs + 1), ntask(runs + 1), task_first(runs + 1);
    tbytes = 0;
    MLG_HIP(rocprim::exclusive_scan(nullptr, tbytes, counts.p, run_start.p, 0u, (size_t)runs,
                                    rocprim::plus<unsigned>(), s));
    tmp.ensure(tbytes + 1);
    MLG_HIP(rocprim::exclusive_scan(tmp.p, tbytes, counts.p, run_start.p, 0u, (size_t)runs,
                                    rocprim::plus<unsigned>(), s));
    hipLaunchKernelGGL(k_task_counts, dim3(ceil_div(runs, 256)), dim3(256), 0, s, (int)runs,
                       counts.p, kMaxTaskPoints, ntask.p);
    MLG_LAUNCH_CHECK();
    tbytes = 0;
    MLG_HIP(rocprim::exclusive_scan(nullptr, tbytes, ntask.p, task_first.p, 0u, (size_t)runs + 1,
                                    rocprim::plus<unsigned>(), s));
    tmp.ensure(tbytes + 1);
    // ntask[runs] is scratch: make it 0 so task_first[runs] is the total
    MLG_HIP(hipMemsetAsync(ntask.p + runs, 0, 4, s));
    MLG_HIP(rocprim::exclusive_scan(tmp.p, tbytes, ntask.p, task_first.p, 0u, (size_t)runs + 1,
                                    rocprim::plus<unsigned>(), s));
    unsigned total = 0;
    MLG_HIP(hipMemcpyAsync(&total, task_first.p + runs, 4, hipMemcpyDeviceToHost, s));
    MLG_HIP(hipStreamSynchronize(s));
    P.ntasks = (int)total;
    P.tasks.alloc(total);
    P.bin_tasks.alloc(P.nbins);
    MLG_HIP(hipMemsetAsync(P.bin_tasks.p, 0, sizeof(int2) * P.nbins, s));
    hipLaunchKernelGGL(k_fill_tasks, dim3(ceil_div(runs, 256)), dim3(256), 0, s, (int)runs, ukeys.p,
                       counts.p, run_start.p, task_first.p, kMaxTaskPoints, P.tasks.p,
                       P.bin_tasks.p);
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

static int tile_edge(int d, int nos, int bs, int prec) {
    // LDS holds kWaves copies of TS^d x bs values; keep it <= 64 KB.
    const int esz = prec == 64 ? 8 : 4;
    int TS = d == 3 ? 8 : (d == 2 ? 16 : 256);
    for (;;) {
        int64_t tc = 1;
        for (int t = 0; t < d; ++t) tc *= TS;
        if ((int64_t)kWaves * tc * bs * esz <= 65536 || TS == 1) break;
        TS /= 2;
    }
    return TS > nos ? nos : TS;
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
    MLG_HIP(hipStreamSynchronize(s));
}

static int patch_side(const NfftPlan &P, const NfftWindow &W) { return P.B + W.w - 1; }

size_t nfft_patch_elems(const NfftPlan &P, const NfftWindow &W, int bs) {
    size_t pd = 1;
    for (int t = 0; t < P.d; ++t) pd *= (size_t)patch_side(P, W);
    return pd * bs * (size_t)P.ntasks;
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
static const T *coords_of(const NfftPlan &P);
template <>
const float *coords_of<float>(const NfftPlan &P) { return P.u32.p; }
template <>
const double *coords_of<double>(const NfftPlan &P) { return P.u64.p; }
template <class T>
static const typename Cplx<T>::type *tw_of(const NfftPlan &P);
template <>
const float2 *tw_of<float>(const NfftPlan &P) { return P.tw32.p; }
template <>
const double2 *tw_of<double>(const NfftPlan &P) { return P.tw64.p; }

template <class T>
static void fft_all(const NfftPlan &P, int bg, typename Cplx<T>::type *grid, int sign,
                    hipStream_t s) {
    const int L = P.nos;
    int logL = 0;
    while ((1 << logL) < L) ++logL;
    const int64_t nq = bg / 2;
    // axis 0 is fastest; line stride for axis t is nos^t * nq
    for (int ax = 0; ax < P.d; ++ax) {
        int64_t inner = nq;
        for (int t = 0; t < ax; ++t) inner *= P.nos;
        int64_t outer = 1;
        for (int t = ax + 1; t < P.d; ++t) outer *= P.nos;
        const int maxlines = std::max(1, 4096 / L);
        int IC = (int)std::min<int64_t>(inner, maxlines);
        while (inner % IC) --IC;
        int LB = std::max(1, maxlines / IC);
        if (LB > outer) LB = (int)outer;
        const size_t lds = (size_t)L * IC * LB * sizeof(typename Cplx<T>::type);
        dim3 grd((unsigned)(inner / IC), (unsigned)((outer + LB - 1) / LB));
        hipLaunchKernelGGL(k_fft<T>, grd, dim3(256), lds, s, grid, L, logL, outer, inner, IC, LB,
                           sign, tw_of<T>(P));
        MLG_LAUNCH_CHECK();
    }
}

template <class T, int D>
static void apply_d(const NfftPlan &P, const NfftWindow &W, int bs, const T *Zs, T *Fs, T *patch,
                    T *grid, hipStream_t s, hipEvent_t *ev) {
    TaskGeom g;
    g.d = D;
    g.nos = P.nos;
    g.B = P.B;
    g.nb = P.nb;
    g.w = W.w;
    g.P = patch_side(P, W);
    g.bs = bs;
    g.n = P.n;
    int PD = 1;
    for (int t = 0; t < D; ++t) PD *= g.P;
    MLG_REQUIRE(256 % bs == 0, MLG_ERR_ARG, "block stride must divide 256");
    // vectors per workgroup: the patch slots of one group must fit the
    // register budget of 256 threads
    int vg = bs;
    while (vg > 1 && (int64_t)PD * vg > (int64_t)kMaxSlots * 256) vg >>= 1;
    MLG_REQUIRE((int64_t)PD * vg <= (int64_t)kMaxSlots * 256, MLG_ERR_RANGE,
                "patch too large for one task (reduce window or bin)");
    const int ngroups = bs / vg;
    const int bg = bs < 2 ? 2 : bs;
    const T beta = (T)W.beta;
    const T *u = coords_of<T>(P);
    if (P.ntasks > 0) {
        const int per_pt = (D * g.P + bs) * (int)sizeof(T);
        int chs = std::min(kMaxTaskPoints, 49152 / per_pt);
        size_t lds = (size_t)chs * per_pt;
        hipLaunchKernelGGL((k_spread<T, D>), dim3(P.ntasks, ngroups), dim3(256), lds, s, g, P.tasks.p,
                           u, Zs, beta, chs, vg, patch);
        MLG_LAUNCH_CHECK();
    }
    if (ev) MLG_HIP(hipEventRecord(ev[1], s));
    const int TS = tile_edge(D, P.nos, bs, sizeof(T) == 8 ? 64 : 32);
    const int ntd = P.nos / TS;
    int ntiles = 1;
    for (int t = 0; t < D; ++t) ntiles *= ntd;
    int TC = 1;
    for (int t = 0; t < D; ++t) TC *= TS;
    hipLaunchKernelGGL((k_gather<T, D>), dim3(ntiles), dim3(256), (size_t)kWaves * TC * bs * sizeof(T),
                       s, g, TS, ntd, P.tasks.p, P.bin_tasks.p, patch, bg, grid);
    MLG_LAUNCH_CHECK();
    if (ev) MLG_HIP(hipEventRecord(ev[2], s));
    using C2 = typename Cplx<T>::type;
    fft_all<T>(P, bg, reinterpret_cast<C2 *>(grid), -1, s);
    int64_t G = 1;
    for (int t = 0; t < D; ++t) G *= P.nos;
    hipLaunchKernelGGL(k_mul<T>, dim3(ceil_div(G * (bg / 2), 256)), dim3(256), 0, s,
                       reinterpret_cast<C2 *>(grid), mult_of<T>(W), G, bg / 2);
    MLG_LAUNCH_CHECK();
    fft_all<T>(P, bg, reinterpret_cast<C2 *>(grid), +1, s);
    if (ev) MLG_HIP(hipEventRecord(ev[3], s));
    if (P.ntasks > 0) {
        const int per_pt = (D * g.P + kWaves * vg) * (int)sizeof(T);
        int chs = std::min(kMaxTaskPoints, 49152 / per_pt);
        size_t lds = (size_t)chs * per_pt;
        hipLaunchKernelGGL((k_interp<T, D>), dim3(P.ntasks, ngroups), dim3(256), lds, s, g, P.tasks.p,
                           u, grid, bg, beta, chs, vg, Fs);
        MLG_LAUNCH_CHECK();
    }
    if (ev) MLG_HIP(hipEventRecord(ev[4], s));
}

template <class T>
void nfft_apply(const NfftPlan &P, const NfftWindow &W, int bs, const T *Zs, T *Fs, T *patch,
                T *grid, hipStream_t s, hipEvent_t *ev) {
    switch (P.d) {
        case 1: apply_d<T, 1>(P, W, bs, Zs, Fs, patch, grid, s, ev); break;
        case 2: apply_d<T, 2>(P, W, bs, Zs, Fs, patch, grid, s, ev); break;
        case 3: apply_d<T, 3>(P, W, bs, Zs, Fs, patch, grid, s, ev); break;
        default: throw Error(MLG_ERR_RANGE, "NFFT layers need d in 1..3");
    }
}

template void nfft_apply<float>(const NfftPlan &, const NfftWindow &, int, const float *, float *,
                                float *, float *, hipStream_t, hipEvent_t *);
template void nfft_apply<double>(const NfftPlan &, const NfftWindow &, int, const double *,
                                 double *, double *, double *, hipStream_t, hipEvent_t *);

}  // namespace mlg
