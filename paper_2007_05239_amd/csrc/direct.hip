// Direct tiled summation of the kernel weight matrix (Sec. 2 case (i):
// W assembled on the fly, O(d n^2) work), zero diagonal:
//     F_i = sum_{j != i} K(x_i - x_j) Z_j     (b vectors)
// with the Gaussian K(y) = exp(-||y||^2 / sigma^2) or the Laplacian RBF
// K(y) = exp(-||y|| / sigma) (Sec. 4 names both).  The coordinates are stored
// centred on the bounding box and divided by sigma (FP64), or multiplied by
// sqrt(log2 e)/sigma (FP32 Gaussian) resp. log2(e)/sigma (FP32 Laplacian), so
// that a weight is exp(-r^2), exp2(-r^2), exp(-r) or exp2(-r) of the scaled
// distance r.
//
// The exp tile x vector block contraction runs on the matrix cores: per
// wavefront, 16 target rows against 16 source points, the 16 x 16 weight
// tile E is formed on the vector ALUs (four entries per lane, in the
// A-operand layout of the 16x16x4 MFMA) and multiplied by the 16 x 16 vector
// tile of Z with four MFMAs (blocks narrower than 16 vectors pad the tile
// with zero columns).  Rows are split over workgroups and the column range
// over a second grid dimension; the column partials are summed in a fixed
// order, so results are reproducible bit for bit.
#include "internal.h"

namespace mlg {

constexpr int kDirectMaxD = 16;
constexpr int kDmRT = 2;       // 16-row target tiles per wavefront (MFMA kernel)
constexpr int kDmRows = 4 * kDmRT * 16;  // target rows per workgroup (4 wavefronts)
constexpr int kDmJC = 128;     // source points per LDS stage (MFMA kernel)

// Weight of a scaled squared distance (see the file header); lap selects the
// Laplacian RBF.
__device__ inline float kweight(float r2, int lap) {
    return __builtin_amdgcn_exp2f(lap ? -__builtin_sqrtf(r2) : -r2);
}
__device__ inline double kweight(double r2, int lap) { return exp(lap ? -sqrt(r2) : -r2); }

// ---- MFMA kernel ------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <class T>
struct Mfma16;
template <>
struct Mfma16<float> {
    typedef f32x4 acc;
    // row of element m of lane li + 16q in the 16 x 16 result
    static __device__ inline int row(int q, int m) { return 4 * q + m; }
    static __device__ inline acc run(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <>
struct Mfma16<double> {
    typedef f64x4 acc;
    static __device__ inline int row(int q, int m) { return q + 4 * m; }
    static __device__ inline acc run(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

// 16x16x4 operand layout: A[i][k] in lane i + 16k, B[k][v] in lane v + 16k;
// the result D[i][v] sits in lane v + 16q, element m, with i = 4q + m for
// the FP32 instruction and i = q + 4m for the FP64 one.  For one 16-point source
// tile, lane i + 16q forms the weights of target i and sources 4q + r
// (r = 0..3): with k = q these are A operands of four MFMAs, the r-th taking
// B = Z[4q + r][v].  The LDS stage keeps Z in exactly that order
// (sz[tile][vtile][lane][r]) so each lane reads its four values at once.
//
// DK = d for d <= 3 (compile time), or 0 for a runtime d <= 16; VT = vector
// tiles of 16 (bs < 16 uses one tile with lanes v >= bs reading zeros).
template <class T, int DK, int VT>
__global__ __launch_bounds__(256) void k_direct_mfma(int64_t n, int d, int bs, int lap,
                                                     const T *__restrict__ x,
                                                     const T *__restrict__ Zs,
                                                     T *__restrict__ out, int64_t jchunk) {
    typedef typename Mfma16<T>::acc acc_t;
    constexpr int DMAX = DK > 0 ? DK : kDirectMaxD;
    if (DK > 0) d = DK;
    __shared__ T sc[kDmJC / 16][DMAX][16];
    __shared__ T sz[kDmJC / 16][VT][64][4];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int li = lane & 15, q = lane >> 4;
    const int64_t row0 = (int64_t)blockIdx.x * kDmRows + wave * (kDmRT * 16);
    T yi[kDmRT][DMAX];
#pragma unroll
    for (int rt = 0; rt < kDmRT; ++rt) {
        const int64_t i = row0 + rt * 16 + li;
#pragma unroll
        for (int k = 0; k < DMAX; ++k) yi[rt][k] = (k < d && i < n) ? x[(int64_t)k * n + i] : T(0);
    }
    acc_t acc[kDmRT][VT];
#pragma unroll
    for (int rt = 0; rt < kDmRT; ++rt)
#pragma unroll
        for (int vt = 0; vt < VT; ++vt) acc[rt][vt] = acc_t{0, 0, 0, 0};

    const int64_t j0 = (int64_t)blockIdx.y * jchunk;
    const int64_t j1 = (j0 + jchunk < n) ? j0 + jchunk : n;
    for (int64_t jb = j0; jb < j1; jb += kDmJC) {
        const int cnt = (int)((j1 - jb) < kDmJC ? (j1 - jb) : kDmJC);
        // every global load of the stage issued before the first LDS write
        constexpr int CI = (DMAX * kDmJC + 255) / 256, ZI = kDmJC * VT * 16 / 256;
        T cv[CI], zv[ZI];
#pragma unroll
        for (int it = 0; it < CI; ++it) {
            const int e = tid + 256 * it;
            const int k = e / kDmJC, jj = e - k * kDmJC;
            cv[it] = (k < d && jj < cnt) ? x[(int64_t)k * n + jb + jj] : T(0);
        }
#pragma unroll
        for (int it = 0; it < ZI; ++it) {
            const int e = tid + 256 * it;
            const int jj = e / (VT * 16), v = e - jj * (VT * 16);
            zv[it] = (jj < cnt && v < bs) ? Zs[(jb + jj) * bs + v] : T(0);
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < CI; ++it) {
            const int e = tid + 256 * it;
            const int k = e / kDmJC, jj = e - k * kDmJC;
            if (k < d) sc[jj >> 4][k][jj & 15] = cv[it];
        }
#pragma unroll
        for (int it = 0; it < ZI; ++it) {
            const int e = tid + 256 * it;
            const int jj = e / (VT * 16), v = e - jj * (VT * 16);
            const int jl = jj & 15;
            sz[jj >> 4][v >> 4][(v & 15) + 16 * (jl >> 2)][jl & 3] = zv[it];
        }
        __syncthreads();
        const int ntile = (cnt + 15) >> 4;
        for (int jt = 0; jt < ntile; ++jt) {
            T xs[DMAX][4];
#pragma unroll
            for (int k = 0; k < DMAX; ++k)
                if (k < d) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) xs[k][r] = sc[jt][k][4 * q + r];
                }
            T zf[VT][4];
#pragma unroll
            for (int vt = 0; vt < VT; ++vt)
#pragma unroll
                for (int r = 0; r < 4; ++r) zf[vt][r] = sz[jt][vt][lane][r];
            const int64_t jg = jb + 16 * jt;
#pragma unroll
            for (int rt = 0; rt < kDmRT; ++rt) {
                T e[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    T r2 = T(0);
#pragma unroll
                    for (int k = 0; k < DMAX; ++k)
                        if (k < d) {
                            const T dk = yi[rt][k] - xs[k][r];
                            r2 += dk * dk;
                        }
                    e[r] = kweight(r2, lap);
                }
                if (jg == row0 + rt * 16) {   // diagonal tile: zero the self pairs
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (4 * q + r == li) e[r] = T(0);
                }
#pragma unroll
                for (int vt = 0; vt < VT; ++vt)
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc[rt][vt] = Mfma16<T>::run(e[r], zf[vt][r], acc[rt][vt]);
            }
        }
    }
    T *o = out + (int64_t)blockIdx.y * n * bs;
#pragma unroll
    for (int rt = 0; rt < kDmRT; ++rt)
#pragma unroll
        for (int vt = 0; vt < VT; ++vt)
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int64_t i = row0 + rt * 16 + Mfma16<T>::row(q, m);
                const int v = vt * 16 + li;
                if (i < n && v < bs) o[i * bs + v] = acc[rt][vt][m];
            }
}

// Fs[e] = sum_{s < S} part[s*n*bs + e], s ascending.
template <class T>
__global__ void k_direct_reduce(int64_t total, int S, const T *__restrict__ part,
                                T *__restrict__ Fs) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    T acc = part[e];
    for (int s = 1; s < S; ++s) acc += part[(int64_t)s * total + e];
    Fs[e] = acc;
}

// ---- coordinates -----------------------------------------------------------------
// Per dimension (one workgroup each): bounding-box midpoint, or NaN if a
// coordinate of that dimension is not finite (fmin/fmax would skip a NaN).
__global__ __launch_bounds__(256) void k_bbox_mid(int64_t n, int d, const double *__restrict__ pts,
                                                  double *__restrict__ mid) {
    __shared__ double lo[256], hi[256];
    __shared__ int bad[256];
    const int k = blockIdx.x;
    double a = pts[k], b = pts[k];
    int nf = 0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const double v = pts[i * d + k];
        nf |= !isfinite(v);
        a = fmin(a, v);
        b = fmax(b, v);
    }
    lo[threadIdx.x] = a;
    hi[threadIdx.x] = b;
    bad[threadIdx.x] = nf;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            lo[threadIdx.x] = fmin(lo[threadIdx.x], lo[threadIdx.x + h]);
            hi[threadIdx.x] = fmax(hi[threadIdx.x], hi[threadIdx.x + h]);
            bad[threadIdx.x] |= bad[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) mid[k] = bad[0] ? __builtin_nan("") : 0.5 * (lo[0] + hi[0]);
}

// x64 = (x - mid) s64, x32 = (x - mid) s32, SoA d x n.
__global__ void k_direct_coords(int64_t n, int d, const double *__restrict__ pts,
                                const double *__restrict__ mid, double s64, double s32,
                                double *__restrict__ x64, float *__restrict__ x32) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int k = 0; k < d; ++k) {
        const double c = pts[i * d + k] - mid[k];
        x64[(int64_t)k * n + i] = c * s64;
        x32[(int64_t)k * n + i] = (float)(c * s32);
    }
}

void direct_coords_into(int64_t n, int d, const double *pts_dev, double sigma, int kernel,
                        double *mid, double *x64, float *x32, hipStream_t s) {
    MLG_REQUIRE(d >= 1 && d <= kDirectMaxD, MLG_ERR_RANGE, "direct summation supports d <= 16");
    hipLaunchKernelGGL(k_bbox_mid, dim3(d), dim3(256), 0, s, n, d, pts_dev, mid);
    MLG_LAUNCH_CHECK();
    const double log2e = 1.4426950408889634;
    const double s32 = (kernel == MLG_KERNEL_LAPLACIAN ? log2e : std::sqrt(log2e)) / sigma;
    hipLaunchKernelGGL(k_direct_coords, dim3(ceil_div(n, 256)), dim3(256), 0, s, n, d, pts_dev, mid,
                       1.0 / sigma, s32, x64, x32);
    MLG_LAUNCH_CHECK();
}

void direct_coords(int64_t n, int d, const double *pts_dev, double sigma, int kernel,
                   DevBuf<double> &x64, DevBuf<float> &x32, hipStream_t s) {
    MLG_REQUIRE(d >= 1 && d <= kDirectMaxD, MLG_ERR_RANGE, "direct summation supports d <= 16");
    DevBuf<double> mid(d);
    x64.alloc((size_t)n * d);
    x32.alloc((size_t)n * d);
    direct_coords_into(n, d, pts_dev, sigma, kernel, mid.p, x64.p, x32.p, s);
    double hm[kDirectMaxD];
    MLG_HIP(hipMemcpyAsync(hm, mid.p, sizeof(double) * d, hipMemcpyDeviceToHost, s));
    MLG_HIP(hipStreamSynchronize(s));
    for (int k = 0; k < d; ++k)
        MLG_REQUIRE(std::isfinite(hm[k]), MLG_ERR_ARG, "point coordinates must be finite");
}

// ---- launch ------------------------------------------------------------------------
// Column splits: enough workgroups to fill the chip, each split a multiple
// of the LDS stage.
static int direct_splits(int64_t n, int rows_per_wg, int stage) {
    const int rb = ceil_div(n, rows_per_wg);
    int S = ceil_div(1024, rb);
    const int maxS = ceil_div(n, 4 * stage);
    if (S > maxS) S = maxS;
    return S < 1 ? 1 : S;
}

static void split_plan(int64_t n, int bs, int &S, int64_t &jchunk) {
    (void)bs;
    const int stage = kDmJC;
    S = direct_splits(n, kDmRows, stage);
    jchunk = (n + S - 1) / S;
    jchunk = (jchunk + stage - 1) / stage * stage;
    S = (int)((n + jchunk - 1) / jchunk);
}

template <class T>
size_t direct_part_size(int64_t n, int bs) {
    int S;
    int64_t jchunk;
    split_plan(n, bs, S, jchunk);
    return S > 1 ? (size_t)S * n * bs : 0;
}

template <class T, int DK>
static void launch_mfma_d(int64_t n, int d, int bs, int lap, const T *x, const T *Zs, T *dst, int S,
                          int64_t jchunk, hipStream_t s) {
    const dim3 grid(ceil_div(n, kDmRows), S);
    switch (bs) {
        case 1:
        case 2:
        case 4:
        case 8:
        case 16:
            hipLaunchKernelGGL((k_direct_mfma<T, DK, 1>), grid, dim3(256), 0, s, n, d, bs, lap, x, Zs, dst,
                               jchunk);
            break;
        case 32:
            hipLaunchKernelGGL((k_direct_mfma<T, DK, 2>), grid, dim3(256), 0, s, n, d, bs, lap, x, Zs, dst,
                               jchunk);
            break;
        case 64:
            hipLaunchKernelGGL((k_direct_mfma<T, DK, 4>), grid, dim3(256), 0, s, n, d, bs, lap, x, Zs, dst,
                               jchunk);
            break;
        default: throw Error(MLG_ERR_ARG, "direct: unsupported block stride");
    }
    MLG_LAUNCH_CHECK();
}

template <class T>
void launch_direct(int64_t n, int d, int kernel, const T *x, int bs, const T *Zs, T *Fs, T *part,
                   size_t part_cap, hipStream_t s) {
    const int lap = kernel == MLG_KERNEL_LAPLACIAN ? 1 : 0;
    MLG_REQUIRE(d >= 1 && d <= kDirectMaxD, MLG_ERR_RANGE, "direct summation supports d <= 16");
    int S;
    int64_t jchunk;
    split_plan(n, bs, S, jchunk);
    T *dst = Fs;
    if (S > 1) {
        MLG_REQUIRE(part && part_cap >= (size_t)S * n * bs, MLG_ERR_ARG, "direct: workspace too small");
        dst = part;
    }
    switch (d) {
        case 1: launch_mfma_d<T, 1>(n, d, bs, lap, x, Zs, dst, S, jchunk, s); break;
        case 2: launch_mfma_d<T, 2>(n, d, bs, lap, x, Zs, dst, S, jchunk, s); break;
        case 3: launch_mfma_d<T, 3>(n, d, bs, lap, x, Zs, dst, S, jchunk, s); break;
        default: launch_mfma_d<T, 0>(n, d, bs, lap, x, Zs, dst, S, jchunk, s); break;
    }
    if (S > 1) {
        const int64_t total = n * bs;
        hipLaunchKernelGGL(k_direct_reduce<T>, dim3(ceil_div(total, 256)), dim3(256), 0, s, total, S,
                           part, Fs);
        MLG_LAUNCH_CHECK();
    }
}

template void launch_direct<float>(int64_t, int, int, const float *, int, const float *, float *,
                                   float *, size_t, hipStream_t);
template void launch_direct<double>(int64_t, int, int, const double *, int, const double *, double *,
                                    double *, size_t, hipStream_t);
template size_t direct_part_size<float>(int64_t, int);
template size_t direct_part_size<double>(int64_t, int);

}  // namespace mlg
