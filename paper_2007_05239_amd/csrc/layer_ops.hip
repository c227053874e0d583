// Entry and exit of a block matvec, around each layer's summation:
//   scatter-in   z_t = D_t^-1/2 x for every layer t, cast to its summation
//                precision, in node order (Sec. 2, L_sym = I - D^-1/2 W D^-1/2);
//   gather-out   y = coef sum_t D_t^-1/2 (F_t - K(0) z_t) in FP64, with the
//                self term of W = W~ - K(0) I (Sec. 4) and the layer mean
//                (1/T) sum_t (Sec. 3); y = x - that for L_sym / L_1.
// The entry kernel gives one thread a row, the exit kernel a row's group of
// kOutVG vectors (D^-1/2 is read once per layer and thread).  The layer sum
// runs in layer order.
#include "internal.h"

namespace mlg {

// Thread per row, vectors in groups of VG = 16 (or bs if smaller): a
// thread reads its row of the column-major block column by column (each
// column access is contiguous across the workgroup's threads), with every
// load of the group issued before the first use, and writes or reads the
// layer's sorted row (bs consecutive values) with vector accesses.
constexpr int kIoVG = 16;

template <class T>
__device__ inline void store_row(void *Zbase, int64_t off, const double (&z)[kIoVG], int cnt) {
    T *dst = reinterpret_cast<T *>(Zbase) + off;
    if constexpr (sizeof(T) == 4) {
        if (cnt == 16) {
#pragma unroll
            for (int j = 0; j < 16; j += 4)
                *reinterpret_cast<float4 *>(dst + j) =
                    make_float4((float)z[j], (float)z[j + 1], (float)z[j + 2], (float)z[j + 3]);
            return;
        }
    }
    for (int j = 0; j < cnt; ++j) dst[j] = (T)z[j];
}

template <class T>
__device__ inline void load_row(const void *Fbase, int64_t off, double (&f)[kIoVG], int cnt) {
    const T *src = reinterpret_cast<const T *>(Fbase) + off;
    if constexpr (sizeof(T) == 4) {
        if (cnt == 16) {
#pragma unroll
            for (int j = 0; j < 16; j += 4) {
                const float4 q = *reinterpret_cast<const float4 *>(src + j);
                f[j] = q.x; f[j + 1] = q.y; f[j + 2] = q.z; f[j + 3] = q.w;
            }
            return;
        }
    }
    for (int j = 0; j < cnt; ++j) f[j] = (double)src[j];
}

__device__ inline void load_block_row(const double *__restrict__ X, int64_t ldx, int64_t i, int b,
                                      int v0, int vgw, double (&x)[kIoVG]) {
#pragma unroll
    for (int j = 0; j < kIoVG; ++j)
        x[j] = (j < vgw && v0 + j < b) ? X[i + (int64_t)(v0 + j) * ldx] : 0.0;
}

// FP32 layer slices are written through an LDS tile of the block's 256 rows
// (row-major, bs + 1 floats per row), so that each block stores one
// contiguous, fully coalesced region of the slice; FP64 slices are stored
// row by row.  kIoTile: the largest block stride with an LDS tile.  (The
// exit kernel reads its slices row by row: one wavefront's rows are already
// one contiguous region there, and an LDS round trip per layer costs more
// than it saves.)
constexpr int kIoTile = 32;

__global__ __launch_bounds__(256) void k_scatter_in(int64_t n, int b, int bs,
                                                    const double *__restrict__ X, int64_t ldx,
                                                    const LayerIO *__restrict__ L, int nl,
                                                    int use_dinv, float *__restrict__ X32) {
    __shared__ float tile[256 * (kIoTile + 1)];
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x;
    const int64_t i = i0 + threadIdx.x;
    const bool live = i < n;
    const int rows = (n - i0) < 256 ? (int)(n - i0) : 256;
    const int vgw = bs < kIoVG ? bs : kIoVG;
    const int ng = (bs + vgw - 1) / vgw;
    const bool tiled = bs <= kIoTile;
    const int ldt = bs + 1;
    constexpr int NG = kIoTile / kIoVG;
    double x[NG][kIoVG];
#pragma unroll
    for (int gi = 0; gi < NG; ++gi) {
        if (tiled && live && gi < ng) load_block_row(X, ldx, i, b, gi * vgw, vgw, x[gi]);
        else
#pragma unroll
            for (int j = 0; j < kIoVG; ++j) x[gi][j] = 0.0;
    }
    // the shared FP32 slice of x (layers marked shared scale it themselves)
    if (X32) {
        if (tiled) {
#pragma unroll
            for (int gi = 0; gi < NG; ++gi)
                if (gi < ng)
#pragma unroll
                    for (int j = 0; j < kIoVG; ++j)
                        if (j < vgw) tile[threadIdx.x * ldt + gi * vgw + j] = (float)x[gi][j];
            __syncthreads();
            float *dst = X32 + i0 * bs;
            for (int e = threadIdx.x; e < rows * bs; e += 256) {
                const int r = e / bs, c = e - r * bs;
                dst[e] = tile[r * ldt + c];
            }
            __syncthreads();
        } else if (live) {
            for (int v0 = 0; v0 < bs; v0 += vgw) {
                double xr[kIoVG];
                load_block_row(X, ldx, i, b, v0, vgw, xr);
                store_row<float>(X32, i * bs + v0, xr, vgw);
            }
        }
    }
    for (int t = 0; t < nl; ++t) {
        const LayerIO d = L[t];
        if (d.shared) continue;
        if (tiled && !d.is64) {
            const double di = (use_dinv && live) ? d.dinv[i] : 1.0;
#pragma unroll
            for (int gi = 0; gi < NG; ++gi)
                if (gi < ng)
#pragma unroll
                    for (int j = 0; j < kIoVG; ++j)
                        if (j < vgw)
                            tile[threadIdx.x * ldt + gi * vgw + j] =
                                (float)(use_dinv ? x[gi][j] * di : x[gi][j]);
            __syncthreads();
            float *dst = reinterpret_cast<float *>(d.Z) + i0 * bs;
            for (int e = threadIdx.x; e < rows * bs; e += 256) {
                const int r = e / bs, c = e - r * bs;
                dst[e] = tile[r * ldt + c];
            }
            __syncthreads();
        } else if (live) {
            const double di = use_dinv ? d.dinv[i] : 1.0;
            for (int v0 = 0; v0 < bs; v0 += vgw) {
                double xr[kIoVG];
                load_block_row(X, ldx, i, b, v0, vgw, xr);
                double z[kIoVG];
#pragma unroll
                for (int j = 0; j < kIoVG; ++j) z[j] = use_dinv ? xr[j] * di : xr[j];
                if (d.is64) store_row<double>(d.Z, i * bs + v0, z, vgw);
                else store_row<float>(d.Z, i * bs + v0, z, vgw);
            }
        }
    }
}

// Exit kernel: one thread per (row, group of kOutVG vectors), the groups of
// a row in adjacent threads, so that a wavefront reads 64 / ng consecutive
// rows of each layer's slice as one region and keeps few registers per
// thread (the one-thread-per-row form held 16 vectors in flight per thread
// at 2 wavefronts per SIMD).  Per vector the arithmetic and its order are
// those of the layer sum described at the top of the file.
constexpr int kOutVG = 8;

__device__ inline void load_row8(const void *Fbase, bool is64, int64_t off, double (&f)[kOutVG],
                                 int cnt) {
    if (!is64) {
        const float *src = reinterpret_cast<const float *>(Fbase) + off;
        if (cnt == kOutVG) {
            const float4 a = *reinterpret_cast<const float4 *>(src);
            const float4 c = *reinterpret_cast<const float4 *>(src + 4);
            f[0] = a.x; f[1] = a.y; f[2] = a.z; f[3] = a.w;
            f[4] = c.x; f[5] = c.y; f[6] = c.z; f[7] = c.w;
            return;
        }
#pragma unroll
        for (int j = 0; j < kOutVG; ++j) f[j] = j < cnt ? (double)src[j] : 0.0;
    } else {
        const double *src = reinterpret_cast<const double *>(Fbase) + off;
        if (cnt == kOutVG) {
#pragma unroll
            for (int j = 0; j < kOutVG; j += 2) {
                const double2 q = *reinterpret_cast<const double2 *>(src + j);
                f[j] = q.x;
                f[j + 1] = q.y;
            }
            return;
        }
#pragma unroll
        for (int j = 0; j < kOutVG; ++j) f[j] = j < cnt ? src[j] : 0.0;
    }
}

__global__ __launch_bounds__(256) void k_gather_out(int64_t n, int b, int bs, int lng,
                                                    const double *__restrict__ X, int64_t ldx,
                                                    double *__restrict__ Y, int64_t ldy,
                                                    const LayerIO *__restrict__ L, int nl,
                                                    int use_dinv, int lsym, double coef) {
    const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = gt >> lng;
    if (i >= n) return;
    const int v0 = (int)(gt & ((1 << lng) - 1)) * kOutVG;
    const int vgw = bs < kOutVG ? bs : kOutVG;
    double x[kOutVG], acc[kOutVG];
#pragma unroll
    for (int j = 0; j < kOutVG; ++j) {
        x[j] = (j < vgw && v0 + j < b) ? X[i + (int64_t)(v0 + j) * ldx] : 0.0;
        acc[j] = 0.0;
    }
    for (int t = 0; t < nl; ++t) {
        const LayerIO d = L[t];
        const double di = use_dinv ? d.dinv[i] : 1.0;
        double f[kOutVG];
        load_row8(d.F, d.is64, i * bs + v0, f, vgw);
#pragma unroll
        for (int j = 0; j < kOutVG; ++j) {
            if (j < vgw) {
                const double zx = use_dinv ? x[j] * di : x[j];
                // the value the summation saw (FP32 layers round it; a shared
                // slice gives the FP32 product of the rounded factors)
                const double z = d.is64 ? zx
                                 : d.shared ? (double)(use_dinv ? (float)x[j] * (float)di : (float)x[j])
                                            : (double)(float)zx;
                double w = f[j] - d.K0 * z;
                if (use_dinv) w *= di;
                acc[j] += w;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < kOutVG; ++j) {
        if (j < vgw && v0 + j < b) {
            double y = coef * acc[j];
            if (lsym) y = x[j] - y;
            Y[i + (int64_t)(v0 + j) * ldy] = y;
        }
    }
}

__global__ void k_fill_ones(int64_t n, double *Xr) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) Xr[i] = 1.0;
}

// flag := 1 if some degree is below thresh (each offender writes the same 1).
__global__ void k_check_degrees(int64_t n, const double *deg, double thresh, int *flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !(deg[i] > thresh)) flag[0] = 1;
}

// dinv[i] = 1/sqrt(deg[i]).
__global__ void k_dinv(int64_t n, const double *deg, double *dinv) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dinv[i] = 1.0 / sqrt(deg[i]);
}

__global__ void k_sorted_f32(int64_t n, const int *__restrict__ perm, const double *__restrict__ src,
                             float *__restrict__ dst) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) dst[p] = (float)src[perm[p]];
}

static inline unsigned blocks_for(int64_t work, int threads) {
    return (unsigned)((work + threads - 1) / threads);
}

void launch_scatter_in(int64_t n, int b, int bs, const double *X, int64_t ldx, const LayerIO *L,
                       int nl, int use_dinv, hipStream_t s, float *X32) {
    MLG_REQUIRE(bs <= 64 && b <= bs, MLG_ERR_ARG, "block too wide");
    hipLaunchKernelGGL(k_scatter_in, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, b, bs, X, ldx, L,
                       nl, use_dinv, X32);
    MLG_LAUNCH_CHECK();
}

void launch_gather_out(int64_t n, int b, int bs, const double *X, int64_t ldx, double *Y,
                       int64_t ldy, const LayerIO *L, int nl, int use_dinv, int lsym, double coef,
                       hipStream_t s) {
    MLG_REQUIRE(bs <= 64 && b <= bs, MLG_ERR_ARG, "block too wide");
    // groups of kOutVG vectors per row; a power-of-two stride above kOutVG
    // is a whole number of groups, so no group reads past its row
    MLG_REQUIRE(bs >= 1 && (bs & (bs - 1)) == 0, MLG_ERR_ARG, "block stride must be a power of two");
    int lng = 0;
    while ((kOutVG << lng) < bs) ++lng;
    hipLaunchKernelGGL(k_gather_out, dim3(blocks_for(n << lng, 256)), dim3(256), 0, s, n, b, bs, lng,
                       X, ldx, Y, ldy, L, nl, use_dinv, lsym, coef);
    MLG_LAUNCH_CHECK();
}

static bool node_runs(hipGraphNode_t node, const void *fn) {
    hipGraphNodeType t;
    if (hipGraphNodeGetType(node, &t) != hipSuccess || t != hipGraphNodeTypeKernel) return false;
    hipKernelNodeParams p{};
    MLG_HIP(hipGraphKernelNodeGetParams(node, &p));
    return p.func == fn;
}

bool is_scatter_in_node(hipGraphNode_t node) {
    return node_runs(node, reinterpret_cast<const void *>(&k_scatter_in));
}

bool is_gather_out_node(hipGraphNode_t node) {
    return node_runs(node, reinterpret_cast<const void *>(&k_gather_out));
}

// The argument lists below follow the kernels' parameter lists exactly (types
// included); the grid, block and function come from the captured node.
void set_scatter_in_node(hipGraphExec_t e, hipGraphNode_t node, int64_t n, int b, int bs,
                         const double *X, int64_t ldx, const LayerIO *L, int nl, int use_dinv,
                         float *X32) {
    hipKernelNodeParams p{};
    MLG_HIP(hipGraphKernelNodeGetParams(node, &p));
    void *args[] = {&n, &b, &bs, &X, &ldx, &L, &nl, &use_dinv, &X32};
    p.kernelParams = args;
    p.extra = nullptr;
    MLG_HIP(hipGraphExecKernelNodeSetParams(e, node, &p));
}

void set_gather_out_node(hipGraphExec_t e, hipGraphNode_t node, int64_t n, int b, int bs,
                         const double *X, int64_t ldx, double *Y, int64_t ldy, const LayerIO *L,
                         int nl, int use_dinv, int lsym, double coef) {
    hipKernelNodeParams p{};
    MLG_HIP(hipGraphKernelNodeGetParams(node, &p));
    int lng = 0;
    while ((kOutVG << lng) < bs) ++lng;
    void *args[] = {&n, &b, &bs, &lng, &X, &ldx, &Y, &ldy, &L, &nl, &use_dinv, &lsym, &coef};
    p.kernelParams = args;
    p.extra = nullptr;
    MLG_HIP(hipGraphExecKernelNodeSetParams(e, node, &p));
}

void launch_fill_ones(int64_t n, double *Xr, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_ones, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, Xr);
    MLG_LAUNCH_CHECK();
}

void launch_check_degrees(int64_t n, const double *deg, double thresh, int *flag, hipStream_t s) {
    hipLaunchKernelGGL(k_check_degrees, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, deg, thresh,
                       flag);
    MLG_LAUNCH_CHECK();
}

void launch_sorted_f32(int64_t n, const int *perm, const double *src, float *dst, hipStream_t s) {
    hipLaunchKernelGGL(k_sorted_f32, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, perm, src, dst);
    MLG_LAUNCH_CHECK();
}

void launch_dinv(int64_t n, const double *deg, double *dinv, hipStream_t s) {
    hipLaunchKernelGGL(k_dinv, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, deg, dinv);
    MLG_LAUNCH_CHECK();
}


}  // namespace mlg
