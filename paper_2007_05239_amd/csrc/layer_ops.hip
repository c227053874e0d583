// Entry and exit of a block matvec, around each layer's summation:
//   scatter-in   z_t = D_t^-1/2 x for every layer t, written in the layer's
//                sorted point order and cast to its summation precision
//                (Sec. 2, L_sym = I - D^-1/2 W D^-1/2);
//   gather-out   y = coef sum_t D_t^-1/2 (F_t - K(0) z_t) in FP64, with the
//                self term of W = W~ - K(0) I (Sec. 4) and the layer mean
//                (1/T) sum_t (Sec. 3); y = x - that for L_sym / L_1.
// Both move 64 rows of the column-major block through LDS so that the
// column-major side and the point-major side are both coalesced.  The layer
// sum runs in layer order.
#include "internal.h"

namespace mlg {

template <class T>
__device__ inline void store_z(void *Z, int64_t idx, double v) {
    reinterpret_cast<T *>(Z)[idx] = (T)v;
}

__global__ __launch_bounds__(256) void k_scatter_in(int64_t n, int b, int bs,
                                                    const double *__restrict__ X, int64_t ldx,
                                                    const LayerIO *__restrict__ L, int nl,
                                                    int use_dinv) {
    __shared__ double tile[64 * 65];
    const int64_t i0 = (int64_t)blockIdx.x * 64;
    const int rows = (int)((n - i0) < 64 ? (n - i0) : 64);
    for (int e = threadIdx.x; e < 64 * b; e += blockDim.x) {
        const int r = e & 63, v = e >> 6;
        if (r < rows) tile[v * 65 + r] = X[i0 + r + (int64_t)v * ldx];
    }
    __syncthreads();
    for (int t = 0; t < nl; ++t) {
        const LayerIO d = L[t];
        for (int e = threadIdx.x; e < rows * bs; e += blockDim.x) {
            const int r = e / bs, v = e - r * bs;
            const int64_t i = i0 + r;
            const int64_t p = d.invperm ? d.invperm[i] : i;
            double z = 0.0;
            if (v < b) {
                z = tile[v * 65 + r];
                if (use_dinv) z *= d.dinv[i];
            }
            if (d.is64) store_z<double>(d.Z, p * bs + v, z);
            else store_z<float>(d.Z, p * bs + v, z);
        }
    }
}

__global__ __launch_bounds__(256) void k_gather_out(int64_t n, int b, int bs,
                                                    const double *__restrict__ X, int64_t ldx,
                                                    double *__restrict__ Y, int64_t ldy,
                                                    const LayerIO *__restrict__ L, int nl,
                                                    int use_dinv, int lsym, double coef) {
    __shared__ double tile[64 * 65];
    const int64_t i0 = (int64_t)blockIdx.x * 64;
    const int rows = (int)((n - i0) < 64 ? (n - i0) : 64);
    for (int e = threadIdx.x; e < 64 * b; e += blockDim.x) {
        const int r = e & 63, v = e >> 6;
        if (r < rows) tile[v * 65 + r] = X[i0 + r + (int64_t)v * ldx];
    }
    __syncthreads();
    // each (row, vector) element is read and rewritten by one thread only
    for (int e = threadIdx.x; e < rows * b; e += blockDim.x) {
        const int r = e / b, v = e - r * b;
        const int64_t i = i0 + r;
        const double x = tile[v * 65 + r];
        double acc = 0.0;
        for (int t = 0; t < nl; ++t) {
            const LayerIO d = L[t];
            const int64_t p = d.invperm ? d.invperm[i] : i;
            const double di = use_dinv ? d.dinv[i] : 1.0;
            double zx = use_dinv ? x * di : x;
            double f, z;
            if (d.is64) {
                f = reinterpret_cast<const double *>(d.F)[p * bs + v];
                z = zx;
            } else {
                f = (double)reinterpret_cast<const float *>(d.F)[p * bs + v];
                z = (double)(float)zx;       // the value the FP32 summation saw
            }
            double w = f - d.K0 * z;
            if (use_dinv) w *= di;
            acc += w;
        }
        double y = coef * acc;
        if (lsym) y = x - y;
        tile[v * 65 + r] = y;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * b; e += blockDim.x) {
        const int r = e & 63, v = e >> 6;
        if (r < rows) Y[i0 + r + (int64_t)v * ldy] = tile[v * 65 + r];
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

// inv[perm[p]] = p.
__global__ void k_invperm(int64_t n, const int *perm, int *inv) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) inv[perm[p]] = (int)p;
}

static inline unsigned blocks_for(int64_t work, int threads) {
    return (unsigned)((work + threads - 1) / threads);
}

void launch_scatter_in(int64_t n, int b, int bs, const double *X, int64_t ldx, const LayerIO *L,
                       int nl, int use_dinv, hipStream_t s) {
    MLG_REQUIRE(bs <= 64 && b <= bs, MLG_ERR_ARG, "block too wide");
    hipLaunchKernelGGL(k_scatter_in, dim3(blocks_for(n, 64)), dim3(256), 0, s, n, b, bs, X, ldx, L, nl,
                       use_dinv);
    MLG_LAUNCH_CHECK();
}

void launch_gather_out(int64_t n, int b, int bs, const double *X, int64_t ldx, double *Y,
                       int64_t ldy, const LayerIO *L, int nl, int use_dinv, int lsym, double coef,
                       hipStream_t s) {
    MLG_REQUIRE(bs <= 64 && b <= bs, MLG_ERR_ARG, "block too wide");
    hipLaunchKernelGGL(k_gather_out, dim3(blocks_for(n, 64)), dim3(256), 0, s, n, b, bs, X, ldx, Y, ldy,
                       L, nl, use_dinv, lsym, coef);
    MLG_LAUNCH_CHECK();
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

void launch_dinv(int64_t n, const double *deg, double *dinv, hipStream_t s) {
    hipLaunchKernelGGL(k_dinv, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, deg, dinv);
    MLG_LAUNCH_CHECK();
}

void launch_invperm(int64_t n, const int *perm, int *inv, hipStream_t s) {
    hipLaunchKernelGGL(k_invperm, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, perm, inv);
    MLG_LAUNCH_CHECK();
}

}  // namespace mlg
