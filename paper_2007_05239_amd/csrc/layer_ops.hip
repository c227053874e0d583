// Block layout changes and the FP64 scalings around each layer's summation:
// z = D^-1/2 x (Sec. 2, L_sym), the self term of W = W~ - K(0) I (Sec. 4),
// and the layer mean (1/T) sum_t (Sec. 3).
#include "internal.h"

namespace mlg {

// Column-major n x b (leading dim ldx) -> point-major Xr[i*b + v].
// One workgroup moves 64 rows through LDS so both sides are coalesced.
__global__ void k_to_rowmajor(int64_t n, int b, const double *__restrict__ X, int64_t ldx,
                              double *__restrict__ Xr) {
    __shared__ double tile[64 * 65];
    const int64_t i0 = (int64_t)blockIdx.x * 64;
    const int rows = (int)((n - i0) < 64 ? (n - i0) : 64);
    for (int e = threadIdx.x; e < 64 * b; e += blockDim.x) {
        int r = e & 63, v = e >> 6;
        if (r < rows) tile[v * 65 + r] = X[i0 + r + (int64_t)v * ldx];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < rows * b; e += blockDim.x) {
        int r = e / b, v = e - r * b;
        Xr[(i0 + r) * b + v] = tile[v * 65 + r];
    }
}

// Y[i + v*ldy] = (lsym ? X[i + v*ldx] - Yr[i*b+v] : Yr[i*b+v]).
__global__ void k_finish(int64_t n, int b, const double *__restrict__ Yr,
                         const double *__restrict__ X, int64_t ldx, double *__restrict__ Y,
                         int64_t ldy, int lsym) {
    __shared__ double tile[64 * 65];
    const int64_t i0 = (int64_t)blockIdx.x * 64;
    const int rows = (int)((n - i0) < 64 ? (n - i0) : 64);
    for (int e = threadIdx.x; e < rows * b; e += blockDim.x) {
        int r = e / b, v = e - r * b;
        tile[v * 65 + r] = Yr[(i0 + r) * b + v];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * b; e += blockDim.x) {
        int r = e & 63, v = e >> 6;
        if (r < rows) {
            double y = tile[v * 65 + r];
            if (lsym) y = X[i0 + r + (int64_t)v * ldx] - y;
            Y[i0 + r + (int64_t)v * ldy] = y;
        }
    }
}

// Zs[p*bs + v] = T(dinv[p] * Xr[perm[p]*b + v]) for v < b, 0 for b <= v < bs.
template <class T>
__global__ void k_pre(int64_t n, int b, int bs, const int *__restrict__ perm,
                      const double *__restrict__ dinv, const double *__restrict__ Xr,
                      T *__restrict__ Zs) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * bs) return;
    const int64_t p = e / bs;
    const int v = (int)(e - p * bs);
    T out = T(0);
    if (v < b) {
        const int64_t i = perm ? perm[p] : p;
        double z = Xr[i * b + v];
        if (dinv) z *= dinv[p];
        out = (T)z;
    }
    Zs[e] = out;
}

// y = coef * dinv[p] * (F - K0 * Z) in FP64, stored (or added) at row perm[p].
template <class T>
__global__ void k_post(int64_t n, int b, int bs, const int *__restrict__ perm,
                       const double *__restrict__ dinv, double coef, double K0,
                       const T *__restrict__ Fs, const T *__restrict__ Zs,
                       double *__restrict__ Yr, int accumulate) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * (int64_t)b) return;
    const int64_t p = e / b;
    const int v = (int)(e - p * b);
    double f = (double)Fs[p * bs + v];
    if (K0 != 0.0) f -= K0 * (double)Zs[p * bs + v];
    double sc = coef;
    if (dinv) sc *= dinv[p];
    const int64_t i = perm ? perm[p] : p;
    double y = sc * f;
    double *dst = Yr + i * b + v;
    *dst = accumulate ? *dst + y : y;
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

// dinv_s[p] = 1/sqrt(deg[perm[p]]).
__global__ void k_dinv(int64_t n, const double *deg, const int *perm, double *dinv_s) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) dinv_s[p] = 1.0 / sqrt(deg[perm ? perm[p] : p]);
}

static inline unsigned blocks_for(int64_t work, int threads) {
    return (unsigned)((work + threads - 1) / threads);
}

void launch_to_rowmajor(int64_t n, int b, const double *X, int64_t ldx, double *Xr, hipStream_t s) {
    hipLaunchKernelGGL(k_to_rowmajor, dim3(blocks_for(n, 64)), dim3(256), 0, s, n, b, X, ldx, Xr);
    MLG_LAUNCH_CHECK();
}

void launch_finish(int64_t n, int b, const double *Yr, const double *X, int64_t ldx, double *Y,
                   int64_t ldy, int lsym, hipStream_t s) {
    hipLaunchKernelGGL(k_finish, dim3(blocks_for(n, 64)), dim3(256), 0, s, n, b, Yr, X, ldx, Y,
                       ldy, lsym);
    MLG_LAUNCH_CHECK();
}

template <class T>
void launch_pre(int64_t n, int b, int bs, const int *perm, const double *dinv, const double *Xr,
                T *Zs, hipStream_t s) {
    hipLaunchKernelGGL(k_pre<T>, dim3(blocks_for(n * bs, 256)), dim3(256), 0, s, n, b, bs, perm,
                       dinv, Xr, Zs);
    MLG_LAUNCH_CHECK();
}

template <class T>
void launch_post(int64_t n, int b, int bs, const int *perm, const double *dinv, double coef,
                 double K0, const T *Fs, const T *Zs, double *Yr, int accumulate, hipStream_t s) {
    hipLaunchKernelGGL(k_post<T>, dim3(blocks_for(n * b, 256)), dim3(256), 0, s, n, b, bs, perm,
                       dinv, coef, K0, Fs, Zs, Yr, accumulate);
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

void launch_dinv(int64_t n, const double *deg, const int *perm, double *dinv_s, hipStream_t s) {
    hipLaunchKernelGGL(k_dinv, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, deg, perm, dinv_s);
    MLG_LAUNCH_CHECK();
}

template void launch_pre<float>(int64_t, int, int, const int *, const double *, const double *,
                                float *, hipStream_t);
template void launch_pre<double>(int64_t, int, int, const int *, const double *, const double *,
                                 double *, hipStream_t);
template void launch_post<float>(int64_t, int, int, const int *, const double *, double, double,
                                 const float *, const float *, double *, int, hipStream_t);
template void launch_post<double>(int64_t, int, int, const int *, const double *, double, double,
                                  const double *, const double *, double *, int, hipStream_t);

}  // namespace mlg
