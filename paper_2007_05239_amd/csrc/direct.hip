// Direct tiled summation of the Gaussian weight matrix (Sec. 2 case (i):
// W assembled on the fly, O(d n^2) work), zero diagonal:
//     F_i = sum_{j != i} exp(-||x_i - x_j||^2 / sigma^2) Z_j     (b vectors)
// Rows are split over workgroups (256 rows each) and the column range over a
// second grid dimension; the column partials are summed in a fixed order, so
// results are reproducible bit for bit.
#include "internal.h"

namespace mlg {

constexpr int kDirectMaxD = 16;
constexpr int kJT = 64;

template <class T>
__device__ inline T kexp(T a);
template <>
__device__ inline float kexp<float>(float a) { return __expf(a); }
template <>
__device__ inline double kexp<double>(double a) { return exp(a); }

template <class T, int BS>
__global__ __launch_bounds__(256) void k_direct(int64_t n, int d, const T *__restrict__ x, T inv_s2,
                                                const T *__restrict__ Zs, T *__restrict__ out,
                                                int64_t jchunk) {
    __shared__ T sx[kDirectMaxD][kJT];
    __shared__ T sz[kJT][BS];
    const int tid = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * 256 + tid;
    const bool valid = i < n;
    T xi[kDirectMaxD];
#pragma unroll
    for (int k = 0; k < kDirectMaxD; ++k) xi[k] = (k < d && valid) ? x[(int64_t)k * n + i] : T(0);
    T acc[BS];
#pragma unroll
    for (int v = 0; v < BS; ++v) acc[v] = T(0);
    const int64_t j0 = (int64_t)blockIdx.y * jchunk;
    const int64_t j1 = (j0 + jchunk < n) ? j0 + jchunk : n;
    for (int64_t jb = j0; jb < j1; jb += kJT) {
        const int cnt = (int)((j1 - jb) < kJT ? (j1 - jb) : kJT);
        __syncthreads();
        for (int e = tid; e < d * kJT; e += 256) {
            int k = e / kJT, jj = e - k * kJT;
            sx[k][jj] = jj < cnt ? x[(int64_t)k * n + jb + jj] : T(0);
        }
        for (int e = tid; e < kJT * BS; e += 256) {
            int jj = e / BS, v = e - jj * BS;
            sz[jj][v] = jj < cnt ? Zs[(jb + jj) * BS + v] : T(0);
        }
        __syncthreads();
        for (int jj = 0; jj < cnt; ++jj) {
            T r2 = T(0);
#pragma unroll
            for (int k = 0; k < kDirectMaxD; ++k) {
                if (k < d) {
                    T dk = xi[k] - sx[k][jj];
                    r2 += dk * dk;
                }
            }
            T e = kexp<T>(-r2 * inv_s2);
            if (jb + jj == i) e = T(0);
#pragma unroll
            for (int v = 0; v < BS; ++v) acc[v] += e * sz[jj][v];
        }
    }
    if (valid) {
        T *o = out + ((int64_t)blockIdx.y * n + i) * BS;
#pragma unroll
        for (int v = 0; v < BS; ++v) o[v] = acc[v];
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

static int direct_splits(int64_t n) {
    const int rb = ceil_div(n, 256);
    int S = ceil_div(1024, rb);
    const int maxS = ceil_div(n, 4 * kJT);
    if (S > maxS) S = maxS;
    return S < 1 ? 1 : S;
}

template <class T>
size_t direct_part_size(int64_t n, int bs) {
    const int S = direct_splits(n);
    return S > 1 ? (size_t)S * n * bs : 0;
}

template <class T, int BS>
static void launch_direct_bs(int64_t n, int d, const T *x, T inv_s2, const T *Zs, T *Fs, T *part,
                             size_t part_cap, hipStream_t s) {
    const int S = direct_splits(n);
    int64_t jchunk = (n + S - 1) / S;
    jchunk = (jchunk + kJT - 1) / kJT * kJT;
    const int Seff = (int)((n + jchunk - 1) / jchunk);
    dim3 grid(ceil_div(n, 256), Seff);
    if (Seff == 1) {
        hipLaunchKernelGGL((k_direct<T, BS>), grid, dim3(256), 0, s, n, d, x, inv_s2, Zs, Fs, jchunk);
        MLG_LAUNCH_CHECK();
        return;
    }
    MLG_REQUIRE(part && part_cap >= (size_t)Seff * n * BS, MLG_ERR_ARG, "direct: workspace too small");
    hipLaunchKernelGGL((k_direct<T, BS>), grid, dim3(256), 0, s, n, d, x, inv_s2, Zs, part, jchunk);
    MLG_LAUNCH_CHECK();
    const int64_t total = n * BS;
    hipLaunchKernelGGL(k_direct_reduce<T>, dim3(ceil_div(total, 256)), dim3(256), 0, s, total, Seff,
                       part, Fs);
    MLG_LAUNCH_CHECK();
}

template <class T>
void launch_direct(int64_t n, int d, const T *x, double inv_s2, int bs, const T *Zs, T *Fs, T *part,
                   size_t part_cap, hipStream_t s) {
    MLG_REQUIRE(d >= 1 && d <= kDirectMaxD, MLG_ERR_RANGE, "direct summation supports d <= 16");
    const T is2 = (T)inv_s2;
    switch (bs) {
        case 1: launch_direct_bs<T, 1>(n, d, x, is2, Zs, Fs, part, part_cap, s); break;
        case 2: launch_direct_bs<T, 2>(n, d, x, is2, Zs, Fs, part, part_cap, s); break;
        case 4: launch_direct_bs<T, 4>(n, d, x, is2, Zs, Fs, part, part_cap, s); break;
        case 8: launch_direct_bs<T, 8>(n, d, x, is2, Zs, Fs, part, part_cap, s); break;
        case 16: launch_direct_bs<T, 16>(n, d, x, is2, Zs, Fs, part, part_cap, s); break;
        case 32: launch_direct_bs<T, 32>(n, d, x, is2, Zs, Fs, part, part_cap, s); break;
        case 64: launch_direct_bs<T, 64>(n, d, x, is2, Zs, Fs, part, part_cap, s); break;
        default: throw Error(MLG_ERR_ARG, "direct: unsupported block stride");
    }
}

template void launch_direct<float>(int64_t, int, const float *, double, int, const float *, float *,
                                   float *, size_t, hipStream_t);
template void launch_direct<double>(int64_t, int, const double *, double, int, const double *,
                                    double *, double *, size_t, hipStream_t);
template size_t direct_part_size<float>(int64_t, int);
template size_t direct_part_size<double>(int64_t, int);

}  // namespace mlg
