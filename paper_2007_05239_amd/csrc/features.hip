// Feature grouping (Sec. 7): a d >= 4 feature space is split into groups of
// dimension <= 3, one graph layer per group, so that every layer can use the
// NFFT fast summation.  This file gathers a group's feature columns into a
// layer's point array on the device, and computes the per-layer kernel width
// as the median of the pairwise distances of a node sample.
#include <algorithm>
#include <cmath>
#include <cstring>

#include <rocprim/rocprim.hpp>

#include "internal.h"

namespace mlg {

namespace {

// out (n x d row-major) = columns cols[0..d) of the n x D row-major features.
__global__ void k_gather_cols(int64_t n, int D, const double *__restrict__ F, int d,
                              const int *__restrict__ cols, double *__restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * d) return;
    const int64_t i = e / d;
    const int k = (int)(e - i * d);
    out[e] = F[i * D + cols[k]];
}

// Squared pairwise distances of the sample rows (a < b, row-major order of
// pairs): r2 = sum over the coordinates in order of the rounded squares (no
// fused multiply-add); stored as the bit pattern of the non-negative double,
// whose unsigned order is the numeric one.  The square root is monotonic, so
// the order statistics of the distances are the square roots of those of r2;
// the host takes the square root of the middle value(s) only.
__global__ void k_pair_dist(int s, int D, const double *__restrict__ F, int d,
                            const int *__restrict__ cols, const int64_t *__restrict__ sample,
                            uint64_t *__restrict__ out) {
#pragma clang fp contract(off)
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t npair = (int64_t)s * (s - 1) / 2;
    if (e >= npair) return;
    // pair index e -> (a, b), a < b, pairs ordered (0,1), (0,2), ..., (1,2), ...
    int a = (int)((2.0 * s - 1.0 - sqrt((2.0 * s - 1.0) * (2.0 * s - 1.0) - 8.0 * (double)e)) / 2.0);
    if (a < 0) a = 0;
    auto start = [s](int64_t aa) { return aa * (2 * (int64_t)s - aa - 1) / 2; };
    while (a > 0 && start(a) > e) --a;
    while (a + 1 < s && start(a + 1) <= e) ++a;
    const int b = (int)(e - start(a)) + a + 1;
    const double *xa = F + sample[a] * D;
    const double *xb = F + sample[b] * D;
    double r2 = 0.0;
    for (int k = 0; k < d; ++k) {
        const double dk = xa[cols[k]] - xb[cols[k]];
        r2 = r2 + dk * dk;
    }
    out[e] = (uint64_t)__double_as_longlong(r2);
}

struct OwnedStream {
    hipStream_t s = nullptr;
    OwnedStream() { MLG_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking)); }
    ~OwnedStream() { if (s) (void)hipStreamDestroy(s); }
};

}  // namespace

void gather_feature_groups(int64_t n, int D, const double *features, bool dev, int T,
                           const int *group_dim, const int *group_cols,
                           std::vector<DevBuf<double>> &pts) {
    MLG_REQUIRE(n >= 1 && D >= 1, MLG_ERR_ARG, "need n >= 1 and D >= 1");
    MLG_REQUIRE(features && group_dim && group_cols, MLG_ERR_ARG, "null argument");
    MLG_REQUIRE(T >= 1 && T <= 1024, MLG_ERR_ARG, "T must be in 1..1024");
    int total = 0;
    for (int t = 0; t < T; ++t) {
        MLG_REQUIRE(group_dim[t] >= 1 && group_dim[t] <= 16, MLG_ERR_RANGE,
                    "group dimensions must be in 1..16");
        total += group_dim[t];
    }
    for (int e = 0; e < total; ++e)
        MLG_REQUIRE(group_cols[e] >= 0 && group_cols[e] < D, MLG_ERR_ARG,
                    "feature index out of range");
    OwnedStream os;
    DevBuf<double> hostcopy;
    const double *F = features;
    if (!dev) {
        upload(hostcopy, features, (size_t)n * D, false, os.s);
        F = hostcopy.p;
    }
    DevBuf<int> cols;
    upload(cols, group_cols, (size_t)total, false, os.s);
    pts.clear();
    pts.resize(T);
    int off = 0;
    for (int t = 0; t < T; ++t) {
        const int d = group_dim[t];
        pts[t].alloc((size_t)n * d);
        hipLaunchKernelGGL(k_gather_cols, dim3(ceil_div(n * d, 256)), dim3(256), 0, os.s, n, D, F, d,
                           cols.p + off, pts[t].p);
        MLG_LAUNCH_CHECK();
        off += d;
    }
    MLG_HIP(hipStreamSynchronize(os.s));
}

double median_pair_distance(int64_t n, int D, const double *features, bool dev, int d,
                            const int *cols_host, int s, const int64_t *sample_host,
                            hipStream_t stream) {
    MLG_REQUIRE(n >= 2 && D >= 1 && d >= 1 && d <= D, MLG_ERR_ARG, "need n >= 2, 1 <= d <= D");
    MLG_REQUIRE(s >= 2 && s <= 8192 && s <= n, MLG_ERR_ARG, "sample size must be in 2..min(n, 8192)");
    MLG_REQUIRE(features && sample_host, MLG_ERR_ARG, "null argument");
    std::vector<int> cols(d);
    for (int k = 0; k < d; ++k) {
        cols[k] = cols_host ? cols_host[k] : k;
        MLG_REQUIRE(cols[k] >= 0 && cols[k] < D, MLG_ERR_ARG, "feature index out of range");
    }
    for (int a = 0; a < s; ++a)
        MLG_REQUIRE(sample_host[a] >= 0 && sample_host[a] < n, MLG_ERR_ARG,
                    "sample index out of range");
    hipStream_t st = stream;
    DevBuf<double> hostcopy;
    const double *F = features;
    if (!dev) {
        upload(hostcopy, features, (size_t)n * D, false, st);
        F = hostcopy.p;
    }
    DevBuf<int> dcols;
    DevBuf<int64_t> dsample;
    upload(dcols, cols.data(), (size_t)d, false, st);
    upload(dsample, sample_host, (size_t)s, false, st);
    const int64_t npair = (int64_t)s * (s - 1) / 2;
    DevBuf<uint64_t> keys(npair), sorted(npair);
    hipLaunchKernelGGL(k_pair_dist, dim3(ceil_div(npair, 256)), dim3(256), 0, st, s, D, F, d, dcols.p,
                       dsample.p, keys.p);
    MLG_LAUNCH_CHECK();
    size_t tbytes = 0;
    MLG_HIP(rocprim::radix_sort_keys(nullptr, tbytes, keys.p, sorted.p, (unsigned)npair, 0, 64, st));
    DevBuf<char> tmp(tbytes);
    MLG_HIP(rocprim::radix_sort_keys(tmp.p, tbytes, keys.p, sorted.p, (unsigned)npair, 0, 64, st));
    uint64_t mid[2] = {0, 0};
    const int64_t h = npair / 2;
    if (npair % 2 == 1) {
        MLG_HIP(hipMemcpyAsync(&mid[0], sorted.p + h, 8, hipMemcpyDeviceToHost, st));
    } else {
        MLG_HIP(hipMemcpyAsync(&mid[0], sorted.p + h - 1, 16, hipMemcpyDeviceToHost, st));
    }
    MLG_HIP(hipStreamSynchronize(st));
    double v0, v1;
    std::memcpy(&v0, &mid[0], 8);
    std::memcpy(&v1, &mid[1], 8);
    v0 = std::sqrt(v0);
    v1 = std::sqrt(v1);
    return npair % 2 == 1 ? v0 : 0.5 * (v0 + v1);
}

}  // namespace mlg
