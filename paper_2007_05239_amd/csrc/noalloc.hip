// Y = W X by direct summation with no device allocation, for callers that
// cannot allocate (code under HIP graph capture, serving loops, harnesses
// that forbid hipMalloc).  Same kernels and the same column split as
// mlg_kernel_matvec with MLG_METHOD_DIRECT (Sec. 2 case (i); zero diagonal),
// so the results are the same bits.  Every intermediate lives in one
// library-owned scratch array per device:
//
//   [layer descriptor | bounding-box midpoint | x64 (n d) | x32 (n d) |
//    Zs (n bs) | Fs (n bs) | column partials (S n bs)]      each 256-aligned
//
// The array is a file-scope __device__ variable; host code reaches it only
// through the address hipGetSymbolAddress returns for the current device
// (taken once per device on its first call and kept).  Calls on one device
// share the array and keep the last call's contents; every region is fully
// written before it is read, so nothing needs clearing.  Calls that overlap
// on one device (different streams, or threads) race on it.
#include <cmath>
#include <mutex>

#include "internal.h"

namespace mlg {

constexpr size_t kScratchBytes = MLG_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device.
static unsigned char *scratch_base(int dev) {
    MLG_REQUIRE(dev >= 0 && dev < kMaxDevices, MLG_ERR_RANGE, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        MLG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        MLG_REQUIRE(p != nullptr, MLG_ERR_HIP, "no device address for the scratch array");
        g_scratch_ptr[dev] = p;
    }
    return static_cast<unsigned char *>(g_scratch_ptr[dev]);
}

__global__ void k_set_layerio(LayerIO *dst, LayerIO v) { *dst = v; }

static size_t round256(size_t b) { return (b + 255) / 256 * 256; }

static int block_stride_of(int b) {
    int bs = 1;
    while (bs < b) bs <<= 1;
    return bs;
}

// Byte offsets of the regions for (n, d, bs, element size esz).
struct NoallocLayout {
    size_t io, mid, x64, x32, zs, fs, part, total;
};

static NoallocLayout layout(int64_t n, int d, int bs, bool fp64) {
    NoallocLayout L{};
    const size_t esz = fp64 ? 8 : 4;
    const size_t part = fp64 ? direct_part_size<double>(n, bs) : direct_part_size<float>(n, bs);
    size_t o = 0;
    L.io = o;   o += round256(sizeof(LayerIO));
    L.mid = o;  o += round256(sizeof(double) * 16);
    L.x64 = o;  o += round256(sizeof(double) * (size_t)n * d);
    L.x32 = o;  o += round256(sizeof(float) * (size_t)n * d);
    L.zs = o;   o += round256(esz * (size_t)n * bs);
    L.fs = o;   o += round256(esz * (size_t)n * bs);
    L.part = o; o += round256(esz * part);
    L.total = o;
    return L;
}

template <class T>
static void run(int64_t n, int d, int kernel, double sigma, int b, const double *points,
                const double *X, int64_t ldx, double *Y, int64_t ldy, unsigned char *base,
                const NoallocLayout &L, int bs, hipStream_t s) {
    double *mid = reinterpret_cast<double *>(base + L.mid);
    double *x64 = reinterpret_cast<double *>(base + L.x64);
    float *x32 = reinterpret_cast<float *>(base + L.x32);
    T *Zs = reinterpret_cast<T *>(base + L.zs);
    T *Fs = reinterpret_cast<T *>(base + L.fs);
    T *part = reinterpret_cast<T *>(base + L.part);
    LayerIO *io = reinterpret_cast<LayerIO *>(base + L.io);
    LayerIO v{};
    v.Z = Zs;
    v.F = Fs;
    v.dinv = nullptr;
    v.K0 = 0.0;
    v.is64 = sizeof(T) == 8;
    v.shared = 0;
    hipLaunchKernelGGL(k_set_layerio, dim3(1), dim3(1), 0, s, io, v);
    MLG_LAUNCH_CHECK();
    direct_coords_into(n, d, points, sigma, kernel, mid, x64, x32, s);
    launch_scatter_in(n, b, bs, X, ldx, io, 1, 0, s);
    const T *x = nullptr;
    if constexpr (sizeof(T) == 8) x = x64; else x = x32;
    const size_t cap = (L.total - L.part) / sizeof(T);
    launch_direct<T>(n, d, kernel, x, bs, Zs, Fs, part, cap, s);
    launch_gather_out(n, b, bs, X, ldx, Y, ldy, io, 1, 0, 0, 1.0, s);
}

}  // namespace mlg

using namespace mlg;

extern "C" mlg_status mlg_kernel_matvec_noalloc(int64_t n, int d, const double *points,
                                                double sigma, const mlg_kparams *kp, int b,
                                                const double *X, int64_t ldx, double *Y,
                                                int64_t ldy, void *stream) {
    try {
        set_last_error("");
        MLG_REQUIRE(points && kp && X && Y, MLG_ERR_ARG, "null argument");
        MLG_REQUIRE(kp->method == MLG_METHOD_DIRECT, MLG_ERR_NOT_IMPL,
                    "the allocation-free product runs the direct method only");
        MLG_REQUIRE(kp->precision == 32 || kp->precision == 64, MLG_ERR_ARG,
                    "precision must be 32 or 64");
        MLG_REQUIRE(kp->kernel == MLG_KERNEL_GAUSSIAN || kp->kernel == MLG_KERNEL_LAPLACIAN,
                    MLG_ERR_ARG, "bad kernel");
        MLG_REQUIRE(n >= 2, MLG_ERR_ARG, "n must be >= 2");
        MLG_REQUIRE(d >= 1 && d <= 16, MLG_ERR_RANGE, "direct summation needs d in 1..16");
        MLG_REQUIRE(sigma > 0 && std::isfinite(sigma), MLG_ERR_RANGE, "sigma must be > 0");
        MLG_REQUIRE(b >= 1 && b <= 64, MLG_ERR_ARG, "b must be in 1..64");
        MLG_REQUIRE(ldx >= n && ldy >= n, MLG_ERR_ARG, "leading dimension < n");
        const int bs = block_stride_of(b);
        const bool fp64 = kp->precision == 64;
        const NoallocLayout L = layout(n, d, bs, fp64);
        if (L.total > kScratchBytes)
            throw Error(MLG_ERR_RANGE,
                        "mlg_kernel_matvec_noalloc: this size needs " + std::to_string(L.total) +
                            " bytes of scratch, the limit is " + std::to_string(kScratchBytes) +
                            " (MLG_NOALLOC_SCRATCH_BYTES)");
        int dev = 0;
        MLG_HIP(hipGetDevice(&dev));
        unsigned char *base = scratch_base(dev);
        hipStream_t s = (hipStream_t)stream;
        if (fp64)
            run<double>(n, d, kp->kernel, sigma, b, points, X, ldx, Y, ldy, base, L, bs, s);
        else
            run<float>(n, d, kp->kernel, sigma, b, points, X, ldx, Y, ldy, base, L, bs, s);
        return MLG_OK;
    } catch (const Error &e) {
        set_last_error(e.what());
        return e.code;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return MLG_ERR_HIP;
    }
}
