// Internal helpers shared by the translation units of libmlg.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/mlg.h"

namespace mlg {

// An error carrying a status code; converted to a return code at the ABI.
struct Error : std::runtime_error {
    mlg_status code;
    Error(mlg_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string &msg);

#define MLG_HIP(call)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess) {                                                          \
            throw ::mlg::Error(e_ == hipErrorOutOfMemory ? MLG_ERR_NOMEM : MLG_ERR_HIP,  \
                               std::string(#call) + ": " + hipGetErrorString(e_) +       \
                                   " at " + __FILE__ + ":" + std::to_string(__LINE__));  \
        }                                                                                \
    } while (0)

#define MLG_REQUIRE(cond, code, msg)                                                     \
    do {                                                                                 \
        if (!(cond)) throw ::mlg::Error(code, msg);                                      \
    } while (0)

#define MLG_LAUNCH_CHECK() MLG_HIP(hipGetLastError())

// Owning device buffer.
template <class T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    explicit DevBuf(size_t count) { alloc(count); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
        return *this;
    }
    ~DevBuf() { release(); }
    void alloc(size_t count) {
        release();
        if (count == 0) return;
        MLG_HIP(hipMalloc((void **)&p, count * sizeof(T)));
        n = count;
    }
    // grow only
    void ensure(size_t count) {
        if (count > n) alloc(count);
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    T *get() const { return p; }
};

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

inline bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// Copies `count` elements into a fresh device buffer from host or device.
template <class T>
void upload(DevBuf<T> &dst, const T *src, size_t count, bool src_on_device, hipStream_t s) {
    dst.alloc(count);
    if (count == 0) return;
    MLG_HIP(hipMemcpyAsync(dst.p, src, count * sizeof(T),
                           src_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
}

// Copies a column-major rows x cols block between leading dimensions dld and
// sld (elements) with contiguous 1-D copies: one copy when both blocks are
// dense, else one per column.
template <class T>
void copy_cols(T *dst, int64_t dld, const T *src, int64_t sld, int64_t rows, int64_t cols,
               hipMemcpyKind kind, hipStream_t s) {
    if (rows == 0 || cols == 0) return;
    if (dld == rows && sld == rows) {
        MLG_HIP(hipMemcpyAsync(dst, src, sizeof(T) * rows * cols, kind, s));
        return;
    }
    for (int64_t c = 0; c < cols; ++c)
        MLG_HIP(hipMemcpyAsync(dst + c * dld, src + c * sld, sizeof(T) * rows, kind, s));
}

}  // namespace mlg
