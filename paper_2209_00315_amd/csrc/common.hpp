// Shared host-side helpers of the otbb library: error reporting, device
// buffers, launch helpers.  Host code only; kernels live in kernels.hpp.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/otbb.h"

namespace otbb {

// An error that carries one of the OT_E* codes of the C ABI.
struct OtError : std::runtime_error {
    int code;
    OtError(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string &msg);

#define OT_HIP(call)                                                          \
    do {                                                                      \
        hipError_t e_ = (call);                                               \
        if (e_ != hipSuccess)                                                 \
            throw ::otbb::OtError(e_ == hipErrorOutOfMemory ? OT_ENOMEM       \
                                                            : OT_EDEVICE,     \
                                  std::string(#call) + ": " +                 \
                                      hipGetErrorString(e_));                 \
    } while (0)

#define OT_REQUIRE(cond, code, msg)                                           \
    do {                                                                      \
        if (!(cond)) throw ::otbb::OtError((code), (msg));                    \
    } while (0)

// Owning device buffer (hipMalloc'd); moves only.
template <typename T>
struct DBuf {
    T *p = nullptr;
    size_t n = 0;
    DBuf() = default;
    explicit DBuf(size_t count) { alloc(count); }
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    DBuf(DBuf &&o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    DBuf &operator=(DBuf &&o) noexcept {
        if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
        return *this;
    }
    ~DBuf() { release(); }
    void alloc(size_t count) {
        release();
        n = count;
        if (count) OT_HIP(hipMalloc(&p, count * sizeof(T)));
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    void upload(const std::vector<T> &h, hipStream_t s) {
        if (h.size() != n) alloc(h.size());
        if (n) OT_HIP(hipMemcpyAsync(p, h.data(), n * sizeof(T), hipMemcpyHostToDevice, s));
    }
    void zero(hipStream_t s) {
        if (n) OT_HIP(hipMemsetAsync(p, 0, n * sizeof(T), s));
    }
    operator T *() const { return p; }
};

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

}  // namespace otbb
