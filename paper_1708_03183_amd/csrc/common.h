// Internal helpers of libdgtile: status propagation, HIP checks, device buffers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/dgtile.h"

namespace dgt {

// A failing call sets the thread-local message and returns its status.
dgt_status fail(dgt_status st, const std::string &msg);

struct Error {
    dgt_status st;
    std::string msg;
};

#define DGT_HIP(call)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            throw ::dgt::Error{DGT_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)

#define DGT_REQUIRE(cond, st, msg)                                  \
    do {                                                            \
        if (!(cond)) throw ::dgt::Error{(st), std::string(msg)};    \
    } while (0)

// Wraps a C-ABI body: converts exceptions into statuses.
template <class F>
dgt_status guard(F &&f) {
    try {
        f();
        return DGT_OK;
    } catch (const Error &e) {
        return fail(e.st, e.msg);
    } catch (const std::bad_alloc &) {
        return fail(DGT_ENOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(DGT_EINVAL, e.what());
    }
}

// Owning device buffer (hipMalloc'd), moved, never copied.
template <class T>
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
        if (count) {
            hipError_t e = hipMalloc(&p, sizeof(T) * count);
            if (e != hipSuccess) { p = nullptr; n = 0; throw Error{DGT_ENOMEM, "hipMalloc failed"}; }
        }
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    void upload(const T *h, size_t count, hipStream_t s) {
        if (count > n) alloc(count);
        if (count) DGT_HIP(hipMemcpyAsync(p, h, sizeof(T) * count, hipMemcpyHostToDevice, s));
    }
    void upload(const std::vector<T> &h, hipStream_t s) { upload(h.data(), h.size(), s); }
    std::vector<T> download(hipStream_t s, size_t count = SIZE_MAX) const {
        if (count == SIZE_MAX) count = n;
        std::vector<T> h(count);
        if (count) DGT_HIP(hipMemcpyAsync(h.data(), p, sizeof(T) * count, hipMemcpyDeviceToHost, s));
        DGT_HIP(hipStreamSynchronize(s));
        return h;
    }
};

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs < 1 ? 1 : (n + bs - 1) / bs); }

}  // namespace dgt
