// Internal helpers shared by the library's translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "tbkpm.h"

namespace tbk {

// Thread-local error text behind tbk_last_error().
void set_error(const char *fmt, ...);
void clear_error();

// Returns the status and records the message.
tbk_status fail(tbk_status st, const char *fmt, ...);

#define TBK_HIP(call)                                                                 \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            return ::tbk::fail(TBK_ERR_DEVICE, "%s failed: %s (%s:%d)", #call,        \
                               hipGetErrorString(e_), __FILE__, __LINE__);            \
    } while (0)

#define TBK_CHECK(cond, st, ...)                                                      \
    do {                                                                              \
        if (!(cond)) return ::tbk::fail((st), __VA_ARGS__);                           \
    } while (0)

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Stream-ordered temporary device buffer, freed on scope exit.
class DevBuf {
  public:
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    hipError_t alloc(size_t bytes, hipStream_t s) {
        release();
        stream_ = s;
        bytes_ = bytes ? bytes : 256;
        return hipMallocAsync(&p_, bytes_, s);
    }
    void release() {
        if (p_) (void)hipFreeAsync(p_, stream_);
        p_ = nullptr;
    }
    template <class T> T *as() const { return static_cast<T *>(p_); }
    size_t bytes() const { return bytes_; }

  private:
    void *p_ = nullptr;
    size_t bytes_ = 0;
    hipStream_t stream_ = nullptr;
};

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Number of XCDs of an MI355X; workgroups are dispatched round-robin over them.
constexpr int kNumXcd = 8;

}  // namespace tbk
