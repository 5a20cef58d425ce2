// Shared host/device helpers of the qtp library (HIP, gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

namespace qtp {

// Internal error type; caught at the C-ABI boundary and turned into a status.
struct Error : std::runtime_error {
  int status;
  Error(int s, const std::string& m) : std::runtime_error(m), status(s) {}
};

#define QTP_HIP(call)                                                        \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess)                                                    \
      throw ::qtp::Error(-3, std::string(#call) + ": " + hipGetErrorString(e_) \
                                 + " (" + __FILE__ + ":" + std::to_string(__LINE__) + ")"); \
  } while (0)

#define QTP_CHECK_LAUNCH() QTP_HIP(hipGetLastError())

#define QTP_REQUIRE(cond, status, msg)                                       \
  do {                                                                       \
    if (!(cond)) throw ::qtp::Error((status), (msg));                       \
  } while (0)

inline int div_up(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// Device buffer owned by the library (stream-ordered allocation).
class DevBuf {
 public:
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : ptr_(o.ptr_), bytes_(o.bytes_) {
    o.ptr_ = nullptr;
    o.bytes_ = 0;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      ptr_ = o.ptr_;
      bytes_ = o.bytes_;
      o.ptr_ = nullptr;
      o.bytes_ = 0;
    }
    return *this;
  }
  void swap(DevBuf& o) noexcept {
    std::swap(ptr_, o.ptr_);
    std::swap(bytes_, o.bytes_);
  }
  ~DevBuf() { release(); }
  void* get() const { return ptr_; }
  size_t bytes() const { return bytes_; }
  template <class T> T* as() const { return static_cast<T*>(ptr_); }
  // Grow to at least `bytes` (contents are not preserved).
  void ensure(size_t bytes) {
    if (bytes <= bytes_) return;
    release();
    size_t b = bytes < 256 ? 256 : bytes;
    QTP_HIP(hipMalloc(&ptr_, b));
    bytes_ = b;
  }
  void release() {
    if (ptr_) (void)hipFree(ptr_);
    ptr_ = nullptr;
    bytes_ = 0;
  }

 private:
  void* ptr_ = nullptr;
  size_t bytes_ = 0;
};

// Pinned, device-visible host memory (coherent), allocated once.
class HostBuf {
 public:
  HostBuf() = default;
  HostBuf(const HostBuf&) = delete;
  HostBuf& operator=(const HostBuf&) = delete;
  ~HostBuf() {
    if (ptr_) (void)hipHostFree(ptr_);
  }
  bool empty() const { return ptr_ == nullptr; }
  void alloc(size_t bytes) {
    if (ptr_) return;
    QTP_HIP(hipHostMalloc(&ptr_, bytes, hipHostMallocDefault));
    QTP_HIP(hipHostGetDevicePointer(&dev_, ptr_, 0));
  }
  template <class T> T* host() const { return static_cast<T*>(ptr_); }
  template <class T> T* dev() const { return static_cast<T*>(dev_); }

 private:
  void* ptr_ = nullptr;
  void* dev_ = nullptr;
};

}  // namespace qtp
