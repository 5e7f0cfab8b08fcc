// Host-side helpers shared by the ABI sources: error reporting, owned and
// borrowed device buffers, host copies of small inputs.
#pragma once

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "common.hpp"

namespace bioem {
namespace host {

inline bioem_status fail(bioem_ctx* ctx, bioem_status st, const char* fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return st;
}

#define HIP_OR_FAIL(ctx, expr)                                                              \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return fail(ctx, e_ == hipErrorOutOfMemory ? BIOEM_ENOMEM : BIOEM_EDEVICE, "%s: %s", \
                  #expr, hipGetErrorString(e_));                                            \
  } while (0)

// Pieces of a fixed device region handed out in order (256-byte aligned,
// never freed): the scratch of the allocation-free posterior.
struct Carve {
  char* base = nullptr;
  size_t cap = 0, off = 0;
  static size_t up(size_t v) { return (v + 255) & ~size_t(255); }
  void* take(size_t bytes) {
    const size_t o = up(off);
    if (!base || o > cap || bytes > cap - o) return nullptr;
    off = o + bytes;
    return base + o;
  }
  size_t left() const { const size_t o = up(off); return o < cap ? cap - o : 0; }
};

// Device buffer that frees itself, or a piece of a Carve it does not own.
struct DevMem {
  void* p = nullptr;
  bool owned = true;
  DevMem() = default;
  DevMem(const DevMem&) = delete;
  DevMem& operator=(const DevMem&) = delete;
  ~DevMem() { if (p && owned) (void)hipFree(p); }
  hipError_t alloc(size_t bytes) { return hipMalloc(&p, bytes ? bytes : 1); }
  // from the carve when one is given (no allocation), else hipMalloc
  hipError_t get(size_t bytes, Carve* c) {
    if (!c) return alloc(bytes);
    owned = false;
    p = c->take(bytes ? bytes : 1);
    return p ? hipSuccess : hipErrorOutOfMemory;
  }
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// A borrowed input made available on the device: used in place when it is
// device memory, copied (stream-ordered) when it is host memory.
struct DevIn {
  DevMem own;
  const void* d = nullptr;
  hipError_t set(const void* src, size_t bytes, bioem_mem mem, hipStream_t s, Carve* c = nullptr) {
    if (!src) { d = nullptr; return hipSuccess; }
    if (mem == BIOEM_MEM_DEVICE) { d = src; return hipSuccess; }
    hipError_t e = own.get(bytes, c);
    if (e != hipSuccess) return e;
    d = own.p;
    return hipMemcpyAsync(own.p, src, bytes, hipMemcpyHostToDevice, s);
  }
  template <class T> const T* as() const { return static_cast<const T*>(d); }
};

// Small inputs are validated on the host; device ones are copied back first.
template <class T>
inline hipError_t to_host(const T* src, size_t count, bioem_mem mem, hipStream_t s, std::vector<T>& out) {
  out.resize(count);
  if (count == 0) return hipSuccess;
  if (mem == BIOEM_MEM_HOST) {
    std::memcpy(out.data(), src, count * sizeof(T));
    return hipSuccess;
  }
  hipError_t e = hipMemcpyAsync(out.data(), src, count * sizeof(T), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

inline bool finite_all(const double* v, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

inline bool valid_mem(int m) { return m == BIOEM_MEM_HOST || m == BIOEM_MEM_DEVICE; }

}  // namespace host
}  // namespace bioem
