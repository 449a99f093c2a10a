// Shared host/device utilities of the sunbloch library: status handling,
// device buffers, complex arithmetic, scans and reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/sunbloch.h"

namespace sun {

// ---------------------------------------------------------------------------
// Errors: internal code throws sun::Error; every C entry point catches it and
// turns it into a status code plus a thread-local message.
// ---------------------------------------------------------------------------
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void set_error(const std::string& msg);
void clear_error();

#define SUN_THROW(code, msg)                                   \
  do {                                                         \
    throw ::sun::Error((code), std::string(__func__) + ": " + (msg)); \
  } while (0)

#define SUN_REQUIRE(cond, code, msg) \
  do {                               \
    if (!(cond)) SUN_THROW((code), (msg)); \
  } while (0)

#define HIP_OK(expr)                                                        \
  do {                                                                      \
    hipError_t _e = (expr);                                                 \
    if (_e != hipSuccess) {                                                 \
      (void)hipGetLastError();                                              \
      throw ::sun::Error(_e == hipErrorOutOfMemory ? SUN_ENOMEM : SUN_EDEVICE, \
                         std::string(#expr) + ": " + hipGetErrorString(_e)); \
    }                                                                       \
  } while (0)

// Check the launch status of the last kernel.
#define HIP_LAUNCH_OK() HIP_OK(hipGetLastError())

// Stream of the entry point being executed on this thread (reset by
// guarded, recorded by as_stream); handed to a caller-installed allocator.
extern thread_local void* t_call_stream;

template <class F>
int guarded(F&& f) {
  try {
    clear_error();
    t_call_stream = nullptr;
    f();
    return SUN_OK;
  } catch (const Error& e) {
    set_error(e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return SUN_ENOMEM;
  } catch (const std::exception& e) {
    set_error(e.what());
    return SUN_EDEVICE;
  }
}

inline hipStream_t as_stream(void* s) {
  t_call_stream = s;
  return reinterpret_cast<hipStream_t>(s);
}

// Device allocations: hipMalloc/hipFree, or the caller's pair installed with
// sun_set_allocator.  Each buffer remembers the pair that allocated it.
struct AllocPair {
  sun_alloc_fn alloc = nullptr;
  sun_release_fn release = nullptr;
  void* ctx = nullptr;
};
void* device_alloc(size_t bytes, AllocPair& used);          // throws SUN_ENOMEM
void device_release(void* p, const AllocPair& used) noexcept;

// ---------------------------------------------------------------------------
// Owning device buffer.
// ---------------------------------------------------------------------------
template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  AllocPair a;
  DevBuf() = default;
  explicit DevBuf(size_t count) { alloc(count); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n), a(o.a) { o.p = nullptr; o.n = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; a = o.a; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t count) {
    release();
    if (count) p = static_cast<T*>(device_alloc(count * sizeof(T), a));
    n = count;
  }
  void release() {
    if (p) device_release(p, a);
    p = nullptr;
    n = 0;
  }
  T* get() const { return p; }
  size_t bytes() const { return n * sizeof(T); }
};

// ---------------------------------------------------------------------------
// Complex numbers (device and host).
// ---------------------------------------------------------------------------
struct cplx {
  double re, im;
};
__host__ __device__ inline cplx cx(double r, double i = 0.0) { return cplx{r, i}; }
__host__ __device__ inline cplx operator+(cplx a, cplx b) { return cplx{a.re + b.re, a.im + b.im}; }
__host__ __device__ inline cplx operator-(cplx a, cplx b) { return cplx{a.re - b.re, a.im - b.im}; }
__host__ __device__ inline cplx operator*(cplx a, cplx b) {
  return cplx{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__host__ __device__ inline cplx operator*(double s, cplx a) { return cplx{s * a.re, s * a.im}; }
__host__ __device__ inline cplx conj(cplx a) { return cplx{a.re, -a.im}; }
__host__ __device__ inline bool is_zero(cplx a) { return a.re == 0.0 && a.im == 0.0; }
__host__ __device__ inline bool is_zero(double a) { return a == 0.0; }
__host__ __device__ inline double absval(double a) { return a < 0 ? -a : a; }
__host__ __device__ inline double absval(cplx a) {
  double r = absval(a.re), i = absval(a.im);
  return r > i ? r : i;  // max-norm: enough for thresholds
}

// ---------------------------------------------------------------------------
// Device-wide exclusive scan of int64 counts (three kernels, deterministic).
// out[i] = sum_{j<i} in[i]; returns the total (synchronises the stream).
// ---------------------------------------------------------------------------
int64_t exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, hipStream_t s);

// max over a double array (non-negative values), result on host.
double device_max(const double* in, int64_t n, hipStream_t s);

// Max of a non-negative int64 array, result on host.
int64_t device_max_i64(const int64_t* in, int64_t n, hipStream_t s);

// Sum of an int64 array, result on host.
int64_t device_sum_i64(const int64_t* in, int64_t n, hipStream_t s);

// bad[0] = 1 if some x[i], i < n, is NaN or infinite (queued on s); and
// a[0] = v (a one-thread kernel, used to reset such flags without memsets).
void flag_nonfinite(const double* x, int64_t n, int* bad, hipStream_t s);
void set_int(int* a, int v, hipStream_t s);

// Per-workgroup LDS limit of the current device, in bytes.
size_t lds_limit();

inline unsigned grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 1 << 30) g = 1 << 30;
  return (unsigned)g;
}

}  // namespace sun
