// Error state, scans and reductions used by the assembly pipeline.
#include <mutex>

#include "common.hpp"

namespace sun {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }

thread_local void* t_call_stream = nullptr;

// ---------------------------------------------------------------------------
// Device allocations (hipMalloc/hipFree or the caller's pair).
// ---------------------------------------------------------------------------
static std::mutex g_alloc_mu;
static AllocPair g_alloc;

void* device_alloc(size_t bytes, AllocPair& used) {
  {
    std::lock_guard<std::mutex> lock(g_alloc_mu);
    used = g_alloc;
  }
  void* p = nullptr;
  if (!used.alloc) {
    HIP_OK(hipMalloc(&p, bytes));
    return p;
  }
  p = used.alloc(bytes, t_call_stream, used.ctx);
  SUN_REQUIRE(p != nullptr, SUN_ENOMEM, "the caller's allocator returned NULL for " + std::to_string(bytes) + " bytes");
  if (reinterpret_cast<uintptr_t>(p) & 255) {
    used.release(p, used.ctx);
    SUN_THROW(SUN_EINVAL, "the caller's allocator returned memory that is not 256-byte aligned");
  }
  return p;
}

void device_release(void* p, const AllocPair& used) noexcept {
  if (!used.release) {
    (void)hipFree(p);
    return;
  }
  // as hipFree does: nothing queued may still use the memory once the
  // caller's allocator may hand it out again
  (void)hipDeviceSynchronize();
  used.release(p, used.ctx);
}

// ---------------------------------------------------------------------------
// Exclusive scan of int64 (block-local scan, recursive scan of block sums,
// then a uniform add).  Fixed summation order: deterministic.
// ---------------------------------------------------------------------------
constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_block(const int64_t* __restrict__ in,
                                                           int64_t* __restrict__ out,
                                                           int64_t* __restrict__ bsum, int64_t n) {
  __shared__ int64_t sh[SCAN_BLOCK];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  int64_t loc[SCAN_ITEMS];
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    int64_t idx = base + i;
    int64_t v = idx < n ? in[idx] : 0;
    loc[i] = s;
    s += v;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  // Hillis-Steele inclusive scan over the per-thread sums
  for (int o = 1; o < SCAN_BLOCK; o <<= 1) {
    int64_t t = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0;
    __syncthreads();
    sh[threadIdx.x] += t;
    __syncthreads();
  }
  int64_t prefix = threadIdx.x ? sh[threadIdx.x - 1] : 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    int64_t idx = base + i;
    if (idx < n) out[idx] = loc[i] + prefix;
  }
  if (threadIdx.x == SCAN_BLOCK - 1) bsum[blockIdx.x] = sh[SCAN_BLOCK - 1];
}

__global__ void k_scan_add(int64_t* __restrict__ out, const int64_t* __restrict__ boff, int64_t n) {
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  const int64_t add = boff[blockIdx.x];
  for (int i = threadIdx.x; i < SCAN_TILE; i += blockDim.x) {
    int64_t idx = base + i;
    if (idx < n) out[idx] += add;
  }
}

static void scan_rec(const int64_t* in, int64_t* out, int64_t n, hipStream_t s) {
  const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  DevBuf<int64_t> bsum(nb), boff(nb);
  hipLaunchKernelGGL(k_scan_block, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, in, out, bsum.get(), n);
  HIP_LAUNCH_OK();
  if (nb > 1) {
    scan_rec(bsum.get(), boff.get(), nb, s);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, out, boff.get(), n);
    HIP_LAUNCH_OK();
  }
  // the temporaries are freed when this returns: make sure the queued kernels
  // that read them have finished
  HIP_OK(hipStreamSynchronize(s));
}

int64_t exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, hipStream_t s) {
  if (n <= 0) return 0;
  scan_rec(in, out, n, s);
  int64_t last_in = 0, last_out = 0;
  HIP_OK(hipMemcpyAsync(&last_in, in + n - 1, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(&last_out, out + n - 1, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  return last_in + last_out;
}

// ---------------------------------------------------------------------------
// Reductions
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_max_partial(const double* __restrict__ in, int64_t n,
                                                     double* __restrict__ part) {
  __shared__ double sh[256];
  double m = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    m = fmax(m, in[i]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < (unsigned)o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// |x| <= DBL_MAX is false exactly for NaN and infinities; threads that find
// one all store the same value.
__global__ void k_flag_nonfinite(int64_t n, const double* __restrict__ x, int* __restrict__ bad) {
  bool b = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b |= !(fabs(x[i]) <= 1.7976931348623157e308);
  if (b) bad[0] = 1;
}

__global__ void k_set_int(int* __restrict__ a, int v) { a[0] = v; }

void flag_nonfinite(const double* x, int64_t n, int* bad, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_flag_nonfinite, dim3(std::min<unsigned>(grid_for(n, 256), 1024)), dim3(256), 0, s, n, x,
                     bad);
  HIP_LAUNCH_OK();
}

void set_int(int* a, int v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, a, v);
  HIP_LAUNCH_OK();
}

double device_max(const double* in, int64_t n, hipStream_t s) {
  if (n <= 0) return 0.0;
  const int nb = 512;
  DevBuf<double> part(nb), fin(1);
  hipLaunchKernelGGL(k_max_partial, dim3(nb), dim3(256), 0, s, in, n, part.get());
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(k_max_partial, dim3(1), dim3(256), 0, s, part.get(), (int64_t)nb, fin.get());
  HIP_LAUNCH_OK();
  double r = 0.0;
  HIP_OK(hipMemcpyAsync(&r, fin.get(), sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  return r;
}

__global__ __launch_bounds__(256) void k_sum_partial(const int64_t* __restrict__ in, int64_t n,
                                                     int64_t* __restrict__ part) {
  __shared__ int64_t sh[256];
  int64_t m = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    m += in[i];
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < (unsigned)o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_maxi_partial(const int64_t* __restrict__ in, int64_t n,
                                                      int64_t* __restrict__ part) {
  __shared__ int64_t sh[256];
  int64_t m = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    m = in[i] > m ? in[i] : m;
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < (unsigned)o && sh[threadIdx.x + o] > sh[threadIdx.x]) sh[threadIdx.x] = sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

int64_t device_max_i64(const int64_t* in, int64_t n, hipStream_t s) {
  if (n <= 0) return 0;
  const int nb = 512;
  DevBuf<int64_t> part(nb), fin(1);
  hipLaunchKernelGGL(k_maxi_partial, dim3(nb), dim3(256), 0, s, in, n, part.get());
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(k_maxi_partial, dim3(1), dim3(256), 0, s, part.get(), (int64_t)nb, fin.get());
  HIP_LAUNCH_OK();
  int64_t r = 0;
  HIP_OK(hipMemcpyAsync(&r, fin.get(), sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  return r;
}

int64_t device_sum_i64(const int64_t* in, int64_t n, hipStream_t s) {
  if (n <= 0) return 0;
  const int nb = 512;
  DevBuf<int64_t> part(nb), fin(1);
  hipLaunchKernelGGL(k_sum_partial, dim3(nb), dim3(256), 0, s, in, n, part.get());
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(k_sum_partial, dim3(1), dim3(256), 0, s, part.get(), (int64_t)nb, fin.get());
  HIP_LAUNCH_OK();
  int64_t r = 0;
  HIP_OK(hipMemcpyAsync(&r, fin.get(), sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  return r;
}

}  // namespace sun

#include "rowpipe.hpp"

namespace sun {

int row_capacity() {
  static int cached = 0;
  if (cached) return cached;
  const size_t lim = lds_limit();
  const size_t static_lds = SORT_THREADS * (sizeof(int) + sizeof(double)) + 1024;
  int cap = ROW_CAP_MAX;
  while (cap > 1024 && (size_t)cap * sizeof(uint64_t) + static_lds > lim) cap >>= 1;
  cached = cap;
  return cap;
}

size_t lds_limit() {
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  int v = 0;
  HIP_OK(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  return (size_t)v;
}

}  // namespace sun

extern "C" const char* sun_last_error(void) { return sun::g_last_error.c_str(); }

extern "C" int sun_set_allocator(sun_alloc_fn alloc, sun_release_fn release, void* ctx) {
  return sun::guarded([&] {
    SUN_REQUIRE((alloc == nullptr) == (release == nullptr), SUN_EINVAL,
                "give both the allocation and the release function, or neither");
    std::lock_guard<std::mutex> lock(sun::g_alloc_mu);
    sun::g_alloc = sun::AllocPair{alloc, release, alloc ? ctx : nullptr};
  });
}
extern "C" int sun_version(void) { return 100; }
