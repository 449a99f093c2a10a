// Row-by-row assembly of a sparse matrix from raw contributions.
//
// A generator enumerates, for each output row, a list of raw contributions
// (column key, value) in any order, possibly with repeated keys.  The
// pipeline turns them into CSR with sorted unique columns:
//   1. count raw contributions per row (the generator run with a counter),
//   2. exclusive scan -> raw offsets,
//   3. fill raw (key, value) pairs,
//   4. per row, one workgroup sorts (key, raw position) pairs in LDS with a
//      bitonic network and sums the values of equal keys in raw order (so the
//      result is bitwise reproducible), optionally dropping exact zeros,
//   5. optional relative threshold against the global max |value|
//      (removes cancellation residues), count kept entries, scan, compact.
//
// This replaces the paper's coordinate-format build + quicksort / radix sort
// + red-black-tree accumulation (Sec. IV, steps 2.2-2.5) with a sort that
// only ever sees one row at a time.
#pragma once

#include "common.hpp"

namespace sun {

constexpr int ROW_CAP_MAX = 16384;  // raw contributions per row (LDS sort size)
constexpr int ROW_CAP_BITS = 14;
constexpr int SORT_THREADS = 256;

// Largest power-of-two sort capacity whose key array fits the device's
// per-workgroup LDS next to the kernel's static LDS (at most ROW_CAP_MAX).
int row_capacity();

template <class V>
struct Counter {
  int64_t n = 0;
  __device__ void operator()(uint64_t, V) { ++n; }
};

// Writes the raw contributions of one row into [pos, end); never past end.
template <class V>
struct Writer {
  uint64_t* key;
  V* val;
  int64_t pos;
  int64_t end;
  __device__ void operator()(uint64_t k, V v) {
    if (pos < end) {
      key[pos] = k;
      val[pos] = v;
    }
    ++pos;
  }
};

template <class G, class V>
__global__ __launch_bounds__(256) void k_rows_count(G g, int64_t rows, int64_t* __restrict__ cnt) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < rows;
       r += (int64_t)gridDim.x * blockDim.x) {
    Counter<V> c;
    g.run((int)r, c);
    cnt[r] = c.n;
  }
}

template <class G, class V>
__global__ __launch_bounds__(256) void k_rows_fill(G g, int64_t rows, const int64_t* __restrict__ off,
                                                   const int64_t* __restrict__ cnt,
                                                   uint64_t* __restrict__ key, V* __restrict__ val,
                                                   int* __restrict__ mismatch) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < rows;
       r += (int64_t)gridDim.x * blockDim.x) {
    Writer<V> w{key, val, off[r], off[r] + cnt[r]};
    g.run((int)r, w);
    if (w.pos != w.end) atomicOr(mismatch, 1);
  }
}

template <class V>
__device__ inline V vzero();
template <>
__device__ inline double vzero<double>() { return 0.0; }
template <>
__device__ inline cplx vzero<cplx>() { return cx(0.0, 0.0); }

__device__ inline double vadd(double a, double b) { return a + b; }
__device__ inline cplx vadd(cplx a, cplx b) { return a + b; }

// One workgroup per row: sort + merge.  Dynamic LDS: ROW_CAP * 8 bytes.
template <class V>
__global__ __launch_bounds__(SORT_THREADS) void k_rows_sort_merge(
    int64_t rows, const int64_t* __restrict__ off, const int64_t* __restrict__ cnt,
    const uint64_t* __restrict__ key, const V* __restrict__ val, uint64_t* __restrict__ mkey,
    V* __restrict__ mval, int64_t* __restrict__ mcnt, double* __restrict__ rowmax, int drop_zero,
    int cap, int* __restrict__ overflow) {
  extern __shared__ uint64_t sk[];
  __shared__ int sh_cnt[SORT_THREADS];
  __shared__ double sh_max[SORT_THREADS];
  const int tid = threadIdx.x;
  for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
    const int64_t o = off[r];
    const int64_t n64 = cnt[r];
    if (n64 > cap) {
      if (tid == 0) {
        atomicOr(overflow, 1);
        mcnt[r] = 0;
        rowmax[r] = 0.0;
      }
      continue;
    }
    const int n = (int)n64;
    if (n == 0) {
      if (tid == 0) {
        mcnt[r] = 0;
        rowmax[r] = 0.0;
      }
      continue;
    }
    int np2 = 1;
    while (np2 < n) np2 <<= 1;
    for (int i = tid; i < np2; i += SORT_THREADS)
      sk[i] = (i < n) ? ((key[o + i] << ROW_CAP_BITS) | (uint64_t)i) : ~0ull;
    __syncthreads();
    // bitonic sort, ascending
    for (int k = 2; k <= np2; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int i = tid; i < np2; i += SORT_THREADS) {
          int l = i ^ j;
          if (l > i) {
            uint64_t a = sk[i], b = sk[l];
            bool up = ((i & k) == 0);
            if ((a > b) == up) {
              sk[i] = b;
              sk[l] = a;
            }
          }
        }
        __syncthreads();
      }
    }
    // each thread owns a contiguous chunk of sorted positions
    const int chunk = (n + SORT_THREADS - 1) / SORT_THREADS;
    const int p0 = tid * chunk;
    const int p1 = min(n, p0 + chunk);
    int kept = 0;
    double lmax = 0.0;
    for (int p = p0; p < p1; ++p) {
      uint64_t kk = sk[p] >> ROW_CAP_BITS;
      if (p > 0 && (sk[p - 1] >> ROW_CAP_BITS) == kk) continue;
      V s = vzero<V>();
      for (int q = p; q < n && (sk[q] >> ROW_CAP_BITS) == kk; ++q)
        s = vadd(s, val[o + (int64_t)(sk[q] & ((1u << ROW_CAP_BITS) - 1))]);
      if (drop_zero && is_zero(s)) continue;
      ++kept;
      lmax = fmax(lmax, absval(s));
    }
    sh_cnt[tid] = kept;
    sh_max[tid] = lmax;
    __syncthreads();
    // inclusive scan of the counts, max reduction
    for (int d = 1; d < SORT_THREADS; d <<= 1) {
      int t = tid >= d ? sh_cnt[tid - d] : 0;
      double m = tid >= d ? sh_max[tid - d] : 0.0;
      __syncthreads();
      sh_cnt[tid] += t;
      sh_max[tid] = fmax(sh_max[tid], m);
      __syncthreads();
    }
    int rank = tid ? sh_cnt[tid - 1] : 0;
    for (int p = p0; p < p1; ++p) {
      uint64_t kk = sk[p] >> ROW_CAP_BITS;
      if (p > 0 && (sk[p - 1] >> ROW_CAP_BITS) == kk) continue;
      V s = vzero<V>();
      for (int q = p; q < n && (sk[q] >> ROW_CAP_BITS) == kk; ++q)
        s = vadd(s, val[o + (int64_t)(sk[q] & ((1u << ROW_CAP_BITS) - 1))]);
      if (drop_zero && is_zero(s)) continue;
      mkey[o + rank] = kk;
      mval[o + rank] = s;
      ++rank;
    }
    if (tid == SORT_THREADS - 1) {
      mcnt[r] = sh_cnt[SORT_THREADS - 1];
      rowmax[r] = sh_max[SORT_THREADS - 1];
    }
    __syncthreads();
  }
}

template <class V>
__global__ __launch_bounds__(256) void k_rows_count_kept(int64_t rows, const int64_t* __restrict__ off,
                                                         const int64_t* __restrict__ mcnt,
                                                         const V* __restrict__ mval, double thr,
                                                         int64_t* __restrict__ kcnt) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < rows;
       r += (int64_t)gridDim.x * blockDim.x) {
    int64_t o = off[r], n = mcnt[r], k = 0;
    for (int64_t i = 0; i < n; ++i) k += (absval(mval[o + i]) > thr);
    kcnt[r] = k;
  }
}

template <class V, class K>
__global__ __launch_bounds__(256) void k_rows_compact(int64_t rows, const int64_t* __restrict__ off,
                                                      const int64_t* __restrict__ mcnt,
                                                      const uint64_t* __restrict__ mkey,
                                                      const V* __restrict__ mval, double thr,
                                                      const int64_t* __restrict__ outoff, int64_t total,
                                                      int* __restrict__ rowptr, K* __restrict__ col,
                                                      V* __restrict__ outval) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < rows;
       r += (int64_t)gridDim.x * blockDim.x) {
    int64_t o = off[r], n = mcnt[r], w = outoff[r];
    if (rowptr) rowptr[r] = (int)w;
    for (int64_t i = 0; i < n; ++i) {
      V v = mval[o + i];
      if (absval(v) > thr) {
        col[w] = (K)mkey[o + i];
        outval[w] = v;
        ++w;
      }
    }
    if (r == rows - 1 && rowptr) rowptr[rows] = (int)total;
  }
}

struct RowAssemblyResult {
  int64_t nnz = 0;
  int64_t raw = 0;
  int64_t max_row_raw = 0;
};

// Run the whole pipeline.  rel_drop > 0: drop |v| <= rel_drop * max|v|;
// drop_zero: drop exact zeros already in the merge step.  Outputs are
// (re)allocated: rowptr int[rows+1] (if want_rowptr), col K[nnz], val V[nnz].
// Synchronises the stream.
template <class G, class V, class K>
RowAssemblyResult assemble_rows(const G& g, int64_t rows, double rel_drop, bool drop_zero,
                                hipStream_t s, DevBuf<int>* rowptr, DevBuf<K>& col,
                                DevBuf<V>& val, DevBuf<int64_t>* row_offsets = nullptr) {
  RowAssemblyResult res;
  if (rows <= 0) SUN_THROW(SUN_EINVAL, "no rows");
  DevBuf<int64_t> cnt(rows), off(rows);
  hipLaunchKernelGGL((k_rows_count<G, V>), dim3(grid_for(rows, 256)), dim3(256), 0, s, g, rows,
                     cnt.get());
  HIP_LAUNCH_OK();
  const int cap = row_capacity();
  res.max_row_raw = device_max_i64(cnt.get(), rows, s);
  if (res.max_row_raw > cap) {
    SUN_THROW(SUN_ENOTSUP, "a row has " + std::to_string(res.max_row_raw) +
                               " raw contributions, more than the LDS sort holds (" + std::to_string(cap) +
                               "); operator too dense for the LDS row sort");
  }
  res.raw = exclusive_scan_i64(cnt.get(), off.get(), rows, s);
  DevBuf<uint64_t> key(res.raw > 0 ? res.raw : 1), mkey(res.raw > 0 ? res.raw : 1);
  DevBuf<V> rval(res.raw > 0 ? res.raw : 1), mval(res.raw > 0 ? res.raw : 1);
  DevBuf<int> flags(2);   // [0] count/fill mismatch, [1] row overflow
  HIP_OK(hipMemsetAsync(flags.get(), 0, 2 * sizeof(int), s));
  hipLaunchKernelGGL((k_rows_fill<G, V>), dim3(grid_for(rows, 256)), dim3(256), 0, s, g, rows,
                     off.get(), cnt.get(), key.get(), rval.get(), flags.get());
  HIP_LAUNCH_OK();
  DevBuf<int64_t> mcnt(rows);
  DevBuf<double> rowmax(rows);
  unsigned sgrid = (unsigned)(rows < 65536 ? rows : 65536);
  hipLaunchKernelGGL((k_rows_sort_merge<V>), dim3(sgrid), dim3(SORT_THREADS),
                     cap * sizeof(uint64_t), s, rows, off.get(), cnt.get(), key.get(),
                     rval.get(), mkey.get(), mval.get(), mcnt.get(), rowmax.get(), drop_zero ? 1 : 0,
                     cap, flags.get() + 1);
  HIP_LAUNCH_OK();
  int hf[2] = {0, 0};
  HIP_OK(hipMemcpyAsync(hf, flags.get(), sizeof(hf), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  if (hf[0]) SUN_THROW(SUN_EDEVICE, "row generator produced different counts in its two passes");
  if (hf[1]) {
    SUN_THROW(SUN_ENOTSUP, "a row has more raw contributions than the LDS sort holds (" +
                               std::to_string(cap) + "); operator too dense for the LDS row sort");
  }
  double thr = 0.0;
  if (rel_drop > 0) thr = rel_drop * device_max(rowmax.get(), rows, s);
  DevBuf<int64_t> kcnt(rows), koff(rows);
  hipLaunchKernelGGL((k_rows_count_kept<V>), dim3(grid_for(rows, 256)), dim3(256), 0, s, rows,
                     off.get(), mcnt.get(), mval.get(), thr, kcnt.get());
  HIP_LAUNCH_OK();
  res.nnz = exclusive_scan_i64(kcnt.get(), koff.get(), rows, s);
  if (rowptr && res.nnz >= (int64_t)INT32_MAX)
    SUN_THROW(SUN_ENOTSUP, "matrix has 2^31 or more nonzeros");
  if (rowptr) rowptr->alloc(rows + 1);
  col.alloc(res.nnz > 0 ? res.nnz : 1);
  val.alloc(res.nnz > 0 ? res.nnz : 1);
  hipLaunchKernelGGL((k_rows_compact<V, K>), dim3(grid_for(rows, 256)), dim3(256), 0, s, rows,
                     off.get(), mcnt.get(), mkey.get(), mval.get(), thr, koff.get(), res.nnz,
                     rowptr ? rowptr->get() : nullptr, col.get(), val.get());
  HIP_LAUNCH_OK();
  if (row_offsets) *row_offsets = std::move(koff);
  HIP_OK(hipStreamSynchronize(s));
  return res;
}

}  // namespace sun
