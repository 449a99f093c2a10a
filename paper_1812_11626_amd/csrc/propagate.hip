// Classical RK4 on the Bloch ODE dv/dt = G(t) v + K(t) (eq. 9; Sec. IV
// step 3.1) with one fused sparse-matrix-vector + stage-update kernel per RK4
// stage.
//
// Fused matrix layout.  All terms with constant weight are merged into one
// CSR row ("static segment"); the free vector K is folded in as an extra
// column with index M that multiplies a constant 1 stored at x[M]; then each
// time-dependent term contributes one further segment of the row.  Per row
// r: [rowptr[r], seg[0][r]) static, [seg[d][r], seg[d+1][r]) dynamic term d
// (the last one ending at rowptr[r+1]).  So a stage computes
//     k_r = sum_static + sum_d c_d(t) sum_dyn_d,
// reading every matrix byte once and no separate K vector.
//
// Kernel.  The rows are cut into blocks of about `block_nnz` nonzeros.  A
// workgroup streams its block's values and column indices with unit stride
// (every lane a different nonzero), multiplies by the gathered x, parks the
// products in LDS, then one lane per row sums its row segments and applies
// the RK4 stage update, so that the row-wise vectors (v, the accumulator,
// the next stage input) are touched once per stage.  Workgroup ids are
// remapped so that each of the 8 XCDs walks one contiguous range of rows,
// keeping the x gathers of neighbouring rows in that XCD's L2.
//
// Stage arithmetic (same order as the textbook formula):
//   s=1: x2 = v + dt/2 k1,  acc = k1
//   s=2: x3 = v + dt/2 k2,  acc = acc + 2 k2
//   s=3: x4 = v + dt   k3,  acc = acc + 2 k3
//   s=4: v  = v + dt/6 (acc + k4)
#include <algorithm>

#include "internal.hpp"

using namespace sun;

struct sun_prop_s {
  const sun_lind_s* lind = nullptr;
  int64_t M = 0;
  int ndyn = 0;
  int64_t nnz = 0;
  DevBuf<int> rowptr, col, seg, blk_row;
  DevBuf<double> val;
  int64_t nblocks = 0;
  int block_nnz = 2048;
  int xcd_remap = 1;
  DevBuf<double> vaug, xa, xb, acc;
};

namespace {

constexpr int kMaxTerms = 32;
constexpr int kMaxDyn = 4;
constexpr int kThreads = 256;

struct TermList {
  int n;
  const int* rowptr[kMaxTerms];
  const int* col[kMaxTerms];
  const double* val[kMaxTerms];
  double w[kMaxTerms];
};

struct DynList {
  int n;
  const int* rowptr[kMaxDyn];
  const int* col[kMaxDyn];
  const double* val[kMaxDyn];
  const double* K[kMaxDyn];   // free vector of a dynamic dissipator term or NULL
};

// Row sizes (mode 0) or row contents (mode 1) of the fused matrix.
__global__ void k_fuse_rows(int64_t M, TermList st, const double* __restrict__ Kst, DynList dy, int mode,
                            int64_t* __restrict__ cnt, const int64_t* __restrict__ off,
                            int* __restrict__ col, double* __restrict__ val, int* __restrict__ seg) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < M;
       r += (int64_t)gridDim.x * blockDim.x) {
    int pos[kMaxTerms];
    for (int a = 0; a < st.n; ++a) pos[a] = st.rowptr[a][r];
    int64_t w = mode ? off[r] : 0;
    int64_t n = 0;
    while (true) {
      int cmin = INT32_MAX;
      for (int a = 0; a < st.n; ++a)
        if (pos[a] < st.rowptr[a][r + 1]) cmin = min(cmin, st.col[a][pos[a]]);
      if (cmin == INT32_MAX) break;
      double s = 0.0;
      for (int a = 0; a < st.n; ++a)
        if (pos[a] < st.rowptr[a][r + 1] && st.col[a][pos[a]] == cmin) {
          s += st.w[a] * st.val[a][pos[a]];
          ++pos[a];
        }
      if (mode) { col[w + n] = cmin; val[w + n] = s; }
      ++n;
    }
    if (Kst && Kst[r] != 0.0) {
      if (mode) { col[w + n] = (int)M; val[w + n] = Kst[r]; }
      ++n;
    }
    for (int d = 0; d < dy.n; ++d) {
      if (mode) seg[(int64_t)d * M + r] = (int)(w + n);
      for (int e = dy.rowptr[d][r]; e < dy.rowptr[d][r + 1]; ++e) {
        if (mode) { col[w + n] = dy.col[d][e]; val[w + n] = dy.val[d][e]; }
        ++n;
      }
      if (dy.K[d] && dy.K[d][r] != 0.0) {
        if (mode) { col[w + n] = (int)M; val[w + n] = dy.K[d][r]; }
        ++n;
      }
    }
    if (!mode) cnt[r] = n;
  }
}

__global__ void k_axpy_into(int64_t M, double w, const double* __restrict__ x, double* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (int64_t)gridDim.x * blockDim.x)
    y[i] += w * x[i];
}

__global__ void k_i64_to_i32(int64_t n, const int64_t* __restrict__ a, int64_t total, int* __restrict__ b) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = (int)a[i];
  if (blockIdx.x == 0 && threadIdx.x == 0) b[n] = (int)total;
}

// Row-block partition: a block starts at every row whose first nonzero lies
// in a new window of `bn` nonzeros.
__global__ void k_block_flags(int64_t M, const int* __restrict__ rowptr, int bn, int64_t* __restrict__ flag) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < M; r += (int64_t)gridDim.x * blockDim.x)
    flag[r] = (r == 0) || (rowptr[r] / bn != rowptr[r - 1] / bn);
}

__global__ void k_block_rows(int64_t M, const int64_t* __restrict__ flag, const int64_t* __restrict__ id,
                             int64_t nb, int* __restrict__ blk_row) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < M; r += (int64_t)gridDim.x * blockDim.x)
    if (flag[r]) blk_row[id[r]] = (int)r;
  if (blockIdx.x == 0 && threadIdx.x == 0) blk_row[nb] = (int)M;
}

__global__ void k_fill(int64_t n, double v, double* __restrict__ a) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

// ---------------------------------------------------------------------------
// The fused stage kernel
// ---------------------------------------------------------------------------
template <int STAGE>
__device__ inline void rk4_update(int r, double k, const double* v, double* acc, double* xout, double dt) {
  const double vr = v[r];
  if (STAGE == 0) {
    xout[r] = vr + (0.5 * dt) * k;
    acc[r] = k;
  } else if (STAGE == 1) {
    xout[r] = vr + (0.5 * dt) * k;
    acc[r] = acc[r] + 2.0 * k;
  } else if (STAGE == 2) {
    xout[r] = vr + dt * k;
    acc[r] = acc[r] + 2.0 * k;
  } else {
    xout[r] = vr + (dt / 6.0) * (acc[r] + k);
  }
}

template <int STAGE>
__global__ __launch_bounds__(kThreads) void k_rk4_stage(
    const int* __restrict__ rowptr, const int* __restrict__ seg, int ndyn, const int* __restrict__ col,
    const double* __restrict__ val, const int* __restrict__ blk_row, int nblocks, int xcd_remap, int cap,
    const double* __restrict__ xin, const double* v, double* acc, double* xout,
    const double* __restrict__ coef, int64_t coef_row, double dt, int M) {
  extern __shared__ double prod[];
  __shared__ double red[kThreads / 64][1 + kMaxDyn];
  int b = blockIdx.x;
  if (xcd_remap) {
    const int q = (nblocks + 7) >> 3;
    b = (b & 7) * q + (b >> 3);
  }
  if (b >= nblocks) return;
  double eps[kMaxDyn];
#pragma unroll
  for (int d = 0; d < kMaxDyn; ++d) eps[d] = d < ndyn ? coef[coef_row * ndyn + d] : 0.0;

  const int r0 = blk_row[b], r1 = blk_row[b + 1];
  const int e0 = rowptr[r0], e1 = rowptr[r1];
  const int n = e1 - e0;
  const int tid = threadIdx.x;
  if (n <= cap) {
    for (int i = tid; i < n; i += kThreads) prod[i] = val[e0 + i] * xin[col[e0 + i]];
    __syncthreads();
    for (int r = r0 + tid; r < r1; r += kThreads) {
      const int a = rowptr[r] - e0;
      const int z = rowptr[r + 1] - e0;
      int send = ndyn ? seg[r] - e0 : z;
      double k = 0.0;
      for (int i = a; i < send; ++i) k += prod[i];
      for (int d = 0; d < ndyn; ++d) {
        const int s0 = send;
        send = (d + 1 < ndyn) ? seg[(int64_t)(d + 1) * M + r] - e0 : z;
        double sd = 0.0;
        for (int i = s0; i < send; ++i) sd += prod[i];
        k += eps[d] * sd;
      }
      rk4_update<STAGE>(r, k, v, acc, xout, dt);
    }
  } else {
    // rows too long for the LDS buffer: the whole workgroup reduces one row
    for (int r = r0; r < r1; ++r) {
      const int a = rowptr[r], z = rowptr[r + 1];
      double part[1 + kMaxDyn];
#pragma unroll
      for (int d = 0; d <= kMaxDyn; ++d) part[d] = 0.0;
      int bounds[2 + kMaxDyn];
      bounds[0] = a;
      for (int d = 0; d < ndyn; ++d) bounds[d + 1] = seg[(int64_t)d * M + r];
      bounds[ndyn + 1] = z;
      for (int sgm = 0; sgm <= ndyn; ++sgm)
        for (int i = bounds[sgm] + tid; i < bounds[sgm + 1]; i += kThreads) part[sgm] += val[i] * xin[col[i]];
      for (int sgm = 0; sgm <= ndyn; ++sgm) {
        double x = part[sgm];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
        if ((tid & 63) == 0) red[tid >> 6][sgm] = x;
      }
      __syncthreads();
      if (tid == 0) {
        double k = 0.0;
        for (int sgm = 0; sgm <= ndyn; ++sgm) {
          double s = 0.0;
          for (int w = 0; w < kThreads / 64; ++w) s += red[w][sgm];
          k += (sgm == 0 ? 1.0 : eps[sgm - 1]) * s;
        }
        rk4_update<STAGE>(r, k, v, acc, xout, dt);
      }
      __syncthreads();
    }
  }
}

void build_partition(sun_prop_s& p, hipStream_t s) {
  const int64_t M = p.M;
  DevBuf<int64_t> flag(M), id(M);
  hipLaunchKernelGGL(k_block_flags, dim3(grid_for(M, 256)), dim3(256), 0, s, M, p.rowptr.get(), p.block_nnz,
                     flag.get());
  HIP_LAUNCH_OK();
  p.nblocks = exclusive_scan_i64(flag.get(), id.get(), M, s);
  p.blk_row.alloc(p.nblocks + 1);
  hipLaunchKernelGGL(k_block_rows, dim3(grid_for(M, 256)), dim3(256), 0, s, M, flag.get(), id.get(), p.nblocks,
                     p.blk_row.get());
  HIP_LAUNCH_OK();
  HIP_OK(hipStreamSynchronize(s));
}

int stage_capacity(int block_nnz) {
  static size_t lim = 0;
  if (!lim) lim = lds_limit();
  int cap = 2 * block_nnz;
  while (cap > 256 && (size_t)cap * sizeof(double) + 1024 > lim) cap >>= 1;
  return cap;
}

template <int STAGE>
void launch_stage(const sun_prop_s& p, const double* xin, double* xout, const double* coef, int64_t row,
                  double dt, hipStream_t s) {
  const int cap = stage_capacity(p.block_nnz);
  const int grid = p.xcd_remap ? (int)(((p.nblocks + 7) / 8) * 8) : (int)p.nblocks;
  hipLaunchKernelGGL((k_rk4_stage<STAGE>), dim3(grid), dim3(kThreads), cap * sizeof(double), s,
                     p.rowptr.get(), p.seg.get(), p.ndyn, p.col.get(), p.val.get(), p.blk_row.get(),
                     (int)p.nblocks, p.xcd_remap, cap, xin, p.vaug.get(), p.acc.get(), xout, coef, row, dt,
                     (int)p.M);
}

}  // namespace

extern "C" int sun_prop_create(sun_lind l, const double* static_w, const int32_t* dyn, int32_t ndyn,
                               void* stream, sun_prop* out) {
  return guarded([&] {
    SUN_REQUIRE(out != nullptr, SUN_EINVAL, "out is NULL");
    *out = nullptr;
    SUN_REQUIRE(l != nullptr && static_w != nullptr, SUN_EINVAL, "NULL argument");
    SUN_REQUIRE(ndyn >= 0 && ndyn <= kMaxDyn, SUN_ENOTSUP, "at most 4 time-dependent terms");
    SUN_REQUIRE(ndyn == 0 || dyn != nullptr, SUN_EINVAL, "dyn is NULL");
    const int nt = l->nH + l->P;
    SUN_REQUIRE(nt <= kMaxTerms, SUN_ENOTSUP, "at most 32 terms");
    hipStream_t s = as_stream(stream);
    const int64_t M = l->basis->M;
    auto p = new sun_prop_s();
    try {
      p->lind = l;
      p->M = M;
      p->ndyn = ndyn;
      TermList st{};
      DynList dy{};
      DevBuf<double> Kst(M);
      HIP_OK(hipMemsetAsync(Kst.get(), 0, M * sizeof(double), s));
      bool anyK = false;
      for (int a = 0; a < nt; ++a) {
        if (static_w[a] == 0.0) continue;
        const DevCSR& m = a < l->nH ? l->QH[a] : l->R[a - l->nH];
        st.rowptr[st.n] = m.rowptr.get();
        st.col[st.n] = m.col.get();
        st.val[st.n] = m.val.get();
        st.w[st.n] = static_w[a];
        ++st.n;
        if (a >= l->nH) {
          hipLaunchKernelGGL(k_axpy_into, dim3(grid_for(M, 256)), dim3(256), 0, s, M, static_w[a],
                             l->K[a - l->nH].get(), Kst.get());
          HIP_LAUNCH_OK();
          anyK = true;
        }
      }
      for (int d = 0; d < ndyn; ++d) {
        const int a = dyn[d];
        SUN_REQUIRE(a >= 0 && a < nt, SUN_EINVAL, "dynamic term index out of range");
        const DevCSR& m = a < l->nH ? l->QH[a] : l->R[a - l->nH];
        dy.rowptr[d] = m.rowptr.get();
        dy.col[d] = m.col.get();
        dy.val[d] = m.val.get();
        dy.K[d] = a < l->nH ? nullptr : l->K[a - l->nH].get();
      }
      dy.n = ndyn;
      DevBuf<int64_t> cnt(M), off(M);
      hipLaunchKernelGGL(k_fuse_rows, dim3(grid_for(M, 128)), dim3(128), 0, s, M, st, anyK ? Kst.get() : nullptr,
                         dy, 0, cnt.get(), nullptr, nullptr, nullptr, nullptr);
      HIP_LAUNCH_OK();
      p->nnz = exclusive_scan_i64(cnt.get(), off.get(), M, s);
      SUN_REQUIRE(p->nnz < (int64_t)INT32_MAX, SUN_ENOTSUP, "fused matrix has 2^31 or more nonzeros");
      p->rowptr.alloc(M + 1);
      p->col.alloc(p->nnz > 0 ? p->nnz : 1);
      p->val.alloc(p->nnz > 0 ? p->nnz : 1);
      p->seg.alloc(ndyn > 0 ? ndyn * M : 1);
      hipLaunchKernelGGL(k_fuse_rows, dim3(grid_for(M, 128)), dim3(128), 0, s, M, st, anyK ? Kst.get() : nullptr,
                         dy, 1, nullptr, off.get(), p->col.get(), p->val.get(), p->seg.get());
      HIP_LAUNCH_OK();
      hipLaunchKernelGGL(k_i64_to_i32, dim3(grid_for(M, 256)), dim3(256), 0, s, M, off.get(), p->nnz,
                         p->rowptr.get());
      HIP_LAUNCH_OK();
      build_partition(*p, s);
      p->vaug.alloc(M + 1);
      p->xa.alloc(M + 1);
      p->xb.alloc(M + 1);
      p->acc.alloc(M + 1);
      for (DevBuf<double>* b : {&p->vaug, &p->xa, &p->xb, &p->acc}) {
        hipLaunchKernelGGL(k_fill, dim3(grid_for(M + 1, 256)), dim3(256), 0, s, M + 1, 0.0, b->get());
        HIP_LAUNCH_OK();
        hipLaunchKernelGGL(k_fill, dim3(1), dim3(1), 0, s, (int64_t)1, 1.0, b->get() + M);
        HIP_LAUNCH_OK();
      }
      HIP_OK(hipStreamSynchronize(s));
    } catch (...) {
      delete p;
      throw;
    }
    *out = p;
  });
}

extern "C" int sun_prop_tune(sun_prop p, int32_t block_nnz, int32_t xcd_remap, void* stream) {
  return guarded([&] {
    SUN_REQUIRE(p != nullptr, SUN_EINVAL, "prop is NULL");
    SUN_REQUIRE(block_nnz >= 256 && block_nnz <= 8192 && (block_nnz & (block_nnz - 1)) == 0, SUN_EINVAL,
                "block_nnz must be a power of two in [256, 8192]");
    p->block_nnz = block_nnz;
    p->xcd_remap = xcd_remap ? 1 : 0;
    build_partition(*p, as_stream(stream));
  });
}

extern "C" int sun_prop_info(sun_prop p, int64_t* nnz_fused, int64_t* nblocks, int64_t* M) {
  return guarded([&] {
    SUN_REQUIRE(p != nullptr, SUN_EINVAL, "prop is NULL");
    if (nnz_fused) *nnz_fused = p->nnz;
    if (nblocks) *nblocks = p->nblocks;
    if (M) *M = p->M;
  });
}

extern "C" int sun_propagate(sun_prop p, double* v, const double* coef, double dt, int64_t steps, void* stream) {
  return guarded([&] {
    SUN_REQUIRE(p != nullptr && v != nullptr, SUN_EINVAL, "NULL argument");
    SUN_REQUIRE(steps >= 0, SUN_EINVAL, "steps must be >= 0");
    SUN_REQUIRE(p->ndyn == 0 || coef != nullptr, SUN_EINVAL, "coef is NULL");
    if (steps == 0) return;
    hipStream_t s = as_stream(stream);
    const int64_t M = p->M;
    HIP_OK(hipMemcpyAsync(p->vaug.get(), v, M * sizeof(double), hipMemcpyDeviceToDevice, s));
    double* va = p->vaug.get();
    double* xa = p->xa.get();
    double* xb = p->xb.get();
    for (int64_t n = 0; n < steps; ++n) {
      launch_stage<0>(*p, va, xa, coef, 2 * n, dt, s);
      launch_stage<1>(*p, xa, xb, coef, 2 * n + 1, dt, s);
      launch_stage<2>(*p, xb, xa, coef, 2 * n + 1, dt, s);
      launch_stage<3>(*p, xa, va, coef, 2 * n + 2, dt, s);
    }
    HIP_LAUNCH_OK();
    HIP_OK(hipMemcpyAsync(v, p->vaug.get(), M * sizeof(double), hipMemcpyDeviceToDevice, s));
  });
}

extern "C" void sun_prop_free(sun_prop p) { delete p; }
