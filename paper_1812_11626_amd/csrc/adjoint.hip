// Discrete adjoint of the RK4 propagation (eq. 9; Sec. IV step 3.1) for the
// gradient of a time-averaged observable
//     J = (1/S) sum_{n = steps-S+1}^{steps} c . v_n
// with respect to parameters theta on which the term coefficients depend:
//     G(t) = sum_a c_a(t) T_a,  K(t) = sum_{a dissipator} c_a(t) K_a,
//     c_a = w_a (static) or the table value c_d(t_k) (time-dependent term d),
//     d c_a / d theta = dstatic[a][theta] or dcoef[k][d][theta].
//
// Reverse sweep of one step n (v' = v + dt/6 (k1 + 2k2 + 2k3 + k4)), with
// lambda = dJ/dv_{n+1}:
//     kb4 = dt/6 lambda,              xb4 = G(t_{n+1})^T kb4
//     kb3 = dt/3 lambda + dt xb4,     xb3 = G(t_{n+1/2})^T kb3
//     kb2 = dt/3 lambda + dt/2 xb3,   xb2 = G(t_{n+1/2})^T kb2
//     kb1 = dt/6 lambda + dt/2 xb2,   xb1 = G(t_n)^T kb1
//     lambda <- lambda + xb4 + xb3 + xb2 + xb1  (+ c/S where v_n enters J)
//     grad   += sum_i sum_a dc_a/dtheta(t_i) kb_i . (T_a x_i + K_a)
// where x_i are the forward stage inputs of step n.  The transposed
// generator runs on the same fused stage kernels (a second propagator built
// from the transposed terms, with the reverse-mode vector updates fused in);
// with at most three parameter-dependent terms those terms are separate
// segments of its rows and each reverse stage also forms
// kb_i . (T_a x_i + K_a) = (T_a^T kb_i) . x_i + kb_i . K_a in the same pass.
// States are checkpointed every `ckpt_every` steps in the forward sweep; the
// backward sweep recomputes one checkpoint interval at a time, except the
// last, whose states and stage inputs the forward sweep leaves in place.
#include <algorithm>
#include <vector>

#include "prop_internal.hpp"

using namespace sun;

struct sun_adj_s {
  const sun_lind_s* lind = nullptr;
  sun_lind_s lindT;             // transposed terms, K = 0
  sun_prop fwd = nullptr, bwd = nullptr;
  std::vector<sun_prop> termp;  // per term: the term alone (unit weight), for the parameter dot products
  // transposed generator with each parameter-dependent term as its own
  // segment (segmented sliced layout), for reverse stages with the dot
  // products fused in; built for the term list revg_terms
  sun_prop revg = nullptr;
  std::vector<int> revg_terms;
  std::vector<double> static_w;
  std::vector<int> dyn;
  int nt = 0, ndyn = 0;
  int64_t M = 0;
  ~sun_adj_s() {
    if (fwd) sun_prop_free(fwd);
    if (bwd) sun_prop_free(bwd);
    if (revg) sun_prop_free(revg);
    for (sun_prop q : termp)
      if (q) sun_prop_free(q);
  }
};

namespace {

// ---------------------------------------------------------------------------
// CSR transpose (count, scan, scatter, per-row sort for a deterministic order)
// ---------------------------------------------------------------------------
__global__ void k_tr_count(int64_t M, const int* __restrict__ rowptr, const int* __restrict__ col,
                           int64_t* __restrict__ cnt) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < M; r += (int64_t)gridDim.x * blockDim.x)
    for (int e = rowptr[r]; e < rowptr[r + 1]; ++e)
      atomicAdd(reinterpret_cast<unsigned long long*>(&cnt[col[e]]), 1ull);
}

__global__ void k_tr_fill(int64_t M, const int* __restrict__ rowptr, const int* __restrict__ col,
                          const double* __restrict__ val, const int64_t* __restrict__ off, int* __restrict__ slot,
                          int* __restrict__ tcol, double* __restrict__ tval) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < M; r += (int64_t)gridDim.x * blockDim.x)
    for (int e = rowptr[r]; e < rowptr[r + 1]; ++e) {
      const int c = col[e];
      const int k = atomicAdd(&slot[c], 1);
      tcol[off[c] + k] = (int)r;
      tval[off[c] + k] = val[e];
    }
}

__global__ void k_tr_sort(int64_t M, const int64_t* __restrict__ off, const int64_t* __restrict__ cnt,
                          int* __restrict__ tcol, double* __restrict__ tval, int* __restrict__ rowptr) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < M; r += (int64_t)gridDim.x * blockDim.x) {
    int* c = tcol + off[r];
    double* v = tval + off[r];
    const int n = (int)cnt[r];
    for (int i = 1; i < n; ++i) {
      const int ci = c[i];
      const double vi = v[i];
      int j = i - 1;
      while (j >= 0 && c[j] > ci) { c[j + 1] = c[j]; v[j + 1] = v[j]; --j; }
      c[j + 1] = ci;
      v[j + 1] = vi;
    }
    rowptr[r] = (int)off[r];
    if (r == M - 1) rowptr[M] = (int)(off[r] + cnt[r]);
  }
}

void transpose(const DevCSR& A, DevCSR& T, hipStream_t s) {
  const int64_t M = A.rows;
  DevBuf<int64_t> cnt(M), off(M);
  DevBuf<int> slot(M);
  HIP_OK(hipMemsetAsync(cnt.get(), 0, M * sizeof(int64_t), s));
  HIP_OK(hipMemsetAsync(slot.get(), 0, M * sizeof(int), s));
  hipLaunchKernelGGL(k_tr_count, dim3(grid_for(M, 256)), dim3(256), 0, s, M, A.rowptr.get(), A.col.get(), cnt.get());
  HIP_LAUNCH_OK();
  const int64_t nnz = exclusive_scan_i64(cnt.get(), off.get(), M, s);
  T.rows = M;
  T.nnz = nnz;
  T.rowptr.alloc(M + 1);
  T.col.alloc(nnz > 0 ? nnz : 1);
  T.val.alloc(nnz > 0 ? nnz : 1);
  hipLaunchKernelGGL(k_tr_fill, dim3(grid_for(M, 256)), dim3(256), 0, s, M, A.rowptr.get(), A.col.get(),
                     A.val.get(), off.get(), slot.get(), T.col.get(), T.val.get());
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(k_tr_sort, dim3(grid_for(M, 64)), dim3(64), 0, s, M, off.get(), cnt.get(), T.col.get(),
                     T.val.get(), T.rowptr.get());
  HIP_LAUNCH_OK();
  HIP_OK(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------------------
// Small vector kernels
// ---------------------------------------------------------------------------
__global__ void k_adj_prep(int64_t M, double* __restrict__ lam, const double* __restrict__ cobs, double cscale,
                           double dt6, double* __restrict__ kb) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (int64_t)gridDim.x * blockDim.x) {
    double l = lam[i];
    if (cscale != 0.0) l = l + cobs[i] * cscale;
    lam[i] = l;
    kb[i] = dt6 * l;
  }
}

// a[i * stride + off] = v for i < n (sets the constant entry x[M] = 1 of
// vectors stored back to back)
__global__ void k_adj_fill_strided(int64_t n, int64_t stride, int64_t off, double v, double* __restrict__ a) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i * stride + off] = v;
}

__global__ void k_adj_fill(int64_t n, double v, double* __restrict__ a) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

constexpr int kDotBlocks = 512;
constexpr int kMaxTheta = 8;
constexpr int kMaxGTerms = 8;

// Running per-thread sums for a time average: each thread of the fixed grid
// (nbj blocks of 256) adds c[i] a_s[i] over its rows i, for the count vectors
// a_s = a0 + s * stride taken from the last to the first, to its own slot of
// run.  The additions into a slot follow the global order of the states
// however the calls split them, so the result does not depend on how the
// states are grouped into calls.
__global__ __launch_bounds__(256) void k_dot_acc_states(int64_t n, const double* __restrict__ c,
                                                        const double* __restrict__ a0, int64_t stride, int64_t count,
                                                        double* __restrict__ run) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double s = run[gid];
  for (int64_t k = count - 1; k >= 0; --k) {
    const double* a = a0 + k * stride;
    for (int64_t i = gid; i < n; i += (int64_t)gridDim.x * blockDim.x) s += c[i] * a[i];
  }
  run[gid] = s;
}

// out[i] = a[i] * w for i < n, out[n] = 0
__global__ void k_adj_scaled(int64_t n, const double* __restrict__ a, double w, double* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = i < n ? a[i] * w : 0.0;
}

// Sum of n partials by one workgroup in a fixed order (strided per lane,
// then a tree), result in sh[0] of lane 0.
__device__ inline double block_sum_fixed(const double* __restrict__ part, int n, double* sh) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += part[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = blockDim.x >> 1; o > 0; o >>= 1) {
    if (threadIdx.x < (unsigned)o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// out[0] += scale * dot(a, b) in a fixed order (two passes)
__global__ __launch_bounds__(256) void k_dot_partial(int64_t n, const double* __restrict__ a,
                                                     const double* __restrict__ b, double* __restrict__ part) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    s += a[i] * b[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < (unsigned)o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_dot_finish(const double* __restrict__ part, int nblk, double scale,
                                                    double* __restrict__ out) {
  __shared__ double sh[256];
  const double s = block_sum_fixed(part, nblk, sh);
  if (threadIdx.x == 0) out[0] += scale * s;
}

// out[th] = sum over y < ny and k < n of part[(y * ntheta + th) * n + k], in a
// fixed order; one workgroup per th.
__global__ __launch_bounds__(256) void k_sum_slots(const double* __restrict__ part, int ny, int ntheta, int n,
                                                   double* __restrict__ out) {
  __shared__ double sh[256];
  double t = 0.0;
  for (int y = 0; y < ny; ++y) t += block_sum_fixed(part + ((int64_t)y * ntheta + blockIdx.x) * n, n, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = t;
}

int dot_blocks(int64_t n) { return (int)std::min<int64_t>(kDotBlocks, std::max<int64_t>(1, (n + 255) / 256)); }

void dot_accumulate(const double* a, const double* b, int64_t n, double scale, double* part, double* out,
                    hipStream_t s) {
  const int nb = dot_blocks(n);
  hipLaunchKernelGGL(k_dot_partial, dim3(nb), dim3(256), 0, s, n, a, b, part);
  hipLaunchKernelGGL(k_dot_finish, dim3(1), dim3(256), 0, s, part, nb, scale, out);
}

// Forward RK4 step of the fused propagator: v (M+1) -> vout (M+1); x2/x3/x4
// receive the stage inputs when non-NULL, else scratch buffers are used.
void forward_step(const sun_prop_s& p, const double* v, double* vout, double* x2, double* x3, double* x4,
                  double* acc, const double* coef, int64_t n, double dt, hipStream_t s) {
  prop_stage(p, 0, v, v, acc, x2, coef, 2 * n, dt, s);
  prop_stage(p, 1, x2, v, acc, x3, coef, 2 * n + 1, dt, s);
  prop_stage(p, 2, x3, v, acc, x4, coef, 2 * n + 1, dt, s);
  prop_stage(p, 3, x4, v, acc, vout, coef, 2 * n + 2, dt, s);   // vout[M] must already be 1
}

}  // namespace

extern "C" int sun_adjoint_create(sun_lind l, const double* static_w, const int32_t* dyn, int32_t ndyn,
                                  void* stream, sun_adj* out) {
  return guarded([&] {
    SUN_REQUIRE(out != nullptr, SUN_EINVAL, "out is NULL");
    *out = nullptr;
    SUN_REQUIRE(l != nullptr && static_w != nullptr, SUN_EINVAL, "NULL argument");
    SUN_REQUIRE(ndyn >= 0 && ndyn <= 1, SUN_ENOTSUP, "the adjoint supports at most one time-dependent term");
    SUN_REQUIRE(ndyn == 0 || dyn != nullptr, SUN_EINVAL, "dyn is NULL");
    const int nt = l->nH + l->P;
    SUN_REQUIRE(nt <= kMaxGTerms, SUN_ENOTSUP, "at most 8 terms");
    hipStream_t s = as_stream(stream);
    auto a = new sun_adj_s();
    try {
      a->lind = l;
      a->nt = nt;
      a->ndyn = ndyn;
      a->M = l->basis->M;
      a->static_w.assign(static_w, static_w + nt);
      a->dyn.assign(dyn, dyn + ndyn);
      sun_lind_s& T = a->lindT;
      T.basis = l->basis;
      T.nH = l->nH;
      T.P = l->P;
      T.QH.resize(l->nH);
      T.R.resize(l->P);
      T.K.resize(l->P);
      for (int h = 0; h < l->nH; ++h) transpose(l->QH[h], T.QH[h], s);
      for (int p = 0; p < l->P; ++p) {
        transpose(l->R[p], T.R[p], s);
        T.K[p].alloc(a->M);
        HIP_OK(hipMemsetAsync(T.K[p].get(), 0, a->M * sizeof(double), s));
      }
      int st = sun_prop_create(l, static_w, dyn, ndyn, stream, &a->fwd);
      if (st != SUN_OK) SUN_THROW(st, std::string("forward propagator: ") + sun_last_error());
      st = sun_prop_create(&a->lindT, static_w, dyn, ndyn, stream, &a->bwd);
      if (st != SUN_OK) SUN_THROW(st, std::string("transposed propagator: ") + sun_last_error());
      HIP_OK(hipStreamSynchronize(s));
    } catch (...) {
      delete a;
      throw;
    }
    *out = a;
  });
}

namespace {

// Stage inputs x2, x3, x4 of a whole checkpoint interval are kept when they
// need at most this many bytes; otherwise they are recomputed per step.
constexpr double kStageStoreBytes = 64.0 * (1ull << 30);

struct Work {
  DevBuf<double> ck;        // checkpoints [(nck) * (M+1)]
  DevBuf<double> per;       // states of one interval [(C+1) * (M+1)]
  DevBuf<double> stg;       // stage inputs of one interval [C][3][M+1] (optional)
  DevBuf<double> x2, x3, x4, acc, lam, lacc, kb4, kb3, kb2, kb1, gpart, jrun, dev_grad, dev_J, dstat;
  DevBuf<double> cw, zero;  // objective weights c/S_avg, and zeros (M+1 each)
};

}  // namespace

extern "C" int sun_adjoint_run(sun_adj a, const double* v0, const double* coef, const double* dstatic,
                               const double* dcoef, int32_t ntheta, const double* cobs, double dt, int64_t steps,
                               int64_t S_avg, int64_t ckpt_every, double* J_out, double* grad_out, void* stream) {
  return guarded([&] {
    SUN_REQUIRE(a != nullptr && v0 != nullptr && cobs != nullptr, SUN_EINVAL, "NULL argument");
    SUN_REQUIRE(ntheta >= 0 && ntheta <= kMaxTheta, SUN_ENOTSUP, "at most 8 parameters");
    SUN_REQUIRE(ntheta == 0 || dstatic != nullptr, SUN_EINVAL, "dstatic is NULL");
    SUN_REQUIRE(a->ndyn == 0 || coef != nullptr, SUN_EINVAL, "coef is NULL");
    SUN_REQUIRE(steps >= 1 && S_avg >= 1 && S_avg <= steps, SUN_EINVAL, "need 1 <= S_avg <= steps");
    SUN_REQUIRE(ckpt_every >= 1, SUN_EINVAL, "ckpt_every must be >= 1");
    SUN_REQUIRE(J_out != nullptr, SUN_EINVAL, "J_out is NULL");
    hipStream_t s = as_stream(stream);
    const sun_prop_s& F = *a->fwd;
    const sun_prop_s& B = *a->bwd;
    const int64_t M = a->M, M1 = M + 1;
    const int64_t C = std::min(ckpt_every, steps);
    const int64_t nck = (steps + C - 1) / C;           // checkpoints at n = 0, C, 2C, ...
    Work w;
    w.ck.alloc(nck * M1);
    w.per.alloc((C + 1) * M1);
    hipLaunchKernelGGL(k_adj_fill_strided, dim3(grid_for(C + 1, 256)), dim3(256), 0, s, C + 1, M1, M, 1.0,
                       w.per.get());
    HIP_LAUNCH_OK();
    const bool keep_stages = 3.0 * (double)C * (double)M1 * 8.0 <= kStageStoreBytes;
    if (keep_stages) {
      w.stg.alloc(3 * C * M1);
      hipLaunchKernelGGL(k_adj_fill_strided, dim3(grid_for(3 * C, 256)), dim3(256), 0, s, 3 * C, M1, M, 1.0,
                         w.stg.get());
      HIP_LAUNCH_OK();
    }
    for (DevBuf<double>* b : {&w.x2, &w.x3, &w.x4, &w.acc, &w.lam, &w.lacc, &w.kb4, &w.kb3, &w.kb2, &w.kb1})
      b->alloc(M1);
    // per-thread running sums of the objective's dot products (nbj blocks of 256)
    const int nbj = dot_blocks(M);
    w.jrun.alloc((size_t)nbj * 256);
    hipLaunchKernelGGL(k_adj_fill, dim3(grid_for((int64_t)nbj * 256, 256)), dim3(256), 0, s, (int64_t)nbj * 256, 0.0,
                       w.jrun.get());
    w.cw.alloc(M1);
    w.zero.alloc(M1);
    hipLaunchKernelGGL(k_adj_scaled, dim3(grid_for(M1, 256)), dim3(256), 0, s, M, cobs, 1.0 / (double)S_avg,
                       w.cw.get());
    hipLaunchKernelGGL(k_adj_fill, dim3(grid_for(M1, 256)), dim3(256), 0, s, M1, 0.0, w.zero.get());
    w.dev_grad.alloc(kMaxTheta);
    w.dev_J.alloc(1);
    w.dstat.alloc(a->nt * (ntheta > 0 ? ntheta : 1));
    HIP_OK(hipMemsetAsync(w.dev_grad.get(), 0, kMaxTheta * sizeof(double), s));
    HIP_OK(hipMemsetAsync(w.dev_J.get(), 0, sizeof(double), s));
    if (ntheta > 0)
      HIP_OK(hipMemcpyAsync(w.dstat.get(), dstatic, a->nt * ntheta * sizeof(double), hipMemcpyHostToDevice, s));
    for (DevBuf<double>* b : {&w.x2, &w.x3, &w.x4, &w.lam, &w.lacc, &w.kb4, &w.kb3, &w.kb2, &w.kb1}) {
      hipLaunchKernelGGL(k_adj_fill, dim3(grid_for(M1, 256)), dim3(256), 0, s, M1, 0.0, b->get());
      hipLaunchKernelGGL(k_adj_fill, dim3(1), dim3(1), 0, s, (int64_t)1, 1.0, b->get() + M);
    }
    HIP_LAUNCH_OK();
    // ---- forward sweep with checkpoints --------------------------------------
    // Up to the last interval the state ping-pongs between the first two
    // interval slots; the last interval's states (and stage inputs) are
    // written where the backward sweep reads them, so it is not recomputed.
    const int64_t nlast = (nck - 1) * C;
    double* cur = w.per.get();
    double* nxt = w.per.get() + M1;
    HIP_OK(hipMemcpyAsync(cur, v0, M * sizeof(double), hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_adj_fill, dim3(1), dim3(1), 0, s, (int64_t)1, 1.0, cur + M);
    hipLaunchKernelGGL(k_adj_fill, dim3(1), dim3(1), 0, s, (int64_t)1, 1.0, nxt + M);
    for (int64_t n = 0; n < nlast; ++n) {
      if (n % C == 0) HIP_OK(hipMemcpyAsync(w.ck.get() + (n / C) * M1, cur, M1 * sizeof(double),
                                            hipMemcpyDeviceToDevice, s));
      forward_step(F, cur, nxt, w.x2.get(), w.x3.get(), w.x4.get(), w.acc.get(), coef, n, dt, s);
      std::swap(cur, nxt);
    }
    if (cur != w.per.get())
      HIP_OK(hipMemcpyAsync(w.per.get(), cur, M1 * sizeof(double), hipMemcpyDeviceToDevice, s));
    auto interval_states = [&](int64_t n0, int64_t n1) {
      double* P0 = w.per.get();
      for (int64_t n = n0; n < n1; ++n) {
        double* sx = keep_stages ? w.stg.get() + 3 * (n - n0) * M1 : nullptr;
        forward_step(F, P0 + (n - n0) * M1, P0 + (n + 1 - n0) * M1, sx ? sx : w.x2.get(),
                     sx ? sx + M1 : w.x3.get(), sx ? sx + 2 * M1 : w.x4.get(), w.acc.get(), coef, n, dt, s);
      }
    };
    interval_states(nlast, steps);
    // ---- parameter-dependent terms ---------------------------------------
    // The terms whose coefficient depends on a parameter.  Up to
    // kMaxRevSeg of them: the reverse stages run on a transposed generator
    // that keeps each of them as its own segment and form the dot products
    // kb . (T_j x + K_j) = (T_jᵀ kb) . x + kb . K_j in the same pass,
    // weighted by dc_j/dtheta, into per-wavefront slots gpart[th * ld + w].
    // More of them: each gets its own static propagator (unit weight, free
    // vector folded in) and one launch per step forms the products, into
    // slots gpart[(y * ntheta + th) * nslot + off_j + w].
    std::vector<int> used_terms;
    if (ntheta > 0) {
      std::vector<bool> used(a->nt, false);
      for (int d = 0; d < a->ndyn; ++d) used[a->dyn[d]] = true;
      for (int t = 0; t < a->nt; ++t)
        for (int th = 0; th < ntheta; ++th)
          if (dstatic[t * ntheta + th] != 0.0) used[t] = true;
      for (int t = 0; t < a->nt; ++t)
        if (used[t]) used_terms.push_back(t);
    }
    auto dyn_slot = [&](int t) {
      for (int d = 0; d < a->ndyn; ++d)
        if (a->dyn[d] == t) return d;
      return -1;
    };
    const bool fused = !used_terms.empty() && (int)used_terms.size() <= kMaxRevSeg;
    RevDot rd;
    struct GTerm { int term, slot; const sun_prop_s* p; int64_t off; };
    std::vector<GTerm> gterms;
    int64_t nslot = 0;
    if (fused) {
      if (!a->revg || a->revg_terms != used_terms) {
        if (a->revg) sun_prop_free(a->revg);
        a->revg = nullptr;
        std::vector<double> w0(a->static_w);
        for (int t : used_terms) w0[t] = 0.0;    // their weights enter as segment coefficients
        sun_prop q = nullptr;
        const int st = sun_prop_create(&a->lindT, w0.data(), used_terms.data(), (int)used_terms.size(), stream, &q);
        if (st != SUN_OK) SUN_THROW(st, std::string("segmented transposed propagator: ") + sun_last_error());
        try {
          prop_build_segments(*q, s);
        } catch (...) {
          sun_prop_free(q);
          throw;
        }
        a->revg = q;
        a->revg_terms = used_terms;
      }
      rd.nseg = (int)used_terms.size();
      for (int d = 0; d < rd.nseg; ++d) {
        const int t = used_terms[d];
        rd.wseg[d] = a->static_w[t];
        rd.slot[d] = dyn_slot(t);
        rd.term[d] = t;
        rd.K[d] = t >= a->lind->nH ? a->lind->K[t - a->lind->nH].get() : nullptr;
      }
      rd.coef = coef;
      rd.ncoef = a->ndyn;
      rd.dstat = w.dstat.get();
      rd.dcoef = dcoef;
      rd.ntheta = ntheta;
      rd.ld = prop_rev_slots(*a->revg);
      nslot = rd.ld;
    } else {
      if (a->termp.size() != (size_t)a->nt) a->termp.assign(a->nt, nullptr);
      for (int t : used_terms) {
        if (!a->termp[t]) {
          std::vector<double> unit(a->nt, 0.0);
          unit[t] = 1.0;
          sun_prop q = nullptr;
          int st = sun_prop_create(const_cast<sun_lind_s*>(a->lind), unit.data(), nullptr, 0, stream, &q);
          if (st != SUN_OK) SUN_THROW(st, std::string("term propagator: ") + sun_last_error());
          // the dot-product kernel reads the sliced layout (small terms start in the stream layout)
          if (q->layout != 1) {
            st = sun_prop_tune_sliced(q, 4096, 32, 1, 1, stream);
            if (st != SUN_OK) {
              sun_prop_free(q);
              SUN_THROW(st, std::string("term propagator layout: ") + sun_last_error());
            }
          }
          a->termp[t] = q;
        }
        gterms.push_back({t, dyn_slot(t), a->termp[t], nslot});
        nslot += prop_dot_slots(*a->termp[t]);
      }
    }
    const int ny = fused ? 1 : kDotStages / kDotStagesPerWave;
    w.gpart.alloc(std::max<int64_t>(1, ny * ntheta * nslot));
    if (ntheta * nslot > 0)
      hipLaunchKernelGGL(k_adj_fill, dim3(grid_for(ny * ntheta * nslot, 256)), dim3(256), 0, s, ny * ntheta * nslot,
                         0.0, w.gpart.get());
    rd.gpart = w.gpart.get();
    std::vector<const sun_prop_s*> gp;
    std::vector<int> gterm, gslot;
    std::vector<int64_t> goff;
    for (const GTerm& g : gterms) {
      gp.push_back(g.p);
      gterm.push_back(g.term);
      gslot.push_back(g.slot);
      goff.push_back(g.off);
    }
    // dot products of the four stages of step n, one launch per step
    auto grad_step = [&](const double* const* xs, const double* const* kbs, const int64_t* krows) {
      if (gp.empty()) return;
      prop_dot(gp.data(), gterm.data(), gslot.data(), goff.data(), (int)gp.size(), xs, kbs, krows, w.dstat.get(),
               dcoef, a->ndyn, ntheta, w.gpart.get(), nslot, s);
    };
    // ---- backward sweep -----------------------------------------------------
    const int64_t first_avg = steps - S_avg + 1;      // J averages v_n for n >= first_avg
    const double dt6 = dt / 6.0;
    double* lam = w.lam.get();
    double* lacc = w.lacc.get();
    for (int64_t ci = nck - 1; ci >= 0; --ci) {
      const int64_t n0 = ci * C, n1 = std::min(steps, n0 + C);
      // recompute the states v_{n0} .. v_{n1} of this interval (the last
      // one is still there from the forward sweep)
      double* P0 = w.per.get();
      if (ci < nck - 1) {
        HIP_OK(hipMemcpyAsync(P0, w.ck.get() + ci * M1, M1 * sizeof(double), hipMemcpyDeviceToDevice, s));
        interval_states(n0, n1);
      }
      // J: the states v_{n+1} of this interval inside the averaging window, in one launch
      const int64_t j0 = std::max(n0 + 1, first_avg);
      if (j0 <= n1)
        hipLaunchKernelGGL(k_dot_acc_states, dim3(nbj), dim3(256), 0, s, M, cobs, P0 + (j0 - n0) * M1, M1,
                           n1 - j0 + 1, w.jrun.get());
      for (int64_t n = n1 - 1; n >= n0; --n) {
        const double* vn = P0 + (n - n0) * M1;
        const bool in_avg = (n + 1) >= first_avg;
        // lambda += c/S (direct dependence of J on v_{n+1}); kb4 = dt/6 lambda.
        // After the first backward step the previous step's last stage
        // (stage 8) has done this already.
        if (n == steps - 1)
          hipLaunchKernelGGL(k_adj_prep, dim3(grid_for(M, 256)), dim3(256), 0, s, M, lam, cobs,
                             in_avg ? 1.0 / (double)S_avg : 0.0, dt6, w.kb4.get());
        // forward stage inputs of step n (kept from the interval recompute,
        // or recomputed here)
        const double *x2 = w.x2.get(), *x3 = w.x3.get(), *x4 = w.x4.get();
        if (keep_stages) {
          x2 = w.stg.get() + 3 * (n - n0) * M1;
          x3 = x2 + M1;
          x4 = x2 + 2 * M1;
        } else {
          prop_stage(F, 0, vn, vn, w.acc.get(), w.x2.get(), coef, 2 * n, dt, s);
          prop_stage(F, 1, w.x2.get(), vn, w.acc.get(), w.x3.get(), coef, 2 * n + 1, dt, s);
          prop_stage(F, 2, w.x3.get(), vn, w.acc.get(), w.x4.get(), coef, 2 * n + 1, dt, s);
        }
        if (fused) {
          // reverse stages with the dot products kb_i . (T_j x_i + K_j) fused in
          const sun_prop_s& G = *a->revg;
          prop_stage_dot(G, 4, w.kb4.get(), lam, lacc, w.kb3.get(), x4, rd, 2 * n + 2, dt, s);
          prop_stage_dot(G, 5, w.kb3.get(), lam, lacc, w.kb2.get(), x3, rd, 2 * n + 1, dt, s);
          prop_stage_dot(G, 6, w.kb2.get(), lam, lacc, w.kb1.get(), x2, rd, 2 * n + 1, dt, s);
          if (n > 0)
            prop_stage_dot(G, 8, w.kb1.get(), n >= first_avg ? w.cw.get() : w.zero.get(), lacc, w.kb4.get(), vn, rd,
                           2 * n, dt, s);
          else
            prop_stage_dot(G, 7, w.kb1.get(), lam, lacc, nullptr, vn, rd, 2 * n, dt, s);
          std::swap(lam, lacc);
          continue;
        }
        // stage 4: kb4 with x4 at t_{n+1}
        prop_stage(B, 4, w.kb4.get(), lam, lacc, w.kb3.get(), coef, 2 * n + 2, dt, s);
        prop_stage(B, 5, w.kb3.get(), lam, lacc, w.kb2.get(), coef, 2 * n + 1, dt, s);
        prop_stage(B, 6, w.kb2.get(), lam, lacc, w.kb1.get(), coef, 2 * n + 1, dt, s);
        // parameter terms: kb_i . (dT/dtheta x_i) for the stage inputs x4, x3, x2, v_n
        // (before the last stage, which overwrites kb4 with the next step's)
        const double* xs[4] = {x4, x3, x2, vn};
        const double* kbs[4] = {w.kb4.get(), w.kb3.get(), w.kb2.get(), w.kb1.get()};
        const int64_t krows[4] = {2 * n + 2, 2 * n + 1, 2 * n + 1, 2 * n};
        grad_step(xs, kbs, krows);
        if (n > 0) {
          // stage 7 and the next step's start: lambda_n += c/S if v_n is averaged
          const bool next_avg = n >= first_avg;
          prop_stage(B, 8, w.kb1.get(), next_avg ? w.cw.get() : w.zero.get(), lacc, w.kb4.get(), coef, 2 * n, dt,
                     s);
        } else {
          prop_stage(B, 7, w.kb1.get(), lam, lacc, nullptr, coef, 2 * n, dt, s);
        }
        std::swap(lam, lacc);
      }
    }
    // fixed-order reductions of the accumulated partials
    if (ntheta > 0 && nslot > 0)
      hipLaunchKernelGGL(k_sum_slots, dim3(ntheta), dim3(256), 0, s, w.gpart.get(), ny, ntheta, (int)nslot,
                         w.dev_grad.get());
    hipLaunchKernelGGL(k_dot_finish, dim3(1), dim3(256), 0, s, w.jrun.get(), nbj * 256, 1.0 / (double)S_avg,
                       w.dev_J.get());
    HIP_LAUNCH_OK();
    double hg[kMaxTheta];
    HIP_OK(hipMemcpyAsync(hg, w.dev_grad.get(), sizeof(hg), hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(J_out, w.dev_J.get(), sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if (grad_out)
      for (int th = 0; th < ntheta; ++th) grad_out[th] = hg[th];
  });
}

extern "C" int sun_adjoint_objective(sun_adj a, const double* v0, const double* coef, const double* cobs,
                                     double dt, int64_t steps, int64_t S_avg, double* J_out, void* stream) {
  return guarded([&] {
    SUN_REQUIRE(a != nullptr && v0 != nullptr && cobs != nullptr && J_out != nullptr, SUN_EINVAL, "NULL argument");
    SUN_REQUIRE(a->ndyn == 0 || coef != nullptr, SUN_EINVAL, "coef is NULL");
    SUN_REQUIRE(steps >= 1 && S_avg >= 1 && S_avg <= steps, SUN_EINVAL, "need 1 <= S_avg <= steps");
    hipStream_t s = as_stream(stream);
    const sun_prop_s& F = *a->fwd;
    const int64_t M = a->M, M1 = M + 1;
    DevBuf<double> v(M1), vn(M1), x2(M1), x3(M1), x4(M1), acc(M1), part(kDotBlocks), J(1);
    for (DevBuf<double>* b : {&v, &vn, &x2, &x3, &x4}) {
      hipLaunchKernelGGL(k_adj_fill, dim3(grid_for(M1, 256)), dim3(256), 0, s, M1, 0.0, b->get());
      hipLaunchKernelGGL(k_adj_fill, dim3(1), dim3(1), 0, s, (int64_t)1, 1.0, b->get() + M);
    }
    HIP_OK(hipMemsetAsync(J.get(), 0, sizeof(double), s));
    HIP_OK(hipMemcpyAsync(v.get(), v0, M * sizeof(double), hipMemcpyDeviceToDevice, s));
    double* cur = v.get();
    double* nxt = vn.get();
    for (int64_t n = 0; n < steps; ++n) {
      forward_step(F, cur, nxt, x2.get(), x3.get(), x4.get(), acc.get(), coef, n, dt, s);
      std::swap(cur, nxt);
      if (n + 1 >= steps - S_avg + 1) dot_accumulate(cobs, cur, M, 1.0 / (double)S_avg, part.get(), J.get(), s);
    }
    HIP_LAUNCH_OK();
    HIP_OK(hipMemcpyAsync(J_out, J.get(), sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
  });
}

extern "C" void sun_adjoint_free(sun_adj a) { delete a; }
