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
  std::vector<double> revg_w;   // the static weights revg was built with
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

// The parameter-dependent terms of a run and the dot-product layout they use.
struct TermSetup {
  std::vector<int> used;        // terms whose coefficient depends on a parameter
  bool fused = false;           // reverse stages with the dot products fused in (<= kMaxRevSeg terms)
  int64_t nslot = 0;            // per-wavefront slots of one parameter
  int ny = 1;                   // slot groups (the per-term path splits the stages over them)
};

int dyn_slot(const sun_adj_s& a, int t) {
  for (int d = 0; d < a.ndyn; ++d)
    if (a.dyn[d] == t) return d;
  return -1;
}

// Find the parameter-dependent terms and build (once, kept with the object)
// the layout their dot products need.  Up to kMaxRevSeg of them: the reverse
// stages run on a transposed generator that keeps each of them as its own
// segment and form kb . (T_j x + K_j) = (T_j^T kb) . x + kb . K_j in the same
// pass, weighted by dc_j/dtheta, into per-wavefront slots gpart[th * ld + w].
// More of them: each gets its own static propagator (unit weight, free
// vector folded in) and one launch per step forms the products, into slots
// gpart[(y * ntheta + th) * nslot + off_j + w].
TermSetup prepare_terms(sun_adj_s& a, const double* dstatic, int ntheta, void* stream) {
  hipStream_t s = as_stream(stream);
  TermSetup ts;
  if (ntheta > 0) {
    std::vector<bool> used(a.nt, false);
    for (int d = 0; d < a.ndyn; ++d) used[a.dyn[d]] = true;
    for (int t = 0; t < a.nt; ++t)
      for (int th = 0; th < ntheta; ++th)
        if (dstatic[t * ntheta + th] != 0.0) used[t] = true;
    for (int t = 0; t < a.nt; ++t)
      if (used[t]) ts.used.push_back(t);
  }
  ts.fused = !ts.used.empty() && (int)ts.used.size() <= kMaxRevSeg;
  if (ts.fused) {
    if (!a.revg || a.revg_terms != ts.used) {
      if (a.revg) sun_prop_free(a.revg);
      a.revg = nullptr;
      std::vector<double> w0(a.static_w);
      for (int t : ts.used) w0[t] = 0.0;    // their weights enter as segment coefficients
      sun_prop q = nullptr;
      const int st = sun_prop_create(&a.lindT, w0.data(), ts.used.data(), (int)ts.used.size(), stream, &q);
      if (st != SUN_OK) SUN_THROW(st, std::string("segmented transposed propagator: ") + sun_last_error());
      try {
        prop_build_segments(*q, s);
      } catch (...) {
        sun_prop_free(q);
        throw;
      }
      a.revg = q;
      a.revg_terms = ts.used;
      a.revg_w = w0;
    }
    ts.nslot = prop_rev_slots(*a.revg);
    ts.ny = 1;
  } else {
    if (a.termp.size() != (size_t)a.nt) a.termp.assign(a.nt, nullptr);
    for (int t : ts.used) {
      if (!a.termp[t]) {
        std::vector<double> unit(a.nt, 0.0);
        unit[t] = 1.0;
        sun_prop q = nullptr;
        int st = sun_prop_create(const_cast<sun_lind_s*>(a.lind), unit.data(), nullptr, 0, stream, &q);
        if (st != SUN_OK) SUN_THROW(st, std::string("term propagator: ") + sun_last_error());
        // the dot-product kernel reads the sliced layout (small terms start in the stream layout)
        if (q->layout != 1) {
          st = sun_prop_tune_sliced(q, 4096, 32, 1, 1, stream);
          if (st != SUN_OK) {
            sun_prop_free(q);
            SUN_THROW(st, std::string("term propagator layout: ") + sun_last_error());
          }
        }
        a.termp[t] = q;
      }
      ts.nslot += prop_dot_slots(*a.termp[t]);
    }
    ts.ny = kDotStages / kDotStagesPerWave;
    if (!ts.used.empty() && !a.bwd) {
      // the transposed generator with every term at its current weight
      const int st = sun_prop_create(&a.lindT, a.static_w.data(), a.dyn.data(), a.ndyn, stream, &a.bwd);
      if (st != SUN_OK) SUN_THROW(st, std::string("transposed propagator: ") + sun_last_error());
    }
  }
  if (ts.used.empty() && !a.bwd) {
    const int st = sun_prop_create(&a.lindT, a.static_w.data(), a.dyn.data(), a.ndyn, stream, &a.bwd);
    if (st != SUN_OK) SUN_THROW(st, std::string("transposed propagator: ") + sun_last_error());
  }
  return ts;
}

// Layout of the caller's workspace: regions of doubles, each starting on a
// 256-byte boundary.
struct WorkLayout {
  int64_t M1 = 0, C = 0, nck = 0;
  int nbj = 0;
  bool keep_stages = false;
  size_t off[32] = {};
  size_t len[32] = {};
  int n = 0;
  size_t bytes = 0;
  size_t add(size_t doubles) {
    const size_t o = bytes;
    off[n] = o;
    len[n] = doubles;
    ++n;
    bytes = o + ((doubles * sizeof(double) + 255) / 256) * 256;
    return o;
  }
};

enum { W_CK, W_PER, W_STG, W_X2, W_X3, W_X4, W_ACC, W_LAM, W_LACC, W_KB4, W_KB3, W_KB2, W_KB1, W_JRUN, W_CW,
       W_ZERO, W_GRAD, W_J, W_DSTAT, W_GPART, W_COUNT };

WorkLayout work_layout(const sun_adj_s& a, const TermSetup& ts, int ntheta, int64_t steps, int64_t ckpt_every,
                       bool keep_stages) {
  WorkLayout L;
  L.M1 = a.M + 1;
  L.C = std::min(ckpt_every, steps);
  L.nck = (steps + L.C - 1) / L.C;
  L.nbj = dot_blocks(a.M);
  L.keep_stages = keep_stages;
  L.add(L.nck * L.M1);                                  // W_CK: checkpoints
  L.add((L.C + 1) * L.M1);                              // W_PER: states of one interval
  L.add(keep_stages ? 3 * L.C * L.M1 : 0);              // W_STG: stage inputs of one interval
  for (int i = W_X2; i <= W_KB1; ++i) L.add(L.M1);      // stage and cotangent vectors
  L.add((size_t)L.nbj * 256);                           // W_JRUN: running sums of the objective
  L.add(L.M1);                                          // W_CW: c / S_avg
  L.add(L.M1);                                          // W_ZERO
  L.add(kMaxTheta);                                     // W_GRAD
  L.add(1);                                             // W_J
  L.add((size_t)a.nt * (ntheta > 0 ? ntheta : 1));      // W_DSTAT
  L.add(std::max<int64_t>(1, ts.ny * ntheta * ts.nslot));   // W_GPART
  return L;
}

bool stages_fit(const sun_adj_s& a, int64_t steps, int64_t ckpt_every) {
  const int64_t C = std::min(ckpt_every, steps);
  return 3.0 * (double)C * (double)(a.M + 1) * 8.0 <= kStageStoreBytes;
}

void check_run_args(const sun_adj_s* a, const double* v0, const double* coef, const double* dstatic, int ntheta,
                    const double* cobs, int64_t steps, int64_t S_avg, int64_t ckpt_every, const double* J_out) {
  SUN_REQUIRE(a != nullptr && v0 != nullptr && cobs != nullptr, SUN_EINVAL, "NULL argument");
  SUN_REQUIRE(ntheta >= 0 && ntheta <= kMaxTheta, SUN_ENOTSUP, "at most 8 parameters");
  SUN_REQUIRE(ntheta == 0 || dstatic != nullptr, SUN_EINVAL, "dstatic is NULL");
  SUN_REQUIRE(a->ndyn == 0 || coef != nullptr, SUN_EINVAL, "coef is NULL");
  SUN_REQUIRE(steps >= 1 && S_avg >= 1 && S_avg <= steps, SUN_EINVAL, "need 1 <= S_avg <= steps");
  SUN_REQUIRE(ckpt_every >= 1, SUN_EINVAL, "ckpt_every must be >= 1");
  SUN_REQUIRE(J_out != nullptr, SUN_EINVAL, "J_out is NULL");
}

// The adjoint run on a workspace laid out by work_layout.
void adjoint_execute(sun_adj_s* a, const TermSetup& ts, const WorkLayout& L, unsigned char* ws, const double* v0,
                     const double* coef, const double* dstatic, const double* dcoef, int32_t ntheta,
                     const double* cobs, double dt, int64_t steps, int64_t S_avg, double* J_out, double* grad_out,
                     hipStream_t s) {
  auto W = [&](int i) { return reinterpret_cast<double*>(ws + L.off[i]); };
  const sun_prop_s& F = *a->fwd;
  prop_require_usable(F);
  const int64_t M = a->M, M1 = L.M1, C = L.C, nck = L.nck;
  const bool keep_stages = L.keep_stages;
  const int nbj = L.nbj;
  double* per = W(W_PER);
  double* stg = W(W_STG);
  double *x2b = W(W_X2), *x3b = W(W_X3), *x4b = W(W_X4), *accb = W(W_ACC);
  double *kb4 = W(W_KB4), *kb3 = W(W_KB3), *kb2 = W(W_KB2), *kb1 = W(W_KB1);
  double* jrun = W(W_JRUN);
  double* cw = W(W_CW);
  double* zero = W(W_ZERO);
  double* dev_grad = W(W_GRAD);
  double* dev_J = W(W_J);
  double* dstat = W(W_DSTAT);
  double* gpart = W(W_GPART);
  hipLaunchKernelGGL(k_adj_fill_strided, dim3(grid_for(C + 1, 256)), dim3(256), 0, s, C + 1, M1, M, 1.0, per);
  HIP_LAUNCH_OK();
  if (keep_stages) {
    hipLaunchKernelGGL(k_adj_fill_strided, dim3(grid_for(3 * C, 256)), dim3(256), 0, s, 3 * C, M1, M, 1.0, stg);
    HIP_LAUNCH_OK();
  }
  // per-thread running sums of the objective's dot products (nbj blocks of 256)
  hipLaunchKernelGGL(k_adj_fill, dim3(grid_for((int64_t)nbj * 256, 256)), dim3(256), 0, s, (int64_t)nbj * 256, 0.0,
                     jrun);
  hipLaunchKernelGGL(k_adj_scaled, dim3(grid_for(M1, 256)), dim3(256), 0, s, M, cobs, 1.0 / (double)S_avg, cw);
  hipLaunchKernelGGL(k_adj_fill, dim3(grid_for(M1, 256)), dim3(256), 0, s, M1, 0.0, zero);
  hipLaunchKernelGGL(k_adj_fill, dim3(1), dim3(256), 0, s, (int64_t)kMaxTheta, 0.0, dev_grad);
  hipLaunchKernelGGL(k_adj_fill, dim3(1), dim3(1), 0, s, (int64_t)1, 0.0, dev_J);
  if (ntheta > 0)
    HIP_OK(hipMemcpyAsync(dstat, dstatic, a->nt * ntheta * sizeof(double), hipMemcpyHostToDevice, s));
  for (int i = W_X2; i <= W_KB1; ++i) {
    if (i == W_ACC) continue;
    hipLaunchKernelGGL(k_adj_fill, dim3(grid_for(M1, 256)), dim3(256), 0, s, M1, 0.0, W(i));
    hipLaunchKernelGGL(k_adj_fill, dim3(1), dim3(1), 0, s, (int64_t)1, 1.0, W(i) + M);
  }
  HIP_LAUNCH_OK();
  // ---- forward sweep with checkpoints --------------------------------------
  // Up to the last interval the state ping-pongs between the first two
  // interval slots; the last interval's states (and stage inputs) are
  // written where the backward sweep reads them, so it is not recomputed.
  const int64_t nlast = (nck - 1) * C;
  double* cur = per;
  double* nxt = per + M1;
  HIP_OK(hipMemcpyAsync(cur, v0, M * sizeof(double), hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(k_adj_fill, dim3(1), dim3(1), 0, s, (int64_t)1, 1.0, cur + M);
  hipLaunchKernelGGL(k_adj_fill, dim3(1), dim3(1), 0, s, (int64_t)1, 1.0, nxt + M);
  for (int64_t n = 0; n < nlast; ++n) {
    if (n % C == 0) HIP_OK(hipMemcpyAsync(W(W_CK) + (n / C) * M1, cur, M1 * sizeof(double),
                                          hipMemcpyDeviceToDevice, s));
    forward_step(F, cur, nxt, x2b, x3b, x4b, accb, coef, n, dt, s);
    std::swap(cur, nxt);
  }
  if (cur != per) HIP_OK(hipMemcpyAsync(per, cur, M1 * sizeof(double), hipMemcpyDeviceToDevice, s));
  auto interval_states = [&](int64_t n0, int64_t n1) {
    for (int64_t n = n0; n < n1; ++n) {
      double* sx = keep_stages ? stg + 3 * (n - n0) * M1 : nullptr;
      forward_step(F, per + (n - n0) * M1, per + (n + 1 - n0) * M1, sx ? sx : x2b, sx ? sx + M1 : x3b,
                   sx ? sx + 2 * M1 : x4b, accb, coef, n, dt, s);
    }
  };
  interval_states(nlast, steps);
  // ---- parameter-dependent terms ---------------------------------------
  RevDot rd;
  struct GTerm { int term, slot; const sun_prop_s* p; int64_t off; };
  std::vector<GTerm> gterms;
  const int64_t nslot = ts.nslot;
  if (ts.fused) {
    prop_require_usable(*a->revg);
    rd.nseg = (int)ts.used.size();
    for (int d = 0; d < rd.nseg; ++d) {
      const int t = ts.used[d];
      rd.wseg[d] = a->static_w[t];
      rd.slot[d] = dyn_slot(*a, t);
      rd.term[d] = t;
      rd.K[d] = t >= a->lind->nH ? a->lind->K[t - a->lind->nH].get() : nullptr;
    }
    rd.coef = coef;
    rd.ncoef = a->ndyn;
    rd.dstat = dstat;
    rd.dcoef = dcoef;
    rd.ntheta = ntheta;
    rd.ld = nslot;
  } else {
    int64_t off = 0;
    for (int t : ts.used) {
      gterms.push_back({t, dyn_slot(*a, t), a->termp[t], off});
      off += prop_dot_slots(*a->termp[t]);
    }
  }
  const int ny = ts.ny;
  if (ntheta * nslot > 0)
    hipLaunchKernelGGL(k_adj_fill, dim3(grid_for(ny * ntheta * nslot, 256)), dim3(256), 0, s, ny * ntheta * nslot,
                       0.0, gpart);
  rd.gpart = gpart;
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
    prop_dot(gp.data(), gterm.data(), gslot.data(), goff.data(), (int)gp.size(), xs, kbs, krows, dstat, dcoef,
             a->ndyn, ntheta, gpart, nslot, s);
  };
  const sun_prop_s* Bp = ts.fused ? nullptr : a->bwd;
  if (Bp) prop_require_usable(*Bp);
  // ---- backward sweep -----------------------------------------------------
  const int64_t first_avg = steps - S_avg + 1;      // J averages v_n for n >= first_avg
  const double dt6 = dt / 6.0;
  double* lam = W(W_LAM);
  double* lacc = W(W_LACC);
  for (int64_t ci = nck - 1; ci >= 0; --ci) {
    const int64_t n0 = ci * C, n1 = std::min(steps, n0 + C);
    // recompute the states v_{n0} .. v_{n1} of this interval (the last
    // one is still there from the forward sweep)
    if (ci < nck - 1) {
      HIP_OK(hipMemcpyAsync(per, W(W_CK) + ci * M1, M1 * sizeof(double), hipMemcpyDeviceToDevice, s));
      interval_states(n0, n1);
    }
    // J: the states v_{n+1} of this interval inside the averaging window, in one launch
    const int64_t j0 = std::max(n0 + 1, first_avg);
    if (j0 <= n1)
      hipLaunchKernelGGL(k_dot_acc_states, dim3(nbj), dim3(256), 0, s, M, cobs, per + (j0 - n0) * M1, M1,
                         n1 - j0 + 1, jrun);
    for (int64_t n = n1 - 1; n >= n0; --n) {
      const double* vn = per + (n - n0) * M1;
      const bool in_avg = (n + 1) >= first_avg;
      // lambda += c/S (direct dependence of J on v_{n+1}); kb4 = dt/6 lambda.
      // After the first backward step the previous step's last stage
      // (stage 8) has done this already.
      if (n == steps - 1)
        hipLaunchKernelGGL(k_adj_prep, dim3(grid_for(M, 256)), dim3(256), 0, s, M, lam, cobs,
                           in_avg ? 1.0 / (double)S_avg : 0.0, dt6, kb4);
      // forward stage inputs of step n (kept from the interval recompute,
      // or recomputed here)
      const double *x2 = x2b, *x3 = x3b, *x4 = x4b;
      if (keep_stages) {
        x2 = stg + 3 * (n - n0) * M1;
        x3 = x2 + M1;
        x4 = x2 + 2 * M1;
      } else {
        prop_stage(F, 0, vn, vn, accb, x2b, coef, 2 * n, dt, s);
        prop_stage(F, 1, x2b, vn, accb, x3b, coef, 2 * n + 1, dt, s);
        prop_stage(F, 2, x3b, vn, accb, x4b, coef, 2 * n + 1, dt, s);
      }
      if (ts.fused) {
        // reverse stages with the dot products kb_i . (T_j x_i + K_j) fused in
        const sun_prop_s& G = *a->revg;
        prop_stage_dot(G, 4, kb4, lam, lacc, kb3, x4, rd, 2 * n + 2, dt, s);
        prop_stage_dot(G, 5, kb3, lam, lacc, kb2, x3, rd, 2 * n + 1, dt, s);
        prop_stage_dot(G, 6, kb2, lam, lacc, kb1, x2, rd, 2 * n + 1, dt, s);
        if (n > 0)
          prop_stage_dot(G, 8, kb1, n >= first_avg ? cw : zero, lacc, kb4, vn, rd, 2 * n, dt, s);
        else
          prop_stage_dot(G, 7, kb1, lam, lacc, nullptr, vn, rd, 2 * n, dt, s);
        std::swap(lam, lacc);
        continue;
      }
      // stage 4: kb4 with x4 at t_{n+1}
      prop_stage(*Bp, 4, kb4, lam, lacc, kb3, coef, 2 * n + 2, dt, s);
      prop_stage(*Bp, 5, kb3, lam, lacc, kb2, coef, 2 * n + 1, dt, s);
      prop_stage(*Bp, 6, kb2, lam, lacc, kb1, coef, 2 * n + 1, dt, s);
      // parameter terms: kb_i . (dT/dtheta x_i) for the stage inputs x4, x3, x2, v_n
      // (before the last stage, which overwrites kb4 with the next step's)
      const double* xs[4] = {x4, x3, x2, vn};
      const double* kbs[4] = {kb4, kb3, kb2, kb1};
      const int64_t krows[4] = {2 * n + 2, 2 * n + 1, 2 * n + 1, 2 * n};
      grad_step(xs, kbs, krows);
      if (n > 0) {
        // stage 7 and the next step's start: lambda_n += c/S if v_n is averaged
        const bool next_avg = n >= first_avg;
        prop_stage(*Bp, 8, kb1, next_avg ? cw : zero, lacc, kb4, coef, 2 * n, dt, s);
      } else {
        prop_stage(*Bp, 7, kb1, lam, lacc, nullptr, coef, 2 * n, dt, s);
      }
      std::swap(lam, lacc);
    }
  }
  // fixed-order reductions of the accumulated partials
  if (ntheta > 0 && nslot > 0)
    hipLaunchKernelGGL(k_sum_slots, dim3(ntheta), dim3(256), 0, s, gpart, ny, ntheta, (int)nslot, dev_grad);
  hipLaunchKernelGGL(k_dot_finish, dim3(1), dim3(256), 0, s, jrun, nbj * 256, 1.0 / (double)S_avg, dev_J);
  HIP_LAUNCH_OK();
  double hg[kMaxTheta];
  HIP_OK(hipMemcpyAsync(hg, dev_grad, sizeof(hg), hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(J_out, dev_J, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  if (grad_out)
    for (int th = 0; th < ntheta; ++th) grad_out[th] = hg[th];
  bool finite = std::isfinite(*J_out);
  for (int th = 0; th < ntheta; ++th) finite = finite && std::isfinite(hg[th]);
  SUN_REQUIRE(finite, SUN_EDIVERGED, "J or its gradient is not finite (the states diverged)");
}

}  // namespace

extern "C" int sun_adjoint_plan(sun_adj a, const double* dstatic, int32_t ntheta, int64_t steps, int64_t ckpt_every,
                                void* stream, size_t* workspace_bytes, size_t* min_workspace_bytes) {
  return guarded([&] {
    SUN_REQUIRE(a != nullptr && workspace_bytes != nullptr, SUN_EINVAL, "NULL argument");
    SUN_REQUIRE(ntheta >= 0 && ntheta <= kMaxTheta, SUN_ENOTSUP, "at most 8 parameters");
    SUN_REQUIRE(ntheta == 0 || dstatic != nullptr, SUN_EINVAL, "dstatic is NULL");
    SUN_REQUIRE(steps >= 1 && ckpt_every >= 1, SUN_EINVAL, "need steps >= 1 and ckpt_every >= 1");
    const TermSetup ts = prepare_terms(*a, dstatic, ntheta, stream);
    const bool keep = stages_fit(*a, steps, ckpt_every);
    *workspace_bytes = work_layout(*a, ts, ntheta, steps, ckpt_every, keep).bytes;
    if (min_workspace_bytes) *min_workspace_bytes = work_layout(*a, ts, ntheta, steps, ckpt_every, false).bytes;
  });
}

extern "C" int sun_adjoint_execute(sun_adj a, const double* v0, const double* coef, const double* dstatic,
                                   const double* dcoef, int32_t ntheta, const double* cobs, double dt, int64_t steps,
                                   int64_t S_avg, int64_t ckpt_every, void* workspace, size_t workspace_bytes,
                                   double* J_out, double* grad_out, void* stream) {
  return guarded([&] {
    check_run_args(a, v0, coef, dstatic, ntheta, cobs, steps, S_avg, ckpt_every, J_out);
    SUN_REQUIRE(workspace != nullptr, SUN_EINVAL, "workspace is NULL");
    SUN_REQUIRE(reinterpret_cast<uintptr_t>(workspace) % 256 == 0, SUN_EINVAL, "workspace must be 256-byte aligned");
    const TermSetup ts = prepare_terms(*a, dstatic, ntheta, stream);
    const WorkLayout full = work_layout(*a, ts, ntheta, steps, ckpt_every, stages_fit(*a, steps, ckpt_every));
    const WorkLayout lean = work_layout(*a, ts, ntheta, steps, ckpt_every, false);
    SUN_REQUIRE(workspace_bytes >= lean.bytes, SUN_ERANGE,
                "workspace too small: " + std::to_string(workspace_bytes) + " < " + std::to_string(lean.bytes) +
                    " bytes (sun_adjoint_plan)");
    const WorkLayout& L = workspace_bytes >= full.bytes ? full : lean;
    adjoint_execute(a, ts, L, static_cast<unsigned char*>(workspace), v0, coef, dstatic, dcoef, ntheta, cobs, dt,
                    steps, S_avg, J_out, grad_out, as_stream(stream));
  });
}

extern "C" int sun_adjoint_run(sun_adj a, const double* v0, const double* coef, const double* dstatic,
                               const double* dcoef, int32_t ntheta, const double* cobs, double dt, int64_t steps,
                               int64_t S_avg, int64_t ckpt_every, double* J_out, double* grad_out, void* stream) {
  return guarded([&] {
    check_run_args(a, v0, coef, dstatic, ntheta, cobs, steps, S_avg, ckpt_every, J_out);
    const TermSetup ts = prepare_terms(*a, dstatic, ntheta, stream);
    const WorkLayout L = work_layout(*a, ts, ntheta, steps, ckpt_every, stages_fit(*a, steps, ckpt_every));
    DevBuf<unsigned char> ws(L.bytes);
    adjoint_execute(a, ts, L, ws.get(), v0, coef, dstatic, dcoef, ntheta, cobs, dt, steps, S_avg, J_out, grad_out,
                    as_stream(stream));
  });
}

extern "C" int sun_adjoint_set_weights(sun_adj a, const double* static_w, void* stream) {
  return guarded([&] {
    SUN_REQUIRE(a != nullptr && static_w != nullptr, SUN_EINVAL, "NULL argument");
    for (int t = a->lind->nH; t < a->nt; ++t)
      SUN_REQUIRE(static_w[t] >= 0.0, SUN_EINVAL, "dissipation rates must be >= 0");
    std::vector<double> w(static_w, static_w + a->nt);
    if (w == a->static_w) return;
    sun_prop f = nullptr;
    const int st = sun_prop_create(const_cast<sun_lind_s*>(a->lind), w.data(), a->dyn.data(), a->ndyn, stream, &f);
    if (st != SUN_OK) SUN_THROW(st, std::string("forward propagator: ") + sun_last_error());
    sun_prop_free(a->fwd);
    a->fwd = f;
    if (a->bwd) {
      sun_prop_free(a->bwd);
      a->bwd = nullptr;    // rebuilt on demand with the new weights
    }
    // the segmented reverse generator has the weights of the terms that are
    // not its segments merged in; it stays valid while those are unchanged
    if (a->revg) {
      bool same = true;
      for (int t = 0; t < a->nt; ++t)
        if (std::find(a->revg_terms.begin(), a->revg_terms.end(), t) == a->revg_terms.end() && w[t] != a->revg_w[t])
          same = false;
      if (!same) {
        sun_prop_free(a->revg);
        a->revg = nullptr;
        a->revg_terms.clear();
      }
    }
    a->static_w = w;
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
