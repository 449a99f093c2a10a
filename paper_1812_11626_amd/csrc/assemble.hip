// Expansion of operators over the SU(N) basis (Sec. IV step 2.1) and
// assembly of the Bloch-form generator (Sec. II eqs. 6, 10, 11; Sec. IV
// steps 2.3-2.5) by contracting the closed-form structure constants with the
// expansion coefficients, row by row, on the GPU.
//
// Contraction primitive.  For a coefficient vector x (expansion of an
// operator X) and complex weights (wf, wd):
//     C[s][n] = sum_m x_m (wf f_smn + wd d_smn).
// With the total (anti)symmetry of f and d this gives every matrix of the
// method:
//     Q_H  = C(h;  1, 0)                      (eq. 6, q_sn = sum_m f_mns h_m)
//     B^T  = C(conj l; 1, 0)                  (B_ls = sum_k conj(l_k) f_kls)
//     A    = C(l; -1, i)                      (A_lm = sum_j l_j z_jlm, z = f + i d)
//     R    = -(1/2) Re(B^T A),  K = (1/N) Im(B^T l)     (eqs. 10, 11)
// Row s of C is built from the operator's sparsity pattern: for an
// off-diagonal s = (j,k) the nonzero m are edges (j,l), (k,l) adjacent to s
// (triangles), the same edge (then n is diagonal), or diagonal generators,
// whose contributions collapse to sum_l x_{D_l} D_l[i] at i = j, k.  For a
// diagonal s = D^l the m are pattern edges (j,k) with j <= l, and (for d)
// the diagonal generators.
// Generators run twice (count, then fill) and must take identical
// floating-point decisions in both passes: no contraction into FMAs.
#pragma clang fp contract(off)

#include <cmath>

#include "internal.hpp"
#include "rowpipe.hpp"

using namespace sun;

namespace {

constexpr double kInvSqrt2 = 0.70710678118654752440;

// ---------------------------------------------------------------------------
// Expansion kernels
// ---------------------------------------------------------------------------
__global__ void k_validate_csr(int n, int nnz, const int* __restrict__ rowptr,
                               const int* __restrict__ col, int* __restrict__ bad) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
    int a = rowptr[r], b = rowptr[r + 1];
    if (r == 0 && a != 0) atomicOr(bad, 1);
    if (r == n - 1 && b != nnz) atomicOr(bad, 1);
    if (b < a) { atomicOr(bad, 1); continue; }
    for (int e = a; e < b; ++e) {
      int c = col[e];
      if (c < 0 || c >= n || (e > a && c <= col[e - 1])) atomicOr(bad, 2);
    }
  }
}

__device__ inline void atomic_max_pos(double* addr, double v) {
  // non-negative doubles order like their bit patterns
  atomicMax(reinterpret_cast<unsigned long long*>(addr), __double_as_longlong(v));
}

__global__ void k_expand_offdiag(BasisDev B, const int* __restrict__ rowptr, const int* __restrict__ col,
                                 const double* __restrict__ re, const double* __restrict__ im,
                                 cplx* __restrict__ x, cplx* __restrict__ diag, double* __restrict__ maxabs) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < B.N; r += gridDim.x * blockDim.x) {
    double m = 0.0;
    for (int e = rowptr[r]; e < rowptr[r + 1]; ++e) {
      const int c = col[e];
      const double vr = re[e], vi = im ? im[e] : 0.0;
      m = fmax(m, fmax(fabs(vr), fabs(vi)));
      if (c == r) {
        diag[r] = cx(vr, vi);
        continue;
      }
      const int p = pair_index(B.N, r, c);
      // S: (X_jk + X_kj)/sqrt2 ; J: i (X_jk - X_kj)/sqrt2, X_jk with j < k
      atomicAdd(&x[p].re, vr * kInvSqrt2);
      atomicAdd(&x[p].im, vi * kInvSqrt2);
      const double sg = (r < c) ? 1.0 : -1.0;   // +i for X_jk, -i for X_kj
      atomicAdd(&x[B.P + p].re, -sg * vi * kInvSqrt2);
      atomicAdd(&x[B.P + p].im, sg * vr * kInvSqrt2);
    }
    atomic_max_pos(maxabs, m);
  }
}

// Diagonal generators: x_{D_l} = c_l (sum_{i<l} X_ii - l X_ll); the trace;
// and xd[i] = sum_l x_{D_l} D_l[i] (suffix sums).  One thread, O(N).
__global__ void k_expand_diag(BasisDev B, const cplx* __restrict__ diag, cplx* __restrict__ x,
                              cplx* __restrict__ xd, cplx* __restrict__ trace) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  cplx pre = cx(0.0);
  for (int l = 1; l < B.N; ++l) {
    pre = pre + diag[l - 1];
    cplx d = (-(double)l) * diag[l];
    x[2 * B.P + l - 1] = B.c[l] * (pre + d);
  }
  *trace = pre + diag[B.N - 1];
  cplx suf = cx(0.0);   // sum_{l > i} x_{D_l} c_l
  for (int i = B.N - 1; i >= 0; --i) {
    cplx own = (i >= 1) ? (-(double)i * B.c[i]) * x[2 * B.P + i - 1] : cx(0.0);
    xd[i] = suf + own;
    if (i >= 1) suf = suf + B.c[i] * x[2 * B.P + i - 1];
  }
}

// max |X_ij - conj(X_ji)|
__global__ void k_hermiticity(int n, const int* __restrict__ rowptr, const int* __restrict__ col,
                              const double* __restrict__ re, const double* __restrict__ im,
                              double* __restrict__ dev) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
    double m = 0.0;
    for (int e = rowptr[r]; e < rowptr[r + 1]; ++e) {
      const int c = col[e];
      double tr = 0.0, ti = 0.0;   // X_cr
      int lo = rowptr[c], hi = rowptr[c + 1] - 1;
      while (lo <= hi) {
        int mid = (lo + hi) >> 1;
        int cc = col[mid];
        if (cc == r) { tr = re[mid]; ti = im ? im[mid] : 0.0; break; }
        if (cc < r) lo = mid + 1; else hi = mid - 1;
      }
      const double vi = im ? im[e] : 0.0;
      m = fmax(m, fmax(fabs(re[e] - tr), fabs(vi + ti)));
    }
    atomic_max_pos(dev, m);
  }
}

// Symmetric off-diagonal adjacency: raw degrees, fill, per-row sort + unique.
__global__ void k_adj_count(int n, const int* __restrict__ rowptr, const int* __restrict__ col,
                            int64_t* __restrict__ deg) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
    for (int e = rowptr[r]; e < rowptr[r + 1]; ++e) {
      int c = col[e];
      if (c == r) continue;
      atomicAdd(reinterpret_cast<unsigned long long*>(&deg[r]), 1ull);
      atomicAdd(reinterpret_cast<unsigned long long*>(&deg[c]), 1ull);
    }
  }
}

__global__ void k_adj_fill(int n, const int* __restrict__ rowptr, const int* __restrict__ col,
                           const int64_t* __restrict__ off, int* __restrict__ slot, int* __restrict__ raw) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
    for (int e = rowptr[r]; e < rowptr[r + 1]; ++e) {
      int c = col[e];
      if (c == r) continue;
      int a = atomicAdd(&slot[r], 1);
      raw[off[r] + a] = c;
      int b = atomicAdd(&slot[c], 1);
      raw[off[c] + b] = r;
    }
  }
}

__global__ void k_adj_sort_unique(int n, const int64_t* __restrict__ off, const int64_t* __restrict__ deg,
                                  int* __restrict__ raw, int64_t* __restrict__ ucnt) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
    int* a = raw + off[r];
    int m = (int)deg[r];
    for (int i = 1; i < m; ++i) {   // insertion sort (rows are short)
      int v = a[i], j = i - 1;
      while (j >= 0 && a[j] > v) { a[j + 1] = a[j]; --j; }
      a[j + 1] = v;
    }
    int u = 0;
    for (int i = 0; i < m; ++i)
      if (i == 0 || a[i] != a[i - 1]) a[u++] = a[i];
    ucnt[r] = u;
  }
}

__global__ void k_adj_compact(int n, const int64_t* __restrict__ off, const int* __restrict__ raw,
                              const int64_t* __restrict__ uoff, const int64_t* __restrict__ ucnt,
                              int total, int* __restrict__ ptr, int* __restrict__ idx) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
    ptr[r] = (int)uoff[r];
    for (int i = 0; i < ucnt[r]; ++i) idx[uoff[r] + i] = raw[off[r] + i];
    if (r == n - 1) ptr[n] = total;
  }
}

__global__ void k_conj(int64_t n, const cplx* __restrict__ a, cplx* __restrict__ b) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    b[i] = conj(a[i]);
}

// ---------------------------------------------------------------------------
// Contraction row generator
// ---------------------------------------------------------------------------
template <class V>
__device__ inline V take(cplx v);
template <>
__device__ inline cplx take<cplx>(cplx v) { return v; }
template <>
__device__ inline double take<double>(cplx v) { return v.re; }

template <class V>
struct ContractGen {
  BasisDev B;
  const cplx* x;
  const cplx* xd;
  const int* adj_ptr;
  const int* adj_idx;
  cplx wf, wd;
  int want_d;

  __device__ bool has_edge(int j, int k) const {
    int lo = adj_ptr[j], hi = adj_ptr[j + 1] - 1;
    while (lo <= hi) {
      int mid = (lo + hi) >> 1;
      int c = adj_idx[mid];
      if (c == k) return true;
      if (c < k) lo = mid + 1; else hi = mid - 1;
    }
    return false;
  }

  template <class E>
  __device__ void put(E& emit, int n, cplx xm, cplx t) const {
    cplx tv = (2.0 * t.im) * wf + (2.0 * t.re) * wd;
    if (is_zero(tv)) return;
    cplx v = xm * tv;
    V out = take<V>(v);
    if (is_zero(out)) return;
    emit((uint64_t)n, out);
  }

  template <class E>
  __device__ void run(int s, E& emit) const {
    const Gen gs = decode(B, s);
    const int N = B.N, P = B.P;
    if (gs.kind != KD) {
      const int j = gs.j, k = gs.k;
      // (1) triangles: m on edge (u,l), n on edge (l,w), {u,w} = {j,k}
      for (int side = 0; side < 2; ++side) {
        const int u = side ? k : j;
        const int w = side ? j : k;
        for (int e = adj_ptr[u]; e < adj_ptr[u + 1]; ++e) {
          const int l = adj_idx[e];
          if (l == j || l == k) continue;
          const int pm = pair_index(N, u, l), pn = pair_index(N, l, w);
          for (int tm = 0; tm < 2; ++tm) {
            const cplx xm = x[tm * P + pm];
            if (is_zero(xm)) continue;
            const Gen gm{tm, min(u, l), max(u, l)};
            for (int tn = 0; tn < 2; ++tn) {
              const Gen gn{tn, min(l, w), max(l, w)};
              put(emit, tn * P + pn, xm, trace3(B, gs, gm, gn));
            }
          }
        }
      }
      // (2) m on the same edge, n = D^l
      if (has_edge(j, k)) {
        const int pe = pair_index(N, j, k);
        const int lhi = want_d ? N - 1 : k;
        for (int tm = 0; tm < 2; ++tm) {
          const cplx xm = x[tm * P + pe];
          if (is_zero(xm)) continue;
          const Gen gm{tm, j, k};
          for (int l = max(j, 1); l <= lhi; ++l) {
            const Gen gn{KD, l, l};
            put(emit, encode_diag(B, l), xm, trace3(B, gs, gm, gn));
          }
        }
      }
      // (3) m diagonal: sum_l x_{D_l} T(s, D_l, n) for n on the same edge,
      //     T(s, D_l, n) = T(n, s, D_l) = n_jk s_kj D_l[j] + n_kj s_jk D_l[k]
      for (int tn = 0; tn < 2; ++tn) {
        const cplx Tj = pentry(tn, j, k) * pentry(gs.kind, k, j);
        const cplx Tk = pentry(tn, k, j) * pentry(gs.kind, j, k);
        const cplx v = wf * ((2.0 * Tj.im) * xd[j] + (2.0 * Tk.im) * xd[k]) +
                       wd * ((2.0 * Tj.re) * xd[j] + (2.0 * Tk.re) * xd[k]);
        V out = take<V>(v);
        if (!is_zero(out)) emit((uint64_t)(tn * P + pair_index(N, j, k)), out);
      }
    } else {
      const int l = gs.j;
      // (1) m, n on the same pattern edge (j,k) with j <= l (<= k for f)
      for (int j = 0; j <= l; ++j) {
        for (int e = adj_ptr[j]; e < adj_ptr[j + 1]; ++e) {
          const int k = adj_idx[e];
          if (k <= j) continue;
          if (!want_d && k < l) continue;
          const int pe = pair_index(N, j, k);
          for (int tm = 0; tm < 2; ++tm) {
            const cplx xm = x[tm * P + pe];
            if (is_zero(xm)) continue;
            const Gen gm{tm, j, k};
            for (int tn = 0; tn < 2; ++tn) {
              const Gen gn{tn, j, k};
              put(emit, tn * P + pe, xm, trace3(B, gs, gm, gn));
            }
          }
        }
      }
      // (2) m diagonal (d only): n = D^b for the nonzero diagonal triples
      if (want_d) {
        for (int a = 1; a < N; ++a) {
          const cplx xm = x[2 * P + a - 1];
          if (is_zero(xm)) continue;
          if (a == l) {
            for (int b = l; b < N; ++b) put(emit, encode_diag(B, b), xm, cx(trace_ddd(B, l, a, b)));
          } else if (a < l) {
            put(emit, encode_diag(B, a), xm, cx(trace_ddd(B, l, a, a)));
          } else {
            put(emit, encode_diag(B, l), xm, cx(trace_ddd(B, l, a, l)));
          }
        }
      }
    }
  }
};

// R = -(1/2) Re(B^T A): row s collects products of row s of B^T with rows of A.
struct SpgemmGen {
  const int* bptr;
  const int* bcol;
  const cplx* bval;
  const int* aptr;
  const int* acol;
  const cplx* aval;
  template <class E>
  __device__ void run(int s, E& emit) const {
    for (int e = bptr[s]; e < bptr[s + 1]; ++e) {
      const int l = bcol[e];
      const cplx bv = bval[e];
      for (int f = aptr[l]; f < aptr[l + 1]; ++f) {
        const cplx av = aval[f];
        const double v = -0.5 * (bv.re * av.re - bv.im * av.im);
        if (v != 0.0) emit((uint64_t)acol[f], v);
      }
    }
  }
};

// Rows of R = -(1/2) Re(B^T A) followed by the entries of the same row of an
// extra real matrix E (the gauge term of a dissipator with a trace); the row
// pipeline merges equal columns in a fixed order.
struct SpgemmPlusGen {
  SpgemmGen g;
  const int* eptr;
  const int* ecol;
  const double* eval;
  template <class E>
  __device__ void run(int s, E& emit) const {
    g.run(s, emit);
    for (int e = eptr[s]; e < eptr[s + 1]; ++e)
      if (eval[e] != 0.0) emit((uint64_t)ecol[e], eval[e]);
  }
};

// Expansion of the gauge Hamiltonian H_c = (i/2)(conj(c) L' - c L'^+) of a
// dissipator L = c 1 + L' (c = Tr(L)/N): h_j = Tr(F_j H_c) = -Im(conj(c) l_j)
// with l_j = Tr(F_j L) = Tr(F_j L'); the same map on the collapsed diagonal.
__global__ void k_gauge_coef(int64_t M, int N, const cplx* __restrict__ x, const cplx* __restrict__ xd, cplx c,
                             cplx* __restrict__ h, cplx* __restrict__ hd) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (int64_t)gridDim.x * blockDim.x) {
    h[i] = cx(c.im * x[i].re - c.re * x[i].im, 0.0);
    if (i < N) hd[i] = cx(c.im * xd[i].re - c.re * xd[i].im, 0.0);
  }
}

// K = (1/N) Im(B^T l)
__global__ void k_free_vector(int64_t M, int N, const int* __restrict__ bptr, const int* __restrict__ bcol,
                              const cplx* __restrict__ bval, const cplx* __restrict__ l,
                              double* __restrict__ K) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < M;
       s += (int64_t)gridDim.x * blockDim.x) {
    cplx acc = cx(0.0);
    for (int e = bptr[s]; e < bptr[s + 1]; ++e) acc = acc + bval[e] * l[bcol[e]];
    K[s] = acc.im / (double)N;
  }
}

// ---------------------------------------------------------------------------
// Dense assembly (operators with many nonzeros: dense or random L, dense H).
// Each row s of C(x; wf, wd) is written into a dense row by the thread that
// generates it (the same contraction generator as the sparse path, so each
// entry is summed in the same order); the sections then meet in one real
// matrix product on the matrix cores:
//   X = [Re B^T | -Im B^T]  (M x 2M),   Y = [Re A ; Im A]  (2M x M),
//   R = -(1/2) X Y = -(1/2) Re(B^T A).
// ---------------------------------------------------------------------------
enum DenseMode : int { DM_REAL = 0, DM_BT = 1, DM_A = 2 };

template <int MODE>
__global__ void k_dense_rows(ContractGen<cplx> g, int64_t M, double* __restrict__ out, int64_t ld) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < M; s += (int64_t)gridDim.x * blockDim.x) {
    double* row = out + s * ld;
    double* row_im = MODE == DM_A ? out + (M + s) * ld : row + M;
    auto emit = [&](uint64_t n, cplx v) {
      row[n] += v.re;
      if (MODE == DM_BT) row_im[n] -= v.im;
      if (MODE == DM_A) row_im[n] += v.im;
    };
    g.run((int)s, emit);
  }
}

// K[s] = (1/N) Im(B^T l)[s] = (1/N) sum_l (X[s][l] Im l_l - X[s][M+l] Re l_l),
// one workgroup per row, fixed-order reduction
__global__ __launch_bounds__(256) void k_dense_free_vector(int64_t M, int N, const double* __restrict__ X,
                                                           const cplx* __restrict__ l, double* __restrict__ K) {
  __shared__ double sh[256];
  for (int64_t s = blockIdx.x; s < M; s += gridDim.x) {
    const double* xr = X + s * 2 * M;
    double a = 0.0;
    for (int64_t j = threadIdx.x; j < M; j += 256) a += xr[j] * l[j].im - xr[M + j] * l[j].re;
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (threadIdx.x < (unsigned)o) sh[threadIdx.x] += sh[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) K[s] = sh[0] / (double)N;
    __syncthreads();
  }
}

// per-row max |a| of a dense M x M matrix (one wavefront per row)
__global__ __launch_bounds__(256) void k_dense_rowmax(int64_t M, const double* __restrict__ a,
                                                      double* __restrict__ rmax) {
  const int lane = threadIdx.x & 63;
  for (int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; r < M;
       r += ((int64_t)gridDim.x * blockDim.x) >> 6) {
    double m = 0.0;
    for (int64_t c = lane; c < M; c += 64) m = fmax(m, fabs(a[r * M + c]));
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_down(m, o, 64));
    if (lane == 0) rmax[r] = m;
  }
}

// CSR of the entries with |a| > thr, in column order: mode 0 counts per row,
// mode 1 fills (one wavefront per row, positions by ballot prefix counts)
template <int FILL>
__global__ __launch_bounds__(256) void k_dense_compress(int64_t M, const double* __restrict__ a, double thr,
                                                        int64_t* __restrict__ cnt, const int64_t* __restrict__ off,
                                                        int* __restrict__ col, double* __restrict__ val) {
  const int lane = threadIdx.x & 63;
  for (int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; r < M;
       r += ((int64_t)gridDim.x * blockDim.x) >> 6) {
    int64_t base = FILL ? off[r] : 0;
    for (int64_t c0 = 0; c0 < M; c0 += 64) {
      const int64_t c = c0 + lane;
      const double v = c < M ? a[r * M + c] : 0.0;
      const bool keep = c < M && fabs(v) > thr;
      const uint64_t mask = __ballot(keep);
      if (FILL && keep) {
        const int64_t pos = base + __popcll(mask & ((1ull << lane) - 1ull));
        col[pos] = (int)c;
        val[pos] = v;
      }
      base += __popcll(mask);
    }
    if (!FILL && lane == 0) cnt[r] = base;
  }
}

__global__ void k_rowptr_from_off(int64_t M, const int64_t* __restrict__ off, int64_t nnz, int* __restrict__ rowptr) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (int64_t)gridDim.x * blockDim.x) {
    rowptr[i] = (int)off[i];
    if (i == 0) rowptr[M] = (int)nnz;
  }
}

__global__ void k_dense_fill(int64_t n, double v, double* __restrict__ a) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

void check_zcsr(const sun_basis_s& b, const sun_zcsr& X, hipStream_t s) {
  SUN_REQUIRE(X.n == b.N, SUN_EINVAL, "operator dimension differs from basis N");
  SUN_REQUIRE(X.nnz >= 0, SUN_EINVAL, "negative nnz");
  SUN_REQUIRE(X.rowptr != nullptr, SUN_EINVAL, "rowptr is NULL");
  SUN_REQUIRE(X.nnz == 0 || (X.col != nullptr && X.re != nullptr), SUN_EINVAL, "col/re is NULL");
  DevBuf<int> bad(1);
  HIP_OK(hipMemsetAsync(bad.get(), 0, sizeof(int), s));
  hipLaunchKernelGGL(k_validate_csr, dim3(grid_for(X.n, 256)), dim3(256), 0, s, X.n, X.nnz, X.rowptr,
                     X.col, bad.get());
  HIP_LAUNCH_OK();
  int h = 0;
  HIP_OK(hipMemcpyAsync(&h, bad.get(), sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  SUN_REQUIRE(h == 0, SUN_EINVAL,
              h & 1 ? "malformed rowptr" : "column indices out of range or not strictly increasing");
}

}  // namespace

namespace sun {

void expand_operator(const sun_basis_s& b, const sun_zcsr& X, Expansion& e, bool want_herm,
                     hipStream_t s) {
  check_zcsr(b, X, s);
  const BasisDev B = b.view();
  e.x.alloc(b.M);
  e.xd.alloc(b.N);
  DevBuf<cplx> diag(b.N), tr(1);
  DevBuf<double> mx(2);
  HIP_OK(hipMemsetAsync(e.x.get(), 0, b.M * sizeof(cplx), s));
  HIP_OK(hipMemsetAsync(diag.get(), 0, b.N * sizeof(cplx), s));
  HIP_OK(hipMemsetAsync(mx.get(), 0, 2 * sizeof(double), s));
  hipLaunchKernelGGL(k_expand_offdiag, dim3(grid_for(b.N, 256)), dim3(256), 0, s, B, X.rowptr, X.col,
                     X.re, X.im, e.x.get(), diag.get(), mx.get());
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(k_expand_diag, dim3(1), dim3(1), 0, s, B, diag.get(), e.x.get(), e.xd.get(), tr.get());
  HIP_LAUNCH_OK();
  if (want_herm) {
    hipLaunchKernelGGL(k_hermiticity, dim3(grid_for(b.N, 256)), dim3(256), 0, s, b.N, X.rowptr, X.col,
                       X.re, X.im, mx.get() + 1);
    HIP_LAUNCH_OK();
  }
  double hm[2];
  HIP_OK(hipMemcpyAsync(hm, mx.get(), sizeof(hm), hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(&e.trace, tr.get(), sizeof(cplx), hipMemcpyDeviceToHost, s));
  // symmetric adjacency
  DevBuf<int64_t> deg(b.N), off(b.N), ucnt(b.N), uoff(b.N);
  HIP_OK(hipMemsetAsync(deg.get(), 0, b.N * sizeof(int64_t), s));
  hipLaunchKernelGGL(k_adj_count, dim3(grid_for(b.N, 256)), dim3(256), 0, s, b.N, X.rowptr, X.col, deg.get());
  HIP_LAUNCH_OK();
  int64_t raw = exclusive_scan_i64(deg.get(), off.get(), b.N, s);
  DevBuf<int> slot(b.N), rawidx(raw > 0 ? raw : 1);
  HIP_OK(hipMemsetAsync(slot.get(), 0, b.N * sizeof(int), s));
  hipLaunchKernelGGL(k_adj_fill, dim3(grid_for(b.N, 256)), dim3(256), 0, s, b.N, X.rowptr, X.col, off.get(),
                     slot.get(), rawidx.get());
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(k_adj_sort_unique, dim3(grid_for(b.N, 64)), dim3(64), 0, s, b.N, off.get(), deg.get(),
                     rawidx.get(), ucnt.get());
  HIP_LAUNCH_OK();
  int64_t tot = exclusive_scan_i64(ucnt.get(), uoff.get(), b.N, s);
  e.adj_ptr.alloc(b.N + 1);
  e.adj_idx.alloc(tot > 0 ? tot : 1);
  hipLaunchKernelGGL(k_adj_compact, dim3(grid_for(b.N, 256)), dim3(256), 0, s, b.N, off.get(), rawidx.get(),
                     uoff.get(), ucnt.get(), (int)tot, e.adj_ptr.get(), e.adj_idx.get());
  HIP_LAUNCH_OK();
  HIP_OK(hipStreamSynchronize(s));
  e.maxabs = hm[0];
  e.herm_dev = hm[1];
}

}  // namespace sun

namespace {

template <class V>
RowAssemblyResult contract(const sun_basis_s& b, const Expansion& e, const cplx* x, const cplx* xd,
                           cplx wf, cplx wd, double rel_drop, bool drop_zero, hipStream_t s,
                           DevBuf<int>& rowptr, DevBuf<int>& col, DevBuf<V>& val) {
  ContractGen<V> g{b.view(), x, xd, e.adj_ptr.get(), e.adj_idx.get(), wf, wd,
                   (wd.re != 0.0 || wd.im != 0.0) ? 1 : 0};
  return assemble_rows<ContractGen<V>, V, int>(g, b.M, rel_drop, drop_zero, s, &rowptr, col, val);
}

constexpr double kRelDrop = 1e-12;

void assemble_hamiltonian(const sun_basis_s& b, const sun_zcsr& H, DevCSR& out, hipStream_t s) {
  Expansion e;
  expand_operator(b, H, e, true, s);
  SUN_REQUIRE(e.herm_dev <= 1e-12 * (e.maxabs > 0 ? e.maxabs : 1.0), SUN_EINVAL,
              "Hamiltonian term is not Hermitian");
  RowAssemblyResult r = contract<double>(b, e, e.x.get(), e.xd.get(), cx(1.0), cx(0.0), kRelDrop, true, s,
                                         out.rowptr, out.col, out.val);
  out.rows = b.M;
  out.nnz = r.nnz;
}

void assemble_dissipator(const sun_basis_s& b, const sun_zcsr& L, DevCSR& out, DevBuf<double>& K,
                         hipStream_t s) {
  Expansion e;
  expand_operator(b, L, e, false, s);
  // A trace c = Tr(L)/N is moved into a Hamiltonian term:
  //   D_{c 1 + L'} = D_{L'} - i[H_c, .],  H_c = (i/2)(conj(c) L' - c L'^+),
  // and L' has the same coefficients l_j as L (the generators are traceless).
  const double tr = fmax(fabs(e.trace.re), fabs(e.trace.im));
  const bool gauge = tr > 1e-12 * b.N * (e.maxabs > 0 ? e.maxabs : 1.0);
  DevCSR Hc;
  if (gauge) {
    const cplx c = cx(e.trace.re / b.N, e.trace.im / b.N);
    DevBuf<cplx> h(b.M), hd(b.N);
    hipLaunchKernelGGL(k_gauge_coef, dim3(grid_for(b.M, 256)), dim3(256), 0, s, b.M, b.N, e.x.get(), e.xd.get(),
                       c, h.get(), hd.get());
    HIP_LAUNCH_OK();
    RowAssemblyResult rh = contract<double>(b, e, h.get(), hd.get(), cx(1.0), cx(0.0), 0.0, true, s, Hc.rowptr,
                                            Hc.col, Hc.val);
    Hc.rows = b.M;
    Hc.nnz = rh.nnz;
  }
  DevBuf<cplx> xc(b.M), xdc(b.N);
  hipLaunchKernelGGL(k_conj, dim3(grid_for(b.M, 256)), dim3(256), 0, s, b.M, e.x.get(), xc.get());
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(k_conj, dim3(grid_for(b.N, 256)), dim3(256), 0, s, (int64_t)b.N, e.xd.get(), xdc.get());
  HIP_LAUNCH_OK();
  DevZCSR BT, A;
  RowAssemblyResult rb = contract<cplx>(b, e, xc.get(), xdc.get(), cx(1.0), cx(0.0), 0.0, true, s,
                                        BT.rowptr, BT.col, BT.val);
  BT.rows = b.M;
  BT.nnz = rb.nnz;
  RowAssemblyResult ra = contract<cplx>(b, e, e.x.get(), e.xd.get(), cx(-1.0), cx(0.0, 1.0), 0.0, true, s,
                                        A.rowptr, A.col, A.val);
  A.rows = b.M;
  A.nnz = ra.nnz;
  SpgemmGen g{BT.rowptr.get(), BT.col.get(), BT.val.get(), A.rowptr.get(), A.col.get(), A.val.get()};
  RowAssemblyResult rr;
  if (gauge) {
    SpgemmPlusGen gp{g, Hc.rowptr.get(), Hc.col.get(), Hc.val.get()};
    rr = assemble_rows<SpgemmPlusGen, double, int>(gp, b.M, kRelDrop, true, s, &out.rowptr, out.col, out.val);
  } else {
    rr = assemble_rows<SpgemmGen, double, int>(g, b.M, kRelDrop, true, s, &out.rowptr, out.col, out.val);
  }
  out.rows = b.M;
  out.nnz = rr.nnz;
  K.alloc(b.M);
  hipLaunchKernelGGL(k_free_vector, dim3(grid_for(b.M, 256)), dim3(256), 0, s, b.M, b.N, BT.rowptr.get(),
                     BT.col.get(), BT.val.get(), e.x.get(), K.get());
  HIP_LAUNCH_OK();
  HIP_OK(hipStreamSynchronize(s));
}


// ---- dense path -------------------------------------------------------------

// Dense M x M matrix -> CSR, dropping |q| <= kRelDrop max|q| (the same rule
// as the sparse path).
void dense_to_csr(int64_t M, const double* a, DevCSR& out, hipStream_t s) {
  DevBuf<double> rmax(M);
  hipLaunchKernelGGL(k_dense_rowmax, dim3(grid_for(M * 64, 256)), dim3(256), 0, s, M, a, rmax.get());
  HIP_LAUNCH_OK();
  const double thr = kRelDrop * device_max(rmax.get(), M, s);
  DevBuf<int64_t> cnt(M), off(M);
  hipLaunchKernelGGL(k_dense_compress<0>, dim3(grid_for(M * 64, 256)), dim3(256), 0, s, M, a, thr, cnt.get(),
                     nullptr, nullptr, nullptr);
  HIP_LAUNCH_OK();
  const int64_t nnz = exclusive_scan_i64(cnt.get(), off.get(), M, s);
  SUN_REQUIRE(nnz < (int64_t)INT32_MAX, SUN_ENOTSUP, "assembled matrix has 2^31 or more nonzeros");
  out.rows = M;
  out.nnz = nnz;
  out.rowptr.alloc(M + 1);
  out.col.alloc(nnz > 0 ? nnz : 1);
  out.val.alloc(nnz > 0 ? nnz : 1);
  hipLaunchKernelGGL(k_dense_compress<1>, dim3(grid_for(M * 64, 256)), dim3(256), 0, s, M, a, thr, nullptr,
                     off.get(), out.col.get(), out.val.get());
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(k_rowptr_from_off, dim3(grid_for(M, 256)), dim3(256), 0, s, M, off.get(), nnz,
                     out.rowptr.get());
  HIP_LAUNCH_OK();
  HIP_OK(hipStreamSynchronize(s));
}

template <int MODE>
void dense_rows(const sun_basis_s& b, const Expansion& e, const cplx* x, const cplx* xd, cplx wf, cplx wd,
                double* out, int64_t ld, hipStream_t s) {
  ContractGen<cplx> g{b.view(), x, xd, e.adj_ptr.get(), e.adj_idx.get(), wf, wd,
                      (wd.re != 0.0 || wd.im != 0.0) ? 1 : 0};
  hipLaunchKernelGGL(k_dense_rows<MODE>, dim3(grid_for(b.M, 64)), dim3(64), 0, s, g, b.M, out, ld);
  HIP_LAUNCH_OK();
}

// The dense path holds M x M arrays: limit it to M^2 < 2^33 entries (N < 300).
void dense_require(int64_t M) {
  SUN_REQUIRE(M * M < ((int64_t)1 << 33), SUN_ENOTSUP, "dense path limited to M^2 < 2^33 entries (N <= 304)");
}

void dense_zero(double* a, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_dense_fill, dim3(std::min<unsigned>(grid_for(n, 256), 65536)), dim3(256), 0, s, n, 0.0, a);
  HIP_LAUNCH_OK();
}

void assemble_hamiltonian_dense(const sun_basis_s& b, const sun_zcsr& H, DevCSR& out, hipStream_t s) {
  Expansion e;
  expand_operator(b, H, e, true, s);
  SUN_REQUIRE(e.herm_dev <= 1e-12 * (e.maxabs > 0 ? e.maxabs : 1.0), SUN_EINVAL,
              "Hamiltonian term is not Hermitian");
  const int64_t M = b.M;
  dense_require(M);
  DevBuf<double> Q((size_t)M * M);
  dense_zero(Q.get(), M * M, s);
  dense_rows<DM_REAL>(b, e, e.x.get(), e.xd.get(), cx(1.0), cx(0.0), Q.get(), M, s);
  dense_to_csr(M, Q.get(), out, s);
}

void assemble_dissipator_dense(const sun_basis_s& b, const sun_zcsr& L, DevCSR& out, DevBuf<double>& K,
                               hipStream_t s) {
  Expansion e;
  expand_operator(b, L, e, false, s);
  const int64_t M = b.M;
  dense_require(M);
  const double tr = fmax(fabs(e.trace.re), fabs(e.trace.im));
  const bool gauge = tr > 1e-12 * b.N * (e.maxabs > 0 ? e.maxabs : 1.0);
  DevBuf<double> R((size_t)M * M);
  dense_zero(R.get(), M * M, s);
  if (gauge) {
    // the trace moves into the Hamiltonian term H_c (see assemble_dissipator)
    const cplx c = cx(e.trace.re / b.N, e.trace.im / b.N);
    DevBuf<cplx> h(M), hd(b.N);
    hipLaunchKernelGGL(k_gauge_coef, dim3(grid_for(M, 256)), dim3(256), 0, s, M, b.N, e.x.get(), e.xd.get(), c,
                       h.get(), hd.get());
    HIP_LAUNCH_OK();
    dense_rows<DM_REAL>(b, e, h.get(), hd.get(), cx(1.0), cx(0.0), R.get(), M, s);
  }
  DevBuf<cplx> xc(M), xdc(b.N);
  hipLaunchKernelGGL(k_conj, dim3(grid_for(M, 256)), dim3(256), 0, s, M, e.x.get(), xc.get());
  hipLaunchKernelGGL(k_conj, dim3(grid_for(b.N, 256)), dim3(256), 0, s, (int64_t)b.N, e.xd.get(), xdc.get());
  HIP_LAUNCH_OK();
  DevBuf<double> X((size_t)M * 2 * M), Y((size_t)2 * M * M);
  dense_zero(X.get(), 2 * M * M, s);
  dense_zero(Y.get(), 2 * M * M, s);
  dense_rows<DM_BT>(b, e, xc.get(), xdc.get(), cx(1.0), cx(0.0), X.get(), 2 * M, s);
  dense_rows<DM_A>(b, e, e.x.get(), e.xd.get(), cx(-1.0), cx(0.0, 1.0), Y.get(), M, s);
  gemm_f64(M, M, 2 * M, -0.5, X.get(), 2 * M, Y.get(), M, gauge ? 1.0 : 0.0, R.get(), M, s);
  K.alloc(M);
  hipLaunchKernelGGL(k_dense_free_vector, dim3((unsigned)std::min<int64_t>(M, 65536)), dim3(256), 0, s, M, b.N,
                     X.get(), e.x.get(), K.get());
  HIP_LAUNCH_OK();
  dense_to_csr(M, R.get(), out, s);
}

// Device memory of the dense path for one dissipator: X, Y and R.
double dense_bytes(int64_t M) { return 5.0 * (double)M * (double)M * 8.0; }

}  // namespace

extern "C" int sun_expand_operator(sun_basis b, const sun_zcsr* X, double* coef_re, double* coef_im,
                                   double* trace, void* stream) {
  return guarded([&] {
    SUN_REQUIRE(b != nullptr && X != nullptr, SUN_EINVAL, "NULL argument");
    hipStream_t s = as_stream(stream);
    Expansion e;
    expand_operator(*b, *X, e, false, s);
    if (coef_re)
      HIP_OK(hipMemcpy2DAsync(coef_re, sizeof(double), e.x.get(), sizeof(cplx), sizeof(double), b->M,
                              hipMemcpyDeviceToDevice, s));
    if (coef_im)
      HIP_OK(hipMemcpy2DAsync(coef_im, sizeof(double), reinterpret_cast<const char*>(e.x.get()) + sizeof(double),
                              sizeof(cplx), sizeof(double), b->M, hipMemcpyDeviceToDevice, s));
    HIP_OK(hipStreamSynchronize(s));
    if (trace) {
      trace[0] = e.trace.re;
      trace[1] = e.trace.im;
    }
  });
}

namespace {

// mode 0: sparse rows (SUN_ENOTSUP past the LDS row capacity); 1: dense path
// for every term; 2: sparse, falling back to the dense path for a term whose
// rows exceed the capacity
int expand_impl(sun_basis b, const sun_zcsr* H, int32_t nH, const sun_zcsr* L, int32_t P, void* stream,
                sun_lind* out, int mode) {
  return guarded([&] {
    SUN_REQUIRE(out != nullptr, SUN_EINVAL, "out is NULL");
    *out = nullptr;
    SUN_REQUIRE(b != nullptr, SUN_EINVAL, "basis is NULL");
    SUN_REQUIRE(nH >= 0 && P >= 0 && nH + P >= 1, SUN_EINVAL, "need at least one term");
    SUN_REQUIRE(nH == 0 || H != nullptr, SUN_EINVAL, "H is NULL");
    SUN_REQUIRE(P == 0 || L != nullptr, SUN_EINVAL, "L is NULL");
    hipStream_t s = as_stream(stream);
    auto lind = new sun_lind_s();
    try {
      lind->basis = b;
      lind->nH = nH;
      lind->P = P;
      lind->QH.resize(nH);
      lind->R.resize(P);
      lind->K.resize(P);
      auto ham = [&](int a) {
        if (mode == 1) return assemble_hamiltonian_dense(*b, H[a], lind->QH[a], s);
        try {
          assemble_hamiltonian(*b, H[a], lind->QH[a], s);
        } catch (const Error& err) {
          if (mode != 2 || err.code != SUN_ENOTSUP) throw;
          assemble_hamiltonian_dense(*b, H[a], lind->QH[a], s);
        }
      };
      auto dis = [&](int p) {
        if (mode == 1) return assemble_dissipator_dense(*b, L[p], lind->R[p], lind->K[p], s);
        try {
          assemble_dissipator(*b, L[p], lind->R[p], lind->K[p], s);
        } catch (const Error& err) {
          if (mode != 2 || err.code != SUN_ENOTSUP) throw;
          assemble_dissipator_dense(*b, L[p], lind->R[p], lind->K[p], s);
        }
      };
      for (int a = 0; a < nH; ++a) ham(a);
      for (int p = 0; p < P; ++p) dis(p);
    } catch (...) {
      delete lind;
      throw;
    }
    *out = lind;
  });
}

}  // namespace

extern "C" int sun_expand_lindbladian(sun_basis b, const sun_zcsr* H, int32_t nH, const sun_zcsr* L,
                                      int32_t P, void* stream, sun_lind* out) {
  return expand_impl(b, H, nH, L, P, stream, out, 2);
}

extern "C" int sun_expand_lindbladian_dense(sun_basis b, const sun_zcsr* H, int32_t nH, const sun_zcsr* L,
                                            int32_t P, void* stream, sun_lind* out) {
  return expand_impl(b, H, nH, L, P, stream, out, 1);
}

extern "C" int sun_lind_nnz(sun_lind l, int32_t which, int32_t index, int64_t* nnz) {
  return guarded([&] {
    SUN_REQUIRE(l != nullptr && nnz != nullptr, SUN_EINVAL, "NULL argument");
    if (which == SUN_TERM_H) {
      SUN_REQUIRE(index >= 0 && index < l->nH, SUN_EINVAL, "term index out of range");
      *nnz = l->QH[index].nnz;
    } else if (which == SUN_TERM_L) {
      SUN_REQUIRE(index >= 0 && index < l->P, SUN_EINVAL, "term index out of range");
      *nnz = l->R[index].nnz;
    } else {
      SUN_THROW(SUN_EINVAL, "which must be SUN_TERM_H or SUN_TERM_L");
    }
  });
}

extern "C" int sun_lind_export(sun_lind l, int32_t which, int32_t index, int32_t* rowptr, int32_t* col,
                               double* val, double* K, void* stream) {
  return guarded([&] {
    SUN_REQUIRE(l != nullptr, SUN_EINVAL, "lind is NULL");
    hipStream_t s = as_stream(stream);
    const DevCSR* m = nullptr;
    if (which == SUN_TERM_H) {
      SUN_REQUIRE(index >= 0 && index < l->nH, SUN_EINVAL, "term index out of range");
      m = &l->QH[index];
    } else if (which == SUN_TERM_L) {
      SUN_REQUIRE(index >= 0 && index < l->P, SUN_EINVAL, "term index out of range");
      m = &l->R[index];
    } else {
      SUN_THROW(SUN_EINVAL, "which must be SUN_TERM_H or SUN_TERM_L");
    }
    if (rowptr)
      HIP_OK(hipMemcpyAsync(rowptr, m->rowptr.get(), (m->rows + 1) * sizeof(int), hipMemcpyDeviceToDevice, s));
    if (col && m->nnz)
      HIP_OK(hipMemcpyAsync(col, m->col.get(), m->nnz * sizeof(int), hipMemcpyDeviceToDevice, s));
    if (val && m->nnz)
      HIP_OK(hipMemcpyAsync(val, m->val.get(), m->nnz * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (K && which == SUN_TERM_L)
      HIP_OK(hipMemcpyAsync(K, l->K[index].get(), m->rows * sizeof(double), hipMemcpyDeviceToDevice, s));
  });
}

extern "C" int sun_lind_device_bytes(sun_lind l, size_t* bytes) {
  return guarded([&] {
    SUN_REQUIRE(l != nullptr && bytes != nullptr, SUN_EINVAL, "NULL argument");
    size_t b = 0;
    for (const std::vector<DevCSR>* v : {&l->QH, &l->R})
      for (const DevCSR& m : *v) b += m.rowptr.bytes() + m.col.bytes() + m.val.bytes();
    for (const DevBuf<double>& k : l->K) b += k.bytes();
    *bytes = b;
  });
}

extern "C" void sun_lind_free(sun_lind l) { delete l; }
