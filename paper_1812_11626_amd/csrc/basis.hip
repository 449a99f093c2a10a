// SU(N) basis metadata, and counting / export of the nonzero structure
// constants (Sec. II, eq. 4; Sec. IV, step 2.2) from their closed forms.
// Generators run twice (count, then fill) and must take identical
// floating-point decisions in both passes: no contraction into FMAs.
#pragma clang fp contract(off)

#include <cmath>

#include "internal.hpp"
#include "rowpipe.hpp"

using namespace sun;

namespace {

// ---------------------------------------------------------------------------
// Enumeration of the structurally possible (b, c) for one first index a.
// Every (b, c) with T(a,b,c) != 0 is visited exactly once; some visited
// entries evaluate to zero in the real or imaginary part and are skipped by
// the caller.  Work item (a, t), t in [0, N), visits one slice of row a:
//   a = pair (j,k):  t = l.  Triangles through vertex l (if l not in {j,k}):
//                    (b, c) = (X_{j,l}, Y_{l,k}) and (X_{k,l}, Y_{l,j});
//                    same-edge with D^l (if l >= 1): (P_{jk}, D^l), (D^l, P_{jk}).
//   a = D^l:         t = j.  Pairs (j,k), k > j, if j <= l: (P_{jk}, P'_{jk});
//                    and the diagonal triples (q,q) q<l, (l,q) q>=l, (q,l) q>l
//                    with q = t (q >= 1).
// ---------------------------------------------------------------------------
template <class F>
__device__ inline void enum_slice(const BasisDev& B, int a, int t, F&& visit) {
  const Gen ga = decode(B, a);
  const int N = B.N;
  if (ga.kind != KD) {
    const int j = ga.j, k = ga.k, l = t;
    if (l != j && l != k) {
      for (int order = 0; order < 2; ++order) {
        int u = order ? k : j;   // vertex shared by a and b
        int w = order ? j : k;   // vertex shared by a and c
        for (int tb = 0; tb < 2; ++tb) {
          Gen gb{tb, min(u, l), max(u, l)};
          for (int tc = 0; tc < 2; ++tc) {
            Gen gc{tc, min(l, w), max(l, w)};
            visit(encode_pair(B, tb, u, l), encode_pair(B, tc, l, w), trace3(B, ga, gb, gc));
          }
        }
      }
    }
    if (l >= 1) {
      Gen gd{KD, l, l};
      for (int tp = 0; tp < 2; ++tp) {
        Gen gp{tp, j, k};
        visit(encode_pair(B, tp, j, k), encode_diag(B, l), trace3(B, ga, gp, gd));
        visit(encode_diag(B, l), encode_pair(B, tp, j, k), trace3(B, ga, gd, gp));
      }
    }
  } else {
    const int l = ga.j, j = t;
    if (j <= l) {
      for (int k = j + 1; k < N; ++k) {
        for (int tb = 0; tb < 2; ++tb) {
          Gen gb{tb, j, k};
          for (int tc = 0; tc < 2; ++tc) {
            Gen gc{tc, j, k};
            visit(encode_pair(B, tb, j, k), encode_pair(B, tc, j, k), trace3(B, ga, gb, gc));
          }
        }
      }
    }
    const int q = t;
    if (q >= 1) {
      if (q < l) visit(encode_diag(B, q), encode_diag(B, q), cx(trace_ddd(B, l, q, q)));
      if (q >= l) visit(encode_diag(B, l), encode_diag(B, q), cx(trace_ddd(B, l, l, q)));
      if (q > l) visit(encode_diag(B, q), encode_diag(B, l), cx(trace_ddd(B, l, q, l)));
    }
  }
}

__global__ __launch_bounds__(256) void k_count_fd(BasisDev B, unsigned long long* out) {
  __shared__ unsigned long long sf[256], sd[256];
  unsigned long long nf = 0, nd = 0;
  const int64_t items = (int64_t)B.M * B.N;
  for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < items;
       w += (int64_t)gridDim.x * blockDim.x) {
    int a = (int)(w / B.N), t = (int)(w % B.N);
    enum_slice(B, a, t, [&](int, int, cplx T) {
      nf += (T.im != 0.0);
      nd += (T.re != 0.0);
    });
  }
  sf[threadIdx.x] = nf;
  sd[threadIdx.x] = nd;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < (unsigned)o) {
      sf[threadIdx.x] += sf[threadIdx.x + o];
      sd[threadIdx.x] += sd[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicAdd(&out[0], sf[0]);
    atomicAdd(&out[1], sd[0]);
  }
}

// Row generator for the export: row a, key = b*M + c, value f or d.
struct ExportGen {
  BasisDev B;
  int which;      // 0 = f, 1 = d
  int canonical;  // 1: only m < n < s (f) or m <= n <= s (d)
  template <class E>
  __device__ void run(int a, E& emit) const {
    for (int t = 0; t < B.N; ++t) {
      enum_slice(B, a, t, [&](int b, int c, cplx T) {
        if (canonical && (which == 0 ? !(a < b && b < c) : !(a <= b && b <= c))) return;
        double v = which == 0 ? 2.0 * T.im : 2.0 * T.re;
        if (v != 0.0) emit((uint64_t)b * (uint64_t)B.M + (uint64_t)c, v);
      });
    }
  }
};

__global__ void k_export_triples(int64_t rows, int64_t M, const int* __restrict__ rowptr,
                                 const uint64_t* __restrict__ key, int* __restrict__ idx) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < rows;
       r += (int64_t)gridDim.x * blockDim.x) {
    for (int e = rowptr[r]; e < rowptr[r + 1]; ++e) {
      idx[3 * (int64_t)e + 0] = (int)r;
      idx[3 * (int64_t)e + 1] = (int)(key[e] / (uint64_t)M);
      idx[3 * (int64_t)e + 2] = (int)(key[e] % (uint64_t)M);
    }
  }
}

}  // namespace

extern "C" int sun_build_basis(int32_t N, void* stream, sun_basis* out) {
  return guarded([&] {
    SUN_REQUIRE(out != nullptr, SUN_EINVAL, "out is NULL");
    *out = nullptr;
    SUN_REQUIRE(N >= 2, SUN_EINVAL, "N must be >= 2");
    SUN_REQUIRE((int64_t)N * N - 1 < (int64_t)INT32_MAX, SUN_EINVAL, "M = N^2-1 must be < 2^31");
    hipStream_t s = as_stream(stream);
    auto b = new sun_basis_s();
    try {
      b->N = N;
      b->P = N * (N - 1) / 2;
      b->M = (int64_t)N * N - 1;
      HIP_OK(hipGetDevice(&b->device));
      std::vector<int> pj(b->P), pk(b->P);
      for (int j = 0; j < N; ++j)
        for (int k = j + 1; k < N; ++k) {
          int p = pair_index(N, j, k);
          pj[p] = j;
          pk[p] = k;
        }
      std::vector<double> c(N, 0.0);
      for (int l = 1; l < N; ++l) c[l] = 1.0 / std::sqrt((double)l * (double)(l + 1));
      b->pj.alloc(b->P);
      b->pk.alloc(b->P);
      b->c.alloc(N);
      HIP_OK(hipMemcpyAsync(b->pj.get(), pj.data(), b->P * sizeof(int), hipMemcpyHostToDevice, s));
      HIP_OK(hipMemcpyAsync(b->pk.get(), pk.data(), b->P * sizeof(int), hipMemcpyHostToDevice, s));
      HIP_OK(hipMemcpyAsync(b->c.get(), c.data(), N * sizeof(double), hipMemcpyHostToDevice, s));
      HIP_OK(hipStreamSynchronize(s));
    } catch (...) {
      delete b;
      throw;
    }
    *out = b;
  });
}

extern "C" int sun_basis_dims(sun_basis b, int32_t* N, int64_t* M) {
  return guarded([&] {
    SUN_REQUIRE(b != nullptr, SUN_EINVAL, "basis is NULL");
    if (N) *N = b->N;
    if (M) *M = b->M;
  });
}

extern "C" int sun_basis_counts(sun_basis b, void* stream, int64_t* nnz_f, int64_t* nnz_d) {
  return guarded([&] {
    SUN_REQUIRE(b != nullptr, SUN_EINVAL, "basis is NULL");
    hipStream_t s = as_stream(stream);
    DevBuf<unsigned long long> out(2);
    HIP_OK(hipMemsetAsync(out.get(), 0, 2 * sizeof(unsigned long long), s));
    const int64_t items = b->M * (int64_t)b->N;
    unsigned grid = grid_for(items, 256);
    if (grid > 16384) grid = 16384;
    hipLaunchKernelGGL(k_count_fd, dim3(grid), dim3(256), 0, s, b->view(), out.get());
    HIP_LAUNCH_OK();
    unsigned long long h[2];
    HIP_OK(hipMemcpyAsync(h, out.get(), sizeof(h), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if (nnz_f) *nnz_f = (int64_t)h[0];
    if (nnz_d) *nnz_d = (int64_t)h[1];
  });
}

extern "C" int sun_basis_export(sun_basis b, int32_t which, int32_t canonical, int32_t* idx, double* val,
                                int64_t cap, int64_t* written, void* stream) {
  return guarded([&] {
    SUN_REQUIRE(b != nullptr, SUN_EINVAL, "basis is NULL");
    SUN_REQUIRE(which == 0 || which == 1, SUN_EINVAL, "which must be 0 (f) or 1 (d)");
    SUN_REQUIRE(canonical == 0 || canonical == 1, SUN_EINVAL, "canonical must be 0 or 1");
    SUN_REQUIRE(b->N <= 64, SUN_ENOTSUP, "export supports N <= 64");
    hipStream_t s = as_stream(stream);
    ExportGen g{b->view(), which, canonical};
    DevBuf<int> rowptr;
    DevBuf<uint64_t> key;
    DevBuf<double> v;
    RowAssemblyResult r = assemble_rows<ExportGen, double, uint64_t>(g, b->M, 0.0, true, s, &rowptr, key, v);
    if (written) *written = r.nnz;
    if (r.nnz > cap) SUN_THROW(SUN_ERANGE, "capacity too small");
    if (r.nnz == 0) return;
    SUN_REQUIRE(idx != nullptr && val != nullptr, SUN_EINVAL, "idx/val is NULL");
    hipLaunchKernelGGL(k_export_triples, dim3(grid_for(b->M, 256)), dim3(256), 0, s, b->M, b->M,
                       rowptr.get(), key.get(), idx);
    HIP_LAUNCH_OK();
    HIP_OK(hipMemcpyAsync(val, v.get(), r.nnz * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIP_OK(hipStreamSynchronize(s));
  });
}

extern "C" void sun_basis_free(sun_basis b) { delete b; }
