// Readout of Bloch vectors (Sec. II eq. 5; Sec. IV step 3.2).
//
// The density matrix is rho = 1/N + sum_j v_j F_j.  With the generator
// entries of the grouped basis (S^(j,k): 1/sqrt2 at (j,k) and (k,j); J^(j,k):
// -i/sqrt2 at (j,k), +i/sqrt2 at (k,j); D^l: c_l on the first l diagonal
// entries and -l c_l on entry l):
//     rho_jk = (v_S - i v_J)/sqrt2,  rho_kj = conj(rho_jk)      (j < k, pair p)
//     rho_ii = 1/N - i c_i v_{D_i} + sum_{l > i} c_l v_{D_l}     (c_0 v_{D_0} = 0)
// The diagonal is a suffix sum over l, taken by one workgroup in a fixed
// order.  Expectation values follow from Tr(F_j F_k) = delta_jk:
//     Tr(rho X) = Tr(X)/N + sum_j v_j Tr(F_j X),
// a dot product with the expansion coefficients of X, reduced in a fixed
// order (results do not depend on timing).
#include "internal.hpp"
#include "readout.hpp"

using namespace sun;

namespace {

constexpr int kRT = 256;   // threads of the readout workgroups

// Off-diagonal entries, one row of rho per blockIdx.y (grid-strided).
__global__ __launch_bounds__(kRT) void k_density_offdiag(BasisDev B, const double* __restrict__ v,
                                                         double* __restrict__ re, double* __restrict__ im) {
  const double r = 0.70710678118654752440;
  const int N = B.N;
  for (int i = blockIdx.y; i < N; i += gridDim.y) {
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < N; k += gridDim.x * blockDim.x) {
      if (k == i) continue;
      const int p = pair_index(N, i, k);
      const int64_t e = (int64_t)i * N + k;
      re[e] = v[p] * r;
      if (im) im[e] = (i < k ? -v[B.P + p] : v[B.P + p]) * r;
    }
  }
}

// Diagonal entries: rho_ii = 1/N + own_i + suffix_i with own_i = -i c_i v_{D_i}
// and suffix_i = sum_{l>i} c_l v_{D_l}.  Thread t owns the contiguous range
// [t*chunk, (t+1)*chunk) of l; chunk totals are combined from the top down by
// one thread, then every thread walks its range from the top.
__global__ __launch_bounds__(kRT) void k_density_diag(BasisDev B, const double* __restrict__ v,
                                                      double* __restrict__ re, double* __restrict__ im) {
  __shared__ double tot[kRT];
  const int N = B.N;
  const int chunk = (N + kRT - 1) / kRT;
  const int lo = threadIdx.x * chunk;
  const int hi = min(N, lo + chunk);
  auto term = [&](int l) { return l >= 1 ? B.c[l] * v[2 * B.P + l - 1] : 0.0; };
  double s = 0.0;
  for (int l = hi - 1; l >= lo; --l) s += term(l);
  tot[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double run = 0.0;   // suffix over the chunks above
    for (int t = kRT - 1; t >= 0; --t) {
      const double x = tot[t];
      tot[t] = run;
      run += x;
    }
  }
  __syncthreads();
  double suf = tot[threadIdx.x];
  const double invN = 1.0 / (double)N;
  for (int i = hi - 1; i >= lo; --i) {
    const double own = i >= 1 ? -(double)i * term(i) : 0.0;
    const int64_t e = (int64_t)i * N + i;
    re[e] = invN + own + suf;
    if (im) im[e] = 0.0;
    suf += term(i);
  }
}

// Partial dot products of nvec vectors with (x_re, x_im); nb blocks per
// vector (blockIdx.x), vectors over blockIdx.y (grid-strided).  With nb == 1
// the block writes the result (plus the constant c) directly.
__global__ __launch_bounds__(kRT) void k_expect_part(int64_t M, const double* __restrict__ v, int64_t nvec,
                                                     int64_t ldv, const double* __restrict__ xre,
                                                     const double* __restrict__ xim, double cre, double cim,
                                                     double* __restrict__ out_re, double* __restrict__ out_im,
                                                     double* __restrict__ part) {
  __shared__ double sr[kRT], si[kRT];
  const int nb = gridDim.x;
  for (int64_t vi = blockIdx.y; vi < nvec; vi += gridDim.y) {
    const double* a = v + vi * ldv;
    double r = 0.0, q = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * kRT + threadIdx.x; j < M; j += (int64_t)nb * kRT) {
      r += a[j] * xre[j];
      if (xim) q += a[j] * xim[j];
    }
    sr[threadIdx.x] = r;
    si[threadIdx.x] = q;
    __syncthreads();
    for (int o = kRT / 2; o > 0; o >>= 1) {
      if (threadIdx.x < (unsigned)o) {
        sr[threadIdx.x] += sr[threadIdx.x + o];
        si[threadIdx.x] += si[threadIdx.x + o];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      if (nb == 1) {
        out_re[vi] = cre + sr[0];
        if (out_im) out_im[vi] = cim + si[0];
      } else {
        part[(vi * nb + blockIdx.x) * 2] = sr[0];
        part[(vi * nb + blockIdx.x) * 2 + 1] = si[0];
      }
    }
    __syncthreads();
  }
}

// Sum of the nb partials of each vector in a fixed order.
__global__ __launch_bounds__(kRT) void k_expect_finish(int64_t nvec, int nb, const double* __restrict__ part,
                                                       double cre, double cim, double* __restrict__ out_re,
                                                       double* __restrict__ out_im) {
  __shared__ double sr[kRT], si[kRT];
  for (int64_t vi = blockIdx.x; vi < nvec; vi += gridDim.x) {
    double r = 0.0, q = 0.0;
    for (int b = threadIdx.x; b < nb; b += kRT) {
      r += part[(vi * nb + b) * 2];
      q += part[(vi * nb + b) * 2 + 1];
    }
    sr[threadIdx.x] = r;
    si[threadIdx.x] = q;
    __syncthreads();
    for (int o = kRT / 2; o > 0; o >>= 1) {
      if (threadIdx.x < (unsigned)o) {
        sr[threadIdx.x] += sr[threadIdx.x + o];
        si[threadIdx.x] += si[threadIdx.x + o];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      out_re[vi] = cre + sr[0];
      if (out_im) out_im[vi] = cim + si[0];
    }
    __syncthreads();
  }
}

}  // namespace

namespace sun {

void expect_launch(int64_t M, const double* v, int64_t nvec, int64_t ldv, const double* xre, const double* xim,
                   double cre, double cim, double* out_re, double* out_im, double* part, int nb, hipStream_t s) {
  if (nvec <= 0) return;
  const unsigned gy = (unsigned)std::min<int64_t>(nvec, 65535);
  if (part == nullptr || nb <= 1) {
    hipLaunchKernelGGL(k_expect_part, dim3(1, gy), dim3(kRT), 0, s, M, v, nvec, ldv, xre, xim, cre, cim, out_re,
                       out_im, nullptr);
  } else {
    hipLaunchKernelGGL(k_expect_part, dim3(nb, gy), dim3(kRT), 0, s, M, v, nvec, ldv, xre, xim, cre, cim, out_re,
                       out_im, part);
    hipLaunchKernelGGL(k_expect_finish, dim3(gy), dim3(kRT), 0, s, nvec, nb, part, cre, cim, out_re, out_im);
  }
  HIP_LAUNCH_OK();
}

}  // namespace sun

extern "C" int sun_bloch_density(sun_basis b, const double* v, double* rho_re, double* rho_im, void* stream) {
  return guarded([&] {
    SUN_REQUIRE(b != nullptr && v != nullptr && rho_re != nullptr, SUN_EINVAL, "NULL argument");
    hipStream_t s = as_stream(stream);
    const BasisDev B = b->view();
    const unsigned gx = grid_for(b->N, kRT);
    const unsigned gy = (unsigned)std::min(b->N, 65535);
    hipLaunchKernelGGL(k_density_offdiag, dim3(gx, gy), dim3(kRT), 0, s, B, v, rho_re, rho_im);
    hipLaunchKernelGGL(k_density_diag, dim3(1), dim3(kRT), 0, s, B, v, rho_re, rho_im);
    HIP_LAUNCH_OK();
  });
}

extern "C" int sun_bloch_expect(sun_basis b, const double* v, int64_t nvec, int64_t ldv, const double* x_re,
                                const double* x_im, const double* trace, double* out_re, double* out_im,
                                void* stream) {
  return guarded([&] {
    SUN_REQUIRE(b != nullptr && x_re != nullptr && out_re != nullptr, SUN_EINVAL, "NULL argument");
    SUN_REQUIRE(nvec >= 0, SUN_EINVAL, "nvec must be >= 0");
    SUN_REQUIRE(nvec == 0 || v != nullptr, SUN_EINVAL, "v is NULL");
    SUN_REQUIRE(nvec <= 1 || ldv >= b->M, SUN_EINVAL, "ldv must be >= M");
    SUN_REQUIRE(out_im == nullptr || x_im != nullptr, SUN_EINVAL, "out_im needs x_im");
    const double inv = 1.0 / (double)b->N;
    const double cre = trace ? trace[0] * inv : 0.0;
    const double cim = trace ? trace[1] * inv : 0.0;
    expect_launch(b->M, v, nvec, ldv, x_re, out_im ? x_im : nullptr, cre, cim, out_re, out_im, nullptr, 1,
                  as_stream(stream));
  });
}
