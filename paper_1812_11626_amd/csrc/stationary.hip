// Stationary state of a time-independent generator (paper Sec. I: the
// asymptotic state of a time-independent GKSL equation is the kernel of the
// Lindbladian; in the Bloch form of eq. 9 it is the solution of G v = -K).
//
// G is far from normal for the driven-dimer class (eigenvalues spread along
// the imaginary axis up to |lambda| ~ 2 sqrt(eps^2 + J^2) (N-1), real parts of
// order one), so Krylov methods on G itself converge slowly.  The time-tau
// map of RK4 is benign instead: with n steps of size dt (tau = n dt),
//     v -> Phi v + phi,   Phi = R4(dt G)^n,
// and the fixed point of one RK4 step, v = v + dt p(dt G)(G v + K) with
// p(z) = 1 + z/2 + z^2/6 + z^3/24, is exactly G v + K = 0 (p(dt G) is
// invertible for a stable step), so the fixed point of the tau-map is the
// stationary state itself.  Every mode with decay rate r contracts by e^{-r
// tau} per map, so (I - Phi) has its spectrum clustered at 1 except for the
// few modes slower than 1/tau, which restarted GMRES resolves in about one
// iteration each.  The map is applied with the propagator's fused stage
// kernels on augmented vectors whose entry M is 0 (the folded free vector
// drops out, giving Phi x); phi is the map applied to the zero state with
// entry M = 1.  Orthogonalisation is classical Gram-Schmidt, twice, with all
// dot products of a pass in one launch (per-block partials summed on the
// host in a fixed order); the small Hessenberg least-squares problem is
// solved on the host with Givens rotations.  The returned residual is the
// true ||G v + K||_2 / ||K||_2, from one stage launch.
#include <cmath>
#include <vector>

#include "prop_internal.hpp"

using namespace sun;

namespace {

constexpr int kStT = 256;
constexpr int kStBlocks = 256;   // partial sums per dot product

__global__ void k_st_fill(int64_t n, double v, double* __restrict__ a) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

// part[i * nb + b] = partial of dot(w, V_i) over block b's strided range (rows < M)
__global__ __launch_bounds__(kStT) void k_st_multidot(int64_t M, const double* __restrict__ w,
                                                      const double* __restrict__ V, int64_t ldv,
                                                      double* __restrict__ part) {
  __shared__ double sh[kStT];
  const int i = blockIdx.y;
  const double* vi = V + (int64_t)i * ldv;
  double s = 0.0;
  for (int64_t j = (int64_t)blockIdx.x * kStT + threadIdx.x; j < M; j += (int64_t)gridDim.x * kStT) s += w[j] * vi[j];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = kStT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < (unsigned)o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(int64_t)i * gridDim.x + blockIdx.x] = sh[0];
}

// w[j] -= sum_{i<k} h[i] V_i[j]   (rows < M; h in device memory)
__global__ void k_st_sub(int64_t M, double* __restrict__ w, const double* __restrict__ V, int64_t ldv, int k,
                         const double* __restrict__ h) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < M; j += (int64_t)gridDim.x * blockDim.x) {
    double s = w[j];
    for (int i = 0; i < k; ++i) s -= h[i] * V[(int64_t)i * ldv + j];
    w[j] = s;
  }
}

// y[j] = a * x[j] + b * y[j]   (rows < M)
__global__ void k_st_axpby(int64_t M, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < M; j += (int64_t)gridDim.x * blockDim.x)
    y[j] = a * x[j] + b * y[j];
}

unsigned st_grid(int64_t M) { return std::min<unsigned>(grid_for(M, kStT), 4096); }

struct Solver {
  sun_prop_s& p;
  hipStream_t s;
  int64_t M, M1;
  double dt;
  int64_t nsteps;
  DevBuf<double> cdev, cur, nxt, xa, acc, part, hdev;

  Solver(sun_prop_s& p_, hipStream_t s_, double dt_, int64_t n_) : p(p_), s(s_), dt(dt_), nsteps(n_) {
    M = p.M;
    M1 = M + 1;
    cdev.alloc(p.ndyn > 0 ? p.ndyn : 1);
    cur.alloc(M1);
    nxt.alloc(M1);
    xa.alloc(M1);
    acc.alloc(M1);
  }

  // dot products of w with V_0..V_{k-1} (leading dimension ldv), summed on
  // the host in a fixed order
  void dots(const double* w, const double* V, int64_t ldv, int k, double* out) {
    const int nb = (int)std::min<int64_t>(kStBlocks, std::max<int64_t>(1, (M + kStT - 1) / kStT));
    if (part.n < (size_t)k * nb) part.alloc((size_t)k * nb);
    hipLaunchKernelGGL(k_st_multidot, dim3(nb, k), dim3(kStT), 0, s, M, w, V, ldv, part.get());
    HIP_LAUNCH_OK();
    std::vector<double> h((size_t)k * nb);
    HIP_OK(hipMemcpyAsync(h.data(), part.get(), h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    for (int i = 0; i < k; ++i) {
      double t = 0.0;
      for (int b = 0; b < nb; ++b) t += h[(size_t)i * nb + b];
      out[i] = t;
    }
  }

  double norm(const double* w) {
    double d = 0.0;
    dots(w, w, 0, 1, &d);
    return std::sqrt(d);
  }

  // out = x propagated over nsteps RK4 steps with the frozen coefficients;
  // entry M of x (0 or 1) decides whether the free vector takes part
  void map(const double* x, double* out, double tail) {
    HIP_OK(hipMemcpyAsync(cur.get(), x, M * sizeof(double), hipMemcpyDeviceToDevice, s));
    for (double* b : {cur.get(), nxt.get(), xa.get(), acc.get()})
      hipLaunchKernelGGL(k_st_fill, dim3(1), dim3(1), 0, s, (int64_t)1, tail, b + M);
    HIP_LAUNCH_OK();
    double* a = cur.get();
    double* b = nxt.get();
    for (int64_t n = 0; n < nsteps; ++n) {
      prop_stage(p, 0, a, a, acc.get(), xa.get(), cdev.get(), 0, dt, s);
      prop_stage(p, 1, xa.get(), a, acc.get(), b, cdev.get(), 0, dt, s);
      prop_stage(p, 2, b, a, acc.get(), xa.get(), cdev.get(), 0, dt, s);
      prop_stage(p, 3, xa.get(), a, acc.get(), b, cdev.get(), 0, dt, s);
      std::swap(a, b);
    }
    HIP_OK(hipMemcpyAsync(out, a, M * sizeof(double), hipMemcpyDeviceToDevice, s));
  }

  // out = G x + K (x[M] = 1 brings the folded free vector in): stage 0 with
  // a zero base vector and dt = 2 stores exactly k = G x + K
  void residual(const double* x, double* out, double* zero) {
    HIP_OK(hipMemcpyAsync(cur.get(), x, M * sizeof(double), hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_st_fill, dim3(1), dim3(1), 0, s, (int64_t)1, 1.0, cur.get() + M);
    HIP_LAUNCH_OK();
    prop_stage(p, 0, cur.get(), zero, acc.get(), out, cdev.get(), 0, 2.0, s);
  }
};

}  // namespace

extern "C" int sun_stationary(sun_prop p, const double* coef, double dt, int64_t steps_per_map, int32_t restart,
                              int32_t max_iter, double tol, double* v, int32_t* iters_out, double* relres_out,
                              void* stream) {
  return guarded([&] {
    SUN_REQUIRE(p != nullptr && v != nullptr, SUN_EINVAL, "NULL argument");
    SUN_REQUIRE(p->ndyn == 0 || coef != nullptr, SUN_EINVAL, "coef is NULL");
    SUN_REQUIRE(dt > 0.0 && std::isfinite(dt), SUN_EINVAL, "dt must be positive");
    SUN_REQUIRE(steps_per_map >= 1, SUN_EINVAL, "steps_per_map must be >= 1");
    SUN_REQUIRE(restart >= 1 && restart <= 1000, SUN_EINVAL, "restart must be in [1, 1000]");
    SUN_REQUIRE(max_iter >= 1, SUN_EINVAL, "max_iter must be >= 1");
    SUN_REQUIRE(tol > 0.0, SUN_EINVAL, "tol must be > 0");
    prop_require_usable(*p);
    if (p->dt_max > 0.0 && dt > p->dt_max)
      SUN_THROW(SUN_EUNSTABLE, "dt exceeds the stable step set by sun_prop_guard_stability");
    hipStream_t s = as_stream(stream);
    Solver S(*p, s, dt, steps_per_map);
    const int64_t M = S.M, M1 = S.M1;
    if (p->ndyn > 0) HIP_OK(hipMemcpyAsync(S.cdev.get(), coef, p->ndyn * sizeof(double), hipMemcpyHostToDevice, s));
    const int m = restart;
    DevBuf<double> V((size_t)(m + 1) * M1), x(M1), phi(M1), w(M1), r(M1), zero(M1);
    for (DevBuf<double>* b : {&x, &phi, &w, &r, &zero})
      hipLaunchKernelGGL(k_st_fill, dim3(st_grid(M1)), dim3(kStT), 0, s, M1, 0.0, b->get());
    HIP_LAUNCH_OK();
    HIP_OK(hipMemcpyAsync(x.get(), v, M * sizeof(double), hipMemcpyDeviceToDevice, s));
    // ||K||: the residual of the zero state
    S.residual(zero.get(), r.get(), zero.get());
    const double knorm = S.norm(r.get());
    auto true_relres = [&]() {
      S.residual(x.get(), r.get(), zero.get());
      const double rn = S.norm(r.get());
      return knorm > 0.0 ? rn / knorm : rn;
    };
    int iters = 0;
    double relres = true_relres();
    if (knorm == 0.0) {
      // no free vector: the maximally mixed state (v = 0) is stationary
      hipLaunchKernelGGL(k_st_fill, dim3(st_grid(M)), dim3(kStT), 0, s, M, 0.0, v);
      HIP_LAUNCH_OK();
      relres = 0.0;
    } else {
      // phi = the map applied to the zero state (free vector only)
      S.map(zero.get(), phi.get(), 1.0);
      const double phinorm = S.norm(phi.get());
      std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m), h(m + 1), h2(m + 1);
      while (relres > tol && iters < max_iter) {
        // r = phi - (x - Phi x)
        S.map(x.get(), w.get(), 0.0);                                  // w = Phi x
        HIP_OK(hipMemcpyAsync(r.get(), phi.get(), M * sizeof(double), hipMemcpyDeviceToDevice, s));
        hipLaunchKernelGGL(k_st_axpby, dim3(st_grid(M)), dim3(kStT), 0, s, M, 1.0, w.get(), 1.0, r.get());
        hipLaunchKernelGGL(k_st_axpby, dim3(st_grid(M)), dim3(kStT), 0, s, M, -1.0, x.get(), 1.0, r.get());
        HIP_LAUNCH_OK();
        const double beta = S.norm(r.get());
        if (!(beta > 0.0) || !std::isfinite(beta)) break;
        std::fill(H.begin(), H.end(), 0.0);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        double* V0 = V.get();
        hipLaunchKernelGGL(k_st_axpby, dim3(st_grid(M)), dim3(kStT), 0, s, M, 1.0 / beta, r.get(), 0.0, V0);
        HIP_LAUNCH_OK();
        int k = 0;
        for (; k < m && iters < max_iter; ++k, ++iters) {
          double* Vk = V0 + (int64_t)k * M1;
          double* Vn = V0 + (int64_t)(k + 1) * M1;
          // Vn = (I - Phi) Vk
          S.map(Vk, Vn, 0.0);
          hipLaunchKernelGGL(k_st_axpby, dim3(st_grid(M)), dim3(kStT), 0, s, M, 1.0, Vk, -1.0, Vn);
          HIP_LAUNCH_OK();
          // classical Gram-Schmidt, twice
          std::fill(h.begin(), h.end(), 0.0);
          for (int pass = 0; pass < 2; ++pass) {
            S.dots(Vn, V0, M1, k + 1, h2.data());
            if (S.hdev.n < (size_t)(m + 1)) S.hdev.alloc(m + 1);
            HIP_OK(hipMemcpyAsync(S.hdev.get(), h2.data(), (k + 1) * sizeof(double), hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL(k_st_sub, dim3(st_grid(M)), dim3(kStT), 0, s, M, Vn, V0, M1, k + 1, S.hdev.get());
            HIP_LAUNCH_OK();
            for (int i = 0; i <= k; ++i) h[i] += h2[i];
          }
          const double hn = S.norm(Vn);
          h[k + 1] = hn;
          if (hn > 0.0) {
            hipLaunchKernelGGL(k_st_axpby, dim3(st_grid(M)), dim3(kStT), 0, s, M, 1.0 / hn, Vn, 0.0, Vn);
            HIP_LAUNCH_OK();
          }
          // Givens rotations on column k of the Hessenberg matrix
          for (int i = 0; i < k; ++i) {
            const double t = cs[i] * h[i] + sn[i] * h[i + 1];
            h[i + 1] = -sn[i] * h[i] + cs[i] * h[i + 1];
            h[i] = t;
          }
          const double d = std::hypot(h[k], h[k + 1]);
          cs[k] = d > 0.0 ? h[k] / d : 1.0;
          sn[k] = d > 0.0 ? h[k + 1] / d : 0.0;
          h[k] = d;
          h[k + 1] = 0.0;
          g[k + 1] = -sn[k] * g[k];
          g[k] = cs[k] * g[k];
          for (int i = 0; i <= k; ++i) H[(size_t)i * m + k] = h[i];
          // the map's residual is G's damped by up to 1/|lambda| for fast
          // modes: end the cycle well below tol in the map's relative
          // residual; the true residual decides about another cycle
          if (std::fabs(g[k + 1]) <= 0.01 * tol * phinorm || hn == 0.0) {
            ++k;
            ++iters;
            break;
          }
        }
        // y = H^{-1} g (upper triangular, k x k); x += V y
        for (int i = k - 1; i >= 0; --i) {
          double t = g[i];
          for (int j = i + 1; j < k; ++j) t -= H[(size_t)i * m + j] * y[j];
          y[i] = t / H[(size_t)i * m + i];
        }
        for (int i = 0; i < k; ++i) {
          hipLaunchKernelGGL(k_st_axpby, dim3(st_grid(M)), dim3(kStT), 0, s, M, y[i], V0 + (int64_t)i * M1, 1.0,
                             x.get());
        }
        HIP_LAUNCH_OK();
        relres = true_relres();
        if (!std::isfinite(relres)) break;
      }
      HIP_OK(hipMemcpyAsync(v, x.get(), M * sizeof(double), hipMemcpyDeviceToDevice, s));
      HIP_OK(hipStreamSynchronize(s));
    }
    if (iters_out) *iters_out = iters;
    if (relres_out) *relres_out = relres;
    SUN_REQUIRE(std::isfinite(relres), SUN_EDIVERGED, "the iteration produced a non-finite state");
    SUN_REQUIRE(relres <= tol, SUN_ENOTCONVERGED,
                "not converged: relative residual " + std::to_string(relres) + " after " + std::to_string(iters) +
                    " iterations (v holds the last iterate)");
  });
}
