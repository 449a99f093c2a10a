// Dense FP64 matrix product on the CDNA matrix cores:
//     C = alpha A B + beta C,   A: M x K,  B: K x N,  C: M x N,  row-major.
// The dense-operator assembly forms the dissipative part as one such product,
// R = -(1/2) Re(B^T A) = -(1/2) [Re B^T | -Im B^T] [Re A ; Im A], a dense
// contraction of M x 2M by 2M x M (Sec. II eq. 10 with dense sections).
//
// Tiling: a workgroup of four wavefronts computes a 128 x 128 tile of C,
// each wavefront a 64 x 64 quarter as 4 x 4 blocks of 16 x 16, with
// v_mfma_f64_16x16x4f64 (a 16 x 4 by 4 x 16 product per instruction, 4
// accumulators per lane).  K advances in steps of 16: the A panel (128 x 16)
// and B panel (16 x 128) are staged in LDS, double-buffered, the next panel
// fetched into registers while the current one is multiplied.  Operand
// layout of the instruction: lane l holds A[l % 16][l / 16] and B[l / 16][l %
// 16]; accumulator r of lane l is C[4 r + l / 16][l % 16] (checked on the
// device with one-hot operands).  Workgroups are
// numbered so that consecutive ones share a band of rows of A (groups of 8
// row tiles), which keeps the A band and the B panels they read in L2.
#include "internal.hpp"

using namespace sun;

namespace {

constexpr int kBM = 128, kBN = 128, kBK = 16;
constexpr int kAP = kBK + 1;      // padded row of the A panel in LDS (row-major)
constexpr int kBP = kBN + 2;      // padded row of the B panel in LDS
constexpr int kGroupM = 8;

typedef double v4d __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_gemm_f64(int64_t M, int64_t N, int64_t K, double alpha,
                                                  const double* __restrict__ A, int64_t lda,
                                                  const double* __restrict__ B, int64_t ldb, double beta,
                                                  double* __restrict__ C, int64_t ldc) {
  __shared__ double As[2][kBM * kAP];
  __shared__ double Bs[2][kBK * kBP];
  // grouped tile order: kGroupM row tiles share their A band
  const int64_t tiles_m = (M + kBM - 1) / kBM, tiles_n = (N + kBN - 1) / kBN;
  const int64_t pid = blockIdx.x;
  const int64_t per_group = (int64_t)kGroupM * tiles_n;
  const int64_t group = pid / per_group;
  const int64_t first_m = group * kGroupM;
  const int64_t gsize = min((int64_t)kGroupM, tiles_m - first_m);
  const int64_t tm = first_m + (pid % per_group) % gsize;
  const int64_t tn = (pid % per_group) / gsize;
  const int64_t row0 = tm * kBM, col0 = tn * kBN;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;

  // global -> register staging: A panel 128 x 16 (8 per thread: row tid/2,
  // columns (tid%2)*8 ..+8), B panel 16 x 128 (8 per thread: row tid/16,
  // columns (tid%16)*8 ..+8)
  const int ar = tid >> 1, ac = (tid & 1) * 8;
  const int br = tid >> 4, bc = (tid & 15) * 8;
  double ra[8], rb[8];
  auto fetch = [&](int64_t k0) {
    const int64_t gr = row0 + ar;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int64_t gk = k0 + ac + i;
      ra[i] = (gr < M && gk < K) ? A[gr * lda + gk] : 0.0;
    }
    const int64_t gk = k0 + br;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int64_t gc = col0 + bc + i;
      rb[i] = (gk < K && gc < N) ? B[gk * ldb + gc] : 0.0;
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int i = 0; i < 8; ++i) As[buf][ar * kAP + ac + i] = ra[i];
#pragma unroll
    for (int i = 0; i < 8; ++i) Bs[buf][br * kBP + bc + i] = rb[i];
  };

  v4d acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

  const int li = lane & 15, lk = lane >> 4;
  const int64_t nk = (K + kBK - 1) / kBK;
  fetch(0);
  stash(0);
  __syncthreads();
  for (int64_t t = 0; t < nk; ++t) {
    const int buf = t & 1;
    if (t + 1 < nk) fetch((t + 1) * kBK);
#pragma unroll
    for (int kk = 0; kk < kBK; kk += 4) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[buf][(wm + i * 16 + li) * kAP + kk + lk];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[buf][(kk + lk) * kBP + wn + j * 16 + li];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (t + 1 < nk) {
      stash(buf ^ 1);
      __syncthreads();
    }
  }
  // epilogue: accumulator r of lane l is C[4 r + l/16][l % 16] of its block
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gr = row0 + wm + i * 16 + 4 * r + lk;
        const int64_t gc = col0 + wn + j * 16 + li;
        if (gr < M && gc < N) {
          double* c = C + gr * ldc + gc;
          *c = beta == 0.0 ? alpha * acc[i][j][r] : alpha * acc[i][j][r] + beta * *c;
        }
      }
}

}  // namespace

namespace sun {

void gemm_f64(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda, const double* B,
              int64_t ldb, double beta, double* C, int64_t ldc, hipStream_t s) {
  if (M <= 0 || N <= 0) return;
  const int64_t tiles = ((M + kBM - 1) / kBM) * ((N + kBN - 1) / kBN);
  SUN_REQUIRE(tiles < (int64_t)INT32_MAX, SUN_ENOTSUP, "matrix product too large for one launch");
  hipLaunchKernelGGL(k_gemm_f64, dim3((unsigned)tiles), dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb, beta, C,
                     ldc);
  HIP_LAUNCH_OK();
}

}  // namespace sun

extern "C" int sun_gemm_f64(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
                            const double* B, int64_t ldb, double beta, double* C, int64_t ldc, void* stream) {
  return guarded([&] {
    SUN_REQUIRE(M >= 0 && N >= 0 && K >= 0, SUN_EINVAL, "negative size");
    SUN_REQUIRE(M == 0 || N == 0 || (C != nullptr && ldc >= N), SUN_EINVAL, "C is NULL or ldc < N");
    SUN_REQUIRE(M == 0 || N == 0 || K == 0 || (A != nullptr && B != nullptr && lda >= K && ldb >= N), SUN_EINVAL,
                "A or B is NULL, or a leading dimension is too small");
    gemm_f64(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, as_stream(stream));
  });
}
