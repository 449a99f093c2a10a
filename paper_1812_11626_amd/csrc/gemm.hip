// Dense FP64 matrix product on the CDNA matrix cores:
//     C = alpha A B + beta C,   A: M x K,  B: K x N,  C: M x N,  row-major.
// The dense-operator assembly forms the dissipative part as one such product,
// R = -(1/2) Re(B^T A) = -(1/2) [Re B^T | -Im B^T] [Re A ; Im A], a dense
// contraction of M x 2M by 2M x M (Sec. II eq. 10 with dense sections).
//
// Tiling: a workgroup of four wavefronts (two workgroups per CU: 214
// registers per lane, 72 KiB of LDS each, so one workgroup's barrier and
// panel writes overlap the other's products) computes a 128 x 128 tile of
// C, each wavefront a 64 x 64 block as 4 x 4 blocks of 16 x 16 with
// v_mfma_f64_16x16x4f64 (a 16 x 4 by 4 x 16 product per instruction, 4
// accumulators per lane).  K advances in panels of 16: the A panel
// (128 x 16) and the B panel (16 x 128) are staged in LDS k-major (A
// transposed on the way in), each
// row padded to 16 mod 32 doubles so that the four k-rows one fragment read
// touches fall on disjoint banks; the LDS panels are double-buffered and the
// next panel is fetched into registers (16-byte loads in the interior)
// while the current one is multiplied, with the fragments of the next
// k-step read from LDS while the current step's 16 products run.  Operand
// layout of the instruction: lane l holds A[l % 16][l / 16] and B[l / 16][l %
// 16]; accumulator r of lane l is C[4 r + l / 16][l % 16] (checked on the
// device with one-hot operands).  Workgroups are numbered so that
// consecutive ones share a band of rows of A (groups of 8 row tiles), which
// keeps the A band and the B panels they read in L2.
#include "internal.hpp"

using namespace sun;

namespace {

constexpr int kBM = 128, kBN = 128, kBK = 16;
constexpr int kWavesM = 2, kWavesN = 2;
constexpr int kThreads = 64 * kWavesM * kWavesN;
constexpr int kGroupM = 8;
constexpr int kPadA = 16, kPadB = 16;        // (kBM + kPadA) and (kBN + kPadB) are 16 mod 32
static_assert((kBM + kPadA) % 32 == 16 && (kBN + kPadB) % 32 == 16, "bank-disjoint k-rows");

typedef double v4d __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kThreads, 2) void k_gemm_f64(int64_t M, int64_t N, int64_t K, double alpha,
                                                       const double* __restrict__ A, int64_t lda,
                                                       const double* __restrict__ B, int64_t ldb, double beta,
                                                       double* __restrict__ C, int64_t ldc) {
  constexpr int TM = kBM / kWavesM, TN = kBN / kWavesN;   // 64 x 64 per wavefront
  constexpr int FM = TM / 16, FN = TN / 16;
  constexpr int SA = kBM + kPadA, SB = kBN + kPadB;       // LDS row strides (k-major panels)
  constexpr int NA = kBM * kBK / kThreads;                 // A doubles fetched per thread (one row, NA k's)
  constexpr int NB = kBK * kBN / kThreads;                 // B doubles fetched per thread (one k, NB columns)
  constexpr int APR = kBK / NA, BPR = kBN / NB;            // threads per A row / per B row
  __shared__ double As[2][kBK * SA];
  __shared__ double Bs[2][kBK * SB];
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
  const int wm = (wave / kWavesN) * TM, wn = (wave % kWavesN) * TN;
  const int li = lane & 15, lk = lane >> 4;
  const int a_r = tid / APR, a_k = (tid % APR) * NA;
  const int b_k = tid / BPR, b_n = (tid % BPR) * NB;
  double ra[NA], rb[NB];
  const bool a_vec = (lda % 2 == 0) && ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
  const bool b_vec = (ldb % 2 == 0) && ((reinterpret_cast<uintptr_t>(B) & 15) == 0);
  auto fetch = [&](int64_t k0) {
    const int64_t gr = row0 + a_r, gk = k0 + a_k;
    if (a_vec && gr < M && gk + NA <= K) {
      const double2* src = reinterpret_cast<const double2*>(A + gr * lda + gk);
#pragma unroll
      for (int i = 0; i < NA / 2; ++i) {
        const double2 t = src[i];
        ra[2 * i] = t.x;
        ra[2 * i + 1] = t.y;
      }
    } else {
#pragma unroll
      for (int i = 0; i < NA; ++i) ra[i] = (gr < M && gk + i < K) ? A[gr * lda + gk + i] : 0.0;
    }
    const int64_t bk = k0 + b_k, bn = col0 + b_n;
    if (b_vec && bk < K && bn + NB <= N) {
      const double2* src = reinterpret_cast<const double2*>(B + bk * ldb + bn);
#pragma unroll
      for (int i = 0; i < NB / 2; ++i) {
        const double2 t = src[i];
        rb[2 * i] = t.x;
        rb[2 * i + 1] = t.y;
      }
    } else {
#pragma unroll
      for (int i = 0; i < NB; ++i) rb[i] = (bk < K && bn + i < N) ? B[bk * ldb + bn + i] : 0.0;
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int i = 0; i < NA; ++i) As[buf][(a_k + i) * SA + a_r] = ra[i];
#pragma unroll
    for (int i = 0; i < NB; ++i) Bs[buf][b_k * SB + b_n + i] = rb[i];
  };

  v4d acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

  const int64_t nk = (K + kBK - 1) / kBK;
  fetch(0);
  stash(0);
  __syncthreads();
  for (int64_t t = 0; t < nk; ++t) {
    const int buf = t & 1;
    if (t + 1 < nk) fetch((t + 1) * kBK);
    double a[2][FM], b[2][FN];   // fragments of the current and the next k-step
#pragma unroll
    for (int i = 0; i < FM; ++i) a[0][i] = As[buf][lk * SA + wm + i * 16 + li];
#pragma unroll
    for (int j = 0; j < FN; ++j) b[0][j] = Bs[buf][lk * SB + wn + j * 16 + li];
#pragma unroll
    for (int kk = 0; kk < kBK; kk += 4) {
      const int c = (kk / 4) & 1;
      if (kk + 4 < kBK) {
#pragma unroll
        for (int i = 0; i < FM; ++i) a[c ^ 1][i] = As[buf][(kk + 4 + lk) * SA + wm + i * 16 + li];
#pragma unroll
        for (int j = 0; j < FN; ++j) b[c ^ 1][j] = Bs[buf][(kk + 4 + lk) * SB + wn + j * 16 + li];
      }
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[c][i], b[c][j], acc[i][j], 0, 0, 0);
    }
    if (t + 1 < nk) {
      stash(buf ^ 1);
      __syncthreads();
    }
  }
  // epilogue: accumulator r of lane l is C[4 r + l/16][l % 16] of its block
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
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
  hipLaunchKernelGGL(k_gemm_f64, dim3((unsigned)tiles), dim3(kThreads), 0, s, M, N, K, alpha, A, lda, B, ldb, beta,
                     C, ldc);
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
