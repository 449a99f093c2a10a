// Dense FP64 matrix product on the CDNA matrix cores:
//     C = alpha A B + beta C,   A: M x K,  B: K x N,  C: M x N,  row-major.
// The dense-operator assembly forms the dissipative part as one such product,
// R = -(1/2) Re(B^T A) = -(1/2) [Re B^T | -Im B^T] [Re A ; Im A], a dense
// contraction of M x 2M by 2M x M (Sec. II eq. 10 with dense sections).
//
// Tiling: a workgroup of four wavefronts computes a 128 x 128 tile of C,
// each wavefront a 64 x 64 quarter as 4 x 4 blocks of 16 x 16, with
// v_mfma_f64_16x16x4f64 (a 16 x 4 by 4 x 16 product per instruction, 4
// accumulators per lane).  K advances in panels of BK (16, or 32 for long
// products): the A panel (128 x BK) and B panel (BK x 128) are staged in LDS,
// double-buffered, the next panel fetched into registers (16-byte loads in
// the interior) while the current one is multiplied.  Operand
// layout of the instruction: lane l holds A[l % 16][l / 16] and B[l / 16][l %
// 16]; accumulator r of lane l is C[4 r + l / 16][l % 16] (checked on the
// device with one-hot operands).  Workgroups are
// numbered so that consecutive ones share a band of rows of A (groups of 8
// row tiles), which keeps the A band and the B panels they read in L2.
#include "internal.hpp"

using namespace sun;

namespace {

constexpr int kBM = 128, kBN = 128;
constexpr int kGroupM = 8;

typedef double v4d __attribute__((ext_vector_type(4)));

// BK: depth of the K panel staged per iteration (16 or 32).  Each thread
// stages BK/2 doubles of the A panel (row tid/2) and BK/2 of the B panel
// (row tid/(256/BK) ... ), as 16-byte loads where the panel is interior.
template <int BK>
__global__ __launch_bounds__(256) void k_gemm_f64(int64_t M, int64_t N, int64_t K, double alpha,
                                                  const double* __restrict__ A, int64_t lda,
                                                  const double* __restrict__ B, int64_t ldb, double beta,
                                                  double* __restrict__ C, int64_t ldc) {
  constexpr int AP = BK + 1;     // padded row of the A panel in LDS (row-major)
  constexpr int BP = kBN + 2;    // padded row of the B panel in LDS
  constexpr int AH = BK / 2;     // A doubles per thread: row tid/2, columns (tid%2)*AH ..
  constexpr int BT = 256 / BK;   // threads per B panel row
  constexpr int BW = kBN / BT;   // B doubles per thread
  __shared__ double As[2][kBM * AP];
  __shared__ double Bs[2][BK * BP];
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

  const int ar = tid >> 1, ac = (tid & 1) * AH;
  const int br = tid / BT, bc = (tid % BT) * BW;
  double ra[AH], rb[BW];
  const bool a_vec = (lda % 2 == 0) && ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
  const bool b_vec = (ldb % 2 == 0) && ((reinterpret_cast<uintptr_t>(B) & 15) == 0);
  auto fetch = [&](int64_t k0) {
    const int64_t gr = row0 + ar;
    const int64_t ga = k0 + ac;
    if (a_vec && gr < M && ga + AH <= K) {
      const double2* src = reinterpret_cast<const double2*>(A + gr * lda + ga);
#pragma unroll
      for (int i = 0; i < AH / 2; ++i) {
        const double2 t = src[i];
        ra[2 * i] = t.x;
        ra[2 * i + 1] = t.y;
      }
    } else {
#pragma unroll
      for (int i = 0; i < AH; ++i) ra[i] = (gr < M && ga + i < K) ? A[gr * lda + ga + i] : 0.0;
    }
    const int64_t gk = k0 + br;
    const int64_t gc = col0 + bc;
    if (b_vec && gk < K && gc + BW <= N) {
      const double2* src = reinterpret_cast<const double2*>(B + gk * ldb + gc);
#pragma unroll
      for (int i = 0; i < BW / 2; ++i) {
        const double2 t = src[i];
        rb[2 * i] = t.x;
        rb[2 * i + 1] = t.y;
      }
    } else {
#pragma unroll
      for (int i = 0; i < BW; ++i) rb[i] = (gk < K && gc + i < N) ? B[gk * ldb + gc + i] : 0.0;
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int i = 0; i < AH; ++i) As[buf][ar * AP + ac + i] = ra[i];
#pragma unroll
    for (int i = 0; i < BW; ++i) Bs[buf][br * BP + bc + i] = rb[i];
  };

  v4d acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

  const int li = lane & 15, lk = lane >> 4;
  const int64_t nk = (K + BK - 1) / BK;
  fetch(0);
  stash(0);
  __syncthreads();
  for (int64_t t = 0; t < nk; ++t) {
    const int buf = t & 1;
    if (t + 1 < nk) fetch((t + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[buf][(wm + i * 16 + li) * AP + kk + lk];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[buf][(kk + lk) * BP + wn + j * 16 + li];
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

// K panel depth used for products of at least kDeepK (longer loops amortise
// the per-iteration barrier and hide the global loads behind more matrix work)
constexpr int64_t kDeepK = 256;

}  // namespace

namespace sun {

void gemm_f64(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda, const double* B,
              int64_t ldb, double beta, double* C, int64_t ldc, hipStream_t s) {
  if (M <= 0 || N <= 0) return;
  const int64_t tiles = ((M + kBM - 1) / kBM) * ((N + kBN - 1) / kBN);
  SUN_REQUIRE(tiles < (int64_t)INT32_MAX, SUN_ENOTSUP, "matrix product too large for one launch");
  if (K >= kDeepK)
    hipLaunchKernelGGL(k_gemm_f64<32>, dim3((unsigned)tiles), dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb, beta,
                       C, ldc);
  else
    hipLaunchKernelGGL(k_gemm_f64<16>, dim3((unsigned)tiles), dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb, beta,
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
