// Library objects shared between translation units.
#pragma once

#include "basis_dev.hpp"
#include "common.hpp"

struct sun_basis_s {
  int N = 0;
  int P = 0;
  int64_t M = 0;
  int device = 0;
  sun::DevBuf<int> pj, pk;     // pair -> (j, k)
  sun::DevBuf<double> c;       // c[l] = 1/sqrt(l(l+1))
  sun::BasisDev view() const {
    sun::BasisDev B;
    B.N = N; B.P = P; B.M = (int)M;
    B.pj = pj.get(); B.pk = pk.get(); B.c = c.get();
    return B;
  }
};

namespace sun {

// Real CSR matrix owned by the library (M x M, sorted unique columns).
struct DevCSR {
  int64_t rows = 0;
  int64_t nnz = 0;
  DevBuf<int> rowptr;
  DevBuf<int> col;
  DevBuf<double> val;
};

// Complex CSR matrix (intermediate sections of the dissipator).
struct DevZCSR {
  int64_t rows = 0;
  int64_t nnz = 0;
  DevBuf<int> rowptr;
  DevBuf<int> col;
  DevBuf<cplx> val;
};

// Expansion of one N x N operator: coefficients, trace, symmetric pattern.
struct Expansion {
  DevBuf<cplx> x;        // [M] x_m = Tr(F_m X)
  DevBuf<cplx> xd;       // [N] sum_l x_{D_l} D_l[i]
  DevBuf<int> adj_ptr;   // [N+1] symmetric off-diagonal pattern of X
  DevBuf<int> adj_idx;
  cplx trace{0, 0};
  double maxabs = 0.0;   // max |X_ij|
  double herm_dev = 0.0; // max |X_ij - conj X_ji| (computed on request)
};

void expand_operator(const sun_basis_s& b, const sun_zcsr& X, Expansion& e,
                     bool want_hermiticity, hipStream_t s);

// C = alpha A B + beta C, FP64, row-major, on the matrix cores (gemm.hip).
void gemm_f64(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda, const double* B,
              int64_t ldb, double beta, double* C, int64_t ldc, hipStream_t s);

}  // namespace sun

struct sun_lind_s {
  const sun_basis_s* basis = nullptr;
  int nH = 0, P = 0;
  std::vector<sun::DevCSR> QH;        // [nH]
  std::vector<sun::DevCSR> R;         // [P], unit rate
  std::vector<sun::DevBuf<double>> K; // [P], unit rate, length M
};
