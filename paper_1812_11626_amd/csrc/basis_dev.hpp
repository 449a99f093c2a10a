// Closed forms of the SU(N) basis and of the triple traces
//     T(a,b,c) = Tr(F_a F_b F_c),   f_abc = 2 Im T,   d_abc = 2 Re T
// (from eq. 4: f_mns = -i Tr(F_s[F_m,F_n]) and d_mns = Tr(F_s{F_m,F_n}), and
// Tr(F_s F_n F_m) = conj Tr(F_s F_m F_n) for Hermitian generators).
//
// The paper states that the nonzero set of f and d is known analytically and
// that each coefficient costs O(1) (Sec. IV, step 2.2) without printing the
// rules.  They follow from the supports of the generators: S^(j,k), J^(j,k)
// live on the two entries (j,k), (k,j); D^l on the diagonal.  A product of
// three generators has a nonzero trace only if
//   (1) all three are off-diagonal and their edges form a triangle j,k,l, or
//   (2) two are off-diagonal on the same edge and the third is some D^l, or
//   (3) all three are diagonal,
// and in each case T is a short sum of products of generator entries.
#pragma once

#include "common.hpp"

namespace sun {

enum Kind : int { KS = 0, KJ = 1, KD = 2 };

struct Gen {
  int kind;  // KS, KJ or KD
  int j, k;  // pair (j<k) for KS/KJ; j = k = l for KD
};

struct BasisDev {
  int N;
  int P;              // N(N-1)/2
  int M;              // N^2 - 1
  const int* pj;      // pair index -> j
  const int* pk;      // pair index -> k
  const double* c;    // c[l] = 1/sqrt(l(l+1)), c[0] = 0
};

__host__ __device__ inline int pair_index(int N, int j, int k) {
  if (j > k) { int t = j; j = k; k = t; }
  return (int)((int64_t)j * (2 * (int64_t)N - j - 1) / 2 + (k - j - 1));
}

__device__ inline Gen decode(const BasisDev& B, int a) {
  Gen g;
  if (a < B.P) { g.kind = KS; g.j = B.pj[a]; g.k = B.pk[a]; }
  else if (a < 2 * B.P) { g.kind = KJ; g.j = B.pj[a - B.P]; g.k = B.pk[a - B.P]; }
  else { g.kind = KD; g.j = g.k = a - 2 * B.P + 1; }
  return g;
}

__device__ inline int encode_pair(const BasisDev& B, int kind, int j, int k) {
  return kind * B.P + pair_index(B.N, j, k);
}
__device__ inline int encode_diag(const BasisDev& B, int l) { return 2 * B.P + l - 1; }

// Diagonal entry x of D^l.
__device__ inline double dval(const BasisDev& B, int l, int x) {
  if (x < l) return B.c[l];
  if (x == l) return -(double)l * B.c[l];
  return 0.0;
}

// Entry (u,v), u != v, of the off-diagonal generator of the given kind on
// the edge {u,v}: S -> 1/sqrt2 on both; J -> -i/sqrt2 at (j,k), +i/sqrt2 at (k,j).
__device__ inline cplx pentry(int kind, int u, int v) {
  const double r = 0.70710678118654752440;
  if (kind == KS) return cx(r, 0.0);
  return (u < v) ? cx(0.0, -r) : cx(0.0, r);
}

// T for two off-diagonal generators on the same edge (p1 then p2) followed by
// D^l:  sum_x (p1)_{x y} (p2)_{y x} D[x] over x,y in {j,k}.
__device__ inline cplx trace_ppd(const BasisDev& B, int k1, int k2, int j, int k, int l) {
  cplx a = pentry(k1, j, k) * pentry(k2, k, j);
  cplx b = pentry(k1, k, j) * pentry(k2, j, k);
  return dval(B, l, j) * a + dval(B, l, k) * b;
}

// T for three diagonal generators: sum_x D_a[x] D_b[x] D_c[x], which is
// (1-a) c_a if a=b=c, c_r if the two smaller indices are equal (q=q<r), else 0.
__device__ inline double trace_ddd(const BasisDev& B, int a, int b, int c) {
  // sort a <= b <= c
  if (a > b) { int t = a; a = b; b = t; }
  if (b > c) { int t = b; b = c; c = t; }
  if (a > b) { int t = a; a = b; b = t; }
  if (a == b && b == c) return (1.0 - (double)a) * B.c[a];
  if (a == b) return B.c[c];
  return 0.0;
}

// General closed-form T(a,b,c) for decoded generators.
__device__ inline cplx trace3(const BasisDev& B, Gen a, Gen b, Gen c) {
  int nd = (a.kind == KD) + (b.kind == KD) + (c.kind == KD);
  if (nd == 3) return cx(trace_ddd(B, a.j, b.j, c.j));
  if (nd == 2) return cx(0.0);
  if (nd == 1) {
    // rotate (cyclic invariance of the trace) so that the diagonal one is last
    if (a.kind == KD) { Gen t = a; a = b; b = c; c = t; }
    else if (b.kind == KD) { Gen t = b; b = a; a = c; c = t; }
    // now c is diagonal; a, b must share their edge
    if (a.j != b.j || a.k != b.k) return cx(0.0);
    return trace_ppd(B, a.kind, b.kind, a.j, a.k, c.j);
  }
  // three off-diagonal generators: a closed walk x -> y -> z -> x
  for (int o = 0; o < 2; ++o) {
    int x = o ? a.k : a.j;
    int y = o ? a.j : a.k;
    int z;
    if (b.j == y) z = b.k;
    else if (b.k == y) z = b.j;
    else continue;
    if (z == x) continue;
    bool ok = (c.j == z && c.k == x) || (c.j == x && c.k == z);
    if (!ok) continue;
    return pentry(a.kind, x, y) * pentry(b.kind, y, z) * pentry(c.kind, z, x);
  }
  return cx(0.0);
}

__device__ inline cplx trace3_idx(const BasisDev& B, int a, int b, int c) {
  return trace3(B, decode(B, a), decode(B, b), decode(B, c));
}

}  // namespace sun
