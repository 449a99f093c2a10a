/*
 * Oracle tier O2 -- TEST INFRASTRUCTURE ONLY (see oracle/__init__.py): used by
 * tests/, __graft_entry__.smoke() and the cpu_baseline leg of bench.py, never
 * by the library.  Plain C99 + OpenMP, double precision, written from the
 * definitions in the paper; shares nothing with the HIP path.
 *
 * 1. The Bloch-form generator by explicit traces (paper Sec. II, eqs. 5, 9):
 *    with rho = 1/N + sum_m v_m F_m and Tr(F_s F_m) = delta_sm,
 *        column m of Q_H :  Tr(F_s (-i [H, F_m]))          (eq. 6)
 *        column m of R_L :  Tr(F_s D_L(F_m)),  D_L(X) = L X L^+ - {L^+ L, X}/2
 *                                                          (eq. 10, unit rate)
 *        K_L             :  Tr(F_s D_L(1)) / N              (eq. 11, unit rate)
 *    Each column is formed as the sparse N x N matrix Y = generator(F_m) from
 *    the few entries of F_m (two for S and J, l+1 for D_l) and the operator's
 *    CSR, then projected onto the basis by index arithmetic:
 *        Tr(S^(j,k) Y) = (Y_jk + Y_kj)/sqrt2,  Tr(J^(j,k) Y) = i (Y_jk - Y_kj)/sqrt2,
 *        Tr(D^l Y)     = (sum_{i<l} Y_ii - l Y_ll) / sqrt(l(l+1)).
 *    No structure constant appears anywhere.  Generator order (grouped): S of
 *    pair p = j(2N-j-1)/2 + k-j-1 at p, J at P+p, D^l at 2P+l-1.
 *
 * 2. Classical RK4 (Sec. IV step 3.1) on dv/dt = (G0 + sum_a c_a(t) G_a) v + K
 *    with CSR matrices, the coefficients tabulated on the half-step grid
 *    (rows 2n, 2n+1, 2n+1, 2n+2 for the stages of step n), rows of every
 *    product split over OpenMP threads.  This is the multi-core CPU timing
 *    baseline.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

typedef struct {
  int32_t n;
  const int32_t* rowptr;
  const int32_t* col;
  const double* re;
  const double* im; /* may be NULL */
} o2_op;

/* ---- small helpers ------------------------------------------------------ */

typedef struct {
  int32_t r, c;
  cplx v;
} entry;

typedef struct {
  entry* e;
  int64_t n, cap;
} elist;

static int el_push(elist* l, int32_t r, int32_t c, cplx v) {
  if (l->n == l->cap) {
    int64_t cap = l->cap ? 2 * l->cap : 256;
    entry* e = (entry*)realloc(l->e, (size_t)cap * sizeof(entry));
    if (!e) return -1;
    l->e = e;
    l->cap = cap;
  }
  l->e[l->n].r = r;
  l->e[l->n].c = c;
  l->e[l->n].v = v;
  l->n++;
  return 0;
}

static int cmp_entry(const void* a, const void* b) {
  const entry* x = (const entry*)a;
  const entry* y = (const entry*)b;
  if (x->r != y->r) return x->r < y->r ? -1 : 1;
  if (x->c != y->c) return x->c < y->c ? -1 : 1;
  return 0;
}

/* sort by (r, c) and add up equal positions; returns the merged count */
static int64_t el_merge(elist* l) {
  if (l->n == 0) return 0;
  qsort(l->e, (size_t)l->n, sizeof(entry), cmp_entry);
  int64_t w = 0;
  for (int64_t i = 1; i < l->n; ++i) {
    if (l->e[i].r == l->e[w].r && l->e[i].c == l->e[w].c)
      l->e[w].v += l->e[i].v;
    else
      l->e[++w] = l->e[i];
  }
  l->n = w + 1;
  return l->n;
}

/* complex CSR owned here */
typedef struct {
  int32_t n;
  int32_t* rowptr;
  int32_t* col;
  cplx* val;
} zmat;

static void zm_free(zmat* m) {
  free(m->rowptr);
  free(m->col);
  free(m->val);
  memset(m, 0, sizeof(*m));
}

/* CSR from a merged entry list (sorted by row, then column) */
static int zm_from_list(int32_t n, const elist* l, zmat* out) {
  out->n = n;
  out->rowptr = (int32_t*)calloc((size_t)n + 1, sizeof(int32_t));
  out->col = (int32_t*)malloc((size_t)(l->n > 0 ? l->n : 1) * sizeof(int32_t));
  out->val = (cplx*)malloc((size_t)(l->n > 0 ? l->n : 1) * sizeof(cplx));
  if (!out->rowptr || !out->col || !out->val) return -1;
  for (int64_t i = 0; i < l->n; ++i) out->rowptr[l->e[i].r + 1]++;
  for (int32_t r = 0; r < n; ++r) out->rowptr[r + 1] += out->rowptr[r];
  for (int64_t i = 0; i < l->n; ++i) {
    out->col[i] = l->e[i].c;
    out->val[i] = l->e[i].v;
  }
  return 0;
}

static int zm_from_op(const o2_op* op, zmat* out) {
  elist l = {0};
  for (int32_t r = 0; r < op->n; ++r)
    for (int32_t e = op->rowptr[r]; e < op->rowptr[r + 1]; ++e)
      if (el_push(&l, r, op->col[e], op->re[e] + I * (op->im ? op->im[e] : 0.0))) return -1;
  el_merge(&l);
  int st = zm_from_list(op->n, &l, out);
  free(l.e);
  return st;
}

/* transpose (not conjugated) */
static int zm_transpose(const zmat* a, zmat* out) {
  elist l = {0};
  for (int32_t r = 0; r < a->n; ++r)
    for (int32_t e = a->rowptr[r]; e < a->rowptr[r + 1]; ++e)
      if (el_push(&l, a->col[e], r, a->val[e])) return -1;
  el_merge(&l);
  int st = zm_from_list(a->n, &l, out);
  free(l.e);
  return st;
}

/* A = L^+ L:  A_ac = sum_k conj(L_ka) L_kc */
static int zm_adjoint_product(const zmat* L, zmat* out) {
  elist l = {0};
  for (int32_t k = 0; k < L->n; ++k)
    for (int32_t e = L->rowptr[k]; e < L->rowptr[k + 1]; ++e)
      for (int32_t f = L->rowptr[k]; f < L->rowptr[k + 1]; ++f)
        if (el_push(&l, L->col[e], L->col[f], conj(L->val[e]) * L->val[f])) return -1;
  el_merge(&l);
  int st = zm_from_list(L->n, &l, out);
  free(l.e);
  return st;
}

/* entries of generator m (grouped order) */
static int gen_entries(int32_t N, int64_t m, elist* F) {
  const int64_t P = (int64_t)N * (N - 1) / 2;
  const double r2 = 1.0 / sqrt(2.0);
  F->n = 0;
  if (m < 2 * P) {
    int64_t q = m < P ? m : m - P;
    int32_t j = 0;
    while (q >= N - 1 - j) {
      q -= N - 1 - j;
      ++j;
    }
    const int32_t k = (int32_t)(j + 1 + q);
    if (m < P) {
      if (el_push(F, j, k, r2) || el_push(F, k, j, r2)) return -1;
    } else {
      if (el_push(F, j, k, -I * r2) || el_push(F, k, j, I * r2)) return -1;
    }
  } else {
    const int32_t l = (int32_t)(m - 2 * P + 1);
    const double c = 1.0 / sqrt((double)l * (l + 1.0));
    for (int32_t i = 0; i < l; ++i)
      if (el_push(F, i, i, c)) return -1;
    if (el_push(F, l, l, -(double)l * c)) return -1;
  }
  return 0;
}

/* Y = generator applied to the sparse X (entries of F), into Y (merged) */
typedef struct {
  int kind;      /* 0: -i[H, X];  1: L X L^+ - {L^+L, X}/2 */
  zmat A, AT;    /* H (kind 0) or L (kind 1), and its transpose */
  zmat B, BT;    /* kind 1: L^+ L and its transpose */
} gen_ctx;

static int apply_gen(const gen_ctx* g, const elist* X, elist* Y) {
  Y->n = 0;
  for (int64_t t = 0; t < X->n; ++t) {
    const int32_t a = X->e[t].r, b = X->e[t].c;
    const cplx x = X->e[t].v;
    if (g->kind == 0) {
      /* (H X)_rb += H_ra x  (column a of H = row a of H^T) */
      for (int32_t e = g->AT.rowptr[a]; e < g->AT.rowptr[a + 1]; ++e)
        if (el_push(Y, g->AT.col[e], b, -I * g->AT.val[e] * x)) return -1;
      /* (X H)_ac += x H_bc */
      for (int32_t e = g->A.rowptr[b]; e < g->A.rowptr[b + 1]; ++e)
        if (el_push(Y, a, g->A.col[e], I * x * g->A.val[e])) return -1;
    } else {
      /* (L X L^+)_rc += L_ra x conj(L_cb) */
      for (int32_t e = g->AT.rowptr[a]; e < g->AT.rowptr[a + 1]; ++e)
        for (int32_t f = g->AT.rowptr[b]; f < g->AT.rowptr[b + 1]; ++f)
          if (el_push(Y, g->AT.col[e], g->AT.col[f], g->AT.val[e] * x * conj(g->AT.val[f]))) return -1;
      /* -(1/2)(L^+L X)_rb = -(1/2) B_ra x */
      for (int32_t e = g->BT.rowptr[a]; e < g->BT.rowptr[a + 1]; ++e)
        if (el_push(Y, g->BT.col[e], b, -0.5 * g->BT.val[e] * x)) return -1;
      /* -(1/2)(X L^+L)_ac = -(1/2) x B_bc */
      for (int32_t e = g->B.rowptr[b]; e < g->B.rowptr[b + 1]; ++e)
        if (el_push(Y, a, g->B.col[e], -0.5 * x * g->B.val[e])) return -1;
    }
  }
  el_merge(Y);
  return 0;
}

/* Bloch coordinates Tr(F_s Y) of the merged sparse Y, appended to (rows,
 * vals) as (s, value) pairs with a nonzero real part; |Im| is tracked in
 * *max_im.  The D coordinates need prefix sums of the diagonal: l runs over
 * the range where they can be nonzero (beyond the last diagonal entry the
 * prefix is the trace, exactly 0 for a traceless Y, and only rounding noise
 * when it is dropped for |Tr Y| <= 1e-14 max|Y|). */
typedef struct {
  int32_t* s;
  double* v;
  int64_t n, cap;
} col_out;

static int co_push(col_out* o, int32_t s, double v) {
  if (o->n == o->cap) {
    int64_t cap = o->cap ? 2 * o->cap : 256;
    int32_t* ns = (int32_t*)realloc(o->s, (size_t)cap * sizeof(int32_t));
    if (!ns) return -1;
    o->s = ns;
    double* nv = (double*)realloc(o->v, (size_t)cap * sizeof(double));
    if (!nv) return -1;
    o->v = nv;
    o->cap = cap;
  }
  o->s[o->n] = s;
  o->v[o->n] = v;
  o->n++;
  return 0;
}

static int project(int32_t N, const elist* Y, col_out* out, double* max_im, elist* scratch) {
  const int64_t P = (int64_t)N * (N - 1) / 2;
  const double r2 = 1.0 / sqrt(2.0);
  double maxabs = 0.0;
  for (int64_t t = 0; t < Y->n; ++t) maxabs = fmax(maxabs, cabs(Y->e[t].v));
  /* off-diagonal: (generator index, value) in a scratch list keyed by r = index */
  scratch->n = 0;
  int32_t dmin = N, dmax = -1;
  for (int64_t t = 0; t < Y->n; ++t) {
    const int32_t a = Y->e[t].r, b = Y->e[t].c;
    const cplx y = Y->e[t].v;
    if (a == b) {
      if (a < dmin) dmin = a;
      if (a > dmax) dmax = a;
      continue;
    }
    const int32_t j = a < b ? a : b, k = a < b ? b : a;
    const int64_t p = (int64_t)j * (2 * N - j - 1) / 2 + (k - j - 1);
    if (el_push(scratch, (int32_t)p, 0, y * r2)) return -1;
    if (el_push(scratch, (int32_t)(P + p), 0, (a < b ? I : -I) * y * r2)) return -1;
  }
  el_merge(scratch);
  for (int64_t t = 0; t < scratch->n; ++t) {
    *max_im = fmax(*max_im, fabs(cimag(scratch->e[t].v)));
    const double v = creal(scratch->e[t].v);
    if (v != 0.0 && co_push(out, scratch->e[t].r, v)) return -1;
  }
  if (dmax < 0) return 0;
  /* diagonal: dense over [dmin, dmax] */
  const int32_t w = dmax - dmin + 1;
  cplx* d = (cplx*)calloc((size_t)w, sizeof(cplx));
  if (!d) return -1;
  for (int64_t t = 0; t < Y->n; ++t)
    if (Y->e[t].r == Y->e[t].c) d[Y->e[t].r - dmin] += Y->e[t].v;
  cplx tr = 0.0;
  for (int32_t i = 0; i < w; ++i) tr += d[i];
  const int32_t lend = cabs(tr) > 1e-14 * maxabs ? N - 1 : dmax;
  cplx prefix = 0.0; /* sum_{i<l} Y_ii */
  for (int32_t l = 1; l <= lend; ++l) {
    const int32_t i = l - 1;
    if (i >= dmin && i <= dmax) prefix += d[i - dmin];
    if (l < dmin) continue;
    const cplx yl = (l >= dmin && l <= dmax) ? d[l - dmin] : 0.0;
    const cplx val = (prefix - (double)l * yl) / sqrt((double)l * (l + 1.0));
    *max_im = fmax(*max_im, fabs(cimag(val)));
    if (creal(val) != 0.0 && co_push(out, (int32_t)(2 * P + l - 1), creal(val))) {
      free(d);
      return -1;
    }
  }
  free(d);
  return 0;
}

static int ctx_init(int kind, const o2_op* op, gen_ctx* g) {
  memset(g, 0, sizeof(*g));
  g->kind = kind;
  if (zm_from_op(op, &g->A) || zm_transpose(&g->A, &g->AT)) return -1;
  if (kind == 1) {
    if (zm_adjoint_product(&g->A, &g->B) || zm_transpose(&g->B, &g->BT)) return -1;
  }
  return 0;
}

static void ctx_free(gen_ctx* g) {
  zm_free(&g->A);
  zm_free(&g->AT);
  zm_free(&g->B);
  zm_free(&g->BT);
}

/* ---- exported ----------------------------------------------------------- */

/* Columns of Q (kind 0, op = H) or R (kind 1, op = L, unit rate) as COO,
 * column-major: col_ptr[M+1] (caller, int64), then *rows / *vals allocated
 * here (free with o2_free).  *max_im: largest |Im| seen (must be rounding
 * noise).  threads <= 0: OpenMP default.  Returns 0, or -1 when out of
 * memory. */
int o2_columns(int kind, const o2_op* op, int threads, int64_t* col_ptr, int32_t** rows, double** vals,
               double* max_im) {
  const int32_t N = op->n;
  const int64_t M = (int64_t)N * N - 1;
  gen_ctx g;
  if (ctx_init(kind, op, &g)) return -1;
#ifdef _OPENMP
  const int nt = threads > 0 ? threads : omp_get_max_threads();
#else
  const int nt = 1;
  (void)threads;
#endif
  /* columns split into nt contiguous ranges, one output list per range */
  col_out* outs = (col_out*)calloc((size_t)nt, sizeof(col_out));
  int64_t* cnt = (int64_t*)calloc((size_t)M + 1, sizeof(int64_t));
  double* mi = (double*)calloc((size_t)nt, sizeof(double));
  int* tfail = (int*)calloc((size_t)nt, sizeof(int));
  int fail = (!outs || !cnt || !mi || !tfail);
  if (!fail) {
#ifdef _OPENMP
#pragma omp parallel num_threads(nt)
#endif
    {
#ifdef _OPENMP
      const int t = omp_get_thread_num();
#else
      const int t = 0;
#endif
      const int64_t m0 = M * t / nt, m1 = M * (t + 1) / nt;
      elist F = {0}, Y = {0}, sc = {0};
      for (int64_t m = m0; m < m1; ++m) {
        const int64_t before = outs[t].n;
        if (gen_entries(N, m, &F) || apply_gen(&g, &F, &Y) || project(N, &Y, &outs[t], &mi[t], &sc)) {
          tfail[t] = 1;
          break;
        }
        cnt[m + 1] = outs[t].n - before;
      }
      free(F.e);
      free(Y.e);
      free(sc.e);
    }
    for (int t = 0; t < nt; ++t) fail |= tfail[t];
  }
  int64_t total = 0;
  if (!fail) {
    col_ptr[0] = 0;
    for (int64_t m = 0; m < M; ++m) col_ptr[m + 1] = col_ptr[m] + cnt[m + 1];
    total = col_ptr[M];
    *rows = (int32_t*)malloc((size_t)(total > 0 ? total : 1) * sizeof(int32_t));
    *vals = (double*)malloc((size_t)(total > 0 ? total : 1) * sizeof(double));
    fail = !*rows || !*vals;
  }
  if (!fail) {
    int64_t o = 0;
    double worst = 0.0;
    for (int t = 0; t < nt; ++t) {
      memcpy(*rows + o, outs[t].s, (size_t)outs[t].n * sizeof(int32_t));
      memcpy(*vals + o, outs[t].v, (size_t)outs[t].n * sizeof(double));
      o += outs[t].n;
      worst = fmax(worst, mi[t]);
    }
    *max_im = worst;
  }
  if (outs)
    for (int t = 0; t < nt; ++t) {
      free(outs[t].s);
      free(outs[t].v);
    }
  free(outs);
  free(cnt);
  free(mi);
  free(tfail);
  ctx_free(&g);
  return fail ? -1 : 0;
}

/* K_s = Tr(F_s D_L(1)) / N at unit rate, into k[M] (zero-filled here). */
int o2_k_vector(const o2_op* op, double* k, double* max_im) {
  const int32_t N = op->n;
  const int64_t M = (int64_t)N * N - 1;
  gen_ctx g;
  if (ctx_init(1, op, &g)) return -1;
  elist X = {0}, Y = {0}, sc = {0};
  col_out o = {0};
  int fail = 0;
  for (int32_t i = 0; i < N && !fail; ++i) fail = el_push(&X, i, i, 1.0);
  double mi = 0.0;
  if (!fail) fail = apply_gen(&g, &X, &Y) || project(N, &Y, &o, &mi, &sc);
  if (!fail) {
    memset(k, 0, (size_t)M * sizeof(double));
    for (int64_t t = 0; t < o.n; ++t) k[o.s[t]] = o.v[t] / N;
    *max_im = mi / N;
  }
  free(X.e);
  free(Y.e);
  free(sc.e);
  free(o.s);
  free(o.v);
  ctx_free(&g);
  return fail ? -1 : 0;
}

void o2_free(void* p) { free(p); }

/* Classical RK4 for dv/dt = (sum_a c_a(t) G_a) v + sum_a c_a(t) K_a, where
 * term a has the CSR matrix (rowptr[a], col[a], val[a]) (M x M) and the free
 * vector K[a] (length M, or NULL), and c_a(t) is column a of the table coef
 * (2*steps+1 rows of nterm values; rows 2n, 2n+1, 2n+1, 2n+2 for the stages
 * of step n).  v (length M) is advanced in place by `steps` steps of size dt;
 * threads <= 0: OpenMP default.  Returns 0, or -1 when out of memory. */
int o2_rk4(int64_t M, int nterm, const int32_t* const* rowptr, const int32_t* const* col,
           const double* const* val, const double* const* K, const double* coef, double dt, int64_t steps,
           double* v, int threads) {
  double* k1 = (double*)malloc((size_t)M * sizeof(double));
  double* k2 = (double*)malloc((size_t)M * sizeof(double));
  double* k3 = (double*)malloc((size_t)M * sizeof(double));
  double* k4 = (double*)malloc((size_t)M * sizeof(double));
  double* x = (double*)malloc((size_t)M * sizeof(double));
  if (!k1 || !k2 || !k3 || !k4 || !x) {
    free(k1); free(k2); free(k3); free(k4); free(x);
    return -1;
  }
#ifdef _OPENMP
  const int nt = threads > 0 ? threads : omp_get_max_threads();
#else
  const int nt = 1;
  (void)threads;
#endif
  for (int64_t n = 0; n < steps; ++n) {
    const double* c0 = coef + (2 * n) * nterm;
    const double* ch = coef + (2 * n + 1) * nterm;
    const double* c1 = coef + (2 * n + 2) * nterm;
    /* k = G(c) xin + K(c) */
#define RHS(kout, xin, c)                                                         \
    do {                                                                          \
      _Pragma("omp parallel for num_threads(nt) schedule(static)")                \
      for (int64_t r = 0; r < M; ++r) {                                           \
        double s = 0.0;                                                           \
        for (int a = 0; a < nterm; ++a) {                                         \
          double t = 0.0;                                                         \
          for (int32_t e = rowptr[a][r]; e < rowptr[a][r + 1]; ++e)               \
            t += val[a][e] * (xin)[col[a][e]];                                    \
          if (K[a]) t += K[a][r];                                                 \
          s += (c)[a] * t;                                                        \
        }                                                                         \
        (kout)[r] = s;                                                            \
      }                                                                           \
    } while (0)
    RHS(k1, v, c0);
#pragma omp parallel for num_threads(nt) schedule(static)
    for (int64_t r = 0; r < M; ++r) x[r] = v[r] + 0.5 * dt * k1[r];
    RHS(k2, x, ch);
#pragma omp parallel for num_threads(nt) schedule(static)
    for (int64_t r = 0; r < M; ++r) x[r] = v[r] + 0.5 * dt * k2[r];
    RHS(k3, x, ch);
#pragma omp parallel for num_threads(nt) schedule(static)
    for (int64_t r = 0; r < M; ++r) x[r] = v[r] + dt * k3[r];
    RHS(k4, x, c1);
#pragma omp parallel for num_threads(nt) schedule(static)
    for (int64_t r = 0; r < M; ++r) v[r] = v[r] + (dt / 6.0) * (k1[r] + 2.0 * k2[r] + 2.0 * k3[r] + k4[r]);
#undef RHS
  }
  free(k1); free(k2); free(k3); free(k4); free(x);
  return 0;
}

/* Number of OpenMP threads a parallel region would use by default. */
int o2_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
