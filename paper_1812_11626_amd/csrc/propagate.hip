// Classical RK4 on the Bloch ODE dv/dt = G(t) v + K(t) (eq. 9; Sec. IV
// step 3.1) with one fused sparse-matrix-vector + stage-update kernel per RK4
// stage.
//
// Fused matrix layout.  All terms with constant weight are merged into one
// CSR row ("static segment"); the free vector K is folded in as an extra
// column with index M that multiplies a constant 1 stored at x[M]; then each
// time-dependent term contributes one further segment of the row.  Per row
// r: [rowptr[r], seg[0][r]) static, [seg[d][r], seg[d+1][r]) dynamic term d
// (the last one ending at rowptr[r+1]).  So a stage computes
//     k_r = sum_static + sum_d c_d(t) sum_dyn_d,
// reading every matrix byte once and no separate K vector.
//
// Kernels, by layout of that matrix (chosen at creation, retunable):
//  * sliced ELL (k_rk4_sell; large generators, at most one time-dependent
//    term): rows packed 64 per slice, one lane per row, compressed column
//    offsets, one wavefront per slice, each XCD on a contiguous slice range;
//  * segmented sliced ELL (k_sell_seg; 2-3 time-dependent terms): the same
//    with each time-dependent term as its own segment of the lane's row;
//  * CSR stream (k_rk4_stage; small generators, or 4 terms): the rows cut
//    into blocks of about `block_nnz` nonzeros; a workgroup streams its
//    block's values and columns with unit stride, multiplies by the gathered
//    x, parks the products in LDS, then one lane per row sums its segments;
//  * resident (k_rk4_resident; tiny generators): one workgroup keeps the
//    state in LDS and runs all steps of a call in one launch.
// Every layout sums a row's segments in nonzero order and applies the RK4
// stage update in the same pass, so the row-wise vectors (v, the
// accumulator, the next stage input) are touched once per stage.
//
// Stage arithmetic (same order as the textbook formula):
//   s=1: x2 = v + dt/2 k1,  acc = k1
//   s=2: x3 = v + dt/2 k2,  acc = acc + 2 k2
//   s=3: x4 = v + dt   k3,  acc = acc + 2 k3
//   s=4: v  = v + dt/6 (acc + k4)
#include <algorithm>
#include <cmath>
#include <atomic>
#include <mutex>

#include "internal.hpp"

using namespace sun;

#include "prop_internal.hpp"
#include "readout.hpp"


namespace {

constexpr int kMaxTerms = 32;
constexpr int kMaxDyn = 4;
constexpr int kThreads = 256;

struct TermList {
  int n;
  const int* rowptr[kMaxTerms];
  const int* col[kMaxTerms];
  const double* val[kMaxTerms];
  double w[kMaxTerms];
};

struct DynList {
  int n;
  const int* rowptr[kMaxDyn];
  const int* col[kMaxDyn];
  const double* val[kMaxDyn];
  const double* K[kMaxDyn];   // free vector of a dynamic dissipator term or NULL
};

// Row sizes (mode 0) or row contents (mode 1) of the fused matrix.
__global__ void k_fuse_rows(int64_t M, TermList st, const double* __restrict__ Kst, DynList dy, int mode,
                            int64_t* __restrict__ cnt, const int64_t* __restrict__ off,
                            int* __restrict__ col, double* __restrict__ val, int* __restrict__ seg) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < M;
       r += (int64_t)gridDim.x * blockDim.x) {
    int pos[kMaxTerms];
    for (int a = 0; a < st.n; ++a) pos[a] = st.rowptr[a][r];
    int64_t w = mode ? off[r] : 0;
    int64_t n = 0;
    while (true) {
      int cmin = INT32_MAX;
      for (int a = 0; a < st.n; ++a)
        if (pos[a] < st.rowptr[a][r + 1]) cmin = min(cmin, st.col[a][pos[a]]);
      if (cmin == INT32_MAX) break;
      double s = 0.0;
      for (int a = 0; a < st.n; ++a)
        if (pos[a] < st.rowptr[a][r + 1] && st.col[a][pos[a]] == cmin) {
          s += st.w[a] * st.val[a][pos[a]];
          ++pos[a];
        }
      if (mode) { col[w + n] = cmin; val[w + n] = s; }
      ++n;
    }
    if (Kst && Kst[r] != 0.0) {
      if (mode) { col[w + n] = (int)M; val[w + n] = Kst[r]; }
      ++n;
    }
    for (int d = 0; d < dy.n; ++d) {
      if (mode) seg[(int64_t)d * M + r] = (int)(w + n);
      for (int e = dy.rowptr[d][r]; e < dy.rowptr[d][r + 1]; ++e) {
        if (mode) { col[w + n] = dy.col[d][e]; val[w + n] = dy.val[d][e]; }
        ++n;
      }
      if (dy.K[d] && dy.K[d][r] != 0.0) {
        if (mode) { col[w + n] = (int)M; val[w + n] = dy.K[d][r]; }
        ++n;
      }
    }
    if (!mode) cnt[r] = n;
  }
}

__global__ void k_axpy_into(int64_t M, double w, const double* __restrict__ x, double* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (int64_t)gridDim.x * blockDim.x)
    y[i] += w * x[i];
}

__global__ void k_i64_to_i32(int64_t n, const int64_t* __restrict__ a, int64_t total, int* __restrict__ b) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = (int)a[i];
  if (blockIdx.x == 0 && threadIdx.x == 0) b[n] = (int)total;
}

// Row-block partition: a block starts at every row whose first nonzero lies
// in a new window of `bn` nonzeros.
__global__ void k_block_flags(int64_t M, const int* __restrict__ rowptr, int bn, int64_t* __restrict__ flag) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < M; r += (int64_t)gridDim.x * blockDim.x)
    flag[r] = (r == 0) || (rowptr[r] / bn != rowptr[r - 1] / bn);
}

__global__ void k_block_rows(int64_t M, const int64_t* __restrict__ flag, const int64_t* __restrict__ id,
                             int64_t nb, int* __restrict__ blk_row) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < M; r += (int64_t)gridDim.x * blockDim.x)
    if (flag[r]) blk_row[id[r]] = (int)r;
  if (blockIdx.x == 0 && threadIdx.x == 0) blk_row[nb] = (int)M;
}

__global__ void k_fill(int64_t n, double v, double* __restrict__ a) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

// ---------------------------------------------------------------------------
// The fused stage kernel
//
// The text between the "[stage-kernel source]" markers in this file defines
// the sliced stage kernel and its launch; bench.py hashes exactly that text to
// tie the committed HBM counter readings to the kernel they were taken on.
// ---------------------------------------------------------------------------
// [stage-kernel source: begin]
template <int STAGE>
__device__ inline void stage_store(int r, double k, double vr, double ar, double* acc, double* xout, double dt) {
  if (STAGE == 0) {
    xout[r] = vr + (0.5 * dt) * k;
    acc[r] = k;
  } else if (STAGE == 1) {
    xout[r] = vr + (0.5 * dt) * k;
    acc[r] = ar + 2.0 * k;
  } else if (STAGE == 2) {
    xout[r] = vr + dt * k;
    acc[r] = ar + 2.0 * k;
  } else if (STAGE == 3) {
    xout[r] = vr + (dt / 6.0) * (ar + k);
  } else if (STAGE == 4) {
    acc[r] = vr + k;
    xout[r] = (dt / 3.0) * vr + dt * k;
  } else if (STAGE == 5) {
    acc[r] = ar + k;
    xout[r] = (dt / 3.0) * vr + (0.5 * dt) * k;
  } else if (STAGE == 6) {
    acc[r] = ar + k;
    xout[r] = (dt / 6.0) * vr + (0.5 * dt) * k;
  } else if (STAGE == 7) {
    acc[r] = ar + k;
  } else {
    // stage 7 followed by the start of the next backward step: the new
    // lambda gets vin (the objective's weight on the state, or 0) added and
    // xout receives dt/6 lambda
    const double l = (ar + k) + vr;
    acc[r] = l;
    xout[r] = (dt / 6.0) * l;
  }
}

// whether a stage reads the accumulator
template <int STAGE>
__device__ constexpr bool reads_acc() { return STAGE != 0 && STAGE != 4; }
// [stage-kernel source: end]

template <int STAGE>
__device__ inline void rk4_update(int r, double k, const double* v, double* acc, double* xout, double dt) {
  const double vr = v[r];
  const double ar = reads_acc<STAGE>() ? acc[r] : 0.0;
  stage_store<STAGE>(r, k, vr, ar, acc, xout, dt);
}

template <int STAGE, int NT>
__global__ __launch_bounds__(NT) void k_rk4_stage(
    const int* __restrict__ rowptr, const int* __restrict__ seg, int ndyn, const int* __restrict__ col,
    const double* __restrict__ val, const int* __restrict__ blk_row, int nblocks, int xcd_remap, int cap,
    const double* __restrict__ xin, const double* v, double* acc, double* xout,
    const double* __restrict__ coef, int64_t coef_row, double dt, int M) {
  extern __shared__ double prod[];
  __shared__ double red[NT / 64][1 + kMaxDyn];
  int b = blockIdx.x;
  if (xcd_remap) {
    const int q = (nblocks + 7) >> 3;
    b = (b & 7) * q + (b >> 3);
  }
  if (b >= nblocks) return;
  double eps[kMaxDyn];
#pragma unroll
  for (int d = 0; d < kMaxDyn; ++d) eps[d] = d < ndyn ? coef[coef_row * ndyn + d] : 0.0;

  const int r0 = blk_row[b], r1 = blk_row[b + 1];
  const int e0 = rowptr[r0], e1 = rowptr[r1];
  const int n = e1 - e0;
  const int tid = threadIdx.x;
  if (n <= cap) {
    // operands of the row this lane finishes in phase 2, fetched early
    const int rr = r0 + tid;
    const bool own = rr < r1;
    int ra = 0, rz = 0, rs = 0;
    double vr = 0.0, ar = 0.0;
    if (own) {
      ra = rowptr[rr];
      rz = rowptr[rr + 1];
      rs = ndyn ? seg[rr] : rz;
      vr = v[rr];
      if (reads_acc<STAGE>()) ar = acc[rr];
    }
    // phase 1: stream the block's nonzeros, kIt per lane per round, with all
    // index/value loads issued before the dependent gathers
    constexpr int kIt = 8;
    for (int base = 0; base < n; base += NT * kIt) {
      int ci[kIt];
      double cv[kIt], xv[kIt];
#pragma unroll
      for (int u = 0; u < kIt; ++u) {
        const int i = base + u * NT + tid;
        ci[u] = i < n ? __builtin_nontemporal_load(col + e0 + i) : M;
        cv[u] = i < n ? __builtin_nontemporal_load(val + e0 + i) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kIt; ++u) xv[u] = xin[ci[u]];
#pragma unroll
      for (int u = 0; u < kIt; ++u) {
        const int i = base + u * NT + tid;
        if (i < n) prod[i] = cv[u] * xv[u];
      }
    }
    __syncthreads();
    // phase 2: one lane per row sums its segments and updates the stage
    for (int r = rr; r < r1; r += NT) {
      if (r != rr) {
        ra = rowptr[r];
        rz = rowptr[r + 1];
        rs = ndyn ? seg[r] : rz;
        vr = v[r];
        if (reads_acc<STAGE>()) ar = acc[r];
      }
      int send = rs - e0;
      const int z = rz - e0;
      double k = 0.0;
      for (int i = ra - e0; i < send; ++i) k += prod[i];
      for (int d = 0; d < ndyn; ++d) {
        const int s0 = send;
        send = (d + 1 < ndyn) ? seg[(int64_t)(d + 1) * M + r] - e0 : z;
        double sd = 0.0;
        for (int i = s0; i < send; ++i) sd += prod[i];
        k += eps[d] * sd;
      }
      stage_store<STAGE>(r, k, vr, ar, acc, xout, dt);
    }
  } else {
    // rows too long for the LDS buffer: the whole workgroup reduces one row
    for (int r = r0; r < r1; ++r) {
      const int a = rowptr[r], z = rowptr[r + 1];
      double part[1 + kMaxDyn];
#pragma unroll
      for (int d = 0; d <= kMaxDyn; ++d) part[d] = 0.0;
      int bounds[2 + kMaxDyn];
      bounds[0] = a;
      for (int d = 0; d < ndyn; ++d) bounds[d + 1] = seg[(int64_t)d * M + r];
      bounds[ndyn + 1] = z;
      for (int sgm = 0; sgm <= ndyn; ++sgm)
        for (int i = bounds[sgm] + tid; i < bounds[sgm + 1]; i += NT) part[sgm] += val[i] * xin[col[i]];
      for (int sgm = 0; sgm <= ndyn; ++sgm) {
        double x = part[sgm];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
        if ((tid & 63) == 0) red[tid >> 6][sgm] = x;
      }
      __syncthreads();
      if (tid == 0) {
        double k = 0.0;
        for (int sgm = 0; sgm <= ndyn; ++sgm) {
          double s = 0.0;
          for (int w = 0; w < NT / 64; ++w) s += red[w][sgm];
          k += (sgm == 0 ? 1.0 : eps[sgm - 1]) * s;
        }
        rk4_update<STAGE>(r, k, v, acc, xout, dt);
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// Sliced-ELL layout.  Rows of length <= long_len are taken in their natural
// order, cut into windows of `sigma` rows, sorted by decreasing length inside
// each window (stable), and packed 64 rows per slice: entry k of the row in
// lane l of slice s sits at off[s] + 64 k + l, so one load instruction of a
// wavefront reads 64 consecutive values.  A slice is as wide as its longest
// row; a shorter row's padding entries hold value 0 and column delta 0 (so
// they gather the slice column's base entry, a valid index); the row walk
// drops their products by selecting on the lane's row length, so they add
// exactly nothing even where the gathered entry is not finite.  Each lane keeps the static length of
// its row so that it can split its sum into the static and the dynamic
// segment.  Longer rows are listed separately and reduced by one wavefront
// each.
// ---------------------------------------------------------------------------
constexpr int kSlice = 64;

// Row taken at position q of the sequence the slices are cut from: the
// natural order (P = 0), or pairs interleaved (S_p at 2p, J_p at 2p+1, the
// D rows after them): the diagonal part of the Hamiltonian couples S_p with
// J_p, P rows apart in the natural order, so with interleaving the rows of a
// contiguous range of slices gather from one range of the state vector
// instead of two.
__device__ inline int64_t seq_row(int64_t q, int64_t P) {
  return q < 2 * P ? ((q & 1) ? P + (q >> 1) : (q >> 1)) : q;
}

__global__ void k_row_class(int64_t M, int64_t P, const int* __restrict__ rowptr, int long_len,
                            int64_t* __restrict__ is_short, int64_t* __restrict__ is_long) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < M; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = seq_row(q, P);
    const int len = rowptr[r + 1] - rowptr[r];
    is_short[q] = len <= long_len;
    is_long[q] = len > long_len;
  }
}

__global__ void k_row_scatter(int64_t M, int64_t P, const int64_t* __restrict__ is_short,
                              const int64_t* __restrict__ spos, const int64_t* __restrict__ lpos,
                              int* __restrict__ short_rows, int* __restrict__ long_rows) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < M; q += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)seq_row(q, P);
    if (is_short[q]) short_rows[spos[q]] = r;
    else long_rows[lpos[q]] = r;
  }
}

// One workgroup per window: bitonic sort of (long_len - len, position) keys.
__global__ __launch_bounds__(256) void k_window_sort(int64_t nshort, int sigma, const int* __restrict__ rowptr,
                                                     const int* __restrict__ short_rows,
                                                     int* __restrict__ sell_row) {
  extern __shared__ uint64_t wk[];
  const int64_t w0 = (int64_t)blockIdx.x * sigma;
  const int n = (int)min((int64_t)sigma, nshort - w0);
  int np2 = 1;
  while (np2 < n) np2 <<= 1;
  for (int i = threadIdx.x; i < np2; i += blockDim.x) {
    if (i < n) {
      const int r = short_rows[w0 + i];
      const uint32_t len = (uint32_t)(rowptr[r + 1] - rowptr[r]);
      wk[i] = ((uint64_t)(0xFFFFFFFFu - len) << 32) | (uint32_t)i;
    } else {
      wk[i] = ~0ull;
    }
  }
  __syncthreads();
  for (int k = 2; k <= np2; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < np2; i += blockDim.x) {
        const int l = i ^ j;
        if (l > i) {
          const uint64_t a = wk[i], b = wk[l];
          if ((a > b) == ((i & k) == 0)) { wk[i] = b; wk[l] = a; }
        }
      }
      __syncthreads();
    }
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    sell_row[w0 + i] = short_rows[w0 + (int64_t)(wk[i] & 0xFFFFFFFFu)];
}

__global__ void k_slice_width(int64_t nslices, int64_t nshort, const int* __restrict__ rowptr,
                              const int* __restrict__ sell_row, int64_t* __restrict__ width_x64) {
  for (int64_t sl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; sl < nslices;
       sl += (int64_t)gridDim.x * blockDim.x) {
    int w = 0;
    for (int l = 0; l < kSlice; ++l) {
      const int64_t i = sl * kSlice + l;
      if (i < nshort) { const int r = sell_row[i]; w = max(w, rowptr[r + 1] - rowptr[r]); }
    }
    width_x64[sl] = (int64_t)w * kSlice;
  }
}

__global__ void k_sell_fill(int64_t nslices, int64_t nshort, const int* __restrict__ rowptr,
                            const int* __restrict__ seg, int ndyn, const int* __restrict__ col,
                            const double* __restrict__ val, const int* __restrict__ sell_row,
                            const int64_t* __restrict__ off64, const int64_t* __restrict__ width_x64,
                            int* __restrict__ sell_off, int* __restrict__ sell_len, int* __restrict__ scol,
                            double* __restrict__ sval, int64_t M, int* __restrict__ sell_seg) {
  const int64_t total = nslices * kSlice;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t sl = i / kSlice;
    const int l = (int)(i % kSlice);
    const int w = (int)(width_x64[sl] / kSlice);
    const int64_t base = off64[sl] + l;
    if (l == 0) sell_off[sl] = (int)off64[sl];
    int len = 0, slen = 0, a = 0;
    if (i < nshort) {
      const int r = sell_row[i];
      a = rowptr[r];
      len = rowptr[r + 1] - a;
      slen = ndyn ? seg[r] - a : len;
    }
    sell_len[i] = (len << 16) | slen;
    if (sell_seg) {
      // row-relative starts of the time-dependent segments, 8 bits each
      // (rows on the sliced path have at most 255 entries here)
      int packed = 0;
      for (int d = 0; d < ndyn; ++d) packed |= (i < nshort ? seg[(int64_t)d * M + sell_row[i]] - a : 0) << (8 * d);
      sell_seg[i] = packed;
    }
    for (int k = 0; k < w; ++k) {
      const int64_t dst = base + (int64_t)k * kSlice;
      if (k < len) { scol[dst] = col[a + k]; sval[dst] = val[a + k]; }
      else { scol[dst] = -1; sval[dst] = 0.0; }     // padding, never read
    }
  }
}

// Column compression.  For every slice column (slice s, entry k) the base is
// the smallest column index over the lanes that hold an entry there; a lane
// stores col - base in 1, 2 or 4 bytes, the width chosen per slice (the
// narrowest that fits every column of the slice).  Padding stores 0.
__global__ void k_group_base(int64_t ngroups, const int* __restrict__ scol, int* __restrict__ gbase,
                             int* __restrict__ gspan) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < ngroups; g += (int64_t)gridDim.x * blockDim.x) {
    int mn = INT32_MAX, mx = -1;
    for (int l = 0; l < kSlice; ++l) {
      const int c = scol[g * kSlice + l];
      if (c >= 0) { mn = min(mn, c); mx = max(mx, c); }
    }
    if (mx < 0) mn = mx = 0;
    gbase[g] = mn;
    gspan[g] = mx - mn;
  }
}

__global__ void k_slice_mode(int64_t nslices, const int* __restrict__ sell_off, const int* __restrict__ gspan,
                             int min_bytes, int64_t* __restrict__ cbytes, int* __restrict__ mode) {
  for (int64_t sl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; sl < nslices; sl += (int64_t)gridDim.x * blockDim.x) {
    const int g0 = sell_off[sl] / kSlice, g1 = sell_off[sl + 1] / kSlice;
    int span = 0;
    for (int g = g0; g < g1; ++g) span = max(span, gspan[g]);
    int m = span < 256 ? 0 : (span < 65536 ? 1 : 2);      // 1, 2 or 4 bytes
    const int mmin = min_bytes >= 4 ? 2 : (min_bytes >= 2 ? 1 : 0);
    m = max(m, mmin);
    mode[sl] = m;
    cbytes[sl] = (int64_t)(g1 - g0) * kSlice << m;
  }
}

__global__ void k_pack_cols(int64_t nslices, const int* __restrict__ sell_off, const int* __restrict__ scol,
                            const int* __restrict__ gbase, const int* __restrict__ mode,
                            const int64_t* __restrict__ coff64, int* __restrict__ sell_coff,
                            unsigned char* __restrict__ cb) {
  const int64_t total = nslices * kSlice;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t sl = i / kSlice;
    const int l = (int)(i % kSlice);
    const int m = mode[sl];
    if (l == 0) sell_coff[sl] = (int)coff64[sl] | m;    // offsets are multiples of 64
    const int g0 = sell_off[sl] / kSlice, g1 = sell_off[sl + 1] / kSlice;
    for (int g = g0; g < g1; ++g) {
      const int c = scol[(int64_t)g * kSlice + l];
      const uint32_t d = c >= 0 ? (uint32_t)(c - gbase[g]) : 0u;
      const int64_t e = (int64_t)(g - g0) * kSlice + l;
      unsigned char* dst = cb + coff64[sl];
      if (m == 0) dst[e] = (unsigned char)d;
      else if (m == 1) reinterpret_cast<uint16_t*>(dst)[e] = (uint16_t)d;
      else reinterpret_cast<uint32_t*>(dst)[e] = d;
    }
  }
}

// [stage-kernel source: begin]
template <bool NTL, class X>
__device__ inline X stream_load(const X* p) {
  if constexpr (NTL) return __builtin_nontemporal_load(p);
  else return *p;
}

template <class T, bool NTL>
__device__ inline int load_delta(const unsigned char* p, int64_t e) {
  return (int)stream_load<NTL>(reinterpret_cast<const T*>(p) + e);
}

// Sum of one lane's row over entries k0 .. wd - 1 of a slice whose column
// deltas are of type T.  k0, wd, cb, gbase and vp - lane are
// wavefront-uniform.
template <class T, int U, bool NTL>
__device__ inline void slice_row_sum(const unsigned char* cb, const int* __restrict__ gbase,
                                     const double* __restrict__ vp, int k0, int wd, int lane, int slen, int len,
                                     const double* __restrict__ xin, double& a0, double& a1) {
  // accumulate in locals with value selects (a select of the target
  // accumulator would force both into scratch memory)
  double s0 = 0.0, s1 = 0.0;
  int k = k0;
  for (; k + U <= wd; k += U) {
    int ci[U];
    double cv[U], xv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ci[u] = gbase[k + u] + load_delta<T, NTL>(cb, (int64_t)(k + u) * kSlice + lane);
      cv[u] = stream_load<NTL>(vp + (int64_t)(k + u) * kSlice);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) xv[u] = xin[ci[u]];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double pr = cv[u] * xv[u];
      s0 += (k + u < slen) ? pr : 0.0;
      s1 += (k + u >= slen && k + u < len) ? pr : 0.0;
    }
  }
  if (k < wd) {
    constexpr int R = U / 2 > 0 ? U / 2 : 1;
    for (; k < wd; k += R) {
      int ci[R];
      double cv[R], xv[R];
#pragma unroll
      for (int u = 0; u < R; ++u) {
        const bool in = k + u < wd;   // uniform
        ci[u] = in ? gbase[k + u] + load_delta<T, NTL>(cb, (int64_t)(k + u) * kSlice + lane) : gbase[0];
        cv[u] = in ? stream_load<NTL>(vp + (int64_t)(k + u) * kSlice) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < R; ++u) xv[u] = xin[ci[u]];
#pragma unroll
      for (int u = 0; u < R; ++u) {
        const double pr = cv[u] * xv[u];
        s0 += (k + u < slen) ? pr : 0.0;
        s1 += (k + u >= slen && k + u < len) ? pr : 0.0;
      }
    }
  }
  a0 = s0;
  a1 = s1;
}

// SPLIT wavefronts per slice (or per long row), workgroups of 4 wavefronts.
// With SPLIT = 1 each wavefront sums its slice's rows alone.  With SPLIT = 2
// or 4 the wavefronts of a slice take consecutive ranges of whole load
// rounds (a long row: interleaved groups of 64 entries), leave their partial
// sums in LDS and the first of them adds them in part order and stores: a
// shorter chain of dependent loads per wavefront and SPLIT times as many
// wavefronts, for generators too small to fill the chip one slice per
// wavefront.
template <int STAGE, int U, bool NTL, int SPLIT>
__global__ __launch_bounds__(256) void k_rk4_sell(
    const int* __restrict__ sell_off, const int* __restrict__ sell_coff, const int* __restrict__ gbase_all,
    const unsigned char* __restrict__ cb_all, const int* __restrict__ sell_row, const int* __restrict__ sell_len,
    const double* __restrict__ sval, int64_t nslices, int64_t nshort,
    const int* __restrict__ long_rows, int64_t nlong, const int* __restrict__ rowptr, const int* __restrict__ seg,
    const int* __restrict__ col, const double* __restrict__ val, int ndyn,
    const double* __restrict__ xin, const double* v, double* acc, double* xout,
    const double* __restrict__ coef, int64_t coef_row, double dt, int xcd_remap) {
  static_assert(SPLIT == 1 || SPLIT == 2 || SPLIT == 4, "1, 2 or 4 wavefronts per slice");
  const int lane = threadIdx.x & 63;
  // Workgroups are dispatched round-robin over the 8 XCDs; with xcd_remap
  // each XCD takes one contiguous range of slices, so the x entries its
  // rows gather stay in that XCD's L2.
  int64_t blk = blockIdx.x;
  if (xcd_remap) {
    const int64_t q = ((int64_t)gridDim.x + 7) >> 3;
    blk = (blk & 7) * q + (blk >> 3);
  }
  // wavefront index, made explicitly uniform so that slice metadata become
  // scalar loads and width tests scalar branches
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int part = wv % SPLIT;
  const int64_t wid = blk * (4 / SPLIT) + wv / SPLIT;
  const double eps = ndyn ? coef[coef_row] : 0.0;
  double a0 = 0.0, a1 = 0.0, vr = 0.0, ar = 0.0;
  int r = 0;
  bool own = false;
  if (wid < nslices) {
    const int64_t i = wid * kSlice + lane;
    const int off = __builtin_amdgcn_readfirstlane(sell_off[wid]);
    const int wd = (__builtin_amdgcn_readfirstlane(sell_off[wid + 1]) - off) / kSlice;   // slice width
    const int coff = __builtin_amdgcn_readfirstlane(sell_coff[wid]);
    own = i < nshort && part == 0;
    r = own ? sell_row[i] : 0;
    const int lens = sell_len[i];
    const int slen = lens & 0xFFFF, len = lens >> 16;
    if (own) {
      vr = v[r];
      if (reads_acc<STAGE>()) ar = acc[r];
    }
    int k0 = 0, k1 = wd;
    if constexpr (SPLIT > 1) {
      // entries per part: a multiple of 4 that does not depend on U, so the
      // parts, and the results, are the same for every U
      const int per = ((wd + SPLIT - 1) / SPLIT + 3) & ~3;
      k0 = min(wd, part * per);
      k1 = min(wd, k0 + per);
    }
    const unsigned char* cb = cb_all + (coff & ~63);
    const int* gbase = gbase_all + off / kSlice;
    const double* vp = sval + off + lane;
    switch (coff & 3) {
      case 0: slice_row_sum<uint8_t, U, NTL>(cb, gbase, vp, k0, k1, lane, slen, len, xin, a0, a1); break;
      case 1: slice_row_sum<uint16_t, U, NTL>(cb, gbase, vp, k0, k1, lane, slen, len, xin, a0, a1); break;
      default: slice_row_sum<uint32_t, U, NTL>(cb, gbase, vp, k0, k1, lane, slen, len, xin, a0, a1); break;
    }
  } else if (wid < nslices + nlong) {
    r = long_rows[wid - nslices];
    const int a = rowptr[r], z = rowptr[r + 1];
    const int sb = ndyn ? seg[r] : z;
    for (int e = a + part * 64 + lane; e < z; e += 64 * SPLIT) {
      const double pr = val[e] * xin[col[e]];
      a0 += e < sb ? pr : 0.0;
      a1 += e < sb ? 0.0 : pr;
    }
    for (int o = 32; o > 0; o >>= 1) {
      a0 += __shfl_down(a0, o, 64);
      a1 += __shfl_down(a1, o, 64);
    }
    own = lane == 0 && part == 0;
    if (own) {
      vr = v[r];
      if (reads_acc<STAGE>()) ar = acc[r];
    }
  }
  if constexpr (SPLIT > 1) {
    __shared__ double red[2][4][64];
    red[0][wv][lane] = a0;
    red[1][wv][lane] = a1;
    __syncthreads();
    if (own) {
      for (int q = 1; q < SPLIT; ++q) {
        a0 += red[0][wv + q][lane];
        a1 += red[1][wv + q][lane];
      }
    }
  }
  if (own) stage_store<STAGE>(r, a0 + eps * a1, vr, ar, acc, xout, dt);
}

// [stage-kernel source: end]

// Adjoint parameter dot products on the sliced layouts of static generators
// T_j (each with its free vector folded in as column M, x[M] = 1), all terms
// and the four RK4 stages of one step in one launch, so each matrix is read
// once per step.  The wavefronts are numbered term after term (wave0); each
// forms, for every stage i, q_i = sum over its rows of kb_i[r] (T_j x_i)[r]
// (one slice, or one long row; every sum in row order), reduced over the
// wavefront in a fixed tree, and adds sum_i dc_jth(t_i) q_i to its own slot
// gpart[th * ld + slot0_j + w] for th < ntheta, with
// dc_jth(t_i) = dstat[term_j * ntheta + th] (+ dcoef[(krow_i * ndyn + slot_j) * ntheta + th]
// for a time-dependent term, slot_j >= 0).  Each slot is updated by one
// wavefront per launch, in stream order.
struct DotView {
  const int *off, *coff, *gbase;
  const unsigned char* cb;
  const int *row, *len;
  const double* sval;
  int64_t nslices, nshort, nlong;
  const int *long_rows, *rowptr, *col;
  const double* val;
  int term, slot;
  int64_t wave0, slot0;
};

struct DotViews {
  int n;
  DotView v[kMaxDotTerms];
};

struct DotStages {
  const double* x[kDotStages];
  const double* kb[kDotStages];
  int64_t krow[kDotStages];
};

// s[i] = sum over one lane's row of a slice (all entries: static generator)
// of val * x_i[col], for the kDotStages stage vectors; U entries per round.
template <class T, int U, bool NTL, int NS>
__device__ inline void slice_row_dots(const unsigned char* cb, const int* __restrict__ gbase,
                                      const double* __restrict__ vp, int wd, int lane, int len,
                                      const double* const* xs, double* s) {
  for (int i = 0; i < NS; ++i) s[i] = 0.0;
  // full rounds without predicates (all loads of a round issued together),
  // then the last wd % U entries
  int k = 0;
  for (; k + U <= wd; k += U) {
    int ci[U];
    double cv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ci[u] = gbase[k + u] + load_delta<T, NTL>(cb, (int64_t)(k + u) * kSlice + lane);
      cv[u] = stream_load<NTL>(vp + (int64_t)(k + u) * kSlice);
    }
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      double xv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) xv[u] = xs[i][ci[u]];
#pragma unroll
      for (int u = 0; u < U; ++u) s[i] += (k + u < len) ? cv[u] * xv[u] : 0.0;
    }
  }
  for (; k < wd; ++k) {
    const int c = gbase[k] + load_delta<T, NTL>(cb, (int64_t)k * kSlice + lane);
    const double v = stream_load<NTL>(vp + (int64_t)k * kSlice);
#pragma unroll
    for (int i = 0; i < NS; ++i) s[i] += (k < len) ? v * xs[i][c] : 0.0;
  }
}

template <int U, bool NTL, int NS>
__global__ __launch_bounds__(256) void k_dot_sell(DotViews dv, int64_t nwaves, DotStages st,
                                                  const double* __restrict__ dstat,
                                                  const double* __restrict__ dcoef, int ndyn, int ntheta,
                                                  double* __restrict__ gpart, int64_t ld, int xcd_remap) {
  // blockIdx.y selects stages [NS * blockIdx.y, NS * blockIdx.y + NS); its
  // slots follow those of the previous y at offset ntheta * ld
  const int sb = NS * blockIdx.y;
  gpart += (int64_t)blockIdx.y * ntheta * ld;
  const double* xs[NS];
  const double* kbs[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    xs[i] = st.x[sb + i];
    kbs[i] = st.kb[sb + i];
  }
  const int lane = threadIdx.x & 63;
  int64_t blk = blockIdx.x;
  if (xcd_remap) {
    const int64_t q = ((int64_t)gridDim.x + 7) >> 3;
    blk = (blk & 7) * q + (blk >> 3);
  }
  const int64_t gw = blk * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (gw >= nwaves) return;
  int j = 0;
  for (int q = 1; q < dv.n; ++q)
    if (dv.v[q].wave0 <= gw) j = q;
  const DotView& D = dv.v[j];
  const int64_t wid = gw - D.wave0;
  double qv[NS];
  if (wid < D.nslices) {
    const int64_t i = wid * kSlice + lane;
    const int off = __builtin_amdgcn_readfirstlane(D.off[wid]);
    const int wd = (__builtin_amdgcn_readfirstlane(D.off[wid + 1]) - off) / kSlice;
    const int coff = __builtin_amdgcn_readfirstlane(D.coff[wid]);
    const bool own = i < D.nshort;
    const int r = own ? D.row[i] : 0;
    const int len = D.len[i] >> 16;
    const unsigned char* cb = D.cb + (coff & ~63);
    const int* gbase = D.gbase + off / kSlice;
    const double* vp = D.sval + off + lane;
    double sv[NS];
    switch (coff & 3) {
      case 0: slice_row_dots<uint8_t, U, NTL, NS>(cb, gbase, vp, wd, lane, len, xs, sv); break;
      case 1: slice_row_dots<uint16_t, U, NTL, NS>(cb, gbase, vp, wd, lane, len, xs, sv); break;
      default: slice_row_dots<uint32_t, U, NTL, NS>(cb, gbase, vp, wd, lane, len, xs, sv); break;
    }
#pragma unroll
    for (int s2 = 0; s2 < NS; ++s2) qv[s2] = own ? kbs[s2][r] * sv[s2] : 0.0;
  } else {
    const int r = D.long_rows[wid - D.nslices];
    double a[NS];
#pragma unroll
    for (int s2 = 0; s2 < NS; ++s2) a[s2] = 0.0;
    for (int e = D.rowptr[r] + lane; e < D.rowptr[r + 1]; e += 64) {
      const double v = D.val[e];
      const int c = D.col[e];
#pragma unroll
      for (int s2 = 0; s2 < NS; ++s2) a[s2] += v * xs[s2][c];
    }
#pragma unroll
    for (int s2 = 0; s2 < NS; ++s2) {
      for (int o = 32; o > 0; o >>= 1) a[s2] += __shfl_xor(a[s2], o, 64);
      qv[s2] = lane == 0 ? kbs[s2][r] * a[s2] : 0.0;
    }
  }
#pragma unroll
  for (int s2 = 0; s2 < NS; ++s2)
    for (int o = 32; o > 0; o >>= 1) qv[s2] += __shfl_xor(qv[s2], o, 64);
  if (lane < ntheta) {
    const double d0 = dstat[D.term * ntheta + lane];
    double add = 0.0;
#pragma unroll
    for (int s2 = 0; s2 < NS; ++s2) {
      double dc = d0;
      if (D.slot >= 0 && dcoef) dc += dcoef[(st.krow[sb + s2] * ndyn + D.slot) * ntheta + lane];
      add += dc * qv[s2];
    }
    gpart[lane * ld + D.slot0 + wid] += add;
  }
}

// Segmented row sums for the reverse stages with fused dot products: ND
// time-dependent segments after the static one, their row-relative starts in
// b[1..ND] (b[0] = 0, b[ND + 1] = len); every segment summed in row order.
template <class T, int U, int ND>
__device__ inline void slice_row_segs(const unsigned char* cb, const int* __restrict__ gbase,
                                      const double* __restrict__ vp, int wd, int lane, const int* b,
                                      const double* __restrict__ xin, double* a) {
#pragma unroll
  for (int q = 0; q <= ND; ++q) a[q] = 0.0;
  int k = 0;
  for (; k + U <= wd; k += U) {
    int ci[U];
    double cv[U], xv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ci[u] = gbase[k + u] + load_delta<T, false>(cb, (int64_t)(k + u) * kSlice + lane);
      cv[u] = vp[(int64_t)(k + u) * kSlice];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) xv[u] = xin[ci[u]];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double pr = cv[u] * xv[u];
#pragma unroll
      for (int q = 0; q <= ND; ++q) a[q] += (k + u >= b[q] && k + u < b[q + 1]) ? pr : 0.0;
    }
  }
  for (; k < wd; ++k) {
    const int c = gbase[k] + load_delta<T, false>(cb, (int64_t)k * kSlice + lane);
    const double pr = vp[(int64_t)k * kSlice] * xin[c];
#pragma unroll
    for (int q = 0; q <= ND; ++q) a[q] += (k >= b[q] && k < b[q + 1]) ? pr : 0.0;
  }
}

// One RK4 stage (forward 0..3 or reverse 4..8) on the segmented sliced
// layout: the static segment plus ND time-dependent segments per row, each
// summed in row order, k = a_0 + sum_d c_d a_{d+1} with c_d from rd (the
// forward layout 2 of 2-3 time-dependent terms).  With DOTS, the reverse
// stages also form the parameter dot products described at RevDot.
template <int STAGE, int ND, bool DOTS>
__global__ __launch_bounds__(256) void k_sell_seg(
    const int* __restrict__ sell_off, const int* __restrict__ sell_coff, const int* __restrict__ gbase_all,
    const unsigned char* __restrict__ cb_all, const int* __restrict__ sell_row, const int* __restrict__ sell_len,
    const int* __restrict__ sell_seg, const double* __restrict__ sval, int64_t nslices, int64_t nshort,
    const int* __restrict__ long_rows, int64_t nlong, const int* __restrict__ rowptr, const int* __restrict__ seg,
    const int* __restrict__ col, const double* __restrict__ val, int64_t M, const double* __restrict__ xin,
    const double* v, double* acc, double* xout, const double* __restrict__ xdot, RevDot rd, int64_t krow,
    double dt, int xcd_remap) {
  const int lane = threadIdx.x & 63;
  int64_t blk = blockIdx.x;
  if (xcd_remap) {
    const int64_t q = ((int64_t)gridDim.x + 7) >> 3;
    blk = (blk & 7) * q + (blk >> 3);
  }
  const int64_t wid = blk * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (wid >= nslices + nlong) return;
  double cseg[ND];
#pragma unroll
  for (int d = 0; d < ND; ++d)
    cseg[d] = rd.wseg[d] + (rd.slot[d] >= 0 ? rd.coef[krow * rd.ncoef + rd.slot[d]] : 0.0);
  double qd[ND];
#pragma unroll
  for (int d = 0; d < ND; ++d) qd[d] = 0.0;
  if (wid < nslices) {
    const int64_t i = wid * kSlice + lane;
    const int off = __builtin_amdgcn_readfirstlane(sell_off[wid]);
    const int wd = (__builtin_amdgcn_readfirstlane(sell_off[wid + 1]) - off) / kSlice;
    const int coff = __builtin_amdgcn_readfirstlane(sell_coff[wid]);
    const bool own = i < nshort;
    const int r = own ? sell_row[i] : 0;
    const int lens = sell_len[i];
    const int packed = sell_seg[i];
    int b[ND + 2];
    b[0] = 0;
#pragma unroll
    for (int d = 0; d < ND; ++d) b[d + 1] = (packed >> (8 * d)) & 255;
    b[ND + 1] = lens >> 16;
    double vr = 0.0, ar = 0.0, xr = 0.0, kr = 0.0;
    if (own) {
      vr = v[r];
      if (reads_acc<STAGE>()) ar = acc[r];
      if (DOTS) {
        xr = xdot[r];
        kr = xin[r];
      }
    }
    const unsigned char* cb = cb_all + (coff & ~63);
    const int* gbase = gbase_all + off / kSlice;
    const double* vp = sval + off + lane;
    double a[ND + 1];
    switch (coff & 3) {
      case 0: slice_row_segs<uint8_t, 8, ND>(cb, gbase, vp, wd, lane, b, xin, a); break;
      case 1: slice_row_segs<uint16_t, 8, ND>(cb, gbase, vp, wd, lane, b, xin, a); break;
      default: slice_row_segs<uint32_t, 8, ND>(cb, gbase, vp, wd, lane, b, xin, a); break;
    }
    if (own) {
      double k = a[0];
#pragma unroll
      for (int d = 0; d < ND; ++d) k += cseg[d] * a[d + 1];
      stage_store<STAGE>(r, k, vr, ar, acc, xout, dt);
      if (DOTS) {
#pragma unroll
        for (int d = 0; d < ND; ++d) qd[d] = a[d + 1] * xr + (rd.K[d] ? kr * rd.K[d][r] : 0.0);
      }
    }
  } else {
    const int r = long_rows[wid - nslices];
    const int e0 = rowptr[r], e1 = rowptr[r + 1];
    int b[ND + 2];
    b[0] = e0;
#pragma unroll
    for (int d = 0; d < ND; ++d) b[d + 1] = seg[(int64_t)d * M + r];
    b[ND + 1] = e1;
    double a[ND + 1];
#pragma unroll
    for (int q = 0; q <= ND; ++q) a[q] = 0.0;
    for (int e = e0 + lane; e < e1; e += 64) {
      const double pr = val[e] * xin[col[e]];
#pragma unroll
      for (int q = 0; q <= ND; ++q) a[q] += (e >= b[q] && e < b[q + 1]) ? pr : 0.0;
    }
#pragma unroll
    for (int q = 0; q <= ND; ++q)
      for (int o = 32; o > 0; o >>= 1) a[q] += __shfl_down(a[q], o, 64);
    if (lane == 0) {
      const double vr = v[r];
      const double ar = reads_acc<STAGE>() ? acc[r] : 0.0;
      double k = a[0];
#pragma unroll
      for (int d = 0; d < ND; ++d) k += cseg[d] * a[d + 1];
      stage_store<STAGE>(r, k, vr, ar, acc, xout, dt);
      if (DOTS) {
        const double xr = xdot[r], kr = xin[r];
#pragma unroll
        for (int d = 0; d < ND; ++d) qd[d] = a[d + 1] * xr + (rd.K[d] ? kr * rd.K[d][r] : 0.0);
      }
    }
  }
  if (!DOTS) return;
#pragma unroll
  for (int d = 0; d < ND; ++d)
    for (int o = 32; o > 0; o >>= 1) qd[d] += __shfl_xor(qd[d], o, 64);
  if (lane < rd.ntheta) {
    double add = 0.0;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      double dc = rd.dstat[rd.term[d] * rd.ntheta + lane];
      if (rd.slot[d] >= 0 && rd.dcoef) dc += rd.dcoef[(krow * rd.ncoef + rd.slot[d]) * rd.ntheta + lane];
      add += dc * qd[d];
    }
    rd.gpart[lane * rd.ld + wid] += add;
  }
}

// ---------------------------------------------------------------------------
// Several instances on one segmented sliced layout (the batched form's
// instance-major path).  KI instance vectors (each M+1 doubles, stride ldv,
// entry M = 1) are advanced by one RK4 stage with per-instance coefficients
// of the ND time-dependent segments, c_{b,d} = w[b][term_d] + u[b][term_d] *
// wave(t); the static segment carries the weights every instance shares.
// One wavefront takes one slice (or long row) for one chunk of KI instances;
// the chunks of a slice are consecutive wavefronts, so the slice's matrix
// data is read from HBM once and served from L2 to the others.  Every
// instance's row sums are formed exactly as k_sell_seg forms them for one
// vector (same segments, same order), so each instance gets the bits of a
// plain propagation with its own coefficients.
// ---------------------------------------------------------------------------
template <class T, int U, int ND, int KI>
__device__ inline void slice_row_segs_multi(const unsigned char* cb, const int* __restrict__ gbase,
                                            const double* __restrict__ vp, int wd, int lane, const int* b,
                                            const double* const* xs, double (*a)[KI]) {
#pragma unroll
  for (int q = 0; q <= ND; ++q)
#pragma unroll
    for (int i = 0; i < KI; ++i) a[q][i] = 0.0;
  int k = 0;
  for (; k + U <= wd; k += U) {
    int ci[U];
    double cv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ci[u] = gbase[k + u] + load_delta<T, false>(cb, (int64_t)(k + u) * kSlice + lane);
      cv[u] = vp[(int64_t)(k + u) * kSlice];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      double xv[KI];
#pragma unroll
      for (int i = 0; i < KI; ++i) xv[i] = xs[i][ci[u]];
#pragma unroll
      for (int i = 0; i < KI; ++i) {
        const double pr = cv[u] * xv[i];
#pragma unroll
        for (int q = 0; q <= ND; ++q) a[q][i] += (k + u >= b[q] && k + u < b[q + 1]) ? pr : 0.0;
      }
    }
  }
  for (; k < wd; ++k) {
    const int c = gbase[k] + load_delta<T, false>(cb, (int64_t)k * kSlice + lane);
    const double cvk = vp[(int64_t)k * kSlice];
#pragma unroll
    for (int i = 0; i < KI; ++i) {
      const double pr = cvk * xs[i][c];
#pragma unroll
      for (int q = 0; q <= ND; ++q) a[q][i] += (k >= b[q] && k < b[q + 1]) ? pr : 0.0;
    }
  }
}

template <int STAGE, int ND, int KI>
__global__ __launch_bounds__(256) void k_sell_multi(
    const int* __restrict__ sell_off, const int* __restrict__ sell_coff, const int* __restrict__ gbase_all,
    const unsigned char* __restrict__ cb_all, const int* __restrict__ sell_row, const int* __restrict__ sell_len,
    const int* __restrict__ sell_seg, const double* __restrict__ sval, int64_t nslices, int64_t nshort,
    const int* __restrict__ long_rows, int64_t nlong, const int* __restrict__ rowptr, const int* __restrict__ seg,
    const int* __restrict__ col, const double* __restrict__ val, int64_t M, MultiCoef mc, const double* xin,
    const double* v, double* acc, double* xout, double dt, int xcd_remap) {
  const int lane = threadIdx.x & 63;
  int64_t blk = blockIdx.x;
  if (xcd_remap) {
    const int64_t q = ((int64_t)gridDim.x + 7) >> 3;
    blk = (blk & 7) * q + (blk >> 3);
  }
  const int64_t gw = blk * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nch = (mc.B + KI - 1) / KI;
  const int64_t wid = gw / nch;
  const int ch = (int)(gw % nch);
  if (wid >= nslices + nlong) return;
  // this chunk's instances (the last chunk repeats its last instance in the
  // unused slots, which are computed but not stored)
  const double* xs[KI];
  int bi[KI];
  double cseg[ND][KI];
  const double ph = mc.wave[mc.widx];
#pragma unroll
  for (int i = 0; i < KI; ++i) {
    const int bb = min(ch * KI + i, mc.B - 1);
    bi[i] = bb;
    xs[i] = xin + (int64_t)bb * mc.ldv;
#pragma unroll
    for (int d = 0; d < ND; ++d)
      cseg[d][i] = mc.w[(int64_t)bb * mc.nt + mc.term[d]] + mc.u[(int64_t)bb * mc.nt + mc.term[d]] * ph;
  }
  if (wid < nslices) {
    const int64_t i = wid * kSlice + lane;
    const int off = __builtin_amdgcn_readfirstlane(sell_off[wid]);
    const int wd = (__builtin_amdgcn_readfirstlane(sell_off[wid + 1]) - off) / kSlice;
    const int coff = __builtin_amdgcn_readfirstlane(sell_coff[wid]);
    const bool own = i < nshort;
    const int r = own ? sell_row[i] : 0;
    const int lens = sell_len[i];
    const int packed = sell_seg[i];
    int b[ND + 2];
    b[0] = 0;
#pragma unroll
    for (int d = 0; d < ND; ++d) b[d + 1] = (packed >> (8 * d)) & 255;
    b[ND + 1] = lens >> 16;
    const unsigned char* cb = cb_all + (coff & ~63);
    const int* gbase = gbase_all + off / kSlice;
    const double* vp = sval + off + lane;
    double a[ND + 1][KI];
    switch (coff & 3) {
      case 0: slice_row_segs_multi<uint8_t, 4, ND, KI>(cb, gbase, vp, wd, lane, b, xs, a); break;
      case 1: slice_row_segs_multi<uint16_t, 4, ND, KI>(cb, gbase, vp, wd, lane, b, xs, a); break;
      default: slice_row_segs_multi<uint32_t, 4, ND, KI>(cb, gbase, vp, wd, lane, b, xs, a); break;
    }
    if (own) {
#pragma unroll
      for (int q = 0; q < KI; ++q) {
        if (ch * KI + q >= mc.B) break;
        const int64_t o = (int64_t)bi[q] * mc.ldv;
        double kk = a[0][q];
#pragma unroll
        for (int d = 0; d < ND; ++d) kk += cseg[d][q] * a[d + 1][q];
        const double vr = v[o + r];
        const double ar = reads_acc<STAGE>() ? acc[o + r] : 0.0;
        stage_store<STAGE>(r, kk, vr, ar, acc + o, xout + o, dt);
      }
    }
  } else {
    const int r = long_rows[wid - nslices];
    const int e0 = rowptr[r], e1 = rowptr[r + 1];
    int b[ND + 2];
    b[0] = e0;
#pragma unroll
    for (int d = 0; d < ND; ++d) b[d + 1] = seg[(int64_t)d * M + r];
    b[ND + 1] = e1;
    double a[ND + 1][KI];
#pragma unroll
    for (int q = 0; q <= ND; ++q)
#pragma unroll
      for (int i = 0; i < KI; ++i) a[q][i] = 0.0;
    for (int e = e0 + lane; e < e1; e += 64) {
      const double ve = val[e];
      const int ce = col[e];
#pragma unroll
      for (int i = 0; i < KI; ++i) {
        const double pr = ve * xs[i][ce];
#pragma unroll
        for (int q = 0; q <= ND; ++q) a[q][i] += (e >= b[q] && e < b[q + 1]) ? pr : 0.0;
      }
    }
#pragma unroll
    for (int q = 0; q <= ND; ++q)
#pragma unroll
      for (int i = 0; i < KI; ++i)
        for (int o = 32; o > 0; o >>= 1) a[q][i] += __shfl_down(a[q][i], o, 64);
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < KI; ++q) {
        if (ch * KI + q >= mc.B) break;
        const int64_t o = (int64_t)bi[q] * mc.ldv;
        double kk = a[0][q];
#pragma unroll
        for (int d = 0; d < ND; ++d) kk += cseg[d][q] * a[d + 1][q];
        const double vr = v[o + r];
        const double ar = reads_acc<STAGE>() ? acc[o + r] : 0.0;
        stage_store<STAGE>(r, kk, vr, ar, acc + o, xout + o, dt);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Resident path for small systems: one workgroup keeps v, two stage vectors
// and the accumulator ((M+1) doubles each, entry M = 1) in LDS and runs every
// RK4 step of a call in one launch, so small N is not bound by four launches
// per step.  Each row is summed in the order of the fused CSR row with a
// separate rounding of every product and sum, as in slice_row_sum (rows of
// at most 64 entries then give the same bits as the sliced kernel).
// ---------------------------------------------------------------------------
constexpr int kResidentThreads = 1024;
constexpr int64_t kResidentMaxNnz = 2500;   // default use of the resident path

__device__ inline void resident_row(const int* __restrict__ rowptr, const int* __restrict__ col,
                                    const double* __restrict__ val, int sb, int r, const double* xin, double& s0,
                                    double& s1) {
#pragma clang fp contract(off)
  const int a = rowptr[r], z = rowptr[r + 1];
  double p0 = 0.0, p1 = 0.0;
  for (int e = a; e < sb; ++e) {
    const double pr = val[e] * xin[col[e]];
    p0 = p0 + pr;
  }
  for (int e = sb; e < z; ++e) {
    const double pr = val[e] * xin[col[e]];
    p1 = p1 + pr;
  }
  s0 = p0;
  s1 = p1;
}

template <int STAGE>
__device__ inline void resident_stage(const int* __restrict__ rowptr, const int* __restrict__ col,
                                      const double* __restrict__ val, const int* __restrict__ seg, int ndyn, int M,
                                      const double* xin, double* v, double* acc, double* xout, double eps,
                                      double dt) {
  for (int r = threadIdx.x; r < M; r += blockDim.x) {
    double a0, a1;
    resident_row(rowptr, col, val, ndyn ? seg[r] : rowptr[r + 1], r, xin, a0, a1);
    const double vr = v[r];
    const double ar = reads_acc<STAGE>() ? acc[r] : 0.0;
    stage_store<STAGE>(r, a0 + eps * a1, vr, ar, acc, xout, dt);
  }
  __syncthreads();
}

__global__ __launch_bounds__(kResidentThreads) void k_rk4_resident(const int* __restrict__ rowptr,
                                                                   const int* __restrict__ col,
                                                                   const double* __restrict__ val,
                                                                   const int* __restrict__ seg, int ndyn, int M,
                                                                   const double* __restrict__ coef, int64_t steps,
                                                                   double dt, double* __restrict__ vg) {
  extern __shared__ double lds[];
  double* sv = lds;
  double* sa = sv + (M + 1);
  double* sb = sa + (M + 1);
  double* sacc = sb + (M + 1);
  for (int i = threadIdx.x; i <= M; i += blockDim.x) {
    sv[i] = i < M ? vg[i] : 1.0;
    sa[i] = 1.0;
    sb[i] = 1.0;
    sacc[i] = 0.0;
  }
  __syncthreads();
  for (int64_t n = 0; n < steps; ++n) {
    const double e0 = ndyn ? coef[2 * n] : 0.0;
    const double eh = ndyn ? coef[2 * n + 1] : 0.0;
    const double e1 = ndyn ? coef[2 * n + 2] : 0.0;
    resident_stage<0>(rowptr, col, val, seg, ndyn, M, sv, sv, sacc, sa, e0, dt);
    resident_stage<1>(rowptr, col, val, seg, ndyn, M, sa, sv, sacc, sb, eh, dt);
    resident_stage<2>(rowptr, col, val, seg, ndyn, M, sb, sv, sacc, sa, eh, dt);
    resident_stage<3>(rowptr, col, val, seg, ndyn, M, sa, sv, sacc, sv, e1, dt);
  }
  for (int i = threadIdx.x; i < M; i += blockDim.x) vg[i] = sv[i];
}

size_t resident_lds_bytes(int64_t M) { return (size_t)(4 * (M + 1)) * sizeof(double); }

// Matrix data and per-row metadata one launch of the sliced stage kernel
// streams (long rows' CSR entries excluded).
int64_t sell_matrix_bytes(const sun_prop_s& p) {
  return p.sell_nnz * 8 + p.sell_col_bytes + (p.sell_nnz / kSlice) * 4 + p.nslices * kSlice * 8 +
         (p.nslices + 1) * 8;
}

// Above this many matrix bytes per launch the stream cannot stay in the
// 256 MB Infinity Cache between launches, and non-temporal loads (which keep
// it from evicting the gathered state vector) are faster; below it ordinary
// loads let it stay there (dimer: 62.0 against 65.9 us per stage at 265 MB,
// 82.1 against 77.5 at 311 MB, 194 against 170 at 732 MB).
constexpr int64_t kNontemporalMinBytes = 288ll << 20;

// Failure injection for tests of the error paths (sun_debug_inject_failure):
// when set, the next layout build throws after it has rewritten part of the
// propagator, as a device allocation failure there would.
std::atomic<int> g_inject_layout_failure{0};

void maybe_inject_layout_failure() {
  if (g_inject_layout_failure.exchange(0) != 0)
    SUN_THROW(SUN_ENOMEM, "injected failure (sun_debug_inject_failure) in the middle of a layout build");
}

// Wavefronts per slice and entries per load round of the sliced stage kernel,
// from the work units (slices + long rows) of one launch: a generator too
// small to give every SIMD several wavefronts gets 2 or 4 per slice, each
// with a shorter chain of dependent loads.  Measured on the dimer, us per
// stage launch with one wavefront per slice and 8 entries per round against
// the choice: N = 101 (241 units) 4.73 / 3.39 (4, 4); N = 201 (813) 4.74 /
// 4.17 (4, 4); N = 301 (1,698) 5.88 / 5.35 (4, 8); N = 701 (8,352) 21.2 /
// 19.1 (4, 8); N = 1001 (16,623) 36.1 / 34.1 (2, 8); N = 1501 (36,662) 114.4
// against 114.5 for (2, 8), so one wavefront per slice from 24,000 units on.
// A given entries-per-round count other than 4 or 8 keeps one wavefront.
void pick_split(sun_prop_s& p, int unroll) {
  const int64_t units = p.nslices + p.nlong;
  int split = units < 12000 ? 4 : (units < 24000 ? 2 : 1);
  int u = units < 1000 ? 4 : 8;
  if (unroll) {
    u = unroll;
    if (u != 4 && u != 8) split = 1;
  }
  p.sell_split = split;
  p.sell_unroll = u;
}

void build_sell(sun_prop_s& p, hipStream_t s) {
  HIP_OK(hipStreamSynchronize(s));   // earlier launches may still read the old layout
  const int64_t M = p.M;
  DevBuf<int64_t> is_short(M), is_long(M), spos(M), lpos(M);
  const int64_t P = p.sell_pairs ? p.lind->basis->P : 0;
  hipLaunchKernelGGL(k_row_class, dim3(grid_for(M, 256)), dim3(256), 0, s, M, P, p.rowptr.get(), p.long_len,
                     is_short.get(), is_long.get());
  HIP_LAUNCH_OK();
  p.nshort = exclusive_scan_i64(is_short.get(), spos.get(), M, s);
  p.nlong = exclusive_scan_i64(is_long.get(), lpos.get(), M, s);
  DevBuf<int> short_rows(p.nshort > 0 ? p.nshort : 1);
  p.long_rows.alloc(p.nlong > 0 ? p.nlong : 1);
  maybe_inject_layout_failure();
  hipLaunchKernelGGL(k_row_scatter, dim3(grid_for(M, 256)), dim3(256), 0, s, M, P, is_short.get(), spos.get(),
                     lpos.get(), short_rows.get(), p.long_rows.get());
  HIP_LAUNCH_OK();
  p.nslices = (p.nshort + kSlice - 1) / kSlice;
  const int64_t padded_rows = p.nslices * kSlice;
  p.sell_row.alloc(padded_rows > 0 ? padded_rows : 1);
  p.sell_len.alloc(padded_rows > 0 ? padded_rows : 1);
  if (p.sell_segs > 0) p.sell_seg.alloc(padded_rows > 0 ? padded_rows : 1);
  else p.sell_seg.release();
  p.sell_off.alloc(p.nslices + 1);
  p.sell_coff.alloc(p.nslices + 1);
  p.sell_nnz = 0;
  p.sell_col_bytes = 0;
  if (p.nshort > 0) {
    const int64_t nwin = (p.nshort + p.sigma - 1) / p.sigma;
    int np2 = 1;
    while (np2 < p.sigma) np2 <<= 1;
    hipLaunchKernelGGL(k_window_sort, dim3((unsigned)nwin), dim3(256), np2 * sizeof(uint64_t), s, p.nshort,
                       p.sigma, p.rowptr.get(), short_rows.get(), p.sell_row.get());
    HIP_LAUNCH_OK();
    DevBuf<int64_t> wx(p.nslices), off64(p.nslices);
    hipLaunchKernelGGL(k_slice_width, dim3(grid_for(p.nslices, 256)), dim3(256), 0, s, p.nslices, p.nshort,
                       p.rowptr.get(), p.sell_row.get(), wx.get());
    HIP_LAUNCH_OK();
    p.sell_nnz = exclusive_scan_i64(wx.get(), off64.get(), p.nslices, s);
    SUN_REQUIRE(p.sell_nnz < (int64_t)INT32_MAX, SUN_ENOTSUP, "sliced layout has 2^31 or more entries");
    DevBuf<int> scol(p.sell_nnz);
    p.sell_val.alloc(p.sell_nnz);
    hipLaunchKernelGGL(k_sell_fill, dim3(grid_for(padded_rows, 256)), dim3(256), 0, s, p.nslices, p.nshort,
                       p.rowptr.get(), p.seg.get(), p.ndyn, p.col.get(), p.val.get(), p.sell_row.get(),
                       off64.get(), wx.get(), p.sell_off.get(), p.sell_len.get(), scol.get(), p.sell_val.get(), M,
                       p.sell_segs > 0 ? p.sell_seg.get() : nullptr);
    HIP_LAUNCH_OK();
    int tot = (int)p.sell_nnz;
    HIP_OK(hipMemcpyAsync(p.sell_off.get() + p.nslices, &tot, sizeof(int), hipMemcpyHostToDevice, s));
    HIP_OK(hipStreamSynchronize(s));
    // column compression
    const int64_t ngroups = p.sell_nnz / kSlice;
    p.sell_base.alloc(ngroups);
    DevBuf<int> gspan(ngroups), mode(p.nslices);
    DevBuf<int64_t> cbytes(p.nslices), coff64(p.nslices);
    hipLaunchKernelGGL(k_group_base, dim3(grid_for(ngroups, 256)), dim3(256), 0, s, ngroups, scol.get(),
                       p.sell_base.get(), gspan.get());
    HIP_LAUNCH_OK();
    hipLaunchKernelGGL(k_slice_mode, dim3(grid_for(p.nslices, 256)), dim3(256), 0, s, p.nslices,
                       p.sell_off.get(), gspan.get(), p.min_col_bytes, cbytes.get(), mode.get());
    HIP_LAUNCH_OK();
    p.sell_col_bytes = exclusive_scan_i64(cbytes.get(), coff64.get(), p.nslices, s);
    SUN_REQUIRE(p.sell_col_bytes < (int64_t)INT32_MAX, SUN_ENOTSUP, "column stream of 2^31 bytes or more");
    p.sell_cb.alloc(p.sell_col_bytes);
    hipLaunchKernelGGL(k_pack_cols, dim3(grid_for(padded_rows, 256)), dim3(256), 0, s, p.nslices,
                       p.sell_off.get(), scol.get(), p.sell_base.get(), mode.get(), coff64.get(),
                       p.sell_coff.get(), p.sell_cb.get());
    HIP_LAUNCH_OK();
    HIP_OK(hipStreamSynchronize(s));
  }
  HIP_OK(hipStreamSynchronize(s));
}

void build_partition(sun_prop_s& p, hipStream_t s) {
  HIP_OK(hipStreamSynchronize(s));   // earlier launches may still read the old partition
  const int64_t M = p.M;
  DevBuf<int64_t> flag(M), id(M);
  hipLaunchKernelGGL(k_block_flags, dim3(grid_for(M, 256)), dim3(256), 0, s, M, p.rowptr.get(), p.block_nnz,
                     flag.get());
  HIP_LAUNCH_OK();
  p.nblocks = exclusive_scan_i64(flag.get(), id.get(), M, s);
  p.blk_row.alloc(p.nblocks + 1);
  maybe_inject_layout_failure();
  hipLaunchKernelGGL(k_block_rows, dim3(grid_for(M, 256)), dim3(256), 0, s, M, flag.get(), id.get(), p.nblocks,
                     p.blk_row.get());
  HIP_LAUNCH_OK();
  HIP_OK(hipStreamSynchronize(s));
}

int stage_capacity(int block_nnz, int threads) {
  static size_t lim = 0;
  if (!lim) lim = lds_limit();
  // single-wave blocks keep their LDS small (occupancy); blocks with a row
  // that does not fit take the row-reduction path instead
  int cap = threads == 64 ? block_nnz + block_nnz / 2 : 2 * block_nnz;
  while (cap > 256 && (size_t)cap * sizeof(double) + 1024 > lim) cap >>= 1;
  return cap;
}

template <int STAGE, int NT>
void launch_stage_nt(const sun_prop_s& p, const double* xin, const double* vin, double* acc, double* xout,
                     const double* coef, int64_t row, double dt, hipStream_t s) {
  const int cap = stage_capacity(p.block_nnz, NT);
  const int grid = p.xcd_remap ? (int)(((p.nblocks + 7) / 8) * 8) : (int)p.nblocks;
  hipLaunchKernelGGL((k_rk4_stage<STAGE, NT>), dim3(grid), dim3(NT), cap * sizeof(double), s,
                     p.rowptr.get(), p.seg.get(), p.ndyn, p.col.get(), p.val.get(), p.blk_row.get(),
                     (int)p.nblocks, p.xcd_remap, cap, xin, vin, acc, xout, coef, row, dt, (int)p.M);
}

// [stage-kernel source: begin]
template <int STAGE>
void launch_stage_v(const sun_prop_s& p, const double* xin, const double* vin, double* acc, double* xout,
                    const double* coef, int64_t row, double dt, hipStream_t s) {
  if (p.layout == 2) {
    sun::prop_seg_stage(p, STAGE, xin, vin, acc, xout, coef, row, dt, s);
    return;
  }
  if (p.layout == 1) {
    const int64_t waves = (p.nslices + p.nlong) * p.sell_split;
    unsigned grid = (unsigned)((waves + 3) / 4);
    if (p.sell_remap) grid = (grid + 7) / 8 * 8;
    auto kern = k_rk4_sell<STAGE, 8, false, 1>;
    switch (p.sell_split * 64 + p.sell_unroll * 2 + p.sell_nt) {
      case 64 + 8: kern = k_rk4_sell<STAGE, 4, false, 1>; break;
      case 64 + 9: kern = k_rk4_sell<STAGE, 4, true, 1>; break;
      case 64 + 12: kern = k_rk4_sell<STAGE, 6, false, 1>; break;
      case 64 + 13: kern = k_rk4_sell<STAGE, 6, true, 1>; break;
      case 64 + 17: kern = k_rk4_sell<STAGE, 8, true, 1>; break;
      case 64 + 24: kern = k_rk4_sell<STAGE, 12, false, 1>; break;
      case 64 + 25: kern = k_rk4_sell<STAGE, 12, true, 1>; break;
      case 64 + 32: kern = k_rk4_sell<STAGE, 16, false, 1>; break;
      case 64 + 33: kern = k_rk4_sell<STAGE, 16, true, 1>; break;
      case 128 + 8: kern = k_rk4_sell<STAGE, 4, false, 2>; break;
      case 128 + 9: kern = k_rk4_sell<STAGE, 4, true, 2>; break;
      case 128 + 16: kern = k_rk4_sell<STAGE, 8, false, 2>; break;
      case 128 + 17: kern = k_rk4_sell<STAGE, 8, true, 2>; break;
      case 256 + 8: kern = k_rk4_sell<STAGE, 4, false, 4>; break;
      case 256 + 9: kern = k_rk4_sell<STAGE, 4, true, 4>; break;
      case 256 + 16: kern = k_rk4_sell<STAGE, 8, false, 4>; break;
      case 256 + 17: kern = k_rk4_sell<STAGE, 8, true, 4>; break;
      default: break;
    }
    hipLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, s, p.sell_off.get(), p.sell_coff.get(),
                       p.sell_base.get(), p.sell_cb.get(), p.sell_row.get(), p.sell_len.get(), p.sell_val.get(),
                       p.nslices, p.nshort, p.long_rows.get(), p.nlong, p.rowptr.get(), p.seg.get(), p.col.get(),
                       p.val.get(), p.ndyn, xin, vin, acc, xout, coef, row, dt, p.sell_remap);
    return;
  }
  switch (p.threads) {
    case 64: launch_stage_nt<STAGE, 64>(p, xin, vin, acc, xout, coef, row, dt, s); break;
    case 128: launch_stage_nt<STAGE, 128>(p, xin, vin, acc, xout, coef, row, dt, s); break;
    default: launch_stage_nt<STAGE, 256>(p, xin, vin, acc, xout, coef, row, dt, s); break;
  }
}

// [stage-kernel source: end]

template <int STAGE>
void launch_stage(const sun_prop_s& p, const double* xin, double* xout, const double* coef, int64_t row,
                  double dt, hipStream_t s) {
  launch_stage_v<STAGE>(p, xin, p.vaug.get(), p.acc.get(), xout, coef, row, dt, s);
}

}  // namespace

namespace sun {

// The failure-injection point of the layout builds, for the batched form's
// re-tiling as well.
void layout_failure_point() { maybe_inject_layout_failure(); }

void prop_require_usable(const sun_prop_s& p) {
  SUN_REQUIRE(p.usable, SUN_EINVAL,
              "propagator layout is incomplete after a failed re-layout; select a layout again (sun_prop_tune*)");
}

void prop_finite_check(const sun_prop_s& p, const double* x, int64_t n, hipStream_t s) {
  if (!p.check_finite || n <= 0) return;
  flag_nonfinite(x, n, p.bad.get(), s);
}

bool prop_finite_result(const sun_prop_s& p, hipStream_t s) {
  if (!p.check_finite) return true;
  int h = 0;
  HIP_OK(hipMemcpyAsync(&h, p.bad.get(), sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  if (h != 0) set_int(p.bad.get(), 0, s);
  return h == 0;
}

void prop_stage(const sun_prop_s& p, int stage, const double* xin, const double* vin, double* acc, double* xout,
                const double* coef, int64_t row, double dt, hipStream_t s) {
  switch (stage) {
    case 0: launch_stage_v<0>(p, xin, vin, acc, xout, coef, row, dt, s); break;
    case 1: launch_stage_v<1>(p, xin, vin, acc, xout, coef, row, dt, s); break;
    case 2: launch_stage_v<2>(p, xin, vin, acc, xout, coef, row, dt, s); break;
    case 3: launch_stage_v<3>(p, xin, vin, acc, xout, coef, row, dt, s); break;
    case 4: launch_stage_v<4>(p, xin, vin, acc, xout, coef, row, dt, s); break;
    case 5: launch_stage_v<5>(p, xin, vin, acc, xout, coef, row, dt, s); break;
    case 6: launch_stage_v<6>(p, xin, vin, acc, xout, coef, row, dt, s); break;
    case 7: launch_stage_v<7>(p, xin, vin, acc, xout, coef, row, dt, s); break;
    default: launch_stage_v<8>(p, xin, vin, acc, xout, coef, row, dt, s); break;
  }
  HIP_LAUNCH_OK();
}

int64_t prop_dot_slots(const sun_prop_s& p) { return p.nslices + p.nlong; }

void prop_dot(const sun_prop_s* const* ps, const int* term, const int* slot, const int64_t* slot0, int n,
              const double* const* xs, const double* const* kbs, const int64_t* krows, const double* dstat,
              const double* dcoef, int ndyn, int ntheta, double* gpart, int64_t ld, hipStream_t s) {
  SUN_REQUIRE(n >= 1 && n <= kMaxDotTerms, SUN_EINVAL, "1 to 8 terms per dot launch");
  DotViews dv{};
  dv.n = n;
  int64_t nw = 0;
  for (int j = 0; j < n; ++j) {
    const sun_prop_s& p = *ps[j];
    SUN_REQUIRE(p.layout == 1 && p.ndyn == 0, SUN_EINVAL, "dot products need static generators in sliced layout");
    DotView& D = dv.v[j];
    D.off = p.sell_off.get();
    D.coff = p.sell_coff.get();
    D.gbase = p.sell_base.get();
    D.cb = p.sell_cb.get();
    D.row = p.sell_row.get();
    D.len = p.sell_len.get();
    D.sval = p.sell_val.get();
    D.nslices = p.nslices;
    D.nshort = p.nshort;
    D.nlong = p.nlong;
    D.long_rows = p.long_rows.get();
    D.rowptr = p.rowptr.get();
    D.col = p.col.get();
    D.val = p.val.get();
    D.term = term[j];
    D.slot = slot[j];
    D.wave0 = nw;
    D.slot0 = slot0[j];
    nw += p.nslices + p.nlong;
  }
  if (nw == 0) return;
  unsigned grid = (unsigned)((nw + 3) / 4);
  const int remap = ps[0]->sell_remap;
  if (remap) grid = (grid + 7) / 8 * 8;
  DotStages st{};
  for (int i = 0; i < kDotStages; ++i) {
    st.x[i] = xs[i];
    st.kb[i] = kbs[i];
    st.krow[i] = krows[i];
  }
  auto kern = ps[0]->sell_nt ? k_dot_sell<4, true, kDotStagesPerWave> : k_dot_sell<4, false, kDotStagesPerWave>;
  hipLaunchKernelGGL(kern, dim3(grid, kDotStages / kDotStagesPerWave), dim3(256), 0, s, dv, nw, st, dstat, dcoef, ndyn,
                     ntheta, gpart, ld, remap);
  HIP_LAUNCH_OK();
}

void prop_build_segments(sun_prop_s& p, hipStream_t s) {
  SUN_REQUIRE(p.ndyn >= 1 && p.ndyn <= kMaxRevSeg, SUN_ENOTSUP, "1 to 3 segments for the fused reverse stages");
  p.usable = 0;
  ++p.layout_gen;
  p.long_len = std::min(p.long_len, 255);   // segment starts are stored in 8 bits
  p.sell_segs = p.ndyn;
  build_sell(p, s);
  p.usable = 1;
}

int64_t prop_rev_slots(const sun_prop_s& p) { return p.nslices + p.nlong; }

template <int STAGE, int ND, int KI>
void launch_sell_multi(const sun_prop_s& p, const double* xin, const double* vin, double* acc, double* xout,
                       const MultiCoef& mc, double dt, hipStream_t s) {
  const int64_t waves = (p.nslices + p.nlong) * ((mc.B + KI - 1) / KI);
  if (waves == 0) return;
  unsigned grid = (unsigned)((waves + 3) / 4);
  if (p.sell_remap) grid = (grid + 7) / 8 * 8;
  hipLaunchKernelGGL((k_sell_multi<STAGE, ND, KI>), dim3(grid), dim3(256), 0, s, p.sell_off.get(), p.sell_coff.get(),
                     p.sell_base.get(), p.sell_cb.get(), p.sell_row.get(), p.sell_len.get(), p.sell_seg.get(),
                     p.sell_val.get(), p.nslices, p.nshort, p.long_rows.get(), p.nlong, p.rowptr.get(), p.seg.get(),
                     p.col.get(), p.val.get(), p.M, mc, xin, vin, acc, xout, dt, p.sell_remap);
}

template <int STAGE, int ND>
void launch_sell_multi_ki(const sun_prop_s& p, const double* xin, const double* vin, double* acc, double* xout,
                          const MultiCoef& mc, int ki, double dt, hipStream_t s) {
  switch (ki) {
    case 2: launch_sell_multi<STAGE, ND, 2>(p, xin, vin, acc, xout, mc, dt, s); break;
    case 4: launch_sell_multi<STAGE, ND, 4>(p, xin, vin, acc, xout, mc, dt, s); break;
    default: launch_sell_multi<STAGE, ND, 8>(p, xin, vin, acc, xout, mc, dt, s); break;
  }
}

template <int STAGE>
void launch_sell_multi_nd(const sun_prop_s& p, const double* xin, const double* vin, double* acc, double* xout,
                          const MultiCoef& mc, int ki, double dt, hipStream_t s) {
  switch (p.ndyn) {
    case 1: launch_sell_multi_ki<STAGE, 1>(p, xin, vin, acc, xout, mc, ki, dt, s); break;
    case 2: launch_sell_multi_ki<STAGE, 2>(p, xin, vin, acc, xout, mc, ki, dt, s); break;
    default: launch_sell_multi_ki<STAGE, 3>(p, xin, vin, acc, xout, mc, ki, dt, s); break;
  }
}

void prop_stage_multi(const sun_prop_s& p, int stage, const double* xin, const double* vin, double* acc,
                      double* xout, const MultiCoef& mc, int ki, double dt, hipStream_t s) {
  SUN_REQUIRE(p.layout == 2 && p.sell_segs == p.ndyn && p.ndyn >= 1 && p.ndyn <= kMaxRevSeg, SUN_EINVAL,
              "the multi-instance stage needs the segmented sliced layout");
  switch (stage) {
    case 0: launch_sell_multi_nd<0>(p, xin, vin, acc, xout, mc, ki, dt, s); break;
    case 1: launch_sell_multi_nd<1>(p, xin, vin, acc, xout, mc, ki, dt, s); break;
    case 2: launch_sell_multi_nd<2>(p, xin, vin, acc, xout, mc, ki, dt, s); break;
    default: launch_sell_multi_nd<3>(p, xin, vin, acc, xout, mc, ki, dt, s); break;
  }
  HIP_LAUNCH_OK();
}

template <int STAGE, bool DOTS>
void launch_sell_seg(const sun_prop_s& p, const double* xin, const double* vin, double* acc, double* xout,
                     const double* xdot, const RevDot& rd, int64_t krow, double dt, hipStream_t s) {
  const int64_t waves = p.nslices + p.nlong;
  if (waves == 0) return;
  unsigned grid = (unsigned)((waves + 3) / 4);
  if (p.sell_remap) grid = (grid + 7) / 8 * 8;
  auto kern = k_sell_seg<STAGE, 1, DOTS>;
  if (rd.nseg == 2) kern = k_sell_seg<STAGE, 2, DOTS>;
  else if (rd.nseg == 3) kern = k_sell_seg<STAGE, 3, DOTS>;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, s, p.sell_off.get(), p.sell_coff.get(), p.sell_base.get(),
                     p.sell_cb.get(), p.sell_row.get(), p.sell_len.get(), p.sell_seg.get(), p.sell_val.get(),
                     p.nslices, p.nshort, p.long_rows.get(), p.nlong, p.rowptr.get(), p.seg.get(), p.col.get(),
                     p.val.get(), p.M, xin, vin, acc, xout, xdot, rd, krow, dt, p.sell_remap);
}

void prop_stage_dot(const sun_prop_s& p, int stage, const double* xin, const double* vin, double* acc, double* xout,
                    const double* xdot, const RevDot& rd, int64_t krow, double dt, hipStream_t s) {
  SUN_REQUIRE(p.sell_segs == rd.nseg && rd.nseg >= 1 && rd.nseg <= kMaxRevSeg && p.ndyn == rd.nseg, SUN_EINVAL,
              "fused reverse stage needs the segmented sliced layout of its terms");
  SUN_REQUIRE(rd.ntheta >= 0 && rd.ntheta <= 64, SUN_EINVAL, "at most 64 parameters per wavefront");
  switch (stage) {
    case 4: launch_sell_seg<4, true>(p, xin, vin, acc, xout, xdot, rd, krow, dt, s); break;
    case 5: launch_sell_seg<5, true>(p, xin, vin, acc, xout, xdot, rd, krow, dt, s); break;
    case 6: launch_sell_seg<6, true>(p, xin, vin, acc, xout, xdot, rd, krow, dt, s); break;
    case 7: launch_sell_seg<7, true>(p, xin, vin, acc, xout, xdot, rd, krow, dt, s); break;
    case 8: launch_sell_seg<8, true>(p, xin, vin, acc, xout, xdot, rd, krow, dt, s); break;
    default: SUN_THROW(SUN_EINVAL, "fused reverse stages are 4..8");
  }
  HIP_LAUNCH_OK();
}

void prop_seg_stage(const sun_prop_s& p, int stage, const double* xin, const double* vin, double* acc, double* xout,
                    const double* coef, int64_t row, double dt, hipStream_t s) {
  RevDot rd;
  rd.nseg = p.ndyn;
  for (int d = 0; d < p.ndyn && d < kMaxRevSeg; ++d) rd.slot[d] = d;   // segment d: coefficient c_d(t)
  rd.coef = coef;
  rd.ncoef = p.ndyn;
  SUN_REQUIRE(p.sell_segs == p.ndyn && p.ndyn >= 1 && p.ndyn <= kMaxRevSeg, SUN_EINVAL,
              "segmented layout does not match the time-dependent terms");
  switch (stage) {
    case 0: launch_sell_seg<0, false>(p, xin, vin, acc, xout, nullptr, rd, row, dt, s); break;
    case 1: launch_sell_seg<1, false>(p, xin, vin, acc, xout, nullptr, rd, row, dt, s); break;
    case 2: launch_sell_seg<2, false>(p, xin, vin, acc, xout, nullptr, rd, row, dt, s); break;
    case 3: launch_sell_seg<3, false>(p, xin, vin, acc, xout, nullptr, rd, row, dt, s); break;
    default: SUN_THROW(SUN_ENOTSUP, "the segmented layout runs the forward stages 0..3");
  }
}

}  // namespace sun

extern "C" int sun_prop_create(sun_lind l, const double* static_w, const int32_t* dyn, int32_t ndyn,
                               void* stream, sun_prop* out) {
  return guarded([&] {
    SUN_REQUIRE(out != nullptr, SUN_EINVAL, "out is NULL");
    *out = nullptr;
    SUN_REQUIRE(l != nullptr && static_w != nullptr, SUN_EINVAL, "NULL argument");
    SUN_REQUIRE(ndyn >= 0 && ndyn <= kMaxDyn, SUN_ENOTSUP, "at most 4 time-dependent terms");
    SUN_REQUIRE(ndyn == 0 || dyn != nullptr, SUN_EINVAL, "dyn is NULL");
    const int nt = l->nH + l->P;
    SUN_REQUIRE(nt <= kMaxTerms, SUN_ENOTSUP, "at most 32 terms");
    for (int a = l->nH; a < nt; ++a)
      SUN_REQUIRE(static_w[a] >= 0.0, SUN_EINVAL, "dissipation rates must be >= 0");
    hipStream_t s = as_stream(stream);
    const int64_t M = l->basis->M;
    auto p = new sun_prop_s();
    try {
      p->lind = l;
      p->M = M;
      p->ndyn = ndyn;
      TermList st{};
      DynList dy{};
      DevBuf<double> Kst(M);
      HIP_OK(hipMemsetAsync(Kst.get(), 0, M * sizeof(double), s));
      bool anyK = false;
      for (int a = 0; a < nt; ++a) {
        if (static_w[a] == 0.0) continue;
        const DevCSR& m = a < l->nH ? l->QH[a] : l->R[a - l->nH];
        st.rowptr[st.n] = m.rowptr.get();
        st.col[st.n] = m.col.get();
        st.val[st.n] = m.val.get();
        st.w[st.n] = static_w[a];
        ++st.n;
        if (a >= l->nH) {
          hipLaunchKernelGGL(k_axpy_into, dim3(grid_for(M, 256)), dim3(256), 0, s, M, static_w[a],
                             l->K[a - l->nH].get(), Kst.get());
          HIP_LAUNCH_OK();
          anyK = true;
        }
      }
      for (int d = 0; d < ndyn; ++d) {
        const int a = dyn[d];
        SUN_REQUIRE(a >= 0 && a < nt, SUN_EINVAL, "dynamic term index out of range");
        const DevCSR& m = a < l->nH ? l->QH[a] : l->R[a - l->nH];
        dy.rowptr[d] = m.rowptr.get();
        dy.col[d] = m.col.get();
        dy.val[d] = m.val.get();
        dy.K[d] = a < l->nH ? nullptr : l->K[a - l->nH].get();
      }
      dy.n = ndyn;
      DevBuf<int64_t> cnt(M), off(M);
      hipLaunchKernelGGL(k_fuse_rows, dim3(grid_for(M, 128)), dim3(128), 0, s, M, st, anyK ? Kst.get() : nullptr,
                         dy, 0, cnt.get(), nullptr, nullptr, nullptr, nullptr);
      HIP_LAUNCH_OK();
      p->nnz = exclusive_scan_i64(cnt.get(), off.get(), M, s);
      SUN_REQUIRE(p->nnz < (int64_t)INT32_MAX, SUN_ENOTSUP, "fused matrix has 2^31 or more nonzeros");
      p->rowptr.alloc(M + 1);
      p->col.alloc(p->nnz > 0 ? p->nnz : 1);
      p->val.alloc(p->nnz > 0 ? p->nnz : 1);
      p->seg.alloc(ndyn > 0 ? ndyn * M : 1);
      hipLaunchKernelGGL(k_fuse_rows, dim3(grid_for(M, 128)), dim3(128), 0, s, M, st, anyK ? Kst.get() : nullptr,
                         dy, 1, nullptr, off.get(), p->col.get(), p->val.get(), p->seg.get());
      HIP_LAUNCH_OK();
      hipLaunchKernelGGL(k_i64_to_i32, dim3(grid_for(M, 256)), dim3(256), 0, s, M, off.get(), p->nnz,
                         p->rowptr.get());
      HIP_LAUNCH_OK();
      build_partition(*p, s);
      // sliced ELL at every size for one time-dependent term: with several
      // wavefronts per slice it is ahead of the CSR stream layout even for
      // small generators (measured on the dimer, us per stage: N = 19, 6,163
      // stored entries, 3.0 against 4.1; N = 51, 48,323, 3.3 against 5.2;
      // N = 71, 94,953, 3.3 against 5.9).  With 2-3 time-dependent terms the
      // segmented sliced layout above 100,000 nonzeros and the stream layout
      // below (5.3 against 7.4 us per stage at 45,773 nonzeros with one
      // wavefront per slice).
      p->layout = ndyn <= 1 ? 1 : (p->nnz > kStreamMaxNnz && ndyn <= kMaxRevSeg ? 2 : 0);
      if (p->layout == 1) {
        build_sell(*p, s);
        p->sell_nt = sell_matrix_bytes(*p) > kNontemporalMinBytes ? 1 : 0;
        pick_split(*p, 0);
      }
      if (p->layout == 2) {
        // 2-3 time-dependent terms: one segment each in the sliced layout
        p->long_len = std::min(p->long_len, 255);
        p->sell_segs = ndyn;
        build_sell(*p, s);
      }
      // one workgroup wins while the whole generator is small (measured on
      // the dimer against the sliced kernel with four wavefronts per slice,
      // us per RK4 step: 5.6 against 8.0 at 140 nonzeros, 9.7 against 11.8
      // at 2,224; slower from 3,135 on, 13.8 against 11.4, and 18.9 against
      // 11.5 at 5,425)
      p->resident = (ndyn <= 1 && p->nnz <= kResidentMaxNnz && resident_lds_bytes(M) <= lds_limit()) ? 1 : 0;
      p->bad.alloc(1);
      set_int(p->bad.get(), 0, s);
      p->vaug.alloc(M + 1);
      p->xa.alloc(M + 1);
      p->xb.alloc(M + 1);
      p->acc.alloc(M + 1);
      for (DevBuf<double>* b : {&p->vaug, &p->xa, &p->xb, &p->acc}) {
        hipLaunchKernelGGL(k_fill, dim3(grid_for(M + 1, 256)), dim3(256), 0, s, M + 1, 0.0, b->get());
        HIP_LAUNCH_OK();
        hipLaunchKernelGGL(k_fill, dim3(1), dim3(1), 0, s, (int64_t)1, 1.0, b->get() + M);
        HIP_LAUNCH_OK();
      }
      HIP_OK(hipStreamSynchronize(s));
    } catch (...) {
      delete p;
      throw;
    }
    *out = p;
  });
}

extern "C" int sun_prop_tune(sun_prop p, int32_t block_nnz, int32_t threads, int32_t xcd_remap,
                             void* stream) {
  return guarded([&] {
    SUN_REQUIRE(p != nullptr, SUN_EINVAL, "prop is NULL");
    SUN_REQUIRE(block_nnz >= 128 && block_nnz <= 8192 && (block_nnz & (block_nnz - 1)) == 0, SUN_EINVAL,
                "block_nnz must be a power of two in [128, 8192]");
    SUN_REQUIRE(threads == 64 || threads == 128 || threads == 256, SUN_EINVAL, "threads must be 64, 128 or 256");
    p->usable = 0;
    ++p->layout_gen;
    p->block_nnz = block_nnz;
    p->threads = threads;
    p->xcd_remap = xcd_remap ? 1 : 0;
    p->resident = 0;
    p->layout = 0;
    build_partition(*p, as_stream(stream));
    p->usable = 1;
  });
}

extern "C" int sun_prop_tune_sliced(sun_prop p, int32_t sigma, int32_t long_len, int32_t min_col_bytes,
                                    int32_t flags, void* stream) {
  return guarded([&] {
    SUN_REQUIRE(p != nullptr, SUN_EINVAL, "prop is NULL");
    SUN_REQUIRE(p->ndyn <= kMaxRevSeg, SUN_ENOTSUP, "the sliced layouts support at most three time-dependent terms");
    SUN_REQUIRE(p->ndyn <= 1 || long_len <= 255, SUN_EINVAL,
                "with 2-3 time-dependent terms long_len must be at most 255");
    SUN_REQUIRE(sigma >= 64 && sigma <= 4096 && (sigma & (sigma - 1)) == 0, SUN_EINVAL,
                "sigma must be a power of two in [64, 4096]");
    SUN_REQUIRE(long_len >= 1 && long_len <= 4096, SUN_EINVAL, "long_len must be in [1, 4096]");
    SUN_REQUIRE(min_col_bytes == 1 || min_col_bytes == 2 || min_col_bytes == 4, SUN_EINVAL,
                "min_col_bytes must be 1, 2 or 4");
    p->sigma = sigma;
    p->long_len = long_len;
    p->min_col_bytes = min_col_bytes;
    const int u = (flags >> 16) & 0xFF;
    SUN_REQUIRE(u == 0 || u == 4 || u == 6 || u == 8 || u == 12 || u == 16, SUN_EINVAL,
                "entries per load round (flags bits 16-23) must be 0, 4, 6, 8, 12 or 16");
    const int split = (flags >> 24) & 7;
    SUN_REQUIRE(split == 0 || split == 1 || split == 2 || split == 4, SUN_EINVAL,
                "wavefronts per slice (flags bits 24-26) must be 0, 1, 2 or 4");
    SUN_REQUIRE(split <= 1 || u == 0 || u == 4 || u == 8, SUN_EINVAL,
                "2 or 4 wavefronts per slice take 4 or 8 entries per load round");
    SUN_REQUIRE((flags & ~0x7FF0007) == 0, SUN_EINVAL, "unknown flag bits");
    p->sell_remap = (flags & 1) ? 1 : 0;
    p->sell_pairs = (flags & 4) ? 1 : 0;
    p->sell_nt = (flags & 2) ? 1 : 0;
    p->usable = 0;
    ++p->layout_gen;
    p->resident = 0;
    p->layout = p->ndyn <= 1 ? 1 : 2;
    p->sell_segs = p->ndyn <= 1 ? 0 : p->ndyn;
    build_sell(*p, as_stream(stream));
    if (split == 0) {
      pick_split(*p, u);
    } else {
      p->sell_split = split;
      p->sell_unroll = u ? u : 8;
    }
    p->usable = 1;
  });
}

extern "C" int sun_prop_info(sun_prop p, int64_t* nnz_fused, int64_t* nblocks, int64_t* M) {
  return guarded([&] {
    SUN_REQUIRE(p != nullptr, SUN_EINVAL, "prop is NULL");
    if (nnz_fused) *nnz_fused = p->nnz;
    if (nblocks) *nblocks = p->layout >= 1 ? p->nslices + p->nlong : p->nblocks;
    if (M) *M = p->M;
  });
}

extern "C" int sun_prop_tune_resident(sun_prop p, int32_t on) {
  return guarded([&] {
    SUN_REQUIRE(p != nullptr, SUN_EINVAL, "prop is NULL");
    if (on) {
      SUN_REQUIRE(p->ndyn <= 1, SUN_ENOTSUP, "the resident path supports at most one time-dependent term");
      SUN_REQUIRE(resident_lds_bytes(p->M) <= lds_limit(), SUN_ENOTSUP, "system too large for one workgroup's LDS");
    }
    p->resident = on ? 1 : 0;
  });
}

extern "C" int sun_prop_layout(sun_prop p, int32_t* layout, int64_t* stored_entries, int64_t* long_rows,
                               int64_t* bytes_per_launch) {
  return guarded([&] {
    SUN_REQUIRE(p != nullptr, SUN_EINVAL, "prop is NULL");
    if (layout) *layout = p->layout;
    if (stored_entries) *stored_entries = p->layout >= 1 ? p->sell_nnz : p->nnz;
    if (long_rows) *long_rows = p->layout >= 1 ? p->nlong : 0;
    if (bytes_per_launch) {
      // matrix stream + per-row metadata, excluding the vectors
      int64_t b = 0;
      if (p->layout >= 1) {
        b = sell_matrix_bytes(*p);
      } else {
        b = p->nnz * 12 + (p->M + 1) * 4 + (int64_t)p->ndyn * p->M * 4;
      }
      *bytes_per_launch = b;
    }
  });
}

namespace {

void check_step_size(const sun_prop_s& p, double dt) {
  if (p.dt_max > 0.0 && std::fabs(dt) > p.dt_max)
    SUN_THROW(SUN_EUNSTABLE, "dt = " + std::to_string(dt) + " exceeds the stable step " + std::to_string(p.dt_max) +
                                 " (|lambda|max ~ " + std::to_string(p.rho_guard) + ")");
}

void require_finite(const sun_prop_s& p, hipStream_t s, int64_t steps) {
  if (!prop_finite_result(p, s))
    SUN_THROW(SUN_EDIVERGED, "the state is not finite after " + std::to_string(steps) +
                                 " RK4 steps (NaN or Inf in v; it is returned as computed)");
}

// HIP-graph replay: a chunk of kGraphSteps RK4 steps (4 launches each) on the
// propagator's own vectors is captured once per layout and step size, with
// the stage kernels reading their coefficient rows from a fixed buffer; each
// replay first copies the chunk's 2 kGraphSteps + 1 rows of the caller's
// table there (stream-ordered after the previous replay).  No memset is
// recorded.  Used where a stage is launch-bound (M <= kGraphMaxRows).
constexpr int64_t kGraphSteps = 64;
constexpr int64_t kGraphMaxRows = 160000;

void reset_graph(sun_prop_s& p) {
  if (p.gexec) (void)hipGraphExecDestroy(p.gexec);
  if (p.graph) (void)hipGraphDestroy(p.graph);
  p.gexec = nullptr;
  p.graph = nullptr;
  p.graph_gen = -1;
}

bool graph_wanted(const sun_prop_s& p, int64_t steps) {
  return p.graph_mode != 0 && !p.resident && steps >= kGraphSteps && (p.graph_mode == 2 || p.M <= kGraphMaxRows);
}

void ensure_graph(sun_prop_s& p, double dt) {
  if (p.gexec && p.graph_gen == p.layout_gen && p.graph_dt == dt) return;
  reset_graph(p);
  if (!p.cap_stream) HIP_OK(hipStreamCreateWithFlags(&p.cap_stream, hipStreamNonBlocking));
  const double* cf = nullptr;
  if (p.ndyn > 0) {
    const size_t need = (size_t)(2 * kGraphSteps + 1) * p.ndyn;
    if (p.gcoef.n < need) p.gcoef.alloc(need);
    cf = p.gcoef.get();
  }
  double* va = p.vaug.get();
  double* xa = p.xa.get();
  double* xb = p.xb.get();
  HIP_OK(hipStreamBeginCapture(p.cap_stream, hipStreamCaptureModeThreadLocal));
  hipGraph_t g = nullptr;
  try {
    for (int64_t j = 0; j < kGraphSteps; ++j) {
      launch_stage<0>(p, va, xa, cf, 2 * j, dt, p.cap_stream);
      launch_stage<1>(p, xa, xb, cf, 2 * j + 1, dt, p.cap_stream);
      launch_stage<2>(p, xb, xa, cf, 2 * j + 1, dt, p.cap_stream);
      launch_stage<3>(p, xa, va, cf, 2 * j + 2, dt, p.cap_stream);
    }
    HIP_LAUNCH_OK();
  } catch (...) {
    (void)hipStreamEndCapture(p.cap_stream, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  HIP_OK(hipStreamEndCapture(p.cap_stream, &g));
  p.graph = g;
  HIP_OK(hipGraphInstantiate(&p.gexec, g, nullptr, nullptr, 0));
  p.graph_gen = p.layout_gen;
  p.graph_dt = dt;
}

}  // namespace

sun_prop_s::~sun_prop_s() {
  reset_graph(*this);
  if (cap_stream) (void)hipStreamDestroy(cap_stream);
}

namespace sun {

size_t prop_device_bytes(const sun_prop_s& p) {
  size_t b = 0;
  for (const DevBuf<int>* x : {&p.rowptr, &p.col, &p.seg, &p.blk_row, &p.sell_row, &p.sell_len, &p.sell_off,
                               &p.sell_coff, &p.sell_base, &p.long_rows, &p.sell_seg, &p.bad})
    b += x->bytes();
  for (const DevBuf<double>* x : {&p.val, &p.vaug, &p.xa, &p.xb, &p.acc, &p.sell_val, &p.rec_part, &p.gcoef})
    b += x->bytes();
  return b + p.sell_cb.bytes();
}

}  // namespace sun

extern "C" int sun_prop_device_bytes(sun_prop p, size_t* bytes) {
  return guarded([&] {
    SUN_REQUIRE(p != nullptr && bytes != nullptr, SUN_EINVAL, "NULL argument");
    *bytes = prop_device_bytes(*p);
  });
}

extern "C" int sun_prop_use_graphs(sun_prop p, int32_t mode) {
  return guarded([&] {
    SUN_REQUIRE(p != nullptr, SUN_EINVAL, "propagator is NULL");
    SUN_REQUIRE(mode >= 0 && mode <= 2, SUN_EINVAL, "mode must be 0, 1 or 2");
    p->graph_mode = mode;
    if (mode == 0) reset_graph(*p);
  });
}

extern "C" int sun_propagate(sun_prop p, double* v, const double* coef, double dt, int64_t steps, void* stream) {
  return guarded([&] {
    SUN_REQUIRE(p != nullptr && v != nullptr, SUN_EINVAL, "NULL argument");
    SUN_REQUIRE(steps >= 0, SUN_EINVAL, "steps must be >= 0");
    SUN_REQUIRE(p->ndyn == 0 || coef != nullptr, SUN_EINVAL, "coef is NULL");
    prop_require_usable(*p);
    check_step_size(*p, dt);
    if (steps == 0) return;
    hipStream_t s = as_stream(stream);
    const int64_t M = p->M;
    if (p->resident) {
      hipLaunchKernelGGL(k_rk4_resident, dim3(1), dim3(kResidentThreads), resident_lds_bytes(M), s,
                         p->rowptr.get(), p->col.get(), p->val.get(), p->seg.get(), p->ndyn, (int)M, coef, steps, dt,
                         v);
      HIP_LAUNCH_OK();
      prop_finite_check(*p, v, M, s);
      require_finite(*p, s, steps);
      return;
    }
    HIP_OK(hipMemcpyAsync(p->vaug.get(), v, M * sizeof(double), hipMemcpyDeviceToDevice, s));
    double* va = p->vaug.get();
    double* xa = p->xa.get();
    double* xb = p->xb.get();
    int64_t n0 = 0;
    if (graph_wanted(*p, steps)) {
      ensure_graph(*p, dt);
      const size_t rows = (size_t)(2 * kGraphSteps + 1) * p->ndyn;
      for (; n0 + kGraphSteps <= steps; n0 += kGraphSteps) {
        if (p->ndyn > 0)
          HIP_OK(hipMemcpyAsync(p->gcoef.get(), coef + (size_t)2 * n0 * p->ndyn, rows * sizeof(double),
                                hipMemcpyDeviceToDevice, s));
        HIP_OK(hipGraphLaunch(p->gexec, s));
      }
    }
    for (int64_t n = n0; n < steps; ++n) {
      launch_stage<0>(*p, va, xa, coef, 2 * n, dt, s);
      launch_stage<1>(*p, xa, xb, coef, 2 * n + 1, dt, s);
      launch_stage<2>(*p, xb, xa, coef, 2 * n + 1, dt, s);
      launch_stage<3>(*p, xa, va, coef, 2 * n + 2, dt, s);
    }
    HIP_LAUNCH_OK();
    prop_finite_check(*p, va, M, s);
    HIP_OK(hipMemcpyAsync(v, p->vaug.get(), M * sizeof(double), hipMemcpyDeviceToDevice, s));
    require_finite(*p, s, steps);
  });
}

// Fixed device array for the allocation-free recording entry point (see
// record_scratch below): 2 * 512 doubles, the most partial sums the
// observable's dot product uses (record_blocks() <= 512).
constexpr int kRecordScratchDoubles = 1024;
static __device__ __align__(256) double scratch[kRecordScratchDoubles];

namespace {

// Body of sun_propagate_record: `part` holds the 2*nb partial sums of the
// observable's dot products (nb = record_blocks(M)); it may be NULL when obs
// is NULL.
int record_blocks(int64_t M) { return (int)std::min<int64_t>(512, std::max<int64_t>(1, (M + 4095) / 4096)); }

void propagate_record(sun_prop_s& P, double* v, const double* coef, double dt, int64_t steps, int64_t every,
                      double* states, int64_t ld, const double* x, double x0, double* obs, double* part,
                      hipStream_t s) {
  sun_prop_s* p = &P;
  const int64_t M = p->M;
  const int nb = record_blocks(M);
  HIP_OK(hipMemcpyAsync(p->vaug.get(), v, M * sizeof(double), hipMemcpyDeviceToDevice, s));
  double* va = p->vaug.get();
  double* xa = p->xa.get();
  double* xb = p->xb.get();
  int64_t rec = 0;
  if (p->resident) {
    // one launch per recording interval (and one for the remaining steps)
    for (int64_t n0 = 0; n0 < steps; n0 += every) {
      const int64_t cnt = std::min<int64_t>(every, steps - n0);
      const double* c = p->ndyn ? coef + 2 * n0 * p->ndyn : nullptr;
      hipLaunchKernelGGL(k_rk4_resident, dim3(1), dim3(kResidentThreads), resident_lds_bytes(M), s,
                         p->rowptr.get(), p->col.get(), p->val.get(), p->seg.get(), p->ndyn, (int)M, c, cnt, dt,
                         va);
      if (cnt == every) {
        if (states)
          HIP_OK(hipMemcpyAsync(states + rec * ld, va, M * sizeof(double), hipMemcpyDeviceToDevice, s));
        if (obs) expect_launch(M, va, 1, M, x, nullptr, x0, 0.0, obs + rec, nullptr, part, nb, s);
        ++rec;
      }
    }
    HIP_LAUNCH_OK();
    prop_finite_check(*p, va, M, s);
    HIP_OK(hipMemcpyAsync(v, va, M * sizeof(double), hipMemcpyDeviceToDevice, s));
    require_finite(*p, s, steps);
    return;
  }
  for (int64_t n = 0; n < steps; ++n) {
    launch_stage<0>(*p, va, xa, coef, 2 * n, dt, s);
    launch_stage<1>(*p, xa, xb, coef, 2 * n + 1, dt, s);
    launch_stage<2>(*p, xb, xa, coef, 2 * n + 1, dt, s);
    launch_stage<3>(*p, xa, va, coef, 2 * n + 2, dt, s);
    if ((n + 1) % every == 0) {
      if (states)
        HIP_OK(hipMemcpyAsync(states + rec * ld, va, M * sizeof(double), hipMemcpyDeviceToDevice, s));
      if (obs) expect_launch(M, va, 1, M, x, nullptr, x0, 0.0, obs + rec, nullptr, part, nb, s);
      ++rec;
    }
  }
  HIP_LAUNCH_OK();
  prop_finite_check(*p, va, M, s);
  HIP_OK(hipMemcpyAsync(v, p->vaug.get(), M * sizeof(double), hipMemcpyDeviceToDevice, s));
  require_finite(*p, s, steps);
}

void check_record_args(const sun_prop_s* p, const double* v, const double* coef, int64_t steps, int64_t every,
                       const double* states, int64_t ld, const double* x, const double* obs) {
  SUN_REQUIRE(p != nullptr && v != nullptr, SUN_EINVAL, "NULL argument");
  SUN_REQUIRE(steps >= 0 && every >= 1, SUN_EINVAL, "steps must be >= 0 and every >= 1");
  SUN_REQUIRE(p->ndyn == 0 || coef != nullptr, SUN_EINVAL, "coef is NULL");
  SUN_REQUIRE(states == nullptr || ld >= p->M, SUN_EINVAL, "ld must be >= M");
  SUN_REQUIRE(obs == nullptr || x != nullptr, SUN_EINVAL, "obs needs x");
  prop_require_usable(*p);
}

// ---------------------------------------------------------------------------
// Allocation-free recording: the observable's partial sums live in a fixed
// file-scope device array instead of a buffer the object allocates on first
// use.  Each device holds its own copy of the array; its address is looked up
// once per device (hipGetSymbolAddress, with that device current) and only
// that address is handed to kernels.  Calls that overlap on one device share
// the array and race.
// ---------------------------------------------------------------------------
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

double* record_scratch() {
  int dev = -1;
  HIP_OK(hipGetDevice(&dev));
  SUN_REQUIRE(dev >= 0 && dev < kMaxDevices, SUN_ENOTSUP, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* ptr = nullptr;
    HIP_OK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    SUN_REQUIRE(ptr != nullptr, SUN_EDEVICE, "hipGetSymbolAddress returned NULL for the record scratch array");
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" int sun_propagate_record(sun_prop p, double* v, const double* coef, double dt, int64_t steps,
                                    int64_t every, double* states, int64_t ld, const double* x, double x0,
                                    double* obs, void* stream) {
  return guarded([&] {
    check_record_args(p, v, coef, steps, every, states, ld, x, obs);
    check_step_size(*p, dt);
    if (steps == 0) return;
    const int nb = record_blocks(p->M);
    if (obs && p->rec_part.n < (size_t)(2 * nb)) p->rec_part.alloc(2 * nb);
    propagate_record(*p, v, coef, dt, steps, every, states, ld, x, x0, obs, p->rec_part.get(), as_stream(stream));
  });
}

extern "C" int sun_propagate_record_noalloc(sun_prop p, double* v, const double* coef, double dt, int64_t steps,
                                            int64_t every, double* states, int64_t ld, const double* x, double x0,
                                            double* obs, void* stream) {
  return guarded([&] {
    check_record_args(p, v, coef, steps, every, states, ld, x, obs);
    check_step_size(*p, dt);
    if (steps == 0) return;
    const int nb = record_blocks(p->M);
    SUN_REQUIRE(2 * nb <= kRecordScratchDoubles, SUN_ENOTSUP,
                "observable partials exceed the fixed scratch array (1024 doubles)");
    double* part = obs ? record_scratch() : nullptr;
    propagate_record(*p, v, coef, dt, steps, every, states, ld, x, x0, obs, part, as_stream(stream));
  });
}

namespace {

// x[i] = a deterministic pseudo-random value in [-1, 1) (splitmix64 of i), x[M] = 0
__global__ void k_spec_init(int64_t M, double* __restrict__ x) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= M; i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t z = (uint64_t)i + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    x[i] = i < M ? (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0 : 0.0;
  }
}

// x = y / sqrt(*n2) on rows < M, x[M] = 0
__global__ void k_spec_scale(int64_t M, const double* __restrict__ y, const double* __restrict__ n2,
                             double* __restrict__ x) {
  const double inv = 1.0 / sqrt(*n2);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= M; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = i < M ? y[i] * inv : 0.0;
}

}  // namespace

namespace {

// |lambda|max of the linear part of G at the frozen coefficients coef (host
// double[ndyn]) by `iters` power-iteration steps (mean growth per application
// over the second half).
double spectral_radius(sun_prop_s& P, const double* coef, int iters, hipStream_t s) {
  sun_prop_s* p = &P;
  const int64_t M = p->M;
  DevBuf<double> x(M + 1), y(M + 1), zero(M + 1), acc(M + 1), n2(iters), cdev(p->ndyn > 0 ? p->ndyn : 1);
  const int nb = (int)std::min<int64_t>(512, std::max<int64_t>(1, (M + 4095) / 4096));
  DevBuf<double> part(2 * nb);
  if (p->ndyn > 0) HIP_OK(hipMemcpyAsync(cdev.get(), coef, p->ndyn * sizeof(double), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_fill, dim3(grid_for(M + 1, 256)), dim3(256), 0, s, M + 1, 0.0, zero.get());
  hipLaunchKernelGGL(k_spec_init, dim3(grid_for(M + 1, 256)), dim3(256), 0, s, M, y.get());
  HIP_LAUNCH_OK();
  // start from the normalised pseudo-random vector
  expect_launch(M, y.get(), 1, M, y.get(), nullptr, 0.0, 0.0, n2.get(), nullptr, part.get(), nb, s);
  hipLaunchKernelGGL(k_spec_scale, dim3(grid_for(M + 1, 256)), dim3(256), 0, s, M, y.get(), n2.get(), x.get());
  HIP_LAUNCH_OK();
  for (int i = 0; i < iters; ++i) {
    // stage 0 with a zero base vector and dt = 2: y = G x (x[M] = 0 leaves K out)
    prop_stage(*p, 0, x.get(), zero.get(), acc.get(), y.get(), cdev.get(), 0, 2.0, s);
    expect_launch(M, y.get(), 1, M, y.get(), nullptr, 0.0, 0.0, n2.get() + i, nullptr, part.get(), nb, s);
    hipLaunchKernelGGL(k_spec_scale, dim3(grid_for(M + 1, 256)), dim3(256), 0, s, M, y.get(), n2.get() + i,
                       x.get());
    HIP_LAUNCH_OK();
  }
  std::vector<double> h(iters);
  HIP_OK(hipMemcpyAsync(h.data(), n2.get(), iters * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  // mean log growth per application over the second half of the iterations
  double acc_log = 0.0;
  const int first = iters / 2;
  for (int i = first; i < iters; ++i) {
    SUN_REQUIRE(h[i] > 0.0 && std::isfinite(h[i]), SUN_ERANGE, "power iteration lost its vector (G x = 0 or overflow)");
    acc_log += 0.5 * std::log(h[i]);
  }
  return std::exp(acc_log / (double)(iters - first));
}

// Smallest |z| on the boundary of classical RK4's stability region
// |1 + z + z^2/2 + z^3/6 + z^4/24| <= 1 over the closed left half-plane:
// 2.6156 (at arg z ~ 122.6 degrees; 2.785 on the negative real axis, 2.828 on
// the imaginary axis).  Any eigenvalue with Re <= 0 and |lambda| dt below it
// is inside the region.
constexpr double kRk4SafeRadius = 2.6;

}  // namespace

extern "C" int sun_prop_spectral_radius(sun_prop p, const double* coef, int32_t iters, double* rho, void* stream) {
  return guarded([&] {
    SUN_REQUIRE(p != nullptr && rho != nullptr, SUN_EINVAL, "NULL argument");
    SUN_REQUIRE(p->ndyn == 0 || coef != nullptr, SUN_EINVAL, "coef is NULL");
    SUN_REQUIRE(iters >= 2 && iters <= 100000, SUN_EINVAL, "iters must be in [2, 100000]");
    prop_require_usable(*p);
    *rho = spectral_radius(*p, coef, iters, as_stream(stream));
  });
}

extern "C" int sun_prop_guard_stability(sun_prop p, const double* coef_lo, const double* coef_hi, int32_t iters,
                                        double limit, double* rho_max, void* stream) {
  return guarded([&] {
    SUN_REQUIRE(p != nullptr, SUN_EINVAL, "prop is NULL");
    if (limit < 0.0) {   // guard off
      p->dt_max = 0.0;
      p->rho_guard = 0.0;
      if (rho_max) *rho_max = 0.0;
      return;
    }
    SUN_REQUIRE(p->ndyn == 0 || (coef_lo != nullptr && coef_hi != nullptr), SUN_EINVAL, "coefficient range is NULL");
    SUN_REQUIRE(iters >= 2 && iters <= 100000, SUN_EINVAL, "iters must be in [2, 100000]");
    prop_require_usable(*p);
    const double lim = limit > 0.0 ? limit : kRk4SafeRadius;
    hipStream_t s = as_stream(stream);
    double worst = 0.0;
    // every corner of the box [coef_lo, coef_hi] of the time-dependent coefficients
    for (int corner = 0; corner < (1 << p->ndyn); ++corner) {
      double c[kMaxDyn] = {};
      for (int d = 0; d < p->ndyn; ++d) c[d] = (corner >> d & 1) ? coef_hi[d] : coef_lo[d];
      worst = std::max(worst, spectral_radius(*p, c, iters, s));
    }
    SUN_REQUIRE(worst > 0.0 && std::isfinite(worst), SUN_ERANGE, "no finite spectral radius estimate");
    p->rho_guard = worst;
    p->dt_max = lim / worst;
    if (rho_max) *rho_max = worst;
  });
}

extern "C" int sun_debug_inject_failure(int32_t site) {
  return guarded([&] {
    SUN_REQUIRE(site == 0 || site == 1, SUN_EINVAL, "site must be 0 (clear) or 1 (the next layout build)");
    g_inject_layout_failure.store(site);
  });
}

extern "C" int sun_prop_check_finite(sun_prop p, int32_t on) {
  return guarded([&] {
    SUN_REQUIRE(p != nullptr, SUN_EINVAL, "prop is NULL");
    p->check_finite = on ? 1 : 0;
  });
}

extern "C" int sun_propagate_profile(sun_prop p, double* v, const double* coef, double dt, int64_t steps,
                                     void* stream, double* stage_ms, int64_t* launches) {
  return guarded([&] {
    SUN_REQUIRE(p != nullptr && v != nullptr && stage_ms != nullptr, SUN_EINVAL, "NULL argument");
    SUN_REQUIRE(steps >= 0, SUN_EINVAL, "steps must be >= 0");
    SUN_REQUIRE(p->ndyn == 0 || coef != nullptr, SUN_EINVAL, "coef is NULL");
    prop_require_usable(*p);
    check_step_size(*p, dt);
    hipStream_t s = as_stream(stream);
    const int64_t M = p->M;
    for (int i = 0; i < 4; ++i) stage_ms[i] = 0.0;
    if (launches) *launches = 4 * steps;
    if (steps == 0) return;
    // one event pair per launch, recorded on the launch stream
    std::vector<hipEvent_t> ev(8 * steps, nullptr);
    struct Guard {
      std::vector<hipEvent_t>& e;
      ~Guard() { for (auto x : e) if (x) (void)hipEventDestroy(x); }
    } guard{ev};
    for (auto& e : ev) HIP_OK(hipEventCreate(&e));
    HIP_OK(hipMemcpyAsync(p->vaug.get(), v, M * sizeof(double), hipMemcpyDeviceToDevice, s));
    double* va = p->vaug.get();
    double* xa = p->xa.get();
    double* xb = p->xb.get();
    for (int64_t n = 0; n < steps; ++n) {
      hipEvent_t* e = &ev[8 * n];
      HIP_OK(hipEventRecord(e[0], s));
      launch_stage<0>(*p, va, xa, coef, 2 * n, dt, s);
      HIP_OK(hipEventRecord(e[1], s));
      HIP_OK(hipEventRecord(e[2], s));
      launch_stage<1>(*p, xa, xb, coef, 2 * n + 1, dt, s);
      HIP_OK(hipEventRecord(e[3], s));
      HIP_OK(hipEventRecord(e[4], s));
      launch_stage<2>(*p, xb, xa, coef, 2 * n + 1, dt, s);
      HIP_OK(hipEventRecord(e[5], s));
      HIP_OK(hipEventRecord(e[6], s));
      launch_stage<3>(*p, xa, va, coef, 2 * n + 2, dt, s);
      HIP_OK(hipEventRecord(e[7], s));
    }
    HIP_LAUNCH_OK();
    prop_finite_check(*p, va, M, s);
    HIP_OK(hipMemcpyAsync(v, p->vaug.get(), M * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIP_OK(hipStreamSynchronize(s));
    require_finite(*p, s, steps);
    for (int64_t n = 0; n < steps; ++n)
      for (int i = 0; i < 4; ++i) {
        float ms = 0.f;
        HIP_OK(hipEventElapsedTime(&ms, ev[8 * n + 2 * i], ev[8 * n + 2 * i + 1]));
        stage_ms[i] += ms;
      }
  });
}

extern "C" void sun_prop_free(sun_prop p) { delete p; }
