// Batched RK4 propagation: many parameter instances of the Bloch ODE
// (eq. 9; Sec. IV step 3.1) advanced together, one launch per RK4 stage for
// all instances of all groups.
//
// Instances are grouped by their assembled system (one sun_lind per group,
// e.g. one group per Hilbert-space dimension N).  Instance b of group g has
// the generator
//     G_b(t) = sum_a c_{b,a}(t) T_a,   K_b(t) = sum_{a dissipator} c_{b,a}(t) K_a,
//     c_{b,a}(t_k) = w[b][a] + u[b][a] * wave[k]
// on the half-step grid t_k (k = 0..2*steps), which covers a drive
// eps_b(t) = E + A_b cos(omega t) on one term and a per-instance rate gamma_b
// on another.
//
// Layout.  Each group keeps one fused CSR whose row r lists the entries of
// T_0 row r, then T_1 row r, ... (the free vector of a dissipator term as an
// extra column M), with the segment boundaries per row.  Rows and columns
// are stored in an interleaved order: generator S_p at 2p, J_p at 2p+1, the
// diagonal generators D_l after them in their own order.  The diagonal part
// of any Hamiltonian couples S_p with J_p, so in the grouped order
// (S_0..S_{P-1}, J_0.., D_1..) every S row gathers from two regions P rows
// apart; interleaved, neighbouring rows gather neighbouring state rows and
// the L2 holds them.  Each row keeps its entries in the grouped column
// order, so the sums are formed exactly as in the plain propagator.  The state of a
// group is row-major [M+1][ld] with the instance index fastest (ld = number
// of instances rounded up to 128), and X[M][b] = 1.
//
// Kernels.  A lane group of T lanes handles one row for a tile of T (one
// instance per lane) or 2T (two per lane, 16-byte gathers) consecutive
// instances, so every nonzero's gather reads contiguous doubles of one state
// row and the matrix row is read once per tile.  k_batch_stage_lds (default)
// takes one (instance tile, block of rows) item per workgroup with the
// block's columns, values and row/segment pointers staged in LDS, items
// numbered tile-major and each XCD taking one eighth of every group;
// k_batch_stage_xlds also stages the block's distinct gathered state rows;
// k_batch_stage (rows of more than 1024 entries) reads the matrix from
// global memory, one wavefront per item; k_batch_rows takes one wavefront
// per (row, tile) with the matrix read through the scalar cache;
// k_batch_pipe keeps two persistent workgroups per CU that stage the next
// block's gathered state rows while summing the current one from LDS.
#include <algorithm>
#include <cstring>
#include <memory>
#include <vector>

#include "prop_internal.hpp"

using namespace sun;

namespace {

constexpr int kMaxBTerms = 8;

struct GroupDev {
  const int* rowptr;     // [M+1]
  const int* segptr;     // [M * nt]: start of segment a of row r at segptr[r * nt + a]
  const int* col;
  const double* val;
  const double* w;       // [B * nt]
  const double* u;       // [B * nt]
  const double* wave;    // [2 * steps + 1]
  double* v;             // [(M+1) * ld]
  double* xa;
  double* xb;
  double* acc;           // [M * ld]
  double dt;
  int M, B, ld, nt, tile, rows_per_item;
  int row_blocks, tiles;
  int64_t item0;         // first work item of this group (per-wavefront path)
  const int* blk_row;    // LDS path: row blocks [blk_row[i], blk_row[i+1])
  int nblk;              // LDS path: number of row blocks (0: per-wavefront path)
  int vec;               // LDS path: instances per lane (tile = tile lanes x vec instances)
  int xlds;              // 1: the gathered state rows are staged in LDS as well (path 3)
  const int* ucol_ptr;   // path 3: distinct columns of block i are ucol[ucol_ptr[i] .. ucol_ptr[i+1])
  const int* ucol;
  const unsigned short* lidx;   // path 3: position of every stored entry's column in its block's list
  int p5;                // 1: one wavefront per (row, tile), matrix through the scalar cache (path 5)
  int p7;                // 1: persistent pipelined staging (path 7)
  int p7_nblk;           // path 7: blocks
  const int4* p7_meta;   // path 7, per block: {blob offset and length in 16-byte units, rows, entries}
  const int* p7_ucol;    // path 7, per block kP7Slots columns, slot s at (s % kP7Half) * 8 + s / kP7Half
  const uint4* p7_blob;  // path 7: the blocks' matrix data
  int p7_nlong;          // path 7: rows summed straight from global memory
  const int* p7_long;
};

}  // namespace

struct sun_batch_s {
  int ngroups = 0;
  std::vector<const sun_lind_s*> lind;
  std::vector<int> B, tile, rows_per_item;
  std::vector<int64_t> M, nnz, steps, done;
  std::vector<int> P;       // pairs of the group's basis (interleaved stored order)
  std::vector<double> dt;
  std::vector<const double*> w, u, wave;
  std::vector<DevBuf<int>> rowptr, segptr, col;
  std::vector<DevBuf<double>> val, v, xa, xb, acc;
  std::vector<int> ld, nt;
  DevBuf<GroupDev> gdev;
  std::vector<GroupDev> ghost;
  std::vector<int> order;   // groups sorted by decreasing remaining steps
  std::vector<std::vector<int>> h_rowptr;   // host copies, for the LDS row-block partition
  std::vector<DevBuf<int>> blk_row;
  std::vector<int> nblk;    // row blocks of the LDS path (0: the group uses the per-wavefront path)
  std::vector<int> path;    // 0: LDS path when every row fits, 1: per-wavefront path, 2: as 0 with two instances
                            // per lane, 3: as 2 with the gathered state rows staged in LDS
  std::vector<int> xl;      // 1 when the group runs path 3
  std::vector<DevBuf<int>> xu_ptr, xu_col;
  std::vector<DevBuf<unsigned short>> xu_lidx;
  // path 4: instance-major state ([B][M+1], grouped order, entry M = 1) on a
  // segmented sliced layout of the group's generator (the terms whose
  // coefficients differ between instances as segments, the rest merged)
  std::vector<sun_prop> mprop;
  std::vector<std::vector<int>> mterm;   // the segment terms
  std::vector<DevBuf<double>> mv, mxa, mxb, macc;
  // path 7: block data (meta as 4 ints per block), slot columns, blobs, long rows
  std::vector<DevBuf<int>> p7_meta, p7_ucol, p7_long;
  std::vector<DevBuf<uint4>> p7_blob;
  std::vector<int> p7_nblk, p7_nlong;
  // 0 after a re-tiling of the group failed part-way: sun_batch_run refuses
  // to advance it (its layout is incomplete) until it is tuned again
  std::vector<int> usable;
  ~sun_batch_s() {
    for (sun_prop q : mprop)
      if (q) sun_prop_free(q);
  }
};

namespace {

// Fused per-term rows: count (mode 0) or fill (mode 1).
struct TermPtrs {
  int n;
  const int* rowptr[kMaxBTerms];
  const int* col[kMaxBTerms];
  const double* val[kMaxBTerms];
  const double* K[kMaxBTerms];
};

// Grouped generator index -> stored row (S_p -> 2p, J_p -> 2p+1, D unchanged);
// P = 0 is the identity.
__device__ __host__ inline int64_t inter(int64_t i, int64_t P) {
  return i < P ? 2 * i : (i < 2 * P ? 2 * (i - P) + 1 : i);
}

__global__ void k_batch_fuse(int64_t M, int64_t P, TermPtrs t, int mode, int64_t* __restrict__ cnt,
                             const int64_t* __restrict__ off, int* __restrict__ segptr, int* __restrict__ col,
                             double* __restrict__ val) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < M; r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = inter(r, P);   // stored row of grouped row r
    int64_t w = mode ? off[q] : 0, n = 0;
    for (int a = 0; a < t.n; ++a) {
      if (mode) segptr[q * t.n + a] = (int)(w + n);
      for (int e = t.rowptr[a][r]; e < t.rowptr[a][r + 1]; ++e) {
        if (mode) { col[w + n] = (int)inter(t.col[a][e], P); val[w + n] = t.val[a][e]; }
        ++n;
      }
      if (t.K[a] && t.K[a][r] != 0.0) {
        if (mode) { col[w + n] = (int)M; val[w + n] = t.K[a][r]; }
        ++n;
      }
    }
    if (!mode) cnt[q] = n;
  }
}

__global__ void k_b_i64_to_i32(int64_t n, const int64_t* __restrict__ a, int64_t total, int* __restrict__ b) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = (int)a[i];
  if (blockIdx.x == 0 && threadIdx.x == 0) b[n] = (int)total;
}

// instance-major [B][M] (grouped order) <-> row-major [M+1][ld] (stored
// order; row M set to 1)
__global__ void k_to_rowmajor(int M, int P, int B, int ld, const double* __restrict__ src, double* __restrict__ dst) {
  const int64_t total = (int64_t)M * ld;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(i / ld), b = (int)(i % ld);
    dst[inter(r, P) * ld + b] = b < B ? src[(int64_t)b * M + r] : 0.0;
  }
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < ld; b += (int64_t)gridDim.x * blockDim.x)
    dst[(int64_t)M * ld + b] = 1.0;
}

__global__ void k_from_rowmajor(int M, int P, int B, int ld, const double* __restrict__ src, double* __restrict__ dst) {
  const int64_t total = (int64_t)M * B;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(i / M), r = (int)(i % M);
    dst[i] = src[inter(r, P) * ld + b];
  }
}

__global__ void k_b_fill(int64_t n, double v, double* __restrict__ a) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

// path 4 state (instance-major [B][ldv], grouped order, entry M = 1) from a
// row-major stored state ([M+1][ld], interleaved order), and back
__global__ void k_rm_to_im(int M, int P, int B, int ld, int64_t ldv, const double* __restrict__ src,
                           double* __restrict__ dst) {
  const int64_t total = (int64_t)B * (M + 1);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(i / (M + 1)), r = (int)(i % (M + 1));
    dst[(int64_t)b * ldv + r] = r < M ? src[inter(r, P) * ld + b] : 1.0;
  }
}

__global__ void k_im_to_rm(int M, int P, int B, int ld, int64_t ldv, const double* __restrict__ src,
                           double* __restrict__ dst) {
  const int64_t total = (int64_t)M * ld;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(i / ld), b = (int)(i % ld);
    dst[inter(r, P) * ld + b] = b < B ? src[(int64_t)b * ldv + r] : 0.0;
  }
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < ld; b += (int64_t)gridDim.x * blockDim.x)
    dst[(int64_t)M * ld + b] = 1.0;
}

// instance-major [B][M] caller layout <-> path 4 state [B][ldv] (entry M = 1)
__global__ void k_to_im(int M, int B, int64_t ldv, const double* __restrict__ src, double* __restrict__ dst) {
  const int64_t total = (int64_t)B * (M + 1);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = i / (M + 1);
    const int r = (int)(i % (M + 1));
    dst[b * ldv + r] = r < M ? src[b * M + r] : 1.0;
  }
}

__global__ void k_from_im(int M, int B, int64_t ldv, const double* __restrict__ src, double* __restrict__ dst) {
  const int64_t total = (int64_t)B * M;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = i / M;
    const int r = (int)(i % M);
    dst[i] = src[b * ldv + r];
  }
}

// One RK4 stage for every active group.  stage_in/stage_out select the
// buffers: stage 0 reads v writes xa, 1 reads xa writes xb, 2 reads xb writes
// xa, 3 reads xa writes v.
template <int STAGE>
__global__ __launch_bounds__(256) void k_batch_stage(const GroupDev* __restrict__ groups, const int* __restrict__ gorder,
                                                     int nactive, int64_t nitems, const int64_t* __restrict__ step) {
  const int lane = threadIdx.x & 63;
  const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t it = __builtin_amdgcn_readfirstlane((int)wave0); it < nitems; it += nwaves) {
    // locate the group of this item (few groups: linear scan over the active ones)
    int gi = 0;
    for (int q = 1; q < nactive; ++q)
      if (groups[gorder[q]].item0 <= it) gi = q;
    const GroupDev& G = groups[gorder[gi]];
    const int64_t local = it - G.item0;
    const int rb = (int)(local / G.tiles), tb = (int)(local % G.tiles);
    const int T = G.tile;
    const int sub = lane / T, bl = lane % T;
    const int b = tb * T + bl;
    const int nt = G.nt;
    const int64_t k0 = 2 * step[gorder[gi]];
    const int krow = STAGE == 0 ? 0 : (STAGE == 3 ? 2 : 1);
    const double ph = G.wave[k0 + krow];
    double coefb[kMaxBTerms];
#pragma unroll
    for (int a = 0; a < kMaxBTerms; ++a)
      coefb[a] = (a < nt && b < G.B) ? G.w[(int64_t)b * nt + a] + G.u[(int64_t)b * nt + a] * ph : 0.0;
    const double* xin = STAGE == 0 ? G.v : (STAGE == 1 ? G.xa : (STAGE == 2 ? G.xb : G.xa));
    double* xout = STAGE == 0 ? G.xa : (STAGE == 1 ? G.xb : (STAGE == 2 ? G.xa : G.v));
    const int rpw = 64 / T;   // rows handled side by side in one wavefront
    const int r_begin = rb * G.rows_per_item;
    const int r_end = min(G.M, r_begin + G.rows_per_item);
    const int ld = G.ld;
    for (int r = r_begin + sub; r < r_end; r += rpw) {
      const int e_end = G.rowptr[r + 1];
      double ysum = 0.0;
      for (int a = 0; a < nt; ++a) {
        const int s0 = G.segptr[(int64_t)r * nt + a];
        const int s1 = (a + 1 < nt) ? G.segptr[(int64_t)r * nt + a + 1] : e_end;
        double s = 0.0;
        int e = s0;
        for (; e + 4 <= s1; e += 4) {
          const int c0 = G.col[e], c1 = G.col[e + 1], c2 = G.col[e + 2], c3 = G.col[e + 3];
          const double v0 = G.val[e], v1 = G.val[e + 1], v2 = G.val[e + 2], v3 = G.val[e + 3];
          const double x0 = xin[(int64_t)c0 * ld + b], x1 = xin[(int64_t)c1 * ld + b];
          const double x2 = xin[(int64_t)c2 * ld + b], x3 = xin[(int64_t)c3 * ld + b];
          s += v0 * x0;
          s += v1 * x1;
          s += v2 * x2;
          s += v3 * x3;
        }
        for (; e < s1; ++e) s += G.val[e] * xin[(int64_t)G.col[e] * ld + b];
        ysum += coefb[a] * s;
      }
      if (b < G.B) {
        const int64_t ix = (int64_t)r * ld + b;
        const double vr = G.v[ix];
        const double dt = G.dt;
        if (STAGE == 0) {
          xout[ix] = vr + (0.5 * dt) * ysum;
          G.acc[ix] = ysum;
        } else if (STAGE == 1) {
          xout[ix] = vr + (0.5 * dt) * ysum;
          G.acc[ix] = G.acc[ix] + 2.0 * ysum;
        } else if (STAGE == 2) {
          xout[ix] = vr + dt * ysum;
          G.acc[ix] = G.acc[ix] + 2.0 * ysum;
        } else {
          xout[ix] = vr + (dt / 6.0) * (G.acc[ix] + ysum);
        }
      }
    }
  }
}

// LDS path: one workgroup per (instance tile, block of rows), the block at
// most kLdsRows rows and kLdsCap stored entries.  The block's columns,
// values, row and segment pointers are staged in LDS, so the gathers of a row
// wait only on LDS reads; each lane group of T lanes sums one row for T
// instances, term by term in row order (the same order and arithmetic as
// k_batch_stage).
constexpr int kLdsCap = 1024;
constexpr int kLdsRows = 128;

// Row stride of the LDS table of tile coefficients c_a(t) (a tile has at most
// 128 instances: T, one per lane, or 128, two per lane).
constexpr int kCfStride = 128;

// Stage arithmetic of one state element: returns the new xout, and the new
// accumulator through acc_out (stages 0-2).
template <int STAGE>
__device__ inline double lds_stage(double vr, double ar, double ysum, double dt, double& acc_out) {
  if (STAGE == 0) {
    acc_out = ysum;
    return vr + (0.5 * dt) * ysum;
  } else if (STAGE == 1) {
    acc_out = ar + 2.0 * ysum;
    return vr + (0.5 * dt) * ysum;
  } else if (STAGE == 2) {
    acc_out = ar + 2.0 * ysum;
    return vr + dt * ysum;
  } else {
    return vr + (dt / 6.0) * (ar + ysum);
  }
}

// One instance tile (T lanes per row, one instance per lane) over the rows
// of the block staged in LDS.
template <int STAGE>
__device__ inline void lds_rows(const GroupDev& G, int64_t k0, int tb, int r0, int nr, const int* s_col,
                                const double* s_val, const int* s_rp, const int* s_seg, const double* s_cf) {
  const int tid = threadIdx.x;
  const int T = G.tile;
  const int ngrp = 256 / T, lg = tid / T, bl = tid % T;
  const int nt = G.nt;
  const int krow = STAGE == 0 ? 0 : (STAGE == 3 ? 2 : 1);
  const double ph = G.wave[k0 + krow];
  const double* xin = STAGE == 0 ? G.v : (STAGE == 1 ? G.xa : (STAGE == 2 ? G.xb : G.xa));
  double* xout = STAGE == 0 ? G.xa : (STAGE == 1 ? G.xb : (STAGE == 2 ? G.xa : G.v));
  const int ld = G.ld;
  const int b = tb * T + bl;
  const double* xb = xin + b;
  (void)ph;
  if (b >= G.B) return;   // a lane past the last instance gathers nothing (the tile's padding)
  for (int lr = lg; lr < nr; lr += ngrp) {
    const int ee = s_rp[lr + 1];
    // the row's own state entries are loaded before its gathers
    const int64_t ix = (int64_t)(r0 + lr) * ld + b;
    const bool own = b < G.B;
    const double vr = own ? G.v[ix] : 0.0;
    const double ar = (own && STAGE != 0) ? G.acc[ix] : 0.0;
    double ysum = 0.0;
    for (int a = 0; a < nt; ++a) {
      const int s0 = s_seg[lr * nt + a];
      const int s1 = (a + 1 < nt) ? s_seg[lr * nt + a + 1] : ee;
      double sacc = 0.0;
      int e = s0;
      for (; e + 4 <= s1; e += 4) {
        const int c0 = s_col[e], c1 = s_col[e + 1], c2 = s_col[e + 2], c3 = s_col[e + 3];
        const double v0 = s_val[e], v1 = s_val[e + 1], v2 = s_val[e + 2], v3 = s_val[e + 3];
        const double x0 = xb[(int64_t)c0 * ld], x1 = xb[(int64_t)c1 * ld];
        const double x2 = xb[(int64_t)c2 * ld], x3 = xb[(int64_t)c3 * ld];
        sacc += v0 * x0;
        sacc += v1 * x1;
        sacc += v2 * x2;
        sacc += v3 * x3;
      }
      for (; e < s1; ++e) sacc += s_val[e] * xb[(int64_t)s_col[e] * ld];
      ysum += s_cf[a * kCfStride + bl] * sacc;
    }
    if (own) {
      double an = 0.0;
      xout[ix] = lds_stage<STAGE>(vr, ar, ysum, G.dt, an);
      if (STAGE != 3) G.acc[ix] = an;
    }
  }
}

// Tile of 2*G.tile instances: G.tile lanes (8, 16, 32 or 64) per row, two
// consecutive instances per lane (16-byte gathers, half the memory
// instructions per byte of one-instance lanes).  Each instance's sums are
// formed in the same order as in lds_rows.
template <int STAGE>
__device__ inline void lds_rows_vec2(const GroupDev& G, int64_t k0, int tb, int r0, int nr, const int* s_col,
                                     const double* s_val, const int* s_rp, const int* s_seg, const double* s_cf) {
  const int tid = threadIdx.x;
  const int lpr = G.tile;              // lanes per row, a power of two
  const int lg = tid / lpr, lane = tid % lpr;
  const int ngrp = 256 / lpr;
  const int nt = G.nt;
  const int krow = STAGE == 0 ? 0 : (STAGE == 3 ? 2 : 1);
  const double ph = G.wave[k0 + krow];
  const double* xin = STAGE == 0 ? G.v : (STAGE == 1 ? G.xa : (STAGE == 2 ? G.xb : G.xa));
  double* xout = STAGE == 0 ? G.xa : (STAGE == 1 ? G.xb : (STAGE == 2 ? G.xa : G.v));
  const int ld = G.ld;                 // a multiple of 128
  const int b = tb * 2 * lpr + 2 * lane;   // instances b and b + 1
  (void)ph;
  const double2* xb = reinterpret_cast<const double2*>(xin + b);
  const int ld2 = ld / 2;
  if (b >= G.B) return;   // a lane past the last instance gathers nothing (the tile's padding)
  for (int lr = lg; lr < nr; lr += ngrp) {
    const int ee = s_rp[lr + 1];
    const int64_t ix = (int64_t)(r0 + lr) * ld + b;
    const bool own0 = b < G.B, own1 = b + 1 < G.B;
    const double2 vr = (own0 || own1) ? *reinterpret_cast<const double2*>(G.v + ix) : make_double2(0.0, 0.0);
    const double2 ar = ((own0 || own1) && STAGE != 0) ? *reinterpret_cast<const double2*>(G.acc + ix)
                                                        : make_double2(0.0, 0.0);
    double y0 = 0.0, y1 = 0.0;
    for (int a = 0; a < nt; ++a) {
      const int s0 = s_seg[lr * nt + a];
      const int s1 = (a + 1 < nt) ? s_seg[lr * nt + a + 1] : ee;
      double p0 = 0.0, p1 = 0.0;
      int e = s0;
      for (; e + 4 <= s1; e += 4) {
        const int c0 = s_col[e], c1 = s_col[e + 1], c2 = s_col[e + 2], c3 = s_col[e + 3];
        const double v0 = s_val[e], v1 = s_val[e + 1], v2 = s_val[e + 2], v3 = s_val[e + 3];
        const double2 x0 = xb[(int64_t)c0 * ld2], x1 = xb[(int64_t)c1 * ld2];
        const double2 x2 = xb[(int64_t)c2 * ld2], x3 = xb[(int64_t)c3 * ld2];
        p0 += v0 * x0.x;
        p1 += v0 * x0.y;
        p0 += v1 * x1.x;
        p1 += v1 * x1.y;
        p0 += v2 * x2.x;
        p1 += v2 * x2.y;
        p0 += v3 * x3.x;
        p1 += v3 * x3.y;
      }
      for (; e < s1; ++e) {
        const double v = s_val[e];
        const double2 xx = xb[(int64_t)s_col[e] * ld2];
        p0 += v * xx.x;
        p1 += v * xx.y;
      }
      const double2 cf = *reinterpret_cast<const double2*>(s_cf + a * kCfStride + 2 * lane);
      y0 += cf.x * p0;
      y1 += cf.y * p1;
    }
    double a0 = 0.0, a1 = 0.0;
    const double o0 = lds_stage<STAGE>(vr.x, ar.x, y0, G.dt, a0);
    const double o1 = lds_stage<STAGE>(vr.y, ar.y, y1, G.dt, a1);
    if (own0 && own1) {
      *reinterpret_cast<double2*>(xout + ix) = make_double2(o0, o1);
      if (STAGE != 3) *reinterpret_cast<double2*>(G.acc + ix) = make_double2(a0, a1);
    } else if (own0) {
      xout[ix] = o0;
      if (STAGE != 3) G.acc[ix] = a0;
    }
  }
}

template <int STAGE, int VEC>
__global__ __launch_bounds__(256) void k_batch_stage_lds(const GroupDev* __restrict__ groups,
                                                         const int* __restrict__ gorder, int nactive,
                                                         const int64_t* __restrict__ step) {
  __shared__ int s_col[kLdsCap];
  __shared__ double s_val[kLdsCap];
  __shared__ int s_rp[kLdsRows + 1];
  __shared__ int s_seg[kLdsRows * kMaxBTerms];
  extern __shared__ double s_cf[];                   // c_a(t) of the tile's instances, [nt][kCfStride]
  const int tid = threadIdx.x;
  // Work item = (instance tile, row block) of one group, numbered tile-major.
  // Workgroups are dispatched round-robin over the 8 XCDs (blockIdx % 8); XCD
  // x takes the x-th eighth of every active group's items and walks it in
  // order, so it sweeps the rows of one instance tile: the state rows that
  // neighbouring rows gather (T doubles each) stay in its L2.  The grid is a
  // multiple of 8.  This kernel takes the groups with VEC instances per lane.
  const int x = blockIdx.x & 7;
  const int64_t K = gridDim.x >> 3;
  auto items = [&](const GroupDev& G) -> int64_t {
    return (G.vec == VEC && !G.xlds) ? (int64_t)G.nblk * G.tiles : 0;
  };
  int64_t total = 0;
  for (int q = 0; q < nactive; ++q) {
    const int64_t n = items(groups[gorder[q]]);
    total += n * (x + 1) / 8 - n * x / 8;
  }
  for (int64_t i = blockIdx.x >> 3; i < total; i += K) {
    int gi = 0;
    int64_t j = i, lo = 0;
    for (;;) {
      const int64_t n = items(groups[gorder[gi]]);
      lo = n * x / 8;
      const int64_t cnt = n * (x + 1) / 8 - lo;
      if (j < cnt || gi + 1 == nactive) break;
      j -= cnt;
      ++gi;
    }
    const GroupDev& G = groups[gorder[gi]];
    const int64_t local = lo + j;
    const int tb = (int)(local / G.nblk);
    const int blk = (int)(local % G.nblk);
    const int r0 = G.blk_row[blk], r1 = G.blk_row[blk + 1];
    const int nr = r1 - r0;
    const int e0 = G.rowptr[r0];
    const int ne = G.rowptr[r1] - e0;
    const int nt = G.nt;
    const int64_t k0 = 2 * step[gorder[gi]];
    const int krow = STAGE == 0 ? 0 : (STAGE == 3 ? 2 : 1);
    const double ph = G.wave[k0 + krow];
    const int tw = G.tile * VEC;                      // instances of this tile
    __syncthreads();   // the previous item's LDS contents are no longer read
    for (int i2 = tid; i2 < ne; i2 += 256) {
      s_col[i2] = G.col[e0 + i2];
      s_val[i2] = G.val[e0 + i2];
    }
    for (int i2 = tid; i2 <= nr; i2 += 256) s_rp[i2] = G.rowptr[r0 + i2] - e0;
    for (int i2 = tid; i2 < nr * nt; i2 += 256) s_seg[i2] = G.segptr[(int64_t)r0 * nt + i2] - e0;
    for (int i2 = tid; i2 < nt * tw; i2 += 256) {
      const int a = i2 / tw, bl = i2 % tw;
      const int b = tb * tw + bl;
      s_cf[a * kCfStride + bl] = b < G.B ? G.w[(int64_t)b * nt + a] + G.u[(int64_t)b * nt + a] * ph : 0.0;
    }
    __syncthreads();
    if constexpr (VEC == 2) lds_rows_vec2<STAGE>(G, k0, tb, r0, nr, s_col, s_val, s_rp, s_seg, s_cf);
    else lds_rows<STAGE>(G, k0, tb, r0, nr, s_col, s_val, s_rp, s_seg, s_cf);
  }
}

// Path 3: the state rows a block gathers are staged in LDS too.  Every row
// block carries the sorted list of its distinct columns (at most
// kXLdsBytes / (8 T) of them for a tile of T instances) and each stored
// entry the 16-bit position of its column in that list.  The staged rows are
// loaded with independent, coalesced 16-byte loads before the row walk, so
// the walk's gathers wait only on LDS, and a state row that several rows of
// the block use is read from the memory system once per block.
constexpr int kXLdsBytes = 32768;

int xlds_cap(int tile) { return kXLdsBytes / (8 * tile); }

template <int STAGE>
__device__ inline void xlds_rows(const GroupDev& G, int64_t k0, int tb, int r0, int nr, const unsigned short* s_lx,
                                 const double* s_val, const int* s_rp, const int* s_seg, const double* s_cf,
                                 const double2* s_x) {
  const int tid = threadIdx.x;
  const int lpr = G.tile;              // lanes per row, a power of two
  const int lg = tid / lpr, lane = tid % lpr;
  const int ngrp = 256 / lpr;
  const int nt = G.nt;
  double* xout = STAGE == 0 ? G.xa : (STAGE == 1 ? G.xb : (STAGE == 2 ? G.xa : G.v));
  const int ld = G.ld;
  const int b = tb * 2 * lpr + 2 * lane;   // instances b and b + 1
  (void)k0;
  for (int lr = lg; lr < nr; lr += ngrp) {
    const int ee = s_rp[lr + 1];
    const int64_t ix = (int64_t)(r0 + lr) * ld + b;
    const bool own0 = b < G.B, own1 = b + 1 < G.B;
    const double2 vr = (own0 || own1) ? *reinterpret_cast<const double2*>(G.v + ix) : make_double2(0.0, 0.0);
    const double2 ar = ((own0 || own1) && STAGE != 0) ? *reinterpret_cast<const double2*>(G.acc + ix)
                                                        : make_double2(0.0, 0.0);
    double y0 = 0.0, y1 = 0.0;
    for (int a = 0; a < nt; ++a) {
      const int s0 = s_seg[lr * nt + a];
      const int s1 = (a + 1 < nt) ? s_seg[lr * nt + a + 1] : ee;
      double p0 = 0.0, p1 = 0.0;
      int e = s0;
      for (; e + 4 <= s1; e += 4) {
        const int c0 = s_lx[e], c1 = s_lx[e + 1], c2 = s_lx[e + 2], c3 = s_lx[e + 3];
        const double v0 = s_val[e], v1 = s_val[e + 1], v2 = s_val[e + 2], v3 = s_val[e + 3];
        const double2 x0 = s_x[c0 * lpr + lane], x1 = s_x[c1 * lpr + lane];
        const double2 x2 = s_x[c2 * lpr + lane], x3 = s_x[c3 * lpr + lane];
        p0 += v0 * x0.x;
        p1 += v0 * x0.y;
        p0 += v1 * x1.x;
        p1 += v1 * x1.y;
        p0 += v2 * x2.x;
        p1 += v2 * x2.y;
        p0 += v3 * x3.x;
        p1 += v3 * x3.y;
      }
      for (; e < s1; ++e) {
        const double v = s_val[e];
        const double2 xx = s_x[s_lx[e] * lpr + lane];
        p0 += v * xx.x;
        p1 += v * xx.y;
      }
      const double2 cf = *reinterpret_cast<const double2*>(s_cf + a * kCfStride + 2 * lane);
      y0 += cf.x * p0;
      y1 += cf.y * p1;
    }
    double a0 = 0.0, a1 = 0.0;
    const double o0 = lds_stage<STAGE>(vr.x, ar.x, y0, G.dt, a0);
    const double o1 = lds_stage<STAGE>(vr.y, ar.y, y1, G.dt, a1);
    if (own0 && own1) {
      *reinterpret_cast<double2*>(xout + ix) = make_double2(o0, o1);
      if (STAGE != 3) *reinterpret_cast<double2*>(G.acc + ix) = make_double2(a0, a1);
    } else if (own0) {
      xout[ix] = o0;
      if (STAGE != 3) G.acc[ix] = a0;
    }
  }
}

// cf_len: doubles of the coefficient table at the start of the dynamic LDS
// (the staged state rows follow it).
template <int STAGE>
__global__ __launch_bounds__(256) void k_batch_stage_xlds(const GroupDev* __restrict__ groups,
                                                          const int* __restrict__ gorder, int nactive,
                                                          const int64_t* __restrict__ step, int cf_len) {
  __shared__ unsigned short s_lx[kLdsCap];
  __shared__ double s_val[kLdsCap];
  __shared__ int s_rp[kLdsRows + 1];
  __shared__ int s_seg[kLdsRows * kMaxBTerms];
  extern __shared__ double s_dyn[];
  double* s_cf = s_dyn;                                        // [nt][kCfStride]
  double2* s_x = reinterpret_cast<double2*>(s_dyn + cf_len);   // [distinct columns][tile / 2]
  const int tid = threadIdx.x;
  // Work items and their walk as in k_batch_stage_lds.
  const int x = blockIdx.x & 7;
  const int64_t K = gridDim.x >> 3;
  auto items = [&](const GroupDev& G) -> int64_t { return G.xlds ? (int64_t)G.nblk * G.tiles : 0; };
  int64_t total = 0;
  for (int q = 0; q < nactive; ++q) {
    const int64_t n = items(groups[gorder[q]]);
    total += n * (x + 1) / 8 - n * x / 8;
  }
  for (int64_t i = blockIdx.x >> 3; i < total; i += K) {
    int gi = 0;
    int64_t j = i, lo = 0;
    for (;;) {
      const int64_t n = items(groups[gorder[gi]]);
      lo = n * x / 8;
      const int64_t cnt = n * (x + 1) / 8 - lo;
      if (j < cnt || gi + 1 == nactive) break;
      j -= cnt;
      ++gi;
    }
    const GroupDev& G = groups[gorder[gi]];
    const int64_t local = lo + j;
    const int tb = (int)(local / G.nblk);
    const int blk = (int)(local % G.nblk);
    const int r0 = G.blk_row[blk], r1 = G.blk_row[blk + 1];
    const int nr = r1 - r0;
    const int e0 = G.rowptr[r0];
    const int ne = G.rowptr[r1] - e0;
    const int u0 = G.ucol_ptr[blk];
    const int nu = G.ucol_ptr[blk + 1] - u0;
    const int nt = G.nt;
    const int lpr = G.tile;
    const int tw = 2 * lpr;
    const int64_t k0 = 2 * step[gorder[gi]];
    const int krow = STAGE == 0 ? 0 : (STAGE == 3 ? 2 : 1);
    const double ph = G.wave[k0 + krow];
    const double* xin = STAGE == 0 ? G.v : (STAGE == 1 ? G.xa : (STAGE == 2 ? G.xb : G.xa));
    const double2* xin2 = reinterpret_cast<const double2*>(xin) + tb * lpr;
    const int ld2 = G.ld / 2;
    __syncthreads();   // the previous item's LDS contents are no longer read
    for (int i2 = tid; i2 < nu * lpr; i2 += 256) {
      const int d = i2 / lpr, q = i2 % lpr;
      s_x[i2] = xin2[(int64_t)G.ucol[u0 + d] * ld2 + q];
    }
    for (int i2 = tid; i2 < ne; i2 += 256) {
      s_lx[i2] = G.lidx[e0 + i2];
      s_val[i2] = G.val[e0 + i2];
    }
    for (int i2 = tid; i2 <= nr; i2 += 256) s_rp[i2] = G.rowptr[r0 + i2] - e0;
    for (int i2 = tid; i2 < nr * nt; i2 += 256) s_seg[i2] = G.segptr[(int64_t)r0 * nt + i2] - e0;
    for (int i2 = tid; i2 < nt * tw; i2 += 256) {
      const int a = i2 / tw, bl = i2 % tw;
      const int b = tb * tw + bl;
      s_cf[a * kCfStride + bl] = b < G.B ? G.w[(int64_t)b * nt + a] + G.u[(int64_t)b * nt + a] * ph : 0.0;
    }
    __syncthreads();
    xlds_rows<STAGE>(G, k0, tb, r0, nr, s_lx, s_val, s_rp, s_seg, s_cf, s_x);
  }
}

// Path 5: one wavefront per (row, instance tile), every group in one tile
// of 64 lanes with VEC consecutive instances per lane (VEC = 2: up to 128
// instances, so each group's matrix row is read once per stage).  The row's
// pointers, columns and values are uniform across the wavefront and are read
// through the scalar cache (constant address space), so each entry costs one
// 16-byte gather per lane and no vector work to broadcast it.  Ordering:
// the grid is the number of wavefronts the device keeps resident, each XCD
// (blockIdx % 8) takes one contiguous eighth of every group's rows, and its
// wavefronts walk that eighth interleaved (wavefront w takes rows w, w + W,
// ...), so the rows in flight on an XCD form a narrow moving window and the
// state rows they gather (neighbouring pairs, a few hundred rows apart) are
// still in that XCD's L2 when the next rows use them.  Each term's entries
// are summed in row order and combined exactly as in the other paths, so the
// results are bitwise the same.  The column and value arrays carry
// kRowPad padding entries: a round of kRowChunk scalar loads may read past
// the last row.
typedef const __attribute__((address_space(4))) int scalar_int;
typedef const __attribute__((address_space(4))) double scalar_dbl;
// global (not generic) pointers: generic loads also count against the
// counter the scalar loads wait on, which would serialise the gathers
typedef double dv2 __attribute__((ext_vector_type(2)));
typedef const __attribute__((address_space(1))) double gconst_dbl;
typedef const __attribute__((address_space(1))) dv2 gconst_dbl2;
typedef __attribute__((address_space(1))) double gdbl;
typedef __attribute__((address_space(1))) dv2 gdbl2;

constexpr int kRowChunk = 8;
constexpr int kRowPad = 16;

template <int STAGE, int VEC>
__global__ __launch_bounds__(64) void k_batch_rows(const GroupDev* __restrict__ groups,
                                                   const int* __restrict__ gorder, int nactive,
                                                   const int64_t* __restrict__ step) {
  extern __shared__ double s_cf[];   // [nt][64 * VEC]: this wavefront's tile coefficients, lane-private
  const int lane = threadIdx.x;
  const int x = blockIdx.x & 7;
  const int64_t W = gridDim.x >> 3;
  const int64_t w = blockIdx.x >> 3;
  constexpr int TW = 64 * VEC;
  for (int q = 0; q < nactive; ++q) {
    const int g = gorder[q];
    const GroupDev& G = groups[g];
    if (!G.p5 || G.vec != VEC) continue;
    const int64_t lo = (int64_t)G.M * x / 8;
    const int64_t n = (int64_t)G.M * (x + 1) / 8 - lo;
    const int nt = G.nt, ld = G.ld, B = G.B;
    const int64_t k0 = 2 * step[g];
    const int krow = STAGE == 0 ? 0 : (STAGE == 3 ? 2 : 1);
    const double ph = G.wave[k0 + krow];
    gconst_dbl* xin = (gconst_dbl*)(STAGE == 0 ? G.v : (STAGE == 1 ? G.xa : (STAGE == 2 ? G.xb : G.xa)));
    gdbl* xout = (gdbl*)(STAGE == 0 ? G.xa : (STAGE == 1 ? G.xb : (STAGE == 2 ? G.xa : G.v)));
    gconst_dbl* gv = (gconst_dbl*)G.v;
    gdbl* gacc = (gdbl*)G.acc;
    scalar_int* rp = (scalar_int*)G.rowptr;
    scalar_int* sp = (scalar_int*)G.segptr;
    scalar_int* col = (scalar_int*)G.col;
    scalar_dbl* val = (scalar_dbl*)G.val;
    int cur = -1;
    for (int64_t i = w; i < n * G.tiles; i += W) {
      const int tb = (int)(i / n);
      const int64_t r = lo + i % n;
      if (tb != cur) {
        for (int a = 0; a < nt; ++a)
#pragma unroll
          for (int j = 0; j < VEC; ++j) {
            const int b = tb * TW + VEC * lane + j;
            s_cf[a * TW + VEC * lane + j] = b < B ? G.w[(int64_t)b * nt + a] + G.u[(int64_t)b * nt + a] * ph : 0.0;
          }
        cur = tb;
      }
      const int b0 = tb * TW + VEC * lane;
      const int64_t ix = r * ld + b0;
      const bool own = b0 < B;
      double vr[VEC], ar[VEC], sum[VEC], y[VEC];
      if constexpr (VEC == 2) {
        const dv2 t = own ? *(gconst_dbl2*)(gv + ix) : dv2{0.0, 0.0};
        const dv2 u = (own && STAGE != 0) ? *(gconst_dbl2*)(gacc + ix) : dv2{0.0, 0.0};
        vr[0] = t.x; vr[1] = t.y; ar[0] = u.x; ar[1] = u.y;
      } else {
        vr[0] = own ? gv[ix] : 0.0;
        ar[0] = (own && STAGE != 0) ? gacc[ix] : 0.0;
      }
#pragma unroll
      for (int j = 0; j < VEC; ++j) { sum[j] = 0.0; y[j] = 0.0; }
      const int e0 = rp[r], e1 = rp[r + 1];
      int a = 0;
      int bnd = nt > 1 ? sp[r * nt + 1] : e1;   // end of segment a
      gconst_dbl* xb = xin + b0;
      for (int e = e0; e < e1; e += kRowChunk) {
        int c[kRowChunk];
        double v[kRowChunk];
#pragma unroll
        for (int k = 0; k < kRowChunk; ++k) {
          c[k] = col[e + k];
          v[k] = val[e + k];
        }
        double xv[kRowChunk][VEC];
#pragma unroll
        for (int k = 0; k < kRowChunk; ++k) {
          if (e + k < e1) {
            // lanes past the group's last instance issue no gather
            if constexpr (VEC == 2) {
              const dv2 t = own ? *(gconst_dbl2*)(xb + (int64_t)c[k] * ld) : dv2{0.0, 0.0};
              xv[k][0] = t.x;
              xv[k][1] = t.y;
            } else {
              xv[k][0] = own ? xb[(int64_t)c[k] * ld] : 0.0;
            }
          }
        }
#pragma unroll
        for (int k = 0; k < kRowChunk; ++k) {
          if (e + k < e1) {
            while (e + k >= bnd) {   // close segment a (and any empty ones after it)
              const double* cf = s_cf + a * TW + VEC * lane;
#pragma unroll
              for (int j = 0; j < VEC; ++j) {
                y[j] += cf[j] * sum[j];
                sum[j] = 0.0;
              }
              ++a;
              bnd = a + 1 < nt ? sp[r * nt + a + 1] : e1;
            }
#pragma unroll
            for (int j = 0; j < VEC; ++j) sum[j] += v[k] * xv[k][j];
          }
        }
      }
      for (; a < nt; ++a) {
        const double* cf = s_cf + a * TW + VEC * lane;
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
          y[j] += cf[j] * sum[j];
          sum[j] = 0.0;
        }
      }
      double o[VEC], an[VEC];
#pragma unroll
      for (int j = 0; j < VEC; ++j) o[j] = lds_stage<STAGE>(vr[j], ar[j], y[j], G.dt, an[j]);
      if constexpr (VEC == 2) {
        if (own && b0 + 1 < B) {
          *(gdbl2*)(xout + ix) = dv2{o[0], o[1]};
          if (STAGE != 3) *(gdbl2*)(gacc + ix) = dv2{an[0], an[1]};
        } else if (own) {
          xout[ix] = o[0];
          if (STAGE != 3) gacc[ix] = an[0];
        }
      } else if (own) {
        xout[ix] = o[0];
        if (STAGE != 3) gacc[ix] = an[0];
      }
    }
  }
}

// Path 7: persistent, software-pipelined staging.  The grid holds two
// workgroups of 512 threads per CU, each walking its own list of items
// (tile of 64 instances, block of rows).  A block is a set of rows taken
// along a walk of the (j, k) pair grid in 4 x 4 tiles (S_p and J_p
// together, the diagonal generators last), so that its rows gather a
// compact neighbourhood of state rows: at most kP7Slots - 1 distinct
// columns, staged in LDS as 64-instance slices of 512 bytes, beside the
// block's matrix data (row list, segment ends, 16-bit slot indices, values;
// at most kP7Blob bytes) and the tile's term coefficients.  While the rows
// of one item are summed from LDS, the loads of the next item's staged data
// are in flight into registers -- the same number of 16-byte loads from
// every thread for every item, at out-of-range buffer offsets (zeros, no
// traffic) where a block or a tile needs fewer, so that every wait the
// compiler places is a fixed count -- together with the column list of the
// item after it; at the end of the item the registers are written to LDS.
// Each state row a block gathers is read from the memory system once per
// block instead of once per stored entry.  Rows with more distinct columns
// than slots are summed straight from global memory, one wavefront per row
// and tile, by a few workgroups per XCD that take no blocks.  Every row adds
// its terms in entry order exactly like the other paths, so the results
// are bitwise the same.
constexpr int kP7Threads = 512;                 // 256 (four per CU, 16-row blocks): 1.23 against 1.04 ms per step
constexpr int kP7Waves = kP7Threads / 64;
constexpr int kP7Half = kP7Threads / 32;        // half-wavefronts: each stages one slot per load
constexpr int kP7Slots = 8 * kP7Half;           // eight 16-byte loads per thread
constexpr int kP7Rows = 4 * kP7Waves;           // four passes of one row per wavefront
constexpr int kP7Blob = 16 * kP7Threads;        // one 16-byte blob load per thread
constexpr int kP7Tile = 64;
constexpr int kP7SegOff = 4 * kP7Rows;   // bytes: int32 rows[kP7Rows], then u16 segment ends [kP7Rows][nt]
constexpr int kP7CfPer = (kMaxBTerms + kP7Waves - 1) / kP7Waves;   // coefficients staged per thread
static_assert(kP7CfPer == 1 || kP7CfPer == 2, "one or two coefficients per thread");

// Each (row, term) segment of a block is padded to an even number of
// entries, and each row's last segment to a multiple of kP7Round entries,
// with entries (kP7Zero, 0.0): slot kP7Zero is never loaded and holds
// zeros, and adding 0 * 0 to a running sum changes no bit of it (the sum
// starts at +0 and round-to-nearest never produces -0 from it), so the row
// walk reads whole rounds of pairs (one 4-byte read of two slot indices,
// one 16-byte read of two values) with the results bitwise unchanged.
constexpr int kP7Round = 8;
static_assert(kP7Round % 2 == 0, "rounds of whole pairs");
constexpr int kP7Zero = kP7Slots - 1;
static_assert(kP7Zero == 7 * kP7Half + kP7Half - 1, "the zero slot is load 7 of the last half-wavefront");
__host__ __device__ inline int p7_lidx_off(int nt) { return kP7SegOff + 2 * kP7Rows * nt; }
__host__ __device__ inline int p7_val_off(int nt, int ne) { return (p7_lidx_off(nt) + 2 * ne + 15) & ~15; }

// The path-7 groups of one launch, in launch order (kernel argument, so the
// item walk runs on scalar registers only).
constexpr int kP7MaxGroups = 16;
constexpr int kP7LongWgs = 32 / kP7Waves;   // workgroups per XCD for the long rows, when there are any
struct P7Plan {
  int ng;
  int klong;              // workgroups per XCD given to the long rows (0: none)
  int g[kP7MaxGroups];
  int nblk[kP7MaxGroups];
  int tiles[kP7MaxGroups];
};

struct P7Loc {
  int g, tb, blk;
};

// Item i of XCD x's share: each group of the plan contributes the x-th
// eighth of its (tile, block) items, numbered tile-major.
__device__ inline bool p7_locate(const P7Plan& plan, int x, int64_t i, P7Loc& L) {
  for (int q = 0; q < plan.ng; ++q) {
    const int64_t n = (int64_t)plan.nblk[q] * plan.tiles[q];
    const int64_t lo = n * x / 8, cnt = n * (x + 1) / 8 - lo;
    if (i < cnt) {
      const int64_t local = lo + i;
      L.g = plan.g[q];
      L.tb = (int)(local / plan.nblk[q]);
      L.blk = (int)(local % plan.nblk[q]);
      return true;
    }
    i -= cnt;
  }
  return false;
}

template <int STAGE>
__device__ inline const double* stage_in(const GroupDev& G) {
  return STAGE == 0 ? G.v : (STAGE == 1 ? G.xa : (STAGE == 2 ? G.xb : G.xa));
}
template <int STAGE>
__device__ inline double* stage_out(const GroupDev& G) {
  return STAGE == 0 ? G.xa : (STAGE == 1 ? G.xb : (STAGE == 2 ? G.xa : G.v));
}

// Every global access of the pipelined kernel goes through global-address-
// space pointers: generic (flat) accesses would also count against the
// counter that LDS reads wait on, so every LDS wait of the row walk would
// wait for the staging loads in flight as well.
typedef unsigned uv4 __attribute__((ext_vector_type(4)));
typedef int iv4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(1))) uv4 g_uv4;
typedef const __attribute__((address_space(1))) iv4 g_iv4;
typedef const __attribute__((address_space(1))) int g_int;

// Buffer resource over `bytes` bytes at p: raw addressing (stride 0, so
// the range check compares the byte offset with `bytes`), and in the last
// descriptor word the 32-bit data format that untyped dword loads use on
// CDNA.  A load at a byte offset past the end returns zeros and touches no
// memory, which is how the lanes of a tile past its group's last instance
// (and unused slots) skip their loads without a branch, so every wait count
// stays fixed.
constexpr int kP7Off = 0x7ffffff0;   // out-of-range offset
constexpr int kRawDwordFormat = 0x00020000;
__device__ inline __amdgpu_buffer_rsrc_t p7_rsrc(const void* p, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, kRawDwordFormat);
}
__device__ inline double p7_load_d(__amdgpu_buffer_rsrc_t r, int off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
// The value of x, opaque to the optimizer: keeps a per-lane choice of
// offset a plain select instead of letting it split the load that uses it
// into two branches (which would cost a branch and a full wait per load).
__device__ inline int opaque(int x) {
  asm volatile("" : "+v"(x));
  return x;
}
__device__ inline double readlane_d(double v, int l) {
  const long long bits = __builtin_bit_cast(long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)bits, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(bits >> 32), l);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

template <int STAGE>
__global__ __launch_bounds__(kP7Threads, 4) void k_batch_pipe(const GroupDev* __restrict__ groups, P7Plan plan,
                                                              const int64_t* __restrict__ step) {
  __shared__ uv4 s_x[kP7Slots * 32];                // slot s: 64 instances of state row ucol[s]
  __shared__ uv4 s_blob[kP7Blob / 16];
  __shared__ double s_cf[kMaxBTerms * kP7Tile];     // c_a(t) of the tile's instances, [a][instance]
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int hw = tid >> 5, l32 = tid & 31;          // staging: half-wavefront hw loads slots hw + kP7Half k
  const int x = blockIdx.x & 7;
  // The last plan.klong workgroups of every XCD take the long rows; the
  // others share the blocks.
  const int64_t K = (gridDim.x >> 3) - plan.klong;
  const int64_t kk = blockIdx.x >> 3;
  const int krow = STAGE == 0 ? 0 : (STAGE == 3 ? 2 : 1);

  uv4 px0, px1, px2, px3, px4, px5, px6, px7, pb;   // named, so they stay in registers
  double pw, pu, pw2 = 0.0, pu2 = 0.0;               // coefficient a = wv (and wv + kP7Waves)
  iv4 cu0, cu1;
  auto issue_cols = [&](const P7Loc& L) {
    g_iv4* q = (g_iv4*)(groups[L.g].p7_ucol + (int64_t)L.blk * kP7Slots + hw * 8);
    cu0 = q[0];
    cu1 = q[1];
  };
  auto issue_stage = [&](const P7Loc& L) {
    const GroupDev& G = groups[L.g];
    const __amdgpu_buffer_rsrc_t rx = p7_rsrc(stage_in<STAGE>(G), (int64_t)(G.M + 1) * G.ld * 8);
    const int inst = L.tb * kP7Tile + 2 * l32;      // this lane's two instances
    const int rowb = G.ld * 8;                      // bytes per state row
    const bool live = inst < G.B;
    const int o = inst * 8;
    // unused slots and the zero slot carry column -1: loaded as zeros, no traffic
#define P7_SLOT(c) __builtin_amdgcn_raw_buffer_load_b128(rx, opaque(live && (c) >= 0 ? (c) * rowb + o : kP7Off), 0, 0)
    px0 = P7_SLOT(cu0.x);
    px1 = P7_SLOT(cu0.y);
    px2 = P7_SLOT(cu0.z);
    px3 = P7_SLOT(cu0.w);
    px4 = P7_SLOT(cu1.x);
    px5 = P7_SLOT(cu1.y);
    px6 = P7_SLOT(cu1.z);
    px7 = P7_SLOT(cu1.w);
#undef P7_SLOT
    // block metadata through the scalar cache (uniform, read-only)
    scalar_int* pm = (scalar_int*)G.p7_meta + 4 * (int64_t)L.blk;
    const int m0 = pm[0], m1 = pm[1];
    pb = ((g_uv4*)G.p7_blob)[m0 + (tid < m1 ? tid : 0)];
    const int a = wv, b = L.tb * kP7Tile + lane;
    const int idx = (a < G.nt && b < G.B) ? b * G.nt + a : 0;
    pw = ((gconst_dbl*)G.w)[idx];
    pu = ((gconst_dbl*)G.u)[idx];
    if constexpr (kP7CfPer == 2) {
      const int a2 = wv + kP7Waves;
      const int idx2 = (a2 < G.nt && b < G.B) ? b * G.nt + a2 : 0;
      pw2 = ((gconst_dbl*)G.w)[idx2];
      pu2 = ((gconst_dbl*)G.u)[idx2];
    }
  };
  auto write_stage = [&](const P7Loc& L) {
    constexpr int SK = kP7Half * 32;   // uv4 units between slot hw + kP7Half k and the next k
    uv4* sx = s_x + hw * 32 + l32;     // slot hw + kP7Half k
    sx[0 * SK] = px0;
    sx[1 * SK] = px1;
    sx[2 * SK] = px2;
    sx[3 * SK] = px3;
    sx[4 * SK] = px4;
    sx[5 * SK] = px5;
    sx[6 * SK] = px6;
    sx[7 * SK] = hw == kP7Half - 1 ? uv4{0u, 0u, 0u, 0u} : px7;   // slot kP7Zero holds zeros
    s_blob[tid] = pb;
    const GroupDev& G = groups[L.g];
    const double ph = G.wave[2 * step[L.g] + krow];   // uniform: a scalar load
    const int a = wv, b = L.tb * kP7Tile + lane;
    if (a < G.nt) s_cf[a * kP7Tile + lane] = b < G.B ? pw + pu * ph : 0.0;
    if constexpr (kP7CfPer == 2)
      if (a + kP7Waves < G.nt) s_cf[(a + kP7Waves) * kP7Tile + lane] = b < G.B ? pw2 + pu2 * ph : 0.0;
  };

  // Rows with more distinct columns than slots: one wavefront per (row,
  // tile), straight from global memory.  Each lane holds one of 64
  // consecutive entries of the row (column and value), and the wavefront
  // gathers 32 entries' state at a time before adding them in entry
  // order, so the chain of dependent loads is one round trip per 32
  // entries.  They go to workgroups of their own (a few per XCD, with no
  // blocks), so that their latency overlaps the pipelines of the others
  // instead of delaying them; the tile's term coefficients go to this
  // wavefront's own area of the staging buffer, which these workgroups do
  // not otherwise use.
  if (kk >= K) {
  double* s_cw = reinterpret_cast<double*>(s_x) + wv * (kMaxBTerms * kP7Tile);
  const int64_t wid = (((kk - K) * 8 + x) * (kP7Threads / 64)) + wv;
  const int64_t nw = (int64_t)plan.klong * 8 * (kP7Threads / 64);
  for (int q = 0; q < plan.ng; ++q) {
    const int g = plan.g[q];
    const GroupDev& G = groups[g];
    if (G.p7_nlong == 0) continue;
    const int nt = G.nt, ld = G.ld;
    const double ph = G.wave[2 * step[g] + krow];
    gconst_dbl* xin = (gconst_dbl*)stage_in<STAGE>(G);
    gdbl* xout = (gdbl*)stage_out<STAGE>(G);
    gconst_dbl* gv = (gconst_dbl*)G.v;
    gdbl* gacc = (gdbl*)G.acc;
    gconst_dbl* gval = (gconst_dbl*)G.val;
    g_int* gcol = (g_int*)G.col;
    for (int64_t it = wid; it < (int64_t)G.p7_nlong * G.tiles; it += nw) {
      const int r = G.p7_long[it / G.tiles];
      const int tb = (int)(it % G.tiles);
      const int b = tb * kP7Tile + lane;         // lanes past the last instance read padding, store nothing
      const bool own = b < G.B;
      for (int a = 0; a < nt; ++a)
        s_cw[a * kP7Tile + lane] = own ? G.w[(int64_t)b * nt + a] + G.u[(int64_t)b * nt + a] * ph : 0.0;
      const int64_t ix = (int64_t)r * ld + b;
      const double vr = gv[ix];
      const double ar = STAGE != 0 ? ((gconst_dbl*)gacc)[ix] : 0.0;
      const int e0 = G.rowptr[r], e_end = G.rowptr[r + 1];
      int a = 0;
      int s1 = nt > 1 ? G.segptr[(int64_t)r * nt + 1] : e_end;   // end of term a
      double ysum = 0.0, sacc = 0.0;
      for (int cb = e0; cb < e_end; cb += 64) {
        const int n = min(64, e_end - cb);
        const int mc = gcol[cb + (lane < n ? lane : 0)];
        const double mv = gval[cb + (lane < n ? lane : 0)];
        for (int k = 0; k < n; k += 32) {
          double xs[32];
#pragma unroll
          for (int j = 0; j < 32; ++j)
            xs[j] = xin[(int64_t)__builtin_amdgcn_readlane(mc, min(k + j, n - 1)) * ld + b];
#pragma unroll
          for (int j = 0; j < 32; ++j) {
            if (k + j < n) {
              const int e = cb + k + j;
              while (e == s1) {                    // term a ends before entry e
                ysum += s_cw[a * kP7Tile + lane] * sacc;
                sacc = 0.0;
                ++a;
                s1 = (a + 1 < nt) ? G.segptr[(int64_t)r * nt + a + 1] : e_end;
              }
              sacc += readlane_d(mv, k + j) * xs[j];
            }
          }
        }
      }
      for (; a < nt; ++a) {                          // the last term, and empty terms after it
        ysum += s_cw[a * kP7Tile + lane] * sacc;
        sacc = 0.0;
      }
      if (own) {
        double an = 0.0;
        xout[ix] = lds_stage<STAGE>(vr, ar, ysum, G.dt, an);
        if (STAGE != 3) gacc[ix] = an;
      }
    }
  }
  return;
  }

  P7Loc cur, nxt, nn;
  int64_t i = kk;
  if (p7_locate(plan, x, i, cur)) {
    issue_cols(cur);
    issue_stage(cur);
    write_stage(cur);
    bool has_nxt = p7_locate(plan, x, i + K, nxt);
    issue_cols(has_nxt ? nxt : cur);
    i += 2 * K;
    __syncthreads();
    for (;;) {
      // LDS holds item `cur`; cu0/cu1 hold (or are loading) the columns of `nxt`
      const GroupDev& G = groups[cur.g];
      scalar_int* pm = (scalar_int*)G.p7_meta + 4 * (int64_t)cur.blk;
      const int nr = pm[2], ne = pm[3], nt = G.nt, ld = G.ld;
      const int* s_rows = reinterpret_cast<const int*>(s_blob);
      const unsigned short* s_seg = reinterpret_cast<const unsigned short*>(
          reinterpret_cast<const char*>(s_blob) + kP7SegOff);
      const unsigned short* s_lx = reinterpret_cast<const unsigned short*>(
          reinterpret_cast<const char*>(s_blob) + p7_lidx_off(nt));
      const double* s_val = reinterpret_cast<const double*>(reinterpret_cast<const char*>(s_blob) +
                                                            p7_val_off(nt, ne));
      const double* sx = reinterpret_cast<const double*>(s_x);
      const int b = cur.tb * kP7Tile + lane;
      const bool own = b < G.B;
      gdbl* gacc = (gdbl*)G.acc;
      gdbl* xout = (gdbl*)stage_out<STAGE>(G);
      // this item's own state entries (rows past the block's last are padded
      // with its first row; the row is the same for the whole wavefront)
      const __amdgpu_buffer_rsrc_t rv = p7_rsrc(G.v, (int64_t)(G.M + 1) * ld * 8);
      const __amdgpu_buffer_rsrc_t ra = p7_rsrc(G.acc, (int64_t)G.M * ld * 8);
      double vr[4], ar[4];
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const int row = __builtin_amdgcn_readfirstlane(s_rows[p * kP7Waves + wv]);
        const int off = opaque(own ? (row * ld + b) * 8 : kP7Off);
        vr[p] = p7_load_d(rv, off);
        ar[p] = STAGE != 0 ? p7_load_d(ra, off) : 0.0;
      }
      // the next item's staged data, and the columns of the one after it
      const bool has_nn = p7_locate(plan, x, i, nn);
      issue_stage(has_nxt ? nxt : cur);
      issue_cols(has_nn ? nn : cur);
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const int lr = p * kP7Waves + wv;
        if (lr < nr && own) {
          // one walk over the row in rounds of kP7Round entries across its
          // terms; term a is closed (ysum += c_a * sum) after the pair that
          // ends it, empty terms where they stand, the last term at the end
          const int rs = lr > 0 ? s_seg[lr * nt - 1] : 0;
          const int re = s_seg[lr * nt + nt - 1];
          const unsigned* l2 = reinterpret_cast<const unsigned*>(s_lx);   // two slot indices per word
          const double2* v2 = reinterpret_cast<const double2*>(s_val);
          double ysum = 0.0, sacc = 0.0;
          int a = 0, s1 = s_seg[lr * nt];
          while (a < nt - 1 && s1 == rs) {
            ysum += s_cf[a * kP7Tile + lane] * sacc;
            sacc = 0.0;
            s1 = s_seg[lr * nt + ++a];
          }
          for (int e = rs; e < re; e += kP7Round) {
            unsigned l[kP7Round / 2];
            double2 v[kP7Round / 2];
            double xv[kP7Round];
#pragma unroll
            for (int q = 0; q < kP7Round / 2; ++q) {
              l[q] = l2[(e >> 1) + q];
              v[q] = v2[(e >> 1) + q];
            }
#pragma unroll
            for (int q = 0; q < kP7Round / 2; ++q) {
              xv[2 * q] = sx[(l[q] & 0xffff) * kP7Tile + lane];
              xv[2 * q + 1] = sx[(l[q] >> 16) * kP7Tile + lane];
            }
#pragma unroll
            for (int q = 0; q < kP7Round / 2; ++q) {
              sacc += v[q].x * xv[2 * q];
              sacc += v[q].y * xv[2 * q + 1];
              while (a < nt - 1 && e + 2 * q + 2 == s1) {
                ysum += s_cf[a * kP7Tile + lane] * sacc;
                sacc = 0.0;
                s1 = s_seg[lr * nt + ++a];
              }
            }
          }
          for (; a < nt; ++a) {
            ysum += s_cf[a * kP7Tile + lane] * sacc;
            sacc = 0.0;
          }
          const int64_t ix = (int64_t)__builtin_amdgcn_readfirstlane(s_rows[lr]) * ld + b;
          double an = 0.0;
          xout[ix] = lds_stage<STAGE>(vr[p], ar[p], ysum, G.dt, an);
          if (STAGE != 3) gacc[ix] = an;
        }
      }
      if (!has_nxt) break;
      __syncthreads();   // every wavefront is done with this item's LDS
      write_stage(nxt);
      __syncthreads();
      cur = nxt;
      nxt = nn;
      has_nxt = has_nn;
      i += K;
    }
  }
}

// Row blocks for path 3: at most max_rows rows, kLdsCap entries and ucap
// distinct columns; with each block's sorted distinct columns and every
// entry's position in them.  False if a single row does not fit.
struct XPart {
  std::vector<int> blk, uptr, ucol;
  std::vector<unsigned short> lidx;
};

bool xlds_partition(const std::vector<int>& rp, const std::vector<int>& col, int max_rows, int ucap, XPart& out) {
  const int M = (int)rp.size() - 1;
  const int ncol = M + 1;                  // the free-vector column M included
  // mark[c]: last block that holds column c; seen[c]: last candidate row
  // examination that counted c (a row examined and left for the next block
  // is examined again, under a new stamp)
  std::vector<int> mark(ncol, -1), seen(ncol, -1);
  out.blk.assign(1, 0);
  int r0 = 0, nb = 0, stamp = 0;
  while (r0 < M) {
    int r1 = r0, used = 0;
    while (r1 < M && r1 - r0 < max_rows && rp[r1 + 1] - rp[r0] <= kLdsCap) {
      int fresh = 0;
      ++stamp;
      for (int e = rp[r1]; e < rp[r1 + 1]; ++e) {
        const int c = col[e];
        if (mark[c] != nb && seen[c] != stamp) { seen[c] = stamp; ++fresh; }
      }
      if (used + fresh > ucap) break;
      for (int e = rp[r1]; e < rp[r1 + 1]; ++e) mark[col[e]] = nb;
      used += fresh;
      ++r1;
    }
    if (r1 == r0) return false;              // the row alone exceeds a limit
    out.blk.push_back(r1);
    r0 = r1;
    ++nb;
  }
  out.uptr.assign(1, 0);
  out.ucol.clear();
  out.lidx.assign(rp[M], 0);
  std::vector<int> u;
  for (int b = 0; b < nb; ++b) {
    const int e0 = rp[out.blk[b]], e1 = rp[out.blk[b + 1]];
    u.assign(col.begin() + e0, col.begin() + e1);
    std::sort(u.begin(), u.end());
    u.erase(std::unique(u.begin(), u.end()), u.end());
    // the kernel's LDS tables hold exactly these limits
    SUN_REQUIRE(e1 - e0 <= kLdsCap && (int)u.size() <= ucap && out.blk[b + 1] - out.blk[b] <= kLdsRows,
                SUN_ENOTSUP, "internal: row block exceeds its LDS limits");
    for (int e = e0; e < e1; ++e)
      out.lidx[e] = (unsigned short)(std::lower_bound(u.begin(), u.end(), col[e]) - u.begin());
    out.ucol.insert(out.ucol.end(), u.begin(), u.end());
    out.uptr.push_back((int)out.ucol.size());
  }
  return true;
}

// Path 7 blocks.  Rows are taken along the pair grid in 4 x 4 tiles of
// (j, k) (stored rows 2p and 2p + 1 of pair p = (j, k), j < k), then the
// diagonal generators in order; consecutive rows join a block while it
// keeps at most max_rows rows, kP7Slots distinct columns and kP7Blob bytes
// of matrix data.  A row that alone exceeds a limit goes to the long list.
struct P7Part {
  std::vector<int> meta;        // 4 ints per block
  std::vector<int> ucol;        // kP7Slots per block, slot s at (s % kP7Half) * 8 + s / kP7Half
  std::vector<uint4> blob;
  std::vector<int> longrows;
};

void p7_partition(int N, int64_t M, int nt, const std::vector<int>& rp, const std::vector<int>& seg,
                  const std::vector<int>& col, const std::vector<double>& val, int max_rows, P7Part& out) {
  const int64_t P = (int64_t)N * (N - 1) / 2;
  std::vector<int> seq;
  seq.reserve(M);
  constexpr int T = 4;
  for (int tj = 0; tj < N; tj += T)
    for (int tk = tj; tk < N; tk += T)
      for (int j = tj; j < std::min(tj + T, N); ++j)
        for (int k = std::max(tk, j + 1); k < std::min(tk + T, N); ++k) {
          const int64_t p = (int64_t)j * (2 * N - j - 1) / 2 + k - j - 1;
          seq.push_back((int)(2 * p));
          seq.push_back((int)(2 * p + 1));
        }
  for (int64_t r = 2 * P; r < M; ++r) seq.push_back((int)r);
  SUN_REQUIRE((int64_t)seq.size() == M, SUN_EDEVICE, "internal: path 7 row walk does not cover the rows");
  // ne counts padded entries: a row of term lengths n_a takes sum ceil2(n_a), rounded up to kP7Round
  auto fits = [&](int rows, int used, int ne) {
    return rows <= max_rows && used <= kP7Slots - 1 && p7_val_off(nt, ne) + 8 * ne <= kP7Blob;
  };
  auto padded_len = [&](int r) {
    int n = 0;
    for (int a = 0; a < nt; ++a) {
      const int s1 = a + 1 < nt ? seg[(int64_t)r * nt + a + 1] : rp[r + 1];
      n += (s1 - seg[(int64_t)r * nt + a] + 1) & ~1;
    }
    return (n + kP7Round - 1) / kP7Round * kP7Round;
  };
  std::vector<int> mark(M + 1, -1), seen(M + 1, -1);
  std::vector<std::vector<int>> blocks;
  std::vector<int> cur;
  int used = 0, ne = 0, stamp = 0, nb = 0;
  auto fresh_of = [&](int r) {
    int fresh = 0;
    ++stamp;
    for (int e = rp[r]; e < rp[r + 1]; ++e) {
      const int c = col[e];
      if (mark[c] != nb && seen[c] != stamp) { seen[c] = stamp; ++fresh; }
    }
    return fresh;
  };
  auto close = [&] {
    if (!cur.empty()) { blocks.push_back(cur); ++nb; }
    cur.clear();
    used = 0;
    ne = 0;
  };
  for (int r : seq) {
    const int len = padded_len(r);
    int fresh = fresh_of(r);
    if (!fits((int)cur.size() + 1, used + fresh, ne + len)) {
      close();
      fresh = fresh_of(r);
      if (!fits(1, fresh, len)) {           // the row alone exceeds a block
        out.longrows.push_back(r);
        continue;
      }
    }
    for (int e = rp[r]; e < rp[r + 1]; ++e) mark[col[e]] = nb;
    cur.push_back(r);
    used += fresh;
    ne += len;
  }
  close();
  out.meta.clear();
  out.ucol.assign(blocks.size() * kP7Slots, 0);
  out.blob.clear();
  std::vector<int> u;
  std::vector<unsigned char> bytes;
  for (size_t bi = 0; bi < blocks.size(); ++bi) {
    const std::vector<int>& rows = blocks[bi];
    u.clear();
    int nent = 0;
    for (int r : rows) {
      u.insert(u.end(), col.begin() + rp[r], col.begin() + rp[r + 1]);
      nent += padded_len(r);
    }
    std::sort(u.begin(), u.end());
    u.erase(std::unique(u.begin(), u.end()), u.end());
    SUN_REQUIRE((int)u.size() <= kP7Slots - 1 && (int)rows.size() <= kP7Rows &&
                    p7_val_off(nt, nent) + 8 * nent <= kP7Blob,
                SUN_EDEVICE, "internal: path 7 block exceeds its limits");
    for (int s = 0; s < kP7Slots; ++s)   // unused slots and the zero slot: -1
      out.ucol[bi * kP7Slots + (s % kP7Half) * 8 + s / kP7Half] = s < (int)u.size() ? u[s] : -1;
    const int nbytes = p7_val_off(nt, nent) + 8 * nent;
    const int n16 = (nbytes + 15) / 16;
    bytes.assign((size_t)n16 * 16, 0);
    int* brow = reinterpret_cast<int*>(bytes.data());
    unsigned short* bseg = reinterpret_cast<unsigned short*>(bytes.data() + kP7SegOff);
    unsigned short* blx = reinterpret_cast<unsigned short*>(bytes.data() + p7_lidx_off(nt));
    double* bval = reinterpret_cast<double*>(bytes.data() + p7_val_off(nt, nent));
    int w = 0;
    for (int lr = 0; lr < kP7Rows; ++lr) brow[lr] = rows[lr < (int)rows.size() ? lr : 0];
    for (int lr = 0; lr < (int)rows.size(); ++lr) {
      const int r = rows[lr];
      for (int a = 0; a < nt; ++a) {
        const int s1 = a + 1 < nt ? seg[(int64_t)r * nt + a + 1] : rp[r + 1];
        for (int e = seg[(int64_t)r * nt + a]; e < s1; ++e) {
          blx[w] = (unsigned short)(std::lower_bound(u.begin(), u.end(), col[e]) - u.begin());
          bval[w] = val[e];
          ++w;
        }
        // pad the segment to a multiple of two, the row's last one to a multiple of kP7Round
        for (; (w & 1) || (a == nt - 1 && w % kP7Round); ++w) {
          blx[w] = (unsigned short)kP7Zero;
          bval[w] = 0.0;
        }
        bseg[lr * nt + a] = (unsigned short)w;
      }
    }
    out.meta.push_back((int)out.blob.size());
    out.meta.push_back(n16);
    out.meta.push_back((int)rows.size());
    out.meta.push_back(nent);
    const size_t at = out.blob.size();
    out.blob.resize(at + n16);
    std::memcpy(out.blob.data() + at, bytes.data(), (size_t)n16 * 16);
    SUN_REQUIRE(out.blob.size() < (size_t)INT32_MAX, SUN_ENOTSUP, "path 7 block data exceeds 2^31 16-byte units");
  }
}

// Row blocks of at most max_rows rows and kLdsCap entries; empty if a single
// row has more than kLdsCap entries (the group then takes the per-wavefront
// path).
std::vector<int> lds_partition(const std::vector<int>& rp, int max_rows) {
  std::vector<int> blk{0};
  const int M = (int)rp.size() - 1;
  int r0 = 0;
  while (r0 < M) {
    if (rp[r0 + 1] - rp[r0] > kLdsCap) return {};
    int r1 = r0 + 1;
    while (r1 < M && r1 - r0 < max_rows && rp[r1 + 1] - rp[r0] <= kLdsCap) ++r1;
    blk.push_back(r1);
    r0 = r1;
  }
  return blk;
}

void refresh_items(sun_batch_s& bt) {
  int64_t item = 0;
  for (int g = 0; g < bt.ngroups; ++g) {
    GroupDev& G = bt.ghost[g];
    // LDS path: a tile of 128 is 64 lanes with two instances each; path 2
    // gives narrower tiles (16, 32, 64) two instances per lane as well
    const bool two = bt.nblk[g] > 0 && (bt.tile[g] == 128 || (bt.path[g] >= 2 && bt.tile[g] >= 16) || bt.xl[g]);
    G.vec = two ? 2 : 1;
    G.tile = two ? bt.tile[g] / 2 : std::min(bt.tile[g], 64);
    G.xlds = bt.xl[g];
    G.ucol_ptr = bt.xl[g] ? bt.xu_ptr[g].get() : nullptr;
    G.ucol = bt.xl[g] ? bt.xu_col[g].get() : nullptr;
    G.lidx = bt.xl[g] ? bt.xu_lidx[g].get() : nullptr;
    G.rows_per_item = bt.rows_per_item[g];
    G.ld = bt.ld[g];
    G.row_blocks = (int)((bt.M[g] + G.rows_per_item - 1) / G.rows_per_item);
    G.tiles = (G.B + G.tile * G.vec - 1) / (G.tile * G.vec);
    G.p5 = bt.path[g] == 5;
    if (G.p5) {              // one wavefront (64 lanes) per (row, tile)
      G.vec = bt.tile[g] == 128 ? 2 : 1;
      G.tile = 64;
      G.tiles = (G.B + 64 * G.vec - 1) / (64 * G.vec);
      G.row_blocks = 0;        // no items of the block kernels
    }
    if (bt.path[g] == 4) {   // advanced by the multi-instance sliced kernel instead
      G.row_blocks = 0;
      G.tiles = 0;
    }
    G.p7 = bt.path[g] == 7;
    G.p7_nblk = bt.p7_nblk[g];
    G.p7_meta = reinterpret_cast<const int4*>(bt.p7_meta[g].get());
    G.p7_ucol = bt.p7_ucol[g].get();
    G.p7_blob = bt.p7_blob[g].get();
    G.p7_nlong = bt.p7_nlong[g];
    G.p7_long = bt.p7_long[g].get();
    if (G.p7) {              // tiles of 64 instances, one per lane; no items of the other kernels
      G.vec = 1;
      G.tile = kP7Tile;
      G.tiles = (G.B + kP7Tile - 1) / kP7Tile;
      G.row_blocks = 0;
    }
  }
  for (int gi : bt.order) {
    GroupDev& G = bt.ghost[gi];
    G.nblk = bt.path[gi] >= 4 ? 0 : bt.nblk[gi];
    G.blk_row = bt.blk_row[gi].get();
    G.item0 = item;
    if (G.nblk == 0) item += (int64_t)G.row_blocks * G.tiles;
  }
}

// Per-wavefront and LDS work items of a group (one of the two is zero).
int64_t wave_items(const GroupDev& G) { return G.nblk > 0 ? 0 : (int64_t)G.row_blocks * G.tiles; }

void repartition(sun_batch_s& bt, int g) {
  const int max_rows = std::min(bt.rows_per_item[g], kLdsRows);
  std::vector<int> blk;
  bt.xl[g] = 0;
  bt.p7_meta[g].release();
  bt.p7_ucol[g].release();
  bt.p7_blob[g].release();
  bt.p7_long[g].release();
  bt.p7_nblk[g] = 0;
  bt.p7_nlong[g] = 0;
  if (bt.path[g] >= 4) {
    bt.xu_ptr[g].release();
    bt.xu_col[g].release();
    bt.xu_lidx[g].release();
    bt.nblk[g] = 0;
    bt.blk_row[g].release();
    if (bt.path[g] == 7) {
      const int64_t M = bt.M[g];
      const int nt = bt.nt[g];
      std::vector<int> hseg((size_t)M * nt), hcol(bt.nnz[g]);
      std::vector<double> hval(bt.nnz[g]);
      if (M > 0)
        HIP_OK(hipMemcpy(hseg.data(), bt.segptr[g].get(), hseg.size() * sizeof(int), hipMemcpyDeviceToHost));
      if (bt.nnz[g] > 0) {
        HIP_OK(hipMemcpy(hcol.data(), bt.col[g].get(), hcol.size() * sizeof(int), hipMemcpyDeviceToHost));
        HIP_OK(hipMemcpy(hval.data(), bt.val[g].get(), hval.size() * sizeof(double), hipMemcpyDeviceToHost));
      }
      layout_failure_point();   // the old layout is gone from here on
      P7Part pp;
      p7_partition(bt.lind[g]->basis->N, M, nt, bt.h_rowptr[g], hseg, hcol, hval,
                   std::min(bt.rows_per_item[g], kP7Rows), pp);
      const int nb = (int)(pp.meta.size() / 4);
      bt.p7_meta[g].alloc(std::max<size_t>(4, pp.meta.size()));
      bt.p7_ucol[g].alloc(std::max<size_t>(1, pp.ucol.size()));
      bt.p7_blob[g].alloc(std::max<size_t>(1, pp.blob.size()));
      bt.p7_long[g].alloc(std::max<size_t>(1, pp.longrows.size()));
      if (nb > 0) {
        HIP_OK(hipMemcpy(bt.p7_meta[g].get(), pp.meta.data(), pp.meta.size() * sizeof(int), hipMemcpyHostToDevice));
        HIP_OK(hipMemcpy(bt.p7_ucol[g].get(), pp.ucol.data(), pp.ucol.size() * sizeof(int), hipMemcpyHostToDevice));
        HIP_OK(hipMemcpy(bt.p7_blob[g].get(), pp.blob.data(), pp.blob.size() * sizeof(uint4), hipMemcpyHostToDevice));
      }
      if (!pp.longrows.empty())
        HIP_OK(hipMemcpy(bt.p7_long[g].get(), pp.longrows.data(), pp.longrows.size() * sizeof(int),
                         hipMemcpyHostToDevice));
      bt.p7_nblk[g] = nb;
      bt.p7_nlong[g] = (int)pp.longrows.size();
    }
    return;
  }
  if (bt.path[g] == 3) {
    std::vector<int> hcol(bt.nnz[g]);
    if (bt.nnz[g] > 0)
      HIP_OK(hipMemcpy(hcol.data(), bt.col[g].get(), bt.nnz[g] * sizeof(int), hipMemcpyDeviceToHost));
    XPart xp;
    if (xlds_partition(bt.h_rowptr[g], hcol, max_rows, xlds_cap(bt.tile[g]), xp)) {
      blk = xp.blk;
      bt.xu_ptr[g].alloc(xp.uptr.size());
      bt.xu_col[g].alloc(std::max<size_t>(1, xp.ucol.size()));
      bt.xu_lidx[g].alloc(std::max<size_t>(1, xp.lidx.size()));
      HIP_OK(hipMemcpy(bt.xu_ptr[g].get(), xp.uptr.data(), xp.uptr.size() * sizeof(int), hipMemcpyHostToDevice));
      if (!xp.ucol.empty())
        HIP_OK(hipMemcpy(bt.xu_col[g].get(), xp.ucol.data(), xp.ucol.size() * sizeof(int), hipMemcpyHostToDevice));
      if (!xp.lidx.empty())
        HIP_OK(hipMemcpy(bt.xu_lidx[g].get(), xp.lidx.data(), xp.lidx.size() * sizeof(unsigned short),
                         hipMemcpyHostToDevice));
      bt.xl[g] = 1;
    }
  }
  if (!bt.xl[g]) {
    bt.xu_ptr[g].release();
    bt.xu_col[g].release();
    bt.xu_lidx[g].release();
    if (bt.path[g] != 1) blk = lds_partition(bt.h_rowptr[g], max_rows);
  }
  bt.nblk[g] = blk.empty() ? 0 : (int)blk.size() - 1;
  if (bt.nblk[g] > 0) {
    bt.blk_row[g].alloc(blk.size());
    HIP_OK(hipMemcpy(bt.blk_row[g].get(), blk.data(), blk.size() * sizeof(int), hipMemcpyHostToDevice));
  } else {
    bt.blk_row[g].release();
  }
}

void upload(sun_batch_s& bt, hipStream_t s) {
  HIP_OK(hipMemcpyAsync(bt.gdev.get(), bt.ghost.data(), bt.ngroups * sizeof(GroupDev), hipMemcpyHostToDevice, s));
  HIP_OK(hipStreamSynchronize(s));
}

void alloc_state(sun_batch_s& bt, int g, hipStream_t s) {
  const int64_t M = bt.M[g];
  const int ld = bt.ld[g];
  bt.v[g].alloc((M + 1) * ld);
  bt.xa[g].alloc((M + 1) * ld);
  bt.xb[g].alloc((M + 1) * ld);
  bt.acc[g].alloc(M * (int64_t)ld);
  for (DevBuf<double>* p : {&bt.v[g], &bt.xa[g], &bt.xb[g]}) {
    hipLaunchKernelGGL(k_b_fill, dim3(grid_for(M * ld, 256)), dim3(256), 0, s, M * (int64_t)ld, 0.0, p->get());
    HIP_LAUNCH_OK();
    hipLaunchKernelGGL(k_b_fill, dim3(grid_for(ld, 256)), dim3(256), 0, s, (int64_t)ld, 1.0, p->get() + M * ld);
    HIP_LAUNCH_OK();
  }
  HIP_OK(hipMemsetAsync(bt.acc[g].get(), 0, M * ld * sizeof(double), s));
  GroupDev& G = bt.ghost[g];
  G.v = bt.v[g].get();
  G.xa = bt.xa[g].get();
  G.xb = bt.xb[g].get();
  G.acc = bt.acc[g].get();
}

int round_up(int x, int m) { return (x + m - 1) / m * m; }

// Path 4 set-up: classify the terms (a term is merged into the static part
// when every instance has the same constant coefficient, u = 0 and equal w),
// build the segmented sliced layout of the others (1 to 3 segments) and the
// instance-major state buffers.
void setup_multi(sun_batch_s& bt, int g, hipStream_t s) {
  if (bt.mprop[g]) return;
  const int nt = bt.nt[g], B = bt.B[g];
  std::vector<double> hw((size_t)B * nt), hu((size_t)B * nt);
  HIP_OK(hipMemcpy(hw.data(), bt.w[g], hw.size() * sizeof(double), hipMemcpyDeviceToHost));
  HIP_OK(hipMemcpy(hu.data(), bt.u[g], hu.size() * sizeof(double), hipMemcpyDeviceToHost));
  std::vector<double> static_w(nt, 0.0);
  std::vector<int> dyn;
  for (int a = 0; a < nt; ++a) {
    bool same = true;
    for (int b = 0; b < B && same; ++b) same = hu[(size_t)b * nt + a] == 0.0 && hw[(size_t)b * nt + a] == hw[a];
    if (same) static_w[a] = hw[a];
    else dyn.push_back(a);
  }
  SUN_REQUIRE(!dyn.empty() && (int)dyn.size() <= kMaxRevSeg, SUN_ENOTSUP,
              "path 4 needs 1 to 3 terms whose coefficients differ between instances");
  for (int a = bt.lind[g]->nH; a < nt; ++a)
    SUN_REQUIRE(static_w[a] >= 0.0, SUN_EINVAL, "dissipation rates must be >= 0");
  sun_prop q = nullptr;
  const int st = sun_prop_create(const_cast<sun_lind_s*>(bt.lind[g]), static_w.data(), dyn.data(), (int)dyn.size(), s, &q);
  if (st != SUN_OK) SUN_THROW(st, std::string("path 4 layout: ") + sun_last_error());
  try {
    prop_build_segments(*q, s);
  } catch (...) {
    sun_prop_free(q);
    throw;
  }
  q->layout = 2;
  q->resident = 0;
  bt.mprop[g] = q;
  bt.mterm[g] = dyn;
  const int64_t n = (int64_t)B * (bt.M[g] + 1);
  for (DevBuf<double>* b : {&bt.mv[g], &bt.mxa[g], &bt.mxb[g], &bt.macc[g]}) {
    b->alloc(n);
    hipLaunchKernelGGL(k_b_fill, dim3(grid_for(n, 256)), dim3(256), 0, s, n, 1.0, b->get());
    HIP_LAUNCH_OK();
  }
}

// One RK4 stage of every active path-4 group.
template <int STAGE>
void launch_multi(sun_batch_s& bt, const std::vector<int>& groups, const int64_t* stepidx, hipStream_t s) {
  for (int g : groups) {
    const sun_prop_s& p = *bt.mprop[g];
    MultiCoef mc;
    mc.w = bt.w[g];
    mc.u = bt.u[g];
    mc.wave = bt.wave[g];
    mc.widx = 2 * stepidx[g] + (STAGE == 0 ? 0 : (STAGE == 3 ? 2 : 1));
    mc.nt = bt.nt[g];
    for (int d = 0; d < (int)bt.mterm[g].size(); ++d) mc.term[d] = bt.mterm[g][d];
    mc.B = bt.B[g];
    mc.ldv = bt.M[g] + 1;
    double* v = bt.mv[g].get();
    double* xa = bt.mxa[g].get();
    double* xb = bt.mxb[g].get();
    const double* xin = STAGE == 0 ? v : (STAGE == 1 ? xa : (STAGE == 2 ? xb : xa));
    double* xout = STAGE == 0 ? xa : (STAGE == 1 ? xb : (STAGE == 2 ? xa : v));
    prop_stage_multi(p, STAGE, xin, v, bt.macc[g].get(), xout, mc, bt.tile[g], bt.dt[g], s);
  }
}

// One RK4 stage over all active groups: the per-wavefront kernel, the LDS
// kernels (one or two instances per lane) and the path-3 kernel, each
// launched only when some group takes it.
struct StageLaunch {
  const GroupDev* gd = nullptr;
  const int* go = nullptr;
  const int64_t* st = nullptr;
  hipStream_t s = nullptr;
  int nactive = 0, cf_len = 0;
  int64_t nitems = 0, grid = 1, bgrid = 8, xgrid = 8;
  bool v1 = false, v2 = false, xl = false;
  bool r1 = false, r2 = false;   // path-5 groups with one / two instances per lane
  int64_t rgrid[3] = {0, 0, 0};  // path-5 grids (resident wavefronts, a multiple of 8), by VEC
  int r_nt = 1;                  // most terms of a path-5 group
  std::vector<P7Plan> p7;        // path-7 groups, at most kP7MaxGroups per launch
  int64_t pgrid = 16;            // path-7 grid (the resident workgroups, a multiple of 8)
};

// Wavefronts of k_batch_rows<*, VEC> the device keeps resident (the least
// over the four stages), rounded down to a multiple of 8 XCDs.
template <int VEC>
int64_t rows_grid(int ncu, size_t lds) {
  int least = INT32_MAX;
  const void* ks[4] = {(const void*)k_batch_rows<0, VEC>, (const void*)k_batch_rows<1, VEC>,
                       (const void*)k_batch_rows<2, VEC>, (const void*)k_batch_rows<3, VEC>};
  for (const void* k : ks) {
    int nb = 0;
    HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, 64, lds));
    least = std::min(least, nb);
  }
  SUN_REQUIRE(least >= 1, SUN_ENOTSUP, "path 5 kernel cannot be resident");
  return std::max<int64_t>(8, (int64_t)least * ncu / 8 * 8);
}

// Workgroups of k_batch_pipe the device keeps resident (the least over the
// four stages, at least one per XCD and two more), rounded down to a
// multiple of 8 XCDs.
int64_t pipe_grid(int ncu) {
  int least = INT32_MAX;
  const void* ks[4] = {(const void*)k_batch_pipe<0>, (const void*)k_batch_pipe<1>, (const void*)k_batch_pipe<2>,
                       (const void*)k_batch_pipe<3>};
  for (const void* k : ks) {
    int nb = 0;
    HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, kP7Threads, 0));
    least = std::min(least, nb);
  }
  SUN_REQUIRE(least >= 1, SUN_ENOTSUP, "path 7 kernel cannot be resident");
  return std::max<int64_t>(16, (int64_t)least * ncu / 8 * 8);
}

template <int STAGE>
void launch_stage(const StageLaunch& L) {
  const size_t cf_bytes = (size_t)L.cf_len * sizeof(double);
  if (L.nitems > 0)
    hipLaunchKernelGGL(k_batch_stage<STAGE>, dim3((unsigned)L.grid), dim3(256), 0, L.s, L.gd, L.go, L.nactive,
                       L.nitems, L.st);
  if (L.v1)
    hipLaunchKernelGGL((k_batch_stage_lds<STAGE, 1>), dim3((unsigned)L.bgrid), dim3(256), cf_bytes, L.s, L.gd, L.go,
                       L.nactive, L.st);
  if (L.v2)
    hipLaunchKernelGGL((k_batch_stage_lds<STAGE, 2>), dim3((unsigned)L.bgrid), dim3(256), cf_bytes, L.s, L.gd, L.go,
                       L.nactive, L.st);
  if (L.xl)
    hipLaunchKernelGGL(k_batch_stage_xlds<STAGE>, dim3((unsigned)L.xgrid), dim3(256), cf_bytes + kXLdsBytes, L.s,
                       L.gd, L.go, L.nactive, L.st, L.cf_len);
  if (L.r1)
    hipLaunchKernelGGL((k_batch_rows<STAGE, 1>), dim3((unsigned)L.rgrid[1]), dim3(64),
                       (size_t)L.r_nt * 64 * sizeof(double), L.s, L.gd, L.go, L.nactive, L.st);
  if (L.r2)
    hipLaunchKernelGGL((k_batch_rows<STAGE, 2>), dim3((unsigned)L.rgrid[2]), dim3(64),
                       (size_t)L.r_nt * 128 * sizeof(double), L.s, L.gd, L.go, L.nactive, L.st);
  for (const P7Plan& plan : L.p7)
    hipLaunchKernelGGL(k_batch_pipe<STAGE>, dim3((unsigned)L.pgrid), dim3(kP7Threads), 0, L.s, L.gd, plan, L.st);
}

}  // namespace

extern "C" int sun_batch_create(const sun_lind* lind, int32_t ngroups, const int32_t* B, const double* const* w,
                                const double* const* u, const double* const* wave, const double* dt,
                                const int64_t* steps, void* stream, sun_batch* out) {
  return guarded([&] {
    SUN_REQUIRE(out != nullptr, SUN_EINVAL, "out is NULL");
    *out = nullptr;
    SUN_REQUIRE(ngroups >= 1 && lind && B && w && u && wave && dt && steps, SUN_EINVAL, "NULL argument");
    hipStream_t s = as_stream(stream);
    auto bt = new sun_batch_s();
    try {
      bt->ngroups = ngroups;
      bt->lind.resize(ngroups);
      bt->B.resize(ngroups);
      bt->tile.assign(ngroups, 64);
      bt->rows_per_item.assign(ngroups, 64);
      bt->M.resize(ngroups);
      bt->P.resize(ngroups);
      bt->nnz.resize(ngroups);
      bt->steps.resize(ngroups);
      bt->done.assign(ngroups, 0);
      bt->dt.resize(ngroups);
      bt->w.resize(ngroups);
      bt->u.resize(ngroups);
      bt->wave.resize(ngroups);
      bt->rowptr.resize(ngroups);
      bt->segptr.resize(ngroups);
      bt->col.resize(ngroups);
      bt->val.resize(ngroups);
      bt->v.resize(ngroups);
      bt->xa.resize(ngroups);
      bt->xb.resize(ngroups);
      bt->acc.resize(ngroups);
      bt->ld.resize(ngroups);
      bt->nt.resize(ngroups);
      bt->ghost.resize(ngroups);
      bt->h_rowptr.resize(ngroups);
      bt->blk_row.resize(ngroups);
      bt->nblk.assign(ngroups, 0);
      bt->path.assign(ngroups, 0);
      bt->xl.assign(ngroups, 0);
      bt->xu_ptr.resize(ngroups);
      bt->xu_col.resize(ngroups);
      bt->xu_lidx.resize(ngroups);
      bt->mprop.assign(ngroups, nullptr);
      bt->mterm.resize(ngroups);
      bt->mv.resize(ngroups);
      bt->mxa.resize(ngroups);
      bt->mxb.resize(ngroups);
      bt->macc.resize(ngroups);
      bt->p7_meta.resize(ngroups);
      bt->p7_ucol.resize(ngroups);
      bt->p7_blob.resize(ngroups);
      bt->p7_long.resize(ngroups);
      bt->p7_nblk.assign(ngroups, 0);
      bt->p7_nlong.assign(ngroups, 0);
      bt->usable.assign(ngroups, 1);
      for (int g = 0; g < ngroups; ++g) {
        const sun_lind_s* l = lind[g];
        SUN_REQUIRE(l != nullptr, SUN_EINVAL, "group system is NULL");
        SUN_REQUIRE(B[g] >= 1, SUN_EINVAL, "every group needs at least one instance");
        SUN_REQUIRE(steps[g] >= 0 && dt[g] > 0.0, SUN_EINVAL, "steps must be >= 0 and dt > 0");
        SUN_REQUIRE(w[g] && u[g] && wave[g], SUN_EINVAL, "coefficient arrays are NULL");
        const int nt = l->nH + l->P;
        SUN_REQUIRE(nt <= kMaxBTerms, SUN_ENOTSUP, "at most 8 terms per group");
        bt->lind[g] = l;
        bt->B[g] = B[g];
        bt->M[g] = l->basis->M;
        bt->P[g] = l->basis->P;
        bt->steps[g] = steps[g];
        bt->dt[g] = dt[g];
        bt->w[g] = w[g];
        bt->u[g] = u[g];
        bt->wave[g] = wave[g];
        bt->nt[g] = nt;
        TermPtrs t{};
        t.n = nt;
        for (int a = 0; a < nt; ++a) {
          const DevCSR& m = a < l->nH ? l->QH[a] : l->R[a - l->nH];
          t.rowptr[a] = m.rowptr.get();
          t.col[a] = m.col.get();
          t.val[a] = m.val.get();
          t.K[a] = a < l->nH ? nullptr : l->K[a - l->nH].get();
        }
        const int64_t M = bt->M[g];
        DevBuf<int64_t> cnt(M), off(M);
        const int64_t P = bt->P[g];
        hipLaunchKernelGGL(k_batch_fuse, dim3(grid_for(M, 128)), dim3(128), 0, s, M, P, t, 0, cnt.get(), nullptr,
                           nullptr, nullptr, nullptr);
        HIP_LAUNCH_OK();
        bt->nnz[g] = exclusive_scan_i64(cnt.get(), off.get(), M, s);
        SUN_REQUIRE(bt->nnz[g] < (int64_t)INT32_MAX, SUN_ENOTSUP, "group matrix has 2^31 or more nonzeros");
        bt->rowptr[g].alloc(M + 1);
        bt->segptr[g].alloc(M * nt);
        // kRowPad zero entries after the last one (path 5 reads ahead)
        bt->col[g].alloc(bt->nnz[g] + kRowPad);
        bt->val[g].alloc(bt->nnz[g] + kRowPad);
        HIP_OK(hipMemsetAsync(bt->col[g].get() + bt->nnz[g], 0, kRowPad * sizeof(int), s));
        HIP_OK(hipMemsetAsync(bt->val[g].get() + bt->nnz[g], 0, kRowPad * sizeof(double), s));
        hipLaunchKernelGGL(k_batch_fuse, dim3(grid_for(M, 128)), dim3(128), 0, s, M, P, t, 1, nullptr, off.get(),
                           bt->segptr[g].get(), bt->col[g].get(), bt->val[g].get());
        HIP_LAUNCH_OK();
        hipLaunchKernelGGL(k_b_i64_to_i32, dim3(grid_for(M, 256)), dim3(256), 0, s, M, off.get(), bt->nnz[g],
                           bt->rowptr[g].get());
        HIP_LAUNCH_OK();
        HIP_OK(hipStreamSynchronize(s));
        bt->h_rowptr[g].resize(M + 1);
        HIP_OK(hipMemcpy(bt->h_rowptr[g].data(), bt->rowptr[g].get(), (M + 1) * sizeof(int), hipMemcpyDeviceToHost));
        repartition(*bt, g);
        bt->ld[g] = round_up(B[g], 128);
        GroupDev& G = bt->ghost[g];
        G = GroupDev{};
        G.rowptr = bt->rowptr[g].get();
        G.segptr = bt->segptr[g].get();
        G.col = bt->col[g].get();
        G.val = bt->val[g].get();
        G.w = w[g];
        G.u = u[g];
        G.wave = wave[g];
        G.dt = dt[g];
        G.M = (int)M;
        G.B = B[g];
        G.nt = nt;
        alloc_state(*bt, g, s);
      }
      bt->order.resize(ngroups);
      for (int g = 0; g < ngroups; ++g) bt->order[g] = g;
      bt->gdev.alloc(ngroups);
      refresh_items(*bt);
      upload(*bt, s);
    } catch (...) {
      delete bt;
      throw;
    }
    *out = bt;
  });
}

extern "C" int sun_batch_set_state(sun_batch bt, int32_t g, const double* V, void* stream) {
  return guarded([&] {
    SUN_REQUIRE(bt != nullptr && V != nullptr, SUN_EINVAL, "NULL argument");
    SUN_REQUIRE(g >= 0 && g < bt->ngroups, SUN_EINVAL, "group index out of range");
    hipStream_t s = as_stream(stream);
    if (bt->path[g] == 4) {
      const int64_t total = (int64_t)bt->B[g] * (bt->M[g] + 1);
      hipLaunchKernelGGL(k_to_im, dim3(grid_for(total, 256)), dim3(256), 0, s, (int)bt->M[g], bt->B[g],
                         bt->M[g] + 1, V, bt->mv[g].get());
      HIP_LAUNCH_OK();
      bt->done[g] = 0;
      return;
    }
    const int64_t total = (bt->M[g] + 1) * bt->ld[g];
    hipLaunchKernelGGL(k_to_rowmajor, dim3(grid_for(total, 256)), dim3(256), 0, s, (int)bt->M[g],
                       bt->P[g], bt->B[g],
                       bt->ld[g], V, bt->v[g].get());
    HIP_LAUNCH_OK();
    bt->done[g] = 0;
  });
}

extern "C" int sun_batch_get_state(sun_batch bt, int32_t g, double* V, void* stream) {
  return guarded([&] {
    SUN_REQUIRE(bt != nullptr && V != nullptr, SUN_EINVAL, "NULL argument");
    SUN_REQUIRE(g >= 0 && g < bt->ngroups, SUN_EINVAL, "group index out of range");
    hipStream_t s = as_stream(stream);
    const int64_t total = bt->M[g] * bt->B[g];
    if (bt->path[g] == 4) {
      hipLaunchKernelGGL(k_from_im, dim3(grid_for(total, 256)), dim3(256), 0, s, (int)bt->M[g], bt->B[g],
                         bt->M[g] + 1, bt->mv[g].get(), V);
      HIP_LAUNCH_OK();
      return;
    }
    hipLaunchKernelGGL(k_from_rowmajor, dim3(grid_for(total, 256)), dim3(256), 0, s, (int)bt->M[g],
                       bt->P[g], bt->B[g],
                       bt->ld[g], bt->v[g].get(), V);
    HIP_LAUNCH_OK();
  });
}

extern "C" int sun_batch_tune(sun_batch bt, int32_t g, int32_t tile, int32_t rows_per_item, int32_t path,
                              void* stream) {
  return guarded([&] {
    SUN_REQUIRE(bt != nullptr, SUN_EINVAL, "batch is NULL");
    SUN_REQUIRE(g >= 0 && g < bt->ngroups, SUN_EINVAL, "group index out of range");
    SUN_REQUIRE(path >= 0 && path <= 7 && path != 6, SUN_EINVAL, "path must be 0, 1, 2, 3, 4, 5 or 7");
    if (path == 7) {
      SUN_REQUIRE(tile == kP7Tile, SUN_EINVAL, "path 7 takes tiles of 64 instances");
      SUN_REQUIRE(rows_per_item >= 1 && rows_per_item <= kP7Rows, SUN_EINVAL,
                  "path 7 takes 1 to " + std::to_string(kP7Rows) + " rows per block");
      SUN_REQUIRE((bt->M[g] + 1) * (int64_t)bt->ld[g] * 8 < (int64_t)kP7Off, SUN_ENOTSUP,
                  "path 7 needs a group state below 2 GiB (32-bit buffer offsets)");
    } else if (path == 4) {
      SUN_REQUIRE(tile == 2 || tile == 4 || tile == 8, SUN_EINVAL, "path 4 takes 2, 4 or 8 instances per wavefront");
    } else if (path == 5) {
      SUN_REQUIRE(tile == 64 || tile == 128, SUN_EINVAL, "path 5 takes tiles of 64 or 128 instances");
    } else {
      SUN_REQUIRE(tile == 8 || tile == 16 || tile == 32 || tile == 64 || tile == 128, SUN_EINVAL,
                  "tile must be 8, 16, 32, 64 or 128");
    }
    SUN_REQUIRE(rows_per_item >= 1 && rows_per_item <= 65536, SUN_EINVAL, "rows_per_item out of range");
    SUN_REQUIRE(path != 3 || tile == 8 || tile == 16 || tile == 32, SUN_EINVAL, "path 3 takes tiles 8, 16 or 32");
    hipStream_t s = as_stream(stream);
    HIP_OK(hipStreamSynchronize(s));
    if (path == 4) setup_multi(*bt, g, s);
    // the state moves with the layout
    const int old = bt->path[g];
    const int M = (int)bt->M[g];
    if (old != 4 && path == 4) {
      const int64_t total = (int64_t)bt->B[g] * (M + 1);
      hipLaunchKernelGGL(k_rm_to_im, dim3(grid_for(total, 256)), dim3(256), 0, s, M, bt->P[g], bt->B[g], bt->ld[g],
                         (int64_t)M + 1, bt->v[g].get(), bt->mv[g].get());
      HIP_LAUNCH_OK();
    } else if (old == 4 && path != 4) {
      const int64_t total = (int64_t)M * bt->ld[g];
      hipLaunchKernelGGL(k_im_to_rm, dim3(grid_for(total, 256)), dim3(256), 0, s, M, bt->P[g], bt->B[g], bt->ld[g],
                         (int64_t)M + 1, bt->mv[g].get(), bt->v[g].get());
      HIP_LAUNCH_OK();
    }
    bt->tile[g] = tile;
    bt->rows_per_item[g] = rows_per_item;
    bt->path[g] = path;
    bt->usable[g] = 0;          // until the new layout is complete
    repartition(*bt, g);
    bt->usable[g] = 1;
    refresh_items(*bt);
    upload(*bt, s);
  });
}

extern "C" int sun_batch_info(sun_batch bt, int32_t g, int64_t* M, int64_t* nnz, int32_t* tile,
                              int32_t* rows_per_item) {
  return guarded([&] {
    SUN_REQUIRE(bt != nullptr, SUN_EINVAL, "batch is NULL");
    SUN_REQUIRE(g >= 0 && g < bt->ngroups, SUN_EINVAL, "group index out of range");
    if (M) *M = bt->M[g];
    if (nnz) *nnz = bt->nnz[g];
    if (tile) *tile = bt->tile[g];
    if (rows_per_item) *rows_per_item = bt->rows_per_item[g];
  });
}

extern "C" int sun_batch_run(sun_batch bt, int64_t nsteps, int32_t only_group, void* stream) {
  return guarded([&] {
    SUN_REQUIRE(bt != nullptr, SUN_EINVAL, "batch is NULL");
    SUN_REQUIRE(nsteps >= 0, SUN_EINVAL, "nsteps must be >= 0");
    SUN_REQUIRE(only_group >= -1 && only_group < bt->ngroups, SUN_EINVAL, "group index out of range");
    hipStream_t s = as_stream(stream);
    // per group: how many steps this call advances it
    std::vector<int64_t> todo(bt->ngroups, 0);
    for (int g = 0; g < bt->ngroups; ++g)
      if (only_group < 0 || only_group == g) todo[g] = std::min(nsteps, bt->steps[g] - bt->done[g]);
    for (int g = 0; g < bt->ngroups; ++g)
      SUN_REQUIRE(todo[g] <= 0 || bt->usable[g], SUN_EINVAL,
                  "group " + std::to_string(g) + " has an incomplete layout after a failed sun_batch_tune; tune it again");
    std::vector<int> ord(bt->ngroups);
    for (int g = 0; g < bt->ngroups; ++g) ord[g] = g;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return todo[a] > todo[b]; });
    bt->order = ord;
    refresh_items(*bt);
    upload(*bt, s);
    int64_t maxn = todo[ord[0]];
    if (maxn <= 0) return;
    // device copies: group order and per-group absolute step index
    DevBuf<int> gorder(bt->ngroups);
    DevBuf<int64_t> stepidx(bt->ngroups);
    HIP_OK(hipMemcpyAsync(gorder.get(), ord.data(), bt->ngroups * sizeof(int), hipMemcpyHostToDevice, s));
    // prefix sums of work items in launch order (per-wavefront and LDS paths)
    std::vector<int64_t> items_upto(bt->ngroups + 1, 0);
    for (int q = 0; q < bt->ngroups; ++q) {
      const GroupDev& G = bt->ghost[ord[q]];
      items_upto[q + 1] = items_upto[q] + wave_items(G);
    }
    // the step index of every group lives in a device table: one row per step
    std::vector<int64_t> table((size_t)maxn * bt->ngroups);
    for (int64_t n = 0; n < maxn; ++n)
      for (int g = 0; g < bt->ngroups; ++g) table[(size_t)n * bt->ngroups + g] = bt->done[g] + n;
    DevBuf<int64_t> steptab(table.size());
    HIP_OK(hipMemcpyAsync(steptab.get(), table.data(), table.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
    int dev = 0, ncu = 0;
    HIP_OK(hipGetDevice(&dev));
    HIP_OK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    // path-5 grids: the resident wavefronts for the largest term count of
    // the groups the call advances
    int p5_nt = 1;
    bool p5_vec[3] = {false, false, false};
    for (int g = 0; g < bt->ngroups; ++g)
      if (todo[g] > 0 && bt->ghost[g].p5) {
        p5_nt = std::max(p5_nt, bt->ghost[g].nt);
        p5_vec[bt->ghost[g].vec] = true;
      }
    int64_t p5_grid[3] = {0, 0, 0};
    bool any_p7 = false;
    for (int g = 0; g < bt->ngroups; ++g) any_p7 = any_p7 || (todo[g] > 0 && bt->ghost[g].p7);
    const int64_t p7_grid = any_p7 ? pipe_grid(ncu) : 16;
    if (p5_vec[1]) p5_grid[1] = rows_grid<1>(ncu, (size_t)p5_nt * 64 * sizeof(double));
    if (p5_vec[2]) p5_grid[2] = rows_grid<2>(ncu, (size_t)p5_nt * 128 * sizeof(double));
    for (int64_t n = 0; n < maxn; ++n) {
      int nactive = 0;
      while (nactive < bt->ngroups && todo[ord[nactive]] > n) ++nactive;
      StageLaunch L;
      L.nactive = nactive;
      L.nitems = items_upto[nactive];
      L.grid = std::max<int64_t>(1, std::min<int64_t>((L.nitems + 3) / 4, (int64_t)ncu * 8));
      int64_t nlds = 0, nx = 0;
      int max_nt = 1;
      for (int q = 0; q < nactive; ++q) {
        const GroupDev& G = bt->ghost[ord[q]];
        if (G.p5) {
          // the kernel's tile of 64 * vec instances stays inside the padded state rows
          SUN_REQUIRE(G.tiles * 64 * G.vec <= G.ld && G.nt <= kMaxBTerms, SUN_ENOTSUP,
                      "internal: path 5 tile exceeds the state rows");
          (G.vec == 2 ? L.r2 : L.r1) = true;
          continue;
        }
        if (G.p7) {
          // every 64-instance tile stays inside the padded state rows
          SUN_REQUIRE(G.tiles * kP7Tile <= G.ld && G.nt <= kMaxBTerms, SUN_ENOTSUP,
                      "internal: path 7 tile exceeds the state rows");
          if (L.p7.empty() || L.p7.back().ng == kP7MaxGroups) L.p7.push_back(P7Plan{});
          P7Plan& pl = L.p7.back();
          if (G.p7_nlong > 0) pl.klong = kP7LongWgs;
          pl.g[pl.ng] = ord[q];
          pl.nblk[pl.ng] = G.p7_nblk;
          pl.tiles[pl.ng] = G.tiles;
          ++pl.ng;
          continue;
        }
        if (G.nblk == 0) continue;
        max_nt = std::max(max_nt, G.nt);
        if (G.xlds) {
          L.xl = true;
          nx += (int64_t)G.nblk * G.tiles;
        } else {
          (G.vec == 2 ? L.v2 : L.v1) = true;
          nlds += (int64_t)G.nblk * G.tiles;
        }
      }
      // grids are multiples of 8 (one share per XCD); path 3 holds ~50 KB of
      // LDS per workgroup, so three per CU are resident
      L.bgrid = std::max<int64_t>(8, (std::min<int64_t>(nlds, (int64_t)ncu * 8) + 7) / 8 * 8);
      L.xgrid = std::max<int64_t>(8, (std::min<int64_t>(nx, (int64_t)ncu * 3) + 7) / 8 * 8);
      L.cf_len = max_nt * kCfStride;
      L.r_nt = p5_nt;
      L.pgrid = p7_grid;
      for (P7Plan& pl : L.p7)   // at least one workgroup per XCD keeps the blocks
        pl.klong = std::min<int>(pl.klong, (int)(L.pgrid / 8) - 1);
      L.rgrid[1] = p5_grid[1];
      L.rgrid[2] = p5_grid[2];
      L.st = steptab.get() + n * bt->ngroups;
      L.gd = bt->gdev.get();
      L.go = gorder.get();
      L.s = s;
      // path-4 groups advanced this step, with their absolute step index
      std::vector<int> multi;
      for (int q = 0; q < nactive; ++q)
        if (bt->path[ord[q]] == 4) multi.push_back(ord[q]);
      std::vector<int64_t> sidx(bt->ngroups, 0);
      for (int g : multi) sidx[g] = bt->done[g] + n;
      launch_stage<0>(L);
      launch_multi<0>(*bt, multi, sidx.data(), s);
      launch_stage<1>(L);
      launch_multi<1>(*bt, multi, sidx.data(), s);
      launch_stage<2>(L);
      launch_multi<2>(*bt, multi, sidx.data(), s);
      launch_stage<3>(L);
      launch_multi<3>(*bt, multi, sidx.data(), s);
    }
    HIP_LAUNCH_OK();
    for (int g = 0; g < bt->ngroups; ++g) bt->done[g] += todo[g];
    // finite check of the states the call advanced (a non-finite entry stays
    // non-finite under RK4, so the end of the call catches any step of it)
    DevBuf<int> bad(1);
    set_int(bad.get(), 0, s);
    for (int g = 0; g < bt->ngroups; ++g)
      if (todo[g] > 0) {
        if (bt->path[g] == 4) flag_nonfinite(bt->mv[g].get(), (int64_t)bt->B[g] * (bt->M[g] + 1), bad.get(), s);
        else flag_nonfinite(bt->v[g].get(), (bt->M[g] + 1) * bt->ld[g], bad.get(), s);
      }
    int h = 0;
    HIP_OK(hipMemcpyAsync(&h, bad.get(), sizeof(int), hipMemcpyDeviceToHost, s));
    // the step table and group order are freed on return
    HIP_OK(hipStreamSynchronize(s));
    SUN_REQUIRE(h == 0, SUN_EDIVERGED, "a batched state is not finite after this call (NaN or Inf)");
  });
}

extern "C" int sun_batch_device_bytes(sun_batch bt, size_t* bytes) {
  return guarded([&] {
    SUN_REQUIRE(bt != nullptr && bytes != nullptr, SUN_EINVAL, "NULL argument");
    size_t b = bt->gdev.bytes();
    for (int g = 0; g < bt->ngroups; ++g) {
      for (const DevBuf<int>* x : {&bt->rowptr[g], &bt->segptr[g], &bt->col[g], &bt->blk_row[g], &bt->xu_ptr[g],
                                   &bt->xu_col[g]})
        b += x->bytes();
      for (const DevBuf<double>* x : {&bt->val[g], &bt->v[g], &bt->xa[g], &bt->xb[g], &bt->acc[g], &bt->mv[g],
                                      &bt->mxa[g], &bt->mxb[g], &bt->macc[g]})
        b += x->bytes();
      b += bt->xu_lidx[g].bytes();
      b += bt->p7_meta[g].bytes() + bt->p7_ucol[g].bytes() + bt->p7_blob[g].bytes() + bt->p7_long[g].bytes();
      if (bt->mprop[g]) b += prop_device_bytes(*bt->mprop[g]);
    }
    *bytes = b;
  });
}

extern "C" void sun_batch_free(sun_batch bt) { delete bt; }

extern "C" int sun_propagate_batched(const sun_lind* lind, int32_t ngroups, const int32_t* B, const double* const* w,
                                     const double* const* u, const double* const* wave, const double* dt,
                                     const int64_t* steps, double* const* V, void* stream) {
  return guarded([&] {
    SUN_REQUIRE(V != nullptr, SUN_EINVAL, "V is NULL");
    for (int g = 0; g < ngroups; ++g) SUN_REQUIRE(V[g] != nullptr, SUN_EINVAL, "V[g] is NULL");
    sun_batch bt = nullptr;
    int st = sun_batch_create(lind, ngroups, B, w, u, wave, dt, steps, stream, &bt);
    if (st != SUN_OK) SUN_THROW(st, sun_last_error());
    std::unique_ptr<sun_batch_s> hold(bt);
    int64_t most = 0;
    for (int g = 0; g < ngroups; ++g) {
      st = sun_batch_set_state(bt, g, V[g], stream);
      if (st != SUN_OK) SUN_THROW(st, sun_last_error());
      most = std::max(most, steps[g]);
    }
    st = sun_batch_run(bt, most, -1, stream);
    const int run_st = st;
    const std::string run_msg = st != SUN_OK ? sun_last_error() : "";
    if (st != SUN_OK && st != SUN_EDIVERGED) SUN_THROW(st, run_msg);
    for (int g = 0; g < ngroups; ++g) {
      st = sun_batch_get_state(bt, g, V[g], stream);
      if (st != SUN_OK) SUN_THROW(st, sun_last_error());
    }
    HIP_OK(hipStreamSynchronize(as_stream(stream)));
    if (run_st != SUN_OK) SUN_THROW(run_st, run_msg);
  });
}
