// Propagator object and stage launcher shared by the plain, profiled and
// adjoint propagation entry points.
#pragma once

#include "internal.hpp"

using sun::DevBuf;

struct sun_prop_s {
  const sun_lind_s* lind = nullptr;
  int64_t M = 0;
  int ndyn = 0;
  int64_t nnz = 0;
  DevBuf<int> rowptr, col, seg, blk_row;
  DevBuf<double> val;
  int64_t nblocks = 0;
  int block_nnz = 1024;
  int threads = 256;
  int xcd_remap = 1;
  DevBuf<double> vaug, xa, xb, acc;
  // sliced-ELL layout (used when ndyn <= 1)
  int layout = 1;            // 0 = CSR stream, 1 = sliced ELL + long rows, 2 = segmented sliced ELL (2-3 dyn terms)
  int sigma = 4096;          // rows sorted by length inside windows of sigma rows
  int long_len = 32;         // rows longer than this use the wave-per-row path
  int min_col_bytes = 1;     // narrowest column-delta width allowed (1, 2 or 4)
  int sell_remap = 1;        // XCD-contiguous slice ranges
  int sell_nt = 0;           // 1: non-temporal loads for the matrix stream
  int sell_pairs = 0;        // 1: slices cut from the pair-interleaved row sequence
  int resident = 0;          // sun_propagate runs every step in one single-workgroup launch
  int sell_unroll = 8;       // entries per lane per load round (4, 6, 8, 12 or 16)
  int sell_split = 1;        // wavefronts per slice of the stage kernel (1, 2 or 4)
  int64_t nshort = 0, nlong = 0, nslices = 0, sell_nnz = 0, sell_col_bytes = 0;
  DevBuf<int> sell_row, sell_len, sell_off, sell_coff, sell_base, long_rows;
  DevBuf<unsigned char> sell_cb;
  DevBuf<double> sell_val;
  DevBuf<double> rec_part;   // partial sums of the recorded observable
  // segmented sliced layout (adjoint reverse stages with dot products): the
  // starts of up to kMaxRevSeg time-dependent segments per lane, 8 bits each
  int sell_segs = 0;
  DevBuf<int> sell_seg;
  // run-time checks
  int usable = 1;            // 0 after a re-layout failed part-way: every launching call refuses
  int check_finite = 1;      // finite check of the state at the end of each propagation call
  DevBuf<int> bad;           // [1] set by the finite check, reset after it is read
  double dt_max = 0.0;       // > 0: stability guard, larger dt is refused (SUN_EUNSTABLE)
  double rho_guard = 0.0;    // |lambda|max estimate behind dt_max
  // HIP-graph replay of chunks of sun_propagate steps, for generators small
  // enough that a stage launch is dominated by launch latency
  int graph_mode = 1;        // 0: never, 1: when M <= kGraphMaxRows (default), 2: always
  int layout_gen = 0;        // bumped by every re-layout; a captured graph is valid for one generation
  int graph_gen = -1;        // generation, and step size, the current graph was captured with
  double graph_dt = 0.0;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  DevBuf<double> gcoef;      // the coefficient rows of the chunk being replayed
  sun_prop_s() = default;
  sun_prop_s(const sun_prop_s&) = delete;
  sun_prop_s& operator=(const sun_prop_s&) = delete;
  ~sun_prop_s();
};

namespace sun {

// Refuse a propagator whose layout is not in a launchable state.
void prop_require_usable(const sun_prop_s& p);
// Device memory the propagator holds (bytes).
size_t prop_device_bytes(const sun_prop_s& p);
// Queue the finite check of x[0..n) (sets p.bad[0]); read and reset it with
// prop_finite_result, which synchronises the stream.  Both are no-ops when
// the propagator's check is off.
void prop_finite_check(const sun_prop_s& p, const double* x, int64_t n, hipStream_t s);
bool prop_finite_result(const sun_prop_s& p, hipStream_t s);

// Largest fused generator (stored nonzeros) that sun_prop_create puts in the
// CSR stream layout rather than the sliced one.
constexpr int64_t kStreamMaxNnz = 100000;

// One launch of stage `stage` of the fused generator on the given vectors.
// Forward RK4 stages 0..3 (see propagate.hip):
//   k = G(t) xin;  0: xout = vin + dt/2 k, acc = k;  1: xout = vin + dt/2 k,
//   acc += 2k;  2: xout = vin + dt k, acc += 2k;  3: xout = vin + dt/6 (acc + k).
// Reverse-mode stages 4..7 (the propagator must hold the transposed
// generator; vin = lambda, acc = lambda accumulator, xout = next cotangent):
//   k = G(t)^T xin;  4: acc = vin + k, xout = dt/3 vin + dt k;
//   5: acc += k, xout = dt/3 vin + dt/2 k;  6: acc += k, xout = dt/6 vin + dt/2 k;
//   7: acc += k;  8: acc = (acc + k) + vin, xout = dt/6 acc (stage 7 fused with
//   the start of the next backward step).
// Vectors have M+1 entries with entry M equal to 1.
void prop_stage(const sun_prop_s& p, int stage, const double* xin, const double* vin, double* acc, double* xout,
                const double* coef, int64_t coef_row, double dt, hipStream_t s);

// Adjoint parameter dot products on static generators T_j (j < n <= 8) in
// sliced layout (no time-dependent term), for the kDotStages RK4 stages of
// one step, all in one launch: adds, for th < ntheta,
//   sum_i dc_jth(t_i) * (kbs[i] . (T_j xs[i]))   (xs[i][M] = 1 brings in T_j's free vector)
// split over prop_dot_slots(*ps[j]) per-wavefront slots
// gpart[(y * ntheta + th) * ld + slot0[j] + w] (y < kDotStages / kDotStagesPerWave
// selects the stages), with dc_jth(t_i) = dstat[term[j] * ntheta + th]
// (+ dcoef[(krows[i] * ndyn + slot[j]) * ntheta + th] when slot[j] >= 0).  The
// slot sums are to be reduced in a fixed order.
constexpr int kMaxDotTerms = 8;
constexpr int kMaxRevSeg = 3;
constexpr int kDotStages = 4;
constexpr int kDotStagesPerWave = 2;   // stages one wavefront takes (1, 2 or 4)
// slots per launch: kDotStages / kDotStagesPerWave groups of ntheta * ld
int64_t prop_dot_slots(const sun_prop_s& p);
void prop_dot(const sun_prop_s* const* ps, const int* term, const int* slot, const int64_t* slot0, int n,
              const double* const* xs, const double* const* kbs, const int64_t* krows, const double* dstat,
              const double* dcoef, int ndyn, int ntheta, double* gpart, int64_t ld, hipStream_t s);

// Reverse stage with the parameter dot products fused in.  The propagator
// holds the transposed generator with every parameter-dependent term as its
// own time-dependent segment (ndyn = nseg <= kMaxRevSeg, in the segmented
// sliced layout of prop_build_segments).  Segment d has the coefficient
// wseg[d] (+ coef[krow * ncoef + slot[d]] when slot[d] >= 0) at this stage's
// time.  Besides the stage update of prop_stage (stages 4..8), every
// wavefront adds, for th < ntheta,
//   sum_d dc_d,th * (sum over its rows r of s_d[r] xdot[r] + xin[r] K_d[r])
// to gpart[th * ld + w] (w = its slice, or nslices + its long row), where
// s_d = T_dᵀ xin is the row's segment sum, K_d the term's free vector (or
// NULL) and dc_d,th = dstat[term[d] * ntheta + th] (+ dcoef[(krow * ncoef +
// slot[d]) * ntheta + th] when slot[d] >= 0): kb . (T_d x + K_d) of the
// forward stage input x = xdot through kb . T_d x = (T_dᵀ kb) . x.
struct RevDot {
  int nseg = 0;
  double wseg[kMaxRevSeg] = {};
  int slot[kMaxRevSeg] = {-1, -1, -1};
  int term[kMaxRevSeg] = {};
  const double* K[kMaxRevSeg] = {};
  const double* coef = nullptr;
  int ncoef = 0;
  const double* dstat = nullptr;
  const double* dcoef = nullptr;
  int ntheta = 0;
  double* gpart = nullptr;
  int64_t ld = 0;
};
void prop_build_segments(sun_prop_s& p, hipStream_t s);
int64_t prop_rev_slots(const sun_prop_s& p);
void prop_stage_dot(const sun_prop_s& p, int stage, const double* xin, const double* vin, double* acc, double* xout,
                    const double* xdot, const RevDot& rd, int64_t krow, double dt, hipStream_t s);
// Per-instance coefficients of the time-dependent segments for the
// multi-instance stage: c_{b,d} = w[b * nt + term[d]] + u[b * nt + term[d]] * wave[widx].
struct MultiCoef {
  const double* w = nullptr;
  const double* u = nullptr;
  const double* wave = nullptr;
  int64_t widx = 0;
  int nt = 0;
  int term[kMaxRevSeg] = {};
  int B = 0;          // instances
  int64_t ldv = 0;    // stride between instance vectors (>= M + 1)
};
// One forward RK4 stage (0..3) for B instance vectors (instance-major, stride
// mc.ldv, entry M = 1) on the segmented sliced layout (layout 2, ndyn =
// number of segments), ki = 2, 4 or 8 instances per wavefront.
void prop_stage_multi(const sun_prop_s& p, int stage, const double* xin, const double* vin, double* acc,
                      double* xout, const MultiCoef& mc, int ki, double dt, hipStream_t s);
// Forward stage 0..3 on the segmented sliced layout (layout 2: 2-3
// time-dependent terms, segment d with coefficient coef[row * ndyn + d]).
void prop_seg_stage(const sun_prop_s& p, int stage, const double* xin, const double* vin, double* acc, double* xout,
                    const double* coef, int64_t row, double dt, hipStream_t s);
// Throws SUN_ENOMEM once after sun_debug_inject_failure(1) (tests of the
// error paths of the layout builds).
void layout_failure_point();

}  // namespace sun
