// Internal declarations shared by the HIP translation units of libadl.
// Nothing here is part of the public C ABI (include/adl.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace adl {

constexpr int kWave = 64;
constexpr int kBlock = 256;             // elementwise and reduction kernels
#ifndef ADL_WAVES_Y
#define ADL_WAVES_Y 4
#endif
#ifndef ADL_MAX_GRID
#define ADL_MAX_GRID 16384
#endif
#ifndef ADL_WAVES_Y2
#define ADL_WAVES_Y2 4
#endif
#ifndef ADL_MAX_GRID2
#define ADL_MAX_GRID2 4096
#endif
#ifndef ADL_MAX_GRID3
#define ADL_MAX_GRID3 1536
#endif
constexpr int kWavesY = ADL_WAVES_Y;     // stencil blocks: waves stacked in y (one strip)
constexpr int kTileBlock = kWave * kWavesY;
constexpr int kMaxGrid = ADL_MAX_GRID;   // blocks of a stencil launch (tiles walked per block)
constexpr int kWavesY2 = ADL_WAVES_Y2;   // two-term kernel: waves (= output rows) per block
constexpr int kTileBlock2 = kWave * kWavesY2;
constexpr int kMaxGrid2 = ADL_MAX_GRID2;
// three-term launches (LDS-staged, three blocks per CU): fewer blocks with
// longer runs of bands, so that the run's prologue (two stages on four rows
// above the run) is spread over more output rows (measured at 4096^2 FP64,
// the headline's steps: 4096 blocks 211 us per launch, 2304 201 us, 1536
// 194 us)
constexpr int kMaxGrid3 = ADL_MAX_GRID3;

enum { BC_PERIODIC = 0, BC_DIRICHLET = 1 };

// Stopping rule of a Newton-Leja sweep (the paper leaves it open; tol is the
// accuracy asked of the result, as Sec. 3 uses it): the truncation error of the
// degree-m interpolant is estimated by the norms of its last kStopWindow
// terms, and the sweep stops at the first m >= kStopWindow with
//   ||d_{m-4} y_{m-4}|| + ... + ||d_m y_m|| <= tol ||p_m||
// (summed oldest first).  Single terms rise and fall by orders of magnitude
// from one Leja point to the next on wide intervals, so one small term is no
// estimate of the error.  The norms of the kStopWindow - 1 terms before a
// decided launch are kept in the control block, slot m mod (kStopWindow - 1).
constexpr int kStopWindow = 5;
constexpr int kStopHist = kStopWindow - 1;

// The stopping test of term m (norm tn of its term d_m y_m, squared norm pn2
// of p_m) against the ring `hist` of the norms of terms m - 4 .. m - 1,
// which it then updates with tn.
__device__ __forceinline__ bool window_stop(double (&hist)[kStopHist], int m, double tn, double pn2, double tol) {
  bool stop = false;
  if (m >= kStopWindow) {
    double est = 0.0;
#pragma unroll
    for (int j = kStopHist; j >= 1; --j) est += hist[(m - j) % kStopHist];
    est += tn;
    stop = est <= tol * sqrt(pn2);
  }
  hist[m % kStopHist] = tn;
  return stop;
}

// Per-sweep control block in device memory.  Written only by the last block
// of a launch (fixed-order reduction), read by the next launch and the host.
struct Ctl {
  int stop;             // 1: every later launch of this sweep returns at once
  int status;           // 0 running, 1 converged, 2 non-finite, 3 degree cap
  int degree;           // Newton terms (matrix applications) so far
  unsigned int ticket;  // arrival counter of the running launch (reset by last block)
  double tn2, pn2;      // ||d y||^2, ||p||^2 of the last term
  double scale;         // power iteration: 1 / lambda_k
  double lam, lam_prev; // power iteration estimates
  double gmin;          // Gershgorin result
  int iters;
  int pad[3];
  double hist[kStopHist];  // ||d_m y_m|| of the latest decided terms, slot m mod kStopHist
};
static_assert(sizeof(Ctl) <= 128, "ctl size");

// The outcome of a sweep as the host reads it: a copy of the control block's
// fields, written by the chunk's one-block decision launch into coherent
// (fine-grained) pinned host memory, fields first and the sequence number
// last with a system-scope release.  The host spins on the number instead of
// copying the control block back and synchronising the stream, which wakes
// the host many microseconds later.  One cache line per op.
struct HostCtl {
  int seq;
  int stop, status, degree;
  int pad[12];
};
static_assert(sizeof(HostCtl) == 64, "one cache line");

// The stored operator.  Coefficients are pre-scaled:
//   kxx = Dxx / hx^2, kyy = Dyy / hy^2, kxy = Dxy / (4 hx hy),
//   ax' = ax / (2 hx), ay' = ay / (2 hy)
struct FieldView {
  const void* kxx;
  const void* kxy;
  const void* kyy;
  const void* ax;   // nullptr: constant axc
  const void* ay;   // nullptr: constant ayc
  double axc, ayc;
  int nx, ny, bc;
  int f32;          // fields stored as float
};

// Tiling of one grid for the stencil kernels.  A tile = one strip of
// 64*vec columns x kWavesY*rows rows (a row band), one block's unit of work;
// wave w of the block computes rows [w*rows, (w+1)*rows) of the tile.  Block b
// takes strip b mod ncb and the run of `bands` consecutive row bands number
// b / ncb, so the rows shared by consecutive bands are re-read from cache.
struct Tiling {
  int vec;      // columns per lane (1 or 2; 2 needs even nx)
  int rows;     // rows per wave and tile
  int ncb, nrb; // strips / row bands
  int bands;    // consecutive row bands per block
  int nblocks;  // ncb * ceil(nrb / bands)
};

// rows_hint <= 0: default rows; vec_hint 0: widest usable, 1 or 2: forced
Tiling make_tiling(int nx, int ny, int rows_hint, int vec_hint = 0);

// ---- launches (stencil.hip) ----------------------------------------------
// y = A x + a1 s1 + a2 s2   (s1 / s2 may be null)
hipError_t launch_apply(const FieldView& f, const Tiling& t, const double* x, double* y,
                        const double* s1, double a1, const double* s2, double a2,
                        hipStream_t st);
// the same, and y2 = (s2 - s1) d2 as a second output (s1, s2 required)
hipError_t launch_apply2(const FieldView& f, const Tiling& t, const double* x, double* y,
                         const double* s1, double a1, const double* s2, double a2, double* y2, double d2,
                         hipStream_t st);

// One launch of a Newton-Leja sweep: terms k+1 .. k+nterms (nterms = 1, or 2
// for the two-term kernel), plus the stopping decision of the previous
// launch's terms (taken by block 0).
struct LejaArgs {
  const void* yin;   // y_k (double at k = 0, else the y storage type)
  void* yout;        // y of the launch's last term, or null (not stored: a replay)
  const double* pin; // p_k (k >= 1; FP64)
  double* p;         // p of the launch's last term (a different buffer from pin), or
                     // null (not stored: a replay of a launch whose earlier term is the result)
  double* pmid;      // two-term launch: p_{k+1}; four-term launch: p_{k+1}; null: not stored
  const double* w2;  // augmented column (first term only), or null
  double w2c;        // s_0 / h
  double shift;      // c + gamma xi_k   (term k+1)
  double shift2;     // c + gamma xi_{k+1} (term k+2)
  double invg;       // 1 / gamma
  double d0, dk1, dk2;  // d_0 (first launch), d_{k+1}, d_{k+2}
  double tol;        // stopping tolerance (window test above)
  int k;             // terms before this launch
  int nterms;        // terms of this launch
  int max_degree;
  int first;         // k == 0: p = d0 y0 + d1 y1, zero-vector test
  int ystore_f32;    // y stored as float
  int yin_f32;       // y_k stored as float
  int stream;        // non-temporal hints on p_k and the written vectors
  int staged;        // two-term launch: input rows staged in LDS (leja2s_kernel)
  double* partials;  // two slots of 6 x (max blocks) values
  long slot_stride;
  int slot;          // slot written by this launch
  int nb_prev;       // the decided launch: block count, terms before it, its terms, its slot
  int k_prev;
  int nterms_prev;
  int slot_prev;
  int decide_only;   // only take the decision of the previous launch (1-block launch)
  Ctl* ctl;
  HostCtl* hctl;     // decision launch: publish the outcome here (device address), or null
  int hseq;          // ... with this sequence number
  hipEvent_t ev_start;  // optional: dispatch-attached timing events
  hipEvent_t ev_stop;
  // four-term launch: terms k+3 and k+4, and p_{k+2}, p_{k+3} (at the end:
  // fields inserted further up move the arguments the other kernels read,
  // which cost the two-term register-frame launch 10 % at 2048^2)
  double shift3, shift4;
  double dk3, dk4;
  double* pmid2;
  double* pmid3;
  int lds_fields;    // four-term launch: stage 1 keeps the field rows in LDS for stages 2-4
  // Replay of a launch of a finished sweep, to store p of one of its earlier
  // terms (the result, when the sweep stopped inside the launch): the same
  // arithmetic on the same y_k and p_k, no stop flag, no decision, no partials
  int replay;
  // The sweep's first launch computing its own stage vector (four-term staged
  // kernel, terms 1 .. 3): yin = u, src = s (or null) of w = A u + s
  int stage;
  const double* src;
};
hipError_t launch_leja_step(const FieldView& f, const Tiling& t, const LejaArgs& a, hipStream_t st);
// two-term launch (terms k+1, k+2; k >= 1) on the two-term tiling
hipError_t launch_leja2_step(const FieldView& f, const Tiling& t, const LejaArgs& a, hipStream_t st);
// tiling of the two-term kernel: strips of 62*vec output columns, bands of kWavesY*rows rows
// (frame: lanes at each strip end whose outputs are not stored -- 1 for the
// two- and three-term kernels, 2 for the four-term staged kernel)
Tiling make_tiling2(int nx, int ny, int rows_hint, int vec_hint = 0, int max_blocks = kMaxGrid2, int frame = 1);
// three-term launch (terms k+1 .. k+3; k = 0 with a.first: y_0 = v, FP64
// Newton vectors, no augmented column) with the input rows staged in LDS, on
// a two-term tiling with two columns per lane; the launch's block partials
// take 9 x nblocks values of its slot
hipError_t launch_leja3_step(const FieldView& f, const Tiling& t, const LejaArgs& a, hipStream_t st);
// four-term launch (terms k+1 .. k+4; k >= 1) with the input rows staged in
// LDS, on a tiling of strips of 60*VEC output columns with two columns per
// lane (make_tiling2 with frame 2); block partials: 12 x nblocks values.
// With a.stage: the sweep's first launch, stage vector w = A u + s and terms
// 1 .. 3 (dk1 .. dk4 = d_0 .. d_3, shift2 .. shift4 = the first three
// shifts), partials as a three-term launch's
hipError_t launch_leja4s_step(const FieldView& f, const Tiling& t, const LejaArgs& a, hipStream_t st);
// four-term launch (terms k+1 .. k+4; k >= 1) on the four-term tiling; the
// launch's block partials take 12 x nblocks values of its slot
hipError_t launch_leja4_step(const FieldView& f, const Tiling& t, const LejaArgs& a, hipStream_t st);
// tiling of the four-term kernel: strips of 56*vec output columns, 8 output rows per block
Tiling make_tiling4(int nx, int ny, int vec_hint = 0);
// A four-term block with output rows J0 .. J0 + kFourTermRows - 1 (J0 a
// multiple of kFourTermRows, at most ny - 1) reads grid rows
// J0 - kFourTermTerms .. J0 + kFourTermRows - 1 + kFourTermTerms: a frame of
// one row per stage on each side, plus the stencil's own neighbour row.  The
// row rule wraps a periodic row index once, so on a periodic grid every such
// row lands inside the grid only if the first block's lowest row is >= -ny
// and the last block's highest row is <= 2 ny - 1 (true for every ny >= 11,
// false for ny = 3, 4, 5 and 9).  Grids where it fails run two terms per
// launch.
constexpr int kFourTermRows = 8;   // output rows per block
constexpr int kFourTermTerms = 4;  // Newton terms per launch
inline bool four_term_rows_fit(int ny, int bc) {
  if (bc != BC_PERIODIC) return true;  // rows outside a Dirichlet grid are zero or edge rows, never loaded
  const int j0_last = kFourTermRows * ((ny - 1) / kFourTermRows);
  return -kFourTermTerms >= -ny && j0_last + kFourTermRows - 1 + kFourTermTerms <= 2 * ny - 1;
}

// power iteration launch k: w = A(x) / ||x||, stopping test of iteration k
struct PowerArgs {
  const double* x;
  double* w;
  double rtol;
  int max_iter;
  int k;
  int nb;            // block count of every power launch (and of the start-vector kernel)
  int decide_only;
  double* partials;  // 3 slots x nb
  Ctl* ctl;
};
hipError_t launch_power_init(const Tiling& t, long n, uint64_t seed, double* w, double* partials,
                             hipStream_t st);
hipError_t launch_power_step(const FieldView& f, const Tiling& t, const PowerArgs& a, hipStream_t st);
hipError_t launch_gershgorin(const FieldView& f, double* partials, Ctl* ctl, hipStream_t st);

// ---- elementwise (stencil.hip) --------------------------------------------
hipError_t launch_ctl_reset(Ctl* ctl, int n, hipStream_t st);
// y = a * x + b * z  (z may be null; y may alias x or z)
hipError_t launch_axpby(long n, double* y, double a, const double* x, double b, const double* z,
                        hipStream_t st);
hipError_t launch_fill(long n, double* y, double v, hipStream_t st);
// y = (x - z) * s   (the difference is formed first, so equal x and z give exact zeros)
hipError_t launch_diff_scale(long n, double* y, const double* x, const double* z, double s, hipStream_t st);
// out_f = (double or float) scale * in   for field preparation
hipError_t launch_prepare_field(long n, const double* in, double scale, void* out, int f32,
                                hipStream_t st);

// ---- learned bound (mlp.hip) -----------------------------------------------
// blocks of a one-pass reduction over n nodes (field statistics, Gershgorin):
// eight nodes per thread, so that the per-block release fence and ticket
// (the cost of such a launch on cache-resident grids) are paid once per 2048
// nodes; at most 1024 blocks
inline int stats_blocks(long n) {
  const long nb = (n + 8L * kBlock - 1) / (8L * kBlock);
  return (int)(nb < 1 ? 1 : (nb > 1024 ? 1024 : nb));
}
// Gershgorin partials of a batched statistics launch, after the statistics'
constexpr long kGershPartials = 6 * 1024;

// One op's share of the batched statistics launch (read by the kernel from
// device memory): blocks [blk0, blk0 + nb_s) reduce its field statistics with
// ctl[0]'s ticket, the next nb_g (0: Gershgorin bound already known) its
// Gershgorin bound with ctl[1]'s, each exactly as the op's own launch would.
struct BoundJob {
  FieldView f;
  double hx, hy;
  double* partials;
  Ctl* ctl;
  int blk0, nb_s, nb_g, pad;
};
static_assert(sizeof(BoundJob) <= 128, "job size");
// jobs[n] and blk0[n + 1] (prefix of nb_s + nb_g, blk0[n] = all blocks) in
// device memory; feats[9 i ..] and gmin[i] receive job i's results.  Resets
// the jobs' ctl[0] and ctl[1] first.
hipError_t launch_bound_stats_many(const BoundJob* jobs, const int* blk0, int n, int nblocks, double dt,
                                   float* feats, double* gmin, hipStream_t st);
hipError_t launch_field_stats(const FieldView& f, double hx, double hy, double dt, float* feats,
                              double* partials, Ctl* ctl, hipStream_t st);
hipError_t launch_mlp_forward(const float* W, const float* X, float* Y, float* cache, int B,
                              hipStream_t st);
hipError_t launch_mlp_backward(const float* W, const float* cache, const float* dY, float* dW,
                               int B, hipStream_t st);
hipError_t launch_mlp_mse_grad(const float* Y, const float* T, float* dY, float* loss, int B, hipStream_t st);
hipError_t launch_mlp_adam(float* W, const float* dW, float* m1, float* m2, int t, float lr,
                           float b1, float b2, float eps, hipStream_t st);

}  // namespace adl
