// Nine-point stencil kernels for gfx950: operator application, the fused
// Newton-Leja term, power iteration, Gershgorin bound, elementwise helpers.
//
// The operator is A = div(D grad .) + div(a .) (Sec. 1 eq. 2, Sec. 2), in the
// conservative central nine-point form
//   (A u)_C = kf_E (u_E - u_C) - kf_W (u_C - u_W) + kf_N (u_N - u_C) - kf_S (u_C - u_S)
//           + kxy_E (u_NE - u_SE) - kxy_W (u_NW - u_SW)
//           + kxy_N (u_NE - u_NW) - kxy_S (u_SE - u_SW)
//           + ax_E u_E - ax_W u_W + ay_N u_N - ay_S u_S
// with face coefficients kf_E = (kxx_C + kxx_E)/2 etc. and pre-scaled
// coefficient fields (kxx = Dxx/hx^2, kxy = Dxy/(4 hx hy), ax' = ax/(2 hx)).
//
// Layout and mapping.  Arrays are [ny][nx], x contiguous.  A tile is one strip
// of 64 * VEC columns by 4 * rows rows; the four waves of a block take the
// four row bands of a tile (stacked in y, so the rows they share are L1 hits),
// each wave computing one row per load group (tile.h).  Block b takes strip
// b mod ncb and a run of consecutive row bands, so the rows shared between
// consecutive bands are re-read from cache soon after their first load.
// Newton-Leja sweeps run one term (leja_kernel), two terms per launch (the
// register-frame kernel leja2_kernel on cache-resident grids, the kernel with
// input rows staged in LDS, leja2s_kernel in staged.h, beyond the caches) or
// four (leja4_kernel, on mid-size grids).
//
// Reductions (norms for the Leja stopping test, power iteration) are fixed
// order: shuffle tree per wave, waves in order, block partials written to
// memory.  One block of the next launch (or a one-block launch closing a
// chunk) sums them in index order and records the decision; worker waves only
// read the stop flag (no agent-scope fence; a kernel boundary makes the
// partials visible).  Results are bitwise reproducible for a given tiling.
#include "bounds.h"
#include "staged.h"

#include <type_traits>

#include <hip/hip_ext.h>

#include <cmath>

namespace adl {

// ---------------------------------------------------------------------------
// Block-wide fixed-order reduction (sums for k < NS, NaN-propagating max for
// the rest); every thread receives the totals.
// ---------------------------------------------------------------------------
template <int NA, int NS>
__device__ __forceinline__ void block_allreduce_at(double (&v)[NA], double* sh) {
#pragma unroll
  for (int k = 0; k < NA; ++k) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double t = __shfl_xor(v[k], o);
      v[k] = (k < NS) ? v[k] + t : nanmax(v[k], t);
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NA; ++k) sh[wave * NA + k] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NA; ++k) {
    double s = sh[k];
    for (int w = 1; w < nw; ++w) s = (k < NS) ? s + sh[w * NA + k] : nanmax(s, sh[w * NA + k]);
    v[k] = s;
  }
}
// the same with a static LDS array (sh: NA * 16 doubles)
template <int NA, int NS>
__device__ __forceinline__ void block_allreduce(double (&v)[NA]) {
  __shared__ double sh[NA * 16];
  block_allreduce_at<NA, NS>(v, sh);
}

// Totals of the block partials written by an earlier launch: part[k * nb + b].
template <int NA, int NS>
__device__ __forceinline__ void partial_totals(const double* __restrict__ part, int nb, double (&tot)[NA]) {
#pragma unroll
  for (int k = 0; k < NA; ++k) {
    double s = 0.0;
    bool any = false;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
      const double v = part[(long)k * nb + i];
      s = (k < NS) ? s + v : (any ? nanmax(s, v) : v);
      any = true;
    }
    tot[k] = s;
  }
  block_allreduce<NA, NS>(tot);
}

// block partial of this launch -> part[k * nb + b]
template <int NA, int NS>
__device__ __forceinline__ void write_partials(double (&acc)[NA], double* __restrict__ part, int nb, int b) {
  block_allreduce<NA, NS>(acc);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NA; ++k) part[(long)k * nb + b] = acc[k];
  }
}

// The tiles of worker block b: strip b mod ncb, row bands
// [(b / ncb) * bands, (b / ncb + 1) * bands).
template <typename TF, typename TX, int VEC, bool ADVF, class Ep>
__device__ __forceinline__ void stencil_block(const FieldView& F, const Tiling& T, const TX* __restrict__ x,
                                              Ep& ep, int b) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform rows
  const int cb = b % T.ncb;
  const int rb0 = (b / T.ncb) * T.bands;
  const int rb1 = min(rb0 + T.bands, T.nrb);
#pragma unroll 1
  for (int rb = rb0; rb < rb1; ++rb) {
    const int j0 = (rb * kWavesY + wave) * T.rows;
    if (j0 < F.ny && !stencil_tile<TF, TX, VEC, ADVF>(F, x, ep, cb, j0, min(j0 + T.rows, F.ny))) break;
  }
}

// ---------------------------------------------------------------------------
// Epilogues
// ---------------------------------------------------------------------------
// out = A x + a1 s1 + a2 s2
template <int VEC>
struct ApplyEp {
  struct Extra {
    double s1[VEC];
    double s2[VEC];
  };
  int nx;
  double* __restrict__ out;
  const double* __restrict__ s1;
  const double* __restrict__ s2;
  double a1, a2;
  double* __restrict__ out2;  // optional second output (s2 - s1) * d2, difference first
  double d2;
  __device__ __forceinline__ bool go() const { return true; }
  __device__ __forceinline__ void load(int j, const Strip& g, Extra& e) {
    if (!g.inside) return;
    const long ro = (long)j * nx;
    if (s1) ldr<double, VEC>(s1 + ro, g.col0, e.s1);
    if (s2) ldr<double, VEC>(s2 + ro, g.col0, e.s2);
  }
  __device__ __forceinline__ void finish(int j, const Strip& g, const double (&Ax)[VEC], const double (&)[VEC],
                                         const Extra& e) {
    if (!g.inside) return;
    const long ro = (long)j * nx;
    double r[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      r[v] = Ax[v];
      if (s1) r[v] += a1 * e.s1[v];
      if (s2) r[v] += a2 * e.s2[v];
    }
    str<double, VEC>(out + ro, g.col0, r);
    if (out2) {
      double q[VEC];
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        const double dlt = e.s2[v] - e.s1[v];
        q[v] = dlt * d2;
      }
      str<double, VEC>(out2 + ro, g.col0, q);
    }
  }
};

template <typename TF, int VEC, bool ADVF>
__global__ __launch_bounds__(kTileBlock) void apply_kernel(FieldView F, Tiling T, const double* __restrict__ x,
                                                       ApplyEp<VEC> ep) {
  stencil_block<TF, double, VEC, ADVF>(F, T, x, ep, blockIdx.x);
}

// One Newton-Leja term (fused): y' = (A y + w2c w2 - shift y) invg,
// p' = p + d_{k+1} y'  (p = d_0 y at k = 0); partial norms of d y' and p'.
template <typename TYO, int VEC, bool FIRST, bool NT>
struct LejaEp {
  struct Extra {
    double p[VEC];
    double w[VEC];
  };
  int nx;
  TYO* __restrict__ yout;
  const double* __restrict__ pin;  // p_k (not on the first term)
  double* __restrict__ p;          // p_{k+1}
  const double* __restrict__ w2;   // only on the first term
  double w2c, shift, invg, d0, dk1;
  double acc[3];  // ||d y'||^2, ||p'||^2, max(|y0|, |w2|)
  int stopflag;   // the sweep's stop flag as loaded at the start of the wave
  __device__ __forceinline__ bool go() const { return __builtin_amdgcn_readfirstlane(stopflag) == 0; }
  __device__ __forceinline__ void load(int j, const Strip& g, Extra& e) {
    if (!g.inside) return;
    const long ro = (long)j * nx;
    if constexpr (FIRST) {
      if (w2) ldr<double, VEC>(w2 + ro, g.col0, e.w);
    } else {
      ldr_s<NT, double, VEC>(pin + ro, g.col0, e.p);
    }
  }
  __device__ __forceinline__ void finish(int j, const Strip& g, const double (&Ax)[VEC], const double (&yc)[VEC],
                                         const Extra& e) {
    if (!g.inside) return;
    const long ro = (long)j * nx;
    double yn[VEC], pn[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      double a = Ax[v];
      if constexpr (FIRST) {
        if (w2) a += w2c * e.w[v];
      }
      const double y1 = (a - shift * yc[v]) * invg;
      const double t = dk1 * y1;
      const double pv = (FIRST ? d0 * yc[v] : e.p[v]) + t;
      yn[v] = y1;
      pn[v] = pv;
      acc[0] += t * t;
      acc[1] += pv * pv;
      if constexpr (FIRST) {
        acc[2] = nanmax(acc[2], fabs(yc[v]));
        if (w2) acc[2] = nanmax(acc[2], fabs(e.w[v]));
      }
    }
    str_s<NT, TYO, VEC>(yout + ro, g.col0, yn);
    str_s<NT, double, VEC>(p + ro, g.col0, pn);
  }
};

// Stopping test of the terms of the previous launch (k_prev+1 ..
// k_prev+nterms_prev, in order) from its block partials, taken by one block
// (fixed-order totals) and recorded in the control block unless an earlier
// launch has already stopped the sweep.
// (dsh: a kernel's dynamic LDS for the reduction (160 doubles), or null for
// a static array; the four-term staged kernel passes its rings, so that it
// holds no static LDS and three blocks fit a CU)
template <bool DYN = false>
__device__ __forceinline__ void leja_decide(const LejaArgs& A, double* dsh = nullptr) {
  // the stop flag travels with the partial sums (a max-reduced value), so its
  // load and the partial loads are in flight together
  const double* part = A.partials + (long)A.slot_prev * A.slot_stride;
  const int nb = A.nb_prev;
  const int nt = A.nterms_prev;
  // tn2 / pn2 of terms 1 .. 4 of the decided launch (sums; term t's partials
  // at rows 3t, 3t + 1), max(|y0|, |w2|) (row 2), flag (max)
  double v[10] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (threadIdx.x == 0)
    v[9] = (double)__hip_atomic_load(&A.ctl->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  bool any = false;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    v[0] += part[i];
    v[1] += part[(long)nb + i];
    const double m = part[2L * nb + i];
    v[8] = any ? nanmax(v[8], m) : m;
    if (nt >= 2) {
      v[2] += part[3L * nb + i];
      v[3] += part[4L * nb + i];
    }
    if (nt >= 3) {
      v[4] += part[6L * nb + i];
      v[5] += part[7L * nb + i];
    }
    if (nt >= 4) {
      v[6] += part[9L * nb + i];
      v[7] += part[10L * nb + i];
    }
    any = true;
  }
  if constexpr (DYN) block_allreduce_at<10, 8>(v, dsh);
  else block_allreduce<10, 8>(v);
  if (v[9] != 0.0) return;  // decided by an earlier launch
  // Terms up to `done` were decided already: a chunk's closing decision
  // launch decides the chunk's last launch, and the first launch of the next
  // chunk is handed the same launch.  Each term enters the window once.
  const int done = A.ctl->degree;
  if (A.k_prev + nt <= done) return;
  // norms of the terms before the decided ones (the window of the test)
  double hist[kStopHist];
#pragma unroll
  for (int i = 0; i < kStopHist; ++i) hist[i] = A.ctl->hist[i];
  int stop = 0, status = 0, degree = A.k_prev + A.nterms_prev;
  double tn2 = 0.0, pn2 = 0.0;
  for (int t = 0; t < nt && !stop; ++t) {
    const int deg = A.k_prev + t + 1;
    if (deg <= done) continue;
    tn2 = v[2 * t];
    pn2 = v[2 * t + 1];
    if (!isfinite(tn2) || !isfinite(pn2)) {
      stop = 1; status = 2; degree = deg;
    } else if (deg == 1 && v[8] == 0.0) {
      stop = 1; status = 1; degree = 0;
    } else if (window_stop(hist, deg, sqrt(tn2), pn2, A.tol)) {
      stop = 1; status = 1; degree = deg;
    } else if (deg >= A.max_degree) {
      stop = 1; status = 3; degree = deg;
    }
  }
  if (threadIdx.x == 0) {
    Ctl* c = A.ctl;
    c->tn2 = tn2;
    c->pn2 = pn2;
#pragma unroll
    for (int i = 0; i < kStopHist; ++i) c->hist[i] = hist[i];
    c->degree = degree;
    c->status = status;
    __hip_atomic_store(&c->stop, stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// The sweep's outcome for the host (thread 0 of the decision launch, after
// leja_decide): the control block's fields (written by this thread, or by an
// earlier launch), then the sequence number with a system-scope release, so
// that a host that sees the number sees the fields too.
__device__ __forceinline__ void publish_outcome(const LejaArgs& A) {
  HostCtl* h = A.hctl;
  const Ctl* c = A.ctl;
  h->stop = __hip_atomic_load(&c->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  h->status = c->status;
  h->degree = c->degree;
  __hip_atomic_store(&h->seq, A.hseq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// The sweep's stop flag, read once per block (thread 0) and broadcast, so that
// a concurrent update of the flag cannot split a block.
__device__ __forceinline__ bool block_stopped(const Ctl* ctl) {
  __shared__ int s_stop;
  if (threadIdx.x == 0) s_stop = __hip_atomic_load(&ctl->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  return s_stop != 0;
}

// One Newton-Leja term, launch k: y_{k+1} from y_k, p_{k+1} = p_k + d_{k+1} y_{k+1}
// into the other p buffer, block partials of the norms.
//
// The stopping decision lags one launch behind the work: an extra block
// (block 0, dispatched first) takes the decision of term k from the partials
// of launch k-1 and records it, while the worker blocks 1 .. nblocks compute
// term k+1 without waiting for it.  A worker wave only checks the stop flag,
// which launches before this one have set, and only after its first loads
// are issued.  If term k turns out to be the last, the term computed by this
// launch is discarded: p_k is still intact in the other p
// buffer, and every later launch sees the flag and skips its work.  No store
// of a worker depends on a reduction, so the launch starts loading at once.
// Waves that skip their work still join the partial-sum barriers, and a wave
// that sees the flag set while its block's other waves did not only leaves
// its part of a discarded term unwritten.
//
// The first term of a sweep (y_0 = v in FP64, the augmented column w2, the
// zero-vector check) is a kernel of its own, so that the other terms'
// register allocation does not carry its extra state.
template <typename TF, typename TYI, typename TYO, int VEC, bool ADVF, bool FIRST, bool NT>
__global__ __launch_bounds__(kTileBlock) void leja_kernel(FieldView F, Tiling T, LejaArgs A) {
  // XCD-contiguous logical blocks: neighbouring tiles, which share halo
  // columns and rows, run on one XCD and meet in its L2
  const int L = A.decide_only ? 0 : xcd_contiguous(blockIdx.x, gridDim.x);
  if (L == 0) {
    if (!FIRST) {
      leja_decide(A);
      if (A.decide_only && A.hctl && threadIdx.x == 0) publish_outcome(A);
    } else if (threadIdx.x == 0) {
      // a new sweep: clear the control block (no block of this launch reads it)
      Ctl c{};
      *A.ctl = c;
    }
    return;
  }
  const int b = L - 1;
  LejaEp<TYO, VEC, FIRST, NT> ep;
  ep.nx = F.nx;
  ep.yout = reinterpret_cast<TYO*>(A.yout);
  ep.pin = FIRST ? nullptr : A.pin;
  ep.p = A.p;
  ep.w2 = FIRST ? A.w2 : nullptr;
  ep.w2c = FIRST ? A.w2c : 0.0;
  ep.shift = A.shift;
  ep.invg = A.invg;
  ep.d0 = A.d0;
  ep.dk1 = A.dk1;
  ep.acc[0] = ep.acc[1] = ep.acc[2] = 0.0;
  ep.stopflag = FIRST ? 0 : __hip_atomic_load(&A.ctl->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  stencil_block<TF, TYI, VEC, ADVF>(F, T, reinterpret_cast<const TYI*>(A.yin), ep, b);
  write_partials<3, 2>(ep.acc, A.partials + (long)A.slot * A.slot_stride, T.nblocks, b);
}

// ---------------------------------------------------------------------------
// Two Newton-Leja terms per launch (k >= 1): y_{k+1} is never written to
// memory.  A block owns a strip of 62*VEC output columns (lanes 1..62 of a
// wave strip that starts VEC columns to the left; lanes 0 and 63 are the
// one-column frame) and marches down a run of row bands, one output row per
// wave per step.  Stage 1 computes y_{k+1} on the step's rows over the
// strip's 64*VEC columns into an LDS ring, each wave keeping the face
// coefficients and p_k of its own row in registers; the one-row frame above is already in the
// ring and one wave adds the frame row below.  After a block barrier, stage 2
// computes y_{k+2} from the ring (x-neighbours by the same DPP shifts) and
// updates p twice: p_{k+1} = p_k + d_{k+1} y_{k+1} and p_{k+2} = p_{k+1} +
// d_{k+2} y_{k+2}.  Per point and pair of terms: read y_k, the fields and
// p_k, write y_{k+2} and p_{k+2} (56 B in FP64 instead of 2 x 56 B); p_{k+1}
// is stored only by a replay of the launch (A.replay), when the sweep
// stopped at term k+1.  Frame positions outside a
// Dirichlet grid hold zero; periodic frames are computed from wrapped loads.
// Stage 2 reads y_{k+1} from LDS rounded to the y storage type, exactly as
// the one-term kernel would read it back; p and the norms use it unrounded.
// ---------------------------------------------------------------------------

// What stage 2 of an output row j needs again from its stage-1 loads: the
// face coefficients of the nine-point stencil at row j (0.5 (kxx_C + kxx_E)
// etc., kxy at the four neighbours, the advection face values) and p_k, kept
// in registers across the block barrier.
template <int VEC>
struct Kept {
  double fE[VEC], fW[VEC], fN[VEC], fS[VEC];
  double mE[VEC], mW[VEC], mN[VEC], mS[VEC];
  double aE[VEC], aW[VEC], aN[VEC], aS[VEC];
  double pk[VEC];
};

// (A x) at row j from the kept coefficients and rows j-1, j, j+1 of x
// (the operation order of stencil_point)
template <int VEC, bool ADVF>
__device__ __forceinline__ void stencil_kept(const Kept<VEC>& kp, const RowN<VEC>& um, const RowN<VEC>& uc,
                                             const RowN<VEC>& up, double axc, double ayc, double (&Ax)[VEC]) {
#pragma unroll
  for (int v = 0; v < VEC; ++v) {
    const double uC = uc.at(v), uW = uc.west(v), uE = uc.east(v);
    const double uN = up.at(v), uS = um.at(v);
    const double uNW = up.west(v), uNE = up.east(v);
    const double uSW = um.west(v), uSE = um.east(v);
    double a = kp.fE[v] * (uE - uC) - kp.fW[v] * (uC - uW);
    a += kp.fN[v] * (uN - uC) - kp.fS[v] * (uC - uS);
    a += kp.mE[v] * (uNE - uSE) - kp.mW[v] * (uNW - uSW);
    a += kp.mN[v] * (uNE - uNW) - kp.mS[v] * (uSE - uSW);
    if constexpr (ADVF) {
      a += kp.aE[v] * uE - kp.aW[v] * uW + kp.aN[v] * uN - kp.aS[v] * uS;
    } else {
      a += axc * (uE - uW) + ayc * (uN - uS);
    }
    Ax[v] = a;
  }
}

// Stage 1 of an output row j (wave-uniform): y_{k+1} at row j into the LDS
// ring, keeping the face coefficients and p_k.  Returns false when the gate
// is closed.
template <typename TF, typename TY, int VEC, bool ADVF, bool NT>
__device__ __forceinline__ bool stage1_own(const FieldView& F, const TY* __restrict__ yin, Stage1Ep<VEC>& ep,
                                           const Strip& g, int j, const double* __restrict__ pin, bool own,
                                           Kept<VEC>& kp) {
  const TF* __restrict__ kxx = reinterpret_cast<const TF*>(F.kxx);
  const TF* __restrict__ kxy = reinterpret_cast<const TF*>(F.kxy);
  const TF* __restrict__ kyy = reinterpret_cast<const TF*>(F.kyy);
  const TF* __restrict__ fax = reinterpret_cast<const TF*>(F.ax);
  const TF* __restrict__ fay = reinterpret_cast<const TF*>(F.ay);
  RowN<VEC> u[3], m[3], k, ac;
  RowC<VEC> gg[3], ay[3];
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    row_n<TY, VEC, MODE_ZERO>(yin, j - 1 + t, F, g, u[t]);
    row_c<TF, VEC, MODE_EDGE>(kyy, j - 1 + t, F, g, gg[t]);
    row_n<TF, VEC, MODE_ZERO>(kxy, j - 1 + t, F, g, m[t]);
    if constexpr (ADVF) row_c<TF, VEC, MODE_ZERO>(fay, j - 1 + t, F, g, ay[t]);
  }
  row_n<TF, VEC, MODE_EDGE>(kxx, j, F, g, k);
  if constexpr (ADVF) row_n<TF, VEC, MODE_ZERO>(fax, j, F, g, ac);
  if (own) ldr_s<NT, double, VEC>(pin + (long)j * F.nx, g.col0, kp.pk);
  if (!ep.go()) return false;
#pragma unroll
  for (int v = 0; v < VEC; ++v) {
    const double kC = k.at(v), kW = k.west(v), kE = k.east(v);
    const double gC = gg[1].c[v], gN = gg[2].c[v], gS = gg[0].c[v];
    kp.fE[v] = 0.5 * (kC + kE);
    kp.fW[v] = 0.5 * (kC + kW);
    kp.fN[v] = 0.5 * (gC + gN);
    kp.fS[v] = 0.5 * (gC + gS);
    kp.mE[v] = m[1].east(v);
    kp.mW[v] = m[1].west(v);
    kp.mN[v] = m[2].at(v);
    kp.mS[v] = m[0].at(v);
    if constexpr (ADVF) {
      kp.aE[v] = ac.east(v);
      kp.aW[v] = ac.west(v);
      kp.aN[v] = ay[2].c[v];
      kp.aS[v] = ay[0].c[v];
    }
  }
  double Ax[VEC];
  stencil_kept<VEC, ADVF>(kp, u[0], u[1], u[2], F.axc, F.ayc, Ax);
  typename Stage1Ep<VEC>::Extra none;
  ep.finish(j, g, Ax, u[1].c, none);
  return true;
}

// The block marches down its run of row bands, kWavesY2 output rows per
// step: stage 1 of a step computes the step's own rows (keeping their fields)
// and the frame row below them into the LDS ring; the frame row above is the
// previous step's last own row, already in the ring (a prologue computes it
// for the first step).  The frame row below is computed again as the next
// step's first own row, from input rows this CU has just read.
template <typename TF, typename TY, int VEC, bool ADVF, bool NT>
__global__ __launch_bounds__(kTileBlock2) void leja2_kernel(FieldView F, Tiling T, LejaArgs A) {
  extern __shared__ double lds[];
  const int L = A.decide_only ? 0 : xcd_contiguous(blockIdx.x, gridDim.x);  // as in leja_kernel
  if (L == 0) {
    if (!A.replay) leja_decide(A);
    return;
  }
  const int b = L - 1;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & (kWave - 1);
  const int W = kWave * VEC;
  const TY* __restrict__ yin = reinterpret_cast<const TY*>(A.yin);
  TY* __restrict__ yout = reinterpret_cast<TY*>(A.yout);
  Stage1Ep<VEC> ep1;
  ep1.lds = lds;
  ep1.ny = F.ny;
  ep1.per = F.bc == BC_PERIODIC;
  ep1.shift = A.shift;
  ep1.invg = A.invg;
  ep1.stopflag = A.replay ? 0 : __hip_atomic_load(&A.ctl->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};  // term k+1: ||d y||^2, ||p||^2; term k+2: the same
  bool live = true;
  const int cb = b % T.ncb;
  const int rb0 = (b / T.ncb) * T.bands;
  const int rb1 = min(rb0 + T.bands, T.nrb);
  const Strip g = strip_at<VEC>(F, cb * (kWave - 2) * VEC - VEC);
  const bool own = lane >= 1 && lane <= kWave - 2 && g.inside;
  const int J0 = rb0 * kWavesY2;
  ep1.r0 = J0 - 1;
  // prologue: the frame row above the run
  constexpr int wfr = kWavesY2 / 2;  // the wave that computes frame rows
  if (wave == wfr - 1) live = stencil_group<TF, TY, VEC, ADVF, 1>(F, yin, ep1, g, J0 - 1);
#pragma unroll 1
  for (int rb = rb0; rb < rb1; ++rb) {
    // own row j = j0 + wave; the frame row below (j0 + kWavesY2) first, so
    // that no kept registers are live during it
    const int j0 = rb * kWavesY2;
    const int j = j0 + wave;
    const bool has = wave < kWavesY2 && j < F.ny;
    const int below = min(j0 + kWavesY2, F.ny);
    if (live && wave == wfr) live = stencil_group<TF, TY, VEC, ADVF, 1>(F, yin, ep1, g, below);
    Kept<VEC> kp;
    if (live && has) live = stage1_own<TF, TY, VEC, ADVF, NT>(F, yin, ep1, g, j, A.pin, own, kp);
    __syncthreads();
    if (live && has) {
      RowN<VEC> u[3];
#pragma unroll
      for (int t = 0; t < 3; ++t) lds_row_n<TY, VEC>(lds, (j - 1 + t - ep1.r0) & (kRing - 1), u[t]);
      double Ax[VEC];
      stencil_kept<VEC, ADVF>(kp, u[0], u[1], u[2], F.axc, F.ayc, Ax);
      if (own) {
        const long ro = (long)j * F.nx;
        const double* y1row = lds + (long)((j - ep1.r0) & (kRing - 1)) * W + lane * VEC;
        double y2[VEC], pm[VEC], p2[VEC];
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          const double t1 = A.dk1 * y1row[v];
          pm[v] = kp.pk[v] + t1;
          y2[v] = (Ax[v] - A.shift2 * u[1].c[v]) * A.invg;
          const double t2 = A.dk2 * y2[v];
          p2[v] = pm[v] + t2;
          acc[0] += t1 * t1;
          acc[1] += pm[v] * pm[v];
          acc[2] += t2 * t2;
          acc[3] += p2[v] * p2[v];
        }
        if (yout) str_s<NT, TY, VEC>(yout + ro, g.col0, y2);
        if (A.pmid) str_s<NT, double, VEC>(A.pmid + ro, g.col0, pm);
        if (A.p) str_s<NT, double, VEC>(A.p + ro, g.col0, p2);
      }
    }
    __syncthreads();
  }
  // block partials: term k+1 at (0, 1, 2), term k+2 at (3, 4, 5)
  block_allreduce<4, 4>(acc);
  if (threadIdx.x == 0 && !A.replay) {
    double* part = A.partials + (long)A.slot * A.slot_stride;
    const int nb = T.nblocks;
    part[0L * nb + b] = acc[0];
    part[1L * nb + b] = acc[1];
    part[2L * nb + b] = 0.0;
    part[3L * nb + b] = acc[2];
    part[4L * nb + b] = acc[3];
    part[5L * nb + b] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// Four Newton-Leja terms per launch (k >= 1), for grids of up to 2^20 points:
// there a two-term launch is mostly fixed cost (measured on MI355X, FP64:
// 5.8 us at 256^2, 8.5 us at 512^2, 16 us at 768^2), which four terms share
// out twice as far.  A block owns kR4 output rows of a strip of 56*VEC
// output columns (lanes 4..59 of a wave strip that starts 4*VEC columns to
// the left).  Stage 1 computes y_{k+1} on the kQ4 = kR4 + 6 rows around them
// from memory into an LDS ring; stage t = 2, 3 computes y_{k+t} on two rows
// fewer from the other ring (x-neighbours by the DPP shifts, so each stage
// leaves one more lane per side invalid: the four frame lanes); stage 4
// computes y_{k+4} on the output rows.  Stage 1 also keeps the centre field
// row of each row it computes in LDS, so that stages 2-4 read no memory
// (LF; 75 KB of LDS per block in FP64, two blocks per CU); the other form
// (LF false: the later stages read the field rows again from memory, 32 KB
// per block) measured slower on every grid once the LDS rows were accessed
// 16 bytes per lane, and the host no longer picks it.  Each wave keeps p of
// its output rows in registers and updates it after every stage:
// p_{k+t} = p_{k+t-1} + d_{k+t} y_{k+t}; p_{k+4} is written with y_{k+4}, and
// p_{k+t} for t < 4 only by a replay of the launch (A.replay), when the
// sweep stopped at term k+t.  Rows and
// columns outside a Dirichlet grid hold zero at every stage; periodic ones are
// computed from wrapped field rows.  Stages read y from LDS rounded to the y
// storage type, as a one-term launch reads it back from memory; p and the
// norms use it unrounded.
// ---------------------------------------------------------------------------
#ifndef ADL_WAVES4
#define ADL_WAVES4 4
#endif
constexpr int kT4 = 4;                    // terms per launch
constexpr int kR4 = 8;                    // output rows per block
constexpr int kQ4 = kR4 + 2 * (kT4 - 1);  // stage-1 rows per block
constexpr int kRing4 = 16;                // rows of each LDS ring
constexpr int kW4 = ADL_WAVES4;           // waves per block
constexpr int kOW4 = (kR4 + kW4 - 1) / kW4;  // output rows per wave
static_assert(kQ4 <= kRing4, "ring rows");
// stage 1 loads rows J0 - kT4 .. J0 + kR4 - 1 + kT4 (the host's periodic
// row check, four_term_rows_fit, assumes this geometry)
static_assert(kR4 == kFourTermRows && kT4 == kFourTermTerms, "four-term geometry");

// Field rows kept in LDS for stages 2-4: stage 1 stores the centre row of
// each field it loads (after the row rule: edge rows for kxx and kyy, zero
// rows for kxy and the advection fields), kQ4 rows per field; a later stage
// takes the x-neighbours by DPP and applies the Dirichlet ghost-column
// selects of the register path (lanes 0 and 63, whose halo element is not
// kept, are frame lanes by then)
template <bool ADVF>
constexpr int kNF4 = ADVF ? 5 : 3;  // kxx, kxy, kyy (, ax', ay')
template <int VEC>
__device__ __forceinline__ double* fld_row(double* flds, int f, int q) {
  return flds + ((long)f * kQ4 + q) * (kWave * VEC) + (threadIdx.x & (kWave - 1)) * VEC;
}
// (all LDS rows of the four-term kernel are accessed with one aligned
// 16-byte access per lane at two columns per lane: two 8-byte accesses at a
// 16-byte lane stride made bank-conflict cycles 1.8x the active LDS cycles)
// y row q of a ring (rounded to the storage type) with its x-neighbours
template <typename TY, int VEC>
__device__ __forceinline__ void ring4_row_n(const double* ring, int q, RowN<VEC>& o) {
  double c[VEC];
  lds_get<VEC>(ring + (long)q * (kWave * VEC) + (threadIdx.x & (kWave - 1)) * VEC, c);
#pragma unroll
  for (int v = 0; v < VEC; ++v) o.c[v] = storage_round<TY>(c[v]);
  o.l = dpp_f64<kDppWaveShr1>(o.c[VEC - 1]);
  o.r = dpp_f64<kDppWaveShl1>(o.c[0]);
}
template <int VEC, int MODE>
__device__ __forceinline__ void lds_field_n(double* flds, int f, int q, const Strip& g, RowN<VEC>& o) {
  lds_get<VEC>(fld_row<VEC>(flds, f, q), o.c);
  const double l = dpp_f64<kDppWaveShr1>(o.c[VEC - 1]);
  const double rr = dpp_f64<kDppWaveShl1>(o.c[0]);
  const double gl = MODE == MODE_EDGE ? o.c[0] : 0.0;
  const double gr = MODE == MODE_EDGE ? o.c[VEC - 1] : 0.0;
  o.l = g.ghostL ? gl : l;
  o.r = g.ghostR ? gr : rr;
}
template <int VEC>
__device__ __forceinline__ void lds_field_c(double* flds, int f, int q, RowC<VEC>& o) {
  lds_get<VEC>(fld_row<VEC>(flds, f, q), o.c);
}

// Stage 1 at grid row r (ring row q): y_{k+1} from memory into `out`, as
// the one-term kernel computes it, and the centre field rows into flds
template <typename TF, typename TY, int VEC, bool ADVF>
__device__ __forceinline__ void stage1_row4(const FieldView& F, const TY* __restrict__ yin, const Strip& g,
                                            double* out, double* flds, int q, int r, double shift, double invg) {
  const TF* __restrict__ kxx = reinterpret_cast<const TF*>(F.kxx);
  const TF* __restrict__ kxy = reinterpret_cast<const TF*>(F.kxy);
  const TF* __restrict__ kyy = reinterpret_cast<const TF*>(F.kyy);
  const TF* __restrict__ fax = reinterpret_cast<const TF*>(F.ax);
  const TF* __restrict__ fay = reinterpret_cast<const TF*>(F.ay);
  RowN<VEC> u[3], m[3], k, ac;
  RowC<VEC> gg[3], ay[3];
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    row_n<TY, VEC, MODE_ZERO>(yin, r - 1 + t, F, g, u[t]);
    row_c<TF, VEC, MODE_EDGE>(kyy, r - 1 + t, F, g, gg[t]);
    row_n<TF, VEC, MODE_ZERO>(kxy, r - 1 + t, F, g, m[t]);
    if constexpr (ADVF) row_c<TF, VEC, MODE_ZERO>(fay, r - 1 + t, F, g, ay[t]);
  }
  row_n<TF, VEC, MODE_EDGE>(kxx, r, F, g, k);
  if constexpr (ADVF) row_n<TF, VEC, MODE_ZERO>(fax, r, F, g, ac);
  double Ax[VEC];
  stencil_point<VEC, ADVF>(u[0], u[1], u[2], gg[0], gg[1], gg[2], m[0], m[1], m[2], k, ac, ay[0], ay[2], F.axc,
                           F.ayc, Ax);
  const bool ghost = F.bc != BC_PERIODIC && (!g.inside || r < 0 || r >= F.ny);
  double y1[VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) y1[v] = ghost ? 0.0 : (Ax[v] - shift * u[1].c[v]) * invg;
  lds_set<VEC>(out + (long)q * (kWave * VEC) + (threadIdx.x & (kWave - 1)) * VEC, y1);
  lds_set<VEC>(fld_row<VEC>(flds, 0, q), k.c);
  lds_set<VEC>(fld_row<VEC>(flds, 1, q), m[1].c);
  lds_set<VEC>(fld_row<VEC>(flds, 2, q), gg[1].c);
  if constexpr (ADVF) {
    lds_set<VEC>(fld_row<VEC>(flds, 3, q), ac.c);
    lds_set<VEC>(fld_row<VEC>(flds, 4, q), ay[1].c);
  }
}

// y_{k+t} (t >= 2) at grid row r (ring row q) from ring `in` holding y_{k+t-1}
// (rows q-1, q, q+1) and the field rows in LDS, written to ring `out` (if
// given): (A y - shift y) / gamma, or zero outside a Dirichlet grid; returns
// y_{k+t} (unrounded) in yt
template <typename TF, typename TY, int VEC, bool ADVF>
__device__ __forceinline__ void stage_from_ring(const FieldView& F, const Strip& g, const double* in, double* out,
                                                double* flds, int q, int r, double shift, double invg,
                                                double (&yt)[VEC]) {
  RowN<VEC> u[3], m[3], k, ac;
  RowC<VEC> gg[3], ay[3];
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    lds_field_c<VEC>(flds, 2, q - 1 + t, gg[t]);
    lds_field_n<VEC, MODE_ZERO>(flds, 1, q - 1 + t, g, m[t]);
    if constexpr (ADVF) lds_field_c<VEC>(flds, 4, q - 1 + t, ay[t]);
    ring4_row_n<TY, VEC>(in, q - 1 + t, u[t]);
  }
  lds_field_n<VEC, MODE_EDGE>(flds, 0, q, g, k);
  if constexpr (ADVF) lds_field_n<VEC, MODE_ZERO>(flds, 3, q, g, ac);
  double Ax[VEC];
  stencil_point<VEC, ADVF>(u[0], u[1], u[2], gg[0], gg[1], gg[2], m[0], m[1], m[2], k, ac, ay[0], ay[2], F.axc,
                           F.ayc, Ax);
  const bool ghost = F.bc != BC_PERIODIC && (!g.inside || r < 0 || r >= F.ny);
#pragma unroll
  for (int v = 0; v < VEC; ++v) yt[v] = ghost ? 0.0 : (Ax[v] - shift * u[1].c[v]) * invg;
  if (out) lds_set<VEC>(out + (long)q * (kWave * VEC) + (threadIdx.x & (kWave - 1)) * VEC, yt);
}

// The same with the field rows read again from memory (cache hits), for
// launches whose blocks would not all fit the chip at once with the LDS field
// rows (two blocks per CU)
template <typename TF, typename TY, int VEC, bool ADVF>
__device__ __forceinline__ void stage_from_ring_g(const FieldView& F, const Strip& g, const double* in, double* out,
                                                  int q, int r, double shift, double invg, double (&yt)[VEC]) {
  const TF* __restrict__ kxx = reinterpret_cast<const TF*>(F.kxx);
  const TF* __restrict__ kxy = reinterpret_cast<const TF*>(F.kxy);
  const TF* __restrict__ kyy = reinterpret_cast<const TF*>(F.kyy);
  const TF* __restrict__ fax = reinterpret_cast<const TF*>(F.ax);
  const TF* __restrict__ fay = reinterpret_cast<const TF*>(F.ay);
  RowN<VEC> u[3], m[3], k, ac;
  RowC<VEC> gg[3], ay[3];
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    row_c<TF, VEC, MODE_EDGE>(kyy, r - 1 + t, F, g, gg[t]);
    row_n<TF, VEC, MODE_ZERO>(kxy, r - 1 + t, F, g, m[t]);
    if constexpr (ADVF) row_c<TF, VEC, MODE_ZERO>(fay, r - 1 + t, F, g, ay[t]);
  }
  row_n<TF, VEC, MODE_EDGE>(kxx, r, F, g, k);
  if constexpr (ADVF) row_n<TF, VEC, MODE_ZERO>(fax, r, F, g, ac);
#pragma unroll
  for (int t = 0; t < 3; ++t) ring4_row_n<TY, VEC>(in, q - 1 + t, u[t]);
  double Ax[VEC];
  stencil_point<VEC, ADVF>(u[0], u[1], u[2], gg[0], gg[1], gg[2], m[0], m[1], m[2], k, ac, ay[0], ay[2], F.axc,
                           F.ayc, Ax);
  const bool ghost = F.bc != BC_PERIODIC && (!g.inside || r < 0 || r >= F.ny);
#pragma unroll
  for (int v = 0; v < VEC; ++v) yt[v] = ghost ? 0.0 : (Ax[v] - shift * u[1].c[v]) * invg;
  if (out) lds_set<VEC>(out + (long)q * (kWave * VEC) + (threadIdx.x & (kWave - 1)) * VEC, yt);
}

// stage t >= 2 from the LDS field rows (LF) or from memory
template <bool LF, typename TF, typename TY, int VEC, bool ADVF>
__device__ __forceinline__ void stage_t(const FieldView& F, const Strip& g, const double* in, double* out,
                                        double* flds, int q, int r, double shift, double invg, double (&yt)[VEC]) {
  if constexpr (LF) stage_from_ring<TF, TY, VEC, ADVF>(F, g, in, out, flds, q, r, shift, invg, yt);
  else stage_from_ring_g<TF, TY, VEC, ADVF>(F, g, in, out, q, r, shift, invg, yt);
}

template <bool LF, typename TF, typename TY, int VEC, bool ADVF>
__global__ __launch_bounds__(kWave * kW4) void leja4_kernel(FieldView F, Tiling T, LejaArgs A) {
  extern __shared__ __attribute__((aligned(16))) double lds[];  // rows accessed 16 bytes per lane
  // XCD-contiguous logical blocks (row-major: column block fastest): the
  // blocks above and below a block, which load half of its rows again, run
  // on the same XCD and find those rows in its L2
  const int L = A.decide_only ? 0 : xcd_contiguous(blockIdx.x, gridDim.x);
  if (L == 0) {
    if (!A.replay) leja_decide(A);
    return;
  }
  if (!A.replay && block_stopped(A.ctl)) return;  // uniform over the block
  const int b = L - 1;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & (kWave - 1);
  const int W = kWave * VEC;
  double* ringA = lds;
  double* ringB = lds + kRing4 * W;
  double* flds = lds + 2 * kRing4 * W;  // kNF4<ADVF> fields x kQ4 rows
  const TY* __restrict__ yin = reinterpret_cast<const TY*>(A.yin);
  TY* __restrict__ yout = reinterpret_cast<TY*>(A.yout);
  const int cb = b % T.ncb;
  const int J0 = (b / T.ncb) * kR4;      // first output row
  const int r0 = J0 - (kT4 - 1);          // grid row of ring row 0
  const Strip g = strip_at<VEC>(F, cb * (kWave - 2 * kT4) * VEC - kT4 * VEC);
  const bool own = lane >= kT4 && lane < kWave - kT4 && g.inside;
  // the wave's output rows o = wave + h kW4 < kR4 (ring rows o + 3)
  int jo[kOW4];
  bool ho[kOW4];
  double pk[kOW4][VEC];
#pragma unroll
  for (int h = 0; h < kOW4; ++h) {
    jo[h] = J0 + wave + h * kW4;
    ho[h] = own && wave + h * kW4 < kR4 && jo[h] < F.ny;
    if (ho[h]) ldr_s<false, double, VEC>(A.pin + (long)jo[h] * F.nx, g.col0, pk[h]);
  }
  double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  // p_{k+t} of the output rows from y_{k+t} in ring `rg`, stored to dst;
  // tn / pn accumulate the term's ||d y||^2 and ||p||^2
  auto update_p = [&](const double* rg, double d, double& tn, double& pn, double* dst) {
#pragma unroll
    for (int h = 0; h < kOW4; ++h) {
      if (ho[h]) {
        double yr[VEC];
        lds_get<VEC>(rg + (long)(jo[h] - r0) * W + lane * VEC, yr);
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          const double tv = d * yr[v];
          pk[h][v] += tv;
          tn += tv * tv;
          pn += pk[h][v] * pk[h][v];
        }
        if (dst) str_s<false, double, VEC>(dst + (long)jo[h] * F.nx, g.col0, pk[h]);
      }
    }
  };
  // stage 1: y_{k+1} on ring rows 0 .. kQ4-1 from memory (and the field rows
  // into LDS)
  if constexpr (LF) {
#pragma unroll 1
    for (int q = wave; q < kQ4; q += kW4)
      stage1_row4<TF, TY, VEC, ADVF>(F, yin, g, ringA, flds, q, r0 + q, A.shift, A.invg);
  } else {
    Stage1Ep<VEC, kRing4> ep1;
    ep1.lds = ringA;
    ep1.r0 = r0;
    ep1.ny = F.ny;
    ep1.per = F.bc == BC_PERIODIC;
    ep1.shift = A.shift;
    ep1.invg = A.invg;
    ep1.stopflag = 0;
#pragma unroll 1
    for (int q = wave; q < kQ4; q += kW4) stencil_group<TF, TY, VEC, ADVF, 1>(F, yin, ep1, g, r0 + q);
  }
  __syncthreads();
  update_p(ringA, A.dk1, acc[0], acc[1], A.pmid);
  // stage 2: ring rows 1 .. kQ4-2, A -> B
  double yt[VEC];
#pragma unroll 1
  for (int q = 1 + wave; q < kQ4 - 1; q += kW4)
    stage_t<LF, TF, TY, VEC, ADVF>(F, g, ringA, ringB, flds, q, r0 + q, A.shift2, A.invg, yt);
  __syncthreads();
  update_p(ringB, A.dk2, acc[2], acc[3], A.pmid2);
  // stage 3: ring rows 2 .. kQ4-3, B -> A (stage 2 and the p update have
  // finished reading A at the barrier above)
#pragma unroll 1
  for (int q = 2 + wave; q < kQ4 - 2; q += kW4)
    stage_t<LF, TF, TY, VEC, ADVF>(F, g, ringB, ringA, flds, q, r0 + q, A.shift3, A.invg, yt);
  __syncthreads();
  update_p(ringA, A.dk3, acc[4], acc[5], A.pmid3);
  // stage 4: the wave's own output rows from A, in registers
#pragma unroll
  for (int h = 0; h < kOW4; ++h) {
    if (wave + h * kW4 >= kR4) continue;  // wave-uniform
    const int q = jo[h] - r0;
    stage_t<LF, TF, TY, VEC, ADVF>(F, g, ringA, nullptr, flds, q, jo[h], A.shift4, A.invg, yt);
    if (ho[h]) {
      const long ro = (long)jo[h] * F.nx;
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        const double tv = A.dk4 * yt[v];
        pk[h][v] += tv;
        acc[6] += tv * tv;
        acc[7] += pk[h][v] * pk[h][v];
      }
      if (yout) str_s<false, TY, VEC>(yout + ro, g.col0, yt);
      if (A.p) str_s<false, double, VEC>(A.p + ro, g.col0, pk[h]);
    }
  }
  // block partials: term t at rows 3t (||d y||^2), 3t + 1 (||p||^2), 3t + 2 (0)
  block_allreduce<8, 8>(acc);
  if (threadIdx.x == 0 && !A.replay) {
    double* part = A.partials + (long)A.slot * A.slot_stride;
    const int nb = T.nblocks;
#pragma unroll
    for (int t = 0; t < kT4; ++t) {
      part[(3L * t) * nb + b] = acc[2 * t];
      part[(3L * t + 1) * nb + b] = acc[2 * t + 1];
      part[(3L * t + 2) * nb + b] = 0.0;
    }
  }
}

template <typename TF, typename TY, int VEC, bool ADVF, bool NT>
__global__ __launch_bounds__(kTileBlock2) void leja2s_kernel(FieldView F, Tiling T, LejaArgs A) {
  extern __shared__ double lds[];
  const int L = A.decide_only ? 0 : xcd_contiguous(blockIdx.x, gridDim.x);
  if (L == 0) {
    if (!A.replay) leja_decide(A);
    return;
  }
  const int b = L - 1;
  const int cb = b % T.ncb;
  const int rb0 = (b / T.ncb) * T.bands;
  const int rb1 = min(rb0 + T.bands, T.nrb);
  StagedIO<TY> io;
  io.yin = reinterpret_cast<const TY*>(A.yin);
  io.yout = reinterpret_cast<TY*>(A.yout);
  io.pin = A.pin;
  io.pmid = A.pmid;
  io.p = A.p;
  io.shift = A.shift;
  io.shift2 = A.shift2;
  io.invg = A.invg;
  io.dk1 = A.dk1;
  io.dk2 = A.dk2;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  staged_run<TF, TY, VEC, ADVF, NT>(
      F, io, lds, cb * (kWave - 2) * VEC - VEC, rb0, rb1,
      A.replay ? 0 : __hip_atomic_load(&A.ctl->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), acc);
  // block partials: term k+1 at (0, 1, 2), term k+2 at (3, 4, 5)
  block_allreduce<4, 4>(acc);
  if (threadIdx.x == 0 && !A.replay) {
    double* part = A.partials + (long)A.slot * A.slot_stride;
    const int nb = T.nblocks;
    part[0L * nb + b] = acc[0];
    part[1L * nb + b] = acc[1];
    part[2L * nb + b] = 0.0;
    part[3L * nb + b] = acc[2];
    part[4L * nb + b] = acc[3];
    part[5L * nb + b] = 0.0;
  }
}

// Three Newton terms per launch with the input rows staged in LDS
// (staged3_run in staged.h), on its own tiling of strips of 62*VEC output
// columns with two columns per lane (the strips of leja2s_kernel, fewer and
// longer runs).  FIRST: the sweep's first launch, terms 1 .. 3 from y_0 = v
// in FP64 (no augmented column among them): block 0 clears the control
// block instead of deciding, p_0 = d_0 y_0 is formed in the march, and the
// first term's third partial row holds max |y_0| (the zero-vector test).
template <typename TF, typename TY, bool ADVF, bool NT, bool FIRST>
__global__ __launch_bounds__(kTileBlock2) void leja3s_kernel(FieldView F, Tiling T, LejaArgs A) {
  extern __shared__ __attribute__((aligned(16))) double lds[];  // rows accessed 16 bytes per lane
  constexpr int VEC = 2;
  const int L = A.decide_only ? 0 : xcd_contiguous(blockIdx.x, gridDim.x);
  if (L == 0) {
    if (FIRST) {
      // a new sweep: clear the control block (no block of this launch reads it)
      if (!A.replay && threadIdx.x == 0) {
        Ctl c{};
        *A.ctl = c;
      }
    } else if (!A.replay) {
      leja_decide(A);
    }
    return;
  }
  const int b = L - 1;
  const int cb = b % T.ncb;
  const int rb0 = (b / T.ncb) * T.bands;
  const int rb1 = min(rb0 + T.bands, T.nrb);
  Staged3IO<TY> io;
  io.yin = reinterpret_cast<const TY*>(A.yin);
  io.yout = reinterpret_cast<TY*>(A.yout);
  // (the first launch reads no p_k: p_0 = d_0 y_0 is formed in the march;
  // its pin is only the base of the stores it drops)
  io.pin = FIRST ? reinterpret_cast<const double*>(A.yin) : A.pin;
  io.p1 = A.pmid;
  io.p2 = A.pmid2;
  io.p = A.p;
  io.y2out = nullptr;
  io.shift = A.shift;
  io.shift2 = A.shift2;
  io.shift3 = A.shift3;
  io.invg = A.invg;
  io.dk1 = A.dk1;
  io.dk2 = A.dk2;
  io.dk3 = A.dk3;
  io.d0 = A.d0;
  double acc[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double (&acc6)[6] = *reinterpret_cast<double(*)[6]>(acc);
  staged3_run<TF, TY, VEC, ADVF, NT, false, FIRST>(
      F, io, lds, cb * (kWave - 2) * VEC - VEC, rb0, rb1,
      (FIRST || A.replay) ? 0 : __hip_atomic_load(&A.ctl->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), acc6,
      acc[6]);
  // block partials: term t (0, 1, 2) at rows 3t (||d y||^2), 3t + 1 (||p||^2),
  // 3t + 2 (0; for the first term of a first launch max |y_0|, the zero test)
  block_allreduce<7, 6>(acc);
  if (threadIdx.x == 0 && !A.replay) {
    double* part = A.partials + (long)A.slot * A.slot_stride;
    const int nb = T.nblocks;
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      part[(3L * t) * nb + b] = acc[2 * t];
      part[(3L * t + 1) * nb + b] = acc[2 * t + 1];
      part[(3L * t + 2) * nb + b] = t == 0 ? acc[6] : 0.0;
    }
  }
}

// Four Newton terms per launch (k >= 1) with the input rows staged in LDS
// (staged4_run in staged.h), on its own tiling of strips of 60*VEC output
// columns with two columns per lane.  No static LDS (the block reductions
// use the dynamic rings), so that three blocks share a CU.
template <typename TF, typename TY, bool ADVF, bool NT, bool STAGE>
__global__ __launch_bounds__(kTileBlock2) void leja4s_kernel(FieldView F, Tiling T, LejaArgs A) {
  extern __shared__ __attribute__((aligned(16))) double lds[];  // rows accessed 16 bytes per lane
  constexpr int VEC = 2;
  const int L = A.decide_only ? 0 : xcd_contiguous(blockIdx.x, gridDim.x);
  if (L == 0) {
    if (STAGE) {
      // a new sweep: clear the control block (no block of this launch reads it)
      if (!A.replay && threadIdx.x == 0) {
        Ctl c{};
        *A.ctl = c;
      }
    } else if (!A.replay) {
      leja_decide<true>(A, lds);
    }
    return;
  }
  const int b = L - 1;
  const int cb = b % T.ncb;
  const int rb0 = (b / T.ncb) * T.bands;
  const int rb1 = min(rb0 + T.bands, T.nrb);
  Staged4IO<TY> io;
  io.yin = reinterpret_cast<const TY*>(A.yin);
  io.yout = reinterpret_cast<TY*>(A.yout);
  io.pin = A.pin;
  io.p1 = A.pmid;
  io.p2 = A.pmid2;
  io.p3 = A.pmid3;
  io.p = A.p;
  io.src = A.src;
  io.shift = A.shift;
  io.shift2 = A.shift2;
  io.shift3 = A.shift3;
  io.shift4 = A.shift4;
  io.invg = A.invg;
  io.dk1 = A.dk1;
  io.dk2 = A.dk2;
  io.dk3 = A.dk3;
  io.dk4 = A.dk4;
  double acc[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double (&acc8)[8] = *reinterpret_cast<double(*)[8]>(acc);
  staged4_run<TF, TY, VEC, ADVF, NT, STAGE>(
      F, io, lds, cb * (kWave - 4) * VEC - 2 * VEC, rb0, rb1,
      (STAGE || A.replay) ? 0 : __hip_atomic_load(&A.ctl->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), acc8,
      acc[8]);
  // block partials: term t (0 .. 3) at rows 3t (||d y||^2), 3t + 1 (||p||^2),
  // 3t + 2 (0); STAGE: the launch's three terms are stages 2 .. 4, and row 2
  // holds max |w| (the first-term zero test)
  __syncthreads();  // (the rings are free again: the reduction's scratch)
  block_allreduce_at<9, 8>(acc, lds);
  if (threadIdx.x == 0 && !A.replay) {
    double* part = A.partials + (long)A.slot * A.slot_stride;
    const int nb = T.nblocks;
    constexpr int first = STAGE ? 1 : 0, nt = STAGE ? 3 : 4;
#pragma unroll
    for (int t = 0; t < nt; ++t) {
      part[(3L * t) * nb + b] = acc[2 * (t + first)];
      part[(3L * t + 1) * nb + b] = acc[2 * (t + first) + 1];
      part[(3L * t + 2) * nb + b] = (STAGE && t == 0) ? acc[8] : 0.0;
    }
  }
}

// Power iteration term: w_{k+1} = A(w_k) / lambda_k, lambda_k = ||w_k|| from
// the partials of the launch that wrote w_k.
template <int VEC>
struct PowerEp {
  struct Extra {};
  int nx;
  double* __restrict__ w;
  double scale;
  double acc[1];
  __device__ __forceinline__ bool go() const { return true; }
  __device__ __forceinline__ void load(int, const Strip&, Extra&) {}
  __device__ __forceinline__ void finish(int j, const Strip& g, const double (&Ax)[VEC], const double (&)[VEC],
                                         const Extra&) {
    if (!g.inside) return;
    double r[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      r[v] = Ax[v] * scale;
      acc[0] += r[v] * r[v];
    }
    str<double, VEC>(w + (long)j * nx, g.col0, r);
  }
};

// Partials of power launch k live in slot k mod 3; the start vector's in slot 2.
// At the start of launch k (k >= 1) lambda_k = ||w_k|| is tested against
// lambda_{k-1} (0 for k = 1), the test of iteration k of the power method.
template <typename TF, int VEC, bool ADVF>
__global__ __launch_bounds__(kTileBlock) void power_kernel(FieldView F, Tiling T, PowerArgs P) {
  Ctl* ctl = P.ctl;
  if (block_stopped(ctl)) return;
  const int k = P.k;
  const long slot = (long)P.nb;
  double t1[1];
  partial_totals<1, 1>(P.partials + ((k + 2) % 3) * slot, P.nb, t1);
  const double lam = sqrt(t1[0]);
  if (k >= 1) {
    double lam_prev = 0.0;
    if (k >= 2) {
      double t0[1];
      partial_totals<1, 1>(P.partials + ((k + 1) % 3) * slot, P.nb, t0);
      lam_prev = sqrt(t0[0]);
    }
    int stop = 0, status = 0;
    if (!isfinite(lam)) {
      stop = 1; status = 2;
    } else if (lam == 0.0) {
      stop = 1; status = 1;
    } else if (fabs(lam - lam_prev) <= P.rtol * lam) {
      stop = 1; status = 1;
    } else if (k >= P.max_iter) {
      stop = 1; status = 3;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      ctl->lam = lam;
      ctl->lam_prev = lam_prev;
      ctl->iters = k;
      ctl->status = status;
      __hip_atomic_store(&ctl->stop, stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (stop) return;
  }
  if (P.decide_only) return;
  PowerEp<VEC> ep;
  ep.nx = F.nx;
  ep.w = P.w;
  ep.scale = lam > 0.0 ? 1.0 / lam : 0.0;
  ep.acc[0] = 0.0;
  stencil_block<TF, double, VEC, ADVF>(F, T, P.x, ep, blockIdx.x);
  write_partials<1, 1>(ep.acc, P.partials + (k % 3) * slot, gridDim.x, blockIdx.x);
}

// splitmix64 output k of the stream seeded with s (Steele, Lea, Flood 2014):
// z = s + (k+1) * golden; two xor-shift-multiply rounds; final xor-shift.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Start vector w_0 = uniform(-1, 1) (splitmix64); its partial norms go to slot 2.
__global__ __launch_bounds__(kBlock) void power_init_kernel(long n, uint64_t seed, double* __restrict__ w,
                                                            double* __restrict__ partials) {
  double acc[1] = {0.0};
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const uint64_t z = splitmix64_at(seed, (uint64_t)i);
    const double u = 2.0 * (double)(z >> 11) * 0x1.0p-53 - 1.0;
    w[i] = u;
    acc[0] += u * u;
  }
  write_partials<1, 1>(acc, partials + 2L * gridDim.x, gridDim.x, blockIdx.x);
}

// Gershgorin: min over rows of A_ii - sum_{j != i} |A_ij| (one thread per node).
template <typename TF, bool ADVF>
__global__ __launch_bounds__(kBlock) void gershgorin_kernel(FieldView F, double* partials, Ctl* ctl) {
  gershgorin_blocks<TF, ADVF>(F, partials, ctl, (int)gridDim.x, (int)blockIdx.x, nullptr);
}

// ---------------------------------------------------------------------------
// Elementwise kernels
// ---------------------------------------------------------------------------
__global__ void ctl_reset_kernel(Ctl* ctl, int n) {
  const int i = threadIdx.x;
  if (i < n) {
    Ctl c{};
    ctl[i] = c;
  }
}

__global__ __launch_bounds__(kBlock) void axpby_kernel(long n, double* y, double a, const double* x, double b,
                                                       const double* z) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    double r = a * x[i];
    if (z) r += b * z[i];
    y[i] = r;
  }
}

__global__ __launch_bounds__(kBlock) void diff_scale_kernel(long n, double* y, const double* x, const double* z,
                                                            double s) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const double d = x[i] - z[i];
    y[i] = d * s;
  }
}

__global__ __launch_bounds__(kBlock) void fill_kernel(long n, double* y, double v) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) y[i] = v;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void prepare_kernel(long n, const double* __restrict__ in, double scale,
                                                         T* __restrict__ out) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    out[i] = (T)(in[i] * scale);
}

// ---------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------
Tiling make_tiling(int nx, int ny, int rows_hint, int vec_hint) {
  Tiling t;
  const bool two = nx % 2 == 0 && nx >= 2 * kWave;
  t.vec = (vec_hint == 1 || !two) ? 1 : 2;
  t.ncb = (nx + kWave * t.vec - 1) / (kWave * t.vec);
  // one row per wave unless asked otherwise (measured best on MI355X from 512^2 to 4096^2)
  int rows = rows_hint > 0 ? rows_hint : 1;
  if (rows > ny) rows = ny;
  t.rows = rows;
  const int band = kWavesY * rows;
  t.nrb = (ny + band - 1) / band;
  // bands per block: the fewest that keep the grid within kMaxGrid blocks
  const long per_strip = kMaxGrid / t.ncb > 0 ? kMaxGrid / t.ncb : 1;
  t.bands = (int)((t.nrb + per_strip - 1) / per_strip);
  t.nblocks = t.ncb * ((t.nrb + t.bands - 1) / t.bands);
  return t;
}

Tiling make_tiling2(int nx, int ny, int rows_hint, int vec_hint, int max_blocks, int frame) {
  Tiling t;
  const bool two = nx % 2 == 0 && nx >= 2 * kWave;
  t.vec = (vec_hint == 1 || !two) ? 1 : 2;
  const int wo = (kWave - 2 * frame) * t.vec;  // output columns of a strip
  t.ncb = (nx + wo - 1) / wo;
  (void)rows_hint;  // one output row per wave
  t.rows = 1;
  t.nrb = (ny + kWavesY2 - 1) / kWavesY2;
  const long per_strip = max_blocks / t.ncb > 0 ? max_blocks / t.ncb : 1;
  t.bands = (int)((t.nrb + per_strip - 1) / per_strip);
  t.nblocks = t.ncb * ((t.nrb + t.bands - 1) / t.bands);
  return t;
}

Tiling make_tiling4(int nx, int ny, int vec_hint) {
  Tiling t;
  const bool two = nx % 2 == 0 && nx >= 2 * kWave;
  t.vec = (vec_hint == 1 || !two) ? 1 : 2;
  const int wo = (kWave - 2 * kT4) * t.vec;  // output columns of a strip
  t.ncb = (nx + wo - 1) / wo;
  t.rows = kR4;
  t.nrb = (ny + kR4 - 1) / kR4;
  t.bands = 1;
  t.nblocks = t.ncb * t.nrb;
  return t;
}

static inline int ew_blocks(long n) {
  long b = (n + kBlock - 1) / kBlock;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (int)b;
}

#define ADL_DISPATCH_TILE(T, F, ...)                                  \
  do {                                                                \
    const bool advf_ = (F).ax != nullptr;                             \
    if ((T).vec == 2) {                                               \
      constexpr int VEC = 2;                                          \
      if (advf_) { constexpr bool ADVF = true; __VA_ARGS__; }         \
      else { constexpr bool ADVF = false; __VA_ARGS__; }              \
    } else {                                                          \
      constexpr int VEC = 1;                                          \
      if (advf_) { constexpr bool ADVF = true; __VA_ARGS__; }         \
      else { constexpr bool ADVF = false; __VA_ARGS__; }              \
    }                                                                 \
  } while (0)

hipError_t launch_apply2(const FieldView& f, const Tiling& t, const double* x, double* y, const double* s1,
                         double a1, const double* s2, double a2, double* y2, double d2, hipStream_t st) {
  if (y2 && (!s1 || !s2)) return hipErrorInvalidValue;
  ADL_DISPATCH_TILE(t, f, {
    ApplyEp<VEC> ep;
    ep.nx = f.nx;
    ep.out = y;
    ep.s1 = s1;
    ep.s2 = s2;
    ep.a1 = a1;
    ep.a2 = a2;
    ep.out2 = y2;
    ep.d2 = d2;
    if (f.f32)
      hipLaunchKernelGGL((apply_kernel<float, VEC, ADVF>), dim3(t.nblocks), dim3(kTileBlock), 0, st, f, t, x, ep);
    else
      hipLaunchKernelGGL((apply_kernel<double, VEC, ADVF>), dim3(t.nblocks), dim3(kTileBlock), 0, st, f, t, x, ep);
  });
  return hipGetLastError();
}

hipError_t launch_apply(const FieldView& f, const Tiling& t, const double* x, double* y, const double* s1,
                        double a1, const double* s2, double a2, hipStream_t st) {
  return launch_apply2(f, t, x, y, s1, a1, s2, a2, nullptr, 0.0, st);
}

template <typename TF, typename TYI, typename TYO, int VEC, bool ADVF, bool FIRST, bool NT>
static void leja_launch(const FieldView& f, const Tiling& t, const LejaArgs& a, hipStream_t st) {
  const dim3 grid(a.decide_only ? 1 : t.nblocks + 1), blk(kTileBlock);
  if (a.ev_start)
    hipExtLaunchKernelGGL((leja_kernel<TF, TYI, TYO, VEC, ADVF, FIRST, NT>), grid, blk, 0, st, a.ev_start,
                          a.ev_stop, 0, f, t, a);
  else
    hipLaunchKernelGGL((leja_kernel<TF, TYI, TYO, VEC, ADVF, FIRST, NT>), grid, blk, 0, st, f, t, a);
}

template <typename TF, int VEC, bool ADVF>
static void leja_dispatch_y(const FieldView& f, const Tiling& t, const LejaArgs& a, hipStream_t st) {
  const bool nt = a.stream && !a.decide_only;
  if (a.first) {  // y_0 = v, FP64
    if (a.ystore_f32) leja_launch<TF, double, float, VEC, ADVF, true, false>(f, t, a, st);
    else leja_launch<TF, double, double, VEC, ADVF, true, false>(f, t, a, st);
  } else if (a.ystore_f32) {
    if (nt) leja_launch<TF, float, float, VEC, ADVF, false, true>(f, t, a, st);
    else leja_launch<TF, float, float, VEC, ADVF, false, false>(f, t, a, st);
  } else {
    if (nt) leja_launch<TF, double, double, VEC, ADVF, false, true>(f, t, a, st);
    else leja_launch<TF, double, double, VEC, ADVF, false, false>(f, t, a, st);
  }
}

hipError_t launch_leja_step(const FieldView& f, const Tiling& t, const LejaArgs& a, hipStream_t st) {
  // later terms read y_k in the storage type and never the augmented column
  if (!a.first && (a.w2 != nullptr || a.yin_f32 != a.ystore_f32 || a.k < 1)) return hipErrorInvalidValue;
  if (!a.first && !a.decide_only && (a.pin == nullptr || a.pin == a.p)) return hipErrorInvalidValue;
  if (a.first && (a.yin_f32 || a.k != 0)) return hipErrorInvalidValue;
  ADL_DISPATCH_TILE(t, f, {
    if (f.f32) leja_dispatch_y<float, VEC, ADVF>(f, t, a, st);
    else leja_dispatch_y<double, VEC, ADVF>(f, t, a, st);
  });
  return hipGetLastError();
}

template <typename TF, typename TY, int VEC, bool ADVF, bool NT>
static void leja2_launch(const FieldView& f, const Tiling& t, const LejaArgs& a, hipStream_t st) {
  const dim3 grid(a.decide_only ? 1 : t.nblocks + 1), blk(kTileBlock2);
  const size_t lds = (size_t)kRing * kWave * VEC * sizeof(double);
  if (a.ev_start)
    hipExtLaunchKernelGGL((leja2_kernel<TF, TY, VEC, ADVF, NT>), grid, blk, lds, st, a.ev_start, a.ev_stop, 0, f, t,
                          a);
  else
    hipLaunchKernelGGL((leja2_kernel<TF, TY, VEC, ADVF, NT>), grid, blk, lds, st, f, t, a);
}

template <typename TF, typename TY, int VEC, bool ADVF, bool NT>
static void leja2s_launch(const FieldView& f, const Tiling& t, const LejaArgs& a, hipStream_t st) {
  const dim3 grid(a.decide_only ? 1 : t.nblocks + 1), blk(kTileBlock2);
  const size_t lds = staged_lds_bytes<VEC, ADVF>();
  if (a.ev_start)
    hipExtLaunchKernelGGL((leja2s_kernel<TF, TY, VEC, ADVF, NT>), grid, blk, lds, st, a.ev_start, a.ev_stop, 0, f,
                          t, a);
  else
    hipLaunchKernelGGL((leja2s_kernel<TF, TY, VEC, ADVF, NT>), grid, blk, lds, st, f, t, a);
}

template <typename TF, typename TY, int VEC, bool ADVF, bool NT>
static void leja2_any(const FieldView& f, const Tiling& t, const LejaArgs& a, hipStream_t st) {
  if (a.staged) leja2s_launch<TF, TY, VEC, ADVF, NT>(f, t, a, st);
  else leja2_launch<TF, TY, VEC, ADVF, NT>(f, t, a, st);
}

template <bool LF, typename TF, typename TY, int VEC, bool ADVF>
static void leja4_launch_lf(const FieldView& f, const Tiling& t, const LejaArgs& a, hipStream_t st) {
  const dim3 grid(a.decide_only ? 1 : t.nblocks + 1), blk(kWave * kW4);
  const size_t lds = (2 * (size_t)kRing4 + (LF ? (size_t)kNF4<ADVF> * kQ4 : 0)) * kWave * VEC * sizeof(double);
  if (a.ev_start)
    hipExtLaunchKernelGGL((leja4_kernel<LF, TF, TY, VEC, ADVF>), grid, blk, lds, st, a.ev_start, a.ev_stop, 0, f, t,
                          a);
  else
    hipLaunchKernelGGL((leja4_kernel<LF, TF, TY, VEC, ADVF>), grid, blk, lds, st, f, t, a);
}
template <typename TF, typename TY, int VEC, bool ADVF>
static void leja4_launch(const FieldView& f, const Tiling& t, const LejaArgs& a, hipStream_t st) {
  if (a.lds_fields) leja4_launch_lf<true, TF, TY, VEC, ADVF>(f, t, a, st);
  else leja4_launch_lf<false, TF, TY, VEC, ADVF>(f, t, a, st);
}

hipError_t launch_leja4_step(const FieldView& f, const Tiling& t, const LejaArgs& a, hipStream_t st) {
  if (a.first || a.k < 1 || a.nterms != kT4 || a.w2 != nullptr || a.yin_f32 != a.ystore_f32 || a.stream)
    return hipErrorInvalidValue;
  if (t.rows != kR4 || t.bands != 1 || t.nblocks != t.ncb * t.nrb) return hipErrorInvalidValue;
  if (!a.decide_only) {
    // p_k is read while the stored p outputs (at least one) are written: all distinct
    const double* o[5] = {a.pin, a.pmid, a.pmid2, a.pmid3, a.p};
    if (a.pin == nullptr || (!a.pmid && !a.pmid2 && !a.pmid3 && !a.p)) return hipErrorInvalidValue;
    for (int i = 1; i < 5; ++i)
      for (int j = 0; j < i; ++j)
        if (o[i] != nullptr && o[i] == o[j]) return hipErrorInvalidValue;
  }
  ADL_DISPATCH_TILE(t, f, {
    if (f.f32) {
      if (a.ystore_f32) leja4_launch<float, float, VEC, ADVF>(f, t, a, st);
      else leja4_launch<float, double, VEC, ADVF>(f, t, a, st);
    } else {
      if (a.ystore_f32) leja4_launch<double, float, VEC, ADVF>(f, t, a, st);
      else leja4_launch<double, double, VEC, ADVF>(f, t, a, st);
    }
  });
  return hipGetLastError();
}

template <typename TF, typename TY, bool ADVF, bool NT, bool FIRST>
static void leja3s_launch_k(const FieldView& f, const Tiling& t, const LejaArgs& a, hipStream_t st) {
  const dim3 grid(a.decide_only ? 1 : t.nblocks + 1), blk(kTileBlock2);
  const size_t lds = staged3_lds_bytes<2, ADVF>();
  if (a.ev_start)
    hipExtLaunchKernelGGL((leja3s_kernel<TF, TY, ADVF, NT, FIRST>), grid, blk, lds, st, a.ev_start, a.ev_stop, 0, f,
                          t, a);
  else
    hipLaunchKernelGGL((leja3s_kernel<TF, TY, ADVF, NT, FIRST>), grid, blk, lds, st, f, t, a);
}

template <typename TF, typename TY, bool ADVF, bool NT>
static void leja3s_launch(const FieldView& f, const Tiling& t, const LejaArgs& a, hipStream_t st) {
  if constexpr (std::is_same_v<TY, double>) {
    if (a.first) {
      leja3s_launch_k<TF, TY, ADVF, NT, true>(f, t, a, st);
      return;
    }
  }
  leja3s_launch_k<TF, TY, ADVF, NT, false>(f, t, a, st);
}

template <typename TF, typename TY, bool NT>
static void leja3s_dispatch(const FieldView& f, const Tiling& t, const LejaArgs& a, hipStream_t st) {
  if (f.ax) leja3s_launch<TF, TY, true, NT>(f, t, a, st);
  else leja3s_launch<TF, TY, false, NT>(f, t, a, st);
}

hipError_t launch_leja3_step(const FieldView& f, const Tiling& t, const LejaArgs& a, hipStream_t st) {
  if (a.nterms != 3 || a.w2 != nullptr || a.yin_f32 != a.ystore_f32 || t.vec != 2) return hipErrorInvalidValue;
  // the first launch (terms 1 .. 3 from y_0 = v, FP64 Newton vectors only) or a later one
  if (a.first ? (a.k != 0 || a.ystore_f32 || a.decide_only || a.pin != nullptr) : a.k < 1)
    return hipErrorInvalidValue;
  if (!a.decide_only) {
    // p_k is read while the stored p outputs (at least one) are written: all distinct
    const double* o[4] = {a.pin, a.pmid, a.pmid2, a.p};
    if ((!a.first && a.pin == nullptr) || (!a.pmid && !a.pmid2 && !a.p)) return hipErrorInvalidValue;
    for (int i = 1; i < 4; ++i)
      for (int j = 0; j < i; ++j)
        if (o[i] != nullptr && o[i] == o[j]) return hipErrorInvalidValue;
  }
  if (a.stream) {
    if (f.f32) {
      if (a.ystore_f32) leja3s_dispatch<float, float, true>(f, t, a, st);
      else leja3s_dispatch<float, double, true>(f, t, a, st);
    } else {
      if (a.ystore_f32) leja3s_dispatch<double, float, true>(f, t, a, st);
      else leja3s_dispatch<double, double, true>(f, t, a, st);
    }
  } else {
    if (f.f32) {
      if (a.ystore_f32) leja3s_dispatch<float, float, false>(f, t, a, st);
      else leja3s_dispatch<float, double, false>(f, t, a, st);
    } else {
      if (a.ystore_f32) leja3s_dispatch<double, float, false>(f, t, a, st);
      else leja3s_dispatch<double, double, false>(f, t, a, st);
    }
  }
  return hipGetLastError();
}

template <typename TF, typename TY, bool ADVF, bool NT, bool STAGE>
static void leja4s_launch_k(const FieldView& f, const Tiling& t, const LejaArgs& a, hipStream_t st) {
  const dim3 grid(a.decide_only ? 1 : t.nblocks + 1), blk(kTileBlock2);
  const size_t lds = staged4_lds_bytes<2, ADVF>();
  if (a.ev_start)
    hipExtLaunchKernelGGL((leja4s_kernel<TF, TY, ADVF, NT, STAGE>), grid, blk, lds, st, a.ev_start, a.ev_stop, 0, f,
                          t, a);
  else
    hipLaunchKernelGGL((leja4s_kernel<TF, TY, ADVF, NT, STAGE>), grid, blk, lds, st, f, t, a);
}

template <typename TF, typename TY, bool ADVF, bool NT>
static void leja4s_launch(const FieldView& f, const Tiling& t, const LejaArgs& a, hipStream_t st) {
  if constexpr (std::is_same_v<TY, double>) {
    if (a.stage) {
      leja4s_launch_k<TF, TY, ADVF, NT, true>(f, t, a, st);
      return;
    }
  }
  leja4s_launch_k<TF, TY, ADVF, NT, false>(f, t, a, st);
}

template <typename TF, typename TY, bool NT>
static void leja4s_dispatch(const FieldView& f, const Tiling& t, const LejaArgs& a, hipStream_t st) {
  if (f.ax) leja4s_launch<TF, TY, true, NT>(f, t, a, st);
  else leja4s_launch<TF, TY, false, NT>(f, t, a, st);
}

hipError_t launch_leja4s_step(const FieldView& f, const Tiling& t, const LejaArgs& a, hipStream_t st) {
  if (a.w2 != nullptr || a.yin_f32 != a.ystore_f32 || t.vec != 2) return hipErrorInvalidValue;
  // the sweep's first launch with its stage vector (terms 1 .. 3 from w = A u
  // + s, FP64 Newton vectors, no p input, not a decision launch), or four
  // later terms
  if (a.stage ? (!a.first || a.k != 0 || a.nterms != 3 || a.ystore_f32 || a.decide_only || a.pin != nullptr)
              : (a.first || a.k < 1 || a.nterms != 4))
    return hipErrorInvalidValue;
  if (!a.decide_only) {
    // p_k is read while the stored p outputs (at least one) are written: all distinct
    const double* o[5] = {a.pin, a.pmid, a.pmid2, a.pmid3, a.p};
    if ((!a.stage && a.pin == nullptr) || (!a.pmid && !a.pmid2 && !a.pmid3 && !a.p)) return hipErrorInvalidValue;
    for (int i = 1; i < 5; ++i)
      for (int j = 0; j < i; ++j)
        if (o[i] != nullptr && o[i] == o[j]) return hipErrorInvalidValue;
  }
  if (a.stream) {
    if (f.f32) {
      if (a.ystore_f32) leja4s_dispatch<float, float, true>(f, t, a, st);
      else leja4s_dispatch<float, double, true>(f, t, a, st);
    } else {
      if (a.ystore_f32) leja4s_dispatch<double, float, true>(f, t, a, st);
      else leja4s_dispatch<double, double, true>(f, t, a, st);
    }
  } else {
    if (f.f32) {
      if (a.ystore_f32) leja4s_dispatch<float, float, false>(f, t, a, st);
      else leja4s_dispatch<float, double, false>(f, t, a, st);
    } else {
      if (a.ystore_f32) leja4s_dispatch<double, float, false>(f, t, a, st);
      else leja4s_dispatch<double, double, false>(f, t, a, st);
    }
  }
  return hipGetLastError();
}

hipError_t launch_leja2_step(const FieldView& f, const Tiling& t, const LejaArgs& a, hipStream_t st) {
  if (a.first || a.k < 1 || a.nterms != 2 || a.w2 != nullptr || a.yin_f32 != a.ystore_f32) return hipErrorInvalidValue;
  // p_k is read while the stored p outputs (at least one) are written: all distinct
  if (!a.decide_only && (a.pin == nullptr || (a.p == nullptr && a.pmid == nullptr) || a.pin == a.p ||
                         a.pin == a.pmid || (a.p != nullptr && a.p == a.pmid)))
    return hipErrorInvalidValue;
  ADL_DISPATCH_TILE(t, f, {
    if (a.stream) {
      if (f.f32) {
        if (a.ystore_f32) leja2_any<float, float, VEC, ADVF, true>(f, t, a, st);
        else leja2_any<float, double, VEC, ADVF, true>(f, t, a, st);
      } else {
        if (a.ystore_f32) leja2_any<double, float, VEC, ADVF, true>(f, t, a, st);
        else leja2_any<double, double, VEC, ADVF, true>(f, t, a, st);
      }
    } else {
      if (f.f32) {
        if (a.ystore_f32) leja2_any<float, float, VEC, ADVF, false>(f, t, a, st);
        else leja2_any<float, double, VEC, ADVF, false>(f, t, a, st);
      } else {
        if (a.ystore_f32) leja2_any<double, float, VEC, ADVF, false>(f, t, a, st);
        else leja2_any<double, double, VEC, ADVF, false>(f, t, a, st);
      }
    }
  });
  return hipGetLastError();
}

hipError_t launch_power_init(const Tiling& t, long n, uint64_t seed, double* w, double* partials, hipStream_t st) {
  hipLaunchKernelGGL(power_init_kernel, dim3(t.nblocks), dim3(kBlock), 0, st, n, seed, w, partials);
  return hipGetLastError();
}

hipError_t launch_power_step(const FieldView& f, const Tiling& t, const PowerArgs& a, hipStream_t st) {
  const dim3 grid(a.decide_only ? 1 : t.nblocks), blk(kTileBlock);
  ADL_DISPATCH_TILE(t, f, {
    if (f.f32) hipLaunchKernelGGL((power_kernel<float, VEC, ADVF>), grid, blk, 0, st, f, t, a);
    else hipLaunchKernelGGL((power_kernel<double, VEC, ADVF>), grid, blk, 0, st, f, t, a);
  });
  return hipGetLastError();
}

hipError_t launch_gershgorin(const FieldView& f, double* partials, Ctl* ctl, hipStream_t st) {
  const int nb = stats_blocks((long)f.nx * f.ny);
  const bool advf = f.ax != nullptr;
  if (f.f32) {
    if (advf) hipLaunchKernelGGL((gershgorin_kernel<float, true>), dim3(nb), dim3(kBlock), 0, st, f, partials, ctl);
    else hipLaunchKernelGGL((gershgorin_kernel<float, false>), dim3(nb), dim3(kBlock), 0, st, f, partials, ctl);
  } else {
    if (advf) hipLaunchKernelGGL((gershgorin_kernel<double, true>), dim3(nb), dim3(kBlock), 0, st, f, partials, ctl);
    else hipLaunchKernelGGL((gershgorin_kernel<double, false>), dim3(nb), dim3(kBlock), 0, st, f, partials, ctl);
  }
  return hipGetLastError();
}

hipError_t launch_ctl_reset(Ctl* ctl, int n, hipStream_t st) {
  hipLaunchKernelGGL(ctl_reset_kernel, dim3(1), dim3(64), 0, st, ctl, n);
  return hipGetLastError();
}

hipError_t launch_axpby(long n, double* y, double a, const double* x, double b, const double* z, hipStream_t st) {
  hipLaunchKernelGGL(axpby_kernel, dim3(ew_blocks(n)), dim3(kBlock), 0, st, n, y, a, x, b, z);
  return hipGetLastError();
}

hipError_t launch_diff_scale(long n, double* y, const double* x, const double* z, double s, hipStream_t st) {
  hipLaunchKernelGGL(diff_scale_kernel, dim3(ew_blocks(n)), dim3(kBlock), 0, st, n, y, x, z, s);
  return hipGetLastError();
}

hipError_t launch_fill(long n, double* y, double v, hipStream_t st) {
  hipLaunchKernelGGL(fill_kernel, dim3(ew_blocks(n)), dim3(kBlock), 0, st, n, y, v);
  return hipGetLastError();
}

hipError_t launch_prepare_field(long n, const double* in, double scale, void* out, int f32, hipStream_t st) {
  if (f32)
    hipLaunchKernelGGL((prepare_kernel<float>), dim3(ew_blocks(n)), dim3(kBlock), 0, st, n, in, scale,
                       reinterpret_cast<float*>(out));
  else
    hipLaunchKernelGGL((prepare_kernel<double>), dim3(ew_blocks(n)), dim3(kBlock), 0, st, n, in, scale,
                       reinterpret_cast<double*>(out));
  return hipGetLastError();
}

}  // namespace adl
