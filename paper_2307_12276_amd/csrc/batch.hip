// Batched momentum bins: many independent operators (grids of different
// sizes, different spectral intervals) advanced by one exponential midpoint
// step (Sec. 2, eq. 4) together.
//
// Work unit: a tile = one wave64 strip of 64*VEC columns x `rows` rows of one
// bin, which the wave marches down row by row (the windows of rows it needs
// in registers, the next row's loads in flight).  Every kernel of a step
// covers the tiles of all bins:
//   stage      w_b = A_b u_b + S_b
//   term k     y_{k+1} = ((A_b - c_b)/gamma_b - xi_k) y_k,
//              p_{b,k+1} = p_{b,k} + d_{b,k+1} y_{k+1},
//              for every bin still running, with the bin's own plan; after
//              the first term two terms per launch by default (y_{k+1} kept
//              in registers), or three with the input rows staged in LDS
//              (blocks of four waves march runs of one strip of a bin)
//   finalize   the decision of the last term, one wave per bin
//   update     u_b += dt p_b for converged bins
// The stopping decision lags one launch behind the work, as for a single
// operator: the first nbins blocks of a term launch are one decision wave per
// bin, which sums the bin's tile partials of the previous launch in a fixed
// order and records the decision; the tile waves only check their bin's stop
// flag (set by an earlier launch) and compute the next term.  When the
// decision recorded in launch k stops a bin, the term launch k computed for it
// is discarded (p_k is intact in the other buffer).  The launches of a step
// (reset, stage, terms, finalize) are captured once in a hipGraph and
// replayed: one graph launch per step.  Kernel boundaries give cross-XCD
// visibility of y_k, so no wave ever waits on another and no agent-scope fence
// is needed.
#include "staged.h"
#include "tile.h"
#include "op.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

namespace adl {

struct BinDesc {
  FieldView f;
  const double* u;
  const double* S;
  double* w;
  void* y0;             // y of launch L's last term in y0 (L odd) or y1 (L even)
  void* y1;
  double* pb[4];        // p_m of degree m: pb[pbuf_index(m)]
  const double* d;      // d_0 .. d_{M-1} of the bin's plan
  const double* shift;  // c + gamma xi_k
  double invg;
  double tol;
  double dt;
  int max_degree;
  int ncb;        // strips of 64*VEC columns (one-term tiles)
  int rows;       // band height
  int ntiles;
  int tile_base;  // first global tile of this bin
  int ncb2;       // strips of 62*VEC output columns (two-term tiles)
  int ntiles2;
  int tile_base2;
  int ncb3;       // three-term blocks: strips of 124 output columns,
  int bands3;     // runs of bands3 bands of four rows,
  int nblocks3;   // ncb3 x runs blocks from block_base3 on
  int block_base3;
  float* y2b[2];   // three-term launches: y of the second-to-last term of launch L (FP32) in y2b[L & 1]
  int active;     // 0: the bin is advanced by the single-op path instead
};

struct BinCtl {
  int stop;
  int status;  // 0 running, 1 converged, 2 non-finite, 3 degree cap
  int degree;
  int upd;     // 1: u already advanced by an earlier update launch of this step
  int inner;   // terms of the stopping launch after the stopping term (their p alone is stored)
  int launch;  // launch index of the stopping term (kNoLaunch until the bin stops)
  double tn2, pn2;
  double hist[kStopHist];  // term norms of the stopping window (as in Ctl)
};

struct BatchArgs {
  const BinDesc* bins;
  const int* tile_bin;   // global one-term tile -> bin
  const int* tile_bin2;  // global two-term tile -> bin
  const int* block_bin3;  // global three-term block -> bin
  BinCtl* ctl;
  double* partials;      // 2 launch parities x tiles x 6
  int total_tiles;
  int total_tiles2;
  int total_blocks3;
  long part_stride;      // doubles per parity
  int L;                 // launch index within the sweep
  int k;                 // terms before this launch
  int kprev, nprev;      // the previous launch: terms before it, its terms (1 or 2)
  int two;               // p buffers in pairs per launch (two-term sweeps)
  int three;             // three-term sweeps: p of launch L's last term in pb[(L & 1) ? 0 : 1]
  int advance;           // tiles of a stopped bin advance u in its due launch (0: timing runs leave u alone)
};

// Launch geometry of the tile kernels: kBWaves independent waves per block,
// each its own unit of work (a tile, or a bin's decision), with no barrier
// or LDS shared between them.  The waves of a block take neighbouring tiles
// of a bin (adjacent strips of a band), which run on one CU and share the
// cache lines at their common edges: against one-wave blocks, HBM traffic of
// a full two-term launch 1.20x -> 1.10x algorithmic and 321 -> 300-306 us.
constexpr int kBWaves = 4;
__device__ __forceinline__ int wave_unit() {
  return (int)blockIdx.x * kBWaves + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
}
inline unsigned blocks_for(long units) { return (unsigned)((units + kBWaves - 1) / kBWaves); }

// buffer of p_m: two-term sweeps keep the terms of a launch in one pair, the
// pairs alternating (a launch never overwrites the p its decision may pick);
// one-term sweeps alternate by degree
__device__ __forceinline__ int pbuf_index(int m, int two) {
  return two ? 2 * ((m >> 1) & 1) + (m & 1) : (m & 1);
}
// three-term sweeps: the p buffer launch L writes (its last term's p; the
// first launch writes pb[1], as pbuf_index(1, .) gives) and the one it reads
__device__ __forceinline__ int pbuf_out3(int L) { return (L & 1) ? 0 : 1; }
__device__ __forceinline__ int pbuf_in3(int L) { return (L & 1) ? 1 : 0; }

// BinCtl::launch before any decision: far from every launch index, so that a
// tile that reads the stop flag set beside it in its own launch, together
// with an older value of `launch`, never takes the update as due
constexpr int kNoLaunch = -1000000;

// The update u_b += dt p_m of a bin that stopped at term m with status 1,
// over rows j0 .. j1-1 and columns c0 .. c1-1 of the bin (a tile's own
// points; one lane per VEC columns).  A bin that stopped at an earlier term m
// of a fused launch is advanced by p_m = p_last - d_last y_last (- d_{m+1}
// y_{m+1} when the launch ran two terms past m, three-term sweeps): that
// launch stored p and y of its last term (and, with three terms, y of the one
// before, in FP32: the term d_{m+1} y_{m+1} is of the order of tol |p| at a
// stop, so its rounding moves p_m by ~1e-7 tol |p|), and no later launch of
// the sweep wrote those buffers of the bin (the launch beside the decision
// writes the other y buffers and the other p buffers, and every later one
// skips the bin).
template <int VEC>
__device__ __forceinline__ void bin_update_rect(const BatchArgs& A, const BinDesc& B, const BinCtl& c,
                                                double* __restrict__ ub, int j0, int j1, int c0, int c1) {
  const int m = c.degree;
  const int back = c.inner;
  const double* __restrict__ pb = B.pb[A.three ? pbuf_out3(c.launch) : pbuf_index(m + back, A.two)];
  const double* __restrict__ yb = reinterpret_cast<const double*>(((c.launch + 1) & 1) ? B.y1 : B.y0);
  const float* __restrict__ yb2 = B.y2b[c.launch & 1];
  const double dm = back > 0 ? B.d[min(m + back, B.max_degree)] : 0.0;
  const double dm2 = back > 1 ? B.d[min(m + 1, B.max_degree)] : 0.0;
  const double dt = B.dt;
  const int nx = B.f.nx;
  const int col0 = c0 + (int)(threadIdx.x & 63) * VEC;
  if (col0 >= c1) return;
  // rows in groups of four, every load of a group issued before its stores
  // (u, p and the y are distinct arrays)
  constexpr int G = 4;
  for (int j = j0; j < j1; j += G) {
    double uu[G][VEC], pp[G][VEC], yy[G][VEC], zz[G][VEC];
#pragma unroll
    for (int q = 0; q < G; ++q) {
      const long ro = (long)min(j + q, j1 - 1) * nx;
      ldr<double, VEC>(ub + ro, col0, uu[q]);
      ldr<double, VEC>(pb + ro, col0, pp[q]);
      if (back > 0) {
        ldr<double, VEC>(yb + ro, col0, yy[q]);
      } else {
#pragma unroll
        for (int v = 0; v < VEC; ++v) yy[q][v] = 0.0;
      }
      if (back > 1) {
        ldr<float, VEC>(yb2 + ro, col0, zz[q]);
      } else {
#pragma unroll
        for (int v = 0; v < VEC; ++v) zz[q][v] = 0.0;
      }
    }
#pragma unroll
    for (int q = 0; q < G; ++q) {
      if (j + q < j1) {
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          double pv = pp[q][v];
          if (back > 0) pv = pv - dm * yy[q][v];
          if (back > 1) pv = pv - dm2 * zz[q][v];
          uu[q][v] = uu[q][v] + dt * pv;
        }
        str<double, VEC>(ub + (long)(j + q) * nx, col0, uu[q]);
      }
    }
  }
}

// A tile of a stopped bin in term launch A.L: the bin's update is due in the
// launch after the one whose decision stopped it (launch c.launch + 2), done
// there by the bin's tiles; the tail's update launch advances the bins whose
// due launch did not run.
__device__ __forceinline__ bool update_due(const BatchArgs& A, const BinCtl& c) {
  return A.advance && c.status == 1 && !c.upd && c.degree > 0 && A.L == c.launch + 2;
}

// ---------------------------------------------------------------------------
__device__ __forceinline__ void wave_sum3(double (&v)[3]) {
#pragma unroll
  for (int q = 0; q < 3; ++q) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double t = __shfl_xor(v[q], o);
      v[q] = (q < 2) ? v[q] + t : nanmax(v[q], t);
    }
  }
}

// Decision for the terms of the previous launch of bin b (kprev+1, and
// kprev+2 after a two-term launch, in order), from that launch's tile
// partials (whole wave; fixed order).
__device__ __forceinline__ bool bin_decide(const BatchArgs& A, const BinDesc& B, int b, bool record) {
  const int nterms = A.nprev;
  const bool two = nterms == 2, three = nterms == 3;
  const int base = three ? B.block_base3 : two ? B.tile_base2 : B.tile_base;
  const int nt = three ? B.nblocks3 : two ? B.ntiles2 : B.ntiles;
  const double* part = A.partials + (long)((A.L - 1) & 1) * A.part_stride + (long)base * 6;
  // a unit's partials: ||d y||^2 and ||p||^2 of its terms at (0, 1), (3, 4)
  // and, after a three-term launch, (2, 5); after a one-term launch entry 2
  // is max |y_0| (the first term's zero check)
  double tot[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  bool any = false;
  for (int t = threadIdx.x & 63; t < nt; t += 64) {
    tot[0] += part[t * 6 + 0];
    tot[1] += part[t * 6 + 1];
    tot[2] = three ? tot[2] + part[t * 6 + 2] : (any ? nanmax(tot[2], part[t * 6 + 2]) : part[t * 6 + 2]);
    tot[3] += part[t * 6 + 3];
    tot[4] += part[t * 6 + 4];
    tot[5] += part[t * 6 + 5];
    any = true;
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double t = __shfl_xor(tot[q], o);
      tot[q] = (q == 2 && !three) ? nanmax(tot[q], t) : tot[q] + t;
    }
  }
  BinCtl* c = A.ctl + b;
  // terms up to `done` were decided already (the finalize launch of an
  // earlier enqueue decided the launch this one is handed again): each term
  // enters the stopping window once
  const int done = c->degree;
  if (A.kprev + nterms <= done) return false;
  double hist[kStopHist];
#pragma unroll
  for (int i = 0; i < kStopHist; ++i) hist[i] = c->hist[i];
  int stop = 0, status = 0, degree = 0;
  double tn2 = 0.0, pn2 = 0.0;
  for (int i = 0; i < nterms && !stop; ++i) {
    if (A.kprev + 1 + i <= done) continue;
    tn2 = i < 2 ? tot[3 * i] : tot[2];
    pn2 = i < 2 ? tot[3 * i + 1] : tot[5];
    degree = A.kprev + 1 + i;
    if (!isfinite(tn2) || !isfinite(pn2)) {
      stop = 1; status = 2;
    } else if (A.kprev == 0 && i == 0 && (three ? tn2 == 0.0 && pn2 == 0.0 : tot[2] == 0.0)) {
      // y_0 = 0 (a three-term first launch has no max |y_0|: with y_0 = 0,
      // and only then, both d_1 y_1 and p_1 = d_0 y_0 + d_1 y_1 vanish)
      stop = 1; status = 1; degree = 0;
    } else if (window_stop(hist, degree, sqrt(tn2), pn2, B.tol)) {
      stop = 1; status = 1;
    } else if (degree >= B.max_degree) {
      stop = 1; status = 3;
    }
  }
  if (record && (threadIdx.x & 63) == 0) {
    c->tn2 = tn2;
    c->pn2 = pn2;
#pragma unroll
    for (int i = 0; i < kStopHist; ++i) c->hist[i] = hist[i];
    c->degree = degree;
    c->status = status;
    // recorded only by the decision that stops the bin: a tile that reads
    // the stop flag set beside it in this launch, with `launch` as it was
    // before, then sees kNoLaunch (never a due launch), not the value of an
    // earlier, non-stopping decision, which would make the current launch
    // look due and advance u twice
    if (stop) {
      c->inner = degree > 0 ? A.kprev + nterms - degree : 0;
      c->launch = A.L - 1;
    }
    __hip_atomic_store(&c->stop, stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  return stop != 0;
}

// marching one-term tiles of the stage launch and of the Newton terms of
// one-term launches (defined with the marching machinery below)
template <typename TF, int VEC, bool ADVF>
__device__ __forceinline__ void batch_stage_tile(const BatchArgs& A, const BinDesc& B, int t);
template <typename TF, int VEC, bool ADVF>
__device__ __forceinline__ void batch_first_tile(const BatchArgs& A, const BinDesc& B, int t);
template <typename TF, int VEC, bool ADVF>
__device__ __forceinline__ void batch_next_tile(const BatchArgs& A, const BinDesc& B, int t);

template <typename TF, int VEC, bool ADVF>
__global__ __launch_bounds__(64 * kBWaves) void batch_stage_kernel(BatchArgs A) {
  const int gt = wave_unit();
  if (gt >= A.total_tiles) return;
  const int b = __builtin_amdgcn_readfirstlane(A.tile_bin[gt]);
  const BinDesc& B = A.bins[b];
  if (!B.active) return;
  batch_stage_tile<TF, VEC, ADVF>(A, B, gt - B.tile_base);
}

__device__ __forceinline__ double* tile_partials(const BatchArgs& A, long tile) {
  return A.partials + (long)(A.L & 1) * A.part_stride + tile * 6;
}

template <typename TF, int VEC, bool ADVF, bool FIRST>
__device__ __forceinline__ void batch_term(const BatchArgs& A, const BinDesc& B, int t) {
  if constexpr (FIRST) batch_first_tile<TF, VEC, ADVF>(A, B, t);
  else batch_next_tile<TF, VEC, ADVF>(A, B, t);
}

// Term launch L (terms k+1 .. k+nterms): blocks [0, nbins) decide the terms
// of launch L-1 of their bin (from its partials), the tile blocks compute the
// launch's terms of their bin unless the bin has stopped.  The first term
// (k = 0, y_0 = w) is a kernel of its own.
template <typename TF, int VEC, bool ADVF, bool FIRST>
__global__ __launch_bounds__(64 * kBWaves) void batch_leja_kernel(BatchArgs A, int nbins) {
  const int w = wave_unit();
  if (w < nbins) {
    const int b = w;
    const BinDesc& B = A.bins[b];
    if (FIRST || !B.active) return;
    if (__hip_atomic_load(&A.ctl[b].stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    bin_decide(A, B, b, true);
    return;
  }
  const int gt = w - nbins;
  if (gt >= A.total_tiles) return;
  const int b = __builtin_amdgcn_readfirstlane(A.tile_bin[gt]);
  const BinDesc& B = A.bins[b];
  if (!B.active) return;
  if (__hip_atomic_load(&A.ctl[b].stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
    const BinCtl& c = A.ctl[b];
    if (!FIRST && update_due(A, c)) {
      const int t = gt - B.tile_base;
      const int rb = t / B.ncb, cb = t - rb * B.ncb;
      const int j0 = rb * B.rows, c0 = cb * kWave * VEC;
      bin_update_rect<VEC>(A, B, c, const_cast<double*>(B.u), j0, min(j0 + B.rows, B.f.ny), c0,
                           min(c0 + kWave * VEC, B.f.nx));
    }
    return;
  }
  if (A.k >= B.max_degree) return;
  batch_term<TF, VEC, ADVF, FIRST>(A, B, gt - B.tile_base);
}

// Two terms per launch (k >= 1) on one wave per tile of 62*VEC output columns
// x `rows` rows (lanes 0 and 63 are the one-column frame): the wave marches
// down its rows with every vertical window in registers -- input rows r ..
// r+2 of y_k, rows r-1 .. r+2 of kyy and kxy (ay'), rows r .. r+1 of kxx
// (ax'), y_{k+1} on rows r-1 .. r+1 -- computing y_{k+1} of row r+1 and then
// y_{k+2} of row r; p_{k+1} and p_{k+2} as for a single operator (p_{k+2}
// stored; the update launch rebuilds p_{k+1} of a bin that stopped there).  Each step
// first issues the loads of the next step's new input row (and of its p_k
// row), so that their latency hides behind the step's arithmetic, and every
// input element of the tile is loaded once.  The x-neighbours of y_{k+1} come
// from DPP shifts within the wave (the frame lanes compute y_{k+1} too), so
// the wave needs neither LDS nor a barrier.

// Memory access of the marching tiles: buffer loads and stores through one
// buffer resource per array (base address in scalar registers), the row's
// byte offset as the scalar offset and the lane's column as a 32-bit vector
// offset.  (A bin's array addresses come from its descriptor in memory; used
// as plain pointers they are generic to the compiler, which then accesses
// them with FLAT instructions -- counted by the LDS/scalar counter too, so
// that every use of a loaded value waits for all loads in flight -- and keeps
// a 64-bit address per lane and load.)  Arrays are limited to 2 GiB (checked
// when a batch is created).
typedef __amdgpu_buffer_rsrc_t Rsrc;
constexpr int kRsrcWord3 = 0x00020000;  // raw buffer, 32-bit data format (CDNA)

__device__ __forceinline__ Rsrc rsrc_of(const void* p) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, 0x7fffffff, kRsrcWord3);
}

template <typename T, int VEC>
__device__ __forceinline__ void bload(Rsrc r, int voff, int soff, T (&c)[VEC]) {
  if constexpr (sizeof(T) == 8 && VEC == 2) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 v = __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
    c[0] = v.x;
    c[1] = v.y;
  } else if constexpr (sizeof(T) == 8) {
    c[0] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  } else if constexpr (VEC == 2) {
    typedef float f2 __attribute__((ext_vector_type(2)));
    const f2 v = __builtin_bit_cast(f2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    c[0] = v.x;
    c[1] = v.y;
  } else {
    c[0] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
  }
}
template <typename T>
__device__ __forceinline__ T bload1(Rsrc r, int voff, int soff) {
  T c[1];
  bload<T, 1>(r, voff, soff, c);
  return c[0];
}
template <int VEC>
__device__ __forceinline__ void bstore(Rsrc r, int voff, int soff, const double (&c)[VEC]) {
  if constexpr (VEC == 2) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
    d2 v;
    v.x = c[0];
    v.y = c[1];
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, v), r, voff, soff, 0);
  } else {
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, c[0]), r, voff, soff, 0);
  }
}

// Wave-uniform copies (scalar registers) of values a tile reads from its
// bin's descriptor: loaded by vector loads, they would otherwise stay in
// vector registers, and so would every address computed from them.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ unsigned long long uni64(unsigned long long v) {
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ double uni(double v) {
  return __longlong_as_double((long long)uni64((unsigned long long)__double_as_longlong(v)));
}
template <typename T>
__device__ __forceinline__ T* uni(T* p) {
  return (T*)uni64((unsigned long long)p);
}

// one lane's part of a row as stored (type T): its VEC values, the halo
// element (lane 0: left, lane 63: right) and the zero-ghost-row flag
template <typename T, int VEC>
struct TRow {
  T c[VEC];
  T h;
  bool zero;
};
template <typename T, int VEC>
struct TRowC {
  T c[VEC];
  bool zero;
};

// a lane's byte offsets in a row: its own columns and its halo column, for
// 8- and 4-byte elements, and its output columns (8-byte)
struct LaneOff {
  int c8, h8, c4, h4, o8;
};

template <typename T, int VEC, int MODE>
__device__ __forceinline__ void trow_load(Rsrc a, int r, const FieldView& F, const LaneOff& lo, TRow<T, VEC>& o) {
  const int row = uni(map_row_any(r, F.ny, F.bc, MODE, o.zero));
  const int soff = row * F.nx * (int)sizeof(T);
  bload<T, VEC>(a, sizeof(T) == 8 ? lo.c8 : lo.c4, soff, o.c);
  o.h = bload1<T>(a, sizeof(T) == 8 ? lo.h8 : lo.h4, soff);
}

template <typename T, int VEC, int MODE>
__device__ __forceinline__ void trowc_load(Rsrc a, int r, const FieldView& F, const LaneOff& lo,
                                           TRowC<T, VEC>& o) {
  const int row = uni(map_row_any(r, F.ny, F.bc, MODE, o.zero));
  bload<T, VEC>(a, sizeof(T) == 8 ? lo.c8 : lo.c4, row * F.nx * (int)sizeof(T), o.c);
}

template <typename T, int CTRL>
__device__ __forceinline__ double dpp_t(T v) {
  if constexpr (sizeof(T) == 8) {
    return dpp_f64<CTRL>(v);
  } else {
    return (double)__int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
  }
}

// a stored row with its x-neighbours (DPP shifts, halo element, Dirichlet
// ghost selects), in FP64, as row_n builds it
template <typename T, int VEC, int MODE>
__device__ __forceinline__ RowN<VEC> rown_of(const TRow<T, VEC>& x, const Strip& g) {
  RowN<VEC> o;
#pragma unroll
  for (int v = 0; v < VEC; ++v) o.c[v] = x.zero ? 0.0 : (double)x.c[v];
  // (shifts taken on every lane, then selected: see ring_rown)
  const double sl = dpp_t<T, kDppWaveShr1>(x.c[VEC - 1]);
  const double sr = dpp_t<T, kDppWaveShl1>(x.c[0]);
  const double l = x.zero ? 0.0 : sl;
  const double rr = x.zero ? 0.0 : sr;
  const double hz = x.zero ? 0.0 : (double)x.h;
  const double gl = MODE == MODE_EDGE ? o.c[0] : 0.0;
  const double gr = MODE == MODE_EDGE ? o.c[VEC - 1] : 0.0;
  o.l = g.ghostL ? gl : (g.useL ? hz : l);
  o.r = g.ghostR ? gr : (g.useR ? hz : rr);
  return o;
}

template <typename T, int VEC>
__device__ __forceinline__ RowC<VEC> rowc_of(const TRowC<T, VEC>& x) {
  RowC<VEC> o;
#pragma unroll
  for (int v = 0; v < VEC; ++v) o.c[v] = x.zero ? 0.0 : (double)x.c[v];
  return o;
}

// y_{k+1} values of a row (zero at ghost positions) with their x-neighbours
template <int VEC>
__device__ __forceinline__ RowN<VEC> rown_y1(const double (&c)[VEC]) {
  RowN<VEC> o;
#pragma unroll
  for (int v = 0; v < VEC; ++v) o.c[v] = c[v];
  o.l = dpp_f64<kDppWaveShr1>(c[VEC - 1]);
  o.r = dpp_f64<kDppWaveShl1>(c[0]);
  return o;
}

// the new rows of one marching step, as stored: input row q of y_k, kyy,
// kxy (ay'), row q-1 of kxx (ax'), and p_k of the step's output row
template <typename TF, int VEC>
struct StepRows {
  TRow<double, VEC> y;
  TRow<TF, VEC> m, k, ax;
  TRowC<TF, VEC> g, ay;
  double p[VEC];
};

// A copy into fresh registers that the compiler cannot merge with its
// source: a step copies the rows it was handed before using them, so that
// their load registers are free again for the loads of the next step,
// and the loop carries each buffer of loads in flight in the same registers
// (otherwise the register allocator may copy a register whose load is still
// in flight at the loop's back edge, and such a copy waits for the load).
__device__ __forceinline__ float vcopy(float v) {
  float o;
  asm("v_mov_b32 %0, %1" : "=v"(o) : "v"(v));
  return o;
}
__device__ __forceinline__ double vcopy(double v) {
  double o;
  asm("v_mov_b64 %0, %1" : "=v"(o) : "v"(v));
  return o;
}
template <typename T, int VEC>
__device__ __forceinline__ TRow<T, VEC> vcopy(const TRow<T, VEC>& x) {
  TRow<T, VEC> o;
#pragma unroll
  for (int v = 0; v < VEC; ++v) o.c[v] = vcopy(x.c[v]);
  o.h = vcopy(x.h);
  o.zero = x.zero;
  return o;
}
template <typename T, int VEC>
__device__ __forceinline__ TRowC<T, VEC> vcopy(const TRowC<T, VEC>& x) {
  TRowC<T, VEC> o;
#pragma unroll
  for (int v = 0; v < VEC; ++v) o.c[v] = vcopy(x.c[v]);
  o.zero = x.zero;
  return o;
}

// the arrays a two-term tile reads, as buffer resources
struct TileIn {
  Rsrc y, p, kxx, kxy, kyy, ax, ay;
};

template <typename TF, int VEC, bool ADVF>
__device__ __forceinline__ void load_step_rows(const FieldView& F, const TileIn& in, const LaneOff& lo, bool own,
                                               int q, bool with_k, int pr, StepRows<TF, VEC>& s) {
  trow_load<double, VEC, MODE_ZERO>(in.y, q, F, lo, s.y);
  trowc_load<TF, VEC, MODE_EDGE>(in.kyy, q, F, lo, s.g);
  trow_load<TF, VEC, MODE_ZERO>(in.kxy, q, F, lo, s.m);
  if constexpr (ADVF) trowc_load<TF, VEC, MODE_ZERO>(in.ay, q, F, lo, s.ay);
  if (with_k) {
    trow_load<TF, VEC, MODE_EDGE>(in.kxx, q - 1, F, lo, s.k);
    if constexpr (ADVF) trow_load<TF, VEC, MODE_ZERO>(in.ax, q - 1, F, lo, s.ax);
  }
  if (own) bload<double, VEC>(in.p, lo.o8, pr * F.nx * 8, s.p);
}

// One stencil application per row on the one-term tiling (a wave per strip
// of 64*VEC columns x `rows` rows, halo elements at the strip edges), with
// the two-term tile's marching: windows of stored rows (y rows r-1, r; kyy,
// kxy, ay' rows r-1, r), each step's new rows (input row r+1, kxx and ax' row
// r, the epilogue's extra input row r) loaded during the step before, two
// buffers taking turns.  fin(r, Ax, y_r, extra_r) consumes each row; `extra`
// (wave-uniform) says whether in.p holds an extra input to load.
template <typename TF, int VEC, bool ADVF, class Fin>
__device__ __forceinline__ void march1(const FieldView& F, const TileIn& in, const LaneOff& lo, const Strip& g,
                                       bool extra, int j0, int j1, Fin&& fin) {
  using RY = TRow<double, VEC>;
  using RF = TRow<TF, VEC>;
  using RC = TRowC<TF, VEC>;
  const bool ld = g.inside && extra;
  StepRows<TF, VEC> s0, s1, na, nb;
  load_step_rows<TF, VEC, ADVF>(F, in, lo, false, j0 - 1, false, j0, s0);
  load_step_rows<TF, VEC, ADVF>(F, in, lo, false, j0, false, j0, s1);
  load_step_rows<TF, VEC, ADVF>(F, in, lo, ld, j0 + 1, true, j0, na);
  RY wy0 = s0.y, wy1 = s1.y;
  RC wgA = s0.g, wgB = s1.g;
  RF wmA = s0.m, wmB = s1.m;
  RC waA = s0.ay, waB = s1.ay;
  auto step = [&](int r, const StepRows<TF, VEC>& held, StepRows<TF, VEC>& nxt) {
    // (nxt was copied out by the step before: its registers are free)
    load_step_rows<TF, VEC, ADVF>(F, in, lo, ld, min(r + 2, j1), true, min(r + 1, j1 - 1), nxt);
    StepRows<TF, VEC> cur;
    cur.y = vcopy(held.y);
    cur.g = vcopy(held.g);
    cur.m = vcopy(held.m);
    cur.k = vcopy(held.k);
    if constexpr (ADVF) {
      cur.ax = vcopy(held.ax);
      cur.ay = vcopy(held.ay);
    }
#pragma unroll
    for (int v = 0; v < VEC; ++v) cur.p[v] = ld ? vcopy(held.p[v]) : 0.0;
    RowN<VEC> xn{};
    RowC<VEC> an0{}, an2{};
    if constexpr (ADVF) {
      xn = rown_of<TF, VEC, MODE_ZERO>(cur.ax, g);
      an0 = rowc_of<TF, VEC>(waA);
      an2 = rowc_of<TF, VEC>(cur.ay);
    }
    const RowN<VEC> uc = rown_of<double, VEC, MODE_ZERO>(wy1, g);
    double Ax[VEC];
    stencil_point<VEC, ADVF>(rown_of<double, VEC, MODE_ZERO>(wy0, g), uc, rown_of<double, VEC, MODE_ZERO>(cur.y, g),
                             rowc_of<TF, VEC>(wgA), rowc_of<TF, VEC>(wgB), rowc_of<TF, VEC>(cur.g),
                             rown_of<TF, VEC, MODE_ZERO>(wmA, g), rown_of<TF, VEC, MODE_ZERO>(wmB, g),
                             rown_of<TF, VEC, MODE_ZERO>(cur.m, g), rown_of<TF, VEC, MODE_EDGE>(cur.k, g), xn, an0,
                             an2, F.axc, F.ayc, Ax);
    fin(r, Ax, uc.c, cur.p);
    wy0 = wy1;
    wy1 = cur.y;
    wgA = wgB;
    wgB = cur.g;
    wmA = wmB;
    wmB = cur.m;
    if constexpr (ADVF) {
      waA = waB;
      waB = cur.ay;
    }
  };
  int r = j0;
#pragma unroll 1
  for (; r + 1 < j1; r += 2) {
    step(r, na, nb);
    step(r + 1, nb, na);
  }
  if (r < j1) step(r, na, nb);
}

// the descriptor's values for a one-term tile, read once into scalar registers
struct TileSetup {
  FieldView F;
  int j0, j1;
  Strip g;
  LaneOff lo;
};
template <int VEC>
__device__ __forceinline__ TileSetup tile_setup(const BinDesc& B, int t) {
  TileSetup s;
  s.F = B.f;
  s.F.nx = uni(s.F.nx);
  s.F.ny = uni(s.F.ny);
  s.F.bc = uni(s.F.bc);
  s.F.axc = uni(s.F.axc);
  s.F.ayc = uni(s.F.ayc);
  const int ncb = uni(B.ncb), rows = uni(B.rows);
  const int rb = t / ncb, cb = t - rb * ncb;
  s.j0 = rb * rows;
  s.j1 = min(s.j0 + rows, s.F.ny);
  s.g = make_strip<VEC>(s.F, cb);
  s.lo = LaneOff{s.g.colc * 8, s.g.hcol * 8, s.g.colc * 4, s.g.hcol * 4, s.g.col0 * 8};
  return s;
}
template <typename TF, bool ADVF>
__device__ __forceinline__ void fields_in(const FieldView& F, TileIn& in) {
  in.kxx = rsrc_of(uni(F.kxx));
  in.kxy = rsrc_of(uni(F.kxy));
  in.kyy = rsrc_of(uni(F.kyy));
  if constexpr (ADVF) {
    in.ax = rsrc_of(uni(F.ax));
    in.ay = rsrc_of(uni(F.ay));
  }
}

// w = A u + S on a one-term tile (S may be absent)
template <typename TF, int VEC, bool ADVF>
__device__ __forceinline__ void batch_stage_tile(const BatchArgs& A, const BinDesc& B, int t) {
  (void)A;
  const TileSetup ts = tile_setup<VEC>(B, t);
  const bool has_s = uni((int)(B.S != nullptr)) != 0;
  TileIn in;
  in.y = rsrc_of(uni(B.u));
  in.p = rsrc_of(uni(has_s ? B.S : B.u));  // (loaded only with a source)
  fields_in<TF, ADVF>(ts.F, in);
  const Rsrc out = rsrc_of(uni(B.w));
  march1<TF, VEC, ADVF>(ts.F, in, ts.lo, ts.g, has_s, ts.j0, ts.j1,
                        [&](int r, const double (&Ax)[VEC], const double (&)[VEC], const double (&sv)[VEC]) {
                          if (!ts.g.inside) return;
                          double o[VEC];
#pragma unroll
                          for (int v = 0; v < VEC; ++v) {
                            o[v] = Ax[v];
                            if (has_s) o[v] += sv[v];
                          }
                          bstore<VEC>(out, ts.lo.o8, r * ts.F.nx * 8, o);
                        });
}

// the first Newton term of every bin's sweep on a one-term tile: y_1 from
// y_0 = w, p_1 = d_0 y_0 + d_1 y_1, the tile's partial norms and max |y_0|
template <typename TF, int VEC, bool ADVF>
__device__ __forceinline__ void batch_first_tile(const BatchArgs& A, const BinDesc& B, int t) {
  const TileSetup ts = tile_setup<VEC>(B, t);
  TileIn in;
  in.y = rsrc_of(uni(B.w));
  in.p = in.y;  // (no extra input)
  fields_in<TF, ADVF>(ts.F, in);
  const Rsrc yout = rsrc_of(uni(((A.L + 1) & 1) ? B.y1 : B.y0));
  const Rsrc pout = rsrc_of(uni(B.pb[pbuf_index(1, A.two)]));
  const double shift = uni(B.shift[0]), invg = uni(B.invg), d0 = uni(B.d[0]), dk1 = uni(B.d[1]);
  double acc[3] = {0.0, 0.0, 0.0};
  march1<TF, VEC, ADVF>(ts.F, in, ts.lo, ts.g, false, ts.j0, ts.j1,
                        [&](int r, const double (&Ax)[VEC], const double (&yc)[VEC], const double (&)[VEC]) {
                          if (!ts.g.inside) return;
                          double yn[VEC], pn[VEC];
#pragma unroll
                          for (int v = 0; v < VEC; ++v) {
                            const double y1 = (Ax[v] - shift * yc[v]) * invg;
                            const double tt = dk1 * y1;
                            const double pv = d0 * yc[v] + tt;
                            yn[v] = y1;
                            pn[v] = pv;
                            acc[0] += tt * tt;
                            acc[1] += pv * pv;
                            acc[2] = nanmax(acc[2], fabs(yc[v]));
                          }
                          const int so = r * ts.F.nx * 8;
                          bstore<VEC>(yout, ts.lo.o8, so, yn);
                          bstore<VEC>(pout, ts.lo.o8, so, pn);
                        });
  wave_sum3(acc);
  if ((threadIdx.x & 63) == 0) {
    double* part = tile_partials(A, B.tile_base + t);
    part[0] = acc[0];
    part[1] = acc[1];
    part[2] = acc[2];
    part[3] = part[4] = part[5] = 0.0;
  }
}

// a later Newton term (k >= 1) of one-term launches: y_{k+1} from y_k,
// p_{k+1} = p_k + d_{k+1} y_{k+1} (p_k the march's extra input row), the
// tile's partial norms
template <typename TF, int VEC, bool ADVF>
__device__ __forceinline__ void batch_next_tile(const BatchArgs& A, const BinDesc& B, int t) {
  const TileSetup ts = tile_setup<VEC>(B, t);
  const int k = A.k;
  TileIn in;
  in.y = rsrc_of(uni((A.L & 1) ? B.y1 : B.y0));
  in.p = rsrc_of(uni(B.pb[pbuf_index(k, A.two)]));
  fields_in<TF, ADVF>(ts.F, in);
  const Rsrc yout = rsrc_of(uni(((A.L + 1) & 1) ? B.y1 : B.y0));
  const Rsrc pout = rsrc_of(uni(B.pb[pbuf_index(k + 1, A.two)]));
  const double shift = uni(B.shift[k]), invg = uni(B.invg), dk1 = uni(B.d[k + 1]);
  double acc[3] = {0.0, 0.0, 0.0};
  march1<TF, VEC, ADVF>(ts.F, in, ts.lo, ts.g, true, ts.j0, ts.j1,
                        [&](int r, const double (&Ax)[VEC], const double (&yc)[VEC], const double (&pk)[VEC]) {
                          if (!ts.g.inside) return;
                          double yn[VEC], pn[VEC];
#pragma unroll
                          for (int v = 0; v < VEC; ++v) {
                            const double y1 = (Ax[v] - shift * yc[v]) * invg;
                            const double tt = dk1 * y1;
                            const double pv = pk[v] + tt;
                            yn[v] = y1;
                            pn[v] = pv;
                            acc[0] += tt * tt;
                            acc[1] += pv * pv;
                          }
                          const int so = r * ts.F.nx * 8;
                          bstore<VEC>(yout, ts.lo.o8, so, yn);
                          bstore<VEC>(pout, ts.lo.o8, so, pn);
                        });
  wave_sum3(acc);
  if ((threadIdx.x & 63) == 0) {
    double* part = tile_partials(A, B.tile_base + t);
    part[0] = acc[0];
    part[1] = acc[1];
    part[2] = acc[2];
    part[3] = part[4] = part[5] = 0.0;
  }
}

// The stencil coefficients of a row's VEC points (Sec. 2, eq. 3 discretised
// as in stencil_point: face averages of kxx and kyy, kxy at the four
// neighbours, the advection values with field advection), computed once by
// stage 1 and applied again by stage 2 to y_{k+1} on the same row.
template <int VEC, bool ADVF>
struct Coef {
  double kE[VEC], kW[VEC], gN[VEC], gS[VEC], mE[VEC], mW[VEC], mN[VEC], mS[VEC];
  double aE[ADVF ? VEC : 1], aW[ADVF ? VEC : 1], yN[ADVF ? VEC : 1], yS[ADVF ? VEC : 1];
};

template <int VEC, bool ADVF>
__device__ __forceinline__ void coef_of(const RowC<VEC>& gm, const RowC<VEC>& gc, const RowC<VEC>& gp,
                                        const RowN<VEC>& mm, const RowN<VEC>& mc, const RowN<VEC>& mp,
                                        const RowN<VEC>& kc, const RowN<VEC>& ac, const RowC<VEC>& ym,
                                        const RowC<VEC>& yp, Coef<VEC, ADVF>& o) {
#pragma unroll
  for (int v = 0; v < VEC; ++v) {
    o.kE[v] = 0.5 * (kc.at(v) + kc.east(v));
    o.kW[v] = 0.5 * (kc.at(v) + kc.west(v));
    o.gN[v] = 0.5 * (gc.c[v] + gp.c[v]);
    o.gS[v] = 0.5 * (gc.c[v] + gm.c[v]);
    o.mE[v] = mc.east(v);
    o.mW[v] = mc.west(v);
    o.mN[v] = mp.at(v);
    o.mS[v] = mm.at(v);
    if constexpr (ADVF) {
      o.aE[v] = ac.east(v);
      o.aW[v] = ac.west(v);
      o.yN[v] = yp.c[v];
      o.yS[v] = ym.c[v];
    }
  }
}

// (A u) at a row's VEC points from its coefficients and rows j-1 (um), j
// (uc), j+1 (up) of u; the same operations in the same order as stencil_point
template <int VEC, bool ADVF>
__device__ __forceinline__ void coef_apply(const Coef<VEC, ADVF>& c, const RowN<VEC>& um, const RowN<VEC>& uc,
                                           const RowN<VEC>& up, double axc, double ayc, double (&Ax)[VEC]) {
#pragma unroll
  for (int v = 0; v < VEC; ++v) {
    const double uC = uc.at(v), uW = uc.west(v), uE = uc.east(v);
    const double uN = up.at(v), uS = um.at(v);
    const double uNW = up.west(v), uNE = up.east(v);
    const double uSW = um.west(v), uSE = um.east(v);
    double a = c.kE[v] * (uE - uC) - c.kW[v] * (uC - uW);
    a += c.gN[v] * (uN - uC) - c.gS[v] * (uC - uS);
    a += c.mE[v] * (uNE - uSE) - c.mW[v] * (uNW - uSW);
    a += c.mN[v] * (uNE - uNW) - c.mS[v] * (uSE - uSW);
    if constexpr (ADVF) {
      a += c.aE[v] * uE - c.aW[v] * uW + c.yN[v] * uN - c.yS[v] * uS;
    } else {
      a += axc * (uE - uW) + ayc * (uN - uS);
    }
    Ax[v] = a;
  }
}

template <typename TF, int VEC, bool ADVF>
__device__ __forceinline__ void batch_term2(const BatchArgs& A, const BinDesc& B, int t) {
  // the descriptor's values, read once: a reference would be re-read after
  // every store of the tile (the compiler cannot rule out that the stores
  // overwrite the descriptor), each time waiting for the loads in flight
  FieldView F = B.f;
  F.nx = uni(F.nx);
  F.ny = uni(F.ny);
  F.bc = uni(F.bc);
  F.axc = uni(F.axc);
  F.ayc = uni(F.ayc);
  const int ncb2 = uni(B.ncb2), rows = uni(B.rows);
  const int rb = t / ncb2, cb = t - rb * ncb2;
  const int j0 = rb * rows, j1 = min(j0 + rows, F.ny);
  const int k = A.k;
  const int lane = threadIdx.x & (kWave - 1);
  const int M = uni(B.max_degree);
  const Strip g = strip_at<VEC>(F, cb * (kWave - 2) * VEC - VEC);
  const bool own = lane >= 1 && lane <= kWave - 2 && g.inside;
  const bool per = F.bc == BC_PERIODIC;
  const LaneOff lo{g.colc * 8, g.hcol * 8, g.colc * 4, g.hcol * 4, g.col0 * 8};
  TileIn in;
  in.y = rsrc_of(uni((A.L & 1) ? B.y1 : B.y0));
  in.p = rsrc_of(uni(B.pb[pbuf_index(k, A.two)]));
  in.kxx = rsrc_of(uni(F.kxx));
  in.kxy = rsrc_of(uni(F.kxy));
  in.kyy = rsrc_of(uni(F.kyy));
  if constexpr (ADVF) {
    in.ax = rsrc_of(uni(F.ax));
    in.ay = rsrc_of(uni(F.ay));
  }
  const Rsrc yout = rsrc_of(uni(((A.L + 1) & 1) ? B.y1 : B.y0));
  // (p_{k+1} is not stored: a bin that stops at term k+1 is advanced by
  // p_{k+2} - d_{k+2} y_{k+2}, both stored, in the update launch)
  const Rsrc pout = rsrc_of(uni(B.pb[pbuf_index(k + 2, A.two)]));
  // (a second term past the bin's degree cap is computed with the last plan
  // entries and discarded by the decision at the cap)
  const double shift1 = uni(B.shift[k]), shift2 = uni(B.shift[min(k + 1, M)]);
  const double dk1 = uni(B.d[k + 1]), dk2 = uni(B.d[min(k + 2, M)]);
  const double invg = uni(B.invg);
  using RY = TRow<double, VEC>;
  using RF = TRow<TF, VEC>;
  using RC = TRowC<TF, VEC>;
  using CF = Coef<VEC, ADVF>;
  // stage 1 on row s: its coefficients from the stored field rows s-1 .. s+1
  // (kept in o_c for stage 2 on the same row one step later), (A y_k)(s) from
  // the stored rows of y_k, then y_{k+1} (zero at ghost positions)
  auto stage1 = [&](int s, const RY& y0, const RY& y1, const RY& y2, const RC& g0, const RC& g1, const RC& g2,
                    const RF& m0, const RF& m1, const RF& m2, const RF& kc, const RF& xc, const RC& a0,
                    const RC& a2, CF& o_c, double (&o)[VEC]) {
    RowN<VEC> xn{};
    RowC<VEC> an0{}, an2{};
    if constexpr (ADVF) {
      xn = rown_of<TF, VEC, MODE_ZERO>(xc, g);
      an0 = rowc_of<TF, VEC>(a0);
      an2 = rowc_of<TF, VEC>(a2);
    }
    coef_of<VEC, ADVF>(rowc_of<TF, VEC>(g0), rowc_of<TF, VEC>(g1), rowc_of<TF, VEC>(g2),
                       rown_of<TF, VEC, MODE_ZERO>(m0, g), rown_of<TF, VEC, MODE_ZERO>(m1, g),
                       rown_of<TF, VEC, MODE_ZERO>(m2, g), rown_of<TF, VEC, MODE_EDGE>(kc, g), xn, an0, an2, o_c);
    const RowN<VEC> u1 = rown_of<double, VEC, MODE_ZERO>(y1, g);
    double Ax[VEC];
    coef_apply<VEC, ADVF>(o_c, rown_of<double, VEC, MODE_ZERO>(y0, g), u1, rown_of<double, VEC, MODE_ZERO>(y2, g),
                          F.axc, F.ayc, Ax);
    const bool ghost = !per && (!g.inside || s < 0 || s >= F.ny);
#pragma unroll
    for (int v = 0; v < VEC; ++v) o[v] = ghost ? 0.0 : (Ax[v] - shift1 * u1.c[v]) * invg;
  };
  // the march starts two rows above the tile: steps r = j0-2 and j0-1 only
  // compute y_{k+1} (and the coefficients) on rows j0-1 and j0.  Windows at
  // step r, as stored: y_k rows r, r+1; kyy, kxy, ay' rows r, r+1; y_{k+1}
  // rows r-1, r (za, zb); the coefficients of row r.  The step's new rows
  // (input row r+2, kxx and ax' row r+1, p_k row r) were loaded during the
  // previous step.
  StepRows<TF, VEC> s0, s1, na, nb;
  load_step_rows<TF, VEC, ADVF>(F, in, lo, false, j0 - 2, false, j0, s0);
  load_step_rows<TF, VEC, ADVF>(F, in, lo, false, j0 - 1, false, j0, s1);
  load_step_rows<TF, VEC, ADVF>(F, in, lo, false, j0, true, j0, na);
  RY wy0 = s0.y, wy1 = s1.y;
  RC wgA = s0.g, wgB = s1.g;
  RF wmA = s0.m, wmB = s1.m;
  RC waA = s0.ay, waB = s1.ay;
  double za[VEC] = {}, zb[VEC] = {};
  CF c0, c1;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  // one marching step: `held` holds the rows loaded during the previous step,
  // the next step's rows go into `nxt` (two buffers taking turns, so that no
  // register holding a load in flight is ever copied: a copy would wait for
  // it; the coefficient buffers take turns likewise).  The loads are issued
  // unconditionally (past the tile's last rows they repeat its last row), so
  // that every step has the same count of loads in flight.  s2: the step
  // computes stage 2 (not at j0-2, j0-1); lp: it loads p_k of the next step's
  // output row.
  auto step = [&](auto s2, auto lp, int r, const StepRows<TF, VEC>& held, StepRows<TF, VEC>& nxt, const CF& c_r,
                  CF& c_next) {
    // (nxt was copied out by the step before: its registers are free)
    load_step_rows<TF, VEC, ADVF>(F, in, lo, own && decltype(lp)::value, min(r + 3, j1 + 1), true,
                                  min(r + 1, j1 - 1), nxt);
    StepRows<TF, VEC> cur;
    cur.y = vcopy(held.y);
    cur.g = vcopy(held.g);
    cur.m = vcopy(held.m);
    cur.k = vcopy(held.k);
    if constexpr (ADVF) {
      cur.ax = vcopy(held.ax);
      cur.ay = vcopy(held.ay);
    }
    if constexpr (decltype(s2)::value) {
#pragma unroll
      for (int v = 0; v < VEC; ++v) cur.p[v] = own ? vcopy(held.p[v]) : 0.0;
    }
    // stage 1: y_{k+1} and the coefficients on row r+1
    double zc[VEC];
    stage1(r + 1, wy0, wy1, cur.y, wgA, wgB, cur.g, wmA, wmB, cur.m, cur.k, cur.ax, waA, cur.ay, c_next, zc);
    // stage 2: y_{k+2} on row r, with row r's coefficients from the step before
    if constexpr (decltype(s2)::value) {
      double Ax[VEC];
      coef_apply<VEC, ADVF>(c_r, rown_y1<VEC>(za), rown_y1<VEC>(zb), rown_y1<VEC>(zc), F.axc, F.ayc, Ax);
      if (own) {
        double y2[VEC], pm[VEC], p2[VEC];
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          const double t1 = dk1 * zb[v];
          pm[v] = cur.p[v] + t1;
          y2[v] = (Ax[v] - shift2 * zb[v]) * invg;
          const double t2 = dk2 * y2[v];
          p2[v] = pm[v] + t2;
          acc[0] += t1 * t1;
          acc[1] += pm[v] * pm[v];
          acc[2] += t2 * t2;
          acc[3] += p2[v] * p2[v];
        }
        const int so = r * F.nx * 8;
        bstore<VEC>(yout, lo.o8, so, y2);
        bstore<VEC>(pout, lo.o8, so, p2);
      }
    }
    // slide the windows down one row
    wy0 = wy1;
    wy1 = cur.y;
    wgA = wgB;
    wgB = cur.g;
    wmA = wmB;
    wmB = cur.m;
    if constexpr (ADVF) {
      waA = waB;
      waB = cur.ay;
    }
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      za[v] = zb[v];
      zb[v] = zc[v];
    }
  };
  using No = std::false_type;
  using Yes = std::true_type;
  step(No{}, No{}, j0 - 2, na, nb, c1, c0);
  step(No{}, Yes{}, j0 - 1, nb, na, c0, c1);
  int r = j0;
#pragma unroll 1
  for (; r + 1 < j1; r += 2) {
    step(Yes{}, Yes{}, r, na, nb, c1, c0);
    step(Yes{}, Yes{}, r + 1, nb, na, c0, c1);
  }
  if (r < j1) step(Yes{}, Yes{}, r, na, nb, c1, c0);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc[q] += __shfl_xor(acc[q], o);
  }
  if (lane == 0) {
    double* part = tile_partials(A, B.tile_base2 + t);
    part[0] = acc[0];
    part[1] = acc[1];
    part[2] = 0.0;
    part[3] = acc[2];
    part[4] = acc[3];
    part[5] = 0.0;
  }
}

template <typename TF, int VEC, bool ADVF>
__global__ __launch_bounds__(64 * kBWaves) void batch_leja2_kernel(BatchArgs A, int nbins) {
  const int w = wave_unit();
  if (w < nbins) {
    const int b = w;
    const BinDesc& B = A.bins[b];
    if (!B.active) return;
    if (__hip_atomic_load(&A.ctl[b].stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    bin_decide(A, B, b, true);
    return;
  }
  const int gt = w - nbins;
  if (gt >= A.total_tiles2) return;
  const int b = __builtin_amdgcn_readfirstlane(A.tile_bin2[gt]);
  const BinDesc& B = A.bins[b];
  if (!B.active) return;
  if (__hip_atomic_load(&A.ctl[b].stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
    const BinCtl& c = A.ctl[b];
    if (update_due(A, c)) {
      // the two-term tile's own points: rows j0 .. j0+rows-1, the strip's
      // 62*VEC output columns
      const int t = gt - B.tile_base2;
      const int rb = t / B.ncb2, cb = t - rb * B.ncb2;
      const int j0 = rb * B.rows, c0 = cb * (kWave - 2) * VEC;
      bin_update_rect<VEC>(A, B, c, const_cast<double*>(B.u), j0, min(j0 + B.rows, B.f.ny), c0,
                           min(c0 + (kWave - 2) * VEC, B.f.nx));
    }
    return;
  }
  if (A.k >= B.max_degree) return;
  batch_term2<TF, VEC, ADVF>(A, B, gt - B.tile_base2);
}

// Three terms per launch with the input rows staged in LDS: blocks [0, ndec)
// hold one decision wave per bin (as the first waves of the tile launches),
// every later block marches one run of bands3 bands (four rows each) of one
// strip of 124 output columns of one bin with staged3_run (two columns per
// lane), and stores y and p of the third term and y of the second (for the
// update of a bin whose stopping term is not the last of its launch).
// FIRST: the sweep's first launch, terms 1 .. 3 from y_0 = w, with
// p_0 = d_0 w formed in the march (no decision: no launch before it).  The block's partials (the three terms' ||d y||^2 and ||p||^2,
// summed over its waves in order) go to the unit partials of the block.
// The blocks keep dispatch order: the XCDs take them round-robin, so the
// blocks of the bins still running late in a sweep are spread over every XCD
// (an XCD-contiguous order, which lets neighbouring strips share L2, left
// those late launches to the one or two XCDs that held those bins' blocks).
constexpr int kStrip3 = (kWave - 2) * 2;  // output columns of a three-term block
// whether a bin's three-term blocks are whole-width strips: Dirichlet bins
// of 128 columns, whose ghost columns on both sides stand in for the frame
// lanes (one strip instead of two, half the work of such bins)
__host__ __device__ inline bool whole_strip(int bc, int nx) { return bc != BC_PERIODIC && nx == 2 * kWave; }


template <typename TF, bool ADVF, bool FIRST>
__global__ __launch_bounds__(kTileBlock2) void batch_leja3s_kernel(BatchArgs A, int nbins, int ndec) {
  extern __shared__ __attribute__((aligned(16))) double lds[];  // rows accessed 16 bytes per lane
  __shared__ double wsum[kWavesY2][6];
  __shared__ int bstop;
  constexpr int VEC = 2;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  if ((int)blockIdx.x < ndec) {
    const int b = (int)blockIdx.x * kWavesY2 + wave;
    if (FIRST || b >= nbins) return;
    const BinDesc& B = A.bins[b];
    if (!B.active) return;
    if (__hip_atomic_load(&A.ctl[b].stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    bin_decide(A, B, b, true);
    return;
  }
  const int bi = (int)blockIdx.x - ndec;
  const int b = __builtin_amdgcn_readfirstlane(A.block_bin3[bi]);
  const BinDesc& B = A.bins[b];
  if (!B.active) return;
  // one read of the stop flag for the whole block (its waves must agree:
  // the march has barriers)
  if (threadIdx.x == 0) bstop = __hip_atomic_load(&A.ctl[b].stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  const int stop = __builtin_amdgcn_readfirstlane(bstop);
  FieldView F = B.f;
  F.nx = uni(F.nx);
  F.ny = uni(F.ny);
  F.bc = uni(F.bc);
  F.axc = uni(F.axc);
  F.ayc = uni(F.ayc);
  const int ubase = uni(B.block_base3);
  const int t = bi - ubase;
  const int ncb3 = uni(B.ncb3), bands = uni(B.bands3);
  const int cb = t % ncb3, run = t / ncb3;
  const int nrb = (F.ny + kWavesY2 - 1) / kWavesY2;
  const int rb0 = run * bands, rb1 = min(rb0 + bands, nrb);
  // a Dirichlet bin 128 columns wide is one strip of all 64 lanes
  const bool whole = whole_strip(F.bc, F.nx);
  const int c0 = whole ? 0 : cb * kStrip3, c1 = whole ? F.nx : min(c0 + kStrip3, F.nx);
  if (stop) {
    const BinCtl& c = A.ctl[b];
    if (update_due(A, c)) {
      // the block's own points, a quarter of its rows per wave
      const int j0 = rb0 * kWavesY2, j1 = min(rb1 * kWavesY2, F.ny);
      const int q = (j1 - j0 + kWavesY2 - 1) / kWavesY2;
      bin_update_rect<VEC>(A, B, c, const_cast<double*>(B.u), j0 + wave * q, min(j0 + (wave + 1) * q, j1), c0, c1);
    }
    return;
  }
  const int k = A.k;
  const int M = uni(B.max_degree);
  if (k >= M) return;
  Staged3IO<double> io;
  io.yin = FIRST ? uni(static_cast<const double*>(B.w))
                 : uni(reinterpret_cast<const double*>((A.L & 1) ? B.y1 : B.y0));
  io.yout = uni(reinterpret_cast<double*>(((A.L + 1) & 1) ? B.y1 : B.y0));
  io.p = uni(B.pb[pbuf_out3(A.L)]);
  io.pin = FIRST ? io.p : uni(B.pb[pbuf_in3(A.L)]);  // (FIRST: not read)
  io.p1 = nullptr;
  io.p2 = nullptr;
  io.d0 = uni(B.d[0]);
  io.y2out = uni(B.y2b[A.L & 1]);
  // (terms past the bin's degree cap are computed with the last plan entries
  // and discarded by the decision at the cap)
  io.shift = uni(B.shift[k]);
  io.shift2 = uni(B.shift[min(k + 1, M)]);
  io.shift3 = uni(B.shift[min(k + 2, M)]);
  io.invg = uni(B.invg);
  io.dk1 = uni(B.d[k + 1]);
  io.dk2 = uni(B.d[min(k + 2, M)]);
  io.dk3 = uni(B.d[min(k + 3, M)]);
  double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double amax = 0.0;  // (the decision tests y_0 = 0 from the first term and p_1)
  staged3_run<TF, double, VEC, ADVF, true, true, FIRST>(F, io, lds, whole ? 0 : c0 - VEC, rb0, rb1, 0, acc, amax,
                                                        whole);
#pragma unroll
  for (int q = 0; q < 6; ++q) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc[q] += __shfl_xor(acc[q], o);
  }
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int q = 0; q < 6; ++q) wsum[wave][q] = acc[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      tot[q] = wsum[0][q];
#pragma unroll
      for (int w = 1; w < kWavesY2; ++w) tot[q] += wsum[w][q];
    }
    double* part = tile_partials(A, (long)ubase + t);
    part[0] = tot[0];
    part[1] = tot[1];
    part[2] = tot[4];
    part[3] = tot[2];
    part[4] = tot[3];
    part[5] = tot[5];
  }
}

// decision of the last launch for every running bin: one wave per bin
__global__ __launch_bounds__(64) void batch_finalize_kernel(BatchArgs A, int nbins) {
  const int b = blockIdx.x;
  if (b >= nbins) return;
  const BinDesc& B = A.bins[b];
  if (!B.active) return;
  if (__hip_atomic_load(&A.ctl[b].stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  if (A.L > 0) bin_decide(A, B, b, true);
}

__global__ __launch_bounds__(256) void batch_reset_kernel(BinCtl* ctl, int nbins) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nbins) {
    BinCtl c{};
    c.launch = kNoLaunch;
    ctl[b] = c;
  }
}

// u_b += dt p_b for converged bins not advanced yet (one wave per tile).  A
// bin that stopped at the first term m of a two-term launch is advanced by
// p_m = p_{m+1} - d_{m+1} y_{m+1}: that launch stored p and y of term m+1
// only, and no later launch of the sweep wrote those buffers of the bin (the
// launch beside the decision writes the other y buffer and the other p pair).
// A.L = the number of term launches the sweep has enqueued; a bin whose due
// launch (c.launch + 2) is among them was advanced there.
template <int VEC>
__global__ __launch_bounds__(64 * kBWaves) void batch_update_kernel(BatchArgs A, double* const* u) {
  const int gt = wave_unit();
  if (gt >= A.total_tiles) return;
  const int b = __builtin_amdgcn_readfirstlane(A.tile_bin[gt]);
  const BinDesc& B = A.bins[b];
  const BinCtl& c = A.ctl[b];
  if (!B.active || c.status != 1 || c.upd || c.degree == 0) return;  // degree 0: p = 0
  if (c.launch + 2 < A.L) return;                                      // advanced in its due launch
  const int t = gt - B.tile_base;
  const int rb = t / B.ncb, cb = t - rb * B.ncb;
  const int j0 = rb * B.rows, j1 = min(j0 + B.rows, B.f.ny);
  const int c0 = cb * kWave * VEC;
  bin_update_rect<VEC>(A, B, c, u[b], j0, j1, c0, min(c0 + kWave * VEC, B.f.nx));
}

// Before a step's sweep continues past the graph: bins that have converged
// were advanced by the graph's update launch; mark them so that the update
// after the continuation leaves them alone.
__global__ __launch_bounds__(256) void batch_mark_kernel(BinCtl* ctl, int nbins) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nbins && ctl[b].status == 1) ctl[b].upd = 1;
}

// The bins' outcomes for the host: one wave copies the control blocks into
// coherent pinned host memory, releases them at system scope, then writes
// the step's publication number (a device counter it advances), which the
// host spins on instead of copying the blocks back and synchronising.
__global__ __launch_bounds__(64) void batch_publish_kernel(const BinCtl* __restrict__ ctl, BinCtl* hbins, int nbins,
                                                           int* dseq, int* hseq) {
  const int lane = threadIdx.x;
  for (int b = lane; b < nbins; b += 64) hbins[b] = ctl[b];
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");  // system scope: the copies before the number
  if (lane == 0) {
    const int s = *dseq + 1;
    *dseq = s;
    __hip_atomic_store(hseq, s, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

}  // namespace adl

using namespace adl;

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct adl_batch {
  std::vector<adl_op*> ops;
  int nbins = 0;
  int vec = 1;
  int f32 = 0;
  bool advf = false;
  int rows = 16;
  int max_degree = kMaxDegreeDefault;
  // workspace slices
  char* ws = nullptr;
  size_t ws_bytes = 0;
  BinDesc* d_bins = nullptr;
  BinCtl* d_ctl = nullptr;
  int* d_tile_bin = nullptr;
  int* d_tile_bin2 = nullptr;
  int* d_block_bin3 = nullptr;
  double* d_partials = nullptr;
  double* d_plans = nullptr;   // nbins x 2 x M
  double** d_uptrs = nullptr;  // nbins
  int* d_seq = nullptr;        // publications so far (device counter)
  // the bins' outcomes as published (coherent pinned host memory): a 64-byte
  // header whose first int is the publication number, then nbins control
  // blocks; hmir_dev is its device address
  unsigned char* hmir = nullptr;
  unsigned char* hmir_dev = nullptr;
  int pubs = 0;                // publications enqueued for execution
  const BinCtl* h_ctl = nullptr;  // the published control blocks (in hmir)
  int total_tiles = 0;
  int total_tiles2 = 0;
  int total_blocks3 = 0;
  long part_stride = 0;  // doubles per launch parity of the partials
  int two = 1;           // two Newton terms per launch after the first
  int three = 0;         // three (LDS-staged blocks; all bins two columns per lane)
  std::vector<BinDesc> bins;
  std::vector<int> tile_bin, tile_bin2, block_bin3;
  std::vector<double> order_key;  // |alpha| dt of each bin's plan (three-term block order)
  // launch state of the sweep being enqueued: launches so far, and the last
  // launch's terms-before and term count (restored after a graph replay)
  int sL = 0, skprev = 0, snprev = 0;
  int gL = 0, gkprev = 0, gnprev = 0, gcovered = 0;
  // plan keys uploaded to d_plans
  std::vector<double> plan_alpha, plan_dt;
  // graph
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<const double*> g_u, g_S;
  double g_dt = 0.0, g_tol = 0.0;
  int g_launches = 0;
  int g_rows = 0;
  int predicted = 0;
};

namespace {

// errors of the batch entry points go to the library's thread-local message
// (adl_last_error), like every other entry point's
int bfail(int code, const char* msg) { return adl::set_error(code, "batch: %s", msg); }

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// two-term tiles: strips of 62*vec output columns (at least as many as the
// one-term tiles of 64*vec columns)
int tiles2_of(int nx, int ny, int vec, int rows) {
  const int w = (kWave - 2) * vec;
  const int ncb = (nx + w - 1) / w;
  const int nrb = (ny + rows - 1) / rows;
  return ncb * nrb;
}

struct BLayout {
  size_t bins, ctl, tile_bin, tile_bin2, block_bin3, partials, plans, uptrs, seq, total;
};

BLayout blayout(int nbins, long max_tiles, int M) {
  BLayout L{};
  size_t o = 0;
  auto take = [&](size_t n) {
    const size_t at = o;
    o = al256(o + n);
    return at;
  };
  L.bins = take(sizeof(BinDesc) * nbins);
  L.ctl = take(sizeof(BinCtl) * nbins);
  L.tile_bin = take(sizeof(int) * max_tiles);
  L.tile_bin2 = take(sizeof(int) * max_tiles);
  L.block_bin3 = take(sizeof(int) * max_tiles);
  L.partials = take(sizeof(double) * 2 * 6 * max_tiles);
  L.plans = take(sizeof(double) * 2 * (size_t)M * nbins);
  L.uptrs = take(sizeof(double*) * nbins);
  L.seq = take(256);
  L.total = o;
  return L;
}

// the most tiles of either kind (one column per lane, one row per tile)
long max_tiles_for(int nbins, adl_op* const* ops) {
  long t = 0;
  for (int b = 0; b < nbins; ++b) t += tiles2_of(ops[b]->nx, ops[b]->ny, 1, 1);
  return t;
}

#define BCHK(expr)                                            \
  do {                                                        \
    hipError_t e_ = (expr);                                   \
    if (e_ != hipSuccess) return bfail(ADL_EHIP, hipGetErrorString(e_)); \
  } while (0)

// The three-term blocks bin by bin in order of decreasing |alpha| dt (the
// bins' order keys): the stiffest bins, whose sweeps run longest, come
// first, so that in the late launches, where only they still run, their
// blocks start at once instead of after the blocks of the bins that have
// stopped (at 256 C4 bins: 3.13-3.24 -> 2.95-3.05 ms per step).
void order_blocks3(adl_batch* B) {
  B->block_bin3.clear();
  int base3 = 0;
  if (B->vec == 2) {
    std::vector<int> ord(B->nbins);
    for (int b = 0; b < B->nbins; ++b) ord[b] = b;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return B->order_key[a] > B->order_key[b]; });
    for (int b : ord) {
      BinDesc& d = B->bins[b];
      d.block_base3 = base3;
      for (int t = 0; t < d.nblocks3; ++t) B->block_bin3.push_back(b);
      base3 += d.nblocks3;
    }
  }
  B->total_blocks3 = base3;
}

void build_tiles(adl_batch* B) {
  B->tile_bin.clear();
  B->tile_bin2.clear();
  B->block_bin3.clear();
  int base = 0, base2 = 0;
  for (int b = 0; b < B->nbins; ++b) {
    adl_op* op = B->ops[b];
    BinDesc& d = B->bins[b];
    const int nrb = (op->ny + B->rows - 1) / B->rows;
    d.ncb = (op->nx + kWave * B->vec - 1) / (kWave * B->vec);
    d.rows = B->rows;
    d.ntiles = d.ncb * nrb;
    d.tile_base = base;
    d.ncb2 = (op->nx + (kWave - 2) * B->vec - 1) / ((kWave - 2) * B->vec);
    d.ntiles2 = d.ncb2 * nrb;
    d.tile_base2 = base2;
    for (int t = 0; t < d.ntiles; ++t) B->tile_bin.push_back(b);
    for (int t = 0; t < d.ntiles2; ++t) B->tile_bin2.push_back(b);
    base += d.ntiles;
    base2 += d.ntiles2;
    // three-term blocks (two columns per lane only): runs of `rows` bands
    // of four rows, i.e. a tile height of 16 rows gives runs of 64 rows
    if (B->vec == 2) {
      const int nband = (op->ny + kWavesY2 - 1) / kWavesY2;
      d.ncb3 = whole_strip(op->bc, op->nx) ? 1 : (op->nx + kStrip3 - 1) / kStrip3;
      d.bands3 = B->rows;
      d.nblocks3 = d.ncb3 * ((nband + d.bands3 - 1) / d.bands3);
    }
  }
  B->total_tiles = base;
  B->total_tiles2 = base2;
  order_blocks3(B);
}

int upload_tiles(adl_batch* B) {
  BCHK(hipMemcpy(B->d_tile_bin, B->tile_bin.data(), sizeof(int) * B->total_tiles, hipMemcpyHostToDevice));
  BCHK(hipMemcpy(B->d_tile_bin2, B->tile_bin2.data(), sizeof(int) * B->total_tiles2, hipMemcpyHostToDevice));
  if (B->total_blocks3 > 0)
    BCHK(hipMemcpy(B->d_block_bin3, B->block_bin3.data(), sizeof(int) * B->total_blocks3, hipMemcpyHostToDevice));
  return ADL_OK;
}

template <typename F>
void dispatch(const adl_batch* B, F&& f) {
  if (B->vec == 2) {
    if (B->f32) {
      if (B->advf) f.template operator()<float, 2, true>(); else f.template operator()<float, 2, false>();
    } else {
      if (B->advf) f.template operator()<double, 2, true>(); else f.template operator()<double, 2, false>();
    }
  } else {
    if (B->f32) {
      if (B->advf) f.template operator()<float, 1, true>(); else f.template operator()<float, 1, false>();
    } else {
      if (B->advf) f.template operator()<double, 1, true>(); else f.template operator()<double, 1, false>();
    }
  }
}

BatchArgs base_args(const adl_batch* B) {
  BatchArgs a{};
  a.bins = B->d_bins;
  a.tile_bin = B->d_tile_bin;
  a.tile_bin2 = B->d_tile_bin2;
  a.block_bin3 = B->d_block_bin3;
  a.ctl = B->d_ctl;
  a.partials = B->d_partials;
  a.total_tiles = B->total_tiles;
  a.total_tiles2 = B->total_tiles2;
  a.total_blocks3 = B->total_blocks3;
  a.part_stride = B->part_stride;
  a.two = B->two;
  a.three = B->three;
  return a;
}

// Enqueue launches covering terms k0+1 .. k0+nterms at least (reset and stage
// first when with_stage), then the decision of the last launch.  Three-term
// sweeps take three terms in every launch; otherwise the first term is a
// launch of its own and later launches take two terms while the batch fuses
// terms and the second stays within the degree cap.  `covered` returns
// the number of terms enqueued (nterms, or one more).  advance = false (the
// autotuner's timing runs): no tile advances u.
int enqueue_sweep(adl_batch* B, int k0, int nterms, bool with_stage, hipStream_t st, int* covered = nullptr,
                  bool advance = true) {
  BatchArgs a = base_args(B);
  a.advance = advance ? 1 : 0;

  if (with_stage) {
    hipLaunchKernelGGL(batch_reset_kernel, dim3((B->nbins + 255) / 256), dim3(256), 0, st, B->d_ctl, B->nbins);
    dispatch(B, [&]<typename TF, int VEC, bool ADVF>() {
      hipLaunchKernelGGL((batch_stage_kernel<TF, VEC, ADVF>), dim3(blocks_for(B->total_tiles)), dim3(64 * kBWaves),
                         0, st, a);
    });
    B->sL = B->skprev = B->snprev = 0;
  }
  int k = k0;
  while (k < k0 + nterms) {
    // three-term sweeps run three terms in every launch, the first included
    // (terms past a bin's degree cap are discarded by its decision there)
    const int n = B->three ? 3 : (k == 0 || !B->two || k + 2 > B->max_degree) ? 1 : 2;
    a.L = B->sL;
    a.k = k;
    a.kprev = B->skprev;
    a.nprev = B->snprev;
    if (n == 1) {
      const dim3 grid(blocks_for((long)B->nbins + B->total_tiles)), blk(64 * kBWaves);
      dispatch(B, [&]<typename TF, int VEC, bool ADVF>() {
        if (a.k == 0)
          hipLaunchKernelGGL((batch_leja_kernel<TF, VEC, ADVF, true>), grid, blk, 0, st, a, B->nbins);
        else
          hipLaunchKernelGGL((batch_leja_kernel<TF, VEC, ADVF, false>), grid, blk, 0, st, a, B->nbins);
      });
    } else if (n == 2) {
      const dim3 grid(blocks_for((long)B->nbins + B->total_tiles2)), blk(64 * kBWaves);
      dispatch(B, [&]<typename TF, int VEC, bool ADVF>() {
        hipLaunchKernelGGL((batch_leja2_kernel<TF, VEC, ADVF>), grid, blk, 0, st, a, B->nbins);
      });
    } else {
      // decision blocks first (one wave per bin)
      const int ndec = (B->nbins + kWavesY2 - 1) / kWavesY2;
      const dim3 grid(ndec + B->total_blocks3), blk(kTileBlock2);
      dispatch(B, [&]<typename TF, int VEC, bool ADVF>() {
        if constexpr (VEC == 2) {
          const size_t lds = staged3_lds_bytes<2, ADVF>();
          if (a.k == 0)
            hipLaunchKernelGGL((batch_leja3s_kernel<TF, ADVF, true>), grid, blk, lds, st, a, B->nbins, ndec);
          else
            hipLaunchKernelGGL((batch_leja3s_kernel<TF, ADVF, false>), grid, blk, lds, st, a, B->nbins, ndec);
        }
      });
    }
    B->skprev = k;
    B->snprev = n;
    ++B->sL;
    k += n;
  }
  a.L = B->sL;
  a.k = k;
  a.kprev = B->skprev;
  a.nprev = B->snprev;
  hipLaunchKernelGGL(batch_finalize_kernel, dim3(B->nbins), dim3(64), 0, st, a, B->nbins);
  BCHK(hipGetLastError());
  if (covered) *covered = k - k0;
  return ADL_OK;
}

// After a sweep's launches: u_b += dt p_b for the bins converged and not yet
// advanced, then the outcomes published to the host mirror.
int enqueue_tail(adl_batch* B, hipStream_t st) {
  BatchArgs a = base_args(B);
  a.L = B->sL;
  if (B->vec == 2)
    hipLaunchKernelGGL((batch_update_kernel<2>), dim3(blocks_for(B->total_tiles)), dim3(64 * kBWaves), 0, st, a,
                       B->d_uptrs);
  else
    hipLaunchKernelGGL((batch_update_kernel<1>), dim3(blocks_for(B->total_tiles)), dim3(64 * kBWaves), 0, st, a,
                       B->d_uptrs);
  hipLaunchKernelGGL(batch_publish_kernel, dim3(1), dim3(64), 0, st, B->d_ctl,
                     reinterpret_cast<BinCtl*>(B->hmir_dev + 64), B->nbins, B->d_seq,
                     reinterpret_cast<int*>(B->hmir_dev));
  BCHK(hipGetLastError());
  return ADL_OK;
}

// Waits until publication number `want` has reached the host mirror (the
// stream is queried every 50 us so that a failed launch ends the wait).
int await_publication(adl_batch* B, int want, hipStream_t st) {
  const int* h = reinterpret_cast<const int*>(B->hmir);
  auto seen = [&] { return __atomic_load_n(h, __ATOMIC_ACQUIRE) == want; };
  auto next = std::chrono::steady_clock::now() + std::chrono::microseconds(50);
  while (!seen()) {
    __builtin_ia32_pause();
    const auto now = std::chrono::steady_clock::now();
    if (now < next) continue;
    next = now + std::chrono::microseconds(50);
    const hipError_t q = hipStreamQuery(st);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess) return bfail(ADL_EHIP, hipGetErrorString(q));
    if (seen()) break;
    return bfail(ADL_EHIP, "batched step ended without publishing its outcome");
  }
  return ADL_OK;
}

int upload_bins(adl_batch* B, double* const* u, const double* const* S, double dt, double tol, hipStream_t st,
                bool& changed) {
  changed = false;
  const int M = B->max_degree + 1;
  std::vector<double> planbuf;
  bool plans_changed = false;
  for (int b = 0; b < B->nbins; ++b) {
    adl_op* op = B->ops[b];
    BinDesc& d = B->bins[b];
    const double* Sb = S ? S[b] : nullptr;
    const int K = substeps_for(op->alpha, dt, op->rho_max);
    const bool active = op->has_bound && op->alpha < 0.0 && K == 1;
    if (d.u != u[b] || d.S != Sb || d.dt != dt || d.tol != tol || d.active != (int)active) changed = true;
    d.f = op->f;
    d.u = u[b];
    d.S = Sb;
    d.w = op->w1;
    d.y0 = op->ybuf[0];
    d.y1 = op->ybuf[1];
    d.pb[0] = op->p2;
    d.pb[1] = op->p;
    d.pb[2] = op->p3;
    d.pb[3] = op->p4;
    // three-term sweeps use pb[0], pb[1] only: the other two hold the y of
    // the second-to-last term of each launch
    d.y2b[0] = reinterpret_cast<float*>(op->p3);
    d.y2b[1] = reinterpret_cast<float*>(op->p4);
    d.tol = tol;
    d.dt = dt;
    d.max_degree = std::min(op->max_degree, B->max_degree);
    d.active = active;
    d.d = B->d_plans + (size_t)b * 2 * M;
    d.shift = d.d + M;
    if (active && (B->plan_alpha[b] != op->alpha || B->plan_dt[b] != dt)) {
      if (!plans_changed) BCHK(hipStreamSynchronize(st));
      Plan& P = get_plan(op, 1, op->alpha, dt);
      d.invg = P.invg;
      planbuf.assign(2 * (size_t)M, 0.0);
      std::copy(P.d.begin(), P.d.begin() + std::min((int)P.d.size(), M), planbuf.begin());
      std::copy(P.shift.begin(), P.shift.begin() + std::min((int)P.shift.size(), M), planbuf.begin() + M);
      BCHK(hipMemcpy(B->d_plans + (size_t)b * 2 * M, planbuf.data(), planbuf.size() * sizeof(double),
                     hipMemcpyHostToDevice));
      B->plan_alpha[b] = op->alpha;
      B->plan_dt[b] = dt;
      B->order_key[b] = std::fabs(op->alpha) * dt;
      plans_changed = true;
    }
  }
  if (plans_changed && B->vec == 2) {
    // (the stream was synchronised above: no launch still reads the table)
    order_blocks3(B);
    if (B->total_blocks3 > 0)
      BCHK(hipMemcpy(B->d_block_bin3, B->block_bin3.data(), sizeof(int) * B->total_blocks3, hipMemcpyHostToDevice));
  }
  if (changed || plans_changed) {
    BCHK(hipStreamSynchronize(st));
    BCHK(hipMemcpy(B->d_bins, B->bins.data(), sizeof(BinDesc) * B->nbins, hipMemcpyHostToDevice));
    std::vector<double*> up(u, u + B->nbins);
    BCHK(hipMemcpy(B->d_uptrs, up.data(), sizeof(double*) * B->nbins, hipMemcpyHostToDevice));
    changed = true;
  }
  (void)st;
  return ADL_OK;
}

// Autotune results of this process, by tuning key.
std::mutex& tune_cache_mu() {
  static std::mutex m;
  return m;
}
std::map<std::string, std::pair<int, double>>& tune_cache() {
  static std::map<std::string, std::pair<int, double>> c;
  return c;
}

// The tuning key of a batch: the GPU's architecture, the storage and
// advection kind, the columns per lane, the Newton terms per launch, the
// candidate heights and the multiset of the bins' grid shapes (nx x ny).
int autotune_key(const adl_batch* B, const int* candidates, int ncand, std::string& key) {
  int dev = 0;
  BCHK(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  BCHK(hipGetDeviceProperties(&prop, dev));
  std::vector<std::pair<int, int>> shapes;
  shapes.reserve(B->nbins);
  for (const adl_op* op : B->ops) shapes.emplace_back(op->nx, op->ny);
  std::sort(shapes.begin(), shapes.end());
  key = std::string(prop.gcnArchName) + "|f32=" + std::to_string(B->f32) + "|adv=" + std::to_string((int)B->advf) +
        "|vec=" + std::to_string(B->vec) + "|two=" + std::to_string(B->two) +
        "|three=" + std::to_string(B->three) + "|cand=";
  for (int c = 0; c < ncand; ++c) key += std::to_string(candidates[c]) + ",";
  key += "|bins=";
  for (const auto& sh : shapes) key += std::to_string(sh.first) + "x" + std::to_string(sh.second) + ",";
  return ADL_OK;
}

int predicted_terms(adl_batch* B, double dt) {
  int mx = 0;
  for (int b = 0; b < B->nbins; ++b) {
    adl_op* op = B->ops[b];
    if (!B->bins[b].active) continue;
    Plan& P = get_plan(op, 1, op->alpha, dt);
    const int m = P.last_degree > 0 ? P.last_degree + 1 : (int)(5.0 * std::sqrt(std::fabs(op->alpha) * dt) + 8.0);
    mx = std::max(mx, m);
  }
  return std::min(std::max(mx, 1), B->max_degree);
}

}  // namespace

extern "C" {

size_t adl_batch_workspace_bytes(int nbins, adl_op* const* ops, int max_degree) {
  if (nbins < 1 || !ops) return 0;
  for (int b = 0; b < nbins; ++b)
    if (!ops[b]) return 0;
  const int M = (max_degree > 0 ? max_degree : kMaxDegreeDefault) + 1;
  return blayout(nbins, max_tiles_for(nbins, ops), M).total;
}

int adl_batch_create(int nbins, adl_op* const* ops, void* workspace, size_t ws_bytes, int tile_rows,
                     adl_batch** out) {
  if (!out) return bfail(ADL_EINVAL, "null out");
  *out = nullptr;
  if (nbins < 1 || !ops) return bfail(ADL_EINVAL, "need nbins >= 1 ops");
  for (int b = 0; b < nbins; ++b)
    if (!ops[b]) return bfail(ADL_EINVAL, "null op in batch");
  const int f32 = ops[0]->f.f32;
  const bool advf = ops[0]->f.ax != nullptr;
  bool all_even = true;
  for (int b = 0; b < nbins; ++b) {
    adl_op* op = ops[b];
    if (op->f.f32 != f32 || (op->f.ax != nullptr) != advf)
      return bfail(ADL_EINVAL, "all bins must share storage mode and advection kind");
    if (op->storage == ADL_STORAGE_FP32_FIELDS_Y) return bfail(ADL_EINVAL, "batch supports FP64 Newton vectors only");
    if (op->nx % 2 != 0 || op->nx < 2 * kWave) all_even = false;
    // (the two-term kernel addresses a vector with 32-bit byte offsets)
    if ((long)op->nx * op->ny * 8 > 0x7fffffffL) return bfail(ADL_EINVAL, "batch bins are limited to 2^28 points");
  }
  if (tile_rows < 0) return bfail(ADL_EINVAL, "tile_rows must be >= 0");
  const int M = kMaxDegreeDefault + 1;
  const long mt = max_tiles_for(nbins, ops);
  const BLayout L = blayout(nbins, mt, M);
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255)) return bfail(ADL_ENOWORKSPACE, "workspace missing or not 256-byte aligned");
  if (ws_bytes < L.total) return bfail(ADL_ENOWORKSPACE, "batch workspace too small");
  adl_batch* B = new (std::nothrow) adl_batch();
  if (!B) return bfail(ADL_EINVAL, "out of host memory");
  B->ops.assign(ops, ops + nbins);
  B->nbins = nbins;
  B->vec = all_even ? 2 : 1;
  // three terms per launch by default where every bin allows them (C4, 256
  // bins: 3.63-3.67 ms per step with two terms per launch, 2.94-3.02 with three)
  B->three = all_even ? 1 : 0;
  B->f32 = f32;
  B->advf = advf;
  B->rows = tile_rows > 0 ? tile_rows : 16;
  B->ws = reinterpret_cast<char*>(workspace);
  B->ws_bytes = ws_bytes;
  B->d_bins = reinterpret_cast<BinDesc*>(B->ws + L.bins);
  B->d_ctl = reinterpret_cast<BinCtl*>(B->ws + L.ctl);
  B->d_tile_bin = reinterpret_cast<int*>(B->ws + L.tile_bin);
  B->d_tile_bin2 = reinterpret_cast<int*>(B->ws + L.tile_bin2);
  B->d_block_bin3 = reinterpret_cast<int*>(B->ws + L.block_bin3);
  B->part_stride = 6 * mt;
  B->d_partials = reinterpret_cast<double*>(B->ws + L.partials);
  B->d_plans = reinterpret_cast<double*>(B->ws + L.plans);
  B->d_uptrs = reinterpret_cast<double**>(B->ws + L.uptrs);
  B->bins.assign(nbins, BinDesc{});
  B->order_key.assign(nbins, 0.0);
  B->plan_alpha.assign(nbins, NAN);
  B->plan_dt.assign(nbins, NAN);
  build_tiles(B);
  hipError_t e = hipMemcpy(B->d_tile_bin, B->tile_bin.data(), sizeof(int) * B->total_tiles, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(B->d_tile_bin2, B->tile_bin2.data(), sizeof(int) * B->total_tiles2, hipMemcpyHostToDevice);
  if (e == hipSuccess && B->total_blocks3 > 0)
    e = hipMemcpy(B->d_block_bin3, B->block_bin3.data(), sizeof(int) * B->total_blocks3, hipMemcpyHostToDevice);
  B->d_seq = reinterpret_cast<int*>(B->ws + L.seq);
  if (e == hipSuccess) e = hipMemset(B->d_seq, 0, sizeof(int));
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void**>(&B->hmir), 64 + sizeof(BinCtl) * nbins,
                      hipHostMallocCoherent | hipHostMallocMapped | hipHostMallocPortable);
  if (e == hipSuccess) {
    std::memset(B->hmir, 0, 64 + sizeof(BinCtl) * nbins);
    e = hipHostGetDevicePointer(reinterpret_cast<void**>(&B->hmir_dev), B->hmir, 0);
  }
  if (e == hipSuccess) e = hipStreamCreate(&B->cap_stream);
  if (e != hipSuccess) {
    if (B->hmir) hipHostFree(B->hmir);
    delete B;
    return bfail(ADL_EHIP, hipGetErrorString(e));
  }
  B->h_ctl = reinterpret_cast<const BinCtl*>(B->hmir + 64);
  *out = B;
  return ADL_OK;
}

int adl_batch_destroy(adl_batch* B) {
  if (!B) return ADL_OK;
  if (B->cap_stream) (void)hipStreamSynchronize(B->cap_stream);
  if (B->gexec) hipGraphExecDestroy(B->gexec);
  if (B->graph) hipGraphDestroy(B->graph);
  if (B->cap_stream) hipStreamDestroy(B->cap_stream);
  if (B->hmir) {
    (void)hipDeviceSynchronize();  // no publication of this batch may still be in flight
    hipHostFree(B->hmir);
  }
  delete B;
  return ADL_OK;
}

int adl_batch_set_tile_rows(adl_batch* B, int rows) {
  if (!B || rows < 1) return bfail(ADL_EINVAL, "tile rows must be positive");
  if (rows == B->rows) return ADL_OK;
  B->rows = rows;
  build_tiles(B);
  const int rc = upload_tiles(B);
  if (rc != ADL_OK) return rc;
  BCHK(hipMemcpy(B->d_bins, B->bins.data(), sizeof(BinDesc) * B->nbins, hipMemcpyHostToDevice));
  BCHK(hipStreamSynchronize(B->cap_stream));
  if (B->gexec) {
    hipGraphExecDestroy(B->gexec);
    B->gexec = nullptr;
  }
  if (B->graph) {
    hipGraphDestroy(B->graph);
    B->graph = nullptr;
  }
  return ADL_OK;
}

int adl_batch_set_term_fusion(adl_batch* B, int mode) {
  if (!B || (mode != 0 && mode != 1 && mode != 3)) return bfail(ADL_EINVAL, "term fusion mode must be 0, 1 or 3");
  if (mode == 3 && B->vec != 2)
    return bfail(ADL_EINVAL, "three terms per launch need every bin at two columns per lane (nx even, >= 128)");
  const int two = mode != 0, three = mode == 3;
  if (two == B->two && three == B->three) return ADL_OK;
  B->two = two;
  B->three = three;
  BCHK(hipStreamSynchronize(B->cap_stream));
  if (B->gexec) {
    hipGraphExecDestroy(B->gexec);
    B->gexec = nullptr;
  }
  if (B->graph) {
    hipGraphDestroy(B->graph);
    B->graph = nullptr;
  }
  return ADL_OK;
}

int adl_batch_get_tile_rows(const adl_batch* B, int* rows) {
  if (!B || !rows) return bfail(ADL_EINVAL, "null argument");
  *rows = B->rows;
  return ADL_OK;
}

// Project autotuner: time the stage + sweep launches of one step (u is not
// modified) for each candidate tile height and keep the fastest.  Results are
// cached per process by the tuning key (autotune_key): a later call with the
// same key installs the cached tile height without timing.
int adl_batch_autotune(adl_batch* B, double* const* u, const double* const* S_half, double dt, double tol,
                       const int* candidates, int ncand, int* best_rows, double* best_ms, void* stream) {
  if (!B || !u || !candidates || ncand < 1) return bfail(ADL_EINVAL, "bad autotune arguments");
  for (int c = 0; c < ncand; ++c)
    if (candidates[c] < 1) return bfail(ADL_EINVAL, "tile height candidates must be positive");
  std::string key;
  {
    const int rc = autotune_key(B, candidates, ncand, key);
    if (rc != ADL_OK) return rc;
  }
  {
    std::lock_guard<std::mutex> g(tune_cache_mu());
    auto it = tune_cache().find(key);
    if (it != tune_cache().end()) {
      const int rc = adl_batch_set_tile_rows(B, it->second.first);
      if (rc != ADL_OK) return rc;
      if (best_rows) *best_rows = it->second.first;
      if (best_ms) *best_ms = it->second.second;
      return ADL_OK;
    }
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  int best = B->rows;
  double bms = INFINITY;
  hipEvent_t e0, e1;
  BCHK(hipEventCreate(&e0));
  BCHK(hipEventCreate(&e1));
  for (int c = 0; c < ncand; ++c) {
    int rc = adl_batch_set_tile_rows(B, candidates[c]);
    if (rc != ADL_OK) return rc;
    bool changed;
    rc = upload_bins(B, u, S_half, dt, tol, st, changed);
    if (rc != ADL_OK) return rc;
    const int nterms = predicted_terms(B, dt);
    float ms_min = INFINITY;
    for (int rep = 0; rep < 3; ++rep) {
      BCHK(hipEventRecord(e0, st));
      rc = enqueue_sweep(B, 0, nterms, true, st, nullptr, false);
      if (rc != ADL_OK) return rc;
      BCHK(hipEventRecord(e1, st));
      BCHK(hipEventSynchronize(e1));
      float ms;
      BCHK(hipEventElapsedTime(&ms, e0, e1));
      if (rep > 0) ms_min = std::min(ms_min, ms);
    }
    if (ms_min < bms) {
      bms = ms_min;
      best = candidates[c];
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  int rc = adl_batch_set_tile_rows(B, best);
  if (rc != ADL_OK) return rc;
  {
    std::lock_guard<std::mutex> g(tune_cache_mu());
    tune_cache()[key] = {best, bms};
  }
  if (best_rows) *best_rows = best;
  if (best_ms) *best_ms = bms;
  return ADL_OK;
}

int adl_batch_midpoint_step(adl_batch* B, double* const* u, const double* const* S_half, double dt, double tol,
                            int use_graph, adl_stats* per_bin, void* stream) {
  if (!B || !u) return bfail(ADL_EINVAL, "null batch or u");
  if (!(dt > 0.0) || !std::isfinite(dt)) return bfail(ADL_EINVAL, "dt must be finite and > 0");
  if (!(tol > 0.0 && tol < 1.0)) return bfail(ADL_EINVAL, "tol must be in (0, 1)");
  for (int b = 0; b < B->nbins; ++b) {
    if (!u[b]) return bfail(ADL_EINVAL, "null u entry");
    if (!B->ops[b]->has_bound) return bfail(ADL_EBOUND, "a bin has no spectral bound");
    if (B->vec == 2 && (reinterpret_cast<uintptr_t>(u[b]) & 15)) return bfail(ADL_EINVAL, "u must be 16-byte aligned");
    if (B->vec == 2 && S_half && S_half[b] && (reinterpret_cast<uintptr_t>(S_half[b]) & 15))
      return bfail(ADL_EINVAL, "S must be 16-byte aligned");
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  bool changed;
  int rc = upload_bins(B, u, S_half, dt, tol, st, changed);
  if (rc != ADL_OK) return rc;
  const int nterms = predicted_terms(B, dt);
  bool any_active = false;
  for (int b = 0; b < B->nbins; ++b) any_active |= B->bins[b].active != 0;

  if (any_active) {
    if (use_graph) {
      const bool rebuild = !B->gexec || changed || nterms > B->g_launches || B->g_rows != B->rows;
      if (rebuild) {
        BCHK(hipStreamSynchronize(B->cap_stream));  // the old graph has finished its last replay
        if (B->gexec) hipGraphExecDestroy(B->gexec);
        if (B->graph) hipGraphDestroy(B->graph);
        B->gexec = nullptr;
        B->graph = nullptr;
        BCHK(hipStreamBeginCapture(B->cap_stream, hipStreamCaptureModeThreadLocal));
        int cov = 0;
        rc = enqueue_sweep(B, 0, nterms, true, B->cap_stream, &cov);
        if (rc == ADL_OK) rc = enqueue_tail(B, B->cap_stream);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(B->cap_stream, &g);
        if (rc != ADL_OK) return rc;
        if (e != hipSuccess) return bfail(ADL_EHIP, hipGetErrorString(e));
        B->graph = g;
        BCHK(hipGraphInstantiate(&B->gexec, B->graph, nullptr, nullptr, 0));
        B->g_launches = nterms;
        B->g_rows = B->rows;
        B->gL = B->sL;
        B->gkprev = B->skprev;
        B->gnprev = B->snprev;
        B->gcovered = cov;
      }
      // the launch state the graph leaves behind
      B->sL = B->gL;
      B->skprev = B->gkprev;
      B->snprev = B->gnprev;
      // order the graph after prior work on the caller's stream
      hipEvent_t ev;
      BCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
      BCHK(hipEventRecord(ev, st));
      BCHK(hipStreamWaitEvent(B->cap_stream, ev, 0));
      BCHK(hipGraphLaunch(B->gexec, B->cap_stream));
      ++B->pubs;
      BCHK(hipEventRecord(ev, B->cap_stream));
      BCHK(hipStreamWaitEvent(st, ev, 0));
      BCHK(hipEventDestroy(ev));
    }
    int launched = 0;
    if (use_graph) {
      launched = B->gcovered;
    } else {
      rc = enqueue_sweep(B, 0, nterms, true, st, &launched);
      if (rc == ADL_OK) rc = enqueue_tail(B, st);
      if (rc != ADL_OK) return rc;
      ++B->pubs;
    }
    // the common path ends here: the graph (or the eager launches) advanced
    // every converged bin and published the outcomes; bins still running
    // continue (their u is advanced after the continuation)
    while (true) {
      rc = await_publication(B, B->pubs, st);
      if (rc != ADL_OK) return rc;
      bool running = false;
      for (int b = 0; b < B->nbins; ++b)
        if (B->bins[b].active && !B->h_ctl[b].stop) running = true;
      if (!running || launched >= B->max_degree) break;
      hipLaunchKernelGGL(batch_mark_kernel, dim3((B->nbins + 255) / 256), dim3(256), 0, st, B->d_ctl, B->nbins);
      BCHK(hipGetLastError());
      const int more = std::min(B->max_degree - launched, std::max(8, launched / 4));
      int cov = 0;
      rc = enqueue_sweep(B, launched, more, false, st, &cov);
      if (rc == ADL_OK) rc = enqueue_tail(B, st);
      if (rc != ADL_OK) return rc;
      ++B->pubs;
      launched += cov;
    }
  }
  // per-bin results; bins outside the kernel (substeps, zero operator) and
  // bins that hit the degree cap take the single-op path (substeps allowed)
  int result = ADL_OK;
  for (int b = 0; b < B->nbins; ++b) {
    adl_op* op = B->ops[b];
    adl_stats s{};
    int code = ADL_OK;
    bool single = !B->bins[b].active;
    if (!single) {
      const BinCtl& c = B->h_ctl[b];
      if (c.status == 1) {
        Plan& P = get_plan(op, 1, op->alpha, dt);
        P.last_degree = c.degree;
        s.matvecs = c.degree + 1;
        s.sweeps = 1;
        s.max_degree = s.last_degree = c.degree;
        s.substeps = 1;
        s.alpha = op->alpha;
      } else if (c.status == 2) {
        code = ADL_ENAN;
      } else {
        single = true;
      }
    }
    if (single) code = adl_exp_midpoint_step(op, u[b], S_half ? S_half[b] : nullptr, dt, tol, &s, stream);
    s.status = code;
    if (per_bin) per_bin[b] = s;
    if (code != ADL_OK && result == ADL_OK) result = code;
  }
  return result;
}

}  // extern "C"
