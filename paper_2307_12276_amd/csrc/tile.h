// Nine-point stencil tiles for gfx950 (direct form).
//
// A wave64 owns a strip of 64*VEC adjacent columns (VEC columns per lane) and
// computes a band of rows of that strip in groups of kGroupRows rows.  For a
// group it issues all of its loads together -- rows j-1 .. j+R of x, kyy and
// kxy (and ay'), rows j .. j+R-1 of kxx (and ax') and of the epilogue's own
// inputs -- and then computes.  Nothing is carried from one group to the
// next: a wave holds few registers, so many waves share a SIMD, and every
// load of a group is in flight at once.  The rows a group shares with the
// groups above and below are re-read through the caches (L1 inside a block,
// L2 inside an XCD), not from HBM.
//
// x-neighbours: DPP whole-wave shifts (wave_shr:1 / wave_shl:1, VALU) give a
// lane the previous lane's last column and the next lane's first column; the
// lanes at the strip edges use a halo element they load themselves.
//
// One code path serves interior and boundary tiles: row indices go through
// the boundary rule (uniform scalar code: periodic wrap, edge row, or a zero
// ghost row) and Dirichlet ghost columns are selects (zero for x, kxy, ax',
// ay'; the edge value for the face averages of kxx and kyy).  A separate
// boundary path would set the register allocation of the whole kernel.
#pragma once

#include "device.h"

namespace adl {

constexpr int kDppWaveShl1 = 0x130;  // lane i <- lane i+1
constexpr int kDppWaveShr1 = 0x138;  // lane i <- lane i-1
constexpr int kGroupRows = 1;        // rows per load group

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
// The same shift where the lane without a source gets zero by the DPP bound
// control, so no register has to hold an old value (for rows whose edge
// lanes' neighbours are not used)
template <int CTRL>
__device__ __forceinline__ double dpp_f64_any(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
// The same shift where the lane without a source (lane 0 for wave_shr:1,
// lane 63 for wave_shl:1) keeps `old` instead of zero: passing the halo
// element as `old` makes the shift deliver it to the edge lane, and no
// select and no zero register are needed.
template <int CTRL>
__device__ __forceinline__ double dpp_f64_keep(double old, double v) {
  const long long b = __double_as_longlong(v);
  const long long o = __double_as_longlong(old);
  const int lo = __builtin_amdgcn_update_dpp((int)(o & 0xffffffffll), (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

struct Strip {
  int col0;     // first column of this lane (may be >= nx in the last strip)
  int colc;     // column of this lane's own loads (in the grid)
  int hcol;     // column of this lane's halo load (in the grid)
  bool lane0, lane63;
  bool inside;  // 0 <= col0 < nx
  bool useL;    // left neighbour = halo element (lane 0)
  bool useR;    // right neighbour = halo element (lane 63)
  bool ghostL;  // Dirichlet: the left neighbour is a ghost column (lane 0 at column 0)
  bool ghostR;  // Dirichlet: the right neighbour is a ghost column (last inside lane)
};

__device__ __forceinline__ int wrap_col(int c, int nx) {
  const int m = c % nx;
  return m < 0 ? m + nx : m;
}

// Columns and neighbour sources of one lane of the strip that starts at
// column i0 (i0 may be negative and the strip may reach past nx: lanes
// outside the grid load, as their own elements, the periodic wrap of their
// columns, or a valid dummy column with Dirichlet boundaries).  Lane 0 loads
// its left halo element, lane 63 its right one; the other lanes re-read their
// own column (a cache hit), so all lanes run the same load.  The DPP shifts
// then deliver every periodic neighbour, and with Dirichlet boundaries the
// ghost neighbours of the edge columns are selects (zero, or the edge value
// for the face averages of kxx and kyy).
template <int VEC>
__device__ __forceinline__ Strip strip_at(const FieldView& F, int i0) {
  const int nx = F.nx;
  const bool per = F.bc == BC_PERIODIC;
  Strip g;
  const int lane = threadIdx.x & (kWave - 1);
  g.col0 = i0 + lane * VEC;
  g.inside = g.col0 >= 0 && g.col0 < nx;
  g.colc = g.inside ? g.col0 : (per ? wrap_col(g.col0, nx) : (g.col0 < 0 ? 0 : nx - VEC));
  g.lane0 = lane == 0;
  g.lane63 = lane == kWave - 1;
  g.useL = g.lane0;
  g.useR = g.lane63 && (g.inside || per);
  const bool lastin = g.inside && g.col0 + VEC >= nx;
  g.ghostL = !per && g.col0 == 0;
  g.ghostR = !per && lastin;
  const int cl = g.col0 - 1, cr = g.col0 + VEC;
  if (g.lane0) g.hcol = (cl >= 0 && cl < nx) ? cl : (per ? wrap_col(cl, nx) : g.colc);
  else if (g.useR) g.hcol = (cr >= 0 && cr < nx) ? cr : (per ? wrap_col(cr, nx) : g.colc);
  else g.hcol = g.colc;
  return g;
}

template <int VEC>
__device__ __forceinline__ Strip make_strip(const FieldView& F, int strip) {
  return strip_at<VEC>(F, strip * kWave * VEC);
}

// ---- row loads -------------------------------------------------------------
// Row `r` of array `a` under the boundary rule MODE: the row index is mapped
// first (uniform: periodic wrap, edge row, or a zero ghost row), then each
// lane loads its own VEC elements and one halo element; the x-neighbours
// come from the DPP shifts, the halo element or a Dirichlet ghost select.
template <typename T, int VEC, int MODE>
__device__ __forceinline__ void row_n(const T* __restrict__ a, int r, const FieldView& F, const Strip& g,
                                      RowN<VEC>& o) {
  bool zero;
  const int row = map_row(r, F.ny, F.bc, MODE, zero);
  const T* rp = a + (long)row * F.nx;
  double c[VEC];
  ldr<T, VEC>(rp, g.colc, c);
  const double h = ld1<T>(rp, g.hcol);
#pragma unroll
  for (int v = 0; v < VEC; ++v) o.c[v] = zero ? 0.0 : c[v];
  const double l = dpp_f64<kDppWaveShr1>(o.c[VEC - 1]);
  const double rr = dpp_f64<kDppWaveShl1>(o.c[0]);
  const double hz = zero ? 0.0 : h;
  // ghost neighbours: zero, or the edge value itself (face averages)
  const double gl = MODE == MODE_EDGE ? o.c[0] : 0.0;
  const double gr = MODE == MODE_EDGE ? o.c[VEC - 1] : 0.0;
  o.l = g.ghostL ? gl : (g.useL ? hz : l);
  o.r = g.ghostR ? gr : (g.useR ? hz : rr);
}

template <typename T, int VEC, int MODE>
__device__ __forceinline__ void row_c(const T* __restrict__ a, int r, const FieldView& F, const Strip& g,
                                      RowC<VEC>& o) {
  bool zero;
  const int row = map_row(r, F.ny, F.bc, MODE, zero);
  double c[VEC];
  ldr<T, VEC>(a + (long)row * F.nx, g.colc, c);
#pragma unroll
  for (int v = 0; v < VEC; ++v) o.c[v] = zero ? 0.0 : c[v];
}

// (A x) at the VEC columns of one lane for output row j, from the rows
// j-1 (um), j (uc), j+1 (up) of x, kyy (gm, gc, gp) and kxy (mm, mc, mp), the
// centre row of kxx (kc) and, with field advection, ax' (ac) and ay' (ym, yp).
template <int VEC, bool ADVF>
__device__ __forceinline__ void stencil_point(const RowN<VEC>& um, const RowN<VEC>& uc, const RowN<VEC>& up,
                                              const RowC<VEC>& gm, const RowC<VEC>& gc, const RowC<VEC>& gp,
                                              const RowN<VEC>& mm, const RowN<VEC>& mc, const RowN<VEC>& mp,
                                              const RowN<VEC>& kc, const RowN<VEC>& ac, const RowC<VEC>& ym,
                                              const RowC<VEC>& yp, double axc, double ayc, double (&Ax)[VEC]) {
#pragma unroll
  for (int v = 0; v < VEC; ++v) {
    const double uC = uc.at(v), uW = uc.west(v), uE = uc.east(v);
    const double uN = up.at(v), uS = um.at(v);
    const double uNW = up.west(v), uNE = up.east(v);
    const double uSW = um.west(v), uSE = um.east(v);
    const double kC = kc.at(v), kW = kc.west(v), kE = kc.east(v);
    const double gC = gc.c[v], gN = gp.c[v], gS = gm.c[v];
    const double mE = mc.east(v), mW = mc.west(v), mN = mp.at(v), mS = mm.at(v);
    double a = 0.5 * (kC + kE) * (uE - uC) - 0.5 * (kC + kW) * (uC - uW);
    a += 0.5 * (gC + gN) * (uN - uC) - 0.5 * (gC + gS) * (uC - uS);
    a += mE * (uNE - uSE) - mW * (uNW - uSW);
    a += mN * (uNE - uNW) - mS * (uSE - uSW);
    if constexpr (ADVF) {
      a += ac.east(v) * uE - ac.west(v) * uW + yp.c[v] * uN - ym.c[v] * uS;
    } else {
      a += axc * (uE - uW) + ayc * (uN - uS);
    }
    Ax[v] = a;
  }
}

// Rows j .. j+R-1 of the strip: all loads first, then R outputs through the
// epilogue (ep.load fetches the epilogue's inputs of a row, ep.finish consumes
// (A x) and the centre values of x; lanes outside the grid skip both).
// ep.go() is asked after the loads are issued: false drops the group and ends
// the wave's work (the epilogue's wave-uniform gate, whose own load is then
// in flight together with the group's loads).
template <typename TF, typename TX, int VEC, bool ADVF, int R, class Ep>
__device__ __forceinline__ bool stencil_group(const FieldView& F, const TX* __restrict__ x, Ep& ep,
                                              const Strip& g, int j) {
  const TF* __restrict__ kxx = reinterpret_cast<const TF*>(F.kxx);
  const TF* __restrict__ kxy = reinterpret_cast<const TF*>(F.kxy);
  const TF* __restrict__ kyy = reinterpret_cast<const TF*>(F.kyy);
  const TF* __restrict__ fax = reinterpret_cast<const TF*>(F.ax);
  const TF* __restrict__ fay = reinterpret_cast<const TF*>(F.ay);
  RowN<VEC> u[R + 2], m[R + 2], k[R], ac[R];
  RowC<VEC> gg[R + 2], ay[R + 2];
  typename Ep::Extra ex[R];
#pragma unroll
  for (int q = 0; q < R + 2; ++q) {
    const int r = j - 1 + q;
    row_n<TX, VEC, MODE_ZERO>(x, r, F, g, u[q]);
    row_c<TF, VEC, MODE_EDGE>(kyy, r, F, g, gg[q]);
    row_n<TF, VEC, MODE_ZERO>(kxy, r, F, g, m[q]);
    if constexpr (ADVF) row_c<TF, VEC, MODE_ZERO>(fay, r, F, g, ay[q]);
  }
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int r = j + q;
    row_n<TF, VEC, MODE_EDGE>(kxx, r, F, g, k[q]);
    if constexpr (ADVF) row_n<TF, VEC, MODE_ZERO>(fax, r, F, g, ac[q]);
    ep.load(r, g, ex[q]);
  }
  if (!ep.go()) return false;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    double Ax[VEC];
    stencil_point<VEC, ADVF>(u[q], u[q + 1], u[q + 2], gg[q], gg[q + 1], gg[q + 2], m[q], m[q + 1], m[q + 2],
                             k[q], ac[q], ay[q], ay[q + 2], F.axc, F.ayc, Ax);
    ep.finish(j + q, g, Ax, u[q + 1].c, ex[q]);
  }
  return true;
}

// Rows [j0, j1) of strip `strip` (one wave), in groups of kGroupRows rows.
// Returns false once the epilogue's gate has closed.
template <typename TF, typename TX, int VEC, bool ADVF, class Ep>
__device__ __forceinline__ bool stencil_tile(const FieldView& F, const TX* __restrict__ x, Ep& ep, int strip,
                                             int j0, int j1) {
  const Strip g = make_strip<VEC>(F, strip);
  constexpr int R = kGroupRows;
  int j = j0;
#pragma unroll 1
  for (; j + R <= j1; j += R)
    if (!stencil_group<TF, TX, VEC, ADVF, R>(F, x, ep, g, j)) return false;
  if constexpr (R > 1) {
#pragma unroll 1
    for (; j < j1; ++j)
      if (!stencil_group<TF, TX, VEC, ADVF, 1>(F, x, ep, g, j)) return false;
  }
  return true;
}

// ---- rows of y_{k+1} kept in LDS (two Newton terms per launch) -----------
// Stage 1 writes y_{k+1} of a strip row into a ring of LDS rows; stage 2
// reads a lane's VEC values back (rounded to the y storage type, as a
// one-term launch would read them from memory) and takes x-neighbours from
// the DPP shifts.  A lane only reads back what it wrote itself.
template <typename TY>
__device__ __forceinline__ double storage_round(double v) {
  return (double)(TY)v;
}

// stage 1 epilogue: y_{k+1} of one strip row into the LDS ring (all lanes)
constexpr int kRing = 8;  // slots of the LDS ring of y_{k+1} rows (a power of two)
static_assert(kRing >= 2 * kWavesY2, "a step writes its rows and the frame below while the previous step's "
                                     "rows are still read");
// ADD: the epilogue of a stage vector w = A x + s instead (add: the row's s
// values, set by the caller before each row)
template <int VEC, int NR = kRing, bool ADD = false>
struct Stage1Ep {
  struct Extra {};
  double add[VEC];
  double* lds;   // [NR][64*VEC]: row r in slot (r - r0) mod NR
  int r0;        // grid row of slot 0 (the row above the block's first tile)
  int ny;
  bool per;
  double shift, invg;
  int stopflag;
  __device__ __forceinline__ bool go() const { return __builtin_amdgcn_readfirstlane(stopflag) == 0; }
  __device__ __forceinline__ void load(int, const Strip&, Extra&) {}
  __device__ __forceinline__ void finish(int r, const Strip& g, const double (&Ax)[VEC], const double (&xc)[VEC],
                                         const Extra&) {
    double* row = lds + (long)((unsigned)(r - r0) % NR) * (kWave * VEC) + (threadIdx.x & (kWave - 1)) * VEC;
    double y[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) y[v] = ADD ? Ax[v] + add[v] : (Ax[v] - shift * xc[v]) * invg;
    if (!per) {
      // uniform branch: only Dirichlet rows and columns have ghost entries
      __asm__ volatile("");
      const bool ghost = !g.inside || r < 0 || r >= ny;
#pragma unroll
      for (int v = 0; v < VEC; ++v) y[v] = ghost ? 0.0 : y[v];
    }
#pragma unroll
    for (int v = 0; v < VEC; ++v) row[v] = y[v];
  }
};

// y_{k+1} row q of LDS (rounded to the storage type) with its x-neighbours
// (lanes 0 and 63, the frame, get zero as the missing neighbour)
template <typename TY, int VEC>
__device__ __forceinline__ void lds_row_n(const double* lds, int q, RowN<VEC>& o) {
  const double* row = lds + (long)q * (kWave * VEC) + (threadIdx.x & (kWave - 1)) * VEC;
#pragma unroll
  for (int v = 0; v < VEC; ++v) o.c[v] = storage_round<TY>(row[v]);
  o.l = dpp_f64_any<kDppWaveShr1>(o.c[VEC - 1]);
  o.r = dpp_f64_any<kDppWaveShl1>(o.c[0]);
}

}  // namespace adl
