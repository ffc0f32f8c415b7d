// Row-marching core of the nine-point stencil kernels (gfx950).
//
// A wave64 owns a strip of 64*VEC adjacent columns (VEC columns per lane) and
// marches down a band of rows [j0, j1).  It keeps the rows j-1, j, j+1 of the
// input vector x and of the kyy / kxy fields and the centre row of kxx in
// registers, so every element is read from memory once per launch plus one
// halo row above and below the band.  The loads of row j+2 are issued before
// row j is computed (software pipelining).
//
// x-neighbours: the left neighbour of a lane's first column is the previous
// lane's last column and the right neighbour of its last column the next
// lane's first column; both come from DPP whole-wave shifts (wave_shr:1 /
// wave_shl:1, VALU instructions).  Lane 0 and lane 63 load their halo element
// (interior tiles: one unmasked load per row and array whose other lanes
// re-read their own column).
//
// Interior strips of interior bands (all of the window in the grid, halo
// columns in the grid) use a path with no boundary logic; the other tiles
// apply the boundary rules (periodic wrap; Dirichlet zero rows/columns for x
// and kxy, edge values for the face averages of kxx and kyy).
#pragma once

#include "device.h"

#include <type_traits>

namespace adl {

constexpr int kDppWaveShl1 = 0x130;  // lane i <- lane i+1
constexpr int kDppWaveShr1 = 0x138;  // lane i <- lane i-1

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

struct Strip {
  int col0;    // first column of this lane
  int lane;
  int hoff;    // interior tiles: column offset of this lane's halo load (-1, VEC or 0)
  bool inside; // col0 < nx
  bool needL;  // this lane's left neighbour is not the previous lane's column
  bool needR;  // this lane's right neighbour is not the next lane's column
  bool lane0, lane63;
};

// A row as loaded (storage type, no conversion): own columns and one halo
// element.  Converted and completed with its x-neighbours one step later.
template <typename T, int VEC>
struct RawRow {
  T c[VEC];
  T h;
};

template <typename T, int VEC>
struct RawC {
  T c[VEC];
};

template <typename T, int VEC>
__device__ __forceinline__ void load_raw(const T* __restrict__ a, long rowoff, const Strip& g, RawRow<T, VEC>& o) {
  if constexpr (VEC == 1) {
    o.c[0] = a[rowoff + g.col0];
  } else if constexpr (sizeof(T) == 8) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 v = *reinterpret_cast<const d2*>(a + rowoff + g.col0);
    o.c[0] = v.x;
    o.c[1] = v.y;
  } else {
    typedef float f2 __attribute__((ext_vector_type(2)));
    const f2 v = *reinterpret_cast<const f2*>(a + rowoff + g.col0);
    o.c[0] = v.x;
    o.c[1] = v.y;
  }
  o.h = a[rowoff + g.col0 + g.hoff];
}

template <typename T, int VEC>
__device__ __forceinline__ void load_raw_c(const T* __restrict__ a, long rowoff, const Strip& g, RawC<T, VEC>& o) {
  if constexpr (VEC == 1) {
    o.c[0] = a[rowoff + g.col0];
  } else if constexpr (sizeof(T) == 8) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 v = *reinterpret_cast<const d2*>(a + rowoff + g.col0);
    o.c[0] = v.x;
    o.c[1] = v.y;
  } else {
    typedef float f2 __attribute__((ext_vector_type(2)));
    const f2 v = *reinterpret_cast<const f2*>(a + rowoff + g.col0);
    o.c[0] = v.x;
    o.c[1] = v.y;
  }
}

template <typename T, int VEC>
__device__ __forceinline__ void finish_row(const RawRow<T, VEC>& in, const Strip& g, RowN<VEC>& o) {
#pragma unroll
  for (int v = 0; v < VEC; ++v) o.c[v] = (double)in.c[v];
  const double h = (double)in.h;
  const double l = dpp_f64<kDppWaveShr1>(o.c[VEC - 1]);
  const double r = dpp_f64<kDppWaveShl1>(o.c[0]);
  o.l = g.lane0 ? h : l;
  o.r = g.lane63 ? h : r;
}

template <typename T, int VEC>
__device__ __forceinline__ void finish_c(const RawC<T, VEC>& in, RowC<VEC>& o) {
#pragma unroll
  for (int v = 0; v < VEC; ++v) o.c[v] = (double)in.c[v];
}

// Centre values of one row (general path: boundary rules).
template <typename T, int VEC>
__device__ __forceinline__ void row_c(const T* __restrict__ a, int r, int mode, int nx, int ny, int bc,
                                      const Strip& g, double (&c)[VEC]) {
  bool zero;
  const int row = map_row(r, ny, bc, mode, zero);
  if (!zero && g.inside) {
    load_c<T, VEC>(a, (long)row * nx + g.col0, c);
  } else {
#pragma unroll
    for (int v = 0; v < VEC; ++v) c[v] = 0.0;
  }
}

// Centre values and x-neighbours of one row (general path).
template <typename T, int VEC>
__device__ __forceinline__ void row_n(const T* __restrict__ a, int r, int mode, int nx, int ny, int bc,
                                      const Strip& g, RowN<VEC>& o) {
  bool zero;
  const int row = map_row(r, ny, bc, mode, zero);
  if (!zero && g.inside) {
    load_c<T, VEC>(a, (long)row * nx + g.col0, o.c);
  } else {
#pragma unroll
    for (int v = 0; v < VEC; ++v) o.c[v] = 0.0;
  }
  o.l = dpp_f64<kDppWaveShr1>(o.c[VEC - 1]);
  o.r = dpp_f64<kDppWaveShl1>(o.c[0]);
  if (g.needL) {
    const int cl = g.col0 - 1;
    double v;
    if (zero) v = 0.0;
    else if (cl >= 0) v = (double)a[(long)row * nx + cl];
    else if (bc == BC_PERIODIC) v = (double)a[(long)row * nx + nx - 1];
    else v = (mode == MODE_EDGE) ? o.c[0] : 0.0;
    o.l = v;
  }
  if (g.needR) {
    const int cr = g.col0 + VEC;
    double v;
    if (zero) v = 0.0;
    else if (cr < nx) v = (double)a[(long)row * nx + cr];
    else if (bc == BC_PERIODIC) v = (double)a[(long)row * nx];
    else v = (mode == MODE_EDGE) ? o.c[VEC - 1] : 0.0;
    o.r = v;
  }
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

// March over rows [j0, j1) of the strip `g`.
//
// INTERIOR (rows j0-1 .. j1 and the halo columns inside the grid, every lane
// inside, j1 - j0 a multiple of 4): rows live in a 4-slot ring (row q in slot
// (q - j0 + 1) mod 4; centre-row arrays in a 2-slot ring) and the loop is
// unrolled by 4, so no register is copied, the loop body has no branches,
// and the loads of rows j+2 (window) and j+1 (centre rows) stay in flight
// while row j is computed.
//
// General tiles (boundary bands or strips): one row per step with the
// boundary rules applied to every load.
template <typename TF, typename TX, int VEC, bool ADVF, bool INTERIOR, class Ep>
__device__ __forceinline__ void march_strip(const FieldView& F, const TX* __restrict__ x, Ep& ep, const Strip& g,
                                            int j0, int j1) {
  const int nx = F.nx, ny = F.ny, bc = F.bc;
  const TF* __restrict__ kxx = reinterpret_cast<const TF*>(F.kxx);
  const TF* __restrict__ kxy = reinterpret_cast<const TF*>(F.kxy);
  const TF* __restrict__ kyy = reinterpret_cast<const TF*>(F.kyy);
  const TF* __restrict__ fax = reinterpret_cast<const TF*>(F.ax);
  const TF* __restrict__ fay = reinterpret_cast<const TF*>(F.ay);
  const double axc = F.axc, ayc = F.ayc;

  if constexpr (INTERIOR) {
    // finished rows (FP64, with x-neighbours): 4-slot ring by row, centre rows 1 slot
    RowN<VEC> u[4], m[4], k, ac;
    RowC<VEC> gg[4], ay[4];
    // raw rows as loaded: 2-slot rings
    RawRow<TX, VEC> ru[2];
    RawRow<TF, VEC> rm[2], rk[2], ra[2];
    RawC<TF, VEC> rg[2], ry[2];
    typename Ep::Extra ex[2];
    auto load_w = [&](int q, int s2) {
      const long off = (long)q * nx;
      load_raw<TX, VEC>(x, off, g, ru[s2]);
      load_raw_c<TF, VEC>(kyy, off, g, rg[s2]);
      load_raw<TF, VEC>(kxy, off, g, rm[s2]);
      if constexpr (ADVF) load_raw_c<TF, VEC>(fay, off, g, ry[s2]);
    };
    auto fin_w = [&](int s2, int s4) {
      finish_row<TX, VEC>(ru[s2], g, u[s4]);
      finish_c<TF, VEC>(rg[s2], gg[s4]);
      finish_row<TF, VEC>(rm[s2], g, m[s4]);
      if constexpr (ADVF) finish_c<TF, VEC>(ry[s2], ay[s4]);
    };
    auto load_k = [&](int q, int s2) {
      const long off = (long)q * nx;
      load_raw<TF, VEC>(kxx, off, g, rk[s2]);
      if constexpr (ADVF) load_raw<TF, VEC>(fax, off, g, ra[s2]);
      ep.template load<false>(q, g, ex[s2]);
    };
    auto fin_k = [&](int s2) {
      finish_row<TF, VEC>(rk[s2], g, k);
      if constexpr (ADVF) finish_row<TF, VEC>(ra[s2], g, ac);
    };
    // step t of a 4-row group at jb (jb - j0 a multiple of 4): output row j = jb + t.
    // Row q of x / kyy / kxy is raw in slot (q - j0 + 1) mod 2 and finished in
    // slot (q - j0 + 1) mod 4; centre row q is raw in slot (q - j0) mod 2.
    auto step = [&](int jb, auto tc, bool prefetch_w, bool prefetch_k) {
      constexpr int t = decltype(tc)::value;
      const int j = jb + t;
      if (prefetch_w) load_w(j + 2, (t + 3) & 1);   // raw slot of row j+2
      if (prefetch_k) load_k(j + 1, (t + 1) & 1);   // raw slot of centre row j+1
      fin_w((t + 2) & 1, (t + 2) & 3);              // row j+1, loaded one step earlier
      fin_k(t & 1);                                 // centre row j, loaded one step earlier
      double Ax[VEC];
      stencil_point<VEC, ADVF>(u[t & 3], u[(t + 1) & 3], u[(t + 2) & 3], gg[t & 3], gg[(t + 1) & 3],
                               gg[(t + 2) & 3], m[t & 3], m[(t + 1) & 3], m[(t + 2) & 3], k, ac, ay[t & 3],
                               ay[(t + 2) & 3], axc, ayc, Ax);
      ep.template finish<false>(j, g, Ax, u[(t + 1) & 3].c, ex[t & 1]);
    };
    using T0 = std::integral_constant<int, 0>;
    using T1 = std::integral_constant<int, 1>;
    using T2 = std::integral_constant<int, 2>;
    using T3 = std::integral_constant<int, 3>;
    // prologue: rows j0-1 and j0 finished, row j0+1 and centre row j0 raw
    load_w(j0 - 1, 0);
    load_w(j0, 1);
    fin_w(0, 0);
    fin_w(1, 1);
    load_w(j0 + 1, 0);
    load_k(j0, 0);
    int jb = j0;
    for (; jb < j1 - 4; jb += 4) {
      step(jb, T0{}, true, true);
      step(jb, T1{}, true, true);
      step(jb, T2{}, true, true);
      step(jb, T3{}, true, true);
    }
    // last group (jb = j1 - 4): window rows up to the halo row j1 = jb + 4 (loaded
    // at step 2), centre rows up to j1 - 1 = jb + 3 (loaded at step 2)
    step(jb, T0{}, true, true);
    step(jb, T1{}, true, true);
    step(jb, T2{}, true, true);
    step(jb, T3{}, false, false);
  } else {
    RowN<VEC> um, uc, up, mm, mc, mp, kc, ac;
    RowC<VEC> gm, gc, gp, ym, yc, yp;
    typename Ep::Extra ec;
    auto load_w = [&](int q, RowN<VEC>& du, RowC<VEC>& dg, RowN<VEC>& dm, RowC<VEC>& dy) {
      row_n<TX, VEC>(x, q, MODE_ZERO, nx, ny, bc, g, du);
      row_c<TF, VEC>(kyy, q, MODE_EDGE, nx, ny, bc, g, dg.c);
      row_n<TF, VEC>(kxy, q, MODE_ZERO, nx, ny, bc, g, dm);
      if constexpr (ADVF) row_c<TF, VEC>(fay, q, MODE_ZERO, nx, ny, bc, g, dy.c);
    };
    auto load_k = [&](int q, RowN<VEC>& dk, RowN<VEC>& da, typename Ep::Extra& de) {
      row_n<TF, VEC>(kxx, q, MODE_EDGE, nx, ny, bc, g, dk);
      if constexpr (ADVF) row_n<TF, VEC>(fax, q, MODE_ZERO, nx, ny, bc, g, da);
      ep.template load<true>(q, g, de);
    };
    load_w(j0 - 1, um, gm, mm, ym);
    load_w(j0, uc, gc, mc, yc);
    load_w(j0 + 1, up, gp, mp, yp);
    load_k(j0, kc, ac, ec);
    for (int j = j0; j < j1; ++j) {
      const bool more = j + 1 < j1;
      RowN<VEC> un, mn, kn, an;
      RowC<VEC> gn, yn;
      typename Ep::Extra en;
      if (more) {
        load_w(j + 2, un, gn, mn, yn);
        load_k(j + 1, kn, an, en);
      }
      double Ax[VEC];
      stencil_point<VEC, ADVF>(um, uc, up, gm, gc, gp, mm, mc, mp, kc, ac, ym, yp, axc, ayc, Ax);
      ep.template finish<true>(j, g, Ax, uc.c, ec);
      if (more) {
        um = uc; uc = up; up = un;
        gm = gc; gc = gp; gp = gn;
        mm = mc; mc = mp; mp = mn;
        if constexpr (ADVF) { ym = yc; yc = yp; yp = yn; ac = an; }
        kc = kn;
        ec = en;
      }
    }
  }
}

// The tile of this wave in a block of kWavesX waves side by side.
template <typename TF, typename TX, int VEC, bool ADVF, class Ep>
__device__ __forceinline__ void march_tile(const FieldView& F, const TX* __restrict__ x, Ep& ep, int cb, int j0,
                                           int j1, int waves_x, int wave) {
  const int lane = threadIdx.x & (kWave - 1);
  Strip g;
  g.lane = lane;
  const int i0 = (cb * waves_x + wave) * kWave * VEC;
  g.col0 = i0 + lane * VEC;
  g.inside = g.col0 < F.nx;
  g.needL = g.inside && lane == 0;
  g.needR = g.inside && (lane == kWave - 1 || g.col0 + VEC >= F.nx);
  g.lane0 = lane == 0;
  g.lane63 = lane == kWave - 1;
  g.hoff = g.lane0 ? -1 : (g.lane63 ? VEC : 0);
  const bool interior = (j0 >= 1) && (j1 <= F.ny - 1) && (i0 >= 1) && (i0 + kWave * VEC < F.nx) &&
                        ((j1 - j0) % 4 == 0) && (j1 - j0 >= 4);
  if (interior) march_strip<TF, TX, VEC, ADVF, true>(F, x, ep, g, j0, j1);
  else march_strip<TF, TX, VEC, ADVF, false>(F, x, ep, g, j0, j1);
}

}  // namespace adl
