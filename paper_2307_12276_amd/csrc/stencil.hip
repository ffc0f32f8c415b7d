// Row-marching nine-point stencil kernels for gfx950.
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
// Layout and mapping.  Arrays are [ny][nx], x contiguous.  A block of four
// wave64s covers 4 * 64 * VEC adjacent columns and a band of `rows` rows;
// each lane owns VEC adjacent columns and marches down the band keeping the
// three rows j-1, j, j+1 of every input in registers, so each element is read
// from HBM once per sweep (plus one halo row per band edge).  x-neighbours come
// from the adjacent lane by cross-lane shuffle; only the strip-edge lanes load
// a halo element.  Loads of row j+2 are issued before row j is computed.
// Block ids are remapped so that each XCD (blocks are dealt round-robin to the
// 8 XCDs) works on a contiguous range of tiles, keeping band-edge halo rows in
// that XCD's L2.
//
// Reductions (norms for the Leja stopping test, power iteration) are fixed
// order: shuffle tree per wave, waves in order, block partials written to
// memory, and the last block to arrive (ticket counter) sums the partials in a
// fixed order.  Results are bitwise reproducible for a given tiling.
#include "device.h"

#include <hip/hip_ext.h>

#include <cmath>

namespace adl {

// ---------------------------------------------------------------------------
// Generic row-marching core.  Ep supplies the per-row extra loads (Extra) and
// the per-row epilogue finish(j, g, Ax, xc, extra).
// ---------------------------------------------------------------------------
template <typename TF, typename TX, int VEC, bool ADVF, class Ep>
__device__ __forceinline__ void march(const FieldView& F, const Tiling& T, const TX* __restrict__ x,
                                      Ep& ep) {
  const int nx = F.nx, ny = F.ny, bc = F.bc;
  const int b = remap_xcd(blockIdx.x, gridDim.x);
  const int rb = b / T.ncb, cb = b - rb * T.ncb;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  LaneGeom g;
  g.lane = lane;
  g.col0 = ((cb * kWavesX + wave) * kWave + lane) * VEC;
  g.inside = g.col0 < nx;
  g.needL = g.inside && lane == 0;
  g.needR = g.inside && (lane == kWave - 1 || g.col0 + VEC >= nx);
  const int j0 = rb * T.rows;
  const int j1 = min(j0 + T.rows, ny);

  const TF* __restrict__ kxx = reinterpret_cast<const TF*>(F.kxx);
  const TF* __restrict__ kxy = reinterpret_cast<const TF*>(F.kxy);
  const TF* __restrict__ kyy = reinterpret_cast<const TF*>(F.kyy);
  const TF* __restrict__ fax = reinterpret_cast<const TF*>(F.ax);
  const TF* __restrict__ fay = reinterpret_cast<const TF*>(F.ay);

  // three-row windows (m = j-1, c = j, p = j+1)
  RowN<VEC> um, uc, up;   // x
  RowC<VEC> gm, gc, gp;   // kyy
  RowN<VEC> mm, mc, mp;   // kxy (x-neighbours are used on the centre row)
  RowC<VEC> ym, yc, yp;   // ay' field
  RowN<VEC> kc, ac;       // kxx, ax' field (centre row only)
  typename Ep::Extra ec;

  load_row_n<TX, VEC>(x, j0 - 1, MODE_ZERO, nx, ny, bc, g, um.c, um.l, um.r);
  load_row_n<TX, VEC>(x, j0, MODE_ZERO, nx, ny, bc, g, uc.c, uc.l, uc.r);
  load_row_n<TX, VEC>(x, j0 + 1, MODE_ZERO, nx, ny, bc, g, up.c, up.l, up.r);
  load_row<TF, VEC>(kyy, j0 - 1, MODE_EDGE, nx, ny, bc, g, gm.c);
  load_row<TF, VEC>(kyy, j0, MODE_EDGE, nx, ny, bc, g, gc.c);
  load_row<TF, VEC>(kyy, j0 + 1, MODE_EDGE, nx, ny, bc, g, gp.c);
  load_row_n<TF, VEC>(kxy, j0 - 1, MODE_ZERO, nx, ny, bc, g, mm.c, mm.l, mm.r);
  load_row_n<TF, VEC>(kxy, j0, MODE_ZERO, nx, ny, bc, g, mc.c, mc.l, mc.r);
  load_row_n<TF, VEC>(kxy, j0 + 1, MODE_ZERO, nx, ny, bc, g, mp.c, mp.l, mp.r);
  load_row_n<TF, VEC>(kxx, j0, MODE_EDGE, nx, ny, bc, g, kc.c, kc.l, kc.r);
  if constexpr (ADVF) {
    load_row<TF, VEC>(fay, j0 - 1, MODE_ZERO, nx, ny, bc, g, ym.c);
    load_row<TF, VEC>(fay, j0, MODE_ZERO, nx, ny, bc, g, yc.c);
    load_row<TF, VEC>(fay, j0 + 1, MODE_ZERO, nx, ny, bc, g, yp.c);
    load_row_n<TF, VEC>(fax, j0, MODE_ZERO, nx, ny, bc, g, ac.c, ac.l, ac.r);
  }
  ep.load(j0, g, ec);

  for (int j = j0; j < j1; ++j) {
    const bool more = (j + 1 < j1);
    RowN<VEC> un, mn, kn, an;
    RowC<VEC> gn, yn;
    typename Ep::Extra en;
    if (more) {  // uniform across the block
      load_row_n<TX, VEC>(x, j + 2, MODE_ZERO, nx, ny, bc, g, un.c, un.l, un.r);
      load_row<TF, VEC>(kyy, j + 2, MODE_EDGE, nx, ny, bc, g, gn.c);
      load_row_n<TF, VEC>(kxy, j + 2, MODE_ZERO, nx, ny, bc, g, mn.c, mn.l, mn.r);
      load_row_n<TF, VEC>(kxx, j + 1, MODE_EDGE, nx, ny, bc, g, kn.c, kn.l, kn.r);
      if constexpr (ADVF) {
        load_row<TF, VEC>(fay, j + 2, MODE_ZERO, nx, ny, bc, g, yn.c);
        load_row_n<TF, VEC>(fax, j + 1, MODE_ZERO, nx, ny, bc, g, an.c, an.l, an.r);
      }
      ep.load(j + 1, g, en);
    }

    double Ax[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      const double uC = uc.at(v), uW = uc.west(v), uE = uc.east(v);
      const double uN = up.at(v), uS = um.at(v);
      const double uNW = up.west(v), uNE = up.east(v);
      const double uSW = um.west(v), uSE = um.east(v);
      const double kC = kc.at(v), kW = kc.west(v), kE = kc.east(v);
      const double gC = gc.c[v], gN = gp.c[v], gS = gm.c[v];
      const double mE = mc.east(v), mW = mc.west(v), mN = mp.at(v), mS = mm.at(v);
      double r = 0.5 * (kC + kE) * (uE - uC) - 0.5 * (kC + kW) * (uC - uW);
      r += 0.5 * (gC + gN) * (uN - uC) - 0.5 * (gC + gS) * (uC - uS);
      r += mE * (uNE - uSE) - mW * (uNW - uSW);
      r += mN * (uNE - uNW) - mS * (uSE - uSW);
      if constexpr (ADVF) {
        r += ac.east(v) * uE - ac.west(v) * uW + yp.c[v] * uN - ym.c[v] * uS;
      } else {
        r += F.axc * (uE - uW) + F.ayc * (uN - uS);
      }
      Ax[v] = r;
    }
    ep.finish(j, g, Ax, uc.c, ec);

    if (more) {
      um = uc; uc = up; up = un;
      gm = gc; gc = gp; gp = gn;
      mm = mc; mc = mp; mp = mn;
      kc = kn;
      if constexpr (ADVF) {
        ym = yc; yc = yp; yp = yn;
        ac = an;
      }
      ec = en;
    }
  }
}

// ---------------------------------------------------------------------------
// Epilogues
// ---------------------------------------------------------------------------
struct NoExtra {};

// out = A x + a1 s1 + a2 s2
template <int VEC>
struct ApplyEp {
  struct Extra {};
  int nx;
  double* __restrict__ out;
  const double* __restrict__ s1;
  const double* __restrict__ s2;
  double a1, a2;
  __device__ __forceinline__ void load(int, const LaneGeom&, Extra&) {}
  __device__ __forceinline__ void finish(int j, const LaneGeom& g, const double (&Ax)[VEC],
                                         const double (&)[VEC], const Extra&) {
    if (!g.inside) return;
    const long off = (long)j * nx + g.col0;
    double r[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) r[v] = Ax[v];
    if (s1) {
      double s[VEC];
      load_c<double, VEC>(s1, off, s);
#pragma unroll
      for (int v = 0; v < VEC; ++v) r[v] += a1 * s[v];
    }
    if (s2) {
      double s[VEC];
      load_c<double, VEC>(s2, off, s);
#pragma unroll
      for (int v = 0; v < VEC; ++v) r[v] += a2 * s[v];
    }
    store_c<double, VEC>(out, off, r);
  }
};

template <typename TF, int VEC, bool ADVF>
__global__ __launch_bounds__(kBlock) void apply_kernel(FieldView F, Tiling T, const double* __restrict__ x,
                                                       ApplyEp<VEC> ep) {
  march<TF, double, VEC, ADVF>(F, T, x, ep);
}

// One Newton-Leja iteration (fused): y' = (A y + w2c w2 - shift y) invg,
// p' = p + d_{k+1} y'  (p = d_0 y at k = 0); norms of d y' and p'.
template <typename TYO, int VEC>
struct LejaEp {
  struct Extra {
    double p[VEC];
    double w[VEC];
  };
  int nx;
  TYO* __restrict__ yout;
  double* __restrict__ p;
  const double* __restrict__ w2;
  double w2c, shift, invg, d0, dk1;
  bool first;
  double acc[3];  // ||d y'||^2, ||p'||^2, max(|y0|, |w2|)
  __device__ __forceinline__ void load(int j, const LaneGeom& g, Extra& e) {
    if (!g.inside) return;
    const long off = (long)j * nx + g.col0;
    if (!first) load_c<double, VEC>(p, off, e.p);
    if (w2) load_c<double, VEC>(w2, off, e.w);
  }
  __device__ __forceinline__ void finish(int j, const LaneGeom& g, const double (&Ax)[VEC],
                                         const double (&yc)[VEC], const Extra& e) {
    if (!g.inside) return;
    const long off = (long)j * nx + g.col0;
    double yn[VEC], pn[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      double a = Ax[v];
      if (w2) a += w2c * e.w[v];
      const double y1 = (a - shift * yc[v]) * invg;
      const double t = dk1 * y1;
      const double pv = (first ? d0 * yc[v] : e.p[v]) + t;
      yn[v] = y1;
      pn[v] = pv;
      acc[0] += t * t;
      acc[1] += pv * pv;
      if (first) {
        acc[2] = nanmax(acc[2], fabs(yc[v]));
        if (w2) acc[2] = nanmax(acc[2], fabs(e.w[v]));
      }
    }
    store_c<TYO, VEC>(yout, off, yn);
    store_c<double, VEC>(p, off, pn);
  }
};

template <typename TF, typename TYI, typename TYO, int VEC, bool ADVF>
__global__ __launch_bounds__(kBlock) void leja_kernel(FieldView F, Tiling T, LejaArgs A) {
  if (A.ctl->stop) return;  // the sweep has already stopped: no-op launch
  LejaEp<TYO, VEC> ep;
  ep.nx = F.nx;
  ep.yout = reinterpret_cast<TYO*>(A.yout);
  ep.p = A.p;
  ep.w2 = A.w2;
  ep.w2c = A.w2c;
  ep.shift = A.shift;
  ep.invg = A.invg;
  ep.d0 = A.d0;
  ep.dk1 = A.dk1;
  ep.first = A.first != 0;
  ep.acc[0] = ep.acc[1] = ep.acc[2] = 0.0;
  march<TF, TYI, VEC, ADVF>(F, T, reinterpret_cast<const TYI*>(A.yin), ep);
  const double tol2 = A.tol2;
  const int k = A.k, maxdeg = A.max_degree;
  const bool first = A.first != 0;
  Ctl* ctl = A.ctl;
  grid_reduce<3, 2>(ep.acc, A.partials, ctl, [=](const double (&tot)[3]) {
    const double tn2 = tot[0], pn2 = tot[1];
    const int deg = k + 1;
    int stop = 0, status = 0, degree = deg;
    if (!isfinite(tn2) || !isfinite(pn2)) {
      stop = 1; status = 2;
    } else if (first && tot[2] == 0.0) {
      stop = 1; status = 1; degree = 0;
    } else if (tn2 <= tol2 * pn2) {
      stop = 1; status = 1;
    } else if (deg >= maxdeg) {
      stop = 1; status = 3;
    }
    ctl->tn2 = tn2;
    ctl->pn2 = pn2;
    ctl->degree = degree;
    ctl->status = status;
    ctl->stop = stop;
  });
}

// Power iteration step: w = scale * A x, lambda = ||w||.
template <int VEC>
struct PowerEp {
  struct Extra {};
  int nx;
  double* __restrict__ w;
  double scale;
  double acc[1];
  __device__ __forceinline__ void load(int, const LaneGeom&, Extra&) {}
  __device__ __forceinline__ void finish(int j, const LaneGeom& g, const double (&Ax)[VEC],
                                         const double (&)[VEC], const Extra&) {
    if (!g.inside) return;
    double r[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      r[v] = Ax[v] * scale;
      acc[0] += r[v] * r[v];
    }
    store_c<double, VEC>(w, (long)j * nx + g.col0, r);
  }
};

template <typename TF, int VEC, bool ADVF>
__global__ __launch_bounds__(kBlock) void power_kernel(FieldView F, Tiling T, const double* __restrict__ x,
                                                       double* __restrict__ w, double rtol, int max_iter,
                                                       double* partials, Ctl* ctl) {
  if (ctl->stop) return;
  PowerEp<VEC> ep;
  ep.nx = F.nx;
  ep.w = w;
  ep.scale = ctl->scale;
  ep.acc[0] = 0.0;
  march<TF, double, VEC, ADVF>(F, T, x, ep);
  grid_reduce<1, 1>(ep.acc, partials, ctl, [=](const double (&tot)[1]) {
    const double lam = sqrt(tot[0]);
    const int it = ctl->iters + 1;
    int stop = 0, status = 0;
    if (!isfinite(lam)) {
      stop = 1; status = 2;
    } else if (lam == 0.0) {
      stop = 1; status = 1;
    } else if (fabs(lam - ctl->lam_prev) <= rtol * lam) {
      stop = 1; status = 1;
    } else if (it >= max_iter) {
      stop = 1; status = 3;
    }
    ctl->lam = lam;
    ctl->lam_prev = lam;
    ctl->scale = lam > 0.0 ? 1.0 / lam : 0.0;
    ctl->iters = it;
    ctl->status = status;
    ctl->stop = stop;
  });
}

// splitmix64 output k of the stream seeded with s (Steele, Lea, Flood 2014):
// z = s + (k+1) * golden; two xor-shift-multiply rounds; final xor-shift.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// w = uniform(-1, 1) start vector; lambda_0 = ||w|| -> scale = 1/lambda_0.
__global__ __launch_bounds__(kBlock) void power_init_kernel(long n, uint64_t seed, double* __restrict__ w,
                                                            double* partials, Ctl* ctl) {
  double acc[1] = {0.0};
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const uint64_t z = splitmix64_at(seed, (uint64_t)i);
    const double u = 2.0 * (double)(z >> 11) * 0x1.0p-53 - 1.0;
    w[i] = u;
    acc[0] += u * u;
  }
  grid_reduce<1, 1>(acc, partials, ctl, [=](const double (&tot)[1]) {
    const double lam = sqrt(tot[0]);
    ctl->scale = lam > 0.0 ? 1.0 / lam : 0.0;
    ctl->lam = lam;
    ctl->lam_prev = 0.0;
    ctl->iters = 0;
    ctl->status = 0;
    ctl->stop = lam > 0.0 ? 0 : 1;
  });
}

// Gershgorin: min over rows of A_ii - sum_{j != i} |A_ij| (one thread per node).
template <typename TF, bool ADVF>
__global__ __launch_bounds__(kBlock) void gershgorin_kernel(FieldView F, double* partials, Ctl* ctl) {
  const int nx = F.nx, ny = F.ny;
  const bool per = F.bc == BC_PERIODIC;
  const TF* kxx = reinterpret_cast<const TF*>(F.kxx);
  const TF* kxy = reinterpret_cast<const TF*>(F.kxy);
  const TF* kyy = reinterpret_cast<const TF*>(F.kyy);
  const TF* fax = reinterpret_cast<const TF*>(F.ax);
  const TF* fay = reinterpret_cast<const TF*>(F.ay);
  double acc[1] = {INFINITY};
  const long n = (long)nx * ny;
  for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += (long)gridDim.x * blockDim.x) {
    const int j = (int)(idx / nx), i = (int)(idx - (long)j * nx);
    const bool hasE = per || i + 1 < nx, hasW = per || i > 0;
    const bool hasN = per || j + 1 < ny, hasS = per || j > 0;
    const int iE = i + 1 < nx ? i + 1 : (per ? 0 : i);
    const int iW = i > 0 ? i - 1 : (per ? nx - 1 : i);
    const int jN = j + 1 < ny ? j + 1 : (per ? 0 : j);
    const int jS = j > 0 ? j - 1 : (per ? ny - 1 : j);
    auto at = [&](const TF* a, int jj, int ii) { return (double)a[(long)jj * nx + ii]; };
    const double kC = at(kxx, j, i), kE = at(kxx, j, iE), kW = at(kxx, j, iW);
    const double gC = at(kyy, j, i), gN = at(kyy, jN, i), gS = at(kyy, jS, i);
    const double mE = hasE ? at(kxy, j, iE) : 0.0, mW = hasW ? at(kxy, j, iW) : 0.0;
    const double mN = hasN ? at(kxy, jN, i) : 0.0, mS = hasS ? at(kxy, jS, i) : 0.0;
    double aE = F.axc, aW = F.axc, aN = F.ayc, aS = F.ayc;
    if constexpr (ADVF) {
      aE = hasE ? at(fax, j, iE) : 0.0;
      aW = hasW ? at(fax, j, iW) : 0.0;
      aN = hasN ? at(fay, jN, i) : 0.0;
      aS = hasS ? at(fay, jS, i) : 0.0;
    }
    const double fe = 0.5 * (kC + kE), fw = 0.5 * (kC + kW), fn = 0.5 * (gC + gN), fs = 0.5 * (gC + gS);
    const double cen = -(fe + fw + fn + fs);
    double rad = 0.0;
    if (hasE) rad += fabs(fe + aE);
    if (hasW) rad += fabs(fw - aW);
    if (hasN) rad += fabs(fn + aN);
    if (hasS) rad += fabs(fs - aS);
    if (hasE && hasN) rad += fabs(mE + mN);
    if (hasW && hasN) rad += fabs(mW + mN);
    if (hasE && hasS) rad += fabs(mE + mS);
    if (hasW && hasS) rad += fabs(mW + mS);
    const double v = cen - rad;
    acc[0] = -nanmax(-acc[0], -v);
  }
  // reduce as a NaN-propagating max of -value
  acc[0] = -acc[0];
  grid_reduce<1, 0>(acc, partials, ctl, [=](const double (&tot)[1]) { ctl->gmin = -tot[0]; });
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
Tiling make_tiling(int nx, int ny, int rows_hint) {
  Tiling t;
  t.vec = (nx % 2 == 0 && nx >= 2 * kWave) ? 2 : 1;
  const int bw = kBlock * t.vec;
  t.ncb = (nx + bw - 1) / bw;
  int rows = rows_hint;
  if (rows <= 0) {
    // aim for >= 2048 blocks on large grids, >= 4 rows per band
    const long target = 2048;
    long nrb_want = (target + t.ncb - 1) / t.ncb;
    rows = (int)((ny + nrb_want - 1) / nrb_want);
    if (rows < 4) rows = 4;
    if (rows > 64) rows = 64;
  }
  if (rows > ny) rows = ny;
  t.rows = rows;
  t.nrb = (ny + rows - 1) / rows;
  t.nblocks = t.ncb * t.nrb;
  return t;
}

static inline int ew_blocks(long n) {
  long b = (n + kBlock - 1) / kBlock;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (int)b;
}

#define ADL_DISPATCH_VEC_ADV(T, F, ...)                    \
  do {                                                     \
    const bool advf_ = (F).ax != nullptr;                  \
    if ((T).vec == 2) {                                    \
      constexpr int VEC = 2;                               \
      if (advf_) { constexpr bool ADVF = true; __VA_ARGS__; }     \
      else { constexpr bool ADVF = false; __VA_ARGS__; }          \
    } else {                                               \
      constexpr int VEC = 1;                               \
      if (advf_) { constexpr bool ADVF = true; __VA_ARGS__; }     \
      else { constexpr bool ADVF = false; __VA_ARGS__; }          \
    }                                                      \
  } while (0)

hipError_t launch_apply(const FieldView& f, const Tiling& t, const double* x, double* y, const double* s1,
                        double a1, const double* s2, double a2, hipStream_t st) {
  ADL_DISPATCH_VEC_ADV(t, f, {
    ApplyEp<VEC> ep;
    ep.nx = f.nx;
    ep.out = y;
    ep.s1 = s1;
    ep.s2 = s2;
    ep.a1 = a1;
    ep.a2 = a2;
    if (f.f32)
      hipLaunchKernelGGL((apply_kernel<float, VEC, ADVF>), dim3(t.nblocks), dim3(kBlock), 0, st, f, t, x, ep);
    else
      hipLaunchKernelGGL((apply_kernel<double, VEC, ADVF>), dim3(t.nblocks), dim3(kBlock), 0, st, f, t, x, ep);
  });
  return hipGetLastError();
}

template <typename TF, typename TYI, typename TYO, int VEC, bool ADVF>
static void leja_launch(const FieldView& f, const Tiling& t, const LejaArgs& a, hipStream_t st) {
  const dim3 grid(t.nblocks), blk(kBlock);
  if (a.ev_start)
    hipExtLaunchKernelGGL((leja_kernel<TF, TYI, TYO, VEC, ADVF>), grid, blk, 0, st, a.ev_start, a.ev_stop, 0, f, t,
                          a);
  else
    hipLaunchKernelGGL((leja_kernel<TF, TYI, TYO, VEC, ADVF>), grid, blk, 0, st, f, t, a);
}

template <typename TF, int VEC, bool ADVF>
static void leja_dispatch_y(const FieldView& f, const Tiling& t, const LejaArgs& a, hipStream_t st) {
  if (a.yin_f32) {
    if (a.ystore_f32) leja_launch<TF, float, float, VEC, ADVF>(f, t, a, st);
    else leja_launch<TF, float, double, VEC, ADVF>(f, t, a, st);
  } else {
    if (a.ystore_f32) leja_launch<TF, double, float, VEC, ADVF>(f, t, a, st);
    else leja_launch<TF, double, double, VEC, ADVF>(f, t, a, st);
  }
}

hipError_t launch_leja_step(const FieldView& f, const Tiling& t, const LejaArgs& a, hipStream_t st) {
  ADL_DISPATCH_VEC_ADV(t, f, {
    if (f.f32) leja_dispatch_y<float, VEC, ADVF>(f, t, a, st);
    else leja_dispatch_y<double, VEC, ADVF>(f, t, a, st);
  });
  return hipGetLastError();
}

hipError_t launch_power_init(int n, uint64_t seed, double* w, double* partials, int nblocks, Ctl* ctl,
                             hipStream_t st) {
  (void)nblocks;
  const int nb = ew_blocks(n) < 1024 ? ew_blocks(n) : 1024;
  hipLaunchKernelGGL(power_init_kernel, dim3(nb), dim3(kBlock), 0, st, (long)n, seed, w, partials, ctl);
  return hipGetLastError();
}

hipError_t launch_power_step(const FieldView& f, const Tiling& t, const double* x, double* w, double rtol,
                             int max_iter, double* partials, Ctl* ctl, hipStream_t st) {
  ADL_DISPATCH_VEC_ADV(t, f, {
    if (f.f32)
      hipLaunchKernelGGL((power_kernel<float, VEC, ADVF>), dim3(t.nblocks), dim3(kBlock), 0, st, f, t, x, w,
                         rtol, max_iter, partials, ctl);
    else
      hipLaunchKernelGGL((power_kernel<double, VEC, ADVF>), dim3(t.nblocks), dim3(kBlock), 0, st, f, t, x, w,
                         rtol, max_iter, partials, ctl);
  });
  return hipGetLastError();
}

hipError_t launch_gershgorin(const FieldView& f, double* partials, Ctl* ctl, hipStream_t st) {
  const long n = (long)f.nx * f.ny;
  const int nb = ew_blocks(n) < 1024 ? ew_blocks(n) : 1024;
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
