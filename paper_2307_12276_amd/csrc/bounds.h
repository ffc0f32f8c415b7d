// Block bodies of the one-pass reductions over the stored operator: the
// Gershgorin bound of the spectrum and the field statistics that feed the
// learned interval.  Each runs as blocks b = 0 .. nb-1 of a reduction, either
// as a whole launch (one op) or as one op's share of a batched launch, with
// the same arithmetic and summation order either way.
#pragma once

#include "device.h"

namespace adl {

// Scale factors of unscaled FP64 fields (Dxx, Dxy, Dyy, ax, ay as the
// caller holds them): the stored form is field * scale, computed here with
// the same product the field preparation stores.
struct FieldScale {
  double xx, xy, yy, ax, ay;
};

// Gershgorin bound: min over rows of A_ii - sum_{j != i} |A_ij| (one thread
// per node), as blocks b of nb; the total goes to ctl->gmin and, if given, *gout.
// RAW: F points at unscaled FP64 fields, scaled by sc on load.
template <typename TF, bool ADVF, bool RAW = false>
__device__ __forceinline__ void gershgorin_blocks(const FieldView& F, double* partials, Ctl* ctl, int nb, int b,
                                                  double* gout, FieldScale sc = FieldScale{}) {
  const int nx = F.nx, ny = F.ny;
  const bool per = F.bc == BC_PERIODIC;
  const TF* kxx = reinterpret_cast<const TF*>(F.kxx);
  const TF* kxy = reinterpret_cast<const TF*>(F.kxy);
  const TF* kyy = reinterpret_cast<const TF*>(F.kyy);
  const TF* fax = reinterpret_cast<const TF*>(F.ax);
  const TF* fay = reinterpret_cast<const TF*>(F.ay);
  double acc[1] = {INFINITY};
  const long n = (long)nx * ny;
  for (long idx = (long)b * blockDim.x + threadIdx.x; idx < n; idx += (long)nb * blockDim.x) {
    const int j = (int)(idx / nx), i = (int)(idx - (long)j * nx);
    const bool hasE = per || i + 1 < nx, hasW = per || i > 0;
    const bool hasN = per || j + 1 < ny, hasS = per || j > 0;
    const int iE = i + 1 < nx ? i + 1 : (per ? 0 : i);
    const int iW = i > 0 ? i - 1 : (per ? nx - 1 : i);
    const int jN = j + 1 < ny ? j + 1 : (per ? 0 : j);
    const int jS = j > 0 ? j - 1 : (per ? ny - 1 : j);
    auto at = [&](const TF* a, int jj, int ii, double s) {
      const double v = (double)a[(long)jj * nx + ii];
      if constexpr (RAW) {
        // the product rounded on its own, as the field preparation stores it
        // (not fused into a following addition)
#pragma clang fp contract(off)
        return v * s;
      } else {
        return v;
      }
    };
    const double kC = at(kxx, j, i, sc.xx), kE = at(kxx, j, iE, sc.xx), kW = at(kxx, j, iW, sc.xx);
    const double gC = at(kyy, j, i, sc.yy), gN = at(kyy, jN, i, sc.yy), gS = at(kyy, jS, i, sc.yy);
    const double mE = hasE ? at(kxy, j, iE, sc.xy) : 0.0, mW = hasW ? at(kxy, j, iW, sc.xy) : 0.0;
    const double mN = hasN ? at(kxy, jN, i, sc.xy) : 0.0, mS = hasS ? at(kxy, jS, i, sc.xy) : 0.0;
    double aE = F.axc, aW = F.axc, aN = F.ayc, aS = F.ayc;
    if constexpr (ADVF) {
      aE = hasE ? at(fax, j, iE, sc.ax) : 0.0;
      aW = hasW ? at(fax, j, iW, sc.ax) : 0.0;
      aN = hasN ? at(fay, jN, i, sc.ay) : 0.0;
      aS = hasS ? at(fay, jS, i, sc.ay) : 0.0;
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
  grid_reduce<1, 0>(acc, partials, ctl, nb, b, [=](const double (&tot)[1]) {
    ctl->gmin = -tot[0];
    if (gout) *gout = -tot[0];
  });
}

// Field statistics: per-node eigenvalues of [[Dxx, Dxy], [Dxy, Dyy]] and |a|
// (sums and maxima), as blocks b of nb; feats[0..8] receive the raw features.
template <typename TF, bool ADVF>
__device__ __forceinline__ void field_stats_blocks(const FieldView& F, double hx, double hy, double dt,
                                                   float* __restrict__ feats, double* partials, Ctl* ctl, int nb,
                                                   int b) {
  const TF* kxx = reinterpret_cast<const TF*>(F.kxx);
  const TF* kxy = reinterpret_cast<const TF*>(F.kxy);
  const TF* kyy = reinterpret_cast<const TF*>(F.kyy);
  const TF* fax = reinterpret_cast<const TF*>(F.ax);
  const TF* fay = reinterpret_cast<const TF*>(F.ay);
  const double sxx = hx * hx, syy = hy * hy, sxy = 4.0 * hx * hy, sax = 2.0 * hx, say = 2.0 * hy;
  const long n = (long)F.nx * F.ny;
  // sums: kpar, kperp', |a|; maxima: kpar, kperp', |a|
  double acc[6] = {0.0, 0.0, 0.0, -INFINITY, -INFINITY, -INFINITY};
  for (long i = (long)b * blockDim.x + threadIdx.x; i < n; i += (long)nb * blockDim.x) {
    const double dxx = (double)kxx[i] * sxx, dyy = (double)kyy[i] * syy, dxy = (double)kxy[i] * sxy;
    const double m = 0.5 * (dxx + dyy);
    const double r = sqrt(0.25 * (dxx - dyy) * (dxx - dyy) + dxy * dxy);
    const double kp = m + r;
    const double kq = fmax(m - r, 0.0) + 1e-30;
    double ax = F.axc * sax, ay = F.ayc * say;
    if constexpr (ADVF) {
      ax = (double)fax[i] * sax;
      ay = (double)fay[i] * say;
    }
    const double am = sqrt(ax * ax + ay * ay);
    acc[0] += kp;
    acc[1] += kq;
    acc[2] += am;
    acc[3] = nanmax(acc[3], kp);
    acc[4] = nanmax(acc[4], kq);
    acc[5] = nanmax(acc[5], am);
  }
  const double nn = (double)n;
  grid_reduce<6, 3>(acc, partials, ctl, nb, b, [=](const double (&tot)[6]) {
    feats[0] = (float)log10(fmax(tot[3], 1e-30));
    feats[1] = (float)log10(fmax(tot[0] / nn, 1e-30));
    feats[2] = (float)log10(tot[4]);
    feats[3] = (float)log10(tot[1] / nn);
    feats[4] = (float)tot[5];
    feats[5] = (float)(tot[2] / nn);
    feats[6] = (float)log10(hx);
    feats[7] = (float)log10(hy);
    feats[8] = (float)log10(dt);
  });
}

}  // namespace adl
