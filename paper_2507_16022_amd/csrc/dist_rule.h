// Distance marginalisation of the per-triple likelihood (eq. lnl_dist_marginalized
// with a prior proportional to D^2 on (0, D_max], Sec. IV B).
//
// In the variables z = dh / sqrt(hh) (data projected on the unit template)
// and s = sqrt(hh) d0 / D_max (template SNR at the largest distance), with
// r = D / D_max:
//     Lbar(z, s) = 3 * int_0^1 r^2 exp(z s / r - s^2 / (2 r^2)) dr
// which is the same as 3 s^3 int_s^inf y^-4 exp(z y - y^2/2) dy (y = s/r).
// Only (z, s) matter: d0 and D_max enter through s alone.
//
// Three evaluation routes, all in FP64:
//   * dr_ln_exact: composite adaptive Gauss-Legendre over r with
//     breakpoints at the stationary points of the log-integrand; used to
//     build the table and for arguments outside it;
//   * a table of ln Lbar on a grid in (z, w), w = ln s for s < 1 and
//     w = s - 1 above (logarithmic resolution where Lbar depends on ln s,
//     linear where it depends on s; w is cheap to form from s), both axes
//     in uniform segments, read with 4x4 tensor-product cubic Lagrange
//     interpolation;
//   * the high-SNR tail (peak far inside the domain and dominant):
//     Gaussian-Hermite quadrature of E[(z + eps)^-4], eps ~ N(0, 1).
#pragma once

#ifndef __HIPCC__
#ifndef __host__
#define __host__
#define __device__
#define __forceinline__ inline
#endif
#endif

#include <math.h>

namespace dotpe {

// table geometry (shared by builder and reader): both axes are split into
// uniform segments, each stored with two guard lines on either side so that
// a stencil never crosses a segment edge.  z (columns): finer where the
// prior-dominated and peak-dominated regimes of the integrand cross; w
// (rows): w = ln s below w = 0 (s < 1) and w = s - 1 above, finer where the
// two maps meet.
constexpr int kDrSeg = 4;       // z segments
constexpr int kDrRowSeg = 4;    // w segments
struct DistTableGeom {
  double ihz[kDrSeg];               // reciprocal steps (whole numbers)
  double zlo[kDrSeg], zhi[kDrSeg];  // z range served by each segment
  int nz[kDrSeg], off[kDrSeg];      // columns per segment (guards included), column offset
  double ihw[kDrRowSeg];            // the same for the rows
  double wlo[kDrRowSeg], whi[kDrRowSeg];
  int nw[kDrRowSeg], roff[kDrRowSeg];
  bool wlog[kDrRowSeg];             // the segment's rows have s = e^w (else s = 1 + w)
  int nrow, ncol;                   // total rows and columns
};

// (strongly negative z, the anti-aligned phases of loud pairs, is smooth and
// takes a coarser step)
constexpr double kDrSegEdge[kDrSeg + 1] = {-64.0, -12.0, 2.0, 14.0, 32.0};
constexpr double kDrSegStep[kDrSeg] = {0.1, 0.05, 0.0125, 0.05};
// w from ln(1e-9) to 19 (s = 20); half steps for 0.135 < s < 3
constexpr double kDrRowEdge[kDrRowSeg + 1] = {-20.75, -2.0, 0.0, 2.0, 19.0};
constexpr double kDrRowStep[kDrRowSeg] = {0.025, 0.0125, 0.0125, 0.025};
constexpr double kDrSMin = 1e-9;     // below: small-s expansion
constexpr int kGH = 12;              // Gauss-Hermite nodes for the tail

__host__ __device__ constexpr DistTableGeom dr_make_geom() {
  DistTableGeom g{};
  int off = 0;
  for (int k = 0; k < kDrSeg; ++k) {
    const double h = kDrSegStep[k];
    g.ihz[k] = 1.0 / h;
    g.zlo[k] = kDrSegEdge[k];
    g.zhi[k] = kDrSegEdge[k + 1];
    g.nz[k] = (int)((kDrSegEdge[k + 1] - kDrSegEdge[k]) / h + 0.5) + 5;
    g.off[k] = off;
    off += g.nz[k];
  }
  g.ncol = off;
  int roff = 0;
  for (int k = 0; k < kDrRowSeg; ++k) {
    const double h = kDrRowStep[k];
    g.ihw[k] = 1.0 / h;
    g.wlo[k] = kDrRowEdge[k];
    g.whi[k] = kDrRowEdge[k + 1];
    g.nw[k] = (int)((kDrRowEdge[k + 1] - kDrRowEdge[k]) / h + 0.5) + 5;
    g.roff[k] = roff;
    g.wlog[k] = kDrRowEdge[k + 1] <= 0.0;
    roff += g.nw[k];
  }
  g.nrow = roff;
  return g;
}

// The geometry as compile-time constants: the reader below folds every
// segment parameter into its instructions (no loads, no registers held).
constexpr DistTableGeom kDrGeom = dr_make_geom();
static_assert(kDrRowEdge[2] == 0.0, "the two row maps meet at w = 0, a segment edge");
// the reader forms positions as (x - edge) / step + 2 with the reciprocal
// step: both must be exact in binary for the builder's nodes to sit at whole
// positions (to rounding)
constexpr bool dr_exact_recip(double h) { return (1.0 / h) * h == 1.0 && (double)(int)(1.0 / h) == 1.0 / h; }
static_assert(dr_exact_recip(kDrSegStep[0]) && dr_exact_recip(kDrSegStep[1]) &&
                  dr_exact_recip(kDrSegStep[2]) && dr_exact_recip(kDrSegStep[3]) &&
                  dr_exact_recip(kDrRowStep[0]) && dr_exact_recip(kDrRowStep[1]) &&
                  dr_exact_recip(kDrRowStep[2]) && dr_exact_recip(kDrRowStep[3]),
              "table steps with whole reciprocals");

// Natural logarithm of a positive normal x: x = m 2^e with m in
// [sqrt(1/2), sqrt(2)), ln m = 2 atanh(t) with t = (m - 1) / (m + 1),
// |t| < 0.172, by the atanh series through t^17 (the rest is below 3e-16).
// About a quarter of the instructions of the math library's version, and
// accurate to a few units in the last place of ln x's absolute value.
__device__ __forceinline__ double dr_log(double x) {
  int e;
  double m = frexp(x, &e);             // m in [1/2, 1)
  if (m < 0.70710678118654752) {
    m *= 2.0;
    --e;
  }
  const double t = (m - 1.0) / (m + 1.0), t2 = t * t;
  double p = 1.0 / 17.0;
  p = fma(p, t2, 1.0 / 15.0);
  p = fma(p, t2, 1.0 / 13.0);
  p = fma(p, t2, 1.0 / 11.0);
  p = fma(p, t2, 1.0 / 9.0);
  p = fma(p, t2, 1.0 / 7.0);
  p = fma(p, t2, 1.0 / 5.0);
  p = fma(p, t2, 1.0 / 3.0);
  p = fma(p, t2, 1.0);
  return fma((double)e, 0.69314718055994531, 2.0 * t * p);
}

// 1 / d for d > 0 of moderate range: the FP32 reciprocal refined by two
// Newton steps in FP64 (relative error squared per step: below 1e-15)
__device__ __forceinline__ double dr_rcp(double d) {
  double y = (double)__builtin_amdgcn_rcpf((float)d);
  y = y * fma(-d, y, 2.0);
  return y * fma(-d, y, 2.0);
}

// z of stored column `col` (any segment)
__device__ inline double dr_col_z(const DistTableGeom& g, int col) {
  int k = 0;
  while (k + 1 < kDrSeg && col >= g.off[k + 1]) ++k;
  return g.zlo[k] + (col - g.off[k] - 2) / g.ihz[k];     // two guard columns below the edge
}

__host__ __device__ __forceinline__ double dr_psi(double r, double a, double b) {
  // log-integrand without the constant ln 3: 2 ln r + a/r - b/(2 r^2)
  return 2.0 * log(r) + a / r - 0.5 * b / (r * r);
}

__host__ __device__ __forceinline__ void dr_gl16(double* x, double* w) {
  // 16-point Gauss-Legendre on [-1, 1] (abscissae, weights)
  const double xs[8] = {0.0950125098376374401853193, 0.2816035507792589132304605,
                        0.4580167776572273863424194, 0.6178762444026437484466718,
                        0.7554044083550030338951012, 0.8656312023878317438804679,
                        0.9445750230732325760779884, 0.9894009349916499325961542};
  const double ws[8] = {0.1894506104550684962853967, 0.1826034150449235888667637,
                        0.1691565193950025381893121, 0.1495959888165767320815017,
                        0.1246289712555338720524763, 0.0951585116824927848099251,
                        0.0622535239386478928628438, 0.0271524594117540948517806};
  for (int k = 0; k < 8; ++k) {
    x[k] = -xs[7 - k]; w[k] = ws[7 - k];
    x[8 + k] = xs[k]; w[8 + k] = ws[k];
  }
}

// integral of exp(psi(r) - pmax) over [lo, hi] with a 16-point rule
__host__ __device__ __forceinline__ double dr_panel(double lo, double hi, double a, double b,
                                                    double pmax, const double* gx, const double* gw) {
  double c = 0.5 * (lo + hi), h = 0.5 * (hi - lo), s = 0.0;
  for (int k = 0; k < 16; ++k) {
    double r = c + h * gx[k];
    if (r > 0.0) s += gw[k] * exp(dr_psi(r, a, b) - pmax);
  }
  return s * h;
}

// ln Lbar(z, s), robust and accurate to ~1e-13 relative.
__host__ __device__ inline __attribute__((noinline)) double dr_ln_exact(double z, double s) {
  if (!(s > 0.0)) return 0.0;
  const double a = z * s, b = s * s;
  double gx[16], gw[16];
  dr_gl16(gx, gw);
  // stationary points of psi: 2 r^2 - a r + b = 0
  double rm = -1.0, rp = -1.0;
  if (a > 0.0 && a * a > 8.0 * b) {
    double sq = sqrt(a * a - 8.0 * b);
    rp = 0.25 * (a + sq);
    rm = 2.0 * b / (a + sq);           // = (a - sq)/4 without cancellation
  }
  double pmax = dr_psi(1.0, a, b);
  bool have_peak = rm > 0.0 && rm < 1.0;
  if (have_peak) pmax = fmax(pmax, dr_psi(rm, a, b));
  // breakpoints
  double pts[48];
  int np = 0;
  pts[np++] = 0.0;
  pts[np++] = 1.0;
  if (have_peak) {
    double d2 = -2.0 / (rm * rm) + 2.0 * a / (rm * rm * rm) - 3.0 * b / (rm * rm * rm * rm);
    double sig = d2 < 0.0 ? 1.0 / sqrt(-d2) : rm;
    pts[np++] = rm;
    const double ks[9] = {0.5, 1, 2, 3, 4, 6, 8, 12, 16};
    for (int k = 0; k < 9; ++k) {
      double lo = rm - ks[k] * sig, hi = rm + ks[k] * sig;
      if (lo > 0.0 && lo < 1.0) pts[np++] = lo;
      if (hi > 0.0 && hi < 1.0) pts[np++] = hi;
    }
  }
  if (rp > 0.0 && rp < 1.0) pts[np++] = rp;
  {
    // decay scale towards r -> 0 from the right end: psi'(1) = 2 - a + b
    double g = 2.0 - a + b;
    if (g > 1.0) {
      const double ks[7] = {1, 2, 4, 8, 16, 32, 64};
      for (int k = 0; k < 7; ++k) {
        double x = 1.0 - ks[k] / g;
        if (x > 0.0 && x < 1.0) pts[np++] = x;
      }
    }
    // near r -> 0 the integrand vanishes like exp(-b / 2r^2); add the scale
    double r0 = sqrt(b) / 8.0;
    if (r0 > 0.0 && r0 < 1.0) pts[np++] = r0;
  }
  // insertion sort
  for (int i = 1; i < np; ++i) {
    double v = pts[i];
    int j = i - 1;
    while (j >= 0 && pts[j] > v) { pts[j + 1] = pts[j]; --j; }
    pts[j + 1] = v;
  }
  // coarse pass: one 16-point panel per interval
  double coarse = 0.0;
  for (int p = 0; p + 1 < np; ++p)
    if (pts[p + 1] > pts[p]) coarse += dr_panel(pts[p], pts[p + 1], a, b, pmax, gx, gw);
  const double tol = 1e-16 * coarse;
  // adaptive refinement with an explicit stack: split a panel until its
  // 16-point value agrees with the sum over its two halves to a relative
  // 1e-14 or an absolute 1e-16 of the coarse total; the number of panel
  // evaluations is capped so the work is bounded for every argument
  double total = 0.0;
  int budget = 4096;
  for (int p = 0; p + 1 < np; ++p) {
    if (pts[p + 1] - pts[p] <= 0.0) continue;
    double st_lo[48], st_hi[48], st_v[48];
    st_lo[0] = pts[p]; st_hi[0] = pts[p + 1];
    st_v[0] = dr_panel(pts[p], pts[p + 1], a, b, pmax, gx, gw);
    int sp = 1;
    while (sp > 0) {
      --sp;
      double lo = st_lo[sp], hi = st_hi[sp], v = st_v[sp];
      double mid = 0.5 * (lo + hi);
      double v1 = dr_panel(lo, mid, a, b, pmax, gx, gw);
      double v2 = dr_panel(mid, hi, a, b, pmax, gx, gw);
      budget -= 2;
      double err = fabs(v1 + v2 - v);
      if (err <= fmax(1e-14 * (v1 + v2), tol) || sp >= 46 || budget <= 0) {
        total += v1 + v2;
      } else {
        st_lo[sp] = lo; st_hi[sp] = mid; st_v[sp] = v1; ++sp;
        st_lo[sp] = mid; st_hi[sp] = hi; st_v[sp] = v2; ++sp;
      }
    }
  }
  return log(3.0) + pmax + log(total);
}

// ln E[(z + eps)^-4], eps ~ N(0,1), by probabilists' Gauss-Hermite nodes
// (the tail formula is used for z >= 8 only, so z + x_k > 2 for every node)
__device__ __forceinline__ double dr_gh_ln_moment(double z, const double* ghx, const double* ghw) {
  double acc = 0.0;
  for (int k = 0; k < kGH; ++k) {
    const double y = dr_rcp(z + ghx[k]);
    const double y2 = y * y;
    acc = fma(ghw[k], y2 * y2, acc);
  }
  return dr_log(acc);
}

// value from the tail formula (peak well inside, Gaussian in y)
__device__ __forceinline__ double dr_ln_tail(double z, double s, const double* ghx,
                                             const double* ghw) {
  const double kLn3Sqrt2Pi = 2.0175508218727823;   // ln(3 sqrt(2 pi))
  return kLn3Sqrt2Pi + 3.0 * dr_log(s) + 0.5 * z * z + dr_gh_ln_moment(z, ghx, ghw);
}

// tail formula valid: Gaussian peak at y ~ z at least 8 sigma above the
// boundary y = s and the boundary region negligible next to it
__device__ __forceinline__ bool dr_tail_ok(double z, double s) {
  if (z < 8.0 || z - s < 8.0) return false;
  const double gap = 0.5 * (z - s) * (z - s) - 4.0 * dr_log(z / s);
  return gap >= 40.0;
}

// 4x4 cubic Lagrange interpolation in the table
__device__ __forceinline__ void dr_lagrange4(double t, double* c) {
  // nodes at -1, 0, 1, 2; t in [0, 1)
  const double tm1 = t - 1.0, tm2 = t - 2.0, tp1 = t + 1.0;
  c[0] = -t * tm1 * tm2 * (1.0 / 6.0);
  c[1] = tp1 * tm1 * tm2 * 0.5;
  c[2] = -tp1 * t * tm2 * 0.5;
  c[3] = tp1 * t * tm1 * (1.0 / 6.0);
}

// ln Lbar at (z, s) from the table; false when (z, s) lies outside it
__device__ __forceinline__ bool dr_table_lookup(const double* tab, double z, double s,
                                                double* out) {
  constexpr DistTableGeom g = kDrGeom;
  const double w = s < 1.0 ? dr_log(s) : s - 1.0;
  if (!(z >= g.zlo[0] && z < g.zhi[kDrSeg - 1] && w >= g.wlo[0] && w < g.whi[kDrRowSeg - 1]))
    return false;
  // each axis' segment: segments are contiguous, so the last one whose lower
  // edge is at or below the coordinate.  The position is formed from the
  // edge and the reciprocal step, which are exact in binary (the guard lines
  // add 2), so the selected constants are immediate operands.
  double zlo = g.zlo[0], ihz = g.ihz[0], wlo = g.wlo[0], ihw = g.ihw[0];
  int nz = g.nz[0], off = g.off[0], nw = g.nw[0], roff = g.roff[0];
#pragma unroll
  for (int q = 1; q < kDrSeg; ++q) {
    if (z >= g.zlo[q]) {
      zlo = g.zlo[q];
      ihz = g.ihz[q];
      nz = g.nz[q];
      off = g.off[q];
    }
  }
#pragma unroll
  for (int q = 1; q < kDrRowSeg; ++q) {
    if (w >= g.wlo[q]) {
      wlo = g.wlo[q];
      ihw = g.ihw[q];
      nw = g.nw[q];
      roff = g.roff[q];
    }
  }
  const double fz = fma(z - zlo, ihz, 2.0), fw = fma(w - wlo, ihw, 2.0);
  const double flz = floor(fz), flw = floor(fw);
  const int jz = (int)flz, jw = (int)flw;
  if (jz < 1 || jz > nz - 3 || jw < 1 || jw > nw - 3) return false;
  double cz[4], cw[4];
  dr_lagrange4(fz - flz, cz);
  dr_lagrange4(fw - flw, cw);
  const double* base = tab + ((roff + jw - 1) * g.ncol + off + (jz - 1));
  double v = 0.0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const double* row = base + a * g.ncol;
    const double rv = cz[0] * row[0] + cz[1] * row[1] + cz[2] * row[2] + cz[3] * row[3];
    v = fma(cw[a], rv, v);
  }
  *out = v;
  return true;
}

// z and s of a triple: z = dh / sqrt(hh), s = sqrt(hh) d0 / D_max (hh > 0)
__device__ __forceinline__ void dr_zs(double dh, double hh, double d0_over_dmax, double& z,
                                      double& s) {
  const double sq = sqrt(hh);
  z = dh / sq;
  s = sq * d0_over_dmax;
}

// full rule: ln Lbar for one triple given dh, hh at distance d0
__device__ __attribute__((always_inline)) inline double dr_ln_marg_body(
    double dh, double hh, double d0_over_dmax, const double* tab, const double* ghx,
    const double* ghw) {
  if (!(hh > 0.0)) return 0.0;
  double z, s;
  dr_zs(dh, hh, d0_over_dmax, z, s);
  if (s < kDrSMin) {
    // Lbar = 1 + 1.5 z s + O(s^2) plus the peak contribution if any
    double v = 1.5 * z * s;
    if (z >= 8.0) {
      double lp = dr_ln_tail(z, s, ghx, ghw);
      v += lp > 0.0 ? lp + log1p(exp(-lp)) : log1p(exp(lp));
    }
    return v;
  }
  if (dr_tail_ok(z, s)) return dr_ln_tail(z, s, ghx, ghw);
  double v;
  if (dr_table_lookup(tab, z, s, &v)) return v;
  return dr_ln_exact(z, s);
}

// The rule as a function (not inlined): for callers with few triples per
// lane, where its registers would otherwise add to their own.
__device__ __attribute__((noinline)) inline double dr_ln_marg(double dh, double hh,
                                                              double d0_over_dmax,
                                                              const double* tab,
                                                              const double* ghx,
                                                              const double* ghw) {
  return dr_ln_marg_body(dh, hh, d0_over_dmax, tab, ghx, ghw);
}

// The rule inlined (the same arithmetic, so the same values), only the
// adaptive quadrature called: for kernels whose lanes evaluate many triples
// in a loop (a call there makes every value live across it occupy a saved
// register).
__device__ __attribute__((always_inline)) inline double dr_ln_marg_inl(
    double dh, double hh, double d0_over_dmax, const double* tab, const double* ghx,
    const double* ghw) {
  return dr_ln_marg_body(dh, hh, d0_over_dmax, tab, ghx, ghw);
}

}  // namespace dotpe
