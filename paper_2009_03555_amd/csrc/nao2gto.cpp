// NAO2GTO: a numerical radial function R(r) on a grid, fitted by a short
// contraction of Gaussians sum_k c_k r^l exp(-a_k r^2), so that the
// exchange build can evaluate its integrals analytically (the paper's
// Introduction and Background: NAOs keep their strict cutoff, their GTO
// fits enter the ERIs).  Host code, run once per radial function before
// planning.
//
// Objective: the weighted squared error sum_i w_i (R(r_i) - f(r_i))^2 with
// w_i = r_i^2 dr_i (trapezoid weights of the radial measure, i.e. the 3-D
// L2 norm of the radial part).  Exponents are even-tempered, a_k = a_0 b^k:
// for given (a_0, b) the coefficients are the weighted linear least-squares
// solution (Householder QR), and (log a_0, log b) is chosen by a grid search
// over a bounded box followed by a Nelder-Mead refinement from the best
// grid point.  Even-tempered exponents keep the fit well conditioned (no two
// exponents collapse onto each other with large cancelling coefficients)
// and the two-parameter search finds the box's global minimum.
#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/hfx.h"

namespace hfx {
hfx_status report_error(hfx_status st, const char *msg);
}

namespace {

// search box of (log a_0, log b): a_0 from 0.1 / r_max^2 to 5 bohr^-2, b from
// 1.5 to 8; the grid has kGridA x kGridB points
constexpr double kBetaLo = 1.5, kBetaHi = 8.0, kA0Hi = 5.0;
constexpr int kGridA = 64, kGridB = 48;

// weighted least squares min |y - A c| for A (n x m, column-major), both
// already scaled by sqrt(w), by Householder QR; false if rank-deficient
bool wls(int n, int m, std::vector<double> a, std::vector<double> y, double *c) {
  for (int j = 0; j < m; ++j) {
    double nrm = 0.0;
    for (int i = j; i < n; ++i) nrm += a[(size_t)j * n + i] * a[(size_t)j * n + i];
    nrm = std::sqrt(nrm);
    if (!(nrm > 0.0)) return false;
    const double alpha = a[(size_t)j * n + j] > 0 ? -nrm : nrm;
    std::vector<double> v(n, 0.0);
    for (int i = j; i < n; ++i) v[i] = a[(size_t)j * n + i];
    v[j] -= alpha;
    double vv = 0.0;
    for (int i = j; i < n; ++i) vv += v[i] * v[i];
    if (vv == 0.0) return false;
    for (int k = j; k < m; ++k) {
      double d = 0.0;
      for (int i = j; i < n; ++i) d += v[i] * a[(size_t)k * n + i];
      d = 2.0 * d / vv;
      for (int i = j; i < n; ++i) a[(size_t)k * n + i] -= d * v[i];
    }
    double d = 0.0;
    for (int i = j; i < n; ++i) d += v[i] * y[i];
    d = 2.0 * d / vv;
    for (int i = j; i < n; ++i) y[i] -= d * v[i];
  }
  for (int j = m - 1; j >= 0; --j) {
    double s = y[j];
    for (int k = j + 1; k < m; ++k) s -= a[(size_t)k * n + j] * c[k];
    const double diag = a[(size_t)j * n + j];
    if (!(std::fabs(diag) > 1e-300)) return false;
    c[j] = s / diag;
  }
  return true;
}

struct Fit {
  int l, n, m;
  const double *r, *R;
  std::vector<double> sw;  // sqrt of the weights
  double lo[2], hi[2];     // box of (log a_0, log b)
  // objective at p = (log a_0, log b), clamped into the box; coefficients
  // into c (if not null); +inf if the least-squares problem is singular
  double cost(const double *p, double *c = nullptr) const {
    const double la = std::min(std::max(p[0], lo[0]), hi[0]);
    const double lb = std::min(std::max(p[1], lo[1]), hi[1]);
    std::vector<double> a((size_t)n * m), y(n), cc(m);
    for (int i = 0; i < n; ++i) {
      const double rl = std::pow(r[i], l);
      y[i] = sw[i] * R[i];
      for (int k = 0; k < m; ++k) a[(size_t)k * n + i] = sw[i] * rl * std::exp(-std::exp(la + k * lb) * r[i] * r[i]);
    }
    if (!wls(n, m, a, y, cc.data())) return INFINITY;
    double s = 0.0;
    for (int i = 0; i < n; ++i) {
      double f = 0.0;
      for (int k = 0; k < m; ++k) f += a[(size_t)k * n + i] * cc[k];
      s += (y[i] - f) * (y[i] - f);
    }
    if (c)
      for (int k = 0; k < m; ++k) c[k] = cc[k];
    return s;
  }
};

}  // namespace

extern "C" hfx_status hfx_nao2gto_fit(int32_t l, int32_t n_r, const double *r, const double *radial, int32_t n_gto,
                                      double *exps_out, double *coefs_out, double *rms_out) {
  using hfx::report_error;
  if (l < 0 || l > HFX_MAX_L) return report_error(HFX_ERR_INVALID, "angular momentum outside 0..HFX_MAX_L");
  if (n_gto < 1 || n_gto > HFX_MAX_PRIM) return report_error(HFX_ERR_INVALID, "n_gto outside 1..HFX_MAX_PRIM");
  if (!r || !radial || !exps_out || !coefs_out) return report_error(HFX_ERR_INVALID, "NULL argument");
  if (n_r < 2 * n_gto + 2) return report_error(HFX_ERR_INVALID, "fewer than 2 n_gto + 2 grid points");
  for (int i = 0; i < n_r; ++i) {
    if (!std::isfinite(r[i]) || !std::isfinite(radial[i]) || r[i] < 0.0)
      return report_error(HFX_ERR_INVALID, "non-finite or negative grid value");
    if (i && !(r[i] > r[i - 1])) return report_error(HFX_ERR_INVALID, "grid not increasing");
  }
  Fit F{l, n_r, n_gto, r, radial, std::vector<double>(n_r), {0, 0}, {0, 0}};
  for (int i = 0; i < n_r; ++i) {
    const double lo = i ? 0.5 * (r[i] - r[i - 1]) : 0.0;
    const double hi = i + 1 < n_r ? 0.5 * (r[i + 1] - r[i]) : 0.0;
    F.sw[i] = std::sqrt(r[i] * r[i] * (lo + hi));
  }
  double norm2 = 0.0;
  for (int i = 0; i < n_r; ++i) norm2 += F.sw[i] * F.sw[i] * radial[i] * radial[i];
  if (!(norm2 > 0.0)) return report_error(HFX_ERR_INVALID, "the radial function is zero on the grid");
  const double rmax = r[n_r - 1];
  F.lo[0] = std::log(0.1 / (rmax * rmax));
  F.hi[0] = std::log(kA0Hi);
  F.lo[1] = std::log(kBetaLo);
  F.hi[1] = n_gto > 1 ? std::log(kBetaHi) : std::log(kBetaLo);
  if (!(F.hi[0] > F.lo[0])) return report_error(HFX_ERR_INVALID, "grid too short for the exponent range");
  // grid search
  double best[2] = {F.lo[0], F.lo[1]}, fbest = INFINITY;
  const int nb = n_gto > 1 ? kGridB : 1;
  for (int i = 0; i < kGridA; ++i)
    for (int j = 0; j < nb; ++j) {
      const double p[2] = {F.lo[0] + (F.hi[0] - F.lo[0]) * i / (kGridA - 1.0),
                           nb > 1 ? F.lo[1] + (F.hi[1] - F.lo[1]) * j / (nb - 1.0) : F.lo[1]};
      const double f = F.cost(p);
      if (f < fbest) {
        fbest = f;
        best[0] = p[0];
        best[1] = p[1];
      }
    }
  if (!std::isfinite(fbest)) return report_error(HFX_ERR_UNSUPPORTED, "no well-posed fit in the exponent box");
  // Nelder-Mead from the best grid point, simplex of one grid step per axis
  const int dim = n_gto > 1 ? 2 : 1;
  double s[3][2], fs[3];
  const double step[2] = {(F.hi[0] - F.lo[0]) / (kGridA - 1.0), (F.hi[1] - F.lo[1]) / (kGridB - 1.0)};
  for (int v = 0; v <= dim; ++v) {
    s[v][0] = best[0];
    s[v][1] = best[1];
    if (v) s[v][v - 1] += step[v - 1];
    for (int d = 0; d < 2; ++d) s[v][d] = std::min(std::max(s[v][d], F.lo[d]), F.hi[d]);
    fs[v] = F.cost(s[v]);
  }
  for (int it = 0; it < 2000; ++it) {
    int o[3] = {0, 1, 2};
    std::sort(o, o + dim + 1, [&](int a, int b) { return fs[a] < fs[b]; });
    const int wv = o[dim];
    double size = 0.0;
    for (int v = 1; v <= dim; ++v)
      for (int d = 0; d < dim; ++d) size = std::max(size, std::fabs(s[o[v]][d] - s[o[0]][d]));
    if (size < 1e-12 || fs[wv] - fs[o[0]] <= 1e-15 * fs[o[0]]) break;
    double cen[2] = {0, 0};
    for (int v = 0; v < dim; ++v)
      for (int d = 0; d < dim; ++d) cen[d] += s[o[v]][d] / dim;
    auto point = [&](double t, double *q) {
      for (int d = 0; d < 2; ++d) q[d] = d < dim ? cen[d] + t * (s[wv][d] - cen[d]) : s[wv][d];
      for (int d = 0; d < 2; ++d) q[d] = std::min(std::max(q[d], F.lo[d]), F.hi[d]);
    };
    double xr[2], xe[2], xc[2];
    point(-1.0, xr);
    const double fr = F.cost(xr);
    if (fr < fs[o[0]]) {
      point(-2.0, xe);
      const double fe = F.cost(xe);
      if (fe < fr) {
        s[wv][0] = xe[0], s[wv][1] = xe[1], fs[wv] = fe;
      } else {
        s[wv][0] = xr[0], s[wv][1] = xr[1], fs[wv] = fr;
      }
    } else if (fr < fs[o[dim - 1]]) {
      s[wv][0] = xr[0], s[wv][1] = xr[1], fs[wv] = fr;
    } else {
      point(fr < fs[wv] ? -0.5 : 0.5, xc);
      const double fc = F.cost(xc);
      if (fc < std::min(fr, fs[wv])) {
        s[wv][0] = xc[0], s[wv][1] = xc[1], fs[wv] = fc;
      } else {  // shrink towards the best vertex
        for (int v = 1; v <= dim; ++v) {
          for (int d = 0; d < dim; ++d) s[o[v]][d] = s[o[0]][d] + 0.5 * (s[o[v]][d] - s[o[0]][d]);
          fs[o[v]] = F.cost(s[o[v]]);
        }
      }
    }
  }
  int bv = 0;
  for (int v = 1; v <= dim; ++v)
    if (fs[v] < fs[bv]) bv = v;
  double p[2] = {std::min(std::max(s[bv][0], F.lo[0]), F.hi[0]), std::min(std::max(s[bv][1], F.lo[1]), F.hi[1])};
  std::vector<double> c(n_gto);
  const double f = F.cost(p, c.data());
  for (int k = 0; k < n_gto; ++k) {
    exps_out[k] = std::exp(p[0] + k * p[1]);
    coefs_out[k] = c[k];
  }
  if (rms_out) *rms_out = std::sqrt(f / norm2);
  return HFX_OK;
}
