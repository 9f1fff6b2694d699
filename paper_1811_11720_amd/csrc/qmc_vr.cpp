// qmc_vr.cpp -- fit of the variance-reduction map (Sec. 2.4).
//
// For each dimension j the per-dimension histogram of |f| over one shifted
// lattice gives the CDF of eq. (CDF) at the bin edges e_b = b / bins:
// C_b = sum_{b' < b} h[b'] / sum h.  The map p of eq. ISfit (PolySingular form
// of App. A.5, with |p2| and |p3|) should be the inverse CDF, so it is fitted
// to the points (C_b, e_b) by unweighted nonlinear least squares:
//   r_b(a) = p(C_b; a) - e_b,  b = 0..bins.
// Levenberg-Marquardt with the analytic Jacobian under the paper's bounds
// p0 >= 1.001, p1 <= -0.001, p2 >= 0, p3 >= 0: a parameter that sits on its
// bound while the gradient points out of the box is held fixed for that step
// (without this, |p3| of a term that wants to vanish flips sign at every step
// and the fit crawls), and every step is projected back into the box.
// Stopping rules follow the paper's defaults (App. A.1): at most 40 iterations,
// step tolerance 3e-3, gradient tolerance 1e-8, cost tolerance 1e-8.  A fit is
// accepted only if p' > 0 on a 4097-point grid; otherwise the identity map is
// returned and the dimension's fallback bit is set.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace qmcv {

namespace {

struct Model {
  // p(y) and its gradient with respect to the six parameters
  static double eval(const double* a, double y, double* grad) {
    const double p0 = a[0], p1 = a[1], p2 = std::fabs(a[2]), p3 = std::fabs(a[3]), p4 = a[4], p5 = a[5];
    const double s2 = a[2] >= 0 ? 1.0 : -1.0, s3 = a[3] >= 0 ? 1.0 : -1.0;
    const double c3 = 1.0 - p2 - p3 - p4 - p5;
    const double f0 = y * (p0 - 1.0) / (p0 - y);
    const double f1 = y * (p1 - 1.0) / (p1 - y);
    const double y2 = y * y, y3 = y2 * y;
    if (grad) {
      grad[0] = p2 * y * (1.0 - y) / ((p0 - y) * (p0 - y));
      grad[1] = p3 * y * (1.0 - y) / ((p1 - y) * (p1 - y));
      grad[2] = s2 * (f0 - y3);
      grad[3] = s3 * (f1 - y3);
      grad[4] = y - y3;
      grad[5] = y2 - y3;
    }
    return p2 * f0 + p3 * f1 + p4 * y + p5 * y2 + c3 * y3;
  }
  static double deriv(const double* a, double y) {
    const double p0 = a[0], p1 = a[1], p2 = std::fabs(a[2]), p3 = std::fabs(a[3]), p4 = a[4], p5 = a[5];
    const double c3 = 1.0 - p2 - p3 - p4 - p5;
    return p2 * p0 * (p0 - 1.0) / ((p0 - y) * (p0 - y)) + p3 * p1 * (p1 - 1.0) / ((p1 - y) * (p1 - y)) + p4 +
           2.0 * p5 * y + 3.0 * c3 * y * y;
  }
};

constexpr double kLo[6] = {1.001, -HUGE_VAL, 0.0, 0.0, -HUGE_VAL, -HUGE_VAL};
constexpr double kHi[6] = {HUGE_VAL, -0.001, HUGE_VAL, HUGE_VAL, HUGE_VAL, HUGE_VAL};

void project(double* a) {
  for (int i = 0; i < 6; ++i) {
    if (!(a[i] >= kLo[i])) a[i] = kLo[i];
    if (!(a[i] <= kHi[i])) a[i] = kHi[i];
  }
}

double cost(const double* a, const std::vector<double>& C, const std::vector<double>& e) {
  double s = 0.0;
  for (size_t b = 0; b < C.size(); ++b) {
    double r = Model::eval(a, C[b], nullptr) - e[b];
    s += r * r;
  }
  return 0.5 * s;
}

// solve the 6x6 system M x = r (Gaussian elimination with partial pivoting)
bool solve6(double M[6][6], double* r) {
  for (int c = 0; c < 6; ++c) {
    int p = c;
    for (int i = c + 1; i < 6; ++i)
      if (std::fabs(M[i][c]) > std::fabs(M[p][c])) p = i;
    if (!(std::fabs(M[p][c]) > 0.0)) return false;
    if (p != c) {
      for (int k = 0; k < 6; ++k) std::swap(M[c][k], M[p][k]);
      std::swap(r[c], r[p]);
    }
    for (int i = c + 1; i < 6; ++i) {
      double f = M[i][c] / M[c][c];
      for (int k = c; k < 6; ++k) M[i][k] -= f * M[c][k];
      r[i] -= f * r[c];
    }
  }
  for (int c = 5; c >= 0; --c) {
    double s = r[c];
    for (int k = c + 1; k < 6; ++k) s -= M[c][k] * r[k];
    r[c] = s / M[c][c];
  }
  return true;
}

bool monotone(const double* a) {
  for (int i = 0; i <= 4096; ++i) {
    double y = i / 4096.0;
    double d = Model::deriv(a, y);
    if (!(d > 0.0) || !std::isfinite(d)) return false;
  }
  return true;
}

}  // namespace

void identity_params(double* a) {
  a[0] = 2.0;
  a[1] = -1.0;
  a[2] = 0.0;
  a[3] = 0.0;
  a[4] = 1.0;
  a[5] = 0.0;
}

// Fit one dimension; returns true if accepted (else `a` holds the identity).
bool fit_dimension(const double* hist, uint32_t bins, double* a) {
  double tot = 0.0;
  for (uint32_t b = 0; b < bins; ++b) tot += hist[b];
  if (!(tot > 0.0) || !std::isfinite(tot)) {
    identity_params(a);
    return false;
  }
  std::vector<double> C(bins + 1), e(bins + 1);
  double run = 0.0;
  for (uint32_t b = 0; b <= bins; ++b) {
    C[b] = std::min(1.0, run / tot);
    e[b] = (double)b / bins;
    if (b < bins) run += hist[b];
  }
  C[bins] = 1.0;
  double x[6] = {1.5, -0.5, 0.01, 0.01, 1.0, 0.0};
  double f = cost(x, C, e);
  double mu = 1e-3;
  const int maxiter = 40;
  const double xtol = 3e-3, gtol = 1e-8, ftol = 1e-8;
  for (int it = 0; it < maxiter; ++it) {
    double A[6][6] = {{0}}, g[6] = {0}, grad[6];
    for (size_t b = 0; b < C.size(); ++b) {
      double r = Model::eval(x, C[b], grad) - e[b];
      for (int i = 0; i < 6; ++i) {
        g[i] += grad[i] * r;
        for (int k = 0; k < 6; ++k) A[i][k] += grad[i] * grad[k];
      }
    }
    // held: on a bound with the descent direction -g leaving the box
    bool held[6];
    double gmax = 0.0;
    for (int i = 0; i < 6; ++i) {
      held[i] = (x[i] <= kLo[i] && g[i] > 0.0) || (x[i] >= kHi[i] && g[i] < 0.0);
      if (!held[i]) gmax = std::max(gmax, std::fabs(g[i]));
    }
    if (gmax <= gtol) break;
    bool accepted = false;
    for (int tries = 0; tries < 12 && !accepted; ++tries) {
      double M[6][6], d[6];
      for (int i = 0; i < 6; ++i) {
        for (int k = 0; k < 6; ++k) M[i][k] = (held[i] || held[k]) ? 0.0 : A[i][k];
        M[i][i] = held[i] ? 1.0 : M[i][i] + mu * std::max(A[i][i], 1e-12);
        d[i] = held[i] ? 0.0 : -g[i];
      }
      if (!solve6(M, d)) {
        mu *= 4.0;
        continue;
      }
      double xn[6];
      for (int i = 0; i < 6; ++i) xn[i] = x[i] + d[i];
      project(xn);
      double fn = cost(xn, C, e);
      if (std::isfinite(fn) && fn < f) {
        bool small = true;
        for (int i = 0; i < 6; ++i) small = small && std::fabs(xn[i] - x[i]) <= xtol * (std::fabs(x[i]) + xtol);
        double df = f - fn;
        std::memcpy(x, xn, sizeof x);
        f = fn;
        mu = std::max(mu / 3.0, 1e-12);
        accepted = true;
        if (small || df <= ftol * f) it = maxiter;  // converged
      } else {
        mu *= 4.0;
      }
    }
    if (!accepted) break;
  }
  if (!monotone(x)) {
    identity_params(a);
    return false;
  }
  std::memcpy(a, x, sizeof x);
  return true;
}

}  // namespace qmcv
