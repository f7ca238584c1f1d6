// Offline stage of Polar Express: the greedy minimax schedule in FP64 on the host.
//
// Theorem 1 (Section 3.1): the optimal composition of odd polynomials is found
// greedily; p_t is the minimax odd quintic approximating 1 on [l_t, u_t] and
// the next interval is [p_t(l_t), 2 - p_t(l_t)] (eq. newbounds).
// Each p_t comes from the degree-5 exchange of Appendix E (Algorithm 3):
// with trial points {lo, x1, x2, hi} solve the 4x4 system of eq. (linearsystem)
// for (a, b, c, E), move x1 < x2 to the positive roots of 5c x^4 + 3b x^2 + a,
// and stop when |E| no longer changes.  Near lo = hi the minimax polynomial is
// the Newton-Schulz quintic (Appendix E); below 1 - 5e-6 we run the exchange.
// Finite precision (Section 3.4, Appendix F): the design interval's lower end
// is cushioned to max(l_t, cushion * u_t) and the quintic is re-centred so that
// p(l_t) + p(u_t) = 2; afterwards each non-Newton-Schulz step is replaced by
// p_t(x / safety).
#include <cmath>
#include <cstring>

#include "pe.h"

namespace {

constexpr double kCushion = 0.02407327424182761;
constexpr double kDegenerate = 1.0 - 5e-6;

struct Quintic {
  double a, b, c;
  double eval(double x) const {
    const double y = x * x;
    return x * (a + y * (b + c * y));
  }
};

// Solve M z = r for a 4x4 system by Gaussian elimination with partial pivoting.
bool solve4(double M[4][4], double r[4], double z[4]) {
  for (int col = 0; col < 4; ++col) {
    int piv = col;
    for (int i = col + 1; i < 4; ++i)
      if (std::fabs(M[i][col]) > std::fabs(M[piv][col])) piv = i;
    if (M[piv][col] == 0.0) return false;
    if (piv != col) {
      for (int j = 0; j < 4; ++j) std::swap(M[col][j], M[piv][j]);
      std::swap(r[col], r[piv]);
    }
    for (int i = col + 1; i < 4; ++i) {
      const double f = M[i][col] / M[col][col];
      for (int j = col; j < 4; ++j) M[i][j] -= f * M[col][j];
      r[i] -= f * r[col];
    }
  }
  for (int i = 3; i >= 0; --i) {
    double s = r[i];
    for (int j = i + 1; j < 4; ++j) s -= M[i][j] * z[j];
    z[i] = s / M[i][i];
  }
  return true;
}

// Minimax odd quintic for the constant 1 on [lo, hi]; returns false if the
// exchange breaks down (singular system or complex critical points).
bool exchange(double lo, double hi, Quintic* out, int* iters, bool* ns5) {
  *ns5 = false;
  if (lo / hi >= kDegenerate) {
    *out = {15.0 / 8.0, -10.0 / 8.0, 3.0 / 8.0};
    *ns5 = true;
    *iters = 0;
    return true;
  }
  double x1 = 0.75 * lo + 0.25 * hi;
  double x2 = 0.25 * lo + 0.75 * hi;
  double prevE = INFINITY;
  Quintic q{0, 0, 0};
  for (int it = 1; it <= 100; ++it) {
    const double pts[4] = {lo, x1, x2, hi};
    double M[4][4], r[4] = {1, 1, 1, 1}, z[4];
    for (int i = 0; i < 4; ++i) {
      const double x = pts[i], x2p = x * x;
      M[i][0] = x;
      M[i][1] = x * x2p;
      M[i][2] = x * x2p * x2p;
      M[i][3] = (i % 2 == 0) ? 1.0 : -1.0;
    }
    if (!solve4(M, r, z)) return false;
    q = {z[0], z[1], z[2]};
    const double E = z[3];
    const double disc = 9.0 * q.b * q.b - 20.0 * q.a * q.c;
    if (!(disc >= 0.0) || q.c == 0.0) return false;
    const double sd = std::sqrt(disc);
    const double y1 = (-3.0 * q.b - sd) / (10.0 * q.c);
    const double y2 = (-3.0 * q.b + sd) / (10.0 * q.c);
    if (!(y1 > 0.0) || !(y2 > 0.0)) return false;
    x1 = std::sqrt(y1);
    x2 = std::sqrt(y2);
    *iters = it;
    if (std::fabs(std::fabs(E) - std::fabs(prevE)) <= 1e-15) {
      *out = q;
      return true;
    }
    prevE = E;
  }
  *out = q;
  return false;
}

}  // namespace

extern "C" void pe_coeff_opts_default(pe_coeff_opts* opts) {
  if (!opts) return;
  opts->cushion = kCushion;
  opts->safety = 1.01;
  opts->safety_on_last = 1;
}

extern "C" pe_status pe_coeffs(double ell, int32_t T, const pe_coeff_opts* opts, double* abc,
                               double* bounds, double* err_bound, int32_t* iters) {
  pe_coeff_opts o;
  pe_coeff_opts_default(&o);
  if (opts) o = *opts;
  if (!abc || !(ell > 0.0) || !(ell < 1.0) || T < 1 || T > 64) return PE_EINVAL;
  if (!(o.safety >= 1.0) || !(o.cushion < 1.0) || !std::isfinite(o.cushion)) return PE_EINVAL;
  const bool tenth = o.cushion < 0.0;
  double l = ell, u = 1.0;
  bool ns5[64];
  if (bounds) {
    bounds[0] = l;
    bounds[1] = u;
  }
  for (int t = 0; t < T; ++t) {
    const double lo = tenth ? std::fmax(l, u / 10.0) : std::fmax(l, o.cushion * u);
    Quintic q;
    int it = 0;
    bool dg = false;
    if (!exchange(lo, u, &q, &it, &dg)) return PE_ENOCONV;
    if (!dg && !tenth) {
      const double k = 2.0 / (q.eval(l) + q.eval(u));
      q.a *= k;
      q.b *= k;
      q.c *= k;
    }
    ns5[t] = dg;
    if (iters) iters[t] = it;
    abc[3 * t + 0] = q.a;
    abc[3 * t + 1] = q.b;
    abc[3 * t + 2] = q.c;
    l = q.eval(l);
    u = 2.0 - l;
    if (bounds) {
      bounds[2 * (t + 1) + 0] = l;
      bounds[2 * (t + 1) + 1] = u;
    }
  }
  if (err_bound) *err_bound = 1.0 - l;
  if (o.safety != 1.0) {
    const double s1 = o.safety, s3 = s1 * s1 * s1, s5 = s3 * s1 * s1;
    for (int t = 0; t < T; ++t) {
      if (ns5[t]) continue;
      if (!o.safety_on_last && t == T - 1) continue;
      abc[3 * t + 0] /= s1;
      abc[3 * t + 1] /= s3;
      abc[3 * t + 2] /= s5;
    }
  }
  return PE_OK;
}
