// Offline stage of Polar Express: the greedy minimax schedule in FP64 on the host.
//
// Theorem 1 (Section 3.1): the optimal composition of odd polynomials is built
// greedily -- p_t is the minimax odd quintic approximating 1 on [l_t, u_t] and
// the next interval is [p_t(l_t), 2 - p_t(l_t)] (eq. newbounds).
//
// Each p_t comes from the degree-5 exchange of Appendix E (Algorithm 3): a
// trial set {lo, x1, x2, hi} on which the error alternates in sign with a
// common magnitude E (eq. linearsystem) determines (a, b, c, E); x1 < x2 then
// move to the interior extrema of the error, the positive roots of
// p'(x) = a + 3b x^2 + 5c x^4 (a quadratic in x^2), until |E| stops changing.
// When lo/hi is within eps^(1/3) of 1 the answer is the Newton-Schulz quintic
// (Algorithm 3's degenerate branch); this library emits its exact
// coefficients (15/8, -10/8, 3/8), as the printed table does.
//
// Finite precision (Section 3.4, Appendix F): Appendix F replaces l_t by a
// cushioned lower end when l_t is far below u_t, stating a ratio-1/10 rule and
// noting that its code uses another factor.  Here the rule is applied to the
// image of the design interval: the cushion r makes the minimax quintic on
// [r u, u] map it onto an interval of ratio 1/10 (levelled error 9/11); r is
// found once by bisection (it is scale-free).  The cushioned quintic is then
// rescaled so that p(l_t) and p(u_t) sit symmetrically about 1, which is what
// the bound update of eq. newbounds needs, and finally every non-Newton-Schulz
// step is replaced by p_t(x / safety).
#include <cmath>
#include <cstring>

#include "pe.h"

namespace {

constexpr double kEps = 1.11e-16;  // Algorithm 3's machine epsilon

struct Odd5 {
  double a = 0, b = 0, c = 0;
  double at(double x) const {
    const double x2 = x * x;
    return x * (a + x2 * (b + x2 * c));
  }
};

struct Fit {
  Odd5 p;
  double E = 0;     // levelled error of the last trial set
  int exchanges = 0;
  bool ns5 = false;
};

// The levelled 4x4 system for trial points t0 < t1 < t2 < t3:
//   p(t_i) + (-1)^i E = 1,  unknowns (a, b, c, E).
// The columns x, x^3, x^5 become nearly parallel as the points cluster
// (Appendix E notes the ill-conditioning as l -> u), so elimination runs in
// long double, which keeps the coefficients accurate where float64 would lose
// six digits on the seventh step of the l = 1e-3 schedule.
bool levelled_solve(const double t[4], double out[4]) {
  long double M[4][5];
  for (int i = 0; i < 4; ++i) {
    const long double x = t[i], x2 = x * x;
    M[i][0] = x;
    M[i][1] = x * x2;
    M[i][2] = x * x2 * x2;
    M[i][3] = (i & 1) ? -1.0L : 1.0L;
    M[i][4] = 1.0L;
  }
  for (int k = 0; k < 4; ++k) {
    int best = k;
    for (int i = k + 1; i < 4; ++i)
      if (fabsl(M[i][k]) > fabsl(M[best][k])) best = i;
    if (M[best][k] == 0.0L) return false;
    if (best != k)
      for (int j = 0; j < 5; ++j) {
        const long double tmp = M[k][j];
        M[k][j] = M[best][j];
        M[best][j] = tmp;
      }
    for (int i = 0; i < 4; ++i) {
      if (i == k) continue;
      const long double f = M[i][k] / M[k][k];
      for (int j = k; j < 5; ++j) M[i][j] -= f * M[k][j];
    }
  }
  for (int i = 0; i < 4; ++i) out[i] = (double)(M[i][4] / M[i][i]);
  return true;
}

// Minimax odd quintic for 1 on [lo, hi] (Algorithm 3).  False on a breakdown
// (singular system, complex or non-positive extrema, no convergence).
bool remez5(double lo, double hi, Fit* f) {
  *f = Fit();
  if (lo / hi >= 1.0 - std::cbrt(kEps)) {
    // the Newton-Schulz quintic; by the time a schedule gets here hi is 1 to
    // within ~1e-9 and the printed table holds the unscaled coefficients
    f->p = {15.0 / 8.0, -10.0 / 8.0, 3.0 / 8.0};
    f->ns5 = true;
    return true;
  }
  // first trial set: the quarter points of Algorithm 3
  double t[4] = {lo, 0.75 * lo + 0.25 * hi, 0.25 * lo + 0.75 * hi, hi};
  double last = INFINITY;
  for (int k = 1; k <= 100; ++k) {
    double z[4];
    if (!levelled_solve(t, z)) return false;
    f->p = {z[0], z[1], z[2]};
    f->E = z[3];
    f->exchanges = k;
    // interior extrema: 5c y^2 + 3b y + a = 0 with y = x^2
    const double A = 5.0 * z[2], B = 3.0 * z[1], C = z[0];
    const double disc = B * B - 4.0 * A * C;
    if (!(disc >= 0.0) || A == 0.0) return false;
    const double r = std::sqrt(disc);
    const double y_lo = (-B - r) / (2.0 * A), y_hi = (-B + r) / (2.0 * A);
    if (!(y_lo > 0.0) || !(y_hi > 0.0)) return false;
    t[1] = std::sqrt(std::fmin(y_lo, y_hi));
    t[2] = std::sqrt(std::fmax(y_lo, y_hi));
    // |E| settles at the rounding level of the solve (a few ulps); stop once
    // it moves by at most 16 eps
    if (std::fabs(std::fabs(f->E) - std::fabs(last)) <= 16.0 * kEps) return true;
    last = f->E;
  }
  return false;
}

// Cushion factor r of the ratio-1/10 rule: the minimax quintic on [r, 1] has
// |E| = (1 - 1/10) / (1 + 1/10) = 9/11.  |E| falls as r grows, so bisection on
// a bracket converges to the spacing of doubles.
double ratio_tenth_cushion() {
  const double target = 9.0 / 11.0;
  double below = 1e-6, above = 0.5;  // |E(below)| > target > |E(above)|
  Fit f;
  for (;;) {
    const double mid = 0.5 * (below + above);
    if (!(mid > below && mid < above)) break;
    if (!remez5(mid, 1.0, &f)) break;
    if (std::fabs(f.E) > target) below = mid;
    else above = mid;
  }
  return 0.5 * (below + above);
}

double default_cushion() {
  static const double r = ratio_tenth_cushion();
  return r;
}

}  // namespace

extern "C" void pe_coeff_opts_default(pe_coeff_opts* opts) {
  if (!opts) return;
  opts->cushion = default_cushion();
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
  // cushion < 0: Algorithm 1's rule as printed, [max(l_t, u_t / 10), u_t],
  // without the rescaling
  const bool alg1_rule = o.cushion < 0.0;
  bool newton_schulz[64];
  double l = ell, u = 1.0;
  if (bounds) {
    bounds[0] = l;
    bounds[1] = u;
  }
  for (int t = 0; t < T; ++t) {
    const double design_lo = alg1_rule ? std::fmax(l, 0.1 * u) : std::fmax(l, o.cushion * u);
    Fit f;
    if (!remez5(design_lo, u, &f)) return PE_ENOCONV;
    Odd5 p = f.p;
    if (!f.ns5 && !alg1_rule) {
      const double k = 2.0 / (p.at(l) + p.at(u));
      p.a *= k;
      p.b *= k;
      p.c *= k;
    }
    newton_schulz[t] = f.ns5;
    if (iters) iters[t] = f.exchanges;
    abc[3 * t + 0] = p.a;
    abc[3 * t + 1] = p.b;
    abc[3 * t + 2] = p.c;
    l = p.at(l);
    u = 2.0 - l;
    if (bounds) {
      bounds[2 * (t + 1) + 0] = l;
      bounds[2 * (t + 1) + 1] = u;
    }
  }
  if (err_bound) *err_bound = 1.0 - l;
  if (o.safety != 1.0) {
    const double s = o.safety, s3 = s * s * s, s5 = s3 * s * s;
    for (int t = 0; t < T; ++t) {
      if (newton_schulz[t]) continue;
      if (!o.safety_on_last && t == T - 1) continue;
      abc[3 * t + 0] /= s;
      abc[3 * t + 1] /= s3;
      abc[3 * t + 2] /= s5;
    }
  }
  return PE_OK;
}

// Degree-3 schedule: the greedy composition (Theorem 1) of the closed-form
// minimax cubics of eq. (deg3_solution), p(x) = beta p_NS(alpha x) with
// p_NS(x) = (3x - x^3)/2, alpha = sqrt(3 / (u^2 + l u + l^2)) and
// beta = 4 / (2 + l u (l + u) alpha^3); the error equioscillates at l, 1/alpha
// and u with E = beta - 1, so l_{t+1} = 1 - E and u_{t+1} = 1 + E.  The safety
// factor as for degree 5; no cushion.  abc receives (a_t, b_t, 0) triples.
extern "C" pe_status pe_coeffs_cubic(double ell, int32_t T, const pe_coeff_opts* opts, double* abc,
                                     double* bounds, double* err_bound) {
  pe_coeff_opts o;
  pe_coeff_opts_default(&o);
  if (opts) o = *opts;
  if (!abc || !(ell > 0.0) || !(ell < 1.0) || T < 1 || T > 64) return PE_EINVAL;
  if (!(o.safety >= 1.0)) return PE_EINVAL;
  double l = ell, u = 1.0;
  if (bounds) {
    bounds[0] = l;
    bounds[1] = u;
  }
  for (int t = 0; t < T; ++t) {
    const double alpha = std::sqrt(3.0 / (u * u + l * u + l * l));
    const double beta = 4.0 / (2.0 + l * u * (l + u) * alpha * alpha * alpha);
    const double a = 1.5 * beta * alpha, b = -0.5 * beta * alpha * alpha * alpha;
    l = l * (a + b * l * l);
    u = 2.0 - l;
    const bool safe = o.safety != 1.0 && (o.safety_on_last || t < T - 1);
    const double s = safe ? o.safety : 1.0;
    abc[3 * t + 0] = a / s;
    abc[3 * t + 1] = b / (s * s * s);
    abc[3 * t + 2] = 0.0;
    if (bounds) {
      bounds[2 * (t + 1) + 0] = l;
      bounds[2 * (t + 1) + 1] = u;
    }
  }
  if (err_bound) *err_bound = 1.0 - l;
  return PE_OK;
}
