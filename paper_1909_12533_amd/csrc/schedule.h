// Host scalar control of the SP2 / SP2ACC expansion (IEEE double):
// Step 1 schedule (polynomial sequence, scale-and-fold parameters, n_max,
// n_min, gap bounds, thresholds of eq. (tau_trunc)), the parameterless
// stopping test of Algorithm 2, the Step 3 homo/lumo estimates, and the
// occupied-subspace error bound of section "Error control".
#pragma once

#include <cmath>
#include <cstdint>
#include <limits>
#include <vector>

namespace sp2 {

// Constant of the stopping criterion of Algorithm 2.
constexpr double C_STOP = 6.8872;
// n_max: first iteration whose bound images are both within 2^-52 of 0 / 1.
constexpr double DELTA_N = 2.220446049250313080847263336181640625e-16;
// scale-and-fold is used while max(l, q) >= DELTA_ACC
constexpr double DELTA_ACC = 1e-2;

struct Sched {
  bool bounds = true;  // false: trace-correcting run (p from traces)
  double w = 1.0;
  int n_max = 0, n_min = 1;
  std::vector<int> p;         // p[0] unused (-1)
  std::vector<double> alpha;  // alpha[0] unused (1)
  std::vector<double> l, q, xi, tau;
};

// Bounds on the spectrum images of X_i: unoccupied in [0, l_i], occupied in
// [1 - q_i, 1].  The polynomial attacks the larger bound (p = 1 when
// l > q; a tie gives p = 0); scale-and-fold picks alpha so that both ends of
// the folded interval have the same image: 2 / (2 - l) for p = 1 and
// 2 / (2 - q) for p = 0.
inline Sched make_schedule(double lmin, double lmax, double homo_ub, double lumo_lb, bool accel, double gamma,
                           double tau_fixed, int cap) {
  Sched s;
  s.bounds = true;
  s.w = lmax - lmin;
  double l = (lmax - lumo_lb) / s.w;
  double q = (homo_ub - lmin) / s.w;
  s.p.push_back(-1);
  s.alpha.push_back(1.0);
  s.l.push_back(l);
  s.q.push_back(q);
  int n_max = cap;
  for (int i = 1; i <= cap; ++i) {
    const int p = (l > q) ? 1 : 0;
    double a = 1.0;
    if (accel && std::fmax(l, q) >= DELTA_ACC) a = (p == 1) ? 2.0 / (2.0 - l) : 2.0 / (2.0 - q);
    double ln, qn;
    if (p == 1) {
      const double e0 = (1.0 - a) * (1.0 - a);
      const double e1 = (1.0 - a + a * l) * (1.0 - a + a * l);
      ln = std::fmax(e0, e1);
      qn = a * q * (2.0 - a * q);
    } else {
      ln = a * l * (2.0 - a * l);
      const double e0 = (1.0 - a + a * q) * (1.0 - a + a * q);
      const double e1 = (1.0 - a) * (1.0 - a);
      qn = std::fmax(e0, e1);
    }
    l = ln;
    q = qn;
    s.p.push_back(p);
    s.alpha.push_back(a);
    s.l.push_back(l);
    s.q.push_back(q);
    if (std::fmax(l, q) <= DELTA_N) {
      n_max = i;
      break;
    }
  }
  s.n_max = n_max;
  s.n_min = n_max + 1;
  for (int i = 1; i <= n_max; ++i)
    if (s.alpha[i] == 1.0) {
      s.n_min = i;
      break;
    }
  s.xi.resize(n_max + 1);
  s.tau.resize(n_max + 1);
  const double g = gamma / (double)(n_max + 1);
  for (int i = 0; i <= n_max; ++i) {
    s.xi[i] = 1.0 - s.q[i] - s.l[i];
    if (tau_fixed > 0.0)
      s.tau[i] = tau_fixed;
    else if (gamma > 0.0)
      s.tau[i] = g * s.xi[i] / (1.0 + g);
    else
      s.tau[i] = 0.0;
  }
  return s;
}

inline Sched make_tc2(double lmin, double lmax, double tau_fixed, int cap) {
  Sched s;
  s.bounds = false;
  s.w = lmax - lmin;
  s.n_max = cap;
  s.n_min = 1;
  s.p.assign(1, -1);
  s.alpha.assign(cap + 1, 1.0);
  s.tau.assign(cap + 1, tau_fixed);
  return s;
}

// coefficients of f_i(X) = a I + b X + c X^2
inline void poly_coeffs(int p, double alpha, double &a, double &b, double &c) {
  if (p == 1) {  // ((1 - alpha) I + alpha X)^2
    a = (1.0 - alpha) * (1.0 - alpha);
    b = 2.0 * alpha * (1.0 - alpha);
    c = alpha * alpha;
  } else {  // 2 alpha X - (alpha X)^2
    a = 0.0;
    b = 2.0 * alpha;
    c = -alpha * alpha;
  }
}

// Rounding noise of e_i = ||X~ - X~^2||_F when the square S = X~^2 is formed
// in low precision: the Frobenius norm of S's rounding error, which behaves
// as kappa sqrt(tr X~) (rounding errors of the ~tr X~ significant rows add up
// at random).  kappa is twice the largest ratio |e_low - e_FP64| / sqrt(tr X~)
// measured at the FP32 / BF16x3 noise floor of the lattice expansions
// (N = 2,048 .. 108,000: FP32 0.7-2.3e-6, BF16x3 4.2-8.1e-6); FP64 squares
// have none at this scale (0).
inline double e_noise(int low_kind, double trX) {
  const double kappa = low_kind == 1 ? 4e-6 : (low_kind == 2 ? 1.6e-5 : 0.0);
  return kappa * std::sqrt(std::fmax(trX, 1.0));
}

// Noise of e_i for an FP64 square of an FP32-stored iterate (the FP32-stored
// FP64 tail): e_i is exact for the stored X~, which differs from the iterate
// of the recursion by its FP32 rounding E, ||E||_F <= 2^-24 ||X~||_F, and
// |e(X~ + E) - e(X~)| <= ||E|| (1 + 2 ||X~||_2 + ||E||) ~ 3 ||E||_F; near a
// projector ||X~||_F^2 ~ tr X~.
inline double e_noise_fp32_storage(double trX) {
  return 3.0 * 5.9604644775390625e-08 * std::sqrt(std::fmax(trX, 1.0));
}

// Step 3 estimates.  e[i], tr[i] of X~_i; p, alpha of the run; sched holds
// the forward bounds in bounds mode.  Returns {homo_ub, lumo_lb} (NaN if none).
// noise[i] (optional): rounding noise of a low-precision e_i (0 for FP64).
inline void homo_lumo(const Sched &s, const std::vector<double> &e, const std::vector<double> &tr,
                      const std::vector<int> &p, const std::vector<double> &alpha, int n, double lmin, double lmax,
                      int64_t N, int64_t n_occ, double &homo, double &lumo, const std::vector<double> *noise = nullptr) {
  // An FP64 e_i below 1e3 * 2^-52 * sqrt(N) is rounding noise rather than an
  // eigenvalue's distance from {0, 1}.  A low-precision e_i is used when it is
  // at least ten times its noise nu_i, and as e_i + nu_i (an upper estimate of
  // the e of the exactly squared iterate).
  const double w = lmax - lmin;
  double bh = std::numeric_limits<double>::infinity();
  double bl = -std::numeric_limits<double>::infinity();
  for (int i = 0; i <= n; ++i) {
    const double nu = noise ? (*noise)[i] : 0.0;
    double ei = e[i];
    if (nu > 0.0) {
      if (!(ei >= 10.0 * nu)) continue;
      ei += nu;
    } else if (!(ei >= 1e3 * DELTA_N * std::sqrt((double)N))) {
      continue;
    }
    if (!(ei < 0.25)) continue;
    const double u = 2.0 * ei / (1.0 + std::sqrt(1.0 - 4.0 * ei));
    bool ok;
    if (s.bounds)
      ok = s.l[i] < 1.0 - u && s.q[i] < 1.0 - u;
    else
      ok = std::fabs(tr[i] - (double)n_occ) < 0.5 - (double)N * u;
    if (!ok) continue;
    double uu = u, qq = u;
    for (int j = i; j >= 1; --j) {
      const double a = alpha[j];
      if (p[j] == 1) {
        uu = (std::sqrt(uu) + a - 1.0) / a;
        qq = qq / ((1.0 + std::sqrt(1.0 - qq)) * a);
      } else {
        uu = uu / ((1.0 + std::sqrt(1.0 - uu)) * a);
        qq = (a - 1.0 + std::sqrt(qq)) / a;
      }
    }
    bh = std::fmin(bh, lmin + qq * w);
    bl = std::fmax(bl, lmax - uu * w);
  }
  homo = std::isfinite(bh) ? bh : std::numeric_limits<double>::quiet_NaN();
  lumo = std::isfinite(bl) ? bl : std::numeric_limits<double>::quiet_NaN();
}

}  // namespace sp2
