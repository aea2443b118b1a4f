// SP2 step controller: choice of sigma_n and the stopping test (Sec. II).
//
// One definition, compiled for the device (every workgroup of a step kernel
// evaluates it on the same FP64 inputs, in the same order, so all agree) and
// for the host (exported as dmpt_sp2_decide for unit tests).
//
// sigma_n: the sign whose update puts Tr X_{n+1} closest to N_occ.  Because
//   Tr X^2 = ||X||_F^2 for symmetric X, the two candidates are ||X||_F^2
//   (sigma = +1, X <- X^2) and 2 Tr X - ||X||_F^2 (sigma = -1, X <- 2X - X^2).
//   Ties choose X^2.
// stop: with the idempotency error eps_n = ||X_n - X_n^2||_F^2 (the sum of
//   (x - x^2)^2 over the spectrum of X_n, >= 0), stop at X_n once at least
//   min_iter steps were taken and either eps_n <= idem_tol, or
//   eps_n >= eps_{n-2} while eps_n < 1/64 (every state is resolved,
//   |x - x^2| < 1/8, and two more steps did not reduce the error) and the
//   rise is at the rounding floor: eps_n <= 128 n u^2, u the unit roundoff
//   of the product X_n^2 (2^-24 for FP32 and the FP32-accurate splits, 2^-16
//   for two BF16 terms, 2^-8 for one): each eigenvalue carries noise of
//   order u, so eps cannot fall much below n u^2; or the previous test rose
//   too, eps_{n-1} >= eps_{n-3}.  One rise far above the floor is not enough:
//   once rounding has put eigenvalues on both sides of 0 (or of 1), the
//   trace no longer shows which side dominates eps, and a sigma that doubles
//   the larger side's deviations raises eps before the floor is reached;
//   the next steps bring it down again.  Without a gap at N_occ a state
//   stays near x = 1/2 and only the step limit ends the recursion.
// bounds: a spectrum inside [0, 1] keeps 0 <= ||X||_F^2 <= n and
//   0 <= Tr X <= n; leaving that envelope (or non-finite traces) means the
//   spectral bounds did not enclose H and the recursion diverges.
#pragma once

#include <math.h>

#if defined(__HIPCC__) || defined(__HIP__)
#define DMPT_HD __host__ __device__
#else
#define DMPT_HD
#endif

namespace dmpt {

enum DecideCode : int {
  kDecideStop = 0,
  kDecideNotConverged = -2,
  kDecideBounds = -3,
  kDecideNonfinite = -4,   // set by the device when an input held NaN/Inf
};

constexpr double kUnresolved = 1.0 / 64.0;
constexpr double kFloorFactor = 128.0;

// Unit roundoff of X_n^2 for a product precision (the values of
// dmpt_precision): two BF16 terms keep 16 bits, one keeps 8, the others 24.
DMPT_HD inline double sp2_unit(int prec) {
  return prec == 1 ? 1.52587890625e-05 : prec == 3 ? 3.90625e-03 : 5.9604644775390625e-08;
}

DMPT_HD inline bool sp2_bounds_ok(double tr, double sq, int n) {
  if (!(isfinite(tr) && isfinite(sq))) return false;
  return !(sq > n + 1.0 || tr < -1.0 || tr > n + 1.0);
}

// Stopping test for X_n: steps = n - 1, eps = eps_n, eps_prevK = eps_{n-K}
// (eps_prev3 is read only when steps >= 3).
DMPT_HD inline bool sp2_should_stop(double eps, double eps_prev1, double eps_prev2, double eps_prev3,
                                    int steps, int n, int min_iter, double idem_tol, double unit) {
  if (steps < min_iter) return false;
  if (eps <= idem_tol) return true;
  if (!(steps >= 2 && eps >= eps_prev2 && eps < kUnresolved)) return false;
  if (eps <= kFloorFactor * n * unit * unit) return true;
  return steps >= 3 && eps_prev1 >= eps_prev3;
}

DMPT_HD inline int sp2_sigma(double tr, double sq, double nocc) {
  const double t_square = sq;
  const double t_other = 2.0 * tr - sq;
  return fabs(t_square - nocc) <= fabs(t_other - nocc) ? 1 : -1;
}

// Decision for iterate X_n given its traces and idempotency errors (the
// oracle's order: bounds, stop, sigma).
DMPT_HD inline int sp2_decide(double tr, double sq, double eps, double eps_prev1, double eps_prev2,
                              double eps_prev3, int steps, int n, double nocc, int min_iter, double idem_tol,
                              int prec) {
  if (!sp2_bounds_ok(tr, sq, n)) return kDecideBounds;
  if (sp2_should_stop(eps, eps_prev1, eps_prev2, eps_prev3, steps, n, min_iter, idem_tol, sp2_unit(prec)))
    return kDecideStop;
  return sp2_sigma(tr, sq, nocc);
}

}  // namespace dmpt
