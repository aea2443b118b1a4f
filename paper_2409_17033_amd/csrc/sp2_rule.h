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
// stop: with e_n = Tr X_n - ||X_n||_F^2 (the sum of x(1-x) over the spectrum
//   of X_n), stop at X_n once at least min_iter steps were taken and either
//   |e_n| <= idem_tol or |e_n| >= |e_{n-2}|: two more steps did not reduce the
//   idempotency error, so the rounding floor of the arithmetic is reached.
// unresolved: |e_n| > 1/4 at the stop means a state is stuck near x = 1/2,
//   i.e. no gap separates the N_occ lowest states (not converged).
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

DMPT_HD inline int sp2_decide(double tr, double sq, double e_prev2, int steps, int n,
                              double nocc, int min_iter, double idem_tol) {
  if (!(isfinite(tr) && isfinite(sq))) return kDecideBounds;
  if (sq > n + 1.0 || tr < -1.0 || tr > n + 1.0) return kDecideBounds;
  const double e = tr - sq;
  if (steps >= min_iter) {
    const double ae = fabs(e);
    if (ae <= idem_tol || (steps >= 2 && ae >= fabs(e_prev2)))
      return ae > 0.25 ? kDecideNotConverged : kDecideStop;
  }
  const double t_square = sq;
  const double t_other = 2.0 * tr - sq;
  return fabs(t_square - nocc) <= fabs(t_other - nocc) ? 1 : -1;
}

}  // namespace dmpt
