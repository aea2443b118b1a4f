/*
 * dmpt.h - C ABI of the MI355X (gfx950) implementation of recursive density
 * matrix perturbation theory in its susceptibility ("dual") form,
 * arXiv 2409.17033 (Niklasson, Habib, Finkelstein, Rubensson).
 *
 * The problem the calls solve, as the paper states it:
 *   given a real symmetric Hamiltonian H (N x N) and N_occ, produce the
 *   zero-temperature density matrix D = theta(mu I - H), Tr D = N_occ
 *   (Sec. II, Eq. DM0); given an observable A = A^T, produce its static
 *   susceptibility chi^A_ij = s * dTr[A D]/dH_ij (Eq. Suscept, computed by the
 *   merged forward sweep Eq. DMSuscept or the backward sweep Eq. DM2); then the
 *   linear response for any number of perturbations H1 is
 *   delta<A> = Tr[chi^A H1] (Eq. dual).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Matrices are DEVICE pointers to row-major FP32 with leading dimension n,
 *    full symmetric storage.  Only the symmetric part of H and A is used
 *    (entry (i,j) and (j,i) are averaged).  Batches (A, chi, H1) are
 *    contiguous stacks of n x n matrices.
 *  - The caller owns all memory, including the device workspace sized by the
 *    matching *_workspace_bytes call.  The library never allocates or frees
 *    device memory and keeps no state between calls; concurrent calls must use
 *    distinct workspaces.
 *  - Work is enqueued on opts->stream (a hipStream_t; NULL = the null stream).
 *    Every call returns after synchronising that stream, because it fills
 *    host-side results (dmpt_info, a0, out).
 *  - Errors are returned as a dmpt_status; nothing is thrown across the ABI.
 *    dmpt_last_error() gives a message for the calling thread.  Arguments are
 *    validated before any HIP call, so DMPT_ERR_ARG never touches the device.
 *  - The spin factor s multiplies chi and a0 (s = 2 for a closed-shell
 *    system, s = 1 for the paper's spin-less chi).  With A := H1 and s = 1 the
 *    susceptibility call returns D^(1) of Eq. DM1/DMPert, because the
 *    recursions are identical (Eq. Equivalence).
 */
#ifndef DMPT_H
#define DMPT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DMPT_ABI_VERSION 8
#define DMPT_MAX_STEPS 255

typedef enum dmpt_status {
  DMPT_OK = 0,
  DMPT_ERR_ARG = 1,            /* invalid argument (null pointer, size, enum) */
  DMPT_ERR_NONFINITE = 2,      /* NaN/Inf in an input matrix */
  DMPT_ERR_NOT_CONVERGED = 3,  /* max_iter reached, or a state stuck at mid-gap (no gap at N_occ) */
  DMPT_ERR_BOUNDS = 4,         /* [emin, emax] did not enclose the spectrum: the recursion left [0,1] */
  DMPT_ERR_DEVICE = 5,         /* a HIP runtime call failed */
  DMPT_ERR_WORKSPACE = 6,      /* workspace missing or smaller than required */
  DMPT_ERR_UNSUPPORTED = 7     /* valid request this library does not implement */
} dmpt_status;

/* Arithmetic of the dense products on the matrix cores (Sec. VI.B).
 * The FP32 master copies of X_n and Y_n, the epilogue updates and all traces
 * are FP32/FP64 in every mode. */
typedef enum dmpt_precision {
  DMPT_FP32 = 0,        /* FP32 operands, FP32 MFMA */
  DMPT_SPLIT_BF16 = 1,  /* Eq. doubleHalf with BF16: x = hi + lo, products hi*hi + hi*lo + lo*hi
                           (lo*lo dropped, Eq. MixPrecMult), FP32 accumulate */
  DMPT_SPLIT3_BF16 = 2, /* three BF16 terms hi+mid+lo (FP32-equivalent operands); the six
                           products of order >= 2^-16 (hh, hm, mh, hl, lh, mm) are kept */
  DMPT_BF16 = 3,        /* one BF16 term (plain BF16 operands), FP32 accumulate */
  DMPT_SPLIT3X_BF16 = 4,/* three BF16 terms stored; the SP2 products X_n^2 keep the six split-3
                           products, the sweep products Y_n X_n + X_n Y_n the two-term ones
                           (hh + hm + mh; mid is the two-term lo).  The SP2 products set the
                           accuracy of D and, through it, of chi; the sweep products tolerate
                           the two-term split. */
  DMPT_SPLIT_FP16 = 5   /* Eq. doubleHalf with FP16 terms (the paper's own double-half split) on
                           power-of-two scaled operands: x 2^s = hi + lo, hi = RNE_fp16(x 2^s),
                           lo = RNE_fp16(x 2^s - hi); products hi*hi + hi*lo + lo*hi, FP32
                           accumulate, result times 2^-(s_a + s_b).  X_n is scaled by 2^14
                           (its entries lie in [-1, 1]); Y_n by the power of two that keeps
                           4.5 ||Y_{n-1}||_F below 2^15, a bound on every entry of Y_n.
                           Eleven-bit terms make the two-term split as accurate as FP32 at
                           the cost of DMPT_SPLIT_BF16. */
} dmpt_precision;

typedef enum dmpt_bounds_mode {
  DMPT_BOUNDS_LANCZOS = 0,     /* Lanczos extreme Ritz values widened by max(residual, 1% of width) */
  DMPT_BOUNDS_GERSHGORIN = 1,  /* Gershgorin discs: always encloses the spectrum */
  DMPT_BOUNDS_GIVEN = 2        /* opts.emin / opts.emax as supplied */
} dmpt_bounds_mode;

typedef enum dmpt_sweep {
  DMPT_SWEEP_FORWARD = 0,  /* Eq. DMSuscept: X and Y updated together, no X_n storage */
  DMPT_SWEEP_ADJOINT = 1   /* Eq. DM0 storing every X_n, then the backward sweep Eq. DM2 */
} dmpt_sweep;

typedef struct dmpt_opts {
  int32_t n;              /* matrix dimension, 1 <= n <= 65536 */
  int32_t nocc;           /* occupied states, 0 <= nocc <= n */
  int32_t precision;      /* dmpt_precision */
  int32_t bounds;         /* dmpt_bounds_mode */
  double emin, emax;      /* spectral bounds, read iff bounds == DMPT_BOUNDS_GIVEN */
  int32_t lanczos_steps;  /* Lanczos iterations for DMPT_BOUNDS_LANCZOS; 0 -> 32 */
  int32_t max_iter;       /* SP2 step limit, <= DMPT_MAX_STEPS; 0 -> 100 */
  int32_t min_iter;       /* steps before the stopping test may fire; < 0 -> 10 */
  int32_t sweep;          /* dmpt_sweep (susceptibility only) */
  double idem_tol;        /* also stop when ||X_n - X_n^2||_F^2 <= idem_tol; 0 -> parameter-free test only */
  int32_t project;        /* susceptibility only: 1 -> finish with the occupied-virtual projection
                             (two sweep steps with X frozen at D: sigma = +1 then -1, in the
                             precision of the recursion; FP32 when it is plain BF16).  When the
                             launch after the last step took sigma = +1 (forward sweep, one
                             precision for all products), its Y is the first of the two and
                             is used as it is.  2 -> DMPT_SPLIT3X_BF16 with refine only: Y is
                             projected in the three-term split (a three-term copy of Y and D's
                             three-term copy, regular tiles) and the correction's delta in the
                             two-term split with D's two-term copy, instead of the two-term and
                             plain-BF16 projections.  What the cheaper projections leave in the
                             occupied-occupied / virtual-virtual blocks (about 2^-16 and 2^-8 of
                             Y and delta) is small in norm but can add up in traces against
                             smooth weights (a dipole Tr[A D1] with A the position); about 6 %
                             more time at n = 8192. */
  int32_t profile;        /* 1 -> time every step-kernel launch with events (dmpt_info.*_ms) */
  int32_t ckpt_interval;  /* ADJOINT sweep only: keep X_n every ckpt_interval steps and recompute
                             the steps in between during the backward sweep; 0 -> keep every X_n */
  int32_t refine;         /* susceptibility, forward sweep with projection only: 1 -> one residual
                             correction of chi after the projection (Appendix, proof of Eq.
                             Equivalence: the exact chi' satisfies [H, chi'] = [D, A] and has no
                             occupied-occupied / virtual-virtual blocks).  With Y the projected
                             sweep result: R = [D, A] - [H, Y] from FP32-accurate products
                             (three-term BF16 split; FP16 split for DMPT_SPLIT_FP16; FP32 for
                             DMPT_FP32), B = [D, R], delta = the forward sweep of B (Eq.
                             DMSuscept with A := B) in plain BF16 products over the recorded
                             sigma sequence, projected with D, and chi' = Y + delta.  On the
                             eigenbasis delta_ij = R_ij / (lambda_i - lambda_j) on the
                             occupied-virtual pairs, the error left in Y there; the sweep only
                             has to be accurate relative to that small correction.  With
                             DMPT_SPLIT3X_BF16 the sweep products of the steps, of the projection
                             and of the correction then run on 256 x 256 output tiles with one
                             FP32 accumulation level (the correction removes what that adds),
                             and each launch's last tiles as two half-K jobs added by a combine
                             launch (dmpt_info.split_tiles*).  2 -> the same correction on the
                             regular tiles only.  0 -> off. */
  double sweep_tol;       /* refine only, 0 <= sweep_tol < 1/4: the sweep products stop at the
                             first X_n with ||X_n - X_n^2||_F^2 <= sweep_tol^2 (every eigenvalue
                             of X_n within sweep_tol of 0 or 1; Y_{n+1} is kept, the recursion of
                             X runs on to its stop), and the correction's sweep stops at the first
                             X_n with ||X_n - X_n^2||_F^2 <= sweep_tol.  Stopped there, the sweep
                             result differs from the converged one by O(sweep_tol) relative on the
                             occupied-virtual pairs only (the projection removes the rest), which
                             is the error the residual correction removes to first order; the
                             correction itself only needs accuracy relative to its small size.
                             0 -> the sweeps run to the end. */
  double spin;            /* s; 0 -> 2 */
  void* stream;           /* hipStream_t */
  void* workspace;        /* device memory owned by the caller */
  size_t workspace_bytes;
} dmpt_opts;

typedef struct dmpt_info {
  int32_t m;                            /* SP2 steps taken (M) */
  int32_t status;                       /* dmpt_status of the call */
  double emin, emax;                    /* bounds used */
  double beta;                          /* -1/(emax - emin), Eq. DM0 */
  double trace_d;                       /* Tr D (FP64) */
  double idem_err;                      /* ||D - D^2||_F^2 (FP64 sum of the step kernel's FP32 values) */
  double elapsed_ms;                    /* device time of the call (events on opts.stream) */
  int8_t sigma[DMPT_MAX_STEPS + 1];     /* sigma_n, n = 1..m, and at n = m + 1 the sigma of the launch after the
                                           last step (it runs before the stop is seen; 0 if it did not run) */
  double trace_x[DMPT_MAX_STEPS + 1];   /* Tr X_n, n = 1..m+1 */
  double sqnorm_x[DMPT_MAX_STEPS + 1];  /* ||X_n||_F^2, n = 1..m+1 */
  double idem_x[DMPT_MAX_STEPS + 1];    /* eps_n = ||X_n - X_n^2||_F^2, n = 1..m+1 (0 if not formed) */
  /* Filled when opts.profile = 1 (event pairs on opts.stream around each launch): */
  double bounds_ms;                     /* spectral bounds + X_1/Y_1 initialisation */
  double step_ms;                       /* sum over the m working step-kernel launches */
  double project_ms;                    /* occupied-virtual projection (or adjoint sweep + projection) */
  double output_ms;                     /* D / chi / a0 output kernel */
  int32_t step_launches;                /* step kernels launched (>= m + 1: the last one decides the stop) */
  int32_t tile;                         /* output tile edge of the step kernel */
  double refine_ms;                     /* residual correction (opts.refine), when profiled */
  int32_t sweep_steps;                  /* sweep steps applied to the returned Y (m without sweep_tol) */
  int32_t correction_steps;             /* sweep steps of the residual correction (0 without refine) */
  int32_t split_tiles;                  /* tiles per step launch run as two half-K jobs and combined
                                           (the tail of the 256 x 256-tile lists of refined runs) */
  int32_t split_tiles_sweep;            /* the same for the projection and correction launches */
} dmpt_info;

/* ABI version compiled into the library (DMPT_ABI_VERSION). */
int32_t dmpt_abi_version(void);

/* Fill *opts with defaults for an n x n problem with nocc occupied states:
 * FP32, Lanczos bounds, max_iter 100, min_iter 10, forward sweep, projection on,
 * spin 2, null stream, no workspace. */
void dmpt_opts_default(dmpt_opts* opts, int32_t n, int32_t nocc);

/* Device workspace (bytes) that dmpt_sp2_density (nobs = 0) or
 * dmpt_susceptibility (nobs >= 1 observables) needs for these options.
 * Returns 0 if the options are invalid. */
size_t dmpt_workspace_bytes(const dmpt_opts* opts, int32_t nobs);

/* Eq. DM0 (Sec. II): D = theta(mu I - H) by the SP2 recursion.
 *   H    device, n x n, read only
 *   D    device, n x n, written (FP32)
 *   info host, optional (NULL allowed), filled on return (also on
 *        NOT_CONVERGED / BOUNDS, where D holds the last iterate). */
dmpt_status dmpt_sp2_density(const float* H, float* D, const dmpt_opts* opts, dmpt_info* info);

/* Eq. DMSuscept (forward, default) or Eq. DM2 (opts.sweep = ADJOINT):
 * chi_k = s * dTr[A_k D]/dH for nobs observables sharing one SP2 recursion.
 *   H    device, n x n
 *   A    device, nobs x n x n (symmetric observables)
 *   chi  device, nobs x n x n, written
 *   D    device, n x n, written if not NULL
 *   a0   host, nobs doubles, a0_k = s * Tr[A_k D] (Eq. expectation), written if not NULL
 *   info host, optional.
 * The adjoint sweep stores every X_n in the workspace, or with opts.ckpt_interval = k
 * every k-th one plus k - 1 recomputation slots (the steps between checkpoints
 * are recomputed with the recorded sigma sequence before they are swept). */
dmpt_status dmpt_susceptibility(const float* H, const float* A, int32_t nobs, float* chi,
                                float* D, double* a0, const dmpt_opts* opts, dmpt_info* info);

/* Device workspace (bytes) for dmpt_response. */
size_t dmpt_response_workspace_bytes(int32_t nobs, int32_t npert, int32_t n);

/* Eq. dual: out[k * npert + p] = Tr[chi_k H1_p] = sum_ij chi_k,ij H1_p,ij, accumulated in FP64.
 *   chi  device, nobs x n x n;  H1 device, npert x n x n
 *   out  host, nobs * npert doubles (row-major), written
 *   workspace  device, >= dmpt_response_workspace_bytes(nobs, npert, n)
 * Limits: nobs, npert >= 1, nobs * npert <= 2^20; formed in groups of up to 8 observables
 * x 64 perturbations (one pass over the group's chi and H1 each). */
dmpt_status dmpt_response(const float* chi, int32_t nobs, const float* H1, int32_t npert,
                          int32_t n, double* out, void* stream, void* workspace,
                          size_t workspace_bytes);

/* dmpt_response for callers that cannot allocate device memory (code under
 * stream capture, serving loops, harnesses that forbid hipMalloc): the same
 * kernels and results, with no workspace argument.  The FP64 partial sums
 * and results live in a library-owned device array of 4 MiB on each device
 * (held until the process ends); the call allocates nothing.  Calls that
 * overlap on one device race on that array.  Sizes whose
 * dmpt_response_workspace_bytes exceeds 4 MiB return DMPT_ERR_WORKSPACE
 * before any device work (at n = 8192, 8 observables x 8 perturbations fit,
 * 8 x 64 do not); other argument errors as dmpt_response.
 * Runs on the device current at the call. */
dmpt_status dmpt_response_static(const float* chi, int32_t nobs, const float* H1, int32_t npert,
                                 int32_t n, double* out, void* stream);

/* ---------------------------------------------------------------------------
 * Non-orthonormal basis (Sec. V.A).  With overlap S and an inverse factor Z
 * (Z^T S Z = I: Z = S^{-1/2} for Loewdin orthonormalisation, or the inverse
 * of the Cholesky factor's transpose) the orthonormal problem is
 *   H_perp = Z^T H Z,  A_perp = Z^T A Z,  D_perp = theta(mu I - H_perp),
 * solved as dmpt_susceptibility does (same opts: precision, sweep, bounds,
 * projection), and mapped back: D = Z D_perp Z^T.  Outputs:
 *   chi_perp  s dTr[A_perp D_perp]/dH_perp, the dual of H_perp-perturbations
 *             (Tr[A_perp D_perp_tau] = Tr[chi_perp H_perp_tau]);
 *   chi_ao    Z chi_perp Z^T, the dual of perturbations of H at fixed S
 *             (Tr[chi_perp Z^T dH Z] = Tr[chi_ao dH]);
 *   D         the density matrix in the atomic-orbital basis;
 *   a0        s Tr[A D] = s Tr[A_perp D_perp] (host, nobs values).
 * H (n x n, symmetric), Z (n x n, any inverse factor) and A (nobs x n x n,
 * symmetric) are device FP32 row-major; chi_perp, chi_ao (nobs x n x n), D
 * and a0 may each be NULL.  The congruences run as FP32 MFMA products on
 * zero-padded copies in the workspace (>= dmpt_nonorth_workspace_bytes).
 * Returns the status of the orthonormal solve (NOT_CONVERGED still maps the
 * last iterate back). */
size_t dmpt_nonorth_workspace_bytes(const dmpt_opts* opts, int32_t nobs);
dmpt_status dmpt_susceptibility_nonorth(const float* H, const float* Z, const float* A, int32_t nobs,
                                        float* chi_perp, float* chi_ao, float* D, double* a0,
                                        const dmpt_opts* opts, dmpt_info* info);

/* ---------------------------------------------------------------------------
 * Fractional occupation at finite electronic temperature (Sec. V.B).
 *   D = f(H) = (exp(beta (H - mu I)) + I)^{-1},  beta = 1 / kT,
 *   chi = s d/dlambda f(H + lambda (A + mu_1 I)) at lambda = 0,
 * canonical: mu with Tr D = N_occ and mu_1 with Tr chi = 0 (the electron
 * count does not move); grand canonical: mu given, mu_1 = 0.
 * Recursive Fermi-operator expansion (the doubling scheme of Niklasson,
 * Phys. Rev. B 66, 155115 (2002)), run on E = D - I/2 so that FP32 keeps
 * the relative precision of the high-temperature start:
 *   E_0 = -(beta / 2^{m+2}) (H - mu I),  E_{k+1} = 2 E_k (I + 4 E_k^2)^{-1},
 * D = I/2 + E_m; each inverse by Newton-Schulz iterations (the spectrum of
 * I + 4 E_k^2 lies in [1, 1 + tanh^2(2^{k-1-m} beta w)], w = max |e - mu|
 * over the bounds, which fixes the start and the iteration count).  The
 * response Y = dE/dlambda of each observable runs alongside:
 *   Y_0 = -(beta / 2^{m+2}) A,  Y_{k+1} = (2 Y_k - 4 E_{k+1} (Y_k E_k + E_k Y_k)) R_k,
 * R_k = (I + 4 E_k^2)^{-1}, symmetrised every step.  mu (canonical) by
 * Newton steps on Tr D(mu) = N_occ with dTr D/dmu = beta Tr[D - D^2]
 * = beta (n/4 - ||E_m||_F^2), safeguarded by bisection; then
 * mu_1 = Tr Y_m / (beta Tr[D - D^2]) and chi = s (Y_m - mu_1 beta (D - D^2)).
 * Products: FP32 MFMA (DMPT_FP32) or the FP16 double-half split
 * (DMPT_SPLIT_FP16: tiled FP16 copies of every operand, scaled by 2^15 for E,
 * 2^16 for E^2, 2^14 for R and T (entry bounds 1/2, 1/4, 1, 1), and by
 * 2^15 / ||M||_F for the responses and their intermediates); other
 * precisions return DMPT_ERR_UNSUPPORTED.
 * H (n x n), A (nobs x n x n) device FP32 symmetric; chi (nobs x n x n) and
 * D (n x n, nullable) device; a0 host (nobs, nullable) = s Tr[A D].  opts:
 * n, nocc, bounds (Lanczos / Gershgorin / given, as for dmpt_sp2_density),
 * spin, stream, workspace (>= dmpt_fermi_workspace_bytes). */
typedef struct dmpt_fermi_opts {
  double kt;             /* k_B T_e > 0, in the energy units of H */
  double mu;             /* grand canonical: the chemical potential; canonical: the first
                            Newton guess (NaN: from the bounds and N_occ / n) */
  double count_tol;      /* canonical: |Tr D - N_occ| target (0: 1e-6 n) */
  int32_t canonical;     /* 1 canonical, 0 grand canonical */
  int32_t doublings;     /* m; 0: smallest m with beta w / 2^m <= 2^-8 */
  int32_t newton_max;    /* canonical: Newton / bisection steps (0: 40) */
  int32_t reserved;      /* must be 0 */
} dmpt_fermi_opts;

typedef struct dmpt_fermi_info {
  double mu;             /* chemical potential used */
  double trace_d;        /* Tr D */
  double emin, emax;     /* spectral bounds */
  int32_t doublings;     /* m of the final run */
  int32_t newton;        /* recursions run to find mu (canonical) */
  int32_t products;      /* matrix products of the final run */
  int32_t reserved;
  double mu1[64];        /* mu_1 per observable (first nobs valid) */
  double elapsed_ms;
} dmpt_fermi_info;

size_t dmpt_fermi_workspace_bytes(const dmpt_opts* opts, const dmpt_fermi_opts* fopts, int32_t nobs);
dmpt_status dmpt_susceptibility_fermi(const float* H, const float* A, int32_t nobs, float* chi, float* D,
                                      double* a0, const dmpt_fermi_opts* fopts, const dmpt_opts* opts,
                                      dmpt_fermi_info* finfo);

/* ---------------------------------------------------------------------------
 * Self-consistent susceptibility (Eq. CP_SCF; Sec. V.C and the Appendix) at
 * zero temperature in an orthonormal basis (Z = I, mu_1 = 0), for an on-site
 * self-consistent field: H = H0 + diag(U_i (n_i - n0_i)), n = s diag(D),
 * n0 = s diag(D(H0)), whose linearised field of a density-matrix change X is
 * G(X) = diag(U_i s X_ii) (self-adjoint, as the dual formulation needs).
 * The susceptibility of A solves chi' = L[A + G(chi')] with L the
 * non-interacting response of H0; the result is chi = s chi'.  G reads only
 * the diagonal, so the iteration state is v = diag(chi'):
 *   F(v) = diag(L[A + diag(U s v)]),  r = F(v) - v,
 *   stop when ||r||_2 <= tol ||F(v)||_2.
 * The SP2 recursion of H0 runs once (X_n stored, adjoint sweep); every
 * iteration is one backward sweep (Eq. DM2) of the diagonal observable
 * diag(U s v), plus the occupied-virtual projection.  Mixers:
 *   LINEAR    v <- v + mix r                           (the paper's c_mix)
 *   ANDERSON  Anderson/Pulay extrapolation over the last anderson_depth
 *             iterates with step mix
 *   LEARNED   v <- v + mix r + (||r|| / sqrt(n)) net(sqrt(n) r / ||r||), net
 *             the BF16 site-local network of dmpt_mixer_*; a step whose
 *             residual does not decrease is rejected and replaced by the
 *             linear step (linear mixing is the fallback and the reference).
 * Inputs: H0, A device n x n; U device n floats; chi device n x n (written).
 * opts: as for dmpt_susceptibility (sweep, spin, workspace are taken from it;
 * the sweep is forced to ADJOINT); workspace >= dmpt_scf_workspace_bytes.
 * info (optional) describes the SP2 recursion of H0; sinfo (optional) the
 * self-consistent loop.  NOT_CONVERGED when max_iter is reached (chi then
 * holds the last iterate). */
typedef enum dmpt_mixer {
  DMPT_MIX_LINEAR = 0,
  DMPT_MIX_ANDERSON = 1,
  DMPT_MIX_LEARNED = 2,
  DMPT_MIX_LEARNED_ANDERSON = 3   /* Anderson extrapolation with the network as its preconditioner:
                                     vb = v - sum_j gamma_j dV_j, rb = r - sum_j gamma_j dR_j, then the
                                     LEARNED step from (vb, rb); rejected like LEARNED */
} dmpt_mixer;

#define DMPT_MAX_SCF 1024

typedef struct dmpt_scf_opts {
  int32_t max_iter;           /* F evaluations, 1 .. DMPT_MAX_SCF */
  int32_t mixer;              /* dmpt_mixer */
  double mix;                 /* c_mix, 0 < mix <= 1 */
  double tol;                 /* relative residual target, > 0 */
  int32_t anderson_depth;     /* ANDERSON: 1 .. 16 */
  int32_t mlp_hidden;         /* LEARNED: hidden width of the network */
  int32_t mlp_window;         /* LEARNED: half-width w of the site window */
  int32_t reserved;           /* must be 0 */
  const uint16_t* mlp_params; /* LEARNED: device, BF16 parameters (dmpt_mixer layout) */
  float* record_v;            /* optional, device, max_iter x n: v of every accepted state */
  float* record_r;            /* optional, device, max_iter x n: r = F(v) - v of every accepted state */
} dmpt_scf_opts;

typedef struct dmpt_scf_info {
  int32_t iters;                   /* F evaluations done (the cost: one backward sweep each, but the first) */
  int32_t converged;               /* 1 if the residual target was met */
  int32_t rejected;                /* ANDERSON / LEARNED steps replaced by the linear step */
  int32_t states;                  /* accepted states, v_0 = 0 included (rows of record_v / record_r) */
  double residual[DMPT_MAX_SCF];   /* ||r|| / ||F(v)|| of every accepted state */
} dmpt_scf_info;

size_t dmpt_scf_workspace_bytes(const dmpt_opts* opts, const dmpt_scf_opts* scf);

dmpt_status dmpt_scf_response(const float* H0, const float* U, const float* A, float* chi,
                              const dmpt_scf_opts* scf, const dmpt_opts* opts, dmpt_info* info,
                              dmpt_scf_info* sinfo);

/* ---------------------------------------------------------------------------
 * Learned mixer network (the LEARNED mixer of dmpt_scf_response; not from the
 * paper, which mixes linearly).  It is applied site by site with shared
 * weights: for a state vector x in R^n, site i sees
 *   z_i = [x_{i-w}, ..., x_{i+w}, E_{i-w}, ..., E_{i+w}, U_i]
 *        (k = 4w + 3 features; x_j = E_j = 0 outside 0..n-1; E the on-site
 *         energies, the diagonal of H0)
 * and outputs y_i = w2 . tanh(W1 z_i + b1) + b2 (hidden width h).  The
 * response of a gapped system is near-sighted, so a window of sites carries
 * the information a preconditioner of the self-consistent loop needs; the
 * on-site energies say which of them are polarisable.
 * BF16 parameters in one vector [W1 (h x k, row-major) | b1 (h) | w2 (h) |
 * b2 (1)]; training minimises the mean squared error over all B n outputs,
 * (1 / (B n)) sum (y - t)^2, with Adam (beta1 0.9, beta2 0.999, eps 1e-8) on
 * FP32 master parameters.  Arrays are device arrays; batches are row-major
 * B x n; U is the n on-site interactions, E the n on-site energies.  Training pairs of the
 * self-consistent loop: x = sqrt(n) r / ||r||, t = sqrt(n) (v* - v - mix r) / ||r||
 * from linear-mixing runs (v* their converged state). */
size_t dmpt_mixer_param_count(int32_t window, int32_t hidden);
/* Scratch for batches of up to `batch` states of size n.  Limits: n <= 65536,
 * window <= 512, hidden <= 4096, batch * n <= 2^20 site rows; 0 (with the
 * error message set) when out of range.  Every mixer call with sizes out of
 * range returns DMPT_ERR_ARG; a workspace smaller than this returns
 * DMPT_ERR_WORKSPACE. */
size_t dmpt_mixer_workspace_bytes(int32_t n, int32_t window, int32_t hidden, int32_t batch);
/* Glorot-uniform weights from a counter-based generator (splitmix64 of seed
 * and index), zero biases; writes the FP32 masters and the BF16 copy. */
dmpt_status dmpt_mixer_init(float* master, uint16_t* params, int32_t window, int32_t hidden, uint64_t seed,
                            void* stream);
dmpt_status dmpt_mixer_forward(const uint16_t* params, int32_t window, int32_t hidden, const float* U, const float* E,
                               int32_t n,
                               const float* x, int32_t batch, float* y, void* stream, void* workspace,
                               size_t workspace_bytes);
/* loss (host) and its gradient (device, FP32, parameter layout) for one batch. */
dmpt_status dmpt_mixer_loss_grad(const uint16_t* params, int32_t window, int32_t hidden, const float* U, const float* E,
                                 int32_t n,
                                 const float* x, const float* t, int32_t batch, float* grad, double* loss,
                                 void* stream, void* workspace, size_t workspace_bytes);
/* steps Adam steps (step counter starting at 1) over minibatches of `batch`
 * consecutive states cycling through the npairs pairs; adam_m and adam_v
 * start at zero (caller-owned, parameter-count floats); loss_history (host,
 * optional) receives the loss of every step. */
dmpt_status dmpt_mixer_train(float* master, uint16_t* params, float* adam_m, float* adam_v, int32_t window,
                             int32_t hidden, const float* U, const float* E, int32_t n, const float* x, const float* t,
                             int32_t npairs, int32_t batch, int32_t steps, double lr, double* loss_history,
                             void* stream, void* workspace, size_t workspace_bytes);

/* Training pairs of the learned mixer from one recorded loop (the LEARNED
 * mixer's data; callers: its trainer).  v, r: device, k x n row-major FP32, the
 * recorded states and residuals (dmpt_scf_opts.record_v / record_r);
 * residual: host, k relative residuals (dmpt_scf_info.residual); vstar:
 * device, n FP32, the loop's converged state.  Every row j with
 * residual[j] >= min_residual (and j < k - 1 when drop_last) gives, in order,
 *   x = sqrt(n) r_j / ||r_j||,   t = sqrt(n) (v* - v_j - mix r_j) / ||r_j||
 * (||r_j|| accumulated in FP64) in rows of x_out, t_out (device, capacity x n);
 * *count (host) receives the number of rows written.  workspace: device,
 * >= dmpt_mixer_rows_workspace_bytes(k).  More kept rows than capacity:
 * DMPT_ERR_ARG, nothing written. */
size_t dmpt_mixer_rows_workspace_bytes(int32_t rows);
dmpt_status dmpt_mixer_pairs(const float* v, const float* r, const double* residual, int32_t k, int32_t n,
                             const float* vstar, double mix, double min_residual, int32_t drop_last,
                             float* x_out, float* t_out, int32_t capacity, int32_t* count, void* stream,
                             void* workspace, size_t workspace_bytes);
/* x_out, t_out (device, npairs x n) = the rows of x, t (device, npairs x n)
 * in one random order (Fisher-Yates on splitmix64 draws of seed; the same
 * seed gives the same order); the outputs must not alias the inputs.
 * workspace: device, >= dmpt_mixer_rows_workspace_bytes(npairs). */
dmpt_status dmpt_mixer_shuffle(const float* x, const float* t, int32_t npairs, int32_t n, uint64_t seed,
                               float* x_out, float* t_out, void* stream, void* workspace, size_t workspace_bytes);

/* Host mirror of the device-side step controller (pure function, no device).
 * Decision for iterate X_n (Sec. II) from FP64 Tr X_n, ||X_n||_F^2, its
 * idempotency error eps = ||X_n - X_n^2||_F^2, the earlier errors
 * eps_prevK = eps_{n-K} (K = 1, 2, 3; eps_prev3 is read only when steps >= 3)
 * and the number of steps taken (steps = n - 1), tested in this order:
 *   -3       : bounds violation (X_n left the [0,1] spectrum envelope)
 *    0       : stop, X_n is the result: steps >= min_iter and either
 *              eps <= idem_tol, or eps >= eps_prev2 with eps < 1/64
 *              (needs steps >= 2) and the rise is at the rounding floor:
 *              eps <= 128 n u^2, u the unit roundoff of X_n^2 in the given
 *              dmpt_precision (2^-16 for DMPT_SPLIT_BF16, 2^-8 for DMPT_BF16,
 *              2^-24 otherwise), or the previous test rose too
 *              (eps_prev1 >= eps_prev3, steps >= 3)
 *   +1 / -1  : sigma_n for the next step (Tr X_{n+1} closest to N_occ).
 * The step limit (max_iter, status NOT_CONVERGED) is applied by the caller.
 * The device makes the same decisions, the stopping test one launch later
 * (eps_n is a by-product of the launch that forms X_n^2). */
int32_t dmpt_sp2_decide(double tr, double sq, double eps, double eps_prev1, double eps_prev2, double eps_prev3,
                        int32_t steps, int32_t n, double nocc, int32_t min_iter, double idem_tol,
                        int32_t precision);

const char* dmpt_status_string(dmpt_status status);
const char* dmpt_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DMPT_H */
