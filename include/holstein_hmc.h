/*
 * holstein_hmc.h - C ABI of the MI355X (gfx950) fermion solver for the
 * Holstein-model hybrid Monte Carlo of Cohen-Stead et al.,
 * "Fast and scalable quantum Monte Carlo simulations of electron-phonon
 * models" (arXiv:2203.01291).
 *
 * The library applies the space-time fermion matrix M of Eq. (M_def),
 * solves the normal equations (M^T M) u = Phi of Eqs. (psi_def, CG) with
 * conjugate gradients, optionally preconditioned by the adiabatic
 * preconditioner of Sec. V (Eqs. P_def, CG_precon, P_change_basis, App. C),
 * evaluates the action S_F = Phi . u (Eq. Sf_Psi) and the phonon force
 * dS_F/dx of Eq. (dSF_dx), and runs the hybrid Monte Carlo update of the
 * phonon field built on them (Sec. III, Algorithm 1; fph_hmc_* below) and
 * the stochastic Green's-function measurements (Sec. VI; fph_meas_*).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Lattice: L x L periodic square lattice, L even and >= 4, N = L*L sites,
 *   site index i = x + L*y.  Hopping K_ij = -t between nearest neighbours
 *   (Eq. V_K_def).  Ltau time slices, Ltau even and >= 2, tau = 0..Ltau-1.
 * Field: x[tau][i] (FP64), row-major, site fastest.  E[tau][i] =
 *   exp(-dtau*(alpha*x[tau][i] - mu)) is the diagonal of exp(-dtau V_tau)
 *   (Eqs. B_def, V_K_def).
 * Vectors: v[r][tau][i] for right-hand side r, site fastest; one
 *   right-hand side holds d = N*Ltau elements.  FP64 (double) unless an
 *   entry point says otherwise; FP32 buffers are float with the same layout.
 * Operator: B_tau = diag(E_tau) C with the checkerboard product
 *   C = P_A P_B ~ exp(-dtau K): P_A (P_B) exponentiates exactly the hopping
 *   of the disjoint 2x2 plaquettes whose lower-left corner has even (odd)
 *   x and y, wrapping periodically; P_B acts first (Sec. II D, "minimal
 *   split" checkerboard; O(dtau^2) error).  Each plaquette factor is
 *   kron(C2, C2), C2 = [[cosh(dtau t), sinh(dtau t)], [sinh(dtau t),
 *   cosh(dtau t)]].
 *   (M v)_tau  = v_tau - E_tau * (C v~_{tau-1}),  v~_{-1} = -v_{Ltau-1};
 *   (M^T w)_tau = w_tau - C^T (E_{tau+1} * w~_{tau+1}),
 *                 w~_{Ltau} = -w_0, E_{Ltau} = E_0.
 *
 * Memory and streams
 * ------------------
 * All data pointers named *_dev are device pointers owned by the caller;
 * the library never frees or retains them past the call.  The library owns
 * only the handle and the workspace allocated by fph_create.  Work is
 * enqueued on the caller's hipStream_t (passed as void*; NULL means the
 * null stream).  A handle must not be used from two streams at once.
 * Entry points that return results on the host (pcg_solve_sync and the
 * other *_sync or host-statistics calls, fph_precond_info) synchronise that
 * stream before returning; the hot path (fph_set_field, fermion_matvec,
 * pcg_solve, fermion_action, fermion_force) only enqueues.
 *
 * Errors
 * ------
 * Every entry point returns FPH_OK (0) on success, a negative FPH_E* code
 * for an argument error detected on the host before anything is enqueued,
 * or FPH_E_HIP for a failed HIP call.  fph_strerror() gives a message.
 * Numerical outcomes of a solve are reported in fph_pcg_stats_t.status.
 */
#ifndef HOLSTEIN_HMC_H
#define HOLSTEIN_HMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FPH_OK 0
#define FPH_E_NULL (-1)       /* a required pointer is NULL               */
#define FPH_E_LATTICE (-2)    /* L odd, < 4 or > 64; Ltau odd, < 2 or > 2048;
                                 Ltau/2 not a product H1*H2 with H1 in
                                 {1,2,3,4,5,8,10,16,20}, H2 <= 32; bad param */
#define FPH_E_NRHS (-3)       /* nrhs < 1 or above the handle's max_rhs   */
#define FPH_E_PREC (-4)       /* unsupported precision / operator code    */
#define FPH_E_NOFIELD (-5)    /* fph_set_field has not been called        */
#define FPH_E_ALIGN (-6)      /* device pointer not 16-byte aligned       */
#define FPH_E_ARG (-7)        /* other invalid argument                   */
#define FPH_E_HIP (-100)      /* a HIP runtime call failed                */

/* Status bits of fph_pcg_stats_t.status. */
#define FPH_ST_CONVERGED 1    /* true relative residual below tol         */
#define FPH_ST_MAXITER 2      /* iteration cap reached                    */
#define FPH_ST_BREAKDOWN 4    /* p.Ap <= 0 or r.z <= 0 in CG              */
#define FPH_ST_NONFINITE 8    /* NaN or Inf met in a scalar of the solve  */
#define FPH_ST_ABORTED 16     /* variant 2: a grid-wide wait ran over its
                                 limit and the launch gave up             */

typedef struct fph_handle_s* fph_handle_t;

typedef struct {
  int32_t L;     /* lattice side, even, >= 4                             */
  int32_t Ltau;  /* number of time slices, even, >= 2                    */
  double dtau;   /* imaginary-time step                                  */
  double t;      /* nearest-neighbour hopping                            */
  double mu;     /* chemical potential                                   */
  double alpha;  /* electron-phonon coupling                             */
} fph_lattice_t;

typedef enum { FPH_OP_M = 0, FPH_OP_MT = 1, FPH_OP_MTM = 2 } fph_op_t;

typedef enum { FPH_F64 = 0, FPH_F32 = 1, FPH_F32_REFINED = 2 } fph_prec_t;

/* Preconditioner operators: F ~ P^{-1}, its transpose, and F F^T. */
typedef enum { FPH_PC_F = 0, FPH_PC_FT = 1, FPH_PC_FFT = 2 } fph_pc_op_t;

typedef struct {
  double tol;           /* stop when |b - M^T M u| / |b| < tol            */
  int32_t maxiter;      /* cap on CG iterations (all precisions)           */
  int32_t use_precond;  /* 1: z = F F^T r (Eq. CG_precon); 0: z = r        */
  int32_t prec;         /* fph_prec_t: FP64 CG, or FP32 CG with FP64
                           reliable updates of the residual (FP32_REFINED) */
  int32_t zero_guess;   /* 1: start from u = 0; 0: u_dev holds the guess   */
  double ru_delta;      /* FP32_REFINED: recompute the FP64 residual when
                           the FP32 residual has fallen by this factor
                           since the last recomputation (0 -> 0.1 with the
                           preconditioner, 0.3 without; at most 0.5); the
                           interval is shortened automatically (delta ->
                           sqrt delta) when a recomputation finds the true
                           residual more than twice the FP32 one          */
  int32_t chunk;        /* pcg_solve_sync: solver slots (iterations or
                           residual evaluations) enqueued between two
                           progress probes (0 -> 16, or 8 when
                           N Ltau > 2^20); variant 2: the
                           largest number of workgroups (0 -> 128)         */
  int32_t variant;      /* 0: the standard (P)CG of pcg_solve (two
                           launches per iteration without preconditioner,
                           four with it); 2: the whole FP32_REFINED solve
                           in one cooperative launch (nrhs == 1, no
                           preconditioner; all workgroups resident,
                           grid-wide exchanges of partial sums instead of
                           kernel boundaries)                              */
  int32_t max_outer;    /* cap on the FP64 residual evaluations after the
                           first one (0 -> 32); a right-hand side that
                           reaches it stops with FPH_ST_MAXITER            */
  int32_t pad;
  double cheb_a1;       /* fph_batch_solve with use_precond: Chebyshev
                           order constants of every system's tables,
                           N_P = floor(db (a1/phi + a2)) (Eq. NP_heuristic;
                           0 -> 1).  pcg_solve takes them from
                           fph_set_field instead.                          */
  double cheb_a2;
} fph_pcg_opts_t;

typedef struct {
  int32_t status;       /* FPH_ST_* bits                                   */
  int32_t iters;        /* CG iterations performed                         */
  int32_t outer_iters;  /* FP64 residual recomputations                    */
  int32_t matvecs;      /* applications of M^T M, all precisions           */
  double rel_resid;     /* final |b - M^T M u| / |b|, evaluated in FP64    */
  double action;        /* S_F = b . u in FP64 (Eq. Sf_Psi)                */
} fph_pcg_stats_t;

/* Library version string. */
const char* fph_version(void);

/* Message for a return code. */
const char* fph_strerror(int code);

/* Create a handle for one lattice and up to max_rhs right-hand sides;
 * allocates all device workspace once (Sec. II C defines the parameters).
 * Returns FPH_E_LATTICE for an unsupported lattice, FPH_E_NRHS for
 * max_rhs < 1.  On error *h is set to NULL. */
int fph_create(fph_handle_t* h, const fph_lattice_t* lat, int32_t max_rhs);

/* Release the handle and its workspace (synchronises the device). */
int fph_destroy(fph_handle_t h);

/* Copy the handle's lattice to *lat and its right-hand-side capacity to
 * *max_rhs (either may be NULL).  Host only. */
int fph_get_lattice(fph_handle_t h, fph_lattice_t* lat, int32_t* max_rhs);

/* Per-field setup from x_dev[Ltau][N] (FP64, device): E = exp(-dtau V)
 * in FP64 and FP32 (Eq. B_def), dbar_i = mean_tau E[tau][i] (Eq. expnVbar),
 * spectral bounds of Bbar = diag(dbar) C enclosing its real eigenvalues,
 * bmin = min(dbar) e^{-4 dtau |t|}, bmax = max(dbar) e^{4 dtau |t|}, and the
 * Chebyshev tables of App. C: N_P(w) = max(1, floor(db (a1/phi_w + a2)))
 * (Eq. NP_heuristic) and c_m(w) by Chebyshev-Gauss quadrature with
 * 2 N_P points (Eq. Cheby-Gauss).  a1, a2 <= 0 select 1.  Enqueue only. */
int fph_set_field(fph_handle_t h, const double* x_dev, double a1, double a2,
                  void* stream);

/* Per-right-hand-side fields, for independent systems of one lattice solved
 * in the same launches (several Markov chains, say): x_dev holds nfields
 * fields [nfields][Ltau][N] (FP64, device), and right-hand side r of the
 * following calls uses field r / rhs_per_field (so at most
 * nfields * rhs_per_field right-hand sides; FPH_E_NRHS otherwise).  Each
 * field gets its own E, dbar, spectral bounds and Chebyshev tables as in
 * fph_set_field, which switches back to one shared field.  fermion_force
 * then writes one gradient per field: grad_dev[f] accumulates the
 * right-hand sides of field f.  Not with pcg_solve variant 2.  nfields is
 * 1..max_rhs.  Enqueue only. */
int fph_set_fields(fph_handle_t h, int32_t nfields, int32_t rhs_per_field, const double* x_dev,
                   double a1, double a2, void* stream);

/* out = op(in) for nrhs right-hand sides sharing the current field
 * (Eq. M_def): op is FPH_OP_M, FPH_OP_MT or FPH_OP_MTM (fused M^T M; the
 * intermediate M v never leaves the chip).  prec FPH_F64: in/out are
 * double; FPH_F32: float (E rounded to nearest FP32).  in and out must not
 * overlap.  Enqueue only. */
int fermion_matvec(fph_handle_t h, int32_t op, int32_t prec, int32_t nrhs,
                   const void* in_dev, void* out_dev, void* stream);

/* Solve (M^T M) u = b for nrhs right-hand sides with (preconditioned)
 * conjugate gradients (Eqs. CG, CG_precon; stopping on the relative
 * residual, Sec. V B).  b_dev, u_dev: double [nrhs][Ltau][N]; u_dev is the
 * initial guess unless opts->zero_guess and receives the solution.
 * stats_dev: device array of nrhs fph_pcg_stats_t, written when the solve
 * ends in stream order (S_F = b . u included).
 *
 * Enqueue only: the call never synchronises and reads nothing back.  Every
 * decision (convergence, FP64 residual evaluation and replacement of the
 * FP32-refined residual, the iteration cap, breakdown) is taken on the
 * device.  The call enqueues a fixed sequence: a start kernel, then
 * 1 + maxiter + max_outer "slots" (each performs one CG iteration or one
 * FP64 residual evaluation per right-hand side; slots after a right-hand
 * side finished return at once, about 1.5 us per launch), then two final
 * kernels; set maxiter near the expected iteration count, since every slot
 * is enqueued.  Only kernel launches are enqueued (no memset or copy), so
 * the sequence can be captured into a hipGraph and replayed.  The host
 * thread may wait for space in the stream's queue while enqueueing a long
 * solve.  Calls on one handle must be ordered on one stream (they share
 * its workspace).  Returns FPH_OK even when a right-hand side did not
 * converge: check stats.status once the stream has reached the end. */
int pcg_solve(fph_handle_t h, int32_t nrhs, const double* b_dev, double* u_dev,
              const fph_pcg_opts_t* opts, fph_pcg_stats_t* stats_dev,
              void* stream);

/* The same solve for callers that want the statistics on the host:
 * stats_host (nrhs entries, may be NULL) is filled on return.  Enqueues the
 * slots of pcg_solve in chunks of opts->chunk (0 -> 16, or 8 above 2^20
 * unknowns per right-hand side); after each chunk
 * a one-wave kernel writes how many right-hand sides are still open into
 * pinned host memory, the host waits for the previous chunk's count only
 * (the GPU always has a chunk queued) and stops enqueueing once it is zero.
 * The result is the one pcg_solve gives.  Blocks the calling thread until
 * the solve has finished on `stream`. */
int pcg_solve_sync(fph_handle_t h, int32_t nrhs, const double* b_dev, double* u_dev,
                   const fph_pcg_opts_t* opts, fph_pcg_stats_t* stats_host,
                   void* stream);

/* grad_dev[Ltau][N] += scale * s * sum_r dS_F/dx for the solutions
 * u_dev[nrhs][Ltau][N] of the current field (Eq. dSF_dx with Lambda = I):
 *   dS_F/dx_{i,tau} = -2 dtau alpha (u - y)_{i,tau} y_{i,tau},
 *   y_tau = E_tau * (C u~_{tau-1}),
 * so that (u - y) = M u.  s = *scale_dev, one double in device memory read
 * when the kernel runs (an upstream gradient that stays on the device), or
 * 1 when scale_dev is NULL.  scale must be finite (FPH_E_ARG).  Enqueue
 * only. */
int fermion_force(fph_handle_t h, int32_t nrhs, const double* u_dev,
                  double* grad_dev, double scale, const double* scale_dev, void* stream);

/* out_dev[r] = b_r . u_r in FP64 for r < nrhs (S_F of Eq. Sf_Psi).
 * Enqueue only. */
int fermion_action(fph_handle_t h, int32_t nrhs, const double* b_dev,
                   const double* u_dev, double* out_dev, void* stream);

/* fermion_action for callers that cannot allocate device memory at all
 * (code under hipGraph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same result, bit for bit, with the partial sums of the
 * dot products kept in a static device array of the library (512 KiB per
 * GPU, held until the process ends) instead of the handle's workspace; the
 * call allocates nothing.  nrhs <= 64 (and <= max_rhs), else FPH_E_NRHS;
 * the current device must be the handle's (FPH_E_ARG).  Every call on a GPU
 * shares that GPU's array: calls that overlap on one GPU (on different
 * streams, or from different host threads) race.  Enqueue only. */
int fermion_action_noalloc(fph_handle_t h, int32_t nrhs, const double* b_dev,
                           const double* u_dev, double* out_dev, void* stream);

/* out = op(in) with the preconditioner of the current field: F ~ P^{-1}
 * = U^dagger Ptilde^{-1} U (Eq. P_change_basis) with each block inverse
 * replaced by its truncated Chebyshev series (Eq. f_A_approx), F^T, or
 * F F^T.  prec FPH_F64 (double) or FPH_F32 (float).  Enqueue only. */
int fph_precond_apply(fph_handle_t h, int32_t op, int32_t prec, int32_t nrhs,
                      const void* in_dev, void* out_dev, void* stream);

/* Copy the preconditioner tables of the current field to the host:
 * bounds_host[2] = {bmin, bmax}; np_host[Ltau] = N_P(w) (may be NULL).
 * Synchronises `stream`. */
int fph_precond_info(fph_handle_t h, double* bounds_host, int32_t* np_host,
                     void* stream);

/* ------------------------------------------------------------------ */
/* Batched solves: many independent systems of uneven size.            */

typedef struct {
  fph_lattice_t lat;    /* L even in [4, 32], Ltau as for fph_create      */
  const double* x_dev;  /* phonon field [Ltau][N] (FP64, device)          */
  int32_t nrhs;         /* right-hand sides of this system (>= 1)          */
  const double* b_dev;  /* [nrhs][Ltau][N] right-hand sides                */
  double* u_dev;        /* [nrhs][Ltau][N] receives the solutions          */
} fph_system_t;

typedef struct fph_batch_s* fph_batch_t;

/* Create a batch over nsys systems (the pointers in sys are recorded and
 * read at every fph_batch_solve).  Allocates the fields E of every system
 * and an FP32 workspace of 5 vectors per right-hand side, and sorts the
 * (system, right-hand side) work items by size, largest first.  Errors:
 * FPH_E_NULL, FPH_E_LATTICE (a system outside the supported range),
 * FPH_E_NRHS (a system with nrhs < 1), FPH_E_HIP. */
int fph_batch_create(fph_batch_t* bh, const fph_system_t* sys, int32_t nsys);

/* Solve every right-hand side of every system, (M^T M) u = b as in
 * pcg_solve, in ONE persistent launch (replayed from a captured hipGraph
 * together with the per-system field setup): each workgroup pulls work
 * items from a queue and runs the item's FP32 conjugate gradients with
 * FP64 residual replacement to opts->tol (Sec. II D, Eq. CG; the paper's
 * stochastic measurements solve many such vectors at once, Sec. VI).
 * With opts->use_precond the iteration is preconditioned by F F^T
 * (Eq. CG_precon; Sec. V A, App. C): each system's dbar, bounds, N_P and
 * Chebyshev coefficients (constants opts->cheb_a1, cheb_a2) are set up with
 * the fields, and the item's workgroup applies the two transforms and the
 * series of every frequency block itself; this needs workgroups of at least
 * L^2/4 threads (FPH_E_ARG otherwise; the default shape qualifies).
 * opts->prec must be FPH_F32_REFINED (FPH_E_PREC).  The replacement factor
 * opts->ru_delta defaults to 0.1 with the preconditioner, 0.3 without.
 * stats_dev: device array with one entry per right-hand side in system
 * order (may be NULL), written in stream order.  Enqueue only (the first
 * call, and a call with another tol, maxiter, ru_delta, use_precond or
 * Chebyshev constants than the last, captures the graph on an internal
 * stream first; fph_batch_tune also captures). */
int fph_batch_solve(fph_batch_t bh, const fph_pcg_opts_t* opts, fph_pcg_stats_t* stats_dev,
                    void* stream);

/* Autotune the launch shape of fph_batch_solve (threads per workgroup and
 * workgroups per compute unit) by timing one solve of each candidate;
 * keeps the fastest.  best_host[3] (may be NULL) receives {threads,
 * plaquettes per thread, workgroups per CU}.  Blocks until done. */
int fph_batch_tune(fph_batch_t bh, const fph_pcg_opts_t* opts, int32_t* best_host, void* stream);

/* Release the batch (synchronises the device). */
int fph_batch_destroy(fph_batch_t bh);


/* ------------------------------------------------------------------ */
/* Hybrid Monte Carlo update of the phonon field (Sec. III).           */
/*
 * Two actions (opts.lambda_action):
 *   0: A = M (Eqs. S_prime, Z_path_orig, S_F),
 *      S'(x) = S_B(x) - dtau*alpha*sum_{i,tau} x_{i,tau}
 *              + 1/2 sum_sigma Phi_sigma . (M^T M)^{-1} Phi_sigma;
 *   1: A = M Lambda (Eqs. Z_path, Lambda_def, S_again),
 *      S(x)  = S_B(x) + 1/2 sum_sigma b_sigma . (M^T M)^{-1} b_sigma,
 *      b_sigma = Lambda(x)^{-T} Phi_sigma, where Lambda couples slice tau
 *      to tau+1 of each site:
 *        Lambda[(i,tau),(i,tau+1)] = s(tau+1) exp(dtau alpha x_{i,tau+1}/2),
 *        s(t) = +1 for t = 0, -1 otherwise (slices mod Ltau);
 * in both, Phi_sigma = A(x)^T R_sigma at the start of an update
 * (Eq. PhiSample-1) and
 *   S_B   = dtau/2 sum_{i,tau} [omega0^2 x^2 + ((x_{tau+1} - x_tau)/dtau)^2]
 *           with x_{i,Ltau} = x_{i,0}                          (Eq. S_B).
 * Kinetic energy p^T Mass^{-1} p / 2 with the Fourier-acceleration mass
 *   Mass = F^{-1} Mtilde F over imaginary time (Sec. III B 1),
 *   Mtilde_w = dtau (m_reg^2 + omega0^2 + 4/dtau^2 sin^2(pi w/Ltau))
 *              / (m_reg^2 + omega0^2),
 * the sine argument being pi w/Ltau (the value the stencil of Eq. dSB_dx
 * gives; the paper's Eq. Qww_def prints 2 pi w/Ltau).  m_reg < 0 or +inf
 * selects Mass = dtau I (no Fourier acceleration).
 * Momenta and forces share the field layout [Ltau][N] (FP64).
 */

typedef struct fph_hmc_s* fph_hmc_t;

typedef struct {
  double omega0;               /* phonon frequency (> 0)                       */
  double m_reg;                /* mass regularisation; < 0 or inf: Mass = dtau I */
  double dt;                   /* integration step Delta t (> 0)               */
  int32_t Nt;                  /* steps per trajectory (>= 1; paper: 100)       */
  int32_t nt;                  /* bosonic sub-steps per step (>= 1; paper: 10)  */
  int32_t nfields;             /* pseudofermion fields, 1..max_rhs (paper: 2)   */
  double a1, a2;               /* Chebyshev-order constants for fph_set_field   */
  int32_t guess;               /* initial guess of each force solve: 0 zero;
                                  1 the previous solution; 2 the linear
                                  extrapolation 2 u_t - u_{t-1} of the last two
                                  (the first solve of a trajectory starts from
                                  zero).  1 and 2 save CG iterations, but the
                                  force error they leave depends on the history
                                  and adds up along the trajectory: at loose
                                  force tolerances they bias H_f - H_i and the
                                  update is reversible only to the tolerance  */
  int32_t lambda_action;       /* 0: the action S' (A = M); 1: S (A = M Lambda) */
  int32_t nchains;             /* independent chains advanced together by
                                  hmc_trajectories (0 or 1: one chain); they
                                  share every launch through per-right-hand-side
                                  fields (fph_set_fields), so the solver handle
                                  needs max_rhs >= nchains * nfields           */
  int32_t pad;
  fph_pcg_opts_t force_solve;  /* solves for the force (paper: tol 1e-5)        */
  fph_pcg_opts_t action_solve; /* solve for S_F at the end (paper: tol 1e-10)   */
} fph_hmc_opts_t;

typedef struct {
  double H_i, H_f;      /* H = S' + K before and after the trajectory (FP64)    */
  double SB_i, SB_f;    /* x-only action: S_B - dtau*alpha*sum x (S') or S_B (S) */
  double SF_i, SF_f;    /* 1/2 sum_sigma Phi.u; SF_i = 1/2 sum |R_sigma|^2      */
  double K_i, K_f;      /* p^T Mass^{-1} p / 2                                  */
  double accept_prob;   /* min(1, exp(-(H_f - H_i)))                            */
  int32_t accepted;     /* 1 if x_dev now holds x_f                             */
  int32_t status;       /* OR of the FPH_ST_* bits of every solve               */
  int32_t solves;       /* pcg_solve calls                                      */
  int32_t cg_iters;     /* CG iterations over all solves and fields             */
  int32_t matvecs;      /* M^T M applications over all solves and fields        */
  int32_t pad;
} fph_hmc_stats_t;

/* Create an HMC context on solver handle h (which must outlive it) with the
 * given options: allocates its device workspace and enqueues, on `stream`,
 * the imaginary-time kernels of the mass (Mass^{-1}, sqrt(Mass), Mass) and of
 * the nt bosonic sub-steps (below).  Errors: FPH_E_NULL, FPH_E_ARG (a
 * non-finite or out-of-range option), FPH_E_NRHS (nfields), FPH_E_HIP. */
int fph_hmc_create(fph_hmc_t* hh, fph_handle_t h, const fph_hmc_opts_t* opts, void* stream);

/* Release the context (synchronises the device). */
int fph_hmc_destroy(fph_hmc_t hh);

/* out_dev[0] = S_B(x) (Eq. S_B), out_dev[1] = -dtau*alpha*sum x (the linear
 * term of Eq. Z_path_orig), both FP64 device scalars.  Enqueue only. */
int bosonic_action(fph_hmc_t hh, const double* x_dev, double* out_dev, void* stream);

/* grad_dev += scale * dS_x/dx for the x-only part of the context's action:
 * dS_B/dx - dtau*alpha for S' (lambda_action 0), dS_B/dx for S, with dS_B/dx
 * of Eq. (dSB_dx), periodic in tau.  Enqueue only. */
int bosonic_force(fph_hmc_t hh, const double* x_dev, double* grad_dev, double scale,
                  void* stream);

typedef enum { FPH_MASS_INV = 0, FPH_MASS_SQRT = 1, FPH_MASS = 2 } fph_mass_op_t;

/* out = op(in) for nvec vectors [Ltau][N]: Mass^{-1}, sqrt(Mass) or Mass
 * (Sec. III B 1, Eq. dynamical_M_def), each a real symmetric circulant over
 * imaginary time applied site by site.  in and out must not overlap.
 * Enqueue only. */
int hmc_mass_apply(fph_hmc_t hh, int32_t op, int32_t nvec, const double* in_dev, double* out_dev,
                   void* stream);

/* The nt bosonic sub-steps of one time step of Algorithm 1, in place:
 *   nt times { p -= h/2 g(x); x += h Mass^{-1} p; p -= h/2 g(x) },
 *   h = dt/nt, g = dS_B/dx - dtau*alpha.
 * The force is linear in x and every operator is diagonal in the Fourier
 * basis, so the nt sub-steps are applied as one exact map per Fourier mode
 * (a 2x2 matrix, plus a constant in the w = 0 mode), i.e. four real
 * circulants over imaginary time.  Enqueue only. */
int hmc_boson_steps(fph_hmc_t hh, double* x_dev, double* p_dev, void* stream);

/* One HMC trial update (Algorithm 1) of the field x_dev [Ltau][N] (a context
 * with one chain; FPH_E_ARG otherwise):
 *   Phi_sigma = A(x_i)^T R_sigma (R_fields_dev [nfields][Ltau][N]);
 *   p = sqrt(Mass) R (R_mom_dev [Ltau][N]);
 *   Nt steps of: p -= dt/2 dS_F/dx; nt bosonic sub-steps; p -= dt/2 dS_F/dx,
 *   the fermion force from pcg_solve with opts.force_solve (each solve
 *   starting from the previous solution) and fermion_force (scale 1/2 per
 *   field); S_F(x_f) from a solve with opts.action_solve;
 *   accept if r_uniform < exp(-(H_f - H_i)).
 * On acceptance x_dev receives x_f; otherwise it is left unchanged.  A
 * trajectory with a non-finite energy, a solve that broke down or met a
 * non-finite value, or an action solve that did not converge is rejected
 * (stats.status tells which).  p_out_dev (may be NULL) receives p_f.  On
 * return the solver handle's field is that of x_dev.  Blocks until done. */
int hmc_trajectory(fph_hmc_t hh, double* x_dev, const double* R_fields_dev,
                   const double* R_mom_dev, double r_uniform, double* p_out_dev,
                   fph_hmc_stats_t* stats_host, void* stream);

/* One HMC trial update of each of the context's nchains independent chains
 * at once (Algorithm 1 per chain, as hmc_trajectory): x_dev [nchains][Ltau][N],
 * R_fields_dev [nchains][nfields][Ltau][N], R_mom_dev [nchains][Ltau][N],
 * r_uniform_host [nchains], p_out_dev [nchains][Ltau][N] (may be NULL),
 * stats_host [nchains] (may be NULL).  Chain k's fields live in the solver
 * as field k of fph_set_fields, its pseudofermions as right-hand sides
 * k*nfields .. k*nfields + nfields - 1; energies and the Metropolis test are
 * per chain, and each accepted chain's x_f replaces its slice of x_dev.
 * The solves of all chains run in the same launches and stop together per
 * right-hand side.  Blocks until done. */
int hmc_trajectories(fph_hmc_t hh, double* x_dev, const double* R_fields_dev,
                     const double* R_mom_dev, const double* r_uniform_host, double* p_out_dev,
                     fph_hmc_stats_t* stats_host, void* stream);

typedef enum {
  FPH_LAMBDA = 0,        /* Lambda      (Eq. Lambda_def)  */
  FPH_LAMBDA_INV = 1,    /* Lambda^{-1} (Eq. Lambda_inv)  */
  FPH_LAMBDA_T = 2,      /* Lambda^T                      */
  FPH_LAMBDA_INV_T = 3   /* Lambda^{-T}                   */
} fph_lambda_op_t;

/* out = op(in) for nvec vectors [Ltau][N], Lambda of the field x_dev (any
 * context; only the lattice's dtau and alpha are used).  Each is one shift
 * in tau per site with a sign and an exponential factor.  in and out must not
 * overlap.  Enqueue only. */
int lambda_apply(fph_hmc_t hh, int32_t op, const double* x_dev, int32_t nvec, const double* in_dev,
                 double* out_dev, void* stream);

/* grad_dev[tau][i] += scale * (-dtau alpha) * sum_r b_r[tau-1][i] u_r[tau-1][i]
 * (slice tau-1 mod Ltau): with A = M Lambda, the one-field force d(b.u)/dx is
 * fermion_force(u) (with b as the right-hand side) plus this term, where
 * b = Lambda^{-T} Phi and u = (M^T M)^{-1} b.  Enqueue only. */
int lambda_force(fph_hmc_t hh, int32_t nrhs, const double* b_dev, const double* u_dev,
                 double* grad_dev, double scale, void* stream);

typedef enum { FPH_MOVE_REFLECT = 0, FPH_MOVE_SWAP = 1 } fph_move_t;

typedef struct {
  double dS;            /* S(x') - S(x)                                        */
  double dS_B;          /* change of the x-only action                         */
  double SF_old;        /* 1/2 sum |R_sigma|^2 = S_F(x)                        */
  double SF_new;        /* S_F(x') from a solve with opts.action_solve          */
  double accept_prob;   /* min(1, exp(-dS))                                    */
  int32_t accepted;     /* 1 if x_dev now holds x'                              */
  int32_t status;       /* OR of the FPH_ST_* bits of the solve                */
  int32_t cg_iters;     /* CG iterations over the fields                        */
  int32_t pad;
} fph_update_stats_t;

/* One Metropolis update by a global move (Sec. IV): kind FPH_MOVE_REFLECT
 * proposes x_i -> -x_i at every tau; FPH_MOVE_SWAP exchanges x_i and x_j
 * (i != j; the paper swaps neighbours).  Phi_sigma = A(x)^T R_sigma is drawn
 * at the current x with the context's action, S_F(x') comes from one solve
 * (opts.action_solve, zero guess), and x' is accepted if
 * r_uniform < exp(-(S(x') - S(x))).  On acceptance x_dev receives x'; a
 * non-converged or non-finite solve rejects.  On return the solver handle's
 * field is that of x_dev.  Errors: FPH_E_ARG for a bad kind or site index,
 * or a context with more than one chain.
 * Blocks until done. */
int hmc_global_update(fph_hmc_t hh, int32_t kind, int32_t i, int32_t j, double* x_dev,
                      const double* R_fields_dev, double r_uniform, fph_update_stats_t* stats_host,
                      void* stream);

/* ------------------------------------------------------------------ */
/* Stochastic Green's-function measurements (Sec. VI).                 */
/*
 * G = M^{-1} estimates the Green's function (Eq. Green_approx); for random
 * vectors xi with <xi xi^T> = I, G ~ (G xi) xi^T (Eq. Hutch_approx), with
 * G xi from (M^T M) v = M^T xi.  Space-time averages over displacements
 * Delta = (dtau, dy, dx) are circular cross-correlations computed with
 * discrete Fourier transforms (Eq. cross_corr).  Result arrays are
 * [Ltau][L][L] doubles indexed [dtau][dy][dx] (the layout of a field).
 * Ncal = N Ltau.  The lattice needs Ltau = P Q with P, Q <= 64.
 */

typedef struct fph_meas_s* fph_meas_t;

/* Create a measurement context on solver handle h (which must outlive it):
 * transform tables and device workspace (six complex grids and max_rhs real
 * vectors).  Errors: FPH_E_NULL, FPH_E_LATTICE (Ltau not a product of two
 * factors <= 64), FPH_E_HIP.  Enqueues the tables on `stream`. */
int fph_meas_create(fph_meas_t* mh, fph_handle_t h, void* stream);

/* Release the context (synchronises the device). */
int fph_meas_destroy(fph_meas_t mh);

/* Unnormalised 3-D DFT over (tau, y, x) of one complex grid (interleaved
 * re/im doubles [Ltau][N][2]): forward exp(-2 pi i k.n / n_d) or inverse
 * exp(+...).  twist = 1 transforms the antiperiodic extension of the grid to
 * 2 Ltau slices on its Ltau odd frequencies: the forward transform first
 * multiplies slice tau by exp(-i pi tau/Ltau), the inverse multiplies its
 * output slice by exp(+i pi tau/Ltau).  in and out must differ.  Enqueue only. */
int meas_fft(fph_meas_t mh, int32_t inverse, int32_t twist, const double* in_dev, double* out_dev,
             void* stream);

/* gxi_dev[n] = G xi_n for nvec real vectors [Ltau][N]: b = M^T xi with the
 * current field, then pcg_solve with *opts (zero guess), in chunks of the
 * handle's max_rhs (Sec. VI B).  stats_host: nvec entries (may be NULL).
 * Blocks until done. */
int green_vectors(fph_meas_t mh, int32_t nvec, const double* xi_dev, double* gxi_dev,
                  const fph_pcg_opts_t* opts, fph_pcg_stats_t* stats_host, void* stream);

/* out_dev[dtau][dy][dx] = (1/nvec) sum_n (1/Ncal) sum_i (Q G xi_n)_{i+Delta} (Q xi_n)_i:
 * the average over space-time of G^ext = Q G Q^T, Q = [I; -I] (Eqs. G_avg-1,
 * G_def-1), estimated with nvec vector pairs (xi_n, G xi_n) (Eq.
 * G_approx_better); dtau in [0, Ltau) (antiperiodic beyond).  The sum runs
 * over the Ncal distinct space-time points.  Enqueue only. */
int green_average(fph_meas_t mh, int32_t nvec, const double* xi_dev, const double* gxi_dev,
                  double* out_dev, void* stream);

/* out_dev[3][Ltau][N]: the averages over space-time of the three products of
 * Green's functions of a four-point measurement (Sec. VI C),
 *   T1 = (1/Ncal) sum_i G_{i+D,i} G_{i+D,i},   T2 = (1/Ncal) sum_i G_{i+D,i+D} G_{i,i},
 *   T3 = (1/Ncal) sum_i G_{i+D,i} G_{i,i+D},
 * each estimated by the average over all pairs n < m of independent vectors
 * (Eq. GG_approx_better) as the cross-correlations
 *   (xi_n . xi_m) * (Gxi_n . Gxi_m),  (xi_n . Gxi_n) * (xi_m . Gxi_m),
 *   (xi_n . Gxi_m) * (xi_m . Gxi_n)   ('.' elementwise, '*' cross-correlation),
 * on the original grid, periodic in tau (the signs of G^ext cancel in each
 * product).  nvec >= 2.  Enqueue only. */
int green_pair_products(fph_meas_t mh, int32_t nvec, const double* xi_dev, const double* gxi_dev,
                        double* out_dev, void* stream);

/* ------------------------------------------------------------------------
 * SSH-type coupling (Sec. II C, closing remark; Sec. III A, force of the SSH
 * model).  The paper states only that the phonon coordinates of the sites
 * enter the hopping matrix K_tau and that the force follows by the product
 * rule through the checkerboard factors.  This library reads it as: bond
 * b = (i, j), j = i + x^ or i + y^, hops with
 *   t_b(x_tau) = t - g (x_{j,tau} - x_{i,tau}),
 * B_tau = diag(E_tau) F_xe F_ye F_xo F_yo with E_tau = exp(-dtau (alpha x_tau - mu))
 * as in the Holstein matrix and F_f = exp(-dtau K_f(x_tau)) for the four bond
 * families (x-bonds from even x, y-bonds from even y, x-bonds from odd x,
 * y-bonds from odd y; F_yo acts first), each a direct sum of two-site blocks
 * [[cosh, sinh], [sinh, cosh]](dtau t_b).  M keeps the block structure of
 * Eq. M_def.  g = 0 gives the Holstein M; alpha = 0 the pure SSH coupling.
 * FP64 only.  Layouts as above: vectors [nrhs][Ltau][N], x [Ltau][N].
 * ------------------------------------------------------------------------ */

typedef struct fph_ssh_s* fph_ssh_t;

/* Context for one lattice (L even in [4, 64], Ltau even >= 2), SSH coupling g
 * and up to max_rhs right-hand sides; allocates its workspace (5 vectors per
 * right-hand side).  Errors: FPH_E_NULL, FPH_E_LATTICE, FPH_E_ARG (g not
 * finite), FPH_E_NRHS, FPH_E_HIP. */
int fph_ssh_create(fph_ssh_t* out, const fph_lattice_t* lat, double g, int32_t max_rhs);

/* Synchronises the device and frees the context.  A context serves one call
 * at a time (its workspace is shared by all its entry points). */
int fph_ssh_destroy(fph_ssh_t c);

/* Copies the field x_dev [Ltau][N] into the context (bond hoppings are
 * formed from it inside the kernels), and sets it on the attached
 * preconditioner's handle.  Enqueue only. */
int ssh_set_field(fph_ssh_t c, const double* x_dev, void* stream);

/* out = M in, M^T in or M^T M in (op FPH_OP_M / _MT / _MTM) for nrhs vectors;
 * in and out must not overlap (FPH_E_ARG).  FPH_E_NOFIELD before
 * ssh_set_field.  Enqueue only. */
int ssh_matvec(fph_ssh_t c, int32_t op, int32_t nrhs, const double* in_dev, double* out_dev,
               void* stream);

/* Let ssh_solve precondition with the adiabatic preconditioner of the
 * Holstein handle h (Sec. V A, Eq. CG_precon): uniform hopping t and the
 * on-site factor of the field.  From now on ssh_set_field also sets h's
 * field (fph_set_field with the Chebyshev-order constants a1, a2).  h must
 * have the same lattice (FPH_E_LATTICE otherwise) and outlive its use; NULL
 * detaches.  The preconditioner uses h's workspace: calls on contexts that
 * share one h (or on h itself) must not overlap.  Host only. */
int ssh_set_preconditioner(fph_ssh_t c, fph_handle_t h, double a1, double a2);

/* (P)CG on (M^T M) u = b (Sec. II D, Eq. CG; Eq. CG_precon with
 * z = F F^T r from the attached Holstein handle when opts->use_precond is 1,
 * FPH_E_ARG if none is attached; FPH_E_NRHS above that handle's max_rhs).
 * opts->prec FPH_F64: FP64 CG; each right-hand side stops on its own at
 * |r| < tol |b| (recursive residual).  FPH_F32_REFINED: FP32 CG (the bond
 * and field tables rounded to FP32) on a correction, with reliable updates
 * of the residual: when a right-hand side's FP32 residual has fallen by
 * opts->ru_delta (0 -> 0.1 with the preconditioner, 0.3 without; at most
 * 0.5) since the last FP64 evaluation, or its FP32 iteration stops, the
 * correction joins the FP64 iterate and the FP64 residual b - M^T M u is
 * evaluated; the right-hand side finishes when that residual is below
 * tol |b|, after opts->max_outer evaluations (0 -> 32) or maxiter FP32
 * iterations (FPH_ST_MAXITER).  Other precisions: FPH_E_PREC.
 * opts->chunk iterations (0 -> 64) are enqueued between host checks.
 * stats_host (nrhs entries, may be NULL) hold the iterations, the FP64
 * evaluations after the first (outer_iters), the FP64 true relative
 * residual and S_F = b . u.  Blocks until done. */
int ssh_solve(fph_ssh_t c, int32_t nrhs, const double* b_dev, double* u_dev,
              const fph_pcg_opts_t* opts, fph_pcg_stats_t* stats_host, void* stream);

/* out_dev[r] = b_r . u_r in FP64 for r < nrhs (S_F of Eq. Sf_Psi for the
 * solutions u of ssh_solve).  Uses the context's workspace.  Enqueue only. */
int ssh_action(fph_ssh_t c, int32_t nrhs, const double* b_dev, const double* u_dev, double* out_dev,
               void* stream);

/* grad_dev [Ltau][N] += scale * s * sum_r dS_F/dx with S_F = b . (M^T M)^{-1} b and
 * u_dev [nrhs][Ltau][N] the solutions (Eq. dSF_dx):
 *   dS_F/dx_{i,tau} = 2 (M u)_tau . (dB_tau/dx_{i,tau}) u~_{tau-1},  u~_{-1} = -u_{Ltau-1},
 * dB by the product rule through the four family factors (Sec. III A) plus
 * the on-site term.  s = *scale_dev (device memory, read when the kernel
 * runs) or 1 when scale_dev is NULL multiplies the result as in
 * fermion_force.  Uses the context's workspace for M u.  Enqueue only. */
int ssh_force(fph_ssh_t c, int32_t nrhs, const double* u_dev, double* grad_dev, double scale,
              const double* scale_dev, void* stream);

/* HMC context (as fph_hmc_create) whose update runs on the SSH operator of
 * ssh: trajectories (hmc_trajectory) and global updates (hmc_global_update)
 * with the action S' = S_B - dtau alpha sum x + 1/2 sum_sigma Phi_sigma .
 * (M^T M)^{-1} Phi_sigma, M the SSH-type matrix, Phi_sigma = M(x_i)^T R_sigma.
 * Solves go through ssh_solve: both solve options must be FPH_F64 or
 * FPH_F32_REFINED (FPH_E_PREC), use_precond needs an attached
 * preconditioner.
 * lambda_action and nchains > 1 are refused (FPH_E_ARG): Lambda belongs to
 * the Holstein coupling and the SSH context has one field.  ssh must outlive
 * the context. */
int fph_hmc_create_ssh(fph_hmc_t* hh, fph_ssh_t ssh, const fph_hmc_opts_t* opts, void* stream);

/* ---------------------------------------------------------- measurement */

/* Copies `bytes` from src_dev to dst_dev (device buffers, 16-byte aligned,
 * not overlapping; bytes a multiple of 16) with one of two access
 * patterns, to measure the HBM bandwidth the GPU sustains: the ceiling
 * against which the fused operator's bandwidth is read.
 *   pattern 0: every workgroup sweeps one common window of the buffer
 *     (grid-stride; nontemporal loads and stores);
 *   pattern 1: workgroup b copies its own contiguous 1/nblocks of the
 *     buffer, as each workgroup of the operator streams its own chunk of
 *     time slices.
 * nblocks <= 0 means one workgroup per compute unit; at most 2^20.
 * 512 threads per workgroup.  FPH_E_NULL, FPH_E_ALIGN or FPH_E_ARG for bad
 * arguments; bytes = 0 does nothing.  Enqueue only. */
int fph_hbm_copy(const void* src_dev, void* dst_dev, int64_t bytes, int32_t nblocks,
                 int32_t pattern, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* HOLSTEIN_HMC_H */
