/*
 * polymat.h - C ABI of the MI355X FFT-CONV library for truncated matrix power
 * series and the NSPT updates of the twisted Eguchi-Kawai model
 * (arXiv:2001.02835): the Euler-Langevin step (with caller-supplied noise or
 * noise drawn on the device), the leapfrog molecular-dynamics trajectory, a
 * stochastic gauge-fixing step, and the action and Wilson-loop series.
 *
 * Series layout (all entry points): a truncated power series in g whose
 * coefficients are N x N complex matrices (Section 2, eq. (4)) is a dense,
 * row-major array of complex128 values (interleaved re, im doubles) of shape
 * [ntrunc + 1][N][N]; element (k, i, j) holds entry (i, j) of the coefficient
 * of g^k.  All operand pointers are DEVICE pointers owned by the caller and
 * must be 16-byte aligned.
 *
 * Execution: every call validates its arguments on the host first.  On any
 * validation failure it returns an error status and enqueues nothing.  On
 * success it only enqueues kernels on `stream` (a hipStream_t, NULL = the
 * default stream) and returns PM_OK without synchronising: results are ready
 * when the stream reaches that point.  Calls never allocate device memory:
 * all scratch space is the caller's `workspace` (device memory, 256-byte
 * aligned, not overlapping any operand), sized by the matching *_size query.
 * A device fault surfaces as PM_ERR_DEVICE on a later call or at the
 * caller's synchronisation.  No C++ exception crosses this interface.
 * Calls enqueue kernel launches only (no memset or copy), so a call can be
 * captured into a HIP graph and replayed (with phase timing off).
 * Host-side state (phase-timing records; otherwise constants) is
 * thread-safe; calls that share one workspace must be ordered on one stream.
 *
 * Precision modes (the per-frequency products only; the transforms, their
 * twiddles and 1/L normalisation, the rescaling and every value stored in a
 * caller's series are FP64):
 *   PM_PREC_FP64   - FP64 MFMA products (the three-real-product form of a
 *                    complex product; the environment variable
 *                    POLYMAT_GEMM_4M=1 selects the four-product form).
 *   PM_PREC_FP32   - Fourier coefficients rounded to FP32, FP32 MFMA products
 *                    with FP32 accumulation.
 *   PM_PREC_BF16X3 - Fourier coefficients split as hi + lo with hi, lo BF16;
 *                    hi*hi + hi*lo + lo*hi on BF16 MFMA with FP32 accumulation.
 *
 * Rescaling g -> s g: both operands of a product are multiplied by s^k at
 * order k before the forward transform and the result by s^-k after the
 * inverse one; in exact arithmetic the product is unchanged, in floating
 * point it balances the magnitudes of the orders.  `scale` > 0 fixes s;
 * `scale` == 0 lets the library choose s on the device from the per-order
 * Frobenius norms of the operands; `scale` < 0 (or NaN/Inf) is invalid.
 */
#ifndef POLYMAT_H
#define POLYMAT_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
enum {
  PM_OK = 0,
  PM_ERR_INVALID = 1,     /* bad size, null/misaligned pointer, overlap, bad scale */
  PM_ERR_WORKSPACE = 2,   /* workspace smaller than the *_size query requires */
  PM_ERR_DEVICE = 3,      /* a HIP call failed (launch error or earlier fault) */
  PM_ERR_UNSUPPORTED = 4, /* valid request outside what is built (e.g. ntrunc > 63) */
  PM_ERR_NONFINITE = 5    /* finiteness check on (polymat_check_enable): a NaN or
                             Inf in an operand, or a result coefficient that is
                             not finite */
};
typedef int pm_status;

/* Precision modes of the per-frequency products. */
enum { PM_PREC_FP64 = 0, PM_PREC_FP32 = 1, PM_PREC_BF16X3 = 2 };

/* Operand forms in a batched problem. */
enum {
  PM_OP_N = 0,  /* the series itself */
  PM_OP_C = 1   /* its Hermitian conjugate series, (X^+)^(k) = (X^(k))^+ */
};

/* Largest supported truncation order: the order-axis transform length is
 * L = max(4, next power of two >= 2 (ntrunc + 1)) and must be <= 128. */
#define PM_MAX_NTRUNC 63
/* Largest supported matrix size N. */
#define PM_MAX_N 4096
/* Largest number of problems in one batched call. */
#define PM_MAX_BATCH 4096

/* Bump on any incompatible change of this header. */
int polymat_abi_version(void);

/* Human-readable text for a status code (static storage, never NULL). */
const char* polymat_strerror(pm_status status);

/* Transform length L used for a truncation order (0 if ntrunc is invalid). */
int polymat_transform_length(int ntrunc);

/*
 * polymat_mul - truncated star product C = A * B (Section 2, eq. (5)):
 *     C^(k) = sum_{l=0..k} A^(l) B^(k-l),   k = 0..ntrunc,
 * computed by FFT-CONV (Section 2, Steps 1-5, eqs. (6)-(9)): the order axis
 * is zero-padded to L >= 2 (ntrunc + 1), transformed per matrix entry with
 * w = exp(+2 pi i / L), multiplied mode by mode as N x N complex matrices,
 * transformed back with w^-1 and 1/L, and truncated to orders 0..ntrunc.
 *
 *   A, B, C    device complex128 [ntrunc+1][n][n].  C may alias A or B
 *              (it is written only after both are consumed, on one stream).
 *   n          1 <= n <= PM_MAX_N.   ntrunc: 0 <= ntrunc <= PM_MAX_NTRUNC.
 *   precision  PM_PREC_* above.     scale: see "Rescaling" above.
 *   workspace  >= polymat_workspace_size(n, ntrunc, precision, 1) bytes.
 * Returns PM_OK or an error status (nothing enqueued on error).
 * With PM_PREC_FP64, ntrunc == 0 and C not aliasing A or B the call takes
 * the direct form of polymat_mul_naive instead (one matrix product against
 * L = 4 mode products plus the transforms; from ntrunc = 1 on the transform
 * path is faster for one product at N = 225); the arguments are validated
 * the same way.
 */
pm_status polymat_mul(const void* A, const void* B, void* C, int n, int ntrunc,
                      int precision, double scale, void* workspace,
                      size_t workspace_bytes, void* stream);

/*
 * polymat_mul_naive - the same product by the direct convolution of eq. (5)
 * (the paper's Naive-CONV, Section 2), in FP64 on the matrix cores:
 *     C^(k) = sum_{l=0..k} op_a(A)^(l) op_b(B)^(k-l),   k = 0..ntrunc,
 * one N x N x (k+1)N complex product per order k, no transform and no
 * rescaling; cost (ntrunc+1)(ntrunc+2)/2 matrix products.
 *   A, B, C    device complex128 [ntrunc+1][n][n]; C must not overlap A or B
 *              (PM_ERR_INVALID).  op_a, op_b: PM_OP_N or PM_OP_C.
 *   n          1 <= n <= PM_MAX_N.   ntrunc: 0 <= ntrunc <= PM_MAX_NTRUNC.
 * No workspace.  Returns PM_OK or an error status (nothing enqueued on error).
 */
pm_status polymat_mul_naive(const void* A, const void* B, void* C, int n, int ntrunc,
                            int op_a, int op_b, void* stream);

/* Workspace bytes for `count` products of one shape (count >= 1), or 0 if
 * the arguments are invalid. */
size_t polymat_workspace_size(int n, int ntrunc, int precision, int count);

/*
 * One problem of a batched call.  C = op_a(A) * op_b(B) with op in PM_OP_*;
 * A, B, C, n, ntrunc and scale as in polymat_mul.  The problems of one call
 * are independent (the batching of Section 2: transforms batched over matrix
 * entries and products batched over modes, here also over problems) and may
 * differ in n and ntrunc.  Every A and B of the call is consumed before any C
 * is written, so a C may alias any operand of the call; two problems must not
 * write overlapping C (PM_ERR_INVALID).
 */
typedef struct {
  const void* A;
  const void* B;
  void* C;
  int n;
  int ntrunc;
  int op_a;
  int op_b;
  double scale;
} pm_problem;

/* Workspace bytes for one batched call over `problems` (host array of
 * `count` entries), or 0 if any problem is invalid. */
size_t polymat_batched_workspace_size(const pm_problem* problems, int count,
                                      int precision);

/*
 * polymat_mul_batched - all problems of a host array in one set of launches
 * (one forward-transform launch, one product launch per precision, one
 * inverse-transform launch for the whole batch).  Same semantics per problem
 * as polymat_mul.  1 <= count <= PM_MAX_BATCH.
 */
pm_status polymat_mul_batched(const pm_problem* problems, int count,
                              int precision, void* workspace,
                              size_t workspace_bytes, void* stream);

/*
 * polymat_mul_noalloc - polymat_mul without a workspace argument, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation).  The workspace is
 * a file-scope device array of PM_NOALLOC_SCRATCH_BYTES bytes inside the
 * library, one per GPU, held from the first use on that GPU until the
 * process ends; the call itself allocates nothing.
 *   A, B, C, n, ntrunc, precision, scale: as in polymat_mul.
 *   stream: its device selects which GPU's array is used.
 * Returns PM_ERR_UNSUPPORTED when polymat_workspace_size(n, ntrunc,
 * precision, 1) exceeds PM_NOALLOC_SCRATCH_BYTES (e.g. N = 225 fits up to
 * ntrunc = 31 in FP64 and up to ntrunc = 63 in FP32 and split BF16), and the
 * errors of polymat_mul otherwise; nothing is enqueued on error.  Results
 * equal those of polymat_mul bitwise (same kernels, same workspace layout).
 * All calls on one GPU share its array: calls that may overlap in time on
 * one GPU (different streams, different host threads) race and must be
 * ordered by the caller.
 */
#define PM_NOALLOC_SCRATCH_BYTES (160u << 20)
pm_status polymat_mul_noalloc(const void* A, const void* B, void* C, int n, int ntrunc,
                              int precision, double scale, void* stream);

/*
 * polymat_check_enable - opt-in finiteness check of polymat_mul and
 * polymat_mul_batched (process-wide, off by default).  The check itself runs
 * on the device in every call: the rescaling step records whether a
 * per-order norm of an operand is not finite (auto scale only), and the
 * inverse transform (Steps 4-5) records whether it stored a non-finite
 * coefficient of C; both words sit in the product's region of the workspace.
 * A NaN or Inf anywhere in A or B reaches every coefficient of C through the
 * order-axis transform, so the second word also covers a fixed scale.
 * With the check on, a call enqueues its kernels, then synchronises `stream`,
 * reads those words back and returns PM_ERR_NONFINITE if any is set (C is
 * written all the same); polymat_mul then always takes the transform path.
 * A call on a stream under graph capture returns PM_ERR_INVALID while the
 * check is on.  The NSPT entry points are not checked.
 */
pm_status polymat_check_enable(int on);

/*
 * polymat_forward_transform - Steps 1-2 alone (eqs. (6)-(7)), FP64:
 *     At^(p) = sum_{k=0..ntrunc} s^k A^(k) w^{kp},  p = 0..L-1,
 * L = polymat_transform_length(ntrunc), s = scale (> 0; no automatic mode).
 *   A   device complex128 [ntrunc+1][n][n];  At  device complex128 [L][n][n]
 *   (must not overlap A).  workspace: >= polymat_transform_workspace_size().
 * Exposed so that the transform can be checked on its own and reused.
 */
pm_status polymat_forward_transform(const void* A, void* At, int n, int ntrunc,
                                    double scale, void* workspace,
                                    size_t workspace_bytes, void* stream);

/*
 * polymat_inverse_transform - Steps 4-5 alone (eqs. (9) and the truncation):
 *     C^(k) = s^-k (1/L) sum_{p=0..L-1} Ct^(p) w^{-kp},  k = 0..ntrunc.
 *   Ct  device complex128 [L][n][n];  C  device complex128 [ntrunc+1][n][n]
 *   (must not overlap Ct).  workspace: >= polymat_transform_workspace_size().
 */
pm_status polymat_inverse_transform(const void* Ct, void* C, int n, int ntrunc,
                                    double scale, void* workspace,
                                    size_t workspace_bytes, void* stream);

/* Workspace bytes of polymat_forward_transform / polymat_inverse_transform
 * (a small table of s^k factors). */
size_t polymat_transform_workspace_size(void);

/*
 * Phase timing for measurement tools.  While enabled, each kernel launch the
 * library makes is bracketed by two HIP events recorded on the caller's
 * stream; polymat_timing_read waits for the recorded events, adds up the
 * elapsed time and the launch count per phase, and clears the record.
 * Timing adds two event records per launch and is off by default; it is not
 * meant to be used under stream capture.
 *   ms[PM_NUM_PHASES], launches[PM_NUM_PHASES]: host arrays (either may be NULL).
 */
enum {
  PM_PHASE_RESCALE = 0,   /* per-order norms and choice of s */
  PM_PHASE_FORWARD = 1,   /* Steps 1-2: rescale, pad, forward transform */
  PM_PHASE_PRODUCT = 2,   /* Step 3: mode-wise complex matrix products */
  PM_PHASE_INVERSE = 3,   /* Steps 4-5: inverse transform, truncation, unscale */
  PM_PHASE_OTHER = 4,     /* NSPT element-wise passes (trace, force and noise) */
  PM_PHASE_RETRUNC = 5,   /* NSPT re-truncation of Fourier-space products */
  PM_PHASE_PIPELINE = 6,  /* persistent launch of all steps of an FP64 batch (and its set-up) */
  PM_NUM_PHASES = 7
};
pm_status polymat_timing_enable(int on);
pm_status polymat_timing_read(double* ms, int* launches);

/*
 * NSPT Euler-Langevin step of the four-dimensional TEK model (Section 2,
 * eqs. (1)-(3)), for `replicas` independent chains at once.
 *
 * Twist: z_{mu nu} = exp(2 pi i k / L) for mu < nu, z_{nu mu} = conj(z_{mu nu}).
 * With every product the truncated star product, for each replica and mu:
 *   S_mu   = U_mu * sum_{nu != mu} ( z_{mu nu} U_nu * U_mu^+ * U_nu^+
 *                                  + z_{mu nu}^* U_nu^+ * U_mu^+ * U_nu )
 *   F^(k)  = i [ D^(k) - Tr(D^(k))/N ],  D = S_mu - S_mu^+   (every order k)
 *   X^(k)  = eps F^(k) + delta_{k,1} sqrt(2 eps) eta_mu,   X^(0) = 0
 *   U_mu  <- exp(i X) * U_mu,  exp(Y) = sum_{m=0..ntrunc} Y^{*m} / m!
 * All four directions are updated from the old links.  The plus sign of the
 * second staple term, the beta absorbed into the rescaled time step and the
 * dropped order-0 drift are this library's reading of eqs. (2)-(3).
 */
typedef struct {
  int n;        /* N = L * L */
  int L;        /* twist lattice size (odd) */
  int k;        /* twist flux */
  int ntrunc;   /* truncation order */
  double eps;   /* rescaled Langevin time step, or the MD step dt (> 0) */
} nspt_params;

/* Workspace bytes for nspt_langevin_step, nspt_langevin_steps, nspt_md_trajectory and the
 * other NSPT calls, or 0 if invalid. */
size_t nspt_workspace_size(int replicas, const nspt_params* params, int precision);

/*
 *   U    device complex128 [replicas][4][ntrunc+1][n][n], updated in place
 *        (order 0 is left unchanged).
 *   eta  device complex128 [replicas][4][n][n]: Hermitian traceless noise.
 *   precision applies to the per-frequency products; U stays FP64.
 * The product rescaling is chosen on the device once per call from the
 * norms of U.
 */
pm_status nspt_langevin_step(void* U, const void* eta, int replicas,
                             const nspt_params* params, int precision,
                             void* workspace, size_t workspace_bytes,
                             void* stream);

/*
 * nspt_noise - the Langevin noise of one step drawn on the device from a
 * counter-based generator, so that a run needs no host-side noise (the
 * paper does not say how its noise is generated; this is the library's
 * choice).  For matrix m = 4 r + mu (replica r, direction mu) and entry pair
 * i <= j: counter (i n + j, m, step, 0) and key (seed, 0) of Philox4x64-10
 * (Salmon et al., SC'11); of its outputs x0, x1, u_a = ((x0 >> 11) + 1) 2^-53,
 * u_b = (x1 >> 11) 2^-53, rho = sqrt(-2 ln u_a), z0 = rho cos(2 pi u_b),
 * z1 = rho sin(2 pi u_b); eta_ij = (z0 + i z1) / sqrt(2) = conj(eta_ji) for
 * i < j, eta_ii = z0, and finally eta_ii -= Tr(eta) / n.  This is the
 * Hermitian traceless (GUE) noise of nspt_langevin_step.
 *   eta       device complex128 [replicas][4][n][n], written.
 *   replicas  1 .. 1024;  n  1 .. PM_MAX_N.
 */
pm_status nspt_noise(void* eta, int replicas, int n, unsigned long long seed,
                     unsigned long long step, void* stream);

/*
 * nspt_langevin_steps - nsteps Euler-Langevin steps (those of
 * nspt_langevin_step) with the noise of nspt_noise for steps step0,
 * step0 + 1, ..., drawn on the device into the workspace.
 *   U       device complex128 [replicas][4][ntrunc+1][n][n], updated in place.
 *   nsteps  1 .. 100000.
 * The workspace is the one of nspt_langevin_step (nspt_workspace_size); U
 * and the workspace must not overlap (PM_ERR_INVALID).
 */
pm_status nspt_langevin_steps(void* U, int replicas, const nspt_params* params,
                              unsigned long long seed, unsigned long long step0, int nsteps,
                              int precision, void* workspace, size_t workspace_bytes,
                              void* stream);

/*
 * One molecular-dynamics trajectory of the NSPT tower (Section 2, eq. (3)
 * and the sentence after it: the truncated tower dU/dt = i (P * U),
 * dP^(k)/dt = F^(k) is integrated by a symplectic integrator, with periodic
 * momentum refreshment), for `replicas` chains at once.
 *
 * The momentum is the series P = sum_{k>=1} g^k P^(k) (no order-0 term),
 * Hermitian traceless at every order; F^(k) is the force of
 * nspt_langevin_step for k >= 1.  The integrator is the leapfrog with step
 * dt = params->eps in kick-drift-kick order:
 *   P <- P + dt/2 F(U);  repeat nsteps times { U_mu <- exp(i dt P_mu) * U_mu;
 *   P <- P + dt F(U) (dt/2 after the last drift) }.
 * All four directions move together (every force from the current links).
 *
 *   U    device complex128 [replicas][4][ntrunc+1][n][n], updated in place
 *        (order 0 is left unchanged).
 *   P    device complex128 [replicas][4][ntrunc+1][n][n], updated in place.
 *   eta  device complex128 [replicas][4][n][n] or NULL.  When not NULL the
 *        momentum is refreshed before the trajectory: P^(1) = eta (Hermitian
 *        traceless), every other order zero.  When NULL the trajectory
 *        continues from the P passed in.
 *   nsteps  number of leapfrog steps, 1 .. 100000.
 * The workspace is the one of nspt_langevin_step (nspt_workspace_size with
 * the same arguments).  U, P, eta and the workspace must not overlap
 * (PM_ERR_INVALID).  One leapfrog step after a refresh equals one
 * nspt_langevin_step with eps = dt^2 / 2 and the same eta.
 */
pm_status nspt_md_trajectory(void* U, void* P, const void* eta, int replicas,
                             const nspt_params* params, int nsteps, int precision,
                             void* workspace, size_t workspace_bytes,
                             void* stream);

/*
 * nspt_gauge_fix - one stochastic gauge-fixing step for `replicas` link sets.
 * The paper uses stochastic gauge fixing in its NSPT runs and omits the
 * details (Section 2); the form here is this library's design.  The reduced
 * model is invariant under U_mu -> Omega U_mu Omega^+ (one Omega for all
 * directions).  With Gamma_mu = U_mu^(0) (the twist eaters) and every
 * product the truncated star product:
 *   G     = sum_mu ( U_mu * Gamma_mu^+ - Gamma_mu^+ * U_mu )
 *   Y^(k) = -(alpha/2) [ D^(k) - Tr(D^(k))/N ],  D = G - G^+,  Y^(0) = 0
 *   U_mu <- Omega * U_mu * Omega^+,  Omega = exp(Y),  for every mu.
 * This is one steepest-ascent step of size alpha of the reduced-model Landau
 * functional sum_mu Re Tr(Omega U_mu Omega^+ Gamma_mu^+).  To first order a
 * pure-gauge fluctuation that is an eigenmode of the conjugations by the
 * twist eaters, with phases phi_nu, is multiplied by
 * 1 - alpha sum_nu |1 - phi_nu|^2; every mode is damped for 0 < alpha < 1/8.
 * Gauge-invariant observables (nspt_action, nspt_wilson_loop) are unchanged
 * up to rounding, and order 0 is left unchanged.
 *   U      device complex128 [replicas][4][ntrunc+1][n][n], updated in place.
 *   alpha  step size, finite and >= 0 (0 returns at once: Omega = 1).
 * params is checked as for nspt_langevin_step (eps > 0), but eps is not
 * used.  precision applies to the products.  The
 * workspace is the one of nspt_langevin_step (nspt_workspace_size); U and
 * the workspace must not overlap (PM_ERR_INVALID).
 */
pm_status nspt_gauge_fix(void* U, int replicas, const nspt_params* params, double alpha,
                         int precision, void* workspace, size_t workspace_bytes,
                         void* stream);

/*
 * nspt_action - the action of eq. (1) at beta = 1 as a series in g, for
 * `replicas` link sets (the observable of the plaquette, i.e. the 1x1
 * Wilson loop: W^(k) = delta_k0 - S^(k) / (12 N)):
 *   S^(k) = sum_{mu != nu} Tr[ delta_k0 1 - z_{mu nu} (U_mu * U_nu * U_mu^+ * U_nu^+)^(k) ]
 *         = 12 N delta_k0 - 2 Re sum_{mu < nu} z_{mu nu} Tr (U_mu * U_nu * U_mu^+ * U_nu^+)^(k).
 *   U    device complex128 [replicas][4][ntrunc+1][n][n] (read only).
 *   S    device float64 [replicas][ntrunc+1], written.
 * precision applies to the products.  The workspace is the one of
 * nspt_langevin_step (nspt_workspace_size); U, S and the workspace must not
 * overlap (PM_ERR_INVALID).
 */
pm_status nspt_action(const void* U, int replicas, const nspt_params* params,
                      int precision, double* S, void* workspace,
                      size_t workspace_bytes, void* stream);

/*
 * nspt_wilson_loop - the a x b Wilson loop of the reduced model as a series
 * in g (the observable whose perturbative coefficients the paper computes,
 * abstract and Section 1), averaged over the six planes:
 *   W^(k) = 1/(6N) sum_{mu<nu} Re z_{mu nu}^{ab} Tr (U_mu^a * U_nu^b * (U_mu^+)^a * (U_nu^+)^b)^(k),
 * with z_{mu nu}^{ab} = exp(2 pi i k a b / L) for mu < nu, so that W = 1 at the
 * twisted vacuum; W(1, 1) = 1 - S / (12 N) with S the series of nspt_action.
 *   U     device complex128 [replicas][4][ntrunc+1][n][n] (read only).
 *   a, b  loop sides, 1 .. 4.
 *   W     device float64 [replicas][ntrunc+1], written.
 * precision applies to the products.  The workspace is the one of
 * nspt_langevin_step (nspt_workspace_size); U, W and the workspace must not
 * overlap (PM_ERR_INVALID).
 */
pm_status nspt_wilson_loop(const void* U, int replicas, const nspt_params* params,
                           int a, int b, int precision, double* W, void* workspace,
                           size_t workspace_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* POLYMAT_H */
