/*
 * sch.h -- C-ABI of the MI355X (gfx950) library for the particle filter of
 * the viscous stochastic Camassa-Holm (SALT) equation, after Cotter, Crisan &
 * Singh, "Data assimilation for the stochastic Camassa-Holm equation using
 * particle filtering: a numerical investigation" (arXiv 2402.06927).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Memory.  Every array argument is a DEVICE pointer to memory the caller
 *    owns (allocated by the caller, e.g. through PyTorch); the library never
 *    allocates, frees or retains user memory.  Calls that need scratch space
 *    take a caller-owned device workspace of at least sch_workspace_bytes()
 *    bytes.  Scalars documented as "host" are plain values.
 *  - Layout.  Row-major, particle-major: a field over the ensemble is
 *    [n_particles][nx] with nodes contiguous; node i sits at x_i = i L / nx on
 *    the periodic interval [0, L).  Noise increments are
 *    [n_particles][n_steps][n_modes].  Floating point is IEEE binary64
 *    throughout; indices are int32.
 *  - Streams.  `stream` is a hipStream_t passed as void* (NULL = the null
 *    stream).  Calls only enqueue work and return, unless documented as
 *    synchronising (the cycle drivers read a few scalars back each step).
 *  - Errors.  Every call returns an int status.  Arguments are validated on
 *    the host before anything is enqueued; on a non-zero status nothing has
 *    been enqueued (validation errors) or the HIP runtime reported a failure
 *    (SCH_E_HIP).  sch_last_error() returns a thread-local message about the
 *    last failure.  Conditions found on the device (a particle whose implicit
 *    solve did not converge or produced a non-finite state) are reported per
 *    particle through the optional `status` arrays, with the same codes.
 *  - The velocity u must equal the Helmholtz image of the momentum m
 *    (H u = M m, see sch_velocity); the library treats m as the prognostic
 *    variable and uses u as the starting guess of the implicit solve.
 */
#ifndef SCH_H
#define SCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SCH_OK 0
#define SCH_E_ARG (-1)          /* null pointer, non-positive size, bad parameter   */
#define SCH_E_SHAPE (-2)        /* size combination the kernels do not support      */
#define SCH_E_NONCONVERGED (-3) /* implicit solve hit picard_max without converging */
#define SCH_E_NONFINITE (-4)    /* a NaN or infinity appeared in a particle state   */
#define SCH_E_DEGENERATE (-5)   /* all weights zero, or the tempering-step cap hit  */
#define SCH_E_HIP (-6)          /* the HIP runtime reported an error                */
#define SCH_E_UNSTABLE (-7)     /* an implicit-step system outside the range where  */
                                /* elimination without pivoting is safe (growth of */
                                /* the eliminated super-diagonal above 2^16)        */

/* Stage tags of the counter-based generator (bits 24..31 of counter word 2). */
#define SCH_TAG_INIT 0u
#define SCH_TAG_FORECAST 1u
#define SCH_TAG_PCN 2u
#define SCH_TAG_ACCEPT 3u
#define SCH_TAG_RESAMPLE 4u
#define SCH_TAG_OBS 5u
#define SCH_TAG_NUDGE 6u

/* Model of section 2 (eqs. schce1, sde1, fde1) with the noise in the modes
 * form dU = sum_q xi_q dW_q of section 2 (the expansion used in earlier SALT
 * work), discretised with P1 elements on nx periodic cells of width L/nx and
 * the implicit midpoint rule in time. */
typedef struct sch_model {
  double L;          /* domain length                                        */
  double alpha;      /* Helmholtz length scale in m = u - alpha^2 u_xx       */
  double mu;         /* viscosity                                            */
  double dt;         /* time step                                            */
  int32_t nx;        /* nodes = cells, >= 64                                 */
  int32_t n_modes;   /* noise modes Q, 1..64                                 */
  const double *xi;  /* device [n_modes][nx]: nodal values of the modes      */
  double picard_tol; /* relative max-norm error of m that ends the solve     */
  int32_t picard_max;/* iteration cap of the implicit solve                  */
} sch_model;

/* Observations of section 3 (eq. obseq): n_obs points x_j = j L / n_obs,
 * the P1 velocity evaluated there, Gaussian errors with std sigma_j. */
typedef struct sch_obs {
  int32_t n_obs;
  const double *y;     /* device [n_obs] */
  const double *sigma; /* device [n_obs] */
} sch_obs;

/* Keys of the Philox4x32-10 counter-based generator (Salmon et al., SC'11):
 * seed is the 64-bit key; cycle and temper_k enter the counter. */
typedef struct sch_rng {
  uint64_t seed;
  uint32_t cycle;
  uint32_t temper_k;
} sch_rng;

/* Per-cycle statistics returned by the cycle drivers (host struct). */
typedef struct sch_cycle_stats {
  double ess;            /* bootstrap: ESS before resampling; tempered: last step */
  int32_t resampled;     /* bootstrap: 1 if the ensemble was resampled            */
  int32_t n_temper;      /* tempered: number of tempering steps                   */
  int64_t picard_iters;  /* implicit-solve iterations summed over the cycle       */
  int64_t n_accept;      /* tempered: pCN acceptances summed over the cycle       */
  int64_t particle_steps;/* model steps integrated (all particles, all windows)   */
  int32_t status;        /* SCH_OK or the first error met                         */
  int32_t n_failed;      /* particles whose forecast window failed (not converged */
                         /* or non-finite): weight zero, replaced when resampled  */
} sch_cycle_stats;

/* Message about the last failure on the calling thread ("" if none). */
const char *sch_last_error(void);
/* Library version, 100 * major + minor. */
int sch_version(void);

/* Workspace sizes in bytes.  `which` is one of the SCH_WS_* values; `extra`
 * is the number of pCN moves per call / per tempering step for SCH_WS_JITTER
 * and SCH_WS_TEMPERED, the checkpoint interval (steps) for SCH_WS_NUDGE_GRAD
 * and SCH_WS_NUDGE, and ignored otherwise.  Returns 0 for invalid
 * arguments. */
#define SCH_WS_RESAMPLE 1
#define SCH_WS_BOOTSTRAP 2
#define SCH_WS_TEMPERED 3
#define SCH_WS_JITTER 4
#define SCH_WS_NUDGE_GRAD 5
#define SCH_WS_NUDGE 6
size_t sch_workspace_bytes(int32_t which, const sch_model *model, int32_t n_particles,
                           int32_t n_steps, int32_t extra);

/* --------------------------------------------------------------------------
 * Noise.  dW[p][n][q] = sqrt(dt) z, z ~ N(0,1) by Box-Muller from one Philox
 * block per mode pair, counter (p, rng->cycle * n_steps + n,
 * (q/2) | tag << 24, rng->temper_k << 16): the iid N(0, dt) prior of the
 * Brownian increments (section 3.1.2).  Modes 2k, 2k+1 share one block.
 * ------------------------------------------------------------------------ */
int sch_draw_increments(const sch_rng *rng, uint32_t tag, int32_t n_particles, int32_t n_steps,
                        int32_t n_modes, double dt, double *dW, void *stream);

/* Raw generator output: out[i][0..3] = Philox4x32-10 of the counter
 * ctr[i][0..3] under the key `seed` (device arrays [n][4] of uint32).  Lets
 * callers check the stream bit for bit against another implementation. */
int sch_philox_blocks(uint64_t seed, int32_t n, const uint32_t *ctr, uint32_t *out, void *stream);

/* --------------------------------------------------------------------------
 * Helmholtz relation, first line of eq. fde1: (M + alpha^2 K) u = M m, with
 * M, K the P1 mass and stiffness matrices.  sch_velocity gives u from m;
 * sch_init_momentum gives m from u (M m = (M + alpha^2 K) u; section 2:
 * m(x,0) from u(x,0)).  In-place use is not allowed.
 * ------------------------------------------------------------------------ */
int sch_velocity(const sch_model *model, int32_t n_particles, const double *m, double *u,
                 void *stream);
int sch_init_momentum(const sch_model *model, int32_t n_particles, const double *u, double *m,
                      void *stream);

/* --------------------------------------------------------------------------
 * sch_ensemble_step: advance every particle n_steps implicit-midpoint steps
 * of eq. fde1,
 *   (m^{n+1} - m^n, phi) + mu dt (d_x m^{n+1/2}, d_x phi)
 *     + (m^{n+1/2} d_x dv, phi) - (m^{n+1/2} dv, d_x phi) = 0,
 *   dv = dt (u^n + u^{n+1})/2 + sum_q xi_q (dW^n_q + dLambda^n_q),
 * each step solved by Picard iteration until the iterate's estimated error
 * c/(1-c) |m_k - m_{k-1}| (c the ratio of the last two changes, used while
 * c < 1/2; the change itself otherwise) is at most picard_tol max|m| in the
 * max norm.  dLambda is the nudging control of
 * eq. "SCH nudge" (NULL = zero).
 *   m, u    in/out [n_particles][nx]
 *   dW      [n_particles][n_steps][n_modes]
 *   dLambda [n_particles][n_steps][n_modes] or NULL
 *   status  out [n_particles] or NULL: SCH_OK, or the code of the first step
 *           that failed (that particle then stops at that step)
 *   iters   out [n_particles] or NULL: implicit-solve iterations summed
 * ------------------------------------------------------------------------ */
int sch_ensemble_step(const sch_model *model, int32_t n_particles, int32_t n_steps, double *m,
                      double *u, const double *dW, const double *dLambda, int32_t *status,
                      int32_t *iters, void *stream);

/* --------------------------------------------------------------------------
 * Observation operator of eq. obseq: out[p][j] = P1 value of u_p at
 * x_j = j L / n_obs (cell floor(j nx / n_obs), located in integers).
 * ------------------------------------------------------------------------ */
int sch_observe(const sch_model *model, int32_t n_obs, int32_t n_particles, const double *u,
                double *out, void *stream);

/* --------------------------------------------------------------------------
 * sch_loglik: negative log of the likelihood weight of eq. loglikeq,
 *   phi[p] = 1/2 sum_j ((P u_p)_j - y_j)^2 / sigma_j^2.
 * A non-finite result is stored as +infinity (weight zero).
 * ------------------------------------------------------------------------ */
int sch_loglik(const sch_model *model, const sch_obs *obs, int32_t n_particles, const double *u,
               double *phi, void *stream);

/* --------------------------------------------------------------------------
 * sch_temper_ess: normalised weights, effective sample size (eq. ess) and the
 * adaptive tempering increment (section 3.1.2).  With s_p = logw_extra[p] -
 * beta phi[p], w[p] = exp(s_p) / sum exp(s), ESS = 1 / sum w^2.
 *   theta      device scalar in/out: temperature before / after the step
 *   n_bisect   > 0: beta = the largest increment <= 1 - theta whose ESS is
 *              >= ess_threshold, found by n_bisect halvings (if the full
 *              remainder keeps the ESS it is taken and theta becomes 1);
 *              == 0: beta = 1 - theta (no search; the bootstrap filter uses
 *              theta = 0, beta = 1 with its carried log-weights)
 *   logw_extra device [n] or NULL (zero)
 *   dtheta     device scalar out: the increment taken
 *   w          device [n] out; logw_out device [n] out or NULL: log w
 *   ess        device scalar out: ESS at the increment taken
 * n_particles <= 65536.  Runs as one workgroup.
 * ------------------------------------------------------------------------ */
int sch_temper_ess(int32_t n_particles, const double *phi, const double *logw_extra,
                   double *theta, double ess_threshold, int32_t n_bisect, double *dtheta,
                   double *w, double *logw_out, double *ess, void *stream);

/* --------------------------------------------------------------------------
 * sch_resample: systematic resampling (section 3.1.1) of normalised weights
 * w[n] with the uniform *u0 (device scalar in [0,1)), in the integer-exact
 * form: q_p = floor(w_p 2^(51 - b - e)), b = ceil(log2 n), e the binary
 * exponent of max w; C_p the inclusive prefix sums of q (exact, < 2^51);
 * T_j = ((j + u0) * C_{n-1}) / n with each operation rounded once;
 * idx[j] = min{ p : C_p > T_j } (clamped to n - 1).  Indices are therefore a
 * pure function of (w, u0), bit-identical to any correct implementation.
 *   cond_ess, cond_threshold: if cond_ess is not NULL and *cond_ess >=
 *   cond_threshold, idx becomes the identity (no resampling), evaluated on
 *   the device.
 * workspace >= sch_workspace_bytes(SCH_WS_RESAMPLE, NULL, n, 0).
 * An all-zero or non-finite weight vector makes idx the identity and sets
 * the device flag *degenerate (int32, may be NULL) to 1.
 * ------------------------------------------------------------------------ */
int sch_resample(int32_t n_particles, const double *w, const double *u0, const double *cond_ess,
                 double cond_threshold, int32_t *idx, int32_t *degenerate, void *workspace,
                 void *stream);

/* sch_gather: dst[j][:] = src[idx[j]][:] for n_rows rows of row_len doubles
 * (src and dst both [n_rows][row_len], not overlapping).  A row whose index
 * lies outside [0, n_rows) is left untouched. */
int sch_gather(int32_t n_rows, int64_t row_len, const int32_t *idx, const double *src,
               double *dst, void *stream);

/* --------------------------------------------------------------------------
 * sch_jitter_pcn: n_jitter preconditioned Crank-Nicolson MCMC moves of each
 * particle's increments at temperature *theta (section 3.1.2, jittering):
 *   dW' = rho dW + sqrt(1 - rho^2) sqrt(dt) z     (z ~ N(0,1), tag PCN,
 *         counter (p, cycle * n_steps + n, pair | tag << 24, temper_k << 16 | j))
 *   rerun the window from (m0, u0) with dW', phi' = sch_loglik of the end;
 *   accept with probability min(1, exp(theta (phi - phi'))) using the uniform
 *   of tag ACCEPT, counter (p, cycle, tag << 24, temper_k << 16 | j).
 * (The paper prints max(1, .); min is the Metropolis rule it describes.)
 * On acceptance dW, phi, m_end, u_end are replaced.  A proposal whose
 * window fails is rejected.
 * With controls (dLambda not NULL; the nudged filter, last paragraph of
 * section 3.1.3: W replaced by W~ in the tempered weights) the window runs
 * with dW' + dLambda, the controls stay fixed, and phi is the potential
 *   J = phi_obs + sum_i (dLambda_i^2 / 2 + dLambda_i dW'_i) / dt,
 * the likelihood plus minus the log of the discrete Girsanov factor.
 *   m0, u0      [n][nx] window-start state (read)
 *   dW          [n][n_steps][n_modes] in/out;  phi [n] in/out
 *   dLambda     [n][n_steps][n_modes] fixed controls (read) or NULL
 *   m_end,u_end [n][nx] in/out: window-end state of the current increments
 *   n_accept    out [n] or NULL
 *   workspace   >= sch_workspace_bytes(SCH_WS_JITTER, model, n, n_steps, n_jitter)
 * ------------------------------------------------------------------------ */
int sch_jitter_pcn(const sch_model *model, const sch_obs *obs, const sch_rng *rng,
                   int32_t n_particles, int32_t n_steps, const double *m0, const double *u0,
                   double *dW, const double *dLambda, double *phi, double *m_end, double *u_end,
                   const double *theta, double rho, int32_t n_jitter, int32_t *n_accept,
                   void *workspace, void *stream);

/* sch_jitter_pcn_noalloc: for callers that cannot allocate device memory --
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  The same moves as sch_jitter_pcn (same kernels, bit-identical
 * results) with every argument but the workspace: the proposal normals and
 * acceptance uniforms, n_jitter * n * n_steps * n_modes + n_jitter * n
 * doubles (plus 512 bytes of alignment), go to a device array of the library
 * of sch_jitter_pcn_noalloc_max_bytes() = 16 MiB, one per GPU, held until
 * the process ends (16 MiB covers 5 moves of 1024 particles x 40 steps x 8
 * modes).  Larger requests fail with SCH_E_SHAPE before any device work.  The
 * call itself allocates nothing; the array's address is looked up once per
 * device on the first call there.  Every call on a GPU uses the same array:
 * calls that overlap on one GPU (different streams, threads or processes
 * sharing a context) race and must be serialised by the caller. */
size_t sch_jitter_pcn_noalloc_max_bytes(void);
int sch_jitter_pcn_noalloc(const sch_model *model, const sch_obs *obs, const sch_rng *rng,
                           int32_t n_particles, int32_t n_steps, const double *m0,
                           const double *u0, double *dW, const double *dLambda, double *phi,
                           double *m_end, double *u_end, const double *theta, double rho,
                           int32_t n_jitter, int32_t *n_accept, void *stream);

/* --------------------------------------------------------------------------
 * Nudging (section 3.1.3).  The control dLambda^n enters each step beside
 * the increment (eq. "SCH nudge": dU^n = sum_q xi_q (dW^n_q + dLambda^n_q)),
 * and the particle's log-weight gains the log of the discrete Girsanov
 * factor (eq. "girsanov DG approx" with the control per step dLambda =
 * Lambda dt):  log G = -sum_n (|dLambda^n|^2 / 2 + dLambda^n . dW^n) / dt.
 * (This is the ratio of the N(0, dt) density of the increment to that of the
 * shifted increment; the continuous form in the paper carries the opposite
 * sign on the stochastic integral.)
 *
 * sch_nudge_grad: for every particle the objective
 *   J = phi(u^S) - log G
 * of one window of n_steps steps from (m0, u0) (phi as in sch_loglik) and its
 * gradient dJ/d(dLambda) by the discrete adjoint of the implicit-midpoint
 * steps: exact for the converged steps, including the dependence of the
 * advecting velocity on the new state through the Helmholtz relation.  The
 * forward pass keeps the state every ckpt_every steps; the reverse pass
 * recomputes each segment from its checkpoint.
 *   m0, u0   [n][nx]; dW, dLambda [n][n_steps][n_modes] or NULL (zero)
 *   J        out [n] (+infinity where a step failed)
 *   grad     out [n][n_steps][n_modes]
 *   status   out [n] or NULL: SCH_OK, or the first failure (forward or adjoint)
 *   workspace >= sch_workspace_bytes(SCH_WS_NUDGE_GRAD, model, n, n_steps,
 *               ckpt_every)
 * ------------------------------------------------------------------------ */
int sch_nudge_grad(const sch_model *model, const sch_obs *obs, int32_t n_particles,
                   int32_t n_steps, const double *m0, const double *u0, const double *dW,
                   const double *dLambda, int32_t ckpt_every, double *J, double *grad,
                   int32_t *status, void *workspace, void *stream);

/* L-BFGS settings of sch_nudge_run (host struct).  The paper optimises with
 * BFGS; the limited-memory form keeps the per-particle state small.
 *   gtol      stop when |grad|_inf <= gtol (1 + |J|)
 *   max_iter  accepted steps per stage
 *   mem       stored correction pairs, 1..16
 *   max_back  step halvings per backtracking (Armijo, c1 = 1e-4) search */
typedef struct sch_lbfgs_opts {
  double gtol;
  int32_t max_iter;
  int32_t mem;
  int32_t max_back;
} sch_lbfgs_opts;

/* sch_nudge_run: the sequential adapted nudging of section 3.1.3 over one
 * window, for every particle: for n = 0 .. n_steps-1, minimise over
 * dLambda^n the objective of the remaining steps n .. n_steps-1 with the
 * later increments and controls set to zero (phi of the window end plus
 * |dLambda^n|^2 / (2 dt)), by L-BFGS started at dLambda^n (warm_start != 0)
 * or at zero; then advance the particle one step with dW^n + dLambda^n.
 *   m, u        in/out [n][nx]: window-start state in, nudged window end out
 *   dW          [n][n_steps][n_modes]: the increments revealed stage by stage
 *   dLambda     [n][n_steps][n_modes]: warm start in (if warm_start), controls out
 *   logG        out [n]: log Girsanov factor of the realised path
 *   lbfgs_status out [n] or NULL: the largest L-BFGS status over the stages
 *               (0 converged, 1 iteration cap, 2 line search failed,
 *               3 objective failed at the starting point)
 *   iters, evals out [n] or NULL: accepted L-BFGS steps and objective
 *               evaluations summed over the stages
 *   status      out [n] or NULL: SCH_OK or the first failed advance (the
 *               particle's later stages still run from the kept state)
 *   workspace   >= sch_workspace_bytes(SCH_WS_NUDGE, model, n, n_steps,
 *                  ckpt_every)
 * Synchronises the stream after every batch of objective evaluations. */
int sch_nudge_run(const sch_model *model, const sch_obs *obs, int32_t n_particles,
                  int32_t n_steps, double *m, double *u, const double *dW, double *dLambda,
                  int32_t warm_start, const sch_lbfgs_opts *opts, int32_t ckpt_every,
                  double *logG, int32_t *lbfgs_status, int32_t *iters, int32_t *evals,
                  int32_t *status, void *workspace, void *stream);

/* --------------------------------------------------------------------------
 * Filter cycles (host-driven sequences of the calls above; they synchronise
 * the stream to read scalars back).
 *
 * sch_pf_bootstrap_cycle -- section 3.1.1: draw increments (tag FORECAST),
 * advance n_steps, multiply the carried weights by the likelihood, and
 * resample (uniform of tag RESAMPLE, counter (0, cycle, tag << 24, 0)) when
 * the ESS falls below ess_frac * n; logw [n] carries normalised log-weights
 * between cycles (zero after a resampling).
 *
 * sch_pf_tempered_cycle -- section 3.1.2: draw increments, run the window,
 * then raise the temperature from 0 to 1 in adaptive steps; after each step
 * resample the particles (window-start state, increments, phi, window-end
 * state; uniform counter (0, cycle, tag << 24, k << 16)) and apply n_jitter
 * pCN moves at the new temperature.  At most max_temper steps
 * (SCH_E_DEGENERATE beyond).  On return m, u hold the window-end states.
 *
 * In both cycles a particle whose forecast window fails (not converged or
 * non-finite) gets phi = +infinity, i.e. zero weight, and is replaced at the
 * next resampling; stats->n_failed counts such particles and the call still
 * succeeds.  SCH_E_DEGENERATE only when every weight vanishes.
 * ------------------------------------------------------------------------ */
int sch_pf_bootstrap_cycle(const sch_model *model, const sch_obs *obs, uint64_t seed,
                           uint32_t cycle, int32_t n_particles, int32_t n_steps, double ess_frac,
                           double *m, double *u, double *logw, void *workspace,
                           sch_cycle_stats *stats, void *stream);

int sch_pf_tempered_cycle(const sch_model *model, const sch_obs *obs, uint64_t seed,
                          uint32_t cycle, int32_t n_particles, int32_t n_steps,
                          double ess_threshold, int32_t n_bisect, double rho, int32_t n_jitter,
                          int32_t max_temper, double *m, double *u, void *workspace,
                          sch_cycle_stats *stats, void *stream);

/* --------------------------------------------------------------------------
 * sch_pf_nudged_cycle -- the nudged filter: section 3.1.3 followed by the
 * tempering and jittering of section 3.1.2 with W replaced by W~ = W + G
 * (last paragraph of section 3.1.3).  Draw the window's increments (tag
 * NUDGE, counter (p, cycle * n_steps + n, pair | tag << 24, 0)), nudge every
 * particle over the window (sch_nudge_run from zero controls, L-BFGS
 * settings opts, checkpoints every ckpt_every steps), give it the potential
 * J = phi(u_end) - log G, then raise the temperature from 0 to 1 in
 * adaptive steps on the weights exp(-dtheta J); after each step resample the
 * particles (window-start state, increments, controls, J, window-end state;
 * uniform as sch_pf_tempered_cycle) and apply n_jitter pCN moves of the
 * increments with the controls fixed (sch_jitter_pcn with dLambda).
 *   m, u       in/out [n][nx]: window-start ensemble in, window-end out
 *   dLambda    out [n][n_steps][n_modes]: the final particles' controls
 *   workspace  >= sch_nudged_workspace_bytes(model, n, n_steps, n_jitter,
 *              ckpt_every)
 * stats->particle_steps counts the forecast and jitter windows (not the
 * objective evaluations of the nudging); stats->picard_iters counts the
 * jitter windows' iterations.  Errors as sch_pf_tempered_cycle; a particle
 * whose nudged window fails gets J = +infinity.
 * ------------------------------------------------------------------------ */
size_t sch_nudged_workspace_bytes(const sch_model *model, int32_t n_particles, int32_t n_steps,
                                  int32_t n_jitter, int32_t ckpt_every);
int sch_pf_nudged_cycle(const sch_model *model, const sch_obs *obs, uint64_t seed,
                        uint32_t cycle, int32_t n_particles, int32_t n_steps,
                        double ess_threshold, int32_t n_bisect, double rho, int32_t n_jitter,
                        int32_t max_temper, const sch_lbfgs_opts *opts, int32_t ckpt_every,
                        double *m, double *u, double *dLambda, void *workspace,
                        sch_cycle_stats *stats, void *stream);

/* sch_pf_nudged_cycle_warm: the nudged filter with given start controls, for
 * a learned warm start of the nudging stages (an extension of section 3.1.3).
 * dLambda [n][n_steps][n_modes] holds the start controls on entry and the
 * final particles' controls on return; mode[p] (device int32 [n]) selects
 * how particle p's stages start:
 *   SCH_NUDGE_KEEP       the window runs with the given controls, no L-BFGS
 *                        steps (its log G and J follow from them)
 *   SCH_NUDGE_FROM_GIVEN each stage's L-BFGS starts from the given control
 *   SCH_NUDGE_FROM_ZERO  plain nudging from zero (the fallback)
 * Everything else as sch_pf_nudged_cycle (same workspace).  Values of mode
 * outside 0..2 are taken as FROM_ZERO. */
#define SCH_NUDGE_KEEP 0
#define SCH_NUDGE_FROM_GIVEN 1
#define SCH_NUDGE_FROM_ZERO 2
int sch_pf_nudged_cycle_warm(const sch_model *model, const sch_obs *obs, uint64_t seed,
                             uint32_t cycle, int32_t n_particles, int32_t n_steps,
                             double ess_threshold, int32_t n_bisect, double rho, int32_t n_jitter,
                             int32_t max_temper, const sch_lbfgs_opts *opts, int32_t ckpt_every,
                             double *m, double *u, double *dLambda, const int32_t *mode,
                             void *workspace, sch_cycle_stats *stats, void *stream);

/* --------------------------------------------------------------------------
 * Gradient-based jitter: preconditioned Crank-Nicolson Langevin moves (pCNL;
 * Cotter, Roberts, Stuart & White, Statist. Sci. 2013), the function-space
 * form of the MALA sampler that the paper names as future work (section 5).
 * For each particle, with x its increments [n_steps][n_modes] (prior
 * N(0, dt I)) and the target exp(-theta phi(x)) N(x; 0, dt I):
 *   v = rho x + sqrt(1 - rho^2) sqrt(dt) z - (1 - rho) dt theta grad phi(x),
 * z and the acceptance uniform drawn exactly as sch_jitter_pcn's, accepted
 * with probability min(1, pi(v) q(v -> x) / (pi(x) q(x -> v))), q the
 * Gaussian density N(rho x - (1 - rho) dt theta grad phi(x), (1 - rho^2) dt I).
 * phi and grad phi come from the discrete adjoint of sch_nudge_grad (one
 * forward + reverse pass per proposal and one at the start; checkpoints every
 * ckpt_every steps).  The drift helps while (1 - rho) dt theta |Hessian of
 * phi| stays below about 1; beyond that the proposals overshoot.
 *   rho in [0, 1);  dW, phi in/out as sch_jitter_pcn (no controls);
 *   m_end, u_end out: the window ends of the final increments (recomputed)
 *   workspace >= sch_pcnl_workspace_bytes(SCH_WS_JITTER, model, n, n_steps,
 *                n_jitter, ckpt_every)
 * sch_pf_tempered_cycle_pcnl: sch_pf_tempered_cycle with these moves
 * (workspace: SCH_WS_TEMPERED); stats->particle_steps counts the forward
 * windows (n_steps each: the gradient at the start, one per proposal and the
 * end-state rerun per tempering step), not the reverse passes.
 * ------------------------------------------------------------------------ */
size_t sch_pcnl_workspace_bytes(int32_t which, const sch_model *model, int32_t n_particles,
                                int32_t n_steps, int32_t n_jitter, int32_t ckpt_every);
int sch_jitter_pcnl(const sch_model *model, const sch_obs *obs, const sch_rng *rng,
                    int32_t n_particles, int32_t n_steps, const double *m0, const double *u0,
                    double *dW, double *phi, double *m_end, double *u_end, const double *theta,
                    double rho, int32_t n_jitter, int32_t ckpt_every, int32_t *n_accept,
                    void *workspace, void *stream);
int sch_pf_tempered_cycle_pcnl(const sch_model *model, const sch_obs *obs, uint64_t seed,
                               uint32_t cycle, int32_t n_particles, int32_t n_steps,
                               double ess_threshold, int32_t n_bisect, double rho,
                               int32_t n_jitter, int32_t max_temper, int32_t ckpt_every,
                               double *m, double *u, void *workspace, sch_cycle_stats *stats,
                               void *stream);

/* --------------------------------------------------------------------------
 * Gradient-based jitter: Hybrid Monte Carlo moves, the second sampler the
 * paper names as future work (section 5), in the function-space form of
 * Beskos, Pinski, Sanz-Serna & Stuart (Stoch. Proc. Appl. 2011).  For each
 * particle, with x its increments [n_steps][n_modes] (prior N(0, dt I)) and
 * the target exp(-theta phi(x)) N(x; 0, dt I): a velocity v = sqrt(dt) z (the
 * normals sch_jitter_pcn draws for the move), then n_leap leapfrog steps of
 * angle h of H(x, v) = theta phi(x) + (|x|^2 + |v|^2) / (2 dt), each a half
 * kick v -= (h/2) dt theta grad phi(x), the rotation
 * (x, v) -> (cos h x + sin h v, -sin h x + cos h v) and a half kick, and the
 * Metropolis test with probability min(1, exp(H(x, v) - H(x', v'))) (the
 * acceptance uniform as sch_jitter_pcn's).  phi and grad phi come from the
 * discrete adjoint of sch_nudge_grad: one forward + reverse pass at the start
 * and n_leap per move (checkpoints every ckpt_every steps).  A trajectory
 * that meets a failed window is rejected.
 *   h in (0, pi), n_leap in 1..64 (else SCH_E_ARG); dW, phi in/out as
 *   sch_jitter_pcn (no controls); m_end, u_end out: the window ends of the
 *   final increments (recomputed)
 *   workspace >= sch_hmc_workspace_bytes(SCH_WS_JITTER, model, n, n_steps,
 *                n_jitter, ckpt_every)
 * sch_pf_tempered_cycle_hmc: sch_pf_tempered_cycle with these moves
 * (workspace: SCH_WS_TEMPERED); stats->particle_steps counts the forward
 * windows (the gradient at the start, n_leap per move and the end-state rerun
 * per tempering step), not the reverse passes.
 * ------------------------------------------------------------------------ */
size_t sch_hmc_workspace_bytes(int32_t which, const sch_model *model, int32_t n_particles,
                               int32_t n_steps, int32_t n_jitter, int32_t ckpt_every);
int sch_jitter_hmc(const sch_model *model, const sch_obs *obs, const sch_rng *rng,
                   int32_t n_particles, int32_t n_steps, const double *m0, const double *u0,
                   double *dW, double *phi, double *m_end, double *u_end, const double *theta,
                   double h, int32_t n_leap, int32_t n_jitter, int32_t ckpt_every,
                   int32_t *n_accept, void *workspace, void *stream);
int sch_pf_tempered_cycle_hmc(const sch_model *model, const sch_obs *obs, uint64_t seed,
                              uint32_t cycle, int32_t n_particles, int32_t n_steps,
                              double ess_threshold, int32_t n_bisect, double h, int32_t n_leap,
                              int32_t n_jitter, int32_t max_temper, int32_t ckpt_every,
                              double *m, double *u, void *workspace, sch_cycle_stats *stats,
                              void *stream);

/* --------------------------------------------------------------------------
 * Matern-type noise (section 2, eqs. noise_solve and noise_solve2), the
 * paper's own noise in place of the modes form.  Per step the space-time
 * white noise is its DG0 approximation: one increment Delta W_i ~ N(0, dt)
 * per cell i = [x_i, x_{i+1}] (cell i beside node i), Delta W_h =
 * sum_i h^{-1/2} 1_{cell i} Delta W_i.  The step's noise Delta U is the P1
 * field U_k of k elliptic solves:
 *   (M + kappa^{-2} K) U_1 = eta b,   b_i = (Delta W_h, phi_i)
 *                                         = sqrt(h) (Delta W_{i-1} + Delta W_i) / 2,
 *   (M + kappa^{-2} K) U_j = M U_{j-1},   j = 2..k,
 * and enters eq. fde1 as dv = dt (u^n + u^{n+1})/2 + Delta U.  The paper
 * takes eta = 1 and k = 3 and leaves kappa open.
 *   kappa  > 0 (kappa h = sqrt(6), where the operator is diagonal, is
 *          rejected);  k in 1..16
 * Errors: SCH_E_ARG for a bad sch_matern, else as the modes-form calls.
 * ------------------------------------------------------------------------ */
typedef struct sch_matern {
  double kappa; /* inverse correlation length of the field  */
  double eta;   /* amplitude                                */
  int32_t k;    /* number of elliptic solves (smoothness)   */
} sch_matern;

/* Delta U of n rows of cell increments: dWc, dU [n][nx] (n <= 65535). */
int sch_matern_field(const sch_model *model, const sch_matern *mt, int32_t n_particles,
                     const double *dWc, double *dU, void *stream);

/* sch_ensemble_step with the Matern-type noise: dWc [n][n_steps][nx] holds
 * the cell increments of every step; m, u, status, iters as sch_ensemble_step
 * (model->xi is not read). */
int sch_ensemble_step_matern(const sch_model *model, const sch_matern *mt, int32_t n_particles,
                             int32_t n_steps, double *m, double *u, const double *dWc,
                             int32_t *status, int32_t *iters, void *stream);

/* Workspace of the Matern-noise calls: which = SCH_WS_JITTER, SCH_WS_TEMPERED
 * or SCH_WS_BOOTSTRAP with extra = n_jitter, SCH_WS_NUDGE_GRAD or SCH_WS_NUDGE
 * with extra = ckpt_every (0 for anything else or invalid sizes). */
size_t sch_matern_workspace_bytes(int32_t which, const sch_model *model, int32_t n_particles,
                                  int32_t n_steps, int32_t extra);

/* sch_jitter_pcn on the cell increments dWc [n][n_steps][nx]: the same pCN
 * proposal per cell (the cells 2k, 2k+1 of a step share one Philox block:
 * tag PCN, counter (p, cycle * n_steps + n, k | tag << 24,
 * temper_k << 16 | j)), the same acceptance uniform, window and likelihood.
 * No controls (sch_jitter_pcn_matern_ctrl takes them).  workspace >=
 * sch_matern_workspace_bytes(SCH_WS_JITTER, ...). */
int sch_jitter_pcn_matern(const sch_model *model, const sch_matern *mt, const sch_obs *obs,
                          const sch_rng *rng, int32_t n_particles, int32_t n_steps,
                          const double *m0, const double *u0, double *dWc, double *phi,
                          double *m_end, double *u_end, const double *theta, double rho,
                          int32_t n_jitter, int32_t *n_accept, void *workspace, void *stream);

/* sch_nudge_grad with the Matern-type noise (section 3.1.3 with the noise of
 * section 2): the controls are per cell, so dWc, dLambdac and grad are
 * [n][n_steps][nx]; each step's noise is the field of the cells dWc + dLambdac,
 * the gradient with respect to the cells is the transpose of the field map
 * applied to dJ/d(Delta U), and J carries the Girsanov term summed over the
 * cells.  workspace >= sch_matern_workspace_bytes(SCH_WS_NUDGE_GRAD, model, n,
 * n_steps, ckpt_every).  Errors as sch_nudge_grad, plus SCH_E_ARG for a bad
 * sch_matern. */
int sch_nudge_grad_matern(const sch_model *model, const sch_matern *mt, const sch_obs *obs,
                          int32_t n_particles, int32_t n_steps, const double *m0,
                          const double *u0, const double *dWc, const double *dLambdac,
                          int32_t ckpt_every, double *J, double *grad, int32_t *status,
                          void *workspace, void *stream);

/* sch_nudge_run with the Matern-type noise: the stage-wise nudging over one
 * window with one control per cell (nx per stage); dWc and dLambdac are
 * [n][n_steps][nx], the other arguments as sch_nudge_run.  workspace >=
 * sch_matern_workspace_bytes(SCH_WS_NUDGE, model, n, n_steps, ckpt_every).
 * The L-BFGS state holds mem correction pairs of nx values per particle. */
int sch_nudge_run_matern(const sch_model *model, const sch_matern *mt, const sch_obs *obs,
                         int32_t n_particles, int32_t n_steps, double *m, double *u,
                         const double *dWc, double *dLambdac, int32_t warm_start,
                         const sch_lbfgs_opts *opts, int32_t ckpt_every, double *logG,
                         int32_t *lbfgs_status, int32_t *iters, int32_t *evals,
                         int32_t *status, void *workspace, void *stream);

/* sch_jitter_pcn_matern with per-cell controls dLambdac [n][n_steps][nx]
 * held fixed (the jittering of the nudged filter, section 3.1.3): the window
 * runs with the cells dWc' + dLambdac and J (in/out) is the nudged potential
 * phi + sum over the cells of (dLambda^2 / 2 + dLambda dW') / dt.  Proposals,
 * uniforms and workspace as sch_jitter_pcn_matern.  SCH_E_ARG without
 * dLambdac. */
int sch_jitter_pcn_matern_ctrl(const sch_model *model, const sch_matern *mt, const sch_obs *obs,
                               const sch_rng *rng, int32_t n_particles, int32_t n_steps,
                               const double *m0, const double *u0, double *dWc,
                               const double *dLambdac, double *J, double *m_end, double *u_end,
                               const double *theta, double rho, int32_t n_jitter,
                               int32_t *n_accept, void *workspace, void *stream);

/* sch_pf_bootstrap_cycle with the Matern-type noise: cell increments drawn as
 * sch_draw_increments with nx values per step (tag FORECAST), the Matern
 * window, likelihood weights and conditional resampling as
 * sch_pf_bootstrap_cycle.  workspace >=
 * sch_matern_workspace_bytes(SCH_WS_BOOTSTRAP, model, n, n_steps, 0). */
int sch_pf_bootstrap_cycle_matern(const sch_model *model, const sch_matern *mt,
                                  const sch_obs *obs, uint64_t seed, uint32_t cycle,
                                  int32_t n_particles, int32_t n_steps, double ess_frac,
                                  double *m, double *u, double *logw, void *workspace,
                                  sch_cycle_stats *stats, void *stream);

/* sch_pf_tempered_cycle with the Matern-type noise: the window's cell
 * increments are drawn as sch_draw_increments with nx values per step (tag
 * FORECAST), the tempering, resampling and jittering as sch_pf_tempered_cycle
 * with sch_jitter_pcn_matern.  workspace >=
 * sch_matern_workspace_bytes(SCH_WS_TEMPERED, model, n, n_steps, n_jitter). */
int sch_pf_tempered_cycle_matern(const sch_model *model, const sch_matern *mt,
                                 const sch_obs *obs, uint64_t seed, uint32_t cycle,
                                 int32_t n_particles, int32_t n_steps, double ess_threshold,
                                 int32_t n_bisect, double rho, int32_t n_jitter,
                                 int32_t max_temper, double *m, double *u, void *workspace,
                                 sch_cycle_stats *stats, void *stream);

/* sch_pf_nudged_cycle with the Matern-type noise (section 3.1.3 with the
 * noise of section 2): the NUDGE-tag cell increments (nx per step), the
 * stage-wise nudging of sch_nudge_run_matern from zero controls, tempering on
 * J = phi - log G (the Girsanov term summed over the cells), resampling, and
 * pCN moves of the cells with the per-cell controls held fixed (the window
 * runs with the cells dW' + dLambda).  dLambdac out [n][n_steps][nx]: the
 * resampled controls.  workspace >= sch_nudged_workspace_bytes_matern(model,
 * n, n_steps, n_jitter, ckpt_every).  Errors as sch_pf_nudged_cycle, plus
 * SCH_E_ARG for a bad sch_matern. */
size_t sch_nudged_workspace_bytes_matern(const sch_model *model, int32_t n_particles,
                                         int32_t n_steps, int32_t n_jitter, int32_t ckpt_every);
int sch_pf_nudged_cycle_matern(const sch_model *model, const sch_matern *mt, const sch_obs *obs,
                               uint64_t seed, uint32_t cycle, int32_t n_particles,
                               int32_t n_steps, double ess_threshold, int32_t n_bisect,
                               double rho, int32_t n_jitter, int32_t max_temper,
                               const sch_lbfgs_opts *opts, int32_t ckpt_every, double *m,
                               double *u, double *dLambdac, void *workspace,
                               sch_cycle_stats *stats, void *stream);

/* --------------------------------------------------------------------------
 * The paper's twin experiments (section 4).
 *
 * sch_paper_init -- the initial ensemble of eq. init_solve: per particle p,
 * DG0 cell values W_i = sqrt(h) z_i ~ N(0, h) (tag INIT, counter
 * (p, 0, pair | tag << 24, 0), cells 2k and 2k + 1 sharing a block), then
 * U^{0,1} solves (I - d_xx) U = |W| in the P1 weak form ((M + K) U_1 = b,
 * b_i = h (|W_{i-1}| + |W_i|) / 2) and U^{0,j+1} = (M + K)^{-1} M U^{0,j} for
 * j = 1, 2; with (alpha, beta) the two normals of counter (p, 1, tag << 24, 0)
 * the velocity is u_p = alpha^2 U^{0,3} + beta^2.  The truth is drawn the same
 * way (the experiments give it its own seed).
 *   u  out [n][nx]; the momenta follow from sch_init_momentum.
 *
 * sch_ensemble_stats -- the statistics of section 4 of the ensemble u [n][nx]
 * against the truth ua [nx], with the nodal Euclidean norm |.|:
 *   out[0] EMRE = (1/n) sum_p |ua - u_p| / |ua|
 *   out[1] RB   = |ua - mean_p u_p| / |ua|
 *   out[2] RES  = (1/(n-1)) sum_p |u_p - mean_p u_p| / |ua|   (0 for n = 1)
 *   workspace  device, at least (nx + 2 n) doubles;  out device [3].
 * Experiment 2 observes half the domain: give the unobserved points of the
 * observation grid sigma = +inf (they then add nothing to any likelihood).
 * ------------------------------------------------------------------------ */
int sch_paper_init(const sch_model *model, uint64_t seed, int32_t n_particles, double *u,
                   void *stream);
int sch_ensemble_stats(int32_t n_particles, int32_t nx, const double *u, const double *ua,
                       double *workspace, double *out, void *stream);

/* --------------------------------------------------------------------------
 * Batched runner: many independent bootstrap filters (sch_pf_bootstrap_cycle
 * semantics, section 3.1.1) of uneven grid and ensemble sizes advanced one
 * assimilation cycle at a time for all of them together.  The forecast of
 * every particle of every instance runs in one persistent kernel per tile
 * class, whose workgroups take (instance, particle) items from a queue,
 * longest first; likelihood, weights, conditional resampling and gathers are
 * batched over instances; all decisions are taken on the device, so a cycle
 * is captured once into a HIP graph and replayed.
 *
 * sch_instance (host struct, one per instance; all arrays device memory the
 * caller keeps alive while the batch exists):
 *   nx, n_particles   grid nodes (64..8192) and particles (1..65536)
 *   xi                [n_modes][nx] noise modes
 *   m, u              in/out [n_particles][nx] ensemble state
 *   logw              in/out [n_particles] normalised log-weights (zero after
 *                     a resampling; start with zeros)
 *   y                 [cycles][n_obs]: row c holds the observations of cycle c
 *   sigma             [n_obs]
 *   seed              generator key of the instance (increments, resampling)
 *   threads           threads per particle (power of two 64..512; 0 = the
 *                     default choice of the model calls, or SCH_TUNE_THREADS)
 * sch_batch_params: physics and filter settings shared by all instances.
 *
 * sch_batch_create lays the batch out in the caller's workspace (at least
 * sch_batch_workspace_bytes) and returns an opaque handle (host memory owned
 * by the library until sch_batch_destroy).  sch_batch_run advances n_cycles
 * cycles, cycle0 .. cycle0 + n_cycles - 1 (the cycle number selects the
 * observation row and the generator counters); with use_graph != 0 the cycle
 * is captured into a HIP graph on first use (on a stream the library creates)
 * and replayed on `stream`; use_graph = 0 enqueues the same kernels directly.
 * sch_batch_read synchronises `stream` and copies
 * per-instance results to host arrays (each may be NULL): the ESS of the last
 * cycle, the number of resamplings since creation, and the first failure of
 * any particle (SCH_OK if none); picard_iters receives the implicit-solve
 * iterations summed since creation.  Calls on one batch must not overlap.
 * ------------------------------------------------------------------------ */
typedef struct sch_instance {
  int32_t nx;
  int32_t n_particles;
  const double *xi;
  double *m;
  double *u;
  double *logw;
  const double *y;
  const double *sigma;
  uint64_t seed;
  int32_t threads;
} sch_instance;

typedef struct sch_batch_params {
  double L, alpha, mu, dt;
  int32_t n_modes;    /* 1..64                                     */
  int32_t n_steps;    /* steps per assimilation window             */
  int32_t n_obs;      /* observation points per instance           */
  double ess_frac;    /* resample when ESS < ess_frac * n_particles */
  double picard_tol;
  int32_t picard_max;
} sch_batch_params;

typedef struct sch_batch sch_batch;

size_t sch_batch_workspace_bytes(const sch_batch_params *params, int32_t n_instances,
                                 const sch_instance *instances);
int sch_batch_create(const sch_batch_params *params, int32_t n_instances,
                     const sch_instance *instances, void *workspace, size_t workspace_bytes,
                     sch_batch **out, void *stream);
int sch_batch_run(sch_batch *batch, uint32_t cycle0, int32_t n_cycles, int32_t use_graph,
                  void *stream);
int sch_batch_read(sch_batch *batch, double *ess, int32_t *resampled, int32_t *status,
                   int64_t *picard_iters, void *stream);
int sch_batch_destroy(sch_batch *batch);

/* --------------------------------------------------------------------------
 * Learned nudging warm start.  A perceptron n_in -> n_hidden -> n_hidden ->
 * n_out with ReLU activations maps a particle's window-start features to the
 * nudging controls of the window; its prediction seeds the L-BFGS stages of
 * sch_nudge_run (warm_start = 1), and a particle whose observation misfit is
 * larger than a threshold calibrated on the training data starts from zero
 * (plain nudging) instead.  Mixed precision on the matrix cores: bfloat16
 * operands (features, weights, activations, back-propagated errors; round to
 * nearest even), float32 accumulation, float32 master weights, biases,
 * gradients and Adam state.  (No passage of the paper: an extension of its
 * nudging step, section 3.1.3.)
 *
 * sch_mlp (host struct):
 *   n_in, n_hidden, n_out   layer sizes
 *   params        device float32 [sch_mlp_param_count]: W1 [H][F], b1 [H],
 *                 W2 [H][H], b2 [H], W3 [O][H], b3 [O] (row-major, out x in)
 *   weights_bf16  device bf16 bits [H F + H H + O H]: W1 | W2 | W3, refreshed
 *                 by sch_mlp_sync and sch_mlp_adam
 * sch_mlp_forward: Y [batch][n_out] (float32) from X [batch][n_in] (bf16
 *   bits); keeps the activations in the workspace
 *   (>= sch_mlp_workspace_bytes(net, batch)).
 * sch_mlp_backward: after sch_mlp_forward on the same X and workspace, the
 *   mean-squared error of Y against T [batch][n_out] (device double *loss,
 *   averaged over all batch x n_out values) and its gradient grad (device
 *   float32, parameter layout).
 * sch_mlp_adam: one Adam step (Kingma & Ba) at step >= 1 on params with the
 *   moments m, v (device float32, parameter layout), then refreshes the
 *   bfloat16 weights.
 * sch_mlp_features: per particle, the misfit y - P u (n_obs values) followed
 *   by u (nx values); X = bf16((x - mean) / sdev) if X is given, raw float32
 *   values into raw and the misfit norm |y - P u|_2 into misfit if given.
 * sch_mlp_encode: X = bf16((raw - mean) / sdev) for stored raw features
 *   [n][cols] (the scaling of sch_mlp_features).
 * sch_mlp_colstats: column means and deviations of A [rows][cols] (float32;
 *   a deviation below 1e-12 is replaced by 1).
 * sch_mlp_targets: T = (dLambda - mean) / sdev as float32 (plain float32 copy
 *   when mean is NULL); dLambda is [n][cols] double.
 * sch_mlp_controls: dLambda = Y sdev + mean as double, or 0 for particles with
 *   misfit[p] > threshold (misfit may be NULL: no fallback); mode (device
 *   int32 [n], or NULL) receives each particle's start mode for
 *   sch_pf_nudged_cycle_warm: keep_mode (SCH_NUDGE_KEEP or
 *   SCH_NUDGE_FROM_GIVEN) where the prediction is used, SCH_NUDGE_FROM_ZERO
 *   (plain nudging) where the misfit is above the threshold.
 * ------------------------------------------------------------------------ */
typedef struct sch_mlp {
  int32_t n_in;
  int32_t n_hidden;
  int32_t n_out;
  float *params;
  uint16_t *weights_bf16;
} sch_mlp;

size_t sch_mlp_param_count(int32_t n_in, int32_t n_hidden, int32_t n_out);
size_t sch_mlp_workspace_bytes(const sch_mlp *net, int32_t batch);
int sch_mlp_sync(const sch_mlp *net, void *stream);
int sch_mlp_forward(const sch_mlp *net, int32_t batch, const uint16_t *X, float *Y,
                    void *workspace, void *stream);
int sch_mlp_backward(const sch_mlp *net, int32_t batch, const uint16_t *X, const float *Y,
                     const float *T, double *loss, float *grad, void *workspace, void *stream);
int sch_mlp_adam(const sch_mlp *net, const float *grad, float *m, float *v, int32_t step,
                 float lr, float beta1, float beta2, float eps, void *stream);
int sch_mlp_features(const sch_model *model, const sch_obs *obs, int32_t n_particles,
                     const double *u, const float *mean, const float *sdev, uint16_t *X,
                     float *raw, double *misfit, void *stream);
int sch_mlp_encode(int32_t n, int32_t cols, const float *raw, const float *mean,
                   const float *sdev, uint16_t *X, void *stream);
int sch_mlp_colstats(int32_t rows, int32_t cols, const float *A, float *mean, float *sdev,
                     void *stream);
int sch_mlp_targets(int32_t n, int32_t cols, const double *dLambda, const float *mean,
                    const float *sdev, float *T, void *stream);
int sch_mlp_controls(int32_t n, int32_t cols, const float *Y, const float *mean,
                     const float *sdev, const double *misfit, double threshold,
                     double *dLambda, int32_t *mode, int32_t keep_mode, void *stream);

/* --------------------------------------------------------------------------
 * Tuning knobs (process-global).  SCH_TUNE_THREADS forces the threads per
 * particle of the model kernels (a power of two in 64..512; 0 = automatic:
 * the smallest power of two giving at most 8 nodes per thread).  A value
 * that leaves more than 16 nodes per thread, or fewer than one, makes the
 * model calls return SCH_E_SHAPE.  sch_tune_get returns the current value
 * (-1 for an unknown key).
 * ------------------------------------------------------------------------ */
#define SCH_TUNE_THREADS 2
int sch_tune_set(int32_t key, int32_t value);
int sch_tune_get(int32_t key);

/* --------------------------------------------------------------------------
 * Kernel timing for benchmarks.  While enabled (on != 0), the cycle drivers
 * bracket every launch with HIP events on the launch stream and, at their
 * synchronisation points, accumulate the elapsed time per kernel class.
 * sch_timing_read copies the totals: ms[k], launches[k] and iters[k] (the
 * implicit-solve iterations done by that class, where it has them) for
 * k < SCH_TK_COUNT; sch_timing_reset zeroes them.  Process-global, not
 * thread-safe: meant for one benchmarking thread.
 * ------------------------------------------------------------------------ */
#define SCH_TK_WINDOW 0   /* forecast window kernel          */
#define SCH_TK_JITTER 1   /* fused pCN jitter kernel         */
#define SCH_TK_TEMPER 2   /* weights / ESS / tempering       */
#define SCH_TK_RESAMPLE 3 /* systematic resampling           */
#define SCH_TK_GATHER 4   /* particle copies after resampling */
#define SCH_TK_OTHER 5    /* likelihood, draws, fills        */
#define SCH_TK_NUDGE 6    /* nudging objective + adjoint     */
#define SCH_TK_ADJOINT 7  /* adjoint evaluations of the gradient-based jitter
                           * (inside SCH_TK_JITTER's time); iters: their
                           * transposed fixed-point iterations, while the
                           * Picard iterations of their forward sweeps are
                           * counted with SCH_TK_JITTER's */
#define SCH_TK_COUNT 8
int sch_timing_enable(int on);
int sch_timing_reset(void);
int sch_timing_read(double *ms, int64_t *launches, int64_t *iters);

#ifdef __cplusplus
}
#endif
#endif /* SCH_H */
