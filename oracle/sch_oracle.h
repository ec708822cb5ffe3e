/*
 * sch_oracle.h -- plain, slow, FP64 CPU oracle for the stochastic Camassa-Holm
 * (SALT) particle filter of Cotter, Crisan & Singh (arXiv 2402.06927).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this code: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no source with the GPU library.
 *
 * Every function follows a passage of the paper (cited by section and
 * equation label) or the textbook definition of the operation.  Where the
 * paper is silent or garbled the reading taken is stated next to the code.
 *
 * Conventions: row-major, particle-major arrays ([particle][node]), node i at
 * x_i = i*h on the periodic interval [0, L), h = L/nx.  All floating point is
 * IEEE binary64; the library is compiled with -ffp-contract=off.
 */
#ifndef SCH_ORACLE_H
#define SCH_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes (same meaning as the product library's, own values) ---- */
enum {
  ORC_OK = 0,
  ORC_E_ARG = -1,
  ORC_E_SINGULAR = -2,
  ORC_E_NONCONVERGED = -3,
  ORC_E_NONFINITE = -4,
  ORC_E_DEGENERATE = -5
};

/* ---- counter-based RNG: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11) ---- */
void orc_philox4x32_10(const uint32_t ctr[4], uint64_t seed, uint32_t out[4]);
double orc_u01(uint32_t hi, uint32_t lo);
void orc_normal_pair(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                     double z[2]);
double orc_uniform(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3);

/* Stage tags placed in bits 24..31 of counter word 2. */
enum {
  ORC_TAG_INIT = 0,
  ORC_TAG_FORECAST = 1,
  ORC_TAG_PCN = 2,
  ORC_TAG_ACCEPT = 3,
  ORC_TAG_RESAMPLE = 4,
  ORC_TAG_OBS = 5,
  ORC_TAG_NUDGE = 6
};

/* dW[p][n][q] = sqrt(dt) * z for particle p, global step (step0 + n), mode q,
 * drawn with the given tag and word-3 value (temper k << 16 | jitter j). */
void orc_draw_increments_rows(uint64_t seed, int32_t p0, int32_t n_particles, int32_t n_steps,
                              int32_t n_modes, uint32_t step0, uint32_t tag, uint32_t word3,
                              double dt, double *dW);
void orc_draw_increments(uint64_t seed, int32_t n_particles, int32_t n_steps, int32_t n_modes,
                         uint32_t step0, uint32_t tag, uint32_t word3, double dt, double *dW);

/* ---- model description ---- */
typedef struct orc_model {
  double L, alpha, mu, dt;
  int32_t nx, n_modes;
  const double *xi; /* [n_modes][nx] nodal values of the noise modes */
  double picard_tol;
  int32_t picard_max;
} orc_model;

/* ---- dense / banded linear algebra ---- */
int orc_dense_solve(int32_t n, const double *A, const double *b, double *x);
int orc_tridiag_pivot_solve(int32_t n, int32_t nrhs, const double *dl, const double *d,
                            const double *du, double *b);
int orc_cyclic_solve(int32_t n, const double *a, const double *b, const double *c,
                     const double *d, double *x);

/* ---- P1 operators on the periodic mesh ---- */
void orc_apply_mass(int32_t nx, double h, const double *f, double *out);
void orc_apply_stiff(int32_t nx, double h, const double *f, double *out);
void orc_apply_advect(int32_t nx, const double *v, const double *f, double *out);
int orc_velocity_from_momentum(const orc_model *md, const double *m, double *u);
int orc_momentum_from_velocity(const orc_model *md, const double *u, double *m);

/* ---- one implicit-midpoint step and windows ---- */
int orc_step(const orc_model *md, double *m, double *u, const double *dW, const double *dLam,
             int32_t *iters);
int orc_window(const orc_model *md, int32_t n_steps, double *m, double *u, const double *dW,
               const double *dLam, int32_t *iters);
int orc_ensemble_window(const orc_model *md, int32_t n_particles, int32_t n_steps, double *m,
                        double *u, const double *dW, const double *dLam, int32_t *status,
                        int32_t *iters, int32_t n_threads);

int orc_step_field(const orc_model *md, double *m, double *u, const double *dU,
                   int32_t *iters);

/* ---- Matern-type noise on the DG0 white noise (k elliptic solves) ---- */
typedef struct orc_matern {
  double kappa, eta;
  int32_t k;
} orc_matern;
int orc_matern_field(int32_t nx, double L, const orc_matern *mt, const double *dWc, double *dU);
int orc_step_matern(const orc_model *md, const orc_matern *mt, double *m, double *u,
                    const double *dWc, int32_t *iters);
int orc_window_matern(const orc_model *md, const orc_matern *mt, int32_t n_steps, double *m,
                      double *u, const double *dWc, int32_t *iters);
int orc_ensemble_window_matern(const orc_model *md, const orc_matern *mt, int32_t n_particles,
                               int32_t n_steps, double *m, double *u, const double *dWc,
                               int32_t *status, int32_t *iters, int32_t n_threads);

/* ---- observations and likelihood ---- */
void orc_observe(int32_t nx, int32_t n_obs, const double *u, double *out);
double orc_nll(int32_t nx, int32_t n_obs, const double *u, const double *y, const double *sigma);
void orc_ensemble_nll(int32_t nx, int32_t n_obs, int32_t n_particles, const double *u,
                      const double *y, const double *sigma, double *phi);

/* ---- weights, ESS, tempering ---- */
double orc_weights(int32_t n, const double *phi, const double *logw_extra, double beta,
                   double *w, double *logw_out);
int orc_temper(int32_t n, const double *phi, double theta, double threshold, int32_t n_bisect,
               double *dtheta, double *w, double *ess);

/* ---- systematic resampling ---- */
int orc_resample_systematic(int32_t n, const double *w, double u0, int32_t *idx);
int orc_resample_textbook(int32_t n, const double *w, double u0, int32_t *idx);

/* ---- pCN jittering ---- */
typedef struct orc_rng {
  uint64_t seed;
  uint32_t cycle, temper_k;
} orc_rng;

void orc_pcn_propose(uint64_t seed, uint32_t particle, uint32_t step0, int32_t n_steps,
                     int32_t n_modes, uint32_t word3, double rho, double dt, const double *cur,
                     double *prop);
int orc_pcn_accept(double theta, double phi_old, double phi_new, double v);
int64_t orc_pcn_linear_chain(uint64_t seed, int32_t n_steps, int32_t n_modes, int32_t n_obs,
                             const double *G, const double *y, double sigma, double theta,
                             double rho, double dt, int32_t n_iter, const double *x0,
                             double *samples);
int orc_jitter_pcn(const orc_model *md, int32_t n_obs, const double *y, const double *sigma,
                   const orc_rng *rng, int32_t n_particles, int32_t n_steps, const double *m0,
                   const double *u0, double *dW, double *phi, double *m_end, double *u_end,
                   double theta, double rho, int32_t n_jitter, int32_t *n_accept,
                   int32_t n_threads);

double orc_nudged_potential(double phi, int32_t len, double dt, const double *dW,
                            const double *dLam);
int orc_jitter_pcn_ctrl(const orc_model *md, int32_t n_obs, const double *y, const double *sigma,
                        const orc_rng *rng, int32_t n_particles, int32_t n_steps,
                        const double *m0, const double *u0, double *dW, const double *dLam,
                        double *phi, double *m_end, double *u_end, double theta, double rho,
                        int32_t n_jitter, int32_t *n_accept, int32_t n_threads);
int64_t orc_pcn_linear_chain_ctrl(uint64_t seed, int32_t n_steps, int32_t n_modes, int32_t n_obs,
                                  const double *G, const double *y, double sigma, double theta,
                                  double rho, double dt, const double *lam, int32_t n_iter,
                                  const double *x0, double *samples);

/* ---- filter cycles ---- */
typedef struct orc_cycle_stats {
  double ess;          /* ESS before resampling (bootstrap) / after last step */
  int32_t resampled;   /* bootstrap: 1 if resampled this cycle */
  int32_t n_temper;    /* tempering steps taken */
  int64_t picard_iters;/* total Picard iterations over the cycle */
  int64_t n_accept;    /* pCN acceptances over the cycle */
  int32_t status;
} orc_cycle_stats;

int orc_bootstrap_cycle(const orc_model *md, int32_t n_obs, const double *y, const double *sigma,
                        uint64_t seed, uint32_t cycle, int32_t n_particles, int32_t n_steps,
                        double ess_frac, double *m, double *u, double *logw,
                        orc_cycle_stats *st, int32_t n_threads);

int orc_tempered_cycle(const orc_model *md, int32_t n_obs, const double *y, const double *sigma,
                       uint64_t seed, uint32_t cycle, int32_t n_particles, int32_t n_steps,
                       double ess_threshold, int32_t n_bisect, double rho, int32_t n_jitter,
                       int32_t max_temper, double *m, double *u, orc_cycle_stats *st,
                       int32_t n_threads);

/* Pin of the tempering loop shared by the tempered drivers (section 3.1.2),
 * with the forward window replaced by a linear-Gaussian plug-in: the window
 * of a particle maps its start state s [ds] and increments xi
 * [n_steps][n_modes] (prior N(0, dt) each, drawn as the SCH forecast) to the
 * end state e = F s + B xi (F [ds][ds], B [ds][n_steps * n_modes]) and its
 * potential is Phi = |G e - y|^2 / (2 sigma^2) (G [n_obs][ds]).  The forecast,
 * the tempering steps, the resampling, the gathers and the pCN jitter (its
 * proposal, counters and acceptance rule) are those of orc_tempered_cycle.
 * x [n][ds] holds the start states on entry and the end states on return.
 * With these Gaussian ingredients the end states after the cycle sample the
 * Kalman filter's posterior, which the tests compare against.
 * `plant` plants a known mistake for the tests' power checks:
 * ORC_PLANT_JITTER_PRE_THETA jitters at the temperature before the step,
 * ORC_PLANT_CUMULATIVE_WEIGHTS resamples with exp(-theta_new Phi) instead of
 * exp(-dtheta Phi). */
enum { ORC_PLANT_NONE = 0, ORC_PLANT_JITTER_PRE_THETA = 1, ORC_PLANT_CUMULATIVE_WEIGHTS = 2,
       ORC_PLANT_HMC_NO_KINETIC = 3 };
int orc_tempered_cycle_linear(int32_t ds, int32_t n_steps, int32_t n_modes, int32_t n_obs,
                              const double *F, const double *B, const double *G, const double *y,
                              double sigma, double dt, uint64_t seed, uint32_t cycle,
                              int32_t n_particles, double ess_threshold, int32_t n_bisect,
                              double rho, int32_t n_jitter, int32_t max_temper, double *x,
                              orc_cycle_stats *st, int32_t plant);

/* ---- nudging objective and its gradient ---- */
int orc_nudge_objective(const orc_model *md, int32_t n_obs, const double *y, const double *sigma,
                        int32_t n_steps, const double *m0, const double *u0, const double *dW,
                        const double *dLam, double *J);
int orc_nudge_grad(const orc_model *md, int32_t n_obs, const double *y, const double *sigma,
                   int32_t n_steps, const double *m0, const double *u0, const double *dW,
                   const double *dLam, double *J, double *grad);
int orc_nudge_grad_tangent(const orc_model *md, int32_t n_obs, const double *y,
                           const double *sigma, int32_t n_steps, const double *m0,
                           const double *u0, const double *dW, const double *dLam,
                           double *grad);

/* ---- L-BFGS and the sequential adapted nudging scheme ---- */
typedef int (*orc_objective)(void *ctx, const double *x, double *f, double *g);
typedef struct {
  double gtol;      /* stop at |g|_inf <= gtol (1 + |f|) */
  int32_t max_iter; /* accepted steps per stage */
  int32_t mem;      /* stored pairs */
  int32_t max_back; /* halvings per line search */
} orc_lbfgs_opts;
int orc_lbfgs(int32_t n, orc_objective fn, void *ctx, double *x, double h0, double gtol,
              int32_t max_iter, int32_t mem, int32_t max_back, double *f_out, int32_t *iters,
              int32_t *evals);
int orc_nudge_particle(const orc_model *md, int32_t n_obs, const double *y, const double *sigma,
                       int32_t n_steps, double *m, double *u, const double *dW, double *dLam,
                       const orc_lbfgs_opts *opt, double *logG, int32_t *iters_total,
                       int32_t *evals_total, int32_t *worst_status);
int orc_nudge_ensemble(const orc_model *md, int32_t n_obs, const double *y, const double *sigma,
                       int32_t n_particles, int32_t n_steps, double *m, double *u, const double *dW,
                       double *dLam, const orc_lbfgs_opts *opt, double *logG, int32_t *iters,
                       int32_t *evals, int32_t *lbfgs_status, int32_t *status, int32_t n_threads);

/* ---- nudged filter: nudging, then tempering and jittering with W~ ---- */
int orc_nudged_cycle(const orc_model *md, int32_t n_obs, const double *y, const double *sigma,
                     uint64_t seed, uint32_t cycle, int32_t n_particles, int32_t n_steps,
                     double ess_threshold, int32_t n_bisect, double rho, int32_t n_jitter,
                     int32_t max_temper, const orc_lbfgs_opts *opt, double *m, double *u,
                     double *m0_out, double *u0_out, double *dW_out, double *dLam_out,
                     double *J_out, orc_cycle_stats *st, int32_t n_threads);

/* The nudged filter with given start controls (the learned warm start of the
 * nudging stages): dLam_start [n][n_steps][n_modes] and, per particle,
 * mode[p] = ORC_NUDGE_KEEP (the window runs with the given controls, no
 * L-BFGS steps), ORC_NUDGE_FROM_GIVEN (the stages' L-BFGS starts from them)
 * or ORC_NUDGE_FROM_ZERO (plain nudging from zero, the fallback).  Otherwise
 * orc_nudged_cycle (which is this call with every particle FROM_ZERO). */
enum { ORC_NUDGE_KEEP = 0, ORC_NUDGE_FROM_GIVEN = 1, ORC_NUDGE_FROM_ZERO = 2 };
int orc_nudged_cycle_warm(const orc_model *md, int32_t n_obs, const double *y,
                          const double *sigma, uint64_t seed, uint32_t cycle, int32_t n_particles,
                          int32_t n_steps, double ess_threshold, int32_t n_bisect, double rho,
                          int32_t n_jitter, int32_t max_temper, const orc_lbfgs_opts *opt,
                          const double *dLam_start, const int32_t *mode, double *m, double *u,
                          double *m0_out, double *u0_out, double *dW_out, double *dLam_out,
                          double *J_out, orc_cycle_stats *st, int32_t n_threads);

/* ---- nudging with the Matern-type noise (controls per cell) ---- */
int orc_matern_transpose(int32_t nx, double L, const orc_matern *mt, const double *g,
                         double *out);
int orc_nudge_grad_matern(const orc_model *md, const orc_matern *mt, int32_t n_obs,
                          const double *y, const double *sigma, int32_t n_steps,
                          const double *m0, const double *u0, const double *dW,
                          const double *dLam, double *J, double *grad);
int orc_nudge_ensemble_matern(const orc_model *md, const orc_matern *mt, int32_t n_obs,
                              const double *y, const double *sigma, int32_t n_particles,
                              int32_t n_steps, double *m, double *u, const double *dW,
                              double *dLam, const orc_lbfgs_opts *opt, double *logG,
                              int32_t *iters, int32_t *evals, int32_t *lbfgs_status,
                              int32_t *status, int32_t n_threads);

/* ---- bootstrap and tempered + jittered filters with the Matern-type noise ---- */
int orc_bootstrap_cycle_matern(const orc_model *md, const orc_matern *mt, int32_t n_obs,
                               const double *y, const double *sigma, uint64_t seed,
                               uint32_t cycle, int32_t n_particles, int32_t n_steps,
                               double ess_frac, double *m, double *u, double *logw,
                               orc_cycle_stats *st, int32_t n_threads);
int orc_jitter_pcn_matern(const orc_model *md, const orc_matern *mt, int32_t n_obs,
                          const double *y, const double *sigma, const orc_rng *rng,
                          int32_t n_particles, int32_t n_steps, const double *m0,
                          const double *u0, double *dWc, double *phi, double *m_end,
                          double *u_end, double theta, double rho, int32_t n_jitter,
                          int32_t *n_accept, int32_t n_threads);

/* orc_jitter_pcn_matern with the per-cell controls dLamc fixed (the nudged
 * filter): the window runs with dWc' + dLamc and J (in/out) is the nudged
 * potential. */
int orc_jitter_pcn_matern_ctrl(const orc_model *md, const orc_matern *mt, int32_t n_obs,
                               const double *y, const double *sigma, const orc_rng *rng,
                               int32_t n_particles, int32_t n_steps, const double *m0,
                               const double *u0, double *dWc, const double *dLamc, double *J,
                               double *m_end, double *u_end, double theta, double rho,
                               int32_t n_jitter, int32_t *n_accept, int32_t n_threads);

/* orc_nudged_cycle with the Matern-type noise: increments and controls per
 * cell, [n][n_steps][nx]. */
int orc_nudged_cycle_matern(const orc_model *md, const orc_matern *mt, int32_t n_obs,
                            const double *y, const double *sigma, uint64_t seed, uint32_t cycle,
                            int32_t n_particles, int32_t n_steps, double ess_threshold,
                            int32_t n_bisect, double rho, int32_t n_jitter, int32_t max_temper,
                            const orc_lbfgs_opts *opt, double *m, double *u, double *m0_out,
                            double *u0_out, double *dW_out, double *dLam_out, double *J_out,
                            orc_cycle_stats *st, int32_t n_threads);
int orc_tempered_cycle_matern(const orc_model *md, const orc_matern *mt, int32_t n_obs,
                              const double *y, const double *sigma, uint64_t seed, uint32_t cycle,
                              int32_t n_particles, int32_t n_steps, double ess_threshold,
                              int32_t n_bisect, double rho, int32_t n_jitter, int32_t max_temper,
                              double *m, double *u, double *m0_out, double *u0_out,
                              double *dWc_out, double *phi_out, orc_cycle_stats *st,
                              int32_t n_threads);

/* ---- gradient-based jitter (pCN Langevin) ---- */
double orc_pcnl_log_ratio(int32_t d, const double *x, double phi_x, const double *g_x,
                          const double *v, double phi_v, const double *g_v, double theta,
                          double rho, double dt);
int64_t orc_pcnl_linear_chain(uint64_t seed, int32_t n_steps, int32_t n_modes, int32_t n_obs,
                              const double *G, const double *y, double sigma, double theta,
                              double rho, double dt, int32_t n_iter, const double *x0,
                              double *samples);
int orc_jitter_pcnl(const orc_model *md, int32_t n_obs, const double *y, const double *sigma,
                    const orc_rng *rng, int32_t n_particles, int32_t n_steps, const double *m0,
                    const double *u0, double *dW, double *phi, double *m_end, double *u_end,
                    double theta, double rho, int32_t n_jitter, int32_t *n_accept,
                    int32_t n_threads);

int orc_tempered_cycle_pcnl(const orc_model *md, int32_t n_obs, const double *y,
                            const double *sigma, uint64_t seed, uint32_t cycle,
                            int32_t n_particles, int32_t n_steps, double ess_threshold,
                            int32_t n_bisect, double rho, int32_t n_jitter, int32_t max_temper,
                            double *m, double *u, orc_cycle_stats *st, int32_t n_threads);

/* ---- gradient-based jitter (Hybrid Monte Carlo on the increments) ----
 * Per move: velocity v ~ N(0, dt I) (the pCN normals sqrt(dt) z of the move),
 * n_leap leapfrog steps of angle h of the Hamiltonian
 * H(x, v) = theta Phi(x) + (|x|^2 + |v|^2) / (2 dt), split as half kicks
 * v -= (h/2) dt theta grad Phi(x) around the exact rotation of the Gaussian
 * part (x, v) -> (cos h x + sin h v, -sin h x + cos h v); accepted with
 * probability min(1, exp(H(x0, v0) - H(xL, vL))).
 * orc_hmc_trajectory_linear: the n_leap steps alone for the linear-Gaussian
 * toy Phi(x) = |G x - y|^2 / (2 sigma^2) (x, v in/out).
 * orc_hmc_linear_chain: n_iter moves of that toy (as orc_pcnl_linear_chain);
 * plant ORC_PLANT_HMC_NO_KINETIC (for tests only) leaves the velocities'
 * energy out of the Metropolis ratio, a mistake that changes the target. */
void orc_hmc_trajectory_linear(int32_t d, int32_t n_obs, const double *G, const double *y,
                               double sigma, double theta, double h, int32_t n_leap, double dt,
                               double *x, double *v);
int64_t orc_hmc_linear_chain(uint64_t seed, int32_t n_steps, int32_t n_modes, int32_t n_obs,
                             const double *G, const double *y, double sigma, double theta,
                             double h, int32_t n_leap, double dt, int32_t n_iter,
                             const double *x0, double *samples, int32_t plant);
int orc_jitter_hmc(const orc_model *md, int32_t n_obs, const double *y, const double *sigma,
                   const orc_rng *rng, int32_t n_particles, int32_t n_steps, const double *m0,
                   const double *u0, double *dW, double *phi, double *m_end, double *u_end,
                   double theta, double h, int32_t n_leap, int32_t n_jitter, int32_t *n_accept,
                   int32_t n_threads);
int orc_tempered_cycle_hmc(const orc_model *md, int32_t n_obs, const double *y,
                           const double *sigma, uint64_t seed, uint32_t cycle,
                           int32_t n_particles, int32_t n_steps, double ess_threshold,
                           int32_t n_bisect, double h, int32_t n_leap, int32_t n_jitter,
                           int32_t max_temper, double *m, double *u, orc_cycle_stats *st,
                           int32_t n_threads);

/* ---- the paper's twin experiments: initialisation and statistics ---- */
int orc_paper_init_from(int32_t nx, double L, const double *W, double alpha, double beta,
                        double *u);
int orc_paper_init(int32_t nx, double L, uint64_t seed, int32_t p0, int32_t n, double *u);
void orc_ensemble_stats(int32_t n, int32_t nx, const double *u, const double *ua, double *out);

#ifdef __cplusplus
}
#endif
#endif
