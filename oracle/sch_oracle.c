/*
 * sch_oracle.c -- plain FP64 CPU oracle for the stochastic Camassa-Holm (SALT)
 * particle filter of Cotter, Crisan & Singh, "Data assimilation for the
 * stochastic Camassa-Holm equation using particle filtering: a numerical
 * investigation" (arXiv 2402.06927).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline of the benchmark, never by the product path.  It shares no code
 * with the GPU library.  Written for clarity, not speed: every array is
 * allocated per call, every solve is a pivoted direct solve, and each step
 * follows the equation it cites.
 *
 * Compiled with -O2 -ffp-contract=off (no fused multiply-add contraction),
 * so the arithmetic is exactly the IEEE operations written here.
 */
#include "sch_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ========================================================================== */
/* Counter-based RNG.                                                          */
/* Philox4x32-10 as published by Salmon, Moraes, Dror & Shaw ("Parallel random */
/* numbers: as easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 bit       */
/* multiplications with the multipliers 0xD2511F53 and 0xCD9E8D57, the high    */
/* halves xor-ed with the other counter words and the round key, the key       */
/* bumped between rounds by the Weyl constants 0x9E3779B9 and 0xBB67AE85.      */
/* The paper itself only fixes the prior of the increments, N(0, dt) per       */
/* entry (section 3.1.2, jittering); the generator is a choice of this build.  */
/* ========================================================================== */

void orc_philox4x32_10(const uint32_t ctr[4], uint64_t seed, uint32_t out[4]) {
  uint32_t key0 = (uint32_t)(seed & 0xffffffffu);
  uint32_t key1 = (uint32_t)(seed >> 32);
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      key0 += 0x9E3779B9u;
      key1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x1 ^ key0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ key1;
    uint32_t y3 = lo0;
    x0 = y0;
    x1 = y1;
    x2 = y2;
    x3 = y3;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

/* The top 53 bits of the 64-bit word (hi:lo), scaled by 2^-53: an exact
 * double in [0, 1). */
double orc_u01(uint32_t hi, uint32_t lo) {
  uint64_t w = ((uint64_t)hi << 32) | (uint64_t)lo;
  return (double)(w >> 11) * (1.0 / 9007199254740992.0);
}

/* Box-Muller: two uniforms u1, u2 from one Philox block; 1 - u1 lies in
 * (0, 1], so the logarithm is finite. */
void orc_normal_pair(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                     double z[2]) {
  uint32_t ctr[4] = {c0, c1, c2, c3}, r[4];
  orc_philox4x32_10(ctr, seed, r);
  double u1 = orc_u01(r[0], r[1]);
  double u2 = orc_u01(r[2], r[3]);
  double rad = sqrt(-2.0 * log(1.0 - u1));
  double ang = 6.283185307179586 * u2;
  z[0] = rad * cos(ang);
  z[1] = rad * sin(ang);
}

double orc_uniform(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3) {
  uint32_t ctr[4] = {c0, c1, c2, c3}, r[4];
  orc_philox4x32_10(ctr, seed, r);
  return orc_u01(r[0], r[1]);
}

/* Brownian increments: iid N(0, dt) per (step, mode) (section 3.1.2:
 * "prior distribution is iid N(0, dt)").  Counter: (particle, global step,
 * mode pair | tag << 24, word3).  Modes 2k and 2k+1 take the pair's z0, z1. */
/* Rows p0 .. p0 + n_particles - 1 of the draw (row p of dW is particle p0 + p). */
void orc_draw_increments_rows(uint64_t seed, int32_t p0, int32_t n_particles, int32_t n_steps,
                              int32_t n_modes, uint32_t step0, uint32_t tag, uint32_t word3,
                              double dt, double *dW) {
  double sdt = sqrt(dt);
  int32_t n_pairs = (n_modes + 1) / 2;
  for (int32_t p = 0; p < n_particles; ++p)
    for (int32_t n = 0; n < n_steps; ++n)
      for (int32_t k = 0; k < n_pairs; ++k) {
        double z[2];
        orc_normal_pair(seed, (uint32_t)(p0 + p), step0 + (uint32_t)n, (uint32_t)k | (tag << 24),
                        word3, z);
        double *row = dW + ((int64_t)p * n_steps + n) * n_modes;
        row[2 * k] = sdt * z[0];
        if (2 * k + 1 < n_modes) row[2 * k + 1] = sdt * z[1];
      }
}

void orc_draw_increments(uint64_t seed, int32_t n_particles, int32_t n_steps, int32_t n_modes,
                         uint32_t step0, uint32_t tag, uint32_t word3, double dt, double *dW) {
  orc_draw_increments_rows(seed, 0, n_particles, n_steps, n_modes, step0, tag, word3, dt, dW);
}

/* ========================================================================== */
/* Linear algebra.                                                             */
/* ========================================================================== */

/* Dense LU with partial pivoting (textbook Gaussian elimination). */
int orc_dense_solve(int32_t n, const double *A, const double *b, double *x) {
  double *M = (double *)malloc(sizeof(double) * (size_t)n * n);
  double *r = (double *)malloc(sizeof(double) * (size_t)n);
  memcpy(M, A, sizeof(double) * (size_t)n * n);
  memcpy(r, b, sizeof(double) * (size_t)n);
  int st = ORC_OK;
  for (int32_t k = 0; k < n && st == ORC_OK; ++k) {
    int32_t piv = k;
    for (int32_t i = k + 1; i < n; ++i)
      if (fabs(M[(size_t)i * n + k]) > fabs(M[(size_t)piv * n + k])) piv = i;
    if (M[(size_t)piv * n + k] == 0.0) {
      st = ORC_E_SINGULAR;
      break;
    }
    if (piv != k) {
      for (int32_t j = 0; j < n; ++j) {
        double t = M[(size_t)k * n + j];
        M[(size_t)k * n + j] = M[(size_t)piv * n + j];
        M[(size_t)piv * n + j] = t;
      }
      double t = r[k];
      r[k] = r[piv];
      r[piv] = t;
    }
    for (int32_t i = k + 1; i < n; ++i) {
      double l = M[(size_t)i * n + k] / M[(size_t)k * n + k];
      if (l == 0.0) continue;
      for (int32_t j = k; j < n; ++j) M[(size_t)i * n + j] -= l * M[(size_t)k * n + j];
      r[i] -= l * r[k];
    }
  }
  if (st == ORC_OK) {
    for (int32_t i = n - 1; i >= 0; --i) {
      double s = r[i];
      for (int32_t j = i + 1; j < n; ++j) s -= M[(size_t)i * n + j] * x[j];
      x[i] = s / M[(size_t)i * n + i];
    }
  }
  free(M);
  free(r);
  return st;
}

/* Tridiagonal Gaussian elimination with partial pivoting (row interchanges),
 * the textbook algorithm behind LAPACK's gtsv.  dl[i] = A[i+1][i],
 * d[i] = A[i][i], du[i] = A[i][i+1].  b is [nrhs][n] and is overwritten with
 * the solution.  Row swaps create fill in a second superdiagonal du2. */
int orc_tridiag_pivot_solve(int32_t n, int32_t nrhs, const double *dl_in, const double *d_in,
                            const double *du_in, double *b) {
  if (n < 1) return ORC_E_ARG;
  double *dl = (double *)malloc(sizeof(double) * (size_t)(n > 1 ? n - 1 : 1));
  double *d = (double *)malloc(sizeof(double) * (size_t)n);
  double *du = (double *)malloc(sizeof(double) * (size_t)(n > 1 ? n - 1 : 1));
  double *du2 = (double *)calloc((size_t)(n > 2 ? n - 2 : 1), sizeof(double));
  memcpy(d, d_in, sizeof(double) * (size_t)n);
  if (n > 1) {
    memcpy(dl, dl_in, sizeof(double) * (size_t)(n - 1));
    memcpy(du, du_in, sizeof(double) * (size_t)(n - 1));
  }
  int st = ORC_OK;
  for (int32_t i = 0; i + 1 < n; ++i) {
    if (fabs(d[i]) >= fabs(dl[i])) {
      /* no interchange: eliminate A[i+1][i] with row i */
      if (d[i] == 0.0) {
        st = ORC_E_SINGULAR;
        break;
      }
      double l = dl[i] / d[i];
      d[i + 1] -= l * du[i];
      for (int32_t r = 0; r < nrhs; ++r) b[(size_t)r * n + i + 1] -= l * b[(size_t)r * n + i];
      if (i + 2 < n) du2[i] = 0.0;
    } else {
      /* interchange rows i and i+1; the old row i+1 becomes the pivot row */
      double l = d[i] / dl[i];
      double old_d1 = d[i + 1];
      d[i] = dl[i];
      d[i + 1] = du[i] - l * old_d1;
      du[i] = old_d1;
      if (i + 2 < n) {
        du2[i] = du[i + 1];
        du[i + 1] = -l * du2[i];
      }
      for (int32_t r = 0; r < nrhs; ++r) {
        double bi = b[(size_t)r * n + i], bi1 = b[(size_t)r * n + i + 1];
        b[(size_t)r * n + i] = bi1;
        b[(size_t)r * n + i + 1] = bi - l * bi1;
      }
    }
  }
  if (st == ORC_OK && d[n - 1] == 0.0) st = ORC_E_SINGULAR;
  if (st == ORC_OK) {
    for (int32_t r = 0; r < nrhs; ++r) {
      double *x = b + (size_t)r * n;
      x[n - 1] = x[n - 1] / d[n - 1];
      if (n > 1) x[n - 2] = (x[n - 2] - du[n - 2] * x[n - 1]) / d[n - 2];
      for (int32_t i = n - 3; i >= 0; --i)
        x[i] = (x[i] - du[i] * x[i + 1] - du2[i] * x[i + 2]) / d[i];
    }
  }
  free(dl);
  free(d);
  free(du);
  free(du2);
  return st;
}

/* Cyclic (periodic) tridiagonal system
 *     a[i] x[i-1] + b[i] x[i] + c[i] x[i+1] = d[i],  indices mod n,  n >= 3,
 * solved by bordering: the first n-1 unknowns form a plain tridiagonal block
 * T, x[n-1] is the border.  Solve T y = d', T z = (border column), then
 * x[n-1] from the Schur complement and x' = y - z x[n-1]. */
int orc_cyclic_solve(int32_t n, const double *a, const double *b, const double *c,
                     const double *d, double *x) {
  if (n < 3) return ORC_E_ARG;
  int32_t m = n - 1;
  double *dl = (double *)malloc(sizeof(double) * (size_t)m);
  double *dd = (double *)malloc(sizeof(double) * (size_t)m);
  double *du = (double *)malloc(sizeof(double) * (size_t)m);
  double *rhs = (double *)calloc((size_t)2 * m, sizeof(double));
  for (int32_t i = 0; i < m; ++i) {
    dd[i] = b[i];
    if (i + 1 < m) {
      dl[i] = a[i + 1];
      du[i] = c[i];
    }
    rhs[i] = d[i];
  }
  /* border column: row 0 couples to x[-1] = x[n-1] via a[0]; row n-2 couples
   * to x[n-1] via c[n-2] */
  rhs[m + 0] += a[0];
  rhs[m + m - 1] += c[m - 1];
  int st = orc_tridiag_pivot_solve(m, 2, dl, dd, du, rhs);
  if (st == ORC_OK) {
    const double *y = rhs, *z = rhs + m;
    /* border row n-1: a[n-1] x[n-2] + b[n-1] x[n-1] + c[n-1] x[0] = d[n-1] */
    double num = d[n - 1] - a[n - 1] * y[m - 1] - c[n - 1] * y[0];
    double den = b[n - 1] - a[n - 1] * z[m - 1] - c[n - 1] * z[0];
    if (den == 0.0) {
      st = ORC_E_SINGULAR;
    } else {
      double xl = num / den;
      for (int32_t i = 0; i < m; ++i) x[i] = y[i] - z[i] * xl;
      x[n - 1] = xl;
    }
  }
  free(dl);
  free(dd);
  free(du);
  free(rhs);
  return st;
}

/* ========================================================================== */
/* P1 finite elements on the uniform periodic mesh (section 2: V_h is the      */
/* continuous piecewise-linear space on N cells of width h = L/N).  Each       */
/* operator is the exact integral of the P1 basis functions:                   */
/*   mass       (phi_j, phi_i)        -> h/6 * (1, 4, 1)                       */
/*   stiffness  (phi_j', phi_i')      -> 1/h * (-1, 2, -1)                     */
/*   advection  (f v_x, phi_i) - (f v, phi_i')  for P1 f, v (eq. sde1 / fde1)  */
/* ========================================================================== */

static inline int32_t wrap(int32_t i, int32_t n) { return (i % n + n) % n; }

void orc_apply_mass(int32_t nx, double h, const double *f, double *out) {
  for (int32_t i = 0; i < nx; ++i)
    out[i] = h / 6.0 * f[wrap(i - 1, nx)] + 2.0 * h / 3.0 * f[i] + h / 6.0 * f[wrap(i + 1, nx)];
}

void orc_apply_stiff(int32_t nx, double h, const double *f, double *out) {
  for (int32_t i = 0; i < nx; ++i)
    out[i] = (-f[wrap(i - 1, nx)] + 2.0 * f[i] - f[wrap(i + 1, nx)]) / h;
}

/* Row i of the advective form b(f, phi_i; v) = (f d_x v, phi_i) - (f v, d_x phi_i)
 * integrated exactly over the two cells touching node i:
 *   cell [x_i, x_{i+1}] contributes  v_{i+1} (f_i + f_{i+1}) / 2
 *   cell [x_{i-1}, x_i] contributes -v_{i-1} (f_{i-1} + f_i) / 2
 * (the h factors of the quadrature and of the derivatives cancel). */
void orc_apply_advect(int32_t nx, const double *v, const double *f, double *out) {
  for (int32_t i = 0; i < nx; ++i) {
    int32_t im = wrap(i - 1, nx), ip = wrap(i + 1, nx);
    out[i] = 0.5 * v[ip] * (f[i] + f[ip]) - 0.5 * v[im] * (f[im] + f[i]);
  }
}

/* Helmholtz relation, first line of eq. fde1:
 *   (u, psi) + alpha^2 (u_x, psi_x) = (m, psi)  for all psi  <=>  (M + alpha^2 K) u = M m. */
int orc_velocity_from_momentum(const orc_model *md, const double *m, double *u) {
  int32_t n = md->nx;
  double h = md->L / n, a2 = md->alpha * md->alpha;
  double *lo = (double *)malloc(sizeof(double) * n), *di = (double *)malloc(sizeof(double) * n);
  double *up = (double *)malloc(sizeof(double) * n), *r = (double *)malloc(sizeof(double) * n);
  for (int32_t i = 0; i < n; ++i) {
    lo[i] = h / 6.0 + a2 * (-1.0 / h);
    di[i] = 2.0 * h / 3.0 + a2 * (2.0 / h);
    up[i] = h / 6.0 + a2 * (-1.0 / h);
  }
  orc_apply_mass(n, h, m, r);
  int st = orc_cyclic_solve(n, lo, di, up, r, u);
  free(lo);
  free(di);
  free(up);
  free(r);
  return st;
}

/* Initial momentum from the initial velocity (section 2, eq. CHe1: m = u -
 * alpha^2 u_xx), in the weak form M m = (M + alpha^2 K) u so that the
 * Helmholtz relation holds exactly for the discrete pair (m, u). */
int orc_momentum_from_velocity(const orc_model *md, const double *u, double *m) {
  int32_t n = md->nx;
  double h = md->L / n, a2 = md->alpha * md->alpha;
  double *lo = (double *)malloc(sizeof(double) * n), *di = (double *)malloc(sizeof(double) * n);
  double *up = (double *)malloc(sizeof(double) * n), *r = (double *)malloc(sizeof(double) * n);
  double *k = (double *)malloc(sizeof(double) * n);
  orc_apply_mass(n, h, u, r);
  orc_apply_stiff(n, h, u, k);
  for (int32_t i = 0; i < n; ++i) {
    r[i] += a2 * k[i];
    lo[i] = h / 6.0;
    di[i] = 2.0 * h / 3.0;
    up[i] = h / 6.0;
  }
  int st = orc_cyclic_solve(n, lo, di, up, r, m);
  free(lo);
  free(di);
  free(up);
  free(r);
  free(k);
  return st;
}

/* ========================================================================== */
/* One implicit-midpoint step, eq. fde1:                                       */
/*   (m^{n+1} - m^n, phi) + mu dt (d_x m^{n+1/2}, d_x phi)                     */
/*     + (m^{n+1/2} d_x dv, phi) - (m^{n+1/2} dv, d_x phi) = 0,                */
/*   dv = dt u^{n+1/2} + dU^n,   H u^{n+1} = M m^{n+1},                        */
/* with the noise in the modes form dU = sum_q xi_q (dW_q + dLambda_q)         */
/* (section 2, the expansion used in earlier SALT work; the nudging control    */
/* enters beside the Brownian increment as in eq. "SCH nudge").                */
/* In matrix form, with A = M + (mu dt/2) K + (1/2) C(dv):                     */
/*   A m^{n+1} = (M - (mu dt/2) K - (1/2) C(dv)) m^n.                          */
/* dv depends on u^{n+1}, so the system is nonlinear.  The paper does not say  */
/* how it is solved; this oracle uses Picard iteration on u^{n+1} (each        */
/* iterate a pivoted linear solve) until the momentum iterate changes by at   */
/* most picard_tol relative in the max norm (reading G5).                      */
/* ========================================================================== */
/* One implicit-midpoint step driven by the nodal noise increment dU (the
 * step's Delta U in dv = dt (u^n + u^{n+1}) / 2 + Delta U, eq. fde1). */
int orc_step_field(const orc_model *md, double *m, double *u, const double *dU,
                   int32_t *iters) {
  int32_t n = md->nx;
  double h = md->L / n, dt = md->dt, mu = md->mu;
  size_t sz = sizeof(double) * (size_t)n;
  double *dv = (double *)malloc(sz), *lo = (double *)malloc(sz), *di = (double *)malloc(sz);
  double *up = (double *)malloc(sz), *rhs = (double *)malloc(sz), *t1 = (double *)malloc(sz);
  double *ms = (double *)malloc(sz), *us = (double *)malloc(sz), *mp = (double *)malloc(sz);

  memcpy(us, u, sz);
  memcpy(mp, m, sz);
  int st = ORC_E_NONCONVERGED;
  int32_t k;
  for (k = 1; k <= md->picard_max; ++k) {
    for (int32_t i = 0; i < n; ++i) dv[i] = dt * 0.5 * (u[i] + us[i]) + dU[i];
    /* rows of A: mass (h/6, 2h/3, h/6) + (mu dt/2) stiffness (-1/h, 2/h, -1/h)
     * + 1/2 advection (-v_{i-1}/2, (v_{i+1}-v_{i-1})/2, v_{i+1}/2) */
    for (int32_t i = 0; i < n; ++i) {
      double vm = dv[wrap(i - 1, n)], vp = dv[wrap(i + 1, n)];
      lo[i] = h / 6.0 + 0.5 * mu * dt * (-1.0 / h) + 0.5 * (-0.5 * vm);
      di[i] = 2.0 * h / 3.0 + 0.5 * mu * dt * (2.0 / h) + 0.5 * (0.5 * vp - 0.5 * vm);
      up[i] = h / 6.0 + 0.5 * mu * dt * (-1.0 / h) + 0.5 * (0.5 * vp);
    }
    /* right-hand side (M - (mu dt/2) K - (1/2) C(dv)) m^n */
    orc_apply_mass(n, h, m, rhs);
    orc_apply_stiff(n, h, m, t1);
    for (int32_t i = 0; i < n; ++i) rhs[i] -= 0.5 * mu * dt * t1[i];
    orc_apply_advect(n, dv, m, t1);
    for (int32_t i = 0; i < n; ++i) rhs[i] -= 0.5 * t1[i];

    int ls = orc_cyclic_solve(n, lo, di, up, rhs, ms);
    if (ls != ORC_OK) {
      st = ls;
      break;
    }
    ls = orc_velocity_from_momentum(md, ms, us);
    if (ls != ORC_OK) {
      st = ls;
      break;
    }
    double diff = 0.0, scale = 0.0;
    int finite = 1;
    for (int32_t i = 0; i < n; ++i) {
      if (!isfinite(ms[i]) || !isfinite(us[i])) finite = 0;
      double dd = fabs(ms[i] - mp[i]);
      if (dd > diff) diff = dd;
      if (fabs(ms[i]) > scale) scale = fabs(ms[i]);
    }
    if (!finite) {
      st = ORC_E_NONFINITE;
      break;
    }
    memcpy(mp, ms, sz);
    /* Stop once the change of the momentum iterate is within tolerance
     * (reading G5 as stated: |m_k - m_{k-1}|_inf <= tol |m_k|_inf).  For a
     * contraction with ratio c the iterate's error is then at most
     * c / (1 - c) tol |m_k|, below tol |m_k| whenever c < 1/2. */
    if (diff <= md->picard_tol * scale) {
      st = ORC_OK;
      break;
    }
  }
  if (iters) *iters = k > md->picard_max ? md->picard_max : k;
  if (st == ORC_OK || st == ORC_E_NONCONVERGED) {
    memcpy(m, ms, sz);
    memcpy(u, us, sz);
  }
  free(dv);
  free(lo);
  free(di);
  free(up);
  free(rhs);
  free(t1);
  free(ms);
  free(us);
  free(mp);
  return st;
}

/* The step with the noise of the modes form: Delta U = sum_q xi_q (dW_q + dLam_q). */
int orc_step(const orc_model *md, double *m, double *u, const double *dW, const double *dLam,
             int32_t *iters) {
  int32_t n = md->nx;
  double *dU = (double *)calloc((size_t)n, sizeof(double));
  for (int32_t q = 0; q < md->n_modes; ++q) {
    double inc = dW[q] + (dLam ? dLam[q] : 0.0);
    for (int32_t i = 0; i < n; ++i) dU[i] += md->xi[(size_t)q * n + i] * inc;
  }
  int st = orc_step_field(md, m, u, dU, iters);
  free(dU);
  return st;
}

/* n_steps consecutive steps; dW and dLam are [n_steps][n_modes]. */
int orc_window(const orc_model *md, int32_t n_steps, double *m, double *u, const double *dW,
               const double *dLam, int32_t *iters) {
  int32_t total = 0;
  for (int32_t s = 0; s < n_steps; ++s) {
    int32_t it = 0;
    int st = orc_step(md, m, u, dW + (size_t)s * md->n_modes,
                      dLam ? dLam + (size_t)s * md->n_modes : NULL, &it);
    total += it;
    if (st != ORC_OK) {
      if (iters) *iters = total;
      return st;
    }
  }
  if (iters) *iters = total;
  return ORC_OK;
}

int orc_ensemble_window(const orc_model *md, int32_t n_particles, int32_t n_steps, double *m,
                        double *u, const double *dW, const double *dLam, int32_t *status,
                        int32_t *iters, int32_t n_threads) {
  int worst = ORC_OK;
  int32_t nx = md->nx, nq = md->n_modes;
#pragma omp parallel for num_threads(n_threads > 0 ? n_threads : 1) schedule(dynamic, 1)
  for (int32_t p = 0; p < n_particles; ++p) {
    int32_t it = 0;
    int st = orc_window(md, n_steps, m + (size_t)p * nx, u + (size_t)p * nx,
                        dW + (size_t)p * n_steps * nq,
                        dLam ? dLam + (size_t)p * n_steps * nq : NULL, &it);
    if (status) status[p] = st;
    if (iters) iters[p] = it;
    if (st != ORC_OK) {
#pragma omp critical
      worst = st;
    }
  }
  return worst;
}

/* ========================================================================== */
/* Matern-type noise (section 2, eqs. noise_solve and noise_solve2): the       */
/* increment of the space-time white noise over a step is piecewise constant,  */
/* Delta W_h = sum_i h^{-1/2} 1_{cell i} Delta W_i with Delta W_i ~ N(0, dt)    */
/* iid per cell (cell i = [x_i, x_{i+1}]), and Delta U = Delta U_k solves       */
/*   (Delta U_j, v) + kappa^{-2} (grad Delta U_j, grad v)                       */
/*       = eta (Delta W_h, v)  (j = 1),   (Delta U_{j-1}, v)  (j > 1)          */
/* for all P1 test functions v: (M + kappa^{-2} K) U_1 = eta b with the load    */
/* vector b_n = (Delta W_h, phi_n) = sqrt(h) (Delta W_{n-1} + Delta W_n) / 2,  */
/* then (M + kappa^{-2} K) U_j = M U_{j-1}.                                     */
/* ========================================================================== */
int orc_matern_field(int32_t nx, double L, const orc_matern *mt, const double *dWc, double *dU) {
  double h = L / nx, ik2 = 1.0 / (mt->kappa * mt->kappa);
  size_t sz = sizeof(double) * (size_t)nx;
  double *a = (double *)malloc(sz), *b = (double *)malloc(sz), *c = (double *)malloc(sz);
  double *rhs = (double *)malloc(sz);
  for (int32_t i = 0; i < nx; ++i) {
    a[i] = h / 6.0 - ik2 / h;
    b[i] = 2.0 * h / 3.0 + 2.0 * ik2 / h;
    c[i] = h / 6.0 - ik2 / h;
    rhs[i] = mt->eta * sqrt(h) * 0.5 * (dWc[wrap(i - 1, nx)] + dWc[i]);
  }
  int st = ORC_OK;
  for (int32_t j = 1; j <= mt->k && st == ORC_OK; ++j) {
    if (j > 1) orc_apply_mass(nx, h, dU, rhs);
    st = orc_cyclic_solve(nx, a, b, c, rhs, dU);
  }
  free(a);
  free(b);
  free(c);
  free(rhs);
  return st;
}

/* The transpose of the linear map dWc -> dU of orc_matern_field: with
 * A = M + kappa^{-2} K and B the load operator (b_n = sqrt(h) (w_{n-1} + w_n)/2),
 * dU = (A^{-1} M)^{k-1} A^{-1} eta B dWc, so the transpose is
 * eta B^T A^{-1} (M A^{-1})^{k-1}: z = A^{-1} g, then z = A^{-1} M z (k - 1
 * times), out_i = eta sqrt(h) (z_i + z_{i+1}) / 2.  (Used by the nudging
 * gradient with the Matern-type noise.) */
int orc_matern_transpose(int32_t nx, double L, const orc_matern *mt, const double *g,
                         double *out) {
  double h = L / nx, ik2 = 1.0 / (mt->kappa * mt->kappa);
  size_t sz = sizeof(double) * (size_t)nx;
  double *a = (double *)calloc((size_t)nx, sizeof(double));
  double *b = (double *)calloc((size_t)nx, sizeof(double));
  double *c = (double *)calloc((size_t)nx, sizeof(double));
  double *z = (double *)malloc(sz), *r = (double *)malloc(sz);
  for (int32_t i = 0; i < nx; ++i) {
    a[i] = h / 6.0 - ik2 / h;
    b[i] = 2.0 * h / 3.0 + 2.0 * ik2 / h;
    c[i] = h / 6.0 - ik2 / h;
  }
  int st = orc_cyclic_solve(nx, a, b, c, g, z);
  for (int32_t j = 2; j <= mt->k && st == ORC_OK; ++j) {
    orc_apply_mass(nx, h, z, r);
    st = orc_cyclic_solve(nx, a, b, c, r, z);
  }
  for (int32_t i = 0; i < nx; ++i) out[i] = mt->eta * sqrt(h) * 0.5 * (z[i] + z[wrap(i + 1, nx)]);
  free(a);
  free(b);
  free(c);
  free(z);
  free(r);
  return st;
}

int orc_step_matern(const orc_model *md, const orc_matern *mt, double *m, double *u,
                    const double *dWc, int32_t *iters) {
  double *dU = (double *)malloc(sizeof(double) * (size_t)md->nx);
  int st = orc_matern_field(md->nx, md->L, mt, dWc, dU);
  if (st == ORC_OK) st = orc_step_field(md, m, u, dU, iters);
  free(dU);
  return st;
}

/* n_steps steps with cell increments dWc [n_steps][nx]. */
int orc_window_matern(const orc_model *md, const orc_matern *mt, int32_t n_steps, double *m,
                      double *u, const double *dWc, int32_t *iters) {
  int32_t total = 0;
  for (int32_t s = 0; s < n_steps; ++s) {
    int32_t it = 0;
    int st = orc_step_matern(md, mt, m, u, dWc + (size_t)s * md->nx, &it);
    total += it;
    if (st != ORC_OK) {
      if (iters) *iters = total;
      return st;
    }
  }
  if (iters) *iters = total;
  return ORC_OK;
}

int orc_ensemble_window_matern(const orc_model *md, const orc_matern *mt, int32_t n_particles,
                               int32_t n_steps, double *m, double *u, const double *dWc,
                               int32_t *status, int32_t *iters, int32_t n_threads) {
  int worst = ORC_OK;
  int32_t nx = md->nx;
#pragma omp parallel for num_threads(n_threads > 0 ? n_threads : 1) schedule(dynamic, 1)
  for (int32_t p = 0; p < n_particles; ++p) {
    int32_t it = 0;
    int st = orc_window_matern(md, mt, n_steps, m + (size_t)p * nx, u + (size_t)p * nx,
                               dWc + (size_t)p * n_steps * nx, &it);
    if (status) status[p] = st;
    if (iters) iters[p] = it;
    if (st != ORC_OK) {
#pragma omp critical
      worst = st;
    }
  }
  return worst;
}

/* ========================================================================== */
/* Observations and likelihood (section 3, eqs. obseq and loglikeq).           */
/* Data grid x_j = j L / n_obs, j = 0..n_obs-1 (the periodic point L is the    */
/* point 0).  The projection onto the data grid is point evaluation of the P1  */
/* field: x_j lies in cell e = floor(j nx / n_obs) at fraction                 */
/* r = (j nx mod n_obs) / n_obs, located with integers so that it is exact.    */
/* ========================================================================== */
void orc_observe(int32_t nx, int32_t n_obs, const double *u, double *out) {
  for (int32_t j = 0; j < n_obs; ++j) {
    int64_t num = (int64_t)j * nx;
    int32_t e = (int32_t)(num / n_obs);
    double r = (double)(num % n_obs) / (double)n_obs;
    out[j] = (1.0 - r) * u[e % nx] + r * u[(e + 1) % nx];
  }
}

/* Negative log of the likelihood weight of eq. loglikeq:
 *   Phi = 1/2 sum_j ((P u)_j - y_j)^2 / sigma_j^2. */
double orc_nll(int32_t nx, int32_t n_obs, const double *u, const double *y, const double *sigma) {
  double *pu = (double *)malloc(sizeof(double) * n_obs);
  orc_observe(nx, n_obs, u, pu);
  long double s = 0.0L;
  for (int32_t j = 0; j < n_obs; ++j) {
    double r = (pu[j] - y[j]) / sigma[j];
    s += (long double)(r * r);
  }
  free(pu);
  return (double)(0.5L * s);
}

void orc_ensemble_nll(int32_t nx, int32_t n_obs, int32_t n_particles, const double *u,
                      const double *y, const double *sigma, double *phi) {
  for (int32_t p = 0; p < n_particles; ++p)
    phi[p] = orc_nll(nx, n_obs, u + (size_t)p * nx, y, sigma);
}

/* ========================================================================== */
/* Normalised weights and the effective sample size (eq. ess):                  */
/*   w_p proportional to exp(logw_extra_p - beta Phi_p),                       */
/*   wbar = w / sum(w),  ESS = 1 / sum(wbar^2).                                 */
/* Evaluated after subtracting the largest exponent so that nothing overflows. */
/* logw_out (optional) receives log(wbar).  Returns the ESS (0 if every weight */
/* vanishes, in which case w is all zero).                                     */
/* ========================================================================== */
double orc_weights(int32_t n, const double *phi, const double *logw_extra, double beta,
                   double *w, double *logw_out) {
  double *s = (double *)malloc(sizeof(double) * n);
  double smax = -INFINITY;
  for (int32_t p = 0; p < n; ++p) {
    double e = logw_extra ? logw_extra[p] : 0.0;
    double t;
    if (beta == 0.0)
      t = e;
    else if (isnan(phi[p]))
      t = -INFINITY;
    else
      t = e - beta * phi[p];
    if (isnan(t)) t = -INFINITY;
    s[p] = t;
    if (t > smax) smax = t;
  }
  if (!(smax > -INFINITY)) {
    for (int32_t p = 0; p < n; ++p) {
      w[p] = 0.0;
      if (logw_out) logw_out[p] = -INFINITY;
    }
    free(s);
    return 0.0;
  }
  long double tot = 0.0L;
  for (int32_t p = 0; p < n; ++p) tot += (long double)exp(s[p] - smax);
  double ltot = (double)logl(tot);
  long double sq = 0.0L;
  for (int32_t p = 0; p < n; ++p) {
    w[p] = (double)((long double)exp(s[p] - smax) / tot);
    if (logw_out) logw_out[p] = (s[p] - smax) - ltot;
    sq += (long double)w[p] * (long double)w[p];
  }
  free(s);
  return (double)(1.0L / sq);
}

/* Adaptive tempering (section 3.1.2): choose the increment dtheta of the
 * temperature so that the ESS of the tempered weights exp(-dtheta Phi) stays
 * at or above the threshold N_p*, with the fewest steps.  The paper "reduces
 * dtheta until the condition holds"; this oracle takes the largest admissible
 * dtheta by bisection (the ESS is non-increasing in dtheta):
 *   rem = 1 - theta; if ESS(rem) >= thr take rem;
 *   else lo = 0, hi = rem, n_bisect times: mid = (lo + hi)/2, keep lo if
 *   ESS(mid) >= thr else hi; take lo (or hi when lo never moved).
 * w receives the normalised weights at the chosen dtheta. */
int orc_temper(int32_t n, const double *phi, double theta, double threshold, int32_t n_bisect,
               double *dtheta, double *w, double *ess) {
  double rem = 1.0 - theta;
  double e = orc_weights(n, phi, NULL, rem, w, NULL);
  if (e >= threshold || n_bisect <= 0) {
    *dtheta = rem;
    *ess = e;
    return ORC_OK;
  }
  double lo = 0.0, hi = rem;
  for (int32_t k = 0; k < n_bisect; ++k) {
    double mid = 0.5 * (lo + hi);
    double em = orc_weights(n, phi, NULL, mid, w, NULL);
    if (em >= threshold)
      lo = mid;
    else
      hi = mid;
  }
  double pick = lo > 0.0 ? lo : hi;
  *dtheta = pick;
  *ess = orc_weights(n, phi, NULL, pick, w, NULL);
  return ORC_OK;
}

/* ========================================================================== */
/* Systematic resampling (section 3.1.1, after Gordon et al.): one uniform u0, */
/* points t_j = (j + u0)/N, and idx_j = the first particle whose cumulative    */
/* weight exceeds t_j.                                                         */
/*                                                                            */
/* Integer-exact form (the contract the GPU must match bit for bit): each      */
/* weight is quantised to q_p = floor(w_p * 2^(51 - b - e)), b = ceil(log2 N), */
/* e = binary exponent of max w (max w < 2^e), so every partial sum C_p of the */
/* q is an exact integer below 2^51.  Then T_j = ((j + u0) * Q) / N with       */
/* Q = C_{N-1}, each operation rounded once, and                               */
/* idx_j = min{ p : C_p > T_j }, clamped to N - 1.                             */
/* ========================================================================== */
int orc_resample_systematic(int32_t n, const double *w, double u0, int32_t *idx) {
  if (n <= 0) return ORC_E_ARG;
  double wmax = 0.0;
  for (int32_t p = 0; p < n; ++p) {
    if (!(w[p] >= 0.0) || isinf(w[p])) return ORC_E_ARG;
    if (w[p] > wmax) wmax = w[p];
  }
  if (wmax == 0.0) return ORC_E_DEGENERATE;
  int e;
  frexp(wmax, &e);
  int b = 0;
  while (((int64_t)1 << b) < (int64_t)n) ++b;
  uint64_t *cum = (uint64_t *)malloc(sizeof(uint64_t) * n);
  uint64_t acc = 0;
  for (int32_t p = 0; p < n; ++p) {
    acc += (uint64_t)floor(ldexp(w[p], 51 - b - e));
    cum[p] = acc;
  }
  if (acc == 0) {
    free(cum);
    return ORC_E_DEGENERATE;
  }
  double Q = (double)acc;
  int32_t p = 0;
  for (int32_t j = 0; j < n; ++j) {
    double t = (double)j + u0;
    t = t * Q;
    t = t / (double)n;
    while (p < n && !((double)cum[p] > t)) ++p;
    idx[j] = p < n ? p : n - 1;
  }
  free(cum);
  return ORC_OK;
}

/* The textbook floating-point version, for the oracle's own checks. */
int orc_resample_textbook(int32_t n, const double *w, double u0, int32_t *idx) {
  if (n <= 0) return ORC_E_ARG;
  long double tot = 0.0L;
  for (int32_t p = 0; p < n; ++p) tot += w[p];
  if (!(tot > 0.0L)) return ORC_E_DEGENERATE;
  long double c = 0.0L;
  int32_t p = 0;
  c = w[0] / tot;
  for (int32_t j = 0; j < n; ++j) {
    long double t = ((long double)j + u0) / (long double)n;
    while (p < n - 1 && !(c > t)) {
      ++p;
      c += w[p] / tot;
    }
    idx[j] = p;
  }
  return ORC_OK;
}

/* ========================================================================== */
/* Jittering by preconditioned Crank-Nicolson MCMC (section 3.1.2).  For each  */
/* particle, starting from its window-start state and increments dW:           */
/*   proposal dW' = rho dW + sqrt(1 - rho^2) zeta,  zeta ~ N(0, dt) iid         */
/*   (the paper's (2-delta)/(2+delta) and sqrt(8 delta)/(2+delta) are rho and  */
/*   sqrt(1 - rho^2) for rho = (2-delta)/(2+delta));                           */
/*   rerun the window with dW', Phi' = negative log-likelihood;                */
/*   accept with probability min(1, exp(theta (Phi - Phi'))).  The paper       */
/*   prints max(1, .), which is never below one; min is the Metropolis rule    */
/*   for the theta-weighted negative log-likelihoods it defines.               */
/* A proposal whose window fails (non-convergence, non-finite state) is        */
/* rejected.  Random numbers: zeta with tag PCN, counter (particle, global     */
/* step, pair | tag, temper k << 16 | j); the acceptance uniform with tag      */
/* ACCEPT, counter (particle, cycle, tag << 24, temper k << 16 | j).           */
/* ========================================================================== */
/* pCN proposal for one particle: prop = rho cur + sqrt(1 - rho^2) zeta with
 * zeta = sqrt(dt) z, z from the PCN-tagged Philox stream. */
void orc_pcn_propose(uint64_t seed, uint32_t particle, uint32_t step0, int32_t n_steps,
                     int32_t n_modes, uint32_t word3, double rho, double dt, const double *cur,
                     double *prop) {
  double srho = sqrt(1.0 - rho * rho);
  double sdt = sqrt(dt);
  int32_t n_pairs = (n_modes + 1) / 2;
  for (int32_t n = 0; n < n_steps; ++n)
    for (int32_t k = 0; k < n_pairs; ++k) {
      double z[2];
      orc_normal_pair(seed, particle, step0 + (uint32_t)n,
                      (uint32_t)k | ((uint32_t)ORC_TAG_PCN << 24), word3, z);
      size_t i0 = (size_t)n * n_modes + 2 * k;
      prop[i0] = rho * cur[i0] + srho * (sdt * z[0]);
      if (2 * k + 1 < n_modes) prop[i0 + 1] = rho * cur[i0 + 1] + srho * (sdt * z[1]);
    }
}

/* Metropolis rule with probability min(1, exp(theta (phi_old - phi_new))):
 * a non-finite proposal is rejected, a non-worse one accepted, otherwise the
 * uniform v decides. */
int orc_pcn_accept(double theta, double phi_old, double phi_new, double v) {
  if (!(phi_new < INFINITY)) return 0;
  double logr = theta * (phi_old - phi_new);
  if (logr >= 0.0) return 1;
  return v < exp(logr);
}

int orc_jitter_pcn(const orc_model *md, int32_t n_obs, const double *y, const double *sigma,
                   const orc_rng *rng, int32_t n_particles, int32_t n_steps, const double *m0,
                   const double *u0, double *dW, double *phi, double *m_end, double *u_end,
                   double theta, double rho, int32_t n_jitter, int32_t *n_accept,
                   int32_t n_threads) {
  int32_t nx = md->nx, nq = md->n_modes;
#pragma omp parallel for num_threads(n_threads > 0 ? n_threads : 1) schedule(dynamic, 1)
  for (int32_t p = 0; p < n_particles; ++p) {
    size_t wlen = (size_t)n_steps * nq;
    double *prop = (double *)malloc(sizeof(double) * wlen);
    double *mm = (double *)malloc(sizeof(double) * nx);
    double *uu = (double *)malloc(sizeof(double) * nx);
    double *dWp = dW + (size_t)p * wlen;
    int32_t acc = 0;
    for (int32_t j = 0; j < n_jitter; ++j) {
      uint32_t w3 = (rng->temper_k << 16) | (uint32_t)j;
      orc_pcn_propose(rng->seed, (uint32_t)p, rng->cycle * (uint32_t)n_steps, n_steps, nq, w3,
                      rho, md->dt, dWp, prop);
      memcpy(mm, m0 + (size_t)p * nx, sizeof(double) * nx);
      memcpy(uu, u0 + (size_t)p * nx, sizeof(double) * nx);
      int32_t it = 0;
      int st = orc_window(md, n_steps, mm, uu, prop, NULL, &it);
      double phi_new = st == ORC_OK ? orc_nll(nx, n_obs, uu, y, sigma) : INFINITY;
      if (!isfinite(phi_new)) phi_new = INFINITY;
      double v = orc_uniform(rng->seed, (uint32_t)p, rng->cycle,
                             (uint32_t)ORC_TAG_ACCEPT << 24, w3);
      if (orc_pcn_accept(theta, phi[p], phi_new, v)) {
        memcpy(dWp, prop, sizeof(double) * wlen);
        phi[p] = phi_new;
        memcpy(m_end + (size_t)p * nx, mm, sizeof(double) * nx);
        memcpy(u_end + (size_t)p * nx, uu, sizeof(double) * nx);
        ++acc;
      }
    }
    if (n_accept) n_accept[p] = acc;
    free(prop);
    free(mm);
    free(uu);
  }
  return ORC_OK;
}

/* Potential of a nudged path for the tempered weights (section 3.1.3, last
 * paragraph: W replaced by W~ = W + G in the log-weights): the negative
 * log-likelihood plus minus the log of the discrete Girsanov factor,
 *   J = phi + sum_i (dLam_i^2 / 2 + dLam_i dW_i) / dt,
 * with dLam the control and dW the Brownian increment of the path. */
double orc_nudged_potential(double phi, int32_t len, double dt, const double *dW,
                            const double *dLam) {
  if (!(phi < INFINITY)) return INFINITY;
  double g = 0.0;
  for (int32_t i = 0; i < len; ++i) g += 0.5 * dLam[i] * dLam[i] / dt + dLam[i] * dW[i] / dt;
  double J = phi + g;
  return isfinite(J) ? J : INFINITY;
}

/* pCN moves of the increments with the control held fixed (jittering of the
 * nudged filter): the proposal and its uniforms are those of orc_jitter_pcn,
 * the window runs with dW' + dLam, and the potential is the nudged J above,
 * so the chain leaves the prior of dW tempered by exp(-theta J) invariant.
 * phi holds J in and out. */
int orc_jitter_pcn_ctrl(const orc_model *md, int32_t n_obs, const double *y, const double *sigma,
                        const orc_rng *rng, int32_t n_particles, int32_t n_steps,
                        const double *m0, const double *u0, double *dW, const double *dLam,
                        double *phi, double *m_end, double *u_end, double theta, double rho,
                        int32_t n_jitter, int32_t *n_accept, int32_t n_threads) {
  int32_t nx = md->nx, nq = md->n_modes;
#pragma omp parallel for num_threads(n_threads > 0 ? n_threads : 1) schedule(dynamic, 1)
  for (int32_t p = 0; p < n_particles; ++p) {
    size_t wlen = (size_t)n_steps * nq;
    double *prop = (double *)malloc(sizeof(double) * wlen);
    double *mm = (double *)malloc(sizeof(double) * nx);
    double *uu = (double *)malloc(sizeof(double) * nx);
    double *dWp = dW + (size_t)p * wlen;
    const double *lam = dLam + (size_t)p * wlen;
    int32_t acc = 0;
    for (int32_t j = 0; j < n_jitter; ++j) {
      uint32_t w3 = (rng->temper_k << 16) | (uint32_t)j;
      orc_pcn_propose(rng->seed, (uint32_t)p, rng->cycle * (uint32_t)n_steps, n_steps, nq, w3,
                      rho, md->dt, dWp, prop);
      memcpy(mm, m0 + (size_t)p * nx, sizeof(double) * nx);
      memcpy(uu, u0 + (size_t)p * nx, sizeof(double) * nx);
      int32_t it = 0;
      int st = orc_window(md, n_steps, mm, uu, prop, lam, &it);
      double phi_new = st == ORC_OK ? orc_nll(nx, n_obs, uu, y, sigma) : INFINITY;
      double J_new = orc_nudged_potential(isfinite(phi_new) ? phi_new : INFINITY, (int32_t)wlen,
                                          md->dt, prop, lam);
      double v = orc_uniform(rng->seed, (uint32_t)p, rng->cycle,
                             (uint32_t)ORC_TAG_ACCEPT << 24, w3);
      if (orc_pcn_accept(theta, phi[p], J_new, v)) {
        memcpy(dWp, prop, sizeof(double) * wlen);
        phi[p] = J_new;
        memcpy(m_end + (size_t)p * nx, mm, sizeof(double) * nx);
        memcpy(u_end + (size_t)p * nx, uu, sizeof(double) * nx);
        ++acc;
      }
    }
    if (n_accept) n_accept[p] = acc;
    free(prop);
    free(mm);
    free(uu);
  }
  return ORC_OK;
}

/* The linear toy chain of orc_pcn_linear_chain with a fixed control lam:
 * the map sees x + lam, and the potential is the nudged J of x,
 *   J(x) = |G (x + lam) - y|^2 / (2 sigma^2) + sum (lam^2 / 2 + lam x) / dt,
 * so x + lam is distributed as the tempered Gaussian posterior of the
 * forcing whatever lam is.  samples is [n_iter][d] of x; returns the number
 * of acceptances. */
int64_t orc_pcn_linear_chain_ctrl(uint64_t seed, int32_t n_steps, int32_t n_modes, int32_t n_obs,
                                  const double *G, const double *y, double sigma, double theta,
                                  double rho, double dt, const double *lam, int32_t n_iter,
                                  const double *x0, double *samples) {
  int32_t d = n_steps * n_modes;
  double *x = (double *)malloc(sizeof(double) * d), *prop = (double *)malloc(sizeof(double) * d);
  double *b = (double *)malloc(sizeof(double) * d);
  memcpy(x, x0, sizeof(double) * d);
  double J = 0.0;
  for (int32_t i = 0; i < d; ++i) b[i] = x[i] + lam[i];
  for (int32_t j = 0; j < n_obs; ++j) {
    double r = -y[j];
    for (int32_t i = 0; i < d; ++i) r += G[(size_t)j * d + i] * b[i];
    J += 0.5 * r * r / (sigma * sigma);
  }
  J = orc_nudged_potential(J, d, dt, x, lam);
  int64_t acc = 0;
  for (int32_t it = 0; it < n_iter; ++it) {
    orc_pcn_propose(seed, 0u, 0u, n_steps, n_modes, (uint32_t)it, rho, dt, x, prop);
    for (int32_t i = 0; i < d; ++i) b[i] = prop[i] + lam[i];
    double Jn = 0.0;
    for (int32_t j = 0; j < n_obs; ++j) {
      double r = -y[j];
      for (int32_t i = 0; i < d; ++i) r += G[(size_t)j * d + i] * b[i];
      Jn += 0.5 * r * r / (sigma * sigma);
    }
    Jn = orc_nudged_potential(Jn, d, dt, prop, lam);
    double v = orc_uniform(seed, 0u, 0u, (uint32_t)ORC_TAG_ACCEPT << 24, (uint32_t)it);
    if (orc_pcn_accept(theta, J, Jn, v)) {
      memcpy(x, prop, sizeof(double) * d);
      J = Jn;
      ++acc;
    }
    memcpy(samples + (size_t)it * d, x, sizeof(double) * d);
  }
  free(x);
  free(prop);
  free(b);
  return acc;
}

/* The same pCN chain with the forward model replaced by a fixed linear map:
 * the increments x (dimension d = n_steps * n_modes, prior N(0, dt I)) are
 * observed as y = G x + noise(sigma), Phi(x) = |G x - y|^2 / (2 sigma^2).
 * Used only to check the proposal and the acceptance rule against the
 * closed-form Gaussian posterior tempered at theta.  samples is
 * [n_iter][d]; returns the number of acceptances. */
int64_t orc_pcn_linear_chain(uint64_t seed, int32_t n_steps, int32_t n_modes, int32_t n_obs,
                             const double *G, const double *y, double sigma, double theta,
                             double rho, double dt, int32_t n_iter, const double *x0,
                             double *samples) {
  int32_t d = n_steps * n_modes;
  double *x = (double *)malloc(sizeof(double) * d), *prop = (double *)malloc(sizeof(double) * d);
  memcpy(x, x0, sizeof(double) * d);
  double phi = 0.0;
  for (int32_t j = 0; j < n_obs; ++j) {
    double r = -y[j];
    for (int32_t i = 0; i < d; ++i) r += G[(size_t)j * d + i] * x[i];
    phi += 0.5 * r * r / (sigma * sigma);
  }
  int64_t acc = 0;
  for (int32_t it = 0; it < n_iter; ++it) {
    uint32_t w3 = (uint32_t)it;
    orc_pcn_propose(seed, 0u, (uint32_t)(it >> 16) * (uint32_t)n_steps, n_steps, n_modes, w3,
                    rho, dt, x, prop);
    double phin = 0.0;
    for (int32_t j = 0; j < n_obs; ++j) {
      double r = -y[j];
      for (int32_t i = 0; i < d; ++i) r += G[(size_t)j * d + i] * prop[i];
      phin += 0.5 * r * r / (sigma * sigma);
    }
    double v = orc_uniform(seed, 0u, (uint32_t)(it >> 16), (uint32_t)ORC_TAG_ACCEPT << 24, w3);
    if (orc_pcn_accept(theta, phi, phin, v)) {
      memcpy(x, prop, sizeof(double) * d);
      phi = phin;
      ++acc;
    }
    memcpy(samples + (size_t)it * d, x, sizeof(double) * d);
  }
  free(x);
  free(prop);
  return acc;
}

/* ========================================================================== */
/* Filter cycles.                                                              */
/* ========================================================================== */

static void gather_rows(double *a, const int32_t *idx, int32_t n, size_t row) {
  double *tmp = (double *)malloc(sizeof(double) * row * (size_t)n);
  for (int32_t j = 0; j < n; ++j) memcpy(tmp + (size_t)j * row, a + (size_t)idx[j] * row,
                                         sizeof(double) * row);
  memcpy(a, tmp, sizeof(double) * row * (size_t)n);
  free(tmp);
}

/* Bootstrap (sampling-importance-resampling) filter, section 3.1.1: propagate
 * every particle through one assimilation window with independent increments,
 * multiply its weight by the likelihood, and resample (systematic) when the
 * ESS falls below ess_frac * N (the paper's N_p* threshold, eq. ess).  Between
 * resamplings the normalised log-weights are carried in logw. */
/* The bootstrap cycle with the modes-form noise (mt == NULL) or the
 * Matern-type noise (mt != NULL: nx cell increments per step). */
static int bootstrap_cycle(const orc_model *md, const orc_matern *mt, int32_t n_obs,
                           const double *y, const double *sigma, uint64_t seed, uint32_t cycle,
                           int32_t n_particles, int32_t n_steps, double ess_frac, double *m,
                           double *u, double *logw, orc_cycle_stats *st, int32_t n_threads) {
  int32_t nx = md->nx, nq = mt ? md->nx : md->n_modes;
  double *dW = (double *)malloc(sizeof(double) * (size_t)n_particles * n_steps * nq);
  int32_t *iters = (int32_t *)malloc(sizeof(int32_t) * n_particles);
  int32_t *stat = (int32_t *)malloc(sizeof(int32_t) * n_particles);
  double *phi = (double *)malloc(sizeof(double) * n_particles);
  double *w = (double *)malloc(sizeof(double) * n_particles);
  int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * n_particles);
  memset(st, 0, sizeof(*st));

  orc_draw_increments(seed, n_particles, n_steps, nq, cycle * (uint32_t)n_steps, ORC_TAG_FORECAST,
                      0u, md->dt, dW);
  if (mt)
    orc_ensemble_window_matern(md, mt, n_particles, n_steps, m, u, dW, stat, iters, n_threads);
  else
    orc_ensemble_window(md, n_particles, n_steps, m, u, dW, NULL, stat, iters, n_threads);
  for (int32_t p = 0; p < n_particles; ++p) {
    st->picard_iters += iters[p];
    phi[p] = stat[p] == ORC_OK ? orc_nll(nx, n_obs, u + (size_t)p * nx, y, sigma) : INFINITY;
    if (!isfinite(phi[p])) phi[p] = INFINITY;
  }
  double ess = orc_weights(n_particles, phi, logw, 1.0, w, logw);
  st->ess = ess;
  int rc = ORC_OK;
  if (ess == 0.0) {
    rc = ORC_E_DEGENERATE;
  } else if (ess < ess_frac * n_particles) {
    double u0 = orc_uniform(seed, 0u, cycle, (uint32_t)ORC_TAG_RESAMPLE << 24, 0u);
    rc = orc_resample_systematic(n_particles, w, u0, idx);
    if (rc == ORC_OK) {
      gather_rows(m, idx, n_particles, (size_t)nx);
      gather_rows(u, idx, n_particles, (size_t)nx);
      for (int32_t p = 0; p < n_particles; ++p) logw[p] = 0.0;
      st->resampled = 1;
    }
  }
  st->status = rc;
  free(dW);
  free(iters);
  free(stat);
  free(phi);
  free(w);
  free(idx);
  return rc;
}

int orc_bootstrap_cycle(const orc_model *md, int32_t n_obs, const double *y, const double *sigma,
                        uint64_t seed, uint32_t cycle, int32_t n_particles, int32_t n_steps,
                        double ess_frac, double *m, double *u, double *logw,
                        orc_cycle_stats *st, int32_t n_threads) {
  return bootstrap_cycle(md, NULL, n_obs, y, sigma, seed, cycle, n_particles, n_steps, ess_frac,
                         m, u, logw, st, n_threads);
}

int orc_bootstrap_cycle_matern(const orc_model *md, const orc_matern *mt, int32_t n_obs,
                               const double *y, const double *sigma, uint64_t seed,
                               uint32_t cycle, int32_t n_particles, int32_t n_steps,
                               double ess_frac, double *m, double *u, double *logw,
                               orc_cycle_stats *st, int32_t n_threads) {
  return bootstrap_cycle(md, mt, n_obs, y, sigma, seed, cycle, n_particles, n_steps, ess_frac, m,
                         u, logw, st, n_threads);
}

/* The tempering loop of section 3.1.2, shared by every tempered driver
 * (modes, pCN-Langevin, Matern-type noise, nudged): the temperature theta
 * climbs from 0 to 1 in adaptive steps; at each step the increment dtheta is
 * the largest with ESS(exp(-dtheta pot)) >= threshold (orc_temper), the
 * ensemble is resampled with those incremental weights (uniform of tag
 * RESAMPLE, counter (0, cycle, tag << 24, k << 16)), every row set of the
 * particles and their potentials are gathered by the same indices, and the
 * jitter moves the increments at the new cumulative temperature (reading
 * G16).  The jitter callback receives theta and the step's RNG keys and
 * writes the per-particle acceptance counts.
 *
 * `plant` exists only for the pins of this loop (ORC_PLANT_*): a nonzero value
 * plants a known mistake so that the tests can show their power. */
typedef void (*jitter_fn)(void *ctx, const orc_rng *rng, double theta, int32_t *acc);
typedef struct {
  double *a;
  size_t len; /* doubles per particle */
} row_set;

static int temper_loop(int32_t n, double *pot, row_set *rows, int32_t n_rows, uint64_t seed,
                       uint32_t cycle, double ess_threshold, int32_t n_bisect, int32_t max_temper,
                       jitter_fn jitter, void *ctx, orc_cycle_stats *st, int32_t plant) {
  double *w = (double *)malloc(sizeof(double) * n);
  int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * n);
  int32_t *acc = (int32_t *)malloc(sizeof(int32_t) * n);
  double theta = 0.0;
  int32_t k = 0;
  int rc = ORC_OK;
  while (theta < 1.0) {
    if (k >= max_temper) {
      rc = ORC_E_DEGENERATE;
      break;
    }
    double dth, ess;
    orc_temper(n, pot, theta, ess_threshold, n_bisect, &dth, w, &ess);
    if (ess == 0.0) {
      rc = ORC_E_DEGENERATE;
      break;
    }
    double theta_new = (dth == 1.0 - theta) ? 1.0 : theta + dth;
    if (plant == ORC_PLANT_CUMULATIVE_WEIGHTS) orc_weights(n, pot, NULL, theta_new, w, NULL);
    double ur = orc_uniform(seed, 0u, cycle, (uint32_t)ORC_TAG_RESAMPLE << 24, (uint32_t)k << 16);
    rc = orc_resample_systematic(n, w, ur, idx);
    if (rc != ORC_OK) break;
    for (int32_t r = 0; r < n_rows; ++r) gather_rows(rows[r].a, idx, n, rows[r].len);
    gather_rows(pot, idx, n, 1);
    orc_rng rg = {seed, cycle, (uint32_t)k};
    jitter(ctx, &rg, plant == ORC_PLANT_JITTER_PRE_THETA ? theta : theta_new, acc);
    for (int32_t p = 0; p < n; ++p) st->n_accept += acc[p];
    st->ess = ess;
    theta = theta_new;
    ++k;
  }
  st->n_temper = k;
  free(w);
  free(idx);
  free(acc);
  return rc;
}

/* The jitters of the SCH drivers behind the callback of temper_loop. */
enum { JIT_PCN = 0, JIT_PCNL = 1, JIT_PCN_CTRL = 2, JIT_MATERN = 3, JIT_HMC = 4 };
static int jitter_matern(const orc_model *md, const orc_matern *mt, int32_t n_obs,
                         const double *y, const double *sigma, const orc_rng *rng,
                         int32_t n_particles, int32_t n_steps, const double *m0, const double *u0,
                         double *dWc, const double *dLamc, double *phi, double *m_end,
                         double *u_end, double theta, double rho, int32_t n_jitter,
                         int32_t *n_accept, int32_t n_threads);
typedef struct {
  int kind;
  const orc_model *md;
  const orc_matern *mt;
  int32_t n_obs, n_particles, n_steps, n_jitter, n_threads;
  const double *y, *sigma, *m0, *u0, *dLam;
  double *dW, *pot, *m, *u;
  double rho;
  double h;       /* HMC: leapfrog angle */
  int32_t n_leap; /* HMC: leapfrog steps per move */
} sch_jitter_ctx;

static void sch_jitter(void *vctx, const orc_rng *rg, double theta, int32_t *acc) {
  sch_jitter_ctx *c = (sch_jitter_ctx *)vctx;
  switch (c->kind) {
    case JIT_PCNL:
      orc_jitter_pcnl(c->md, c->n_obs, c->y, c->sigma, rg, c->n_particles, c->n_steps, c->m0,
                      c->u0, c->dW, c->pot, c->m, c->u, theta, c->rho, c->n_jitter, acc,
                      c->n_threads);
      break;
    case JIT_HMC:
      orc_jitter_hmc(c->md, c->n_obs, c->y, c->sigma, rg, c->n_particles, c->n_steps, c->m0,
                     c->u0, c->dW, c->pot, c->m, c->u, theta, c->h, c->n_leap, c->n_jitter, acc,
                     c->n_threads);
      break;
    case JIT_PCN_CTRL:
      orc_jitter_pcn_ctrl(c->md, c->n_obs, c->y, c->sigma, rg, c->n_particles, c->n_steps,
                          c->m0, c->u0, c->dW, c->dLam, c->pot, c->m, c->u, theta, c->rho,
                          c->n_jitter, acc, c->n_threads);
      break;
    case JIT_MATERN:
      jitter_matern(c->md, c->mt, c->n_obs, c->y, c->sigma, rg, c->n_particles, c->n_steps,
                    c->m0, c->u0, c->dW, c->dLam, c->pot, c->m, c->u, theta, c->rho, c->n_jitter,
                    acc, c->n_threads);
      break;
    default:
      orc_jitter_pcn(c->md, c->n_obs, c->y, c->sigma, rg, c->n_particles, c->n_steps, c->m0,
                     c->u0, c->dW, c->pot, c->m, c->u, theta, c->rho, c->n_jitter, acc,
                     c->n_threads);
  }
}

/* Tempered and jittered filter, section 3.1.2.  Each particle is the pair
 * (window-start state, increments over the window).  After the forecast, the
 * temperature climbs from 0 to 1 in the steps of temper_loop; after every
 * step the ensemble is resampled with the tempered weights exp(-dtheta Phi)
 * and every particle's increments are moved by n_jitter pCN steps targeting
 * the posterior tempered at the new cumulative theta.  Only then does the
 * window end state become the next cycle's start state. */
/* The tempered cycle with pCN moves (pcnl == 0) or pCN-Langevin moves. */
static int tempered_cycle(const orc_model *md, int32_t n_obs, const double *y,
                          const double *sigma, uint64_t seed, uint32_t cycle, int32_t n_particles,
                          int32_t n_steps, double ess_threshold, int32_t n_bisect, double rho,
                          int32_t n_jitter, int32_t max_temper, double *m, double *u,
                          orc_cycle_stats *st, int32_t n_threads, int kind, double h,
                          int32_t n_leap) {
  int32_t nx = md->nx, nq = md->n_modes;
  size_t state = (size_t)n_particles * nx, wlen = (size_t)n_particles * n_steps * nq;
  double *m0 = (double *)malloc(sizeof(double) * state), *u0 = (double *)malloc(sizeof(double) * state);
  double *dW = (double *)malloc(sizeof(double) * wlen);
  double *phi = (double *)malloc(sizeof(double) * n_particles);
  int32_t *iters = (int32_t *)malloc(sizeof(int32_t) * n_particles);
  int32_t *stat = (int32_t *)malloc(sizeof(int32_t) * n_particles);
  memset(st, 0, sizeof(*st));
  memcpy(m0, m, sizeof(double) * state);
  memcpy(u0, u, sizeof(double) * state);

  orc_draw_increments(seed, n_particles, n_steps, nq, cycle * (uint32_t)n_steps, ORC_TAG_FORECAST,
                      0u, md->dt, dW);
  orc_ensemble_window(md, n_particles, n_steps, m, u, dW, NULL, stat, iters, n_threads);
  for (int32_t p = 0; p < n_particles; ++p) {
    st->picard_iters += iters[p];
    phi[p] = stat[p] == ORC_OK ? orc_nll(nx, n_obs, u + (size_t)p * nx, y, sigma) : INFINITY;
    if (!isfinite(phi[p])) phi[p] = INFINITY;
  }
  row_set rows[5] = {{m0, (size_t)nx}, {u0, (size_t)nx}, {m, (size_t)nx}, {u, (size_t)nx},
                     {dW, (size_t)n_steps * nq}};
  sch_jitter_ctx jc = {kind, md, NULL, n_obs, n_particles, n_steps, n_jitter, n_threads, y,
                       sigma, m0, u0, NULL, dW, phi, m, u, rho, h, n_leap};
  int rc = temper_loop(n_particles, phi, rows, 5, seed, cycle, ess_threshold, n_bisect,
                       max_temper, sch_jitter, &jc, st, ORC_PLANT_NONE);
  st->status = rc;
  free(m0);
  free(u0);
  free(dW);
  free(phi);
  free(iters);
  free(stat);
  return rc;
}

int orc_tempered_cycle(const orc_model *md, int32_t n_obs, const double *y, const double *sigma,
                       uint64_t seed, uint32_t cycle, int32_t n_particles, int32_t n_steps,
                       double ess_threshold, int32_t n_bisect, double rho, int32_t n_jitter,
                       int32_t max_temper, double *m, double *u, orc_cycle_stats *st,
                       int32_t n_threads) {
  return tempered_cycle(md, n_obs, y, sigma, seed, cycle, n_particles, n_steps, ess_threshold,
                        n_bisect, rho, n_jitter, max_temper, m, u, st, n_threads, JIT_PCN, 0.0,
                        0);
}

/* The tempered cycle with the gradient-based pCN-Langevin jitter
 * (orc_jitter_pcnl) in place of pCN. */
int orc_tempered_cycle_pcnl(const orc_model *md, int32_t n_obs, const double *y,
                            const double *sigma, uint64_t seed, uint32_t cycle,
                            int32_t n_particles, int32_t n_steps, double ess_threshold,
                            int32_t n_bisect, double rho, int32_t n_jitter, int32_t max_temper,
                            double *m, double *u, orc_cycle_stats *st, int32_t n_threads) {
  return tempered_cycle(md, n_obs, y, sigma, seed, cycle, n_particles, n_steps, ess_threshold,
                        n_bisect, rho, n_jitter, max_temper, m, u, st, n_threads, JIT_PCNL, 0.0,
                        0);
}

/* The tempered cycle with the Hybrid Monte Carlo jitter (orc_jitter_hmc) in
 * place of pCN. */
int orc_tempered_cycle_hmc(const orc_model *md, int32_t n_obs, const double *y,
                           const double *sigma, uint64_t seed, uint32_t cycle,
                           int32_t n_particles, int32_t n_steps, double ess_threshold,
                           int32_t n_bisect, double h, int32_t n_leap, int32_t n_jitter,
                           int32_t max_temper, double *m, double *u, orc_cycle_stats *st,
                           int32_t n_threads) {
  return tempered_cycle(md, n_obs, y, sigma, seed, cycle, n_particles, n_steps, ess_threshold,
                        n_bisect, 0.0, n_jitter, max_temper, m, u, st, n_threads, JIT_HMC, h,
                        n_leap);
}

/* The linear-Gaussian plug-in of the tempering loop (declared in the header
 * with its meaning): e = F s + B xi, Phi = |G e - y|^2 / (2 sigma^2). */
typedef struct {
  int32_t ds, d, n_obs;
  const double *F, *B, *G, *y;
  double sigma;
} lin_model;

static double lin_window(const lin_model *lm, const double *s, const double *xi, double *e) {
  for (int32_t i = 0; i < lm->ds; ++i) {
    double a = 0.0;
    for (int32_t j = 0; j < lm->ds; ++j) a += lm->F[(size_t)i * lm->ds + j] * s[j];
    for (int32_t j = 0; j < lm->d; ++j) a += lm->B[(size_t)i * lm->d + j] * xi[j];
    e[i] = a;
  }
  double phi = 0.0;
  for (int32_t o = 0; o < lm->n_obs; ++o) {
    double r = -lm->y[o];
    for (int32_t i = 0; i < lm->ds; ++i) r += lm->G[(size_t)o * lm->ds + i] * e[i];
    phi += 0.5 * r * r / (lm->sigma * lm->sigma);
  }
  return phi;
}

typedef struct {
  const lin_model *lm;
  int32_t n_particles, n_steps, n_modes, n_jitter;
  double rho, dt;
  const double *x0;
  double *xi, *pot, *x;
} lin_jitter_ctx;

/* n_jitter pCN moves of every particle's increments at temperature theta, with
 * the proposal, counters and acceptance rule of orc_jitter_pcn. */
static void lin_jitter(void *vctx, const orc_rng *rg, double theta, int32_t *acc) {
  lin_jitter_ctx *c = (lin_jitter_ctx *)vctx;
  const lin_model *lm = c->lm;
  double *prop = (double *)malloc(sizeof(double) * lm->d);
  double *e = (double *)malloc(sizeof(double) * lm->ds);
  for (int32_t p = 0; p < c->n_particles; ++p) {
    double *xp = c->xi + (size_t)p * lm->d;
    acc[p] = 0;
    for (int32_t j = 0; j < c->n_jitter; ++j) {
      uint32_t w3 = (rg->temper_k << 16) | (uint32_t)j;
      orc_pcn_propose(rg->seed, (uint32_t)p, rg->cycle * (uint32_t)c->n_steps, c->n_steps,
                      c->n_modes, w3, c->rho, c->dt, xp, prop);
      double phin = lin_window(lm, c->x0 + (size_t)p * lm->ds, prop, e);
      double v = orc_uniform(rg->seed, (uint32_t)p, rg->cycle, (uint32_t)ORC_TAG_ACCEPT << 24, w3);
      if (orc_pcn_accept(theta, c->pot[p], phin, v)) {
        memcpy(xp, prop, sizeof(double) * lm->d);
        memcpy(c->x + (size_t)p * lm->ds, e, sizeof(double) * lm->ds);
        c->pot[p] = phin;
        ++acc[p];
      }
    }
  }
  free(prop);
  free(e);
}

int orc_tempered_cycle_linear(int32_t ds, int32_t n_steps, int32_t n_modes, int32_t n_obs,
                              const double *F, const double *B, const double *G, const double *y,
                              double sigma, double dt, uint64_t seed, uint32_t cycle,
                              int32_t n_particles, double ess_threshold, int32_t n_bisect,
                              double rho, int32_t n_jitter, int32_t max_temper, double *x,
                              orc_cycle_stats *st, int32_t plant) {
  if (ds <= 0 || n_steps <= 0 || n_modes <= 0 || n_obs <= 0 || n_particles <= 0) return ORC_E_ARG;
  lin_model lm = {ds, n_steps * n_modes, n_obs, F, B, G, y, sigma};
  size_t state = (size_t)n_particles * ds, wlen = (size_t)n_particles * lm.d;
  double *x0 = (double *)malloc(sizeof(double) * state);
  double *xi = (double *)malloc(sizeof(double) * wlen);
  double *pot = (double *)malloc(sizeof(double) * n_particles);
  memset(st, 0, sizeof(*st));
  memcpy(x0, x, sizeof(double) * state);
  orc_draw_increments(seed, n_particles, n_steps, n_modes, cycle * (uint32_t)n_steps,
                      ORC_TAG_FORECAST, 0u, dt, xi);
  for (int32_t p = 0; p < n_particles; ++p)
    pot[p] = lin_window(&lm, x0 + (size_t)p * ds, xi + (size_t)p * lm.d, x + (size_t)p * ds);
  row_set rows[3] = {{x0, (size_t)ds}, {x, (size_t)ds}, {xi, (size_t)lm.d}};
  lin_jitter_ctx jc = {&lm, n_particles, n_steps, n_modes, n_jitter, rho, dt, x0, xi, pot, x};
  int rc = temper_loop(n_particles, pot, rows, 3, seed, cycle, ess_threshold, n_bisect,
                       max_temper, lin_jitter, &jc, st, plant);
  st->status = rc;
  free(x0);
  free(xi);
  free(pot);
  return rc;
}

/* ========================================================================== */
/* Nudging (section 3.1.3).                                                    */
/*                                                                            */
/* A control dLambda^n in R^Q enters beside the Brownian increment in every    */
/* step (eq. "SCH nudge", modes form): dU^n = sum_q xi_q (dW^n_q + dLambda^n_q).*/
/* The objective of one window from the state (m0, u0) over n_steps steps is   */
/*   J = Phi(u^N) + sum_n ( |dLambda^n|^2 / 2 + dLambda^n . dW^n ) / dt,        */
/* i.e. the negative log-likelihood plus minus the log of the discrete         */
/* Girsanov factor (eq. "girsanov DG approx" with Lambda = dLambda / dt; the   */
/* sign follows from the ratio of the Gaussian densities of dW + dLambda       */
/* under the model and under the nudged proposal).  Minimising J maximises the */
/* weight W~ = W + G read as log-weights.                                      */
/*                                                                            */
/* Gradient.  With s = m^n + m^{n+1} the step solves                            */
/*   F(s) = A(dv) s - 2 M m^n = 0,  dv = (dt/2) R s + dU^n,  R = H^{-1} M,      */
/* where A(dv) = M + (mu dt/2) K + (1/2) C(dv).  Writing C(v) f = D(f) v,       */
/*   dF/ds = Jac = A(dv) + (dt/4) D(s) R,  dF/dm^n = -2 M,  dF/ddU = D(s)/2.    */
/* Reverse sweep: lambda_N = R^T P^T diag(1/sigma^2) (P u^N - y); per step,     */
/*   nu = Jac^{-T} lambda_{n+1},  lambda_n = 2 M nu - lambda_{n+1},             */
/*   dJ/ddU^n = -(1/2) D(s)^T nu,                                               */
/*   dJ/ddLambda^n_q = xi_q . dJ/ddU^n + (dLambda^n_q + dW^n_q) / dt.           */
/* Jac^T nu = lambda is solved by the fixed point                              */
/*   nu <- A^{-T} (lambda - (dt/4) M H^{-1} D(s)^T nu),                         */
/* each A^{-T} and H^{-1} a pivoted cyclic solve, to picard_tol.               */
/* ========================================================================== */

/* (D(f)^T w)_j = (f_{j-1} + f_j)/2 w_{j-1} - (f_j + f_{j+1})/2 w_{j+1} */
static void advect_transpose(int32_t n, const double *f, const double *w, double *out) {
  for (int32_t j = 0; j < n; ++j) {
    int32_t jm = wrap(j - 1, n), jp = wrap(j + 1, n);
    out[j] = 0.5 * (f[jm] + f[j]) * w[jm] - 0.5 * (f[j] + f[jp]) * w[jp];
  }
}

static double girsanov_term(int32_t n_steps, int32_t nq, double dt, const double *dW,
                            const double *dLam) {
  double g = 0.0;
  if (!dLam) return 0.0;
  for (int32_t i = 0; i < n_steps * nq; ++i)
    g += 0.5 * dLam[i] * dLam[i] / dt + dLam[i] * dW[i] / dt;
  return g;
}

/* P^T (P u - y) / sigma^2, scattered back to the nodes */
static void obs_adjoint(int32_t nx, int32_t n_obs, const double *u, const double *y,
                        const double *sigma, double *out) {
  double *pu = (double *)malloc(sizeof(double) * n_obs);
  orc_observe(nx, n_obs, u, pu);
  for (int32_t i = 0; i < nx; ++i) out[i] = 0.0;
  for (int32_t j = 0; j < n_obs; ++j) {
    int64_t num = (int64_t)j * nx;
    int32_t e = (int32_t)(num / n_obs);
    double r = (double)(num % n_obs) / (double)n_obs;
    double res = (pu[j] - y[j]) / (sigma[j] * sigma[j]);
    out[e % nx] += (1.0 - r) * res;
    out[(e + 1) % nx] += r * res;
  }
  free(pu);
}

int orc_nudge_objective(const orc_model *md, int32_t n_obs, const double *y, const double *sigma,
                        int32_t n_steps, const double *m0, const double *u0, const double *dW,
                        const double *dLam, double *J) {
  int32_t nx = md->nx;
  double *m = (double *)malloc(sizeof(double) * nx), *u = (double *)malloc(sizeof(double) * nx);
  memcpy(m, m0, sizeof(double) * nx);
  memcpy(u, u0, sizeof(double) * nx);
  int32_t it;
  int st = orc_window(md, n_steps, m, u, dW, dLam, &it);
  *J = orc_nll(nx, n_obs, u, y, sigma) + girsanov_term(n_steps, md->n_modes, md->dt, dW, dLam);
  free(m);
  free(u);
  return st;
}

/* rows of A(dv) */
static void step_rows(const orc_model *md, const double *dv, double *lo, double *di, double *up) {
  int32_t n = md->nx;
  double h = md->L / n, dt = md->dt, mu = md->mu;
  for (int32_t i = 0; i < n; ++i) {
    double vm = dv[wrap(i - 1, n)], vp = dv[wrap(i + 1, n)];
    lo[i] = h / 6.0 + 0.5 * mu * dt * (-1.0 / h) + 0.5 * (-0.5 * vm);
    di[i] = 2.0 * h / 3.0 + 0.5 * mu * dt * (2.0 / h) + 0.5 * (0.5 * vp - 0.5 * vm);
    up[i] = h / 6.0 + 0.5 * mu * dt * (-1.0 / h) + 0.5 * (0.5 * vp);
  }
}

/* H w = z (Helmholtz matrix, pivoted cyclic solve) */
static int helm_solve(const orc_model *md, const double *z, double *w) {
  int32_t n = md->nx;
  double h = md->L / n, a2 = md->alpha * md->alpha;
  double *lo = (double *)malloc(sizeof(double) * n), *di = (double *)malloc(sizeof(double) * n);
  double *up = (double *)malloc(sizeof(double) * n);
  for (int32_t i = 0; i < n; ++i) {
    lo[i] = h / 6.0 + a2 * (-1.0 / h);
    di[i] = 2.0 * h / 3.0 + a2 * (2.0 / h);
    up[i] = h / 6.0 + a2 * (-1.0 / h);
  }
  int st = orc_cyclic_solve(n, lo, di, up, z, w);
  free(lo);
  free(di);
  free(up);
  return st;
}

/* dU^n = sum_q xi_q (dW^n_q + dLambda^n_q) (modes form, mt == NULL), or the
 * Matern-type field of the cells dW^n + dLambda^n (eq. "SCH nudge" with the
 * noise of eq. noise_solve2). */
static int noise_field(const orc_model *md, const orc_matern *mt, const double *dW,
                       const double *dLam, double *dU) {
  int32_t n = md->nx;
  if (mt) {
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    for (int32_t i = 0; i < n; ++i) w[i] = dW[i] + (dLam ? dLam[i] : 0.0);
    int st = orc_matern_field(n, md->L, mt, w, dU);
    free(w);
    return st;
  }
  for (int32_t i = 0; i < n; ++i) dU[i] = 0.0;
  for (int32_t q = 0; q < md->n_modes; ++q) {
    double inc = dW[q] + (dLam ? dLam[q] : 0.0);
    for (int32_t i = 0; i < n; ++i) dU[i] += md->xi[(size_t)q * n + i] * inc;
  }
  return ORC_OK;
}

/* The objective and its gradient with the modes-form noise (mt == NULL,
 * controls [n_steps][n_modes]) or the Matern-type noise (controls per cell,
 * [n_steps][nx]). */
static int nudge_grad(const orc_model *md, const orc_matern *mt, int32_t n_obs, const double *y,
                      const double *sigma, int32_t n_steps, const double *m0, const double *u0,
                      const double *dW, const double *dLam, double *J, double *grad) {
  int32_t nx = md->nx, nq = mt ? md->nx : md->n_modes;
  double h = md->L / nx, dt = md->dt;
  size_t sz = sizeof(double) * nx;
  double *M = (double *)malloc(sz * (size_t)(n_steps + 1)), *U = (double *)malloc(sz * (size_t)(n_steps + 1));
  double *dUf = (double *)malloc(sz);
  memcpy(M, m0, sz);
  memcpy(U, u0, sz);
  int st = ORC_OK;
  for (int32_t n = 0; n < n_steps && st == ORC_OK; ++n) {
    memcpy(M + (size_t)(n + 1) * nx, M + (size_t)n * nx, sz);
    memcpy(U + (size_t)(n + 1) * nx, U + (size_t)n * nx, sz);
    int32_t it;
    st = noise_field(md, mt, dW + (size_t)n * nq, dLam ? dLam + (size_t)n * nq : NULL, dUf);
    if (st == ORC_OK)
      st = orc_step_field(md, M + (size_t)(n + 1) * nx, U + (size_t)(n + 1) * nx, dUf, &it);
  }
  const double *uN = U + (size_t)n_steps * nx;
  *J = orc_nll(nx, n_obs, uN, y, sigma) + girsanov_term(n_steps, nq, dt, dW, dLam);

  double *lam = (double *)malloc(sz), *tmp = (double *)malloc(sz), *tmp2 = (double *)malloc(sz);
  double *nu = (double *)malloc(sz), *nun = (double *)malloc(sz), *s = (double *)malloc(sz);
  double *dv = (double *)malloc(sz), *dU = (double *)malloc(sz), *rhs = (double *)malloc(sz);
  double *lo = (double *)malloc(sz), *di = (double *)malloc(sz), *up = (double *)malloc(sz);
  double *tlo = (double *)malloc(sz), *tup = (double *)malloc(sz), *g = (double *)malloc(sz);
  /* seed lambda_N = M H^{-1} P^T residual */
  obs_adjoint(nx, n_obs, uN, y, sigma, tmp);
  if (st == ORC_OK) st = helm_solve(md, tmp, tmp2);
  orc_apply_mass(nx, h, tmp2, lam);
  for (int32_t n = n_steps - 1; n >= 0 && st == ORC_OK; --n) {
    const double *mn = M + (size_t)n * nx, *mn1 = M + (size_t)(n + 1) * nx;
    const double *un = U + (size_t)n * nx, *un1 = U + (size_t)(n + 1) * nx;
    noise_field(md, mt, dW + (size_t)n * nq, dLam ? dLam + (size_t)n * nq : NULL, dU);
    for (int32_t i = 0; i < nx; ++i) {
      s[i] = mn[i] + mn1[i];
      dv[i] = dt * 0.5 * (un[i] + un1[i]) + dU[i];
    }
    step_rows(md, dv, lo, di, up);
    /* A^T rows: sub = up[i-1], diag = di[i], super = lo[i+1] */
    for (int32_t i = 0; i < nx; ++i) {
      tlo[i] = up[wrap(i - 1, nx)];
      tup[i] = lo[wrap(i + 1, nx)];
    }
    st = orc_cyclic_solve(nx, tlo, di, tup, lam, nu);
    int conv = 0;
    for (int32_t k = 0; k < md->picard_max && st == ORC_OK; ++k) {
      advect_transpose(nx, s, nu, tmp);
      st = helm_solve(md, tmp, tmp2);
      if (st != ORC_OK) break;
      orc_apply_mass(nx, h, tmp2, tmp);
      for (int32_t i = 0; i < nx; ++i) rhs[i] = lam[i] - 0.25 * dt * tmp[i];
      st = orc_cyclic_solve(nx, tlo, di, tup, rhs, nun);
      double diff = 0.0, scale = 0.0;
      for (int32_t i = 0; i < nx; ++i) {
        double d = fabs(nun[i] - nu[i]);
        if (d > diff) diff = d;
        if (fabs(nun[i]) > scale) scale = fabs(nun[i]);
      }
      memcpy(nu, nun, sz);
      /* the stopping rule of the forward step: the change within tolerance */
      if (diff <= md->picard_tol * scale) {
        conv = 1;
        break;
      }
    }
    if (st == ORC_OK && !conv) st = ORC_E_NONCONVERGED;
    /* gradient with respect to dU^n, then the modes or the cells */
    advect_transpose(nx, s, nu, g);
    if (mt) {
      for (int32_t i = 0; i < nx; ++i) g[i] *= -0.5;
      orc_matern_transpose(nx, md->L, mt, g, tmp2);
      for (int32_t i = 0; i < nx; ++i) {
        double l = dLam ? dLam[(size_t)n * nq + i] : 0.0;
        grad[(size_t)n * nq + i] = tmp2[i] + (l + dW[(size_t)n * nq + i]) / dt;
      }
    } else {
      for (int32_t q = 0; q < nq; ++q) {
        double acc = 0.0;
        for (int32_t i = 0; i < nx; ++i) acc += md->xi[(size_t)q * nx + i] * (-0.5 * g[i]);
        double l = dLam ? dLam[(size_t)n * nq + q] : 0.0;
        grad[(size_t)n * nq + q] = acc + (l + dW[(size_t)n * nq + q]) / dt;
      }
    }
    /* lambda_n = 2 M nu - lambda_{n+1} */
    orc_apply_mass(nx, h, nu, tmp);
    for (int32_t i = 0; i < nx; ++i) lam[i] = 2.0 * tmp[i] - lam[i];
  }
  free(M); free(U); free(lam); free(tmp); free(tmp2); free(nu); free(nun); free(s); free(dv);
  free(dU); free(rhs); free(lo); free(di); free(up); free(tlo); free(tup); free(g); free(dUf);
  return st;
}

int orc_nudge_grad(const orc_model *md, int32_t n_obs, const double *y, const double *sigma,
                   int32_t n_steps, const double *m0, const double *u0, const double *dW,
                   const double *dLam, double *J, double *grad) {
  return nudge_grad(md, NULL, n_obs, y, sigma, n_steps, m0, u0, dW, dLam, J, grad);
}

/* orc_nudge_grad with the Matern-type noise: dW, dLam and grad per cell
 * [n_steps][nx]; J carries the Girsanov term summed over the cells. */
int orc_nudge_grad_matern(const orc_model *md, const orc_matern *mt, int32_t n_obs,
                          const double *y, const double *sigma, int32_t n_steps,
                          const double *m0, const double *u0, const double *dW,
                          const double *dLam, double *J, double *grad) {
  return nudge_grad(md, mt, n_obs, y, sigma, n_steps, m0, u0, dW, dLam, J, grad);
}

/* Forward-mode (tangent-linear) gradient with dense matrices, for small nx:
 * for every control component (n0, q) the perturbation of m is propagated
 * through the linearised steps dm^{n+1} = Jac^{-1}(2 M dm^n - D(s) d(dU)/2) - dm^n
 * with Jac = A + (dt/4) D(s) H^{-1} M assembled densely and solved by dense LU.
 * Independent of the reverse sweep's transposed solves. */
int orc_nudge_grad_tangent(const orc_model *md, int32_t n_obs, const double *y,
                           const double *sigma, int32_t n_steps, const double *m0,
                           const double *u0, const double *dW, const double *dLam,
                           double *grad) {
  int32_t nx = md->nx, nq = md->n_modes;
  double h = md->L / nx, dt = md->dt;
  size_t sz = sizeof(double) * nx, sz2 = sizeof(double) * (size_t)nx * nx;
  double *M = (double *)malloc(sz * (size_t)(n_steps + 1)), *U = (double *)malloc(sz * (size_t)(n_steps + 1));
  memcpy(M, m0, sz);
  memcpy(U, u0, sz);
  int st = ORC_OK;
  for (int32_t n = 0; n < n_steps && st == ORC_OK; ++n) {
    memcpy(M + (size_t)(n + 1) * nx, M + (size_t)n * nx, sz);
    memcpy(U + (size_t)(n + 1) * nx, U + (size_t)n * nx, sz);
    int32_t it;
    st = orc_step(md, M + (size_t)(n + 1) * nx, U + (size_t)(n + 1) * nx, dW + (size_t)n * nq,
                  dLam ? dLam + (size_t)n * nq : NULL, &it);
  }
  /* dense R = H^{-1} M */
  double *R = (double *)malloc(sz2), *col = (double *)malloc(sz), *e = (double *)malloc(sz);
  double *Jm = (double *)malloc(sz2), *dm = (double *)malloc(sz), *rhs = (double *)malloc(sz);
  double *tmp = (double *)malloc(sz), *dUd = (double *)malloc(sz), *s = (double *)malloc(sz);
  double *dv = (double *)malloc(sz), *dU = (double *)malloc(sz), *lo = (double *)malloc(sz);
  double *di = (double *)malloc(sz), *up = (double *)malloc(sz), *x = (double *)malloc(sz);
  double *adjN = (double *)malloc(sz), *t2 = (double *)malloc(sz);
  for (int32_t j = 0; j < nx && st == ORC_OK; ++j) {
    for (int32_t i = 0; i < nx; ++i) e[i] = i == j ? 1.0 : 0.0;
    orc_apply_mass(nx, h, e, tmp);
    st = helm_solve(md, tmp, col);
    for (int32_t i = 0; i < nx; ++i) R[(size_t)i * nx + j] = col[i];
  }
  /* dPhi/dm^N = R^T P^T residual, as a row vector */
  obs_adjoint(nx, n_obs, U + (size_t)n_steps * nx, y, sigma, t2);
  for (int32_t j = 0; j < nx; ++j) {
    double a = 0.0;
    for (int32_t i = 0; i < nx; ++i) a += R[(size_t)i * nx + j] * t2[i];
    adjN[j] = a;
  }
  for (int32_t n0 = 0; n0 < n_steps && st == ORC_OK; ++n0)
    for (int32_t q = 0; q < nq && st == ORC_OK; ++q) {
      for (int32_t i = 0; i < nx; ++i) dm[i] = 0.0;
      for (int32_t n = n0; n < n_steps && st == ORC_OK; ++n) {
        const double *mn = M + (size_t)n * nx, *mn1 = M + (size_t)(n + 1) * nx;
        const double *un = U + (size_t)n * nx, *un1 = U + (size_t)(n + 1) * nx;
        noise_field(md, NULL, dW + (size_t)n * nq, dLam ? dLam + (size_t)n * nq : NULL, dU);
        for (int32_t i = 0; i < nx; ++i) {
          s[i] = mn[i] + mn1[i];
          dv[i] = dt * 0.5 * (un[i] + un1[i]) + dU[i];
        }
        step_rows(md, dv, lo, di, up);
        /* Jac = A + (dt/4) D(s) R, column by column: D(s) R e_j = C(R e_j) s */
        for (int32_t i = 0; i < (int32_t)((size_t)nx * nx); ++i) Jm[i] = 0.0;
        for (int32_t i = 0; i < nx; ++i) {
          Jm[(size_t)i * nx + wrap(i - 1, nx)] += lo[i];
          Jm[(size_t)i * nx + i] += di[i];
          Jm[(size_t)i * nx + wrap(i + 1, nx)] += up[i];
        }
        for (int32_t j = 0; j < nx; ++j) {
          for (int32_t i = 0; i < nx; ++i) col[i] = R[(size_t)i * nx + j];
          orc_apply_advect(nx, col, s, tmp);
          for (int32_t i = 0; i < nx; ++i) Jm[(size_t)i * nx + j] += 0.25 * dt * tmp[i];
        }
        orc_apply_mass(nx, h, dm, rhs);
        for (int32_t i = 0; i < nx; ++i) rhs[i] *= 2.0;
        if (n == n0) {
          for (int32_t i = 0; i < nx; ++i) dUd[i] = md->xi[(size_t)q * nx + i];
          orc_apply_advect(nx, dUd, s, tmp); /* C(d dU) s = D(s) d dU */
          for (int32_t i = 0; i < nx; ++i) rhs[i] -= 0.5 * tmp[i];
        }
        st = orc_dense_solve(nx, Jm, rhs, x);
        for (int32_t i = 0; i < nx; ++i) dm[i] = x[i] - dm[i];
      }
      double a = 0.0;
      for (int32_t i = 0; i < nx; ++i) a += adjN[i] * dm[i];
      double l = dLam ? dLam[(size_t)n0 * nq + q] : 0.0;
      grad[(size_t)n0 * nq + q] = a + (l + dW[(size_t)n0 * nq + q]) / dt;
    }
  free(M); free(U); free(R); free(col); free(e); free(Jm); free(dm); free(rhs); free(tmp);
  free(dUd); free(s); free(dv); free(dU); free(lo); free(di); free(up); free(x); free(adjN);
  free(t2);
  return st;
}

/* ========================================================================== */
/* L-BFGS with backtracking Armijo search.  The paper optimises the nudging    */
/* objective with BFGS through an automatic adjoint (section 3.1.3); here the  */
/* limited-memory variant (Nocedal & Wright, Algorithms 7.4/7.5):              */
/*  * stop when |g|_inf <= gtol (1 + |f|) or after max_iter accepted steps;     */
/*  * direction by the two-loop recursion over the last `mem` pairs, with      */
/*    H0 = gamma I, gamma = s.y / y.y of the newest pair, or gamma = h0 when    */
/*    no pair is stored (the caller passes dt: the inverse Hessian of the       */
/*    Girsanov term);                                                          */
/*  * a direction with g.p >= 0 drops the memory and restarts from -h0 g;      */
/*  * trial x + a p, a = 1, 1/2, ... (at most max_back halvings); accept when   */
/*    f(trial) is finite and f(trial) <= f + c1 a g.p + 1e-13 |f|, c1 = 1e-4:   */
/*    the last term lets a step pass whose decrease is below the rounding of f  */
/*    near the optimum, where the plain test fails on rounding alone;          */
/*  * the pair (s, y) is kept when s.y > 1e-10 |s|_2 |y|_2.                     */
/* The objective returns 0, or > 0 when it cannot be evaluated at x (a trial  */
/* point is then rejected like one failing the Armijo test), or < 0 for a hard */
/* error that ends the run.                                                    */
/* Status: 0 converged, 1 iteration cap, 2 line search failed, 3 objective     */
/* failed at the starting point (x unchanged), < 0 hard objective error.       */
/* ========================================================================== */
int orc_lbfgs(int32_t n, orc_objective fn, void *ctx, double *x, double h0, double gtol,
              int32_t max_iter, int32_t mem, int32_t max_back, double *f_out, int32_t *iters,
              int32_t *evals) {
  double *g = (double *)malloc(sizeof(double) * n), *p = (double *)malloc(sizeof(double) * n);
  double *xt = (double *)malloc(sizeof(double) * n), *gt = (double *)malloc(sizeof(double) * n);
  double *S = (double *)malloc(sizeof(double) * n * mem), *Y = (double *)malloc(sizeof(double) * n * mem);
  double *rho = (double *)malloc(sizeof(double) * mem), *al = (double *)malloc(sizeof(double) * mem);
  int32_t head = 0, count = 0, k = 0, ne = 0, status = 1;
  double f;
  int st = fn(ctx, x, &f, g);
  ++ne;
  if (st != 0) status = st < 0 ? st : 3;
  while (st == 0) {
    double gmax = 0.0;
    for (int32_t i = 0; i < n; ++i) gmax = fmax(gmax, fabs(g[i]));
    if (gmax <= gtol * (1.0 + fabs(f))) {
      status = 0;
      break;
    }
    if (k >= max_iter) {
      status = 1;
      break;
    }
    /* two-loop recursion: newest pair first, then oldest first */
    for (int32_t i = 0; i < n; ++i) p[i] = -g[i];
    for (int32_t c = 0; c < count; ++c) {
      int32_t j = (head - 1 - c + mem) % mem;
      double d = 0.0;
      for (int32_t i = 0; i < n; ++i) d += S[j * n + i] * p[i];
      al[j] = rho[j] * d;
      for (int32_t i = 0; i < n; ++i) p[i] -= al[j] * Y[j * n + i];
    }
    double gamma = h0;
    if (count > 0) {
      int32_t j = (head - 1 + mem) % mem;
      double sy = 0.0, yy = 0.0;
      for (int32_t i = 0; i < n; ++i) {
        sy += S[j * n + i] * Y[j * n + i];
        yy += Y[j * n + i] * Y[j * n + i];
      }
      gamma = sy / yy;
    }
    for (int32_t i = 0; i < n; ++i) p[i] *= gamma;
    for (int32_t c = count - 1; c >= 0; --c) {
      int32_t j = (head - 1 - c + mem) % mem;
      double d = 0.0;
      for (int32_t i = 0; i < n; ++i) d += Y[j * n + i] * p[i];
      double b = rho[j] * d;
      for (int32_t i = 0; i < n; ++i) p[i] += (al[j] - b) * S[j * n + i];
    }
    double gp = 0.0;
    for (int32_t i = 0; i < n; ++i) gp += g[i] * p[i];
    if (!(gp < 0.0)) {
      count = 0;
      head = 0;
      gp = 0.0;
      for (int32_t i = 0; i < n; ++i) {
        p[i] = -h0 * g[i];
        gp += g[i] * p[i];
      }
    }
    /* backtracking */
    double a = 1.0, ft = 0.0;
    int accepted = 0;
    for (int32_t b = 0; b <= max_back; ++b) {
      for (int32_t i = 0; i < n; ++i) xt[i] = x[i] + a * p[i];
      st = fn(ctx, xt, &ft, gt);
      ++ne;
      if (st < 0) break;
      if (st == 0 && isfinite(ft) && ft <= f + 1e-4 * a * gp + 1e-13 * fabs(f)) {
        accepted = 1;
        break;
      }
      st = 0;
      a *= 0.5;
    }
    if (st < 0) {
      status = st;
      break;
    }
    if (!accepted) {
      status = 2;
      break;
    }
    double sy = 0.0, ss = 0.0, yy = 0.0;
    for (int32_t i = 0; i < n; ++i) {
      double si = xt[i] - x[i], yi = gt[i] - g[i];
      S[head * n + i] = si;
      Y[head * n + i] = yi;
      sy += si * yi;
      ss += si * si;
      yy += yi * yi;
    }
    if (sy > 1e-10 * sqrt(ss) * sqrt(yy)) {
      rho[head] = 1.0 / sy;
      head = (head + 1) % mem;
      if (count < mem) ++count;
    }
    memcpy(x, xt, sizeof(double) * n);
    memcpy(g, gt, sizeof(double) * n);
    f = ft;
    ++k;
  }
  *f_out = f;
  if (iters) *iters = k;
  if (evals) *evals = ne;
  free(g); free(p); free(xt); free(gt); free(S); free(Y); free(rho); free(al);
  return status;
}

/* Objective of one adapted stage: from (m, u) run `n_steps` steps with zero
 * Brownian increments, the control x in the first step only and zero control
 * afterwards; f = Phi(u^N) + |x|^2 / (2 dt). */
typedef struct {
  const orc_model *md;
  const orc_matern *mt;
  int32_t n_obs, n_steps, nq;
  const double *y, *sigma, *m, *u;
  double *dW, *dLam, *grad;
} stage_ctx;

static int stage_objective(void *vctx, const double *x, double *f, double *g) {
  stage_ctx *c = (stage_ctx *)vctx;
  int32_t nq = c->nq;
  memcpy(c->dLam, x, sizeof(double) * nq);
  int st = nudge_grad(c->md, c->mt, c->n_obs, c->y, c->sigma, c->n_steps, c->m, c->u, c->dW,
                      c->dLam, f, c->grad);
  memcpy(g, c->grad, sizeof(double) * nq);
  return st == ORC_OK ? 0 : 1; /* any failure rejects the point */
}

/* Sequential adapted nudging of one particle over a window (section 3.1.3,
 * the stage-by-stage scheme): for each step n the control dLambda^n is
 * optimised with the later increments and controls set to zero, then the
 * increment dW^n is revealed and the state advanced with dW^n + dLambda^n.
 * dLam holds the warm start on entry and the controls on exit; logG is the
 * log Girsanov factor of the realised path. */
static int nudge_particle(const orc_model *md, const orc_matern *mt, int32_t n_obs,
                          const double *y, const double *sigma, int32_t n_steps, double *m,
                          double *u, const double *dW, double *dLam, const orc_lbfgs_opts *opt,
                          double *logG, int32_t *iters_total, int32_t *evals_total,
                          int32_t *worst_status) {
  int32_t nx = md->nx, nq = mt ? md->nx : md->n_modes;
  stage_ctx c;
  c.md = md;
  c.mt = mt;
  c.nq = nq;
  c.n_obs = n_obs;
  c.y = y;
  c.sigma = sigma;
  c.m = m;
  c.u = u;
  c.dW = (double *)calloc((size_t)n_steps * nq, sizeof(double));
  c.dLam = (double *)calloc((size_t)n_steps * nq, sizeof(double));
  c.grad = (double *)calloc((size_t)n_steps * nq, sizeof(double));
  double lg = 0.0;
  int32_t it_tot = 0, ev_tot = 0, worst = 0;
  int st = ORC_OK;
  for (int32_t n = 0; n < n_steps; ++n) {
    c.n_steps = n_steps - n;
    double *x = dLam + (size_t)n * nq, f;
    int32_t it = 0, ev = 0;
    int ls = orc_lbfgs(nq, stage_objective, &c, x, md->dt, opt->gtol, opt->max_iter, opt->mem,
                       opt->max_back, &f, &it, &ev);
    it_tot += it;
    ev_tot += ev;
    if (ls < 0) {
      st = ls;
      break;
    }
    if (ls > worst) worst = ls;
    int32_t pit;
    double *dUs = (double *)malloc(sizeof(double) * (size_t)nx);
    st = noise_field(md, mt, dW + (size_t)n * nq, x, dUs);
    if (st == ORC_OK) st = orc_step_field(md, m, u, dUs, &pit);
    free(dUs);
    if (st != ORC_OK) break;
    for (int32_t q = 0; q < nq; ++q)
      lg -= 0.5 * x[q] * x[q] / md->dt + x[q] * dW[(size_t)n * nq + q] / md->dt;
  }
  (void)nx;
  free(c.dW);
  free(c.dLam);
  free(c.grad);
  *logG = lg;
  if (iters_total) *iters_total = it_tot;
  if (evals_total) *evals_total = ev_tot;
  if (worst_status) *worst_status = worst;
  return st;
}

int orc_nudge_particle(const orc_model *md, int32_t n_obs, const double *y, const double *sigma,
                       int32_t n_steps, double *m, double *u, const double *dW, double *dLam,
                       const orc_lbfgs_opts *opt, double *logG, int32_t *iters_total,
                       int32_t *evals_total, int32_t *worst_status) {
  return nudge_particle(md, NULL, n_obs, y, sigma, n_steps, m, u, dW, dLam, opt, logG,
                        iters_total, evals_total, worst_status);
}

/* mode (NULL: every particle nudged from the controls in dLam) selects per
 * particle how its stages start: ORC_NUDGE_KEEP uses the controls in dLam as
 * they are (no L-BFGS steps), ORC_NUDGE_FROM_GIVEN runs the stages' L-BFGS
 * from them, ORC_NUDGE_FROM_ZERO zeroes them first. */
static int nudge_ensemble_modes(const orc_model *md, const orc_matern *mt, int32_t n_obs,
                                const double *y, const double *sigma, int32_t n_particles,
                                int32_t n_steps, double *m, double *u, const double *dW,
                                double *dLam, const int32_t *mode, const orc_lbfgs_opts *opt,
                                double *logG, int32_t *iters, int32_t *evals,
                                int32_t *lbfgs_status, int32_t *status, int32_t n_threads) {
  int32_t nx = md->nx, nq = mt ? md->nx : md->n_modes;
  int worst = ORC_OK;
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads > 0 ? n_threads : 1)
  for (int32_t p = 0; p < n_particles; ++p) {
    int32_t mp = mode ? mode[p] : ORC_NUDGE_FROM_GIVEN;
    double *lam = dLam + (size_t)p * n_steps * nq;
    orc_lbfgs_opts op = *opt;
    if (mp == ORC_NUDGE_FROM_ZERO) memset(lam, 0, sizeof(double) * (size_t)n_steps * nq);
    if (mp == ORC_NUDGE_KEEP) op.max_iter = 0;
    int st = nudge_particle(md, mt, n_obs, y, sigma, n_steps, m + (size_t)p * nx,
                            u + (size_t)p * nx, dW + (size_t)p * n_steps * nq, lam, &op,
                            logG + p, iters ? iters + p : NULL, evals ? evals + p : NULL,
                            lbfgs_status ? lbfgs_status + p : NULL);
    if (status) status[p] = st;
    if (st != ORC_OK) {
#pragma omp critical
      if (worst == ORC_OK) worst = st;
    }
  }
  return worst;
}

static int nudge_ensemble(const orc_model *md, const orc_matern *mt, int32_t n_obs,
                          const double *y, const double *sigma, int32_t n_particles,
                          int32_t n_steps, double *m, double *u, const double *dW, double *dLam,
                          const orc_lbfgs_opts *opt, double *logG, int32_t *iters, int32_t *evals,
                          int32_t *lbfgs_status, int32_t *status, int32_t n_threads) {
  return nudge_ensemble_modes(md, mt, n_obs, y, sigma, n_particles, n_steps, m, u, dW, dLam,
                              NULL, opt, logG, iters, evals, lbfgs_status, status, n_threads);
}

int orc_nudge_ensemble(const orc_model *md, int32_t n_obs, const double *y, const double *sigma,
                       int32_t n_particles, int32_t n_steps, double *m, double *u, const double *dW,
                       double *dLam, const orc_lbfgs_opts *opt, double *logG, int32_t *iters,
                       int32_t *evals, int32_t *lbfgs_status, int32_t *status, int32_t n_threads) {
  return nudge_ensemble(md, NULL, n_obs, y, sigma, n_particles, n_steps, m, u, dW, dLam, opt,
                        logG, iters, evals, lbfgs_status, status, n_threads);
}

/* Sequential adapted nudging with the Matern-type noise: controls per cell,
 * dW and dLam [n][n_steps][nx]; otherwise as orc_nudge_ensemble. */
int orc_nudge_ensemble_matern(const orc_model *md, const orc_matern *mt, int32_t n_obs,
                              const double *y, const double *sigma, int32_t n_particles,
                              int32_t n_steps, double *m, double *u, const double *dW,
                              double *dLam, const orc_lbfgs_opts *opt, double *logG,
                              int32_t *iters, int32_t *evals, int32_t *lbfgs_status,
                              int32_t *status, int32_t n_threads) {
  return nudge_ensemble(md, mt, n_obs, y, sigma, n_particles, n_steps, m, u, dW, dLam, opt, logG,
                        iters, evals, lbfgs_status, status, n_threads);
}

/* ========================================================================== */
/* Nudged filter: section 3.1.3 followed by the tempering and jittering of    */
/* section 3.1.2 with W replaced by W~ (last paragraph of section 3.1.3).     */
/* ========================================================================== */

static int jitter_matern(const orc_model *md, const orc_matern *mt, int32_t n_obs,
                         const double *y, const double *sigma, const orc_rng *rng,
                         int32_t n_particles, int32_t n_steps, const double *m0, const double *u0,
                         double *dWc, const double *dLamc, double *phi, double *m_end,
                         double *u_end, double theta, double rho, int32_t n_jitter,
                         int32_t *n_accept, int32_t n_threads);

/* One assimilation cycle: the increments of the window are drawn (tag
 * NUDGE) and revealed stage by stage to the sequential nudging of every
 * particle (orc_nudge_particle from zero controls); each particle gets the
 * potential J = phi(u_end) - log G of its nudged path; the temperature then
 * rises from 0 to 1 in adaptive steps on the weights exp(-dtheta J) (as in
 * orc_tempered_cycle); after each step the particles are resampled
 * (window-start state, increments, controls, J, window-end state) and their
 * increments jittered by n_jitter pCN moves with the controls fixed.
 * On return m, u hold the window-end states; the optional outputs (NULL to
 * skip) receive the final window-start states m0_out, u0_out [n][nx], the
 * increments dW_out and controls dLam_out [n][n_steps][n_modes] and the
 * potentials J_out [n].  st->n_accept counts accepted pCN moves;
 * st->picard_iters is not filled. */
static int nudged_cycle(const orc_model *md, const orc_matern *mt, int32_t n_obs,
                        const double *y, const double *sigma, uint64_t seed, uint32_t cycle,
                        int32_t n_particles, int32_t n_steps, double ess_threshold,
                        int32_t n_bisect, double rho, int32_t n_jitter, int32_t max_temper,
                        const orc_lbfgs_opts *opt, const double *dLam_start,
                        const int32_t *mode, double *m, double *u, double *m0_out,
                        double *u0_out, double *dW_out, double *dLam_out, double *J_out,
                        orc_cycle_stats *st, int32_t n_threads) {
  int32_t nx = md->nx, nq = mt ? md->nx : md->n_modes;
  size_t state = (size_t)n_particles * nx, wlen = (size_t)n_particles * n_steps * nq;
  double *m0 = (double *)malloc(sizeof(double) * state), *u0 = (double *)malloc(sizeof(double) * state);
  double *dW = (double *)malloc(sizeof(double) * wlen);
  double *dLam = (double *)calloc(wlen, sizeof(double));
  double *J = (double *)malloc(sizeof(double) * n_particles);
  double *logG = (double *)malloc(sizeof(double) * n_particles);
  int32_t *stat = (int32_t *)malloc(sizeof(int32_t) * n_particles);
  memset(st, 0, sizeof(*st));
  memcpy(m0, m, sizeof(double) * state);
  memcpy(u0, u, sizeof(double) * state);

  orc_draw_increments(seed, n_particles, n_steps, nq, cycle * (uint32_t)n_steps, ORC_TAG_NUDGE,
                      0u, md->dt, dW);
  if (dLam_start) memcpy(dLam, dLam_start, sizeof(double) * wlen);
  nudge_ensemble_modes(md, mt, n_obs, y, sigma, n_particles, n_steps, m, u, dW, dLam,
                       dLam_start ? mode : NULL, opt, logG, NULL, NULL, NULL, stat, n_threads);
  for (int32_t p = 0; p < n_particles; ++p) {
    double phi = stat[p] == ORC_OK ? orc_nll(nx, n_obs, u + (size_t)p * nx, y, sigma) : INFINITY;
    J[p] = (isfinite(phi) && isfinite(logG[p])) ? phi - logG[p] : INFINITY;
    if (!isfinite(J[p])) J[p] = INFINITY;
  }
  row_set rows[6] = {{m0, (size_t)nx}, {u0, (size_t)nx}, {m, (size_t)nx}, {u, (size_t)nx},
                     {dW, (size_t)n_steps * nq}, {dLam, (size_t)n_steps * nq}};
  sch_jitter_ctx jc = {mt ? JIT_MATERN : JIT_PCN_CTRL, md, mt, n_obs, n_particles, n_steps,
                       n_jitter, n_threads, y, sigma, m0, u0, dLam, dW, J, m, u, rho, 0.0, 0};
  int rc = temper_loop(n_particles, J, rows, 6, seed, cycle, ess_threshold, n_bisect, max_temper,
                       sch_jitter, &jc, st, ORC_PLANT_NONE);
  st->status = rc;
  if (m0_out) memcpy(m0_out, m0, sizeof(double) * state);
  if (u0_out) memcpy(u0_out, u0, sizeof(double) * state);
  if (dW_out) memcpy(dW_out, dW, sizeof(double) * wlen);
  if (dLam_out) memcpy(dLam_out, dLam, sizeof(double) * wlen);
  if (J_out) memcpy(J_out, J, sizeof(double) * n_particles);
  free(m0);
  free(u0);
  free(dW);
  free(dLam);
  free(J);
  free(logG);
  free(stat);
  return rc;
}

int orc_nudged_cycle(const orc_model *md, int32_t n_obs, const double *y, const double *sigma,
                     uint64_t seed, uint32_t cycle, int32_t n_particles, int32_t n_steps,
                     double ess_threshold, int32_t n_bisect, double rho, int32_t n_jitter,
                     int32_t max_temper, const orc_lbfgs_opts *opt, double *m, double *u,
                     double *m0_out, double *u0_out, double *dW_out, double *dLam_out,
                     double *J_out, orc_cycle_stats *st, int32_t n_threads) {
  return nudged_cycle(md, NULL, n_obs, y, sigma, seed, cycle, n_particles, n_steps, ess_threshold,
                      n_bisect, rho, n_jitter, max_temper, opt, NULL, NULL, m, u, m0_out, u0_out,
                      dW_out, dLam_out, J_out, st, n_threads);
}

int orc_nudged_cycle_warm(const orc_model *md, int32_t n_obs, const double *y,
                          const double *sigma, uint64_t seed, uint32_t cycle, int32_t n_particles,
                          int32_t n_steps, double ess_threshold, int32_t n_bisect, double rho,
                          int32_t n_jitter, int32_t max_temper, const orc_lbfgs_opts *opt,
                          const double *dLam_start, const int32_t *mode, double *m, double *u,
                          double *m0_out, double *u0_out, double *dW_out, double *dLam_out,
                          double *J_out, orc_cycle_stats *st, int32_t n_threads) {
  if (!dLam_start || !mode) return ORC_E_ARG;
  for (int32_t p = 0; p < n_particles; ++p)
    if (mode[p] < ORC_NUDGE_KEEP || mode[p] > ORC_NUDGE_FROM_ZERO) return ORC_E_ARG;
  return nudged_cycle(md, NULL, n_obs, y, sigma, seed, cycle, n_particles, n_steps, ess_threshold,
                      n_bisect, rho, n_jitter, max_temper, opt, dLam_start, mode, m, u, m0_out,
                      u0_out, dW_out, dLam_out, J_out, st, n_threads);
}

/* orc_nudged_cycle with the Matern-type noise: the NUDGE-tag draws, the
 * controls and the jitter act on the cells ([n][n_steps][nx]); the window,
 * its gradient and the pCN moves use the Matern field of dW + dLam. */
int orc_nudged_cycle_matern(const orc_model *md, const orc_matern *mt, int32_t n_obs,
                            const double *y, const double *sigma, uint64_t seed, uint32_t cycle,
                            int32_t n_particles, int32_t n_steps, double ess_threshold,
                            int32_t n_bisect, double rho, int32_t n_jitter, int32_t max_temper,
                            const orc_lbfgs_opts *opt, double *m, double *u, double *m0_out,
                            double *u0_out, double *dW_out, double *dLam_out, double *J_out,
                            orc_cycle_stats *st, int32_t n_threads) {
  return nudged_cycle(md, mt, n_obs, y, sigma, seed, cycle, n_particles, n_steps, ess_threshold,
                      n_bisect, rho, n_jitter, max_temper, opt, NULL, NULL, m, u, m0_out, u0_out,
                      dW_out, dLam_out, J_out, st, n_threads);
}

/* ========================================================================== */
/* Tempered + jittered filter with the Matern-type noise of section 2: the     */
/* increments are the cell values Delta W_i of the DG0 white noise per step    */
/* ([n][n_steps][nx], N(0, dt) each), drawn, resampled and moved by pCN        */
/* exactly as the mode increments of orc_tempered_cycle (the pCN proposal and  */
/* its counters with nx in place of the number of modes).                      */
/* ========================================================================== */
/* pCN moves of the cell increments; with controls lam (the nudged filter,
 * section 3.1.3) the window runs with the cells dW' + lam and the potential is
 * the nudged J of orc_nudged_potential summed over the cells, as in
 * orc_jitter_pcn_ctrl. */
static int jitter_matern(const orc_model *md, const orc_matern *mt, int32_t n_obs,
                         const double *y, const double *sigma, const orc_rng *rng,
                         int32_t n_particles, int32_t n_steps, const double *m0, const double *u0,
                         double *dWc, const double *dLamc, double *phi, double *m_end,
                         double *u_end, double theta, double rho, int32_t n_jitter,
                         int32_t *n_accept, int32_t n_threads) {
  int32_t nx = md->nx;
#pragma omp parallel for num_threads(n_threads > 0 ? n_threads : 1) schedule(dynamic, 1)
  for (int32_t p = 0; p < n_particles; ++p) {
    size_t wlen = (size_t)n_steps * nx;
    double *prop = (double *)malloc(sizeof(double) * wlen);
    double *cells = dLamc ? (double *)malloc(sizeof(double) * wlen) : prop;
    double *mm = (double *)malloc(sizeof(double) * nx);
    double *uu = (double *)malloc(sizeof(double) * nx);
    double *cur = dWc + (size_t)p * wlen;
    const double *lam = dLamc ? dLamc + (size_t)p * wlen : NULL;
    int32_t acc = 0;
    for (int32_t j = 0; j < n_jitter; ++j) {
      uint32_t w3 = (rng->temper_k << 16) | (uint32_t)j;
      orc_pcn_propose(rng->seed, (uint32_t)p, rng->cycle * (uint32_t)n_steps, n_steps, nx, w3,
                      rho, md->dt, cur, prop);
      if (lam)
        for (size_t i = 0; i < wlen; ++i) cells[i] = prop[i] + lam[i];
      memcpy(mm, m0 + (size_t)p * nx, sizeof(double) * nx);
      memcpy(uu, u0 + (size_t)p * nx, sizeof(double) * nx);
      int32_t it = 0;
      int st = orc_window_matern(md, mt, n_steps, mm, uu, cells, &it);
      double phi_new = st == ORC_OK ? orc_nll(nx, n_obs, uu, y, sigma) : INFINITY;
      if (!isfinite(phi_new)) phi_new = INFINITY;
      if (lam) phi_new = orc_nudged_potential(phi_new, (int32_t)wlen, md->dt, prop, lam);
      double v = orc_uniform(rng->seed, (uint32_t)p, rng->cycle,
                             (uint32_t)ORC_TAG_ACCEPT << 24, w3);
      if (orc_pcn_accept(theta, phi[p], phi_new, v)) {
        memcpy(cur, prop, sizeof(double) * wlen);
        phi[p] = phi_new;
        memcpy(m_end + (size_t)p * nx, mm, sizeof(double) * nx);
        memcpy(u_end + (size_t)p * nx, uu, sizeof(double) * nx);
        ++acc;
      }
    }
    if (n_accept) n_accept[p] = acc;
    if (cells != prop) free(cells);
    free(prop);
    free(mm);
    free(uu);
  }
  return ORC_OK;
}

int orc_jitter_pcn_matern(const orc_model *md, const orc_matern *mt, int32_t n_obs,
                          const double *y, const double *sigma, const orc_rng *rng,
                          int32_t n_particles, int32_t n_steps, const double *m0,
                          const double *u0, double *dWc, double *phi, double *m_end,
                          double *u_end, double theta, double rho, int32_t n_jitter,
                          int32_t *n_accept, int32_t n_threads) {
  return jitter_matern(md, mt, n_obs, y, sigma, rng, n_particles, n_steps, m0, u0, dWc, NULL,
                       phi, m_end, u_end, theta, rho, n_jitter, n_accept, n_threads);
}

int orc_jitter_pcn_matern_ctrl(const orc_model *md, const orc_matern *mt, int32_t n_obs,
                               const double *y, const double *sigma, const orc_rng *rng,
                               int32_t n_particles, int32_t n_steps, const double *m0,
                               const double *u0, double *dWc, const double *dLamc, double *J,
                               double *m_end, double *u_end, double theta, double rho,
                               int32_t n_jitter, int32_t *n_accept, int32_t n_threads) {
  return jitter_matern(md, mt, n_obs, y, sigma, rng, n_particles, n_steps, m0, u0, dWc, dLamc, J,
                       m_end, u_end, theta, rho, n_jitter, n_accept, n_threads);
}

/* One cycle: draw the cell increments (tag FORECAST, counter (p, cycle *
 * n_steps + n, pair | tag << 24, 0)), run the window, then temper, resample
 * (window-start state, increments, phi, window-end state) and jitter as
 * orc_tempered_cycle.  Optional outputs (NULL to skip): the final
 * window-start states m0_out, u0_out, increments dWc_out and phi_out. */
int orc_tempered_cycle_matern(const orc_model *md, const orc_matern *mt, int32_t n_obs,
                              const double *y, const double *sigma, uint64_t seed, uint32_t cycle,
                              int32_t n_particles, int32_t n_steps, double ess_threshold,
                              int32_t n_bisect, double rho, int32_t n_jitter, int32_t max_temper,
                              double *m, double *u, double *m0_out, double *u0_out,
                              double *dWc_out, double *phi_out, orc_cycle_stats *st,
                              int32_t n_threads) {
  int32_t nx = md->nx;
  size_t state = (size_t)n_particles * nx, wlen = (size_t)n_particles * n_steps * nx;
  double *m0 = (double *)malloc(sizeof(double) * state), *u0 = (double *)malloc(sizeof(double) * state);
  double *dWc = (double *)malloc(sizeof(double) * wlen);
  double *phi = (double *)malloc(sizeof(double) * n_particles);
  int32_t *iters = (int32_t *)malloc(sizeof(int32_t) * n_particles);
  int32_t *stat = (int32_t *)malloc(sizeof(int32_t) * n_particles);
  memset(st, 0, sizeof(*st));
  memcpy(m0, m, sizeof(double) * state);
  memcpy(u0, u, sizeof(double) * state);
  orc_draw_increments(seed, n_particles, n_steps, nx, cycle * (uint32_t)n_steps, ORC_TAG_FORECAST,
                      0u, md->dt, dWc);
  orc_ensemble_window_matern(md, mt, n_particles, n_steps, m, u, dWc, stat, iters, n_threads);
  for (int32_t p = 0; p < n_particles; ++p) {
    st->picard_iters += iters[p];
    phi[p] = stat[p] == ORC_OK ? orc_nll(nx, n_obs, u + (size_t)p * nx, y, sigma) : INFINITY;
    if (!isfinite(phi[p])) phi[p] = INFINITY;
  }
  row_set rows[5] = {{m0, (size_t)nx}, {u0, (size_t)nx}, {m, (size_t)nx}, {u, (size_t)nx},
                     {dWc, (size_t)n_steps * nx}};
  sch_jitter_ctx jc = {JIT_MATERN, md, mt, n_obs, n_particles, n_steps, n_jitter, n_threads, y,
                       sigma, m0, u0, NULL, dWc, phi, m, u, rho, 0.0, 0};
  int rc = temper_loop(n_particles, phi, rows, 5, seed, cycle, ess_threshold, n_bisect,
                       max_temper, sch_jitter, &jc, st, ORC_PLANT_NONE);
  st->status = rc;
  if (m0_out) memcpy(m0_out, m0, sizeof(double) * state);
  if (u0_out) memcpy(u0_out, u0, sizeof(double) * state);
  if (dWc_out) memcpy(dWc_out, dWc, sizeof(double) * wlen);
  if (phi_out) memcpy(phi_out, phi, sizeof(double) * n_particles);
  free(m0);
  free(u0);
  free(dWc);
  free(phi);
  free(iters);
  free(stat);
  return rc;
}

/* ========================================================================== */
/* The paper's twin experiments (section 4).                                  */
/* ========================================================================== */
/* Initial velocity of eq. init_solve from given draws: W [nx] holds the DG0
 * cell values (N(0, h) samples), U^{0,1} solves (I - d_xx) U = |W| in the P1
 * weak form, (M + K) U_1 = b with b_n = (|W|, phi_n) = h (|W_{n-1}| + |W_n|)
 * / 2, then (M + K) U_{j+1} = M U_j twice; u = alpha^2 U^{0,3} + beta^2.  This
 * is the Matern-type field with kappa = 1, k = 3 and eta sqrt(h) = h. */
int orc_paper_init_from(int32_t nx, double L, const double *W, double alpha, double beta,
                        double *u) {
  double h = L / nx;
  orc_matern mt = {1.0, sqrt(h), 3};
  double *aw = (double *)calloc((size_t)nx, sizeof(double));
  for (int32_t i = 0; i < nx; ++i) aw[i] = fabs(W[i]);
  int st = orc_matern_field(nx, L, &mt, aw, u);
  for (int32_t i = 0; i < nx; ++i) u[i] = alpha * alpha * u[i] + beta * beta;
  free(aw);
  return st;
}

/* Particles p0 .. p0 + n - 1 of the paper's initial ensemble: the cell values
 * W_i = sqrt(h) z with z from tag INIT, counter (p, 0, pair | tag << 24, 0)
 * (cells 2k, 2k+1 share a block), and (alpha, beta) the pair of counter
 * (p, 1, tag << 24, 0).  u [n][nx]. */
int orc_paper_init(int32_t nx, double L, uint64_t seed, int32_t p0, int32_t n, double *u) {
  double h = L / nx;
  double *W = (double *)malloc(sizeof(double) * (size_t)nx);
  int st = ORC_OK;
  for (int32_t p = 0; p < n && st == ORC_OK; ++p) {
    orc_draw_increments_rows(seed, p0 + p, 1, 1, nx, 0u, ORC_TAG_INIT, 0u, h, W);
    double ab[2];
    orc_normal_pair(seed, (uint32_t)(p0 + p), 1u, (uint32_t)ORC_TAG_INIT << 24, 0u, ab);
    st = orc_paper_init_from(nx, L, W, ab[0], ab[1], u + (size_t)p * nx);
  }
  free(W);
  return st;
}

/* Ensemble statistics of section 4 against the truth ua [nx], with the nodal
 * Euclidean norm: out[0] = EMRE = (1/N) sum_n |ua - u_n| / |ua|,
 * out[1] = RB = |ua - mean_n u_n| / |ua|,
 * out[2] = RES = (1/(N-1)) sum_n |u_n - mean u| / |ua| (N > 1; 0 for N = 1). */
void orc_ensemble_stats(int32_t n, int32_t nx, const double *u, const double *ua, double *out) {
  double *mean = (double *)calloc((size_t)nx, sizeof(double));
  for (int32_t p = 0; p < n; ++p)
    for (int32_t i = 0; i < nx; ++i) mean[i] += u[(size_t)p * nx + i];
  for (int32_t i = 0; i < nx; ++i) mean[i] /= n;
  long double na = 0.0L, nb = 0.0L, se = 0.0L, ss = 0.0L;
  for (int32_t i = 0; i < nx; ++i) {
    na += (long double)ua[i] * ua[i];
    nb += (long double)(ua[i] - mean[i]) * (ua[i] - mean[i]);
  }
  for (int32_t p = 0; p < n; ++p) {
    long double a = 0.0L, b = 0.0L;
    for (int32_t i = 0; i < nx; ++i) {
      double d = ua[i] - u[(size_t)p * nx + i], e = u[(size_t)p * nx + i] - mean[i];
      a += (long double)d * d;
      b += (long double)e * e;
    }
    se += sqrtl(a);
    ss += sqrtl(b);
  }
  long double nrm = sqrtl(na);
  out[0] = (double)(se / n / nrm);
  out[1] = (double)(sqrtl(nb) / nrm);
  out[2] = n > 1 ? (double)(ss / (n - 1) / nrm) : 0.0;
  free(mean);
}

/* ========================================================================== */
/* Gradient-based jitter: the preconditioned Crank-Nicolson Langevin move      */
/* (pCNL; Cotter, Roberts, Stuart & White, Statist. Sci. 2013) on the          */
/* increments x of a particle, prior N(0, dt I), target proportional to        */
/* exp(-theta Phi(x)) N(x; 0, dt I).  The Crank-Nicolson step of the           */
/* preconditioned Langevin equation gives the proposal                         */
/*   v = rho x + sqrt(1 - rho^2) sqrt(dt) z - (1 - rho) dt theta grad Phi(x),  */
/* with rho = (2 - delta)/(2 + delta) as for pCN (the pCN proposal plus a      */
/* drift), and the move is accepted with the Metropolis-Hastings probability   */
/* min(1, pi(v) q(v -> x) / (pi(x) q(x -> v))), q(x -> v) the Gaussian density */
/* of the proposal: N(v; rho x - (1 - rho) dt theta grad Phi(x), (1 - rho^2) dt I).*/
/* The paper names MALA/HMC jittering as future work (section 5).              */
/* ========================================================================== */
static double pcnl_log_q(int32_t d, const double *from, const double *to, const double *g_from,
                         double rho, double dt, double theta) {
  long double s = 0.0L;
  for (int32_t i = 0; i < d; ++i) {
    double r = to[i] - (rho * from[i] - (1.0 - rho) * dt * theta * g_from[i]);
    s += (long double)r * r;
  }
  return (double)(-s / (2.0L * (1.0L - (long double)rho * rho) * dt));
}

static double pcnl_log_target(int32_t d, const double *x, double phi, double theta, double dt) {
  long double s = 0.0L;
  for (int32_t i = 0; i < d; ++i) s += (long double)x[i] * x[i];
  return (double)(-(long double)theta * phi - s / (2.0L * dt));
}

/* log of the acceptance ratio of the move x -> v (phi and grad Phi at both). */
double orc_pcnl_log_ratio(int32_t d, const double *x, double phi_x, const double *g_x,
                          const double *v, double phi_v, const double *g_v, double theta,
                          double rho, double dt) {
  return pcnl_log_target(d, v, phi_v, theta, dt) + pcnl_log_q(d, v, x, g_v, rho, dt, theta) -
         pcnl_log_target(d, x, phi_x, theta, dt) - pcnl_log_q(d, x, v, g_x, rho, dt, theta);
}

/* accept iff the ratio is finite and (log r >= 0 or u < exp(log r)) */
static int pcnl_accept(double logr, double u) {
  if (!(logr > -INFINITY) || logr != logr) return 0;
  if (logr >= 0.0) return 1;
  return u < exp(logr);
}

/* The linear-Gaussian toy of orc_pcn_linear_chain moved by pCNL: Phi(x) =
 * |G x - y|^2 / (2 sigma^2), grad Phi = G^T (G x - y) / sigma^2 exactly;
 * proposals and uniforms with the same counters. */
int64_t orc_pcnl_linear_chain(uint64_t seed, int32_t n_steps, int32_t n_modes, int32_t n_obs,
                              const double *G, const double *y, double sigma, double theta,
                              double rho, double dt, int32_t n_iter, const double *x0,
                              double *samples) {
  int32_t d = n_steps * n_modes;
  double *x = (double *)malloc(sizeof(double) * d), *v = (double *)malloc(sizeof(double) * d);
  double *gx = (double *)calloc((size_t)d, sizeof(double)), *gv = (double *)calloc((size_t)d, sizeof(double));
  double *res = (double *)malloc(sizeof(double) * (n_obs > 0 ? n_obs : 1));
  memcpy(x, x0, sizeof(double) * d);
  /* Phi and its gradient at a point */
#define TOY_EVAL(pt, phi_out, g_out)                                        \
  do {                                                                      \
    double acc_ = 0.0;                                                      \
    for (int32_t j = 0; j < n_obs; ++j) {                                   \
      double r = -y[j];                                                     \
      for (int32_t i = 0; i < d; ++i) r += G[(size_t)j * d + i] * (pt)[i];  \
      res[j] = r;                                                           \
      acc_ += 0.5 * r * r / (sigma * sigma);                                \
    }                                                                       \
    for (int32_t i = 0; i < d; ++i) {                                       \
      double s = 0.0;                                                       \
      for (int32_t j = 0; j < n_obs; ++j) s += G[(size_t)j * d + i] * res[j]; \
      (g_out)[i] = s / (sigma * sigma);                                     \
    }                                                                       \
    (phi_out) = acc_;                                                       \
  } while (0)
  double phi = 0.0, phin = 0.0;
  TOY_EVAL(x, phi, gx);
  int64_t acc = 0;
  for (int32_t it = 0; it < n_iter; ++it) {
    uint32_t w3 = (uint32_t)it;
    orc_pcn_propose(seed, 0u, (uint32_t)(it >> 16) * (uint32_t)n_steps, n_steps, n_modes, w3,
                    rho, dt, x, v);
    for (int32_t i = 0; i < d; ++i) v[i] -= (1.0 - rho) * dt * theta * gx[i];
    TOY_EVAL(v, phin, gv);
    double lr = orc_pcnl_log_ratio(d, x, phi, gx, v, phin, gv, theta, rho, dt);
    double u = orc_uniform(seed, 0u, (uint32_t)(it >> 16), (uint32_t)ORC_TAG_ACCEPT << 24, w3);
    if (pcnl_accept(lr, u)) {
      memcpy(x, v, sizeof(double) * d);
      memcpy(gx, gv, sizeof(double) * d);
      phi = phin;
      ++acc;
    }
    memcpy(samples + (size_t)it * d, x, sizeof(double) * d);
  }
#undef TOY_EVAL
  free(x);
  free(v);
  free(gx);
  free(gv);
  free(res);
  return acc;
}

/* Phi of a particle's window with increments x, and grad Phi with respect to
 * x (the adjoint of orc_nudge_grad without controls: its gradient carries the
 * Girsanov term x / dt, which is removed).  Phi = +inf for a failed window. */
static int pcnl_eval(const orc_model *md, int32_t n_obs, const double *y, const double *sigma,
                     int32_t n_steps, const double *m0, const double *u0, const double *x,
                     double *phi, double *g) {
  int32_t d = n_steps * md->n_modes;
  double J = INFINITY;
  int st = orc_nudge_grad(md, n_obs, y, sigma, n_steps, m0, u0, x, NULL, &J, g);
  if (st != ORC_OK || !isfinite(J)) {
    *phi = INFINITY;
    return st != ORC_OK ? st : ORC_E_NONFINITE;
  }
  for (int32_t i = 0; i < d; ++i) g[i] -= x[i] / md->dt;
  *phi = J;
  return ORC_OK;
}

/* n_jitter pCNL moves of every particle's increments dW [n][n_steps][Q] at
 * temperature theta; proposal normals and uniforms as orc_jitter_pcn (tags
 * PCN and ACCEPT, the same counters).  phi [n] in/out.  On return m_end,
 * u_end hold the window ends of the final increments (recomputed). */
int orc_jitter_pcnl(const orc_model *md, int32_t n_obs, const double *y, const double *sigma,
                    const orc_rng *rng, int32_t n_particles, int32_t n_steps, const double *m0,
                    const double *u0, double *dW, double *phi, double *m_end, double *u_end,
                    double theta, double rho, int32_t n_jitter, int32_t *n_accept,
                    int32_t n_threads) {
  int32_t nx = md->nx, nq = md->n_modes, d = n_steps * nq;
#pragma omp parallel for num_threads(n_threads > 0 ? n_threads : 1) schedule(dynamic, 1)
  for (int32_t p = 0; p < n_particles; ++p) {
    double *x = dW + (size_t)p * d;
    double *v = (double *)malloc(sizeof(double) * d), *gx = (double *)malloc(sizeof(double) * d);
    double *gv = (double *)malloc(sizeof(double) * d);
    const double *mp = m0 + (size_t)p * nx, *up = u0 + (size_t)p * nx;
    double phx = phi[p], phv = 0.0, dummy;
    pcnl_eval(md, n_obs, y, sigma, n_steps, mp, up, x, &dummy, gx);
    int32_t acc = 0;
    for (int32_t j = 0; j < n_jitter; ++j) {
      uint32_t w3 = (rng->temper_k << 16) | (uint32_t)j;
      orc_pcn_propose(rng->seed, (uint32_t)p, rng->cycle * (uint32_t)n_steps, n_steps, nq, w3,
                      rho, md->dt, x, v);
      for (int32_t i = 0; i < d; ++i) v[i] -= (1.0 - rho) * md->dt * theta * gx[i];
      pcnl_eval(md, n_obs, y, sigma, n_steps, mp, up, v, &phv, gv);
      double u = orc_uniform(rng->seed, (uint32_t)p, rng->cycle, (uint32_t)ORC_TAG_ACCEPT << 24,
                             w3);
      double lr = isfinite(phv) && isfinite(phx)
                      ? orc_pcnl_log_ratio(d, x, phx, gx, v, phv, gv, theta, rho, md->dt)
                      : -INFINITY;
      if (isfinite(phv) && !isfinite(phx)) lr = INFINITY; /* leave a failed state at once */
      if (pcnl_accept(lr, u)) {
        memcpy(x, v, sizeof(double) * d);
        memcpy(gx, gv, sizeof(double) * d);
        phx = phv;
        ++acc;
      }
    }
    phi[p] = phx;
    if (n_accept) n_accept[p] = acc;
    double *me = m_end + (size_t)p * nx, *ue = u_end + (size_t)p * nx;
    memcpy(me, mp, sizeof(double) * nx);
    memcpy(ue, up, sizeof(double) * nx);
    int32_t it = 0;
    orc_window(md, n_steps, me, ue, x, NULL, &it);
    free(v);
    free(gx);
    free(gv);
  }
  return ORC_OK;
}

/* ========================================================================== */
/* Gradient-based jitter: Hybrid Monte Carlo on the increments x of a particle */
/* (prior N(0, dt I), target proportional to exp(-theta Phi(x)) N(x; 0, dt I)),*/
/* the second sampler the paper names as future work (section 5).  With the    */
/* velocity v distributed as the prior, the Hamiltonian is                     */
/*   H(x, v) = theta Phi(x) + (|x|^2 + |v|^2) / (2 dt)                         */
/* and its flow dx/dt = v, dv/dt = -x - dt theta grad Phi(x) is split into     */
/* kicks v -= tau dt theta grad Phi(x) (the Phi part) and the exact flow of the*/
/* Gaussian part, a rotation of (x, v) by the angle tau.  One leapfrog step of */
/* angle h is a half kick, the rotation and a half kick (Strang splitting:     */
/* reversible and volume-preserving), so the Metropolis test on               */
/* exp(H(x0, v0) - H(xL, vL)) makes the move exact for the tempered target     */
/* (Beskos, Pinski, Sanz-Serna & Stuart, Stoch. Proc. Appl. 2011, for the      */
/* function-space form).  v0 is the pCN normals sqrt(dt) z of the move (tag    */
/* PCN), the uniform that of orc_jitter_pcn (tag ACCEPT).                      */
/* ========================================================================== */
static void hmc_kick(int32_t d, double tau, double dt, double theta, const double *g,
                     double *v) {
  for (int32_t i = 0; i < d; ++i) v[i] -= tau * dt * theta * g[i];
}

static void hmc_rotate(int32_t d, double c, double s, double *x, double *v) {
  for (int32_t i = 0; i < d; ++i) {
    double xi = x[i], vi = v[i];
    x[i] = c * xi + s * vi;
    v[i] = -s * xi + c * vi;
  }
}

static long double hmc_gauss(int32_t d, const double *x, const double *v, double dt) {
  long double s = 0.0L;
  for (int32_t i = 0; i < d; ++i) s += (long double)x[i] * x[i] + (long double)v[i] * v[i];
  return s / (2.0L * dt);
}

/* The linear-Gaussian toy: Phi(x) = |G x - y|^2 / (2 sigma^2) and its
 * gradient G^T (G x - y) / sigma^2 (G [n_obs][d]). */
static double toy_eval(int32_t d, int32_t n_obs, const double *G, const double *y, double sigma,
                       const double *x, double *g, double *res) {
  double phi = 0.0;
  for (int32_t j = 0; j < n_obs; ++j) {
    double r = -y[j];
    for (int32_t i = 0; i < d; ++i) r += G[(size_t)j * d + i] * x[i];
    res[j] = r;
    phi += 0.5 * r * r / (sigma * sigma);
  }
  for (int32_t i = 0; i < d; ++i) {
    double a = 0.0;
    for (int32_t j = 0; j < n_obs; ++j) a += G[(size_t)j * d + i] * res[j];
    g[i] = a / (sigma * sigma);
  }
  return phi;
}

void orc_hmc_trajectory_linear(int32_t d, int32_t n_obs, const double *G, const double *y,
                               double sigma, double theta, double h, int32_t n_leap, double dt,
                               double *x, double *v) {
  double *g = (double *)malloc(sizeof(double) * d);
  double *res = (double *)malloc(sizeof(double) * (n_obs > 0 ? n_obs : 1));
  double c = cos(h), s = sin(h);
  toy_eval(d, n_obs, G, y, sigma, x, g, res);
  for (int32_t l = 0; l < n_leap; ++l) {
    hmc_kick(d, 0.5 * h, dt, theta, g, v);
    hmc_rotate(d, c, s, x, v);
    toy_eval(d, n_obs, G, y, sigma, x, g, res);
    hmc_kick(d, 0.5 * h, dt, theta, g, v);
  }
  free(g);
  free(res);
}

int64_t orc_hmc_linear_chain(uint64_t seed, int32_t n_steps, int32_t n_modes, int32_t n_obs,
                             const double *G, const double *y, double sigma, double theta,
                             double h, int32_t n_leap, double dt, int32_t n_iter,
                             const double *x0, double *samples, int32_t plant) {
  int32_t d = n_steps * n_modes;
  double *x = (double *)malloc(sizeof(double) * d), *xp = (double *)malloc(sizeof(double) * d);
  double *v0 = (double *)malloc(sizeof(double) * d), *v = (double *)malloc(sizeof(double) * d);
  double *g = (double *)malloc(sizeof(double) * d);
  double *res = (double *)malloc(sizeof(double) * (n_obs > 0 ? n_obs : 1));
  memcpy(x, x0, sizeof(double) * d);
  double phi = toy_eval(d, n_obs, G, y, sigma, x, g, res);
  int64_t acc = 0;
  for (int32_t it = 0; it < n_iter; ++it) {
    uint32_t w3 = (uint32_t)it;
    orc_pcn_propose(seed, 0u, (uint32_t)(it >> 16) * (uint32_t)n_steps, n_steps, n_modes, w3, 0.0,
                    dt, x, v0);
    memcpy(xp, x, sizeof(double) * d);
    memcpy(v, v0, sizeof(double) * d);
    orc_hmc_trajectory_linear(d, n_obs, G, y, sigma, theta, h, n_leap, dt, xp, v);
    double phin = toy_eval(d, n_obs, G, y, sigma, xp, g, res);
    if (plant == ORC_PLANT_HMC_NO_KINETIC) {
      memset(v0, 0, sizeof(double) * d);
      memset(v, 0, sizeof(double) * d);
    }
    double lr = (double)(((long double)theta * phi + hmc_gauss(d, x, v0, dt)) -
                         ((long double)theta * phin + hmc_gauss(d, xp, v, dt)));
    double u = orc_uniform(seed, 0u, (uint32_t)(it >> 16), (uint32_t)ORC_TAG_ACCEPT << 24, w3);
    if (pcnl_accept(lr, u)) {
      memcpy(x, xp, sizeof(double) * d);
      phi = phin;
      ++acc;
    }
    memcpy(samples + (size_t)it * d, x, sizeof(double) * d);
  }
  free(x);
  free(xp);
  free(v0);
  free(v);
  free(g);
  free(res);
  return acc;
}

/* n_jitter HMC moves of every particle's increments dW [n][n_steps][Q] at
 * temperature theta, n_leap leapfrog steps of angle h each; Phi and grad Phi
 * of a window from the adjoint (pcnl_eval), the gradient at the current state
 * carried from move to move.  A trajectory that meets a failed window is
 * rejected; a failed current state is left for any finite proposal.  phi [n]
 * in/out; m_end, u_end: the window ends of the final increments. */
int orc_jitter_hmc(const orc_model *md, int32_t n_obs, const double *y, const double *sigma,
                   const orc_rng *rng, int32_t n_particles, int32_t n_steps, const double *m0,
                   const double *u0, double *dW, double *phi, double *m_end, double *u_end,
                   double theta, double h, int32_t n_leap, int32_t n_jitter, int32_t *n_accept,
                   int32_t n_threads) {
  int32_t nx = md->nx, nq = md->n_modes, d = n_steps * nq;
  if (!(h > 0.0) || n_leap < 1) return ORC_E_ARG;
  double c = cos(h), s = sin(h);
#pragma omp parallel for num_threads(n_threads > 0 ? n_threads : 1) schedule(dynamic, 1)
  for (int32_t p = 0; p < n_particles; ++p) {
    double *x = dW + (size_t)p * d;
    double *xp = (double *)malloc(sizeof(double) * d), *v0 = (double *)malloc(sizeof(double) * d);
    double *v = (double *)malloc(sizeof(double) * d), *gx = (double *)malloc(sizeof(double) * d);
    double *gp = (double *)malloc(sizeof(double) * d);
    const double *mp = m0 + (size_t)p * nx, *up = u0 + (size_t)p * nx;
    double phx = phi[p], php = INFINITY, dummy;
    if (pcnl_eval(md, n_obs, y, sigma, n_steps, mp, up, x, &dummy, gx) != ORC_OK)
      memset(gx, 0, sizeof(double) * d); /* a failed state: any finite proposal leaves it */
    int32_t acc = 0;
    for (int32_t j = 0; j < n_jitter; ++j) {
      uint32_t w3 = (rng->temper_k << 16) | (uint32_t)j;
      orc_pcn_propose(rng->seed, (uint32_t)p, rng->cycle * (uint32_t)n_steps, n_steps, nq, w3,
                      0.0, md->dt, x, v0);
      memcpy(xp, x, sizeof(double) * d);
      memcpy(v, v0, sizeof(double) * d);
      memcpy(gp, gx, sizeof(double) * d);
      int ok = 1;
      for (int32_t l = 0; l < n_leap && ok; ++l) {
        hmc_kick(d, 0.5 * h, md->dt, theta, gp, v);
        hmc_rotate(d, c, s, xp, v);
        ok = pcnl_eval(md, n_obs, y, sigma, n_steps, mp, up, xp, &php, gp) == ORC_OK;
        if (ok) hmc_kick(d, 0.5 * h, md->dt, theta, gp, v);
      }
      if (!ok) php = INFINITY;
      double u = orc_uniform(rng->seed, (uint32_t)p, rng->cycle, (uint32_t)ORC_TAG_ACCEPT << 24,
                             w3);
      double lr = -INFINITY;
      if (isfinite(php) && isfinite(phx))
        lr = (double)(((long double)theta * phx + hmc_gauss(d, x, v0, md->dt)) -
                      ((long double)theta * php + hmc_gauss(d, xp, v, md->dt)));
      if (isfinite(php) && !isfinite(phx)) lr = INFINITY; /* leave a failed state at once */
      if (pcnl_accept(lr, u)) {
        memcpy(x, xp, sizeof(double) * d);
        memcpy(gx, gp, sizeof(double) * d);
        phx = php;
        ++acc;
      }
    }
    phi[p] = phx;
    if (n_accept) n_accept[p] = acc;
    double *me = m_end + (size_t)p * nx, *ue = u_end + (size_t)p * nx;
    memcpy(me, mp, sizeof(double) * nx);
    memcpy(ue, up, sizeof(double) * nx);
    int32_t it = 0;
    orc_window(md, n_steps, me, ue, x, NULL, &it);
    free(xp);
    free(v0);
    free(v);
    free(gx);
    free(gp);
  }
  return ORC_OK;
}
