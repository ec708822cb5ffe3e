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
void orc_draw_increments(uint64_t seed, int32_t n_particles, int32_t n_steps, int32_t n_modes,
                         uint32_t step0, uint32_t tag, uint32_t word3, double dt, double *dW) {
  double sdt = sqrt(dt);
  int32_t n_pairs = (n_modes + 1) / 2;
  for (int32_t p = 0; p < n_particles; ++p)
    for (int32_t n = 0; n < n_steps; ++n)
      for (int32_t k = 0; k < n_pairs; ++k) {
        double z[2];
        orc_normal_pair(seed, (uint32_t)p, step0 + (uint32_t)n, (uint32_t)k | (tag << 24), word3,
                        z);
        double *row = dW + ((int64_t)p * n_steps + n) * n_modes;
        row[2 * k] = sdt * z[0];
        if (2 * k + 1 < n_modes) row[2 * k + 1] = sdt * z[1];
      }
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
/* iterate a pivoted linear solve) until the momentum changes by at most       */
/* picard_tol relative in the max norm.                                        */
/* ========================================================================== */
int orc_step(const orc_model *md, double *m, double *u, const double *dW, const double *dLam,
             int32_t *iters) {
  int32_t n = md->nx;
  double h = md->L / n, dt = md->dt, mu = md->mu;
  size_t sz = sizeof(double) * (size_t)n;
  double *dU = (double *)calloc((size_t)n, sizeof(double));
  double *dv = (double *)malloc(sz), *lo = (double *)malloc(sz), *di = (double *)malloc(sz);
  double *up = (double *)malloc(sz), *rhs = (double *)malloc(sz), *t1 = (double *)malloc(sz);
  double *ms = (double *)malloc(sz), *us = (double *)malloc(sz), *mp = (double *)malloc(sz);

  for (int32_t q = 0; q < md->n_modes; ++q) {
    double inc = dW[q] + (dLam ? dLam[q] : 0.0);
    for (int32_t i = 0; i < n; ++i) dU[i] += md->xi[(size_t)q * n + i] * inc;
  }
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
  free(dU);
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
int orc_bootstrap_cycle(const orc_model *md, int32_t n_obs, const double *y, const double *sigma,
                        uint64_t seed, uint32_t cycle, int32_t n_particles, int32_t n_steps,
                        double ess_frac, double *m, double *u, double *logw,
                        orc_cycle_stats *st, int32_t n_threads) {
  int32_t nx = md->nx, nq = md->n_modes;
  double *dW = (double *)malloc(sizeof(double) * (size_t)n_particles * n_steps * nq);
  int32_t *iters = (int32_t *)malloc(sizeof(int32_t) * n_particles);
  int32_t *stat = (int32_t *)malloc(sizeof(int32_t) * n_particles);
  double *phi = (double *)malloc(sizeof(double) * n_particles);
  double *w = (double *)malloc(sizeof(double) * n_particles);
  int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * n_particles);
  memset(st, 0, sizeof(*st));

  orc_draw_increments(seed, n_particles, n_steps, nq, cycle * (uint32_t)n_steps, ORC_TAG_FORECAST,
                      0u, md->dt, dW);
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

/* Tempered and jittered filter, section 3.1.2.  Each particle is the pair
 * (window-start state, increments over the window).  After the forecast, the
 * temperature theta climbs from 0 to 1 in adaptive steps; after every step the
 * ensemble is resampled with the tempered weights exp(-dtheta Phi) and every
 * particle's increments are moved by n_jitter pCN steps targeting the
 * posterior tempered at the new cumulative theta.  Only then does the window
 * end state become the next cycle's start state. */
int orc_tempered_cycle(const orc_model *md, int32_t n_obs, const double *y, const double *sigma,
                       uint64_t seed, uint32_t cycle, int32_t n_particles, int32_t n_steps,
                       double ess_threshold, int32_t n_bisect, double rho, int32_t n_jitter,
                       int32_t max_temper, double *m, double *u, orc_cycle_stats *st,
                       int32_t n_threads) {
  int32_t nx = md->nx, nq = md->n_modes;
  size_t state = (size_t)n_particles * nx, wlen = (size_t)n_particles * n_steps * nq;
  double *m0 = (double *)malloc(sizeof(double) * state), *u0 = (double *)malloc(sizeof(double) * state);
  double *dW = (double *)malloc(sizeof(double) * wlen);
  double *phi = (double *)malloc(sizeof(double) * n_particles);
  double *w = (double *)malloc(sizeof(double) * n_particles);
  int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * n_particles);
  int32_t *iters = (int32_t *)malloc(sizeof(int32_t) * n_particles);
  int32_t *stat = (int32_t *)malloc(sizeof(int32_t) * n_particles);
  int32_t *acc = (int32_t *)malloc(sizeof(int32_t) * n_particles);
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
  double theta = 0.0;
  int32_t k = 0;
  int rc = ORC_OK;
  while (theta < 1.0) {
    if (k >= max_temper) {
      rc = ORC_E_DEGENERATE;
      break;
    }
    double dth, ess;
    orc_temper(n_particles, phi, theta, ess_threshold, n_bisect, &dth, w, &ess);
    if (ess == 0.0) {
      rc = ORC_E_DEGENERATE;
      break;
    }
    double theta_new = (dth == 1.0 - theta) ? 1.0 : theta + dth;
    double ur = orc_uniform(seed, 0u, cycle, (uint32_t)ORC_TAG_RESAMPLE << 24, (uint32_t)k << 16);
    rc = orc_resample_systematic(n_particles, w, ur, idx);
    if (rc != ORC_OK) break;
    gather_rows(m0, idx, n_particles, (size_t)nx);
    gather_rows(u0, idx, n_particles, (size_t)nx);
    gather_rows(m, idx, n_particles, (size_t)nx);
    gather_rows(u, idx, n_particles, (size_t)nx);
    gather_rows(dW, idx, n_particles, (size_t)n_steps * nq);
    gather_rows(phi, idx, n_particles, 1);
    orc_rng rg = {seed, cycle, (uint32_t)k};
    orc_jitter_pcn(md, n_obs, y, sigma, &rg, n_particles, n_steps, m0, u0, dW, phi, m, u,
                   theta_new, rho, n_jitter, acc, n_threads);
    for (int32_t p = 0; p < n_particles; ++p) st->n_accept += acc[p];
    st->ess = ess;
    theta = theta_new;
    ++k;
  }
  st->n_temper = k;
  st->status = rc;
  free(m0);
  free(u0);
  free(dW);
  free(phi);
  free(w);
  free(idx);
  free(iters);
  free(stat);
  free(acc);
  return rc;
}
