/* Drives every family of the oracle's entry points on small inputs, for a
 * build with the address and undefined-behaviour sanitizers
 * (tests/test_oracle_sanitize.py).  Exits 0 when every call returns a valid
 * status; the sanitizers abort on the first invalid access. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "sch_oracle.h"

#define NX 64
#define NP 6
#define NS 4
#define NQ 4
#define NO 8

static void check(int ok, const char *what) {
  if (!ok) {
    fprintf(stderr, "FAILED: %s\n", what);
    exit(1);
  }
}

int main(void) {
  const double L = 40.0, h = L / NX;
  static double xi[NQ * NX], m[NP * NX], u[NP * NX], dW[NP * NS * NQ], dL[NP * NS * NQ];
  static double y[NO], sig[NO], phi[NP], w[NP], grad[NS * NQ];
  static double cells[NP * NS * NX], field[NX];
  int32_t st[NP], it[NP], idx[NP], acc[NP];
  for (int q = 0; q < NQ; ++q)
    for (int i = 0; i < NX; ++i) {
      const double x = 6.283185307179586 * (q / 2 + 1) * i * h / L;
      xi[q * NX + i] = 0.05 * (q % 2 ? cos(x) : sin(x));
    }
  orc_model md = {L, 1.0, 0.01, 0.025, NX, NQ, xi, 1e-13, 50};
  for (int p = 0; p < NP; ++p)
    for (int i = 0; i < NX; ++i) {
      const double c = cosh((i * h - 20.0 - p) / 2.0);
      u[p * NX + i] = 0.2 / (c * c);
    }
  for (int p = 0; p < NP; ++p)
    check(orc_momentum_from_velocity(&md, u + p * NX, m + p * NX) == ORC_OK, "momentum");
  for (int o = 0; o < NO; ++o) {
    y[o] = 0.1;
    sig[o] = 0.05;
  }

  /* generator, linear algebra, window, observation, weights, resampling */
  uint32_t ctr[4] = {1, 2, 3, 4}, out[4];
  orc_philox4x32_10(ctr, 7u, out);
  orc_draw_increments(7u, NP, NS, NQ, 0u, ORC_TAG_FORECAST, 0u, md.dt, dW);
  check(orc_ensemble_window(&md, NP, NS, m, u, dW, NULL, st, it, 1) == ORC_OK, "window");
  orc_ensemble_nll(NX, NO, NP, u, y, sig, phi);
  double ess = orc_weights(NP, phi, NULL, 1.0, w, NULL);
  check(ess > 0.0, "weights");
  check(orc_resample_systematic(NP, w, 0.3, idx) == ORC_OK, "resample");
  check(orc_resample_textbook(NP, w, 0.3, idx) == ORC_OK, "resample textbook");
  double dth;
  check(orc_temper(NP, phi, 0.0, 0.5 * NP, 50, &dth, w, &ess) == ORC_OK, "temper");

  /* filters */
  orc_cycle_stats cs;
  double logw[NP] = {0};
  check(orc_bootstrap_cycle(&md, NO, y, sig, 7u, 0u, NP, NS, 0.5, m, u, logw, &cs, 1) >=
            ORC_E_DEGENERATE,
        "bootstrap");
  orc_tempered_cycle(&md, NO, y, sig, 7u, 1u, NP, NS, 0.5 * NP, 50, 0.9, 2, 100, m, u, &cs, 1);
  check(cs.n_temper >= 1, "tempered");
  orc_tempered_cycle_pcnl(&md, NO, y, sig, 7u, 2u, NP, NS, 0.5 * NP, 50, 0.9, 2, 100, m, u, &cs,
                          1);
  check(cs.n_temper >= 1, "tempered pcnl");
  {
    double F[4] = {0.9, 0.1, -0.1, 0.9}, B[2 * NS * NQ], G[4] = {1, 0, 0.5, 1};
    double yl[2] = {0.1, 0.2};
    double x[NP * 2] = {0};
    for (int i = 0; i < 2 * NS * NQ; ++i) B[i] = 0.1 * ((i % 5) - 2);
    check(orc_tempered_cycle_linear(2, NS, NQ, 2, F, B, G, yl, 0.1, md.dt, 7u, 0u, NP, 0.5 * NP,
                                    50, 0.5, 3, 100, x, &cs, ORC_PLANT_NONE) == ORC_OK,
          "tempered linear");
  }

  /* nudging: gradient, tangent, L-BFGS stages, nudged filter */
  double J;
  memset(dL, 0, sizeof dL);
  check(orc_nudge_grad(&md, NO, y, sig, NS, m, u, dW, dL, &J, grad) == ORC_OK, "nudge grad");
  check(orc_nudge_grad_tangent(&md, NO, y, sig, NS, m, u, dW, dL, grad) == ORC_OK,
        "nudge tangent");
  orc_lbfgs_opts opt = {1e-8, 5, 8, 30};
  double logG[NP];
  int32_t lst[NP];
  orc_nudge_ensemble(&md, NO, y, sig, NP, NS, m, u, dW, dL, &opt, logG, it, acc, lst, st, 1);
  orc_nudged_cycle(&md, NO, y, sig, 7u, 3u, NP, NS, 0.5 * NP, 50, 0.9, 2, 100, &opt, m, u, NULL,
                   NULL, NULL, NULL, NULL, &cs, 1);

  /* Matern-type noise: field, transpose, window, jitter, cycles, nudging */
  orc_matern mt = {1.0, 1.0, 3};
  orc_draw_increments(8u, NP, NS, NX, 0u, ORC_TAG_FORECAST, 0u, md.dt, cells);
  check(orc_matern_field(NX, L, &mt, cells, field) == ORC_OK, "matern field");
  {
    static double tr[NX];
    check(orc_matern_transpose(NX, L, &mt, field, tr) == ORC_OK, "matern transpose");
  }
  orc_ensemble_window_matern(&md, &mt, NP, NS, m, u, cells, st, it, 1);
  orc_tempered_cycle_matern(&md, &mt, NO, y, sig, 7u, 4u, NP, NS, 0.5 * NP, 50, 0.9, 2, 100, m,
                            u, NULL, NULL, NULL, NULL, &cs, 1);
  orc_bootstrap_cycle_matern(&md, &mt, NO, y, sig, 7u, 5u, NP, NS, 0.5, m, u, logw, &cs, 1);
  {
    static double gc[NS * NX], lc[NP * NS * NX];
    memset(lc, 0, sizeof lc);
    check(orc_nudge_grad_matern(&md, &mt, NO, y, sig, NS, m, u, cells, lc, &J, gc) == ORC_OK,
          "nudge grad matern");
    orc_lbfgs_opts o2 = {1e-8, 3, 8, 30};
    orc_nudge_ensemble_matern(&md, &mt, NO, y, sig, 2, NS, m, u, cells, lc, &o2, logG, it, acc,
                              lst, st, 1);
    orc_nudged_cycle_matern(&md, &mt, NO, y, sig, 7u, 6u, 2, NS, 1.0, 50, 0.9, 1, 100, &o2, m, u,
                            NULL, NULL, NULL, NULL, NULL, &cs, 1);
  }

  /* the paper's experiments: initial ensemble and statistics */
  double stats[3];
  check(orc_paper_init(NX, L, 9u, 0, NP, u) == ORC_OK, "paper init");
  orc_ensemble_stats(NP, NX, u, u, stats);
  printf("oracle sanitizer driver: ok\n");
  return 0;
}
