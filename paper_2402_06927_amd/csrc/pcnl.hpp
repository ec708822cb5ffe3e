// pcnl.hpp -- the gradient-based jitter: preconditioned Crank-Nicolson
// Langevin moves (pCNL; Cotter, Roberts, Stuart & White, Statist. Sci. 2013)
// of every particle's increments x (prior N(0, dt I)) towards the tempered
// posterior exp(-theta Phi(x)) N(x; 0, dt I):
//   v = rho x + sqrt(1 - rho^2) sqrt(dt) z - (1 - rho) dt theta grad Phi(x),
// accepted with the Metropolis-Hastings ratio of target and Gaussian proposal
// densities.  Phi and grad Phi come from the discrete adjoint (k_nudge_grad
// with the increments as dW and no controls: its gradient then carries the
// Girsanov term x / dt, removed here).  The paper names MALA/HMC jittering as
// future work (section 5); the Hybrid Monte Carlo move is below.
#pragma once

#include "device.hpp"

namespace sch {

// g -= x / dt: the adjoint's gradient without the Girsanov term.
__global__ void k_pcnl_grad(int64_t total, double idt, const double* x, double* g) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < total;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    g[i] -= x[i] * idt;
}

// v = rho x + srho zeta - c theta g, zeta = sqrt(dt) z, c = (1 - rho) dt.
__global__ void k_pcnl_propose(int64_t total, double rho, double srho, double c,
                               const double* theta, const double* x, const double* g,
                               const double* zeta, double* v) {
  const double ct = c * *theta;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < total;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    v[i] = (rho * x[i] + srho * zeta[i]) - ct * g[i];
}

// Metropolis-Hastings step of one particle (one wavefront): the adjoint's
// gradient at v is corrected in place (gv -= v / dt), phi(v) = J(v) when the
// window succeeded; log r = log pi(v) + log q(v -> x) - log pi(x) - log q(x -> v)
// with log pi(x) = -theta phi(x) - |x|^2 / (2 dt) and
// log q(x -> v) = -|v - rho x + c theta g(x)|^2 / (2 (1 - rho^2) dt).  A state
// whose window failed (phi = inf) is left for any finite proposal.  On
// acceptance x, g(x) and phi take the proposal's values.
__global__ void __launch_bounds__(kWave) k_pcnl_accept(int d, double rho, double dt,
                                                       const double* theta, const double* vacc,
                                                       const int* status, const double* Jv,
                                                       double* x, double* gx, double* phi,
                                                       const double* v, double* gv, int* acc,
                                                       int first) {
  const int p = blockIdx.x, l = threadIdx.x;
  const double th = *theta, c = (1.0 - rho) * dt * th, idt = 1.0 / dt;
  double* xp = x + static_cast<size_t>(p) * d;
  double* gxp = gx + static_cast<size_t>(p) * d;
  const double* vp = v + static_cast<size_t>(p) * d;
  double* gvp = gv + static_cast<size_t>(p) * d;
  double sv = 0.0, sx = 0.0, sb = 0.0, sf = 0.0;  // |v|^2, |x|^2, backward and forward residuals
  for (int i = l; i < d; i += kWave) {
    const double g = gvp[i] - vp[i] * idt;
    gvp[i] = g;
    const double rb = xp[i] - (rho * vp[i] - c * g);
    const double rf = vp[i] - (rho * xp[i] - c * gxp[i]);
    sv = fma(vp[i], vp[i], sv);
    sx = fma(xp[i], xp[i], sx);
    sb = fma(rb, rb, sb);
    sf = fma(rf, rf, sf);
  }
  sv = wave_sum(sv);
  sx = wave_sum(sx);
  sb = wave_sum(sb);
  sf = wave_sum(sf);
  const double jv = Jv[p];
  const double phv = (status[p] == SCH_OK && fabs(jv) <= 1.7976931348623157e308) ? jv : INFINITY;
  const double phx = phi[p];
  bool accept = false;
  if (phv < INFINITY) {
    if (!(phx < INFINITY)) {
      accept = true;
    } else {
      const double qd = 2.0 * (1.0 - rho * rho) * dt;
      const double lr = (-th * phv - sv / (2.0 * dt) - sb / qd) - (-th * phx - sx / (2.0 * dt) - sf / qd);
      accept = lr >= 0.0 ? true : vacc[p] < exp(lr);
    }
  }
  if (accept) {
    for (int i = l; i < d; i += kWave) {
      xp[i] = vp[i];
      gxp[i] = gvp[i];
    }
  }
  if (l == 0) {
    if (accept) phi[p] = phv;
    acc[p] = (first ? 0 : acc[p]) + (accept ? 1 : 0);
  }
}

// ---------------------------------------------------------------------------
// Hybrid Monte Carlo moves of the increments x (prior N(0, dt I)) towards
// exp(-theta Phi(x)) N(x; 0, dt I), the second sampler the paper names as
// future work: velocity v ~ N(0, dt I) (the pCN draws sqrt(dt) z of the
// move), n_leap leapfrog steps of angle h of H(x, v) = theta Phi(x) +
// (|x|^2 + |v|^2) / (2 dt), each a half kick v -= (h/2) dt theta grad Phi(x),
// the rotation of (x, v) by h (the exact flow of the Gaussian part) and a
// half kick; accepted with probability min(1, exp(H(x0, v0) - H(xL, vL))).
// ---------------------------------------------------------------------------

// One leapfrog step up to its gradient evaluation.  first: the trajectory
// starts at (x, zeta) with the gradient gx of the current state (one half
// kick); otherwise it continues at (xp, v) with the gradient gp of its last
// evaluation (that step's closing half kick, then this step's opening one).
// Then the rotation by h (c = cos h, s = sin h) into (xp, v).  A particle
// whose last evaluation failed is marked in bad.  a = (h/2) dt.
__global__ void k_hmc_step(int64_t total, int d, int first, double a, const double* theta,
                           double c, double s, const double* x, const double* gx,
                           const double* zeta, double* xp, double* v, const double* gp,
                           const int* status, int* bad) {
  const double at = a * *theta;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < total;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    double xi, vi;
    if (first) {
      xi = x[i];
      vi = zeta[i];
      vi -= at * gx[i];
    } else {
      xi = xp[i];
      vi = v[i];
      const double g = gp[i];
      vi -= at * g;
      vi -= at * g;
      const int64_t p = i / d;
      if (status[p] != SCH_OK) bad[p] = 1;
    }
    xp[i] = c * xi + s * vi;
    v[i] = -s * xi + c * vi;
  }
}

// Metropolis test of one particle's trajectory (one wavefront): the closing
// half kick with the gradient gp at its end (already without the Girsanov
// term, k_pcnl_grad), then log r = H(x, zeta) - H(xp, v) with
// H(x, v) = theta phi(x) + (|x|^2 + |v|^2) / (2 dt).  A trajectory with a
// failed evaluation is rejected; a failed current state is left for any
// finite proposal.  On acceptance x, gx and phi take the proposal's values.
__global__ void __launch_bounds__(kWave) k_hmc_accept(int d, double a, double dt,
                                                      const double* theta, const double* vacc,
                                                      const int* status, const int* bad,
                                                      const double* Jp, double* x, double* gx,
                                                      double* phi, const double* xp,
                                                      const double* gp, double* v,
                                                      const double* zeta, int* acc,
                                                      int first) {
  const int p = blockIdx.x, l = threadIdx.x;
  const double th = *theta, at = a * th;
  double* xq = x + static_cast<size_t>(p) * d;
  double* gxq = gx + static_cast<size_t>(p) * d;
  const double* xpq = xp + static_cast<size_t>(p) * d;
  const double* gpq = gp + static_cast<size_t>(p) * d;
  double* vq = v + static_cast<size_t>(p) * d;
  const double* zq = zeta + static_cast<size_t>(p) * d;
  double s0 = 0.0, s1 = 0.0;  // |x|^2 + |zeta|^2 and |xp|^2 + |v|^2
  for (int i = l; i < d; i += kWave) {
    const double vi = vq[i] - at * gpq[i];
    vq[i] = vi;
    s0 = fma(xq[i], xq[i], s0);
    s0 = fma(zq[i], zq[i], s0);
    s1 = fma(xpq[i], xpq[i], s1);
    s1 = fma(vi, vi, s1);
  }
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  const double jp = Jp[p];
  const double php = (status[p] == SCH_OK && !bad[p] && fabs(jp) <= 1.7976931348623157e308)
                         ? jp
                         : INFINITY;
  const double phx = phi[p];
  bool accept = false;
  if (php < INFINITY) {
    if (!(phx < INFINITY)) {
      accept = true;
    } else {
      const double lr = (th * phx + s0 / (2.0 * dt)) - (th * php + s1 / (2.0 * dt));
      accept = lr >= 0.0 ? true : vacc[p] < exp(lr);
    }
  }
  if (accept) {
    for (int i = l; i < d; i += kWave) {
      xq[i] = xpq[i];
      gxq[i] = gpq[i];
    }
  }
  if (l == 0) {
    if (accept) phi[p] = php;
    acc[p] = (first ? 0 : acc[p]) + (accept ? 1 : 0);
  }
}

}  // namespace sch
