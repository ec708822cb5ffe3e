// abi.hip -- the C-ABI of include/sch.h: argument validation, kernel
// selection and launch, and the host-driven filter cycles.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <mutex>
#include <string>
#include <vector>

#include "adjoint.hpp"
#include "host.hpp"
#include "filter.hpp"
#include "model.hpp"
#include "pcnl.hpp"

using namespace sch;

namespace {
// Scratch layout shared by the cycle drivers.
struct CycleWs {
  double *zeta, *vacc;                               // pCN random numbers
  double *m0, *u0, *scratch, *dW, *phi, *w, *scal;  // scal: theta, dtheta, ess, u0
  int *idx, *status, *iters, *degenerate;
  unsigned long long *cum, *acc;                     // acc: [0] iters, [1] accepts
};

// With the Matern-type noise (matern != 0) nq is nx (the cells of a step),
// and zeta is the jitter kernel's stage [n][ns][nx] for the proposals (its
// random numbers are drawn in the kernel; no vacc).
CycleWs carve_cycle(void* base, int which, int nx, int nq, int n, int ns, size_t* bytes,
                    int n_jitter = 0, int matern = 0) {
  Carve c(base);
  CycleWs w{};
  const size_t state = static_cast<size_t>(n) * nx, inc = static_cast<size_t>(n) * ns * nq;
  if (which == SCH_WS_JITTER || which == SCH_WS_TEMPERED) {
    if (matern) {
      w.zeta = c.take<double>(n_jitter > 0 ? inc : 0);
    } else {
      w.zeta = c.take<double>(inc * static_cast<size_t>(n_jitter));
      w.vacc = c.take<double>(static_cast<size_t>(n) * n_jitter);
    }
    if (which == SCH_WS_JITTER) {
      if (bytes) *bytes = c.off + 256;
      return w;
    }
  }
  if (which == SCH_WS_TEMPERED) {
    w.m0 = c.take<double>(state);
    w.u0 = c.take<double>(state);
  }
  w.scratch = c.take<double>(state > inc ? state : inc);
  w.dW = c.take<double>(inc);
  w.phi = c.take<double>(n);
  w.w = c.take<double>(n);
  w.scal = c.take<double>(8);
  w.idx = c.take<int>(n);
  w.status = c.take<int>(n);
  w.iters = c.take<int>(n);
  w.degenerate = c.take<int>(4);
  w.cum = c.take<unsigned long long>(n);
  w.acc = c.take<unsigned long long>(4);
  if (bytes) *bytes = c.off + 256;
  return w;
}

// M != null: the Matern-type noise, dW holds cells [n][n_steps][nx].
int launch_window(const sch_model& md, const Tile& tl, int n, int n_steps, double* m, double* u,
                  const double* dW, const double* dLam, int* status, int* iters,
                  unsigned long long* iters_acc, hipStream_t st, const MaternDev* M = nullptr) {
  WindowArgs A{};
  A.P = make_params(md);
  A.n_steps = n_steps;
  A.m = m;
  A.u = u;
  A.dW = dW;
  A.dLam = dLam;
  A.status = status;
  A.iters = iters;
  A.iters_acc = iters_acc;
  if (M) A.M = *M;
  const HelmConst K = make_helm(md, tl);
  return with_tile(tl, [&]<int PM, int NT, bool FULL>() -> int {
    if (M)
      hipLaunchKernelGGL((k_window<PM, NT, FULL, true>), dim3(n), dim3(NT), 0, st, A, K);
    else
      hipLaunchKernelGGL((k_window<PM, NT, FULL>), dim3(n), dim3(NT), 0, st, A, K);
    CHECK_LAUNCH();
    return SCH_OK;
  });
}

// Constants of the Matern-type noise for the model's grid and tile.
int make_matern(const sch_model& md, const sch_matern* mt, const Tile& tl, MaternDev& M) {
  if (!mt || !(mt->kappa > 0) || !std::isfinite(mt->kappa) || !std::isfinite(mt->eta) ||
      mt->k < 1 || mt->k > 16)
    return fail(SCH_E_ARG, "need 0 < kappa < inf, finite eta and 1 <= k <= 16");
  const double h = md.L / md.nx, a2 = 1.0 / (mt->kappa * mt->kappa);
  if (!(std::fabs(h / 6.0 - a2 / h) > 1e-12 * (2.0 * h / 3.0 + 2.0 * a2 / h)))
    return fail(SCH_E_ARG, "kappa h = sqrt(6): the Matern operator is diagonal");
  M.K = make_helm_op(h, md.nx, a2, tl);
  M.load = mt->eta * std::sqrt(h) * 0.5;
  M.h = h;
  M.k = mt->k;
  return SCH_OK;
}

int launch_helm(const sch_model& md, const Tile& tl, int n, const double* in, double* out,
                int mode, hipStream_t st) {
  HelmArgs A;
  A.P = make_params(md);
  A.in = in;
  A.out = out;
  A.mode = mode;
  const HelmConst K = make_helm(md, tl);
  return with_tile(tl, [&]<int PM, int NT, bool FULL>() -> int {
    hipLaunchKernelGGL((k_helmholtz<PM, NT, FULL>), dim3(n), dim3(NT), 0, st, A, K);
    CHECK_LAUNCH();
    return SCH_OK;
  });
}

// Nudging scratch: checkpoints [n][n_segments][2][nx], segment states
// [n][ckpt_every + 1][2][nx] and two iteration counters; for sch_nudge_run
// also the batched L-BFGS state.
struct NudgeWs {
  double *ckpt, *seg;
  unsigned long long* acc;
  LbfgsState lb;
  double* inc1;
  int *worst, *iters, *evals, *status, *tmp;
};

NudgeWs carve_nudge(void* base, bool full, int nx, int nq, int n, int ns, int ce, size_t* bytes) {
  Carve c(base);
  NudgeWs w{};
  const size_t nseg = static_cast<size_t>((ns + ce - 1) / ce);
  w.ckpt = c.take<double>(static_cast<size_t>(n) * nseg * 2 * nx);
  w.seg = c.take<double>(static_cast<size_t>(n) * (ce + 1) * 2 * nx);
  w.acc = c.take<unsigned long long>(2);
  if (full) {
    const size_t v = static_cast<size_t>(n) * nq, mq = v * kLbfgsMaxMem;
    w.lb.x = c.take<double>(v);
    w.lb.g = c.take<double>(v);
    w.lb.p = c.take<double>(v);
    w.lb.xt = c.take<double>(v);
    w.lb.gt = c.take<double>(v);
    w.lb.ft = c.take<double>(n);
    w.lb.f = c.take<double>(n);
    w.lb.gp = c.take<double>(n);
    w.lb.a = c.take<double>(n);
    w.lb.S = c.take<double>(mq);
    w.lb.Y = c.take<double>(mq);
    w.lb.rho = c.take<double>(static_cast<size_t>(n) * kLbfgsMaxMem);
    int** ints[] = {&w.lb.head, &w.lb.count, &w.lb.k, &w.lb.nback, &w.lb.phase,
                    &w.lb.lstat, &w.lb.active, &w.lb.est, &w.lb.evals, &w.worst,
                    &w.iters, &w.evals, &w.status, &w.tmp};
    for (int** ip : ints) *ip = c.take<int>(n);
    w.lb.n_active = c.take<unsigned int>(1);
    w.inc1 = c.take<double>(v);
  }
  if (bytes) *bytes = c.off + 256;
  return w;
}

int launch_nudge_grad(const sch_model& md, const Tile& tl, const sch_obs& ob, int n,
                      int n_steps, int ctrl_steps, const double* m0, const double* u0,
                      const double* dW, const double* dLam, int ce, double* J, double* grad,
                      int* status, const int* active, const NudgeWs& W, hipStream_t st,
                      const MaternDev* M = nullptr) {
  NudgeArgs A;
  A.P = make_params(md);
  A.n_steps = n_steps;
  A.ctrl_steps = ctrl_steps;
  A.ckpt_every = ce;
  A.m0 = m0;
  A.u0 = u0;
  A.dW = dW;
  A.dLam = dLam;
  A.n_obs = ob.n_obs;
  A.y = ob.y;
  A.sigma = ob.sigma;
  A.J = J;
  A.grad = grad;
  A.status = status;
  A.active = active;
  A.ckpt = W.ckpt;
  A.seg = W.seg;
  A.iters_acc = W.acc;
  if (M) A.M = *M;
  // The adjoint kernel holds more per node than the window (the reverse
  // sweep's source, checkpoints, the transposed solve's right-hand side):
  // on 16 nodes per thread it spills and ran 7-110% slower than on twice the
  // threads with 8 nodes each at every grid measured, so a 16-node tile is
  // doubled where 512 threads allow it.  The Matern-noise kernels keep the
  // caller's tile, to which the noise operator's constants belong.
  const Tile ta = (!M && tl.pmax == 16 && tl.nt <= 256) ? tile_for(md.nx, 2 * tl.nt) : tl;
  const HelmConst K = make_helm(md, ta);
  return with_tile(ta, [&]<int PM, int NT, bool FULL>() -> int {
    if (M)
      hipLaunchKernelGGL((k_nudge_grad<PM, NT, FULL, true>), dim3(n), dim3(NT), 0, st, A, K);
    else
      hipLaunchKernelGGL((k_nudge_grad<PM, NT, FULL>), dim3(n), dim3(NT), 0, st, A, K);
    CHECK_LAUNCH();
    return SCH_OK;
  });
}

// Scratch of the gradient-based jitters: the proposal draws (as pCN), the
// adjoint's scratch, the proposal, the gradients at the current state and at
// the proposal, J, statuses and acceptance counts; for Hybrid Monte Carlo
// (hmc) also the velocity and a per-particle failure flag, and the leapfrog
// angle and step count.
struct PcnlWs {
  double *zeta, *vacc, *v, *gx, *gv, *J;
  int *status, *acc;
  NudgeWs nws;
  int ce;
  double *vel;
  int* bad;
  bool hmc;
  double h;
  int n_leap;
};

PcnlWs carve_pcnl(void* base, int nx, int nq, int n, int ns, int n_jitter, int ce,
                  size_t* bytes, bool hmc = false) {
  Carve c(base);
  PcnlWs w{};
  const size_t inc = static_cast<size_t>(n) * ns * nq;
  w.zeta = c.take<double>(inc * static_cast<size_t>(n_jitter));
  w.vacc = c.take<double>(static_cast<size_t>(n) * n_jitter);
  w.v = c.take<double>(inc);
  w.gx = c.take<double>(inc);
  w.gv = c.take<double>(inc);
  w.J = c.take<double>(n);
  w.status = c.take<int>(n);
  w.acc = c.take<int>(n);
  if (hmc) {
    w.vel = c.take<double>(inc);
    w.bad = c.take<int>(n);
  }
  w.hmc = hmc;
  size_t nb = 0;
  carve_nudge(nullptr, false, nx, nq, n, ns, ce, &nb);
  char* nbase = c.take<char>(nb);
  w.nws = carve_nudge(nbase, false, nx, nq, n, ns, ce, nullptr);
  w.ce = ce;
  if (bytes) *bytes = c.off + 256;
  return w;
}

int check_obs(const sch_obs* ob) {
  if (!ob || ob->n_obs < 1 || !ob->y || !ob->sigma) return fail(SCH_E_ARG, "bad observations");
  return SCH_OK;
}

// Draws the pCN random numbers (zeta [n_jitter][n][n_steps][n_modes],
// vacc [n_jitter][n]) and launches the fused jitter kernel.
int launch_jitter(const sch_model& md, const Tile& tl, const sch_obs& ob, uint64_t seed,
                  uint32_t cycle, uint32_t temper_k, int n, int n_steps, const double* m0,
                  const double* u0, double* dW, double* phi, double* m_end, double* u_end,
                  const double* theta, double rho, int n_jitter, int* n_accept,
                  unsigned long long* accept_acc, unsigned long long* iters_acc, double* zeta,
                  double* vacc, const double* dLam, hipStream_t st, const MaternDev* M = nullptr) {
  if (!M) {
    const int64_t work = static_cast<int64_t>(n_jitter) * n * n_steps * ((md.n_modes + 1) / 2);
    hipLaunchKernelGGL(k_draw_pcn, dim3(grid_for(work, 256)), dim3(256), 0, st, seed,
                       cycle * static_cast<uint32_t>(n_steps), cycle, temper_k << 16, n_jitter, n,
                       n_steps, md.n_modes, std::sqrt(md.dt), zeta, vacc);
    CHECK_LAUNCH();
  }
  JitterArgs A{};
  A.P = make_params(md);
  A.n_steps = n_steps;
  A.m0 = m0;
  A.u0 = u0;
  A.dW = dW;
  A.phi = phi;
  A.m_end = m_end;
  A.u_end = u_end;
  A.theta = theta;
  A.rho = rho;
  A.n_jitter = n_jitter;
  A.n_accept = n_accept;
  A.accept_acc = accept_acc;
  A.iters_acc = iters_acc;
  A.n_obs = ob.n_obs;
  A.y = ob.y;
  A.sigma = ob.sigma;
  A.zeta = zeta;
  A.vacc = vacc;
  A.dLam = dLam;
  A.seed = seed;
  A.cycle = cycle;
  A.temper_k = temper_k;
  if (M) {
    A.M = *M;
    A.stage = zeta;
  }
  const size_t dyn = M ? 0 : 2 * sizeof(double) * static_cast<size_t>(n_steps) * md.n_modes;
  if (dyn > 32768) return fail(SCH_E_SHAPE, "n_steps * n_modes too large for the jitter kernel");
  const HelmConst K = make_helm(md, tl);
  return with_tile(tl, [&]<int PM, int NT, bool FULL>() -> int {
    // the workgroup's LDS (static solver and window arrays plus the
    // increments) must fit the 160 KiB of a compute unit
    constexpr size_t kStatic = sizeof(RowLds<NT>) + sizeof(AuxLds<PM, NT>);
    if (kStatic + dyn > 160 * 1024)
      return fail(SCH_E_SHAPE, "n_steps * n_modes too large for the jitter kernel at nx = %d",
                  md.nx);
    if (M && dLam)
      hipLaunchKernelGGL((k_jitter<PM, NT, FULL, true, true>), dim3(n), dim3(NT), 0, st, A, K);
    else if (M)
      hipLaunchKernelGGL((k_jitter<PM, NT, FULL, true>), dim3(n), dim3(NT), 0, st, A, K);
    else
      hipLaunchKernelGGL((k_jitter<PM, NT, FULL>), dim3(n), dim3(NT), dyn, st, A, K);
    CHECK_LAUNCH();
    return SCH_OK;
  });
}


// One batched adjoint evaluation of the gradient-based jitter at the
// increments x into g (defined with the timing below: its launches form the
// timing class SCH_TK_ADJOINT).
int adjoint_eval(const sch_model& md, const Tile& tl, const sch_obs& ob, int n, int n_steps,
                 const double* m0, const double* u0, const double* x, double* g,
                 const PcnlWs& P, hipStream_t st);

// n_jitter pCN-Langevin moves of every particle's increments dW (pcnl.hpp):
// the proposal draws as launch_jitter, one adjoint evaluation at the current
// increments and one per proposal, the Metropolis-Hastings step per particle;
// then the window ends of the final increments are recomputed into
// (m_end, u_end).
int launch_pcnl(const sch_model& md, const Tile& tl, const sch_obs& ob, uint64_t seed,
                uint32_t cycle, uint32_t temper_k, int n, int n_steps, const double* m0,
                const double* u0, double* dW, double* phi, double* m_end, double* u_end,
                const double* theta, double rho, int n_jitter, int* n_accept,
                unsigned long long* iters_acc, const PcnlWs& P, hipStream_t st) {
  const int Q = md.n_modes, d = n_steps * Q;
  const int64_t total = static_cast<int64_t>(n) * d;
  const int gb = grid_for(total, 256);
  {
    const int64_t work = static_cast<int64_t>(n_jitter) * n * n_steps * ((Q + 1) / 2);
    hipLaunchKernelGGL(k_draw_pcn, dim3(grid_for(work, 256)), dim3(256), 0, st, seed,
                       cycle * static_cast<uint32_t>(n_steps), cycle, temper_k << 16, n_jitter, n,
                       n_steps, Q, std::sqrt(md.dt), P.zeta, P.vacc);
    CHECK_LAUNCH();
  }
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, P.nws.acc, 2);
  if (int rc = adjoint_eval(md, tl, ob, n, n_steps, m0, u0, dW, P.gx, P, st)) return rc;
  hipLaunchKernelGGL(k_pcnl_grad, dim3(gb), dim3(256), 0, st, total, 1.0 / md.dt, dW, P.gx);
  int* acc = n_accept ? n_accept : P.acc;
  const double srho = std::sqrt(1.0 - rho * rho), c = (1.0 - rho) * md.dt;
  for (int j = 0; j < n_jitter; ++j) {
    hipLaunchKernelGGL(k_pcnl_propose, dim3(gb), dim3(256), 0, st, total, rho, srho, c, theta, dW,
                       P.gx, P.zeta + static_cast<size_t>(j) * total, P.v);
    if (int rc = adjoint_eval(md, tl, ob, n, n_steps, m0, u0, P.v, P.gv, P, st)) return rc;
    hipLaunchKernelGGL(k_pcnl_accept, dim3(n), dim3(kWave), 0, st, d, rho, md.dt, theta,
                       P.vacc + static_cast<size_t>(j) * n, P.status, P.J, dW, P.gx, phi, P.v,
                       P.gv, acc, j == 0 ? 1 : 0);
    CHECK_LAUNCH();
  }
  if (n_jitter == 0) return SCH_OK;
  const size_t state = sizeof(double) * static_cast<size_t>(n) * md.nx;
  HIP_TRY(hipMemcpyAsync(m_end, m0, state, hipMemcpyDeviceToDevice, st));
  HIP_TRY(hipMemcpyAsync(u_end, u0, state, hipMemcpyDeviceToDevice, st));
  return launch_window(md, tl, n, n_steps, m_end, u_end, dW, nullptr, nullptr, nullptr,
                       iters_acc, st);
}

// n_jitter Hybrid Monte Carlo moves (pcnl.hpp) of every particle's
// increments: the draws as pCN (the normals give the velocities), the
// gradient at the current state, then per move n_leap leapfrog steps, each
// one adjoint evaluation at its new position, and the Metropolis test; the
// window ends of the final increments are recomputed as for pCNL.
int launch_hmc(const sch_model& md, const Tile& tl, const sch_obs& ob, uint64_t seed,
               uint32_t cycle, uint32_t temper_k, int n, int n_steps, const double* m0,
               const double* u0, double* dW, double* phi, double* m_end, double* u_end,
               const double* theta, int n_jitter, int* n_accept,
               unsigned long long* iters_acc, const PcnlWs& P, hipStream_t st) {
  const int Q = md.n_modes, d = n_steps * Q;
  const int64_t total = static_cast<int64_t>(n) * d;
  const int gb = grid_for(total, 256);
  {
    const int64_t work = static_cast<int64_t>(n_jitter) * n * n_steps * ((Q + 1) / 2);
    hipLaunchKernelGGL(k_draw_pcn, dim3(grid_for(work, 256)), dim3(256), 0, st, seed,
                       cycle * static_cast<uint32_t>(n_steps), cycle, temper_k << 16, n_jitter, n,
                       n_steps, Q, std::sqrt(md.dt), P.zeta, P.vacc);
    CHECK_LAUNCH();
  }
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, P.nws.acc, 2);
  if (int rc = adjoint_eval(md, tl, ob, n, n_steps, m0, u0, dW, P.gx, P, st)) return rc;
  hipLaunchKernelGGL(k_pcnl_grad, dim3(gb), dim3(256), 0, st, total, 1.0 / md.dt, dW, P.gx);
  int* acc = n_accept ? n_accept : P.acc;
  const double a = (0.5 * P.h) * md.dt, c = std::cos(P.h), s = std::sin(P.h);
  for (int j = 0; j < n_jitter; ++j) {
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, 256)), dim3(256), 0, st, P.bad, 0, n);
    const double* zj = P.zeta + static_cast<size_t>(j) * total;
    for (int l = 0; l < P.n_leap; ++l) {
      hipLaunchKernelGGL(k_hmc_step, dim3(gb), dim3(256), 0, st, total, d, l == 0 ? 1 : 0, a,
                         theta, c, s, dW, P.gx, zj, P.v, P.vel, P.gv, P.status, P.bad);
      if (int rc = adjoint_eval(md, tl, ob, n, n_steps, m0, u0, P.v, P.gv, P, st)) return rc;
      hipLaunchKernelGGL(k_pcnl_grad, dim3(gb), dim3(256), 0, st, total, 1.0 / md.dt, P.v, P.gv);
    }
    hipLaunchKernelGGL(k_hmc_accept, dim3(n), dim3(kWave), 0, st, d, a, md.dt, theta,
                       P.vacc + static_cast<size_t>(j) * n, P.status, P.bad, P.J, dW, P.gx, phi,
                       P.v, P.gv, P.vel, zj, acc, j == 0 ? 1 : 0);
    CHECK_LAUNCH();
  }
  if (n_jitter == 0) return SCH_OK;
  const size_t state = sizeof(double) * static_cast<size_t>(n) * md.nx;
  HIP_TRY(hipMemcpyAsync(m_end, m0, state, hipMemcpyDeviceToDevice, st));
  HIP_TRY(hipMemcpyAsync(u_end, u0, state, hipMemcpyDeviceToDevice, st));
  return launch_window(md, tl, n, n_steps, m_end, u_end, dW, nullptr, nullptr, nullptr,
                       iters_acc, st);
}

// Event-based timing of kernel classes (see sch_timing_enable).
struct Timing {
  bool on = false;
  double ms[SCH_TK_COUNT] = {};
  long long launches[SCH_TK_COUNT] = {};
  long long iters[SCH_TK_COUNT] = {};
  struct Pend {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Pend> pend;
  std::vector<hipEvent_t> pool;
  hipEvent_t get() {
    if (pool.empty()) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      return e;
    }
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
};
Timing g_tm;

struct TimedScope {
  int kind;
  hipStream_t st;
  hipEvent_t a = nullptr;
  // kind < 0: no timing
  TimedScope(int k, hipStream_t s) : kind(k), st(s) {
    if (k >= 0 && g_tm.on && (a = g_tm.get())) (void)hipEventRecord(a, st);
  }
  ~TimedScope() {
    if (!a) return;
    hipEvent_t b = g_tm.get();
    if (!b) return;
    (void)hipEventRecord(b, st);
    g_tm.pend.push_back({kind, a, b});
  }
};

int adjoint_eval(const sch_model& md, const Tile& tl, const sch_obs& ob, int n, int n_steps,
                 const double* m0, const double* u0, const double* x, double* g,
                 const PcnlWs& P, hipStream_t st) {
  TimedScope ts(SCH_TK_ADJOINT, st);
  return launch_nudge_grad(md, tl, ob, n, n_steps, n_steps, m0, u0, x, nullptr, P.ce, P.J, g,
                           P.status, nullptr, P.nws, st);
}

// Called after a stream synchronisation: all pending events have completed.
void timing_flush() {
  for (auto& p : g_tm.pend) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      g_tm.ms[p.kind] += ms;
      g_tm.launches[p.kind] += 1;
    }
    g_tm.pool.push_back(p.a);
    g_tm.pool.push_back(p.b);
  }
  g_tm.pend.clear();
}

}  // namespace

// ===========================================================================
// The tempering stage of the tempered and nudged cycles (section 3.1.2):
// W.phi holds each particle's potential (phi, or J = phi - log G for the
// nudged filter), W.m0/W.u0 the window-start states, W.dW the increments,
// (m, u) the window-end states, and dLam the fixed controls or null.  The
// temperature rises from 0 to 1 in adaptive steps; after each step the
// particles are resampled (start state, increments, controls, potential, end
// state) and jittered.  W.acc[0] and W.status hold the forecast's Picard
// iterations and statuses on entry.  M != null: the Matern-type noise (the
// increments are cells [n][n_steps][nx]).
int temper_loop(const sch_model& md, const Tile& tl, const sch_obs& ob, uint64_t seed,
                uint32_t cycle, int n, int n_steps, double thr, int n_bisect, double rho,
                int n_jitter, int max_temper, double* m, double* u, double* dLam,
                const CycleWs& W, sch_cycle_stats* stats, hipStream_t st,
                const MaternDev* M = nullptr, const PcnlWs* PW = nullptr) {
  void* stream = st;
  const int nx = md.nx, Q = M ? md.nx : md.n_modes;
  const size_t state = static_cast<size_t>(n) * nx, inc = static_cast<size_t>(n) * n_steps * Q;
  hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, st, W.scal, 0.0, int64_t(1));  // theta = 0
  int k = 0, rc = SCH_OK;
  double theta = 0.0, ess = 0.0;
  unsigned long long adj_iters[2] = {0, 0};  // forward and transposed, while timing
  int64_t psteps = static_cast<int64_t>(n) * n_steps;
  while (theta < 1.0) {
    if (k >= max_temper) {
      rc = SCH_E_DEGENERATE;
      fail(rc, "tempering did not reach theta = 1 in %d steps", max_temper);
      break;
    }
    {
      TimedScope ts(SCH_TK_TEMPER, st);
      if (int r2 = sch_temper_ess(n, W.phi, nullptr, W.scal + 0, thr, n_bisect, W.scal + 1, W.w,
                                  nullptr, W.scal + 2, stream))
        return r2;
    }
    {
      TimedScope ts(SCH_TK_RESAMPLE, st);
      hipLaunchKernelGGL(k_draw_uniform, dim3(1), dim3(64), 0, st, seed, 0u, cycle,
                         SCH_TAG_RESAMPLE << 24, static_cast<uint32_t>(k) << 16, W.scal + 3);
      if (int r2 = sch_resample(n, W.w, W.scal + 3, nullptr, 0.0, W.idx, W.degenerate, W.cum, stream))
        return r2;
    }
    {
      TimedScope ts(SCH_TK_GATHER, st);
      double* fields[4] = {W.m0, W.u0, m, u};
      for (double* f : fields) {
        if (int r2 = sch_gather(n, nx, W.idx, f, W.scratch, stream)) return r2;
        HIP_TRY(hipMemcpyAsync(f, W.scratch, sizeof(double) * state, hipMemcpyDeviceToDevice, st));
      }
      if (int r2 = sch_gather(n, static_cast<int64_t>(n_steps) * Q, W.idx, W.dW, W.scratch, stream))
        return r2;
      HIP_TRY(hipMemcpyAsync(W.dW, W.scratch, sizeof(double) * inc, hipMemcpyDeviceToDevice, st));
      if (int r2 = sch_gather(n, 1, W.idx, W.phi, W.scratch, stream)) return r2;
      HIP_TRY(hipMemcpyAsync(W.phi, W.scratch, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
      if (dLam) {
        if (int r2 = sch_gather(n, static_cast<int64_t>(n_steps) * Q, W.idx, dLam, W.scratch,
                                stream))
          return r2;
        HIP_TRY(hipMemcpyAsync(dLam, W.scratch, sizeof(double) * inc, hipMemcpyDeviceToDevice,
                               st));
      }
    }
    if (n_jitter > 0 && PW) {
      TimedScope ts(SCH_TK_JITTER, st);
      if (PW->hmc) {
        if (int r2 = launch_hmc(md, tl, ob, seed, cycle, static_cast<uint32_t>(k), n, n_steps,
                                W.m0, W.u0, W.dW, W.phi, m, u, W.scal + 0, n_jitter, nullptr,
                                W.acc + 2, *PW, st))
          return r2;
      } else {
        if (int r2 = launch_pcnl(md, tl, ob, seed, cycle, static_cast<uint32_t>(k), n, n_steps,
                                 W.m0, W.u0, W.dW, W.phi, m, u, W.scal + 0, rho, n_jitter,
                                 nullptr, W.acc + 2, *PW, st))
          return r2;
      }
      hipLaunchKernelGGL(k_sum_i32_u64, dim3(1), dim3(256), 0, st, n, PW->acc, W.acc + 1);
      if (g_tm.on)
        HIP_TRY(hipMemcpyAsync(adj_iters, PW->nws.acc, sizeof adj_iters, hipMemcpyDeviceToHost,
                               st));
      // forward windows: the gradient at the start, one per proposal (n_leap per HMC
      // move), the end-state rerun
      psteps += static_cast<int64_t>(n) * n_steps *
                (static_cast<int64_t>(n_jitter) * (PW->hmc ? PW->n_leap : 1) + 2);
    } else if (n_jitter > 0) {
      TimedScope ts(SCH_TK_JITTER, st);
      if (int r2 = launch_jitter(md, tl, ob, seed, cycle, static_cast<uint32_t>(k), n, n_steps,
                                 W.m0, W.u0, W.dW, W.phi, m, u, W.scal + 0, rho, n_jitter,
                                 nullptr, W.acc + 1, W.acc + 2, W.zeta, W.vacc, dLam, st, M))
        return r2;
      psteps += static_cast<int64_t>(n) * n_steps * n_jitter;
    }
    HIP_TRY(hipMemcpyAsync(&theta, W.scal + 0, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(&ess, W.scal + 2, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    timing_flush();
    // the adjoint evaluations of a gradient-based stage: the Picard iterations
    // of their forward sweeps count with the stage's, the transposed ones with
    // their own class
    g_tm.iters[SCH_TK_JITTER] += static_cast<long long>(adj_iters[0]);
    g_tm.iters[SCH_TK_ADJOINT] += static_cast<long long>(adj_iters[1]);
    adj_iters[0] = adj_iters[1] = 0;
    ++k;
    if (!(ess > 0.0)) {
      rc = SCH_E_DEGENERATE;
      fail(rc, "all weights vanished in cycle %u", cycle);
      break;
    }
  }
  unsigned long long acc[3] = {0, 0, 0};
  std::vector<int> status(n);
  HIP_TRY(hipMemcpyAsync(acc, W.acc, sizeof acc, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(status.data(), W.status, sizeof(int) * n, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  timing_flush();
  g_tm.iters[SCH_TK_WINDOW] += static_cast<long long>(acc[0]);
  g_tm.iters[SCH_TK_JITTER] += static_cast<long long>(acc[2]);
  stats->ess = ess;
  stats->n_temper = k;
  stats->picard_iters = static_cast<int64_t>(acc[0] + acc[2]);
  stats->n_accept = static_cast<int64_t>(acc[1]);
  stats->particle_steps = psteps;
  for (int p = 0; p < n; ++p) stats->n_failed += status[p] != SCH_OK;
  stats->status = rc;
  return rc;
}

extern "C" {

int sch_tune_set(int32_t key, int32_t value) {
  if (key == SCH_TUNE_THREADS && (value == 0 || (value >= 64 && value <= 512 &&
                                                 (value & (value - 1)) == 0))) {
    g_tune_threads = value;
    return SCH_OK;
  }
  return fail(SCH_E_ARG, "bad tuning key %d or value %d", key, value);
}

int sch_tune_get(int32_t key) {
  if (key == SCH_TUNE_THREADS) return g_tune_threads;
  return -1;
}

int sch_timing_enable(int on) {
  g_tm.on = on != 0;
  return SCH_OK;
}

int sch_timing_reset(void) {
  for (int k = 0; k < SCH_TK_COUNT; ++k) {
    g_tm.ms[k] = 0.0;
    g_tm.launches[k] = 0;
    g_tm.iters[k] = 0;
  }
  return SCH_OK;
}

int sch_timing_read(double* ms, int64_t* launches, int64_t* iters) {
  for (int k = 0; k < SCH_TK_COUNT; ++k) {
    if (ms) ms[k] = g_tm.ms[k];
    if (launches) launches[k] = g_tm.launches[k];
    if (iters) iters[k] = g_tm.iters[k];
  }
  return SCH_OK;
}

const char* sch_last_error(void) { return g_err.c_str(); }

int sch_version(void) { return 100; }

size_t sch_workspace_bytes(int32_t which, const sch_model* model, int32_t n, int32_t n_steps,
                           int32_t extra) {
  if (n < 1) return 0;
  if (which == SCH_WS_RESAMPLE) return static_cast<size_t>(n) * sizeof(unsigned long long) + 256;
  if (!model || extra < 0) return 0;
  size_t bytes = 0;
  if (which == SCH_WS_NUDGE_GRAD || which == SCH_WS_NUDGE) {
    if (n_steps < 1 || extra < 1) return 0;
    carve_nudge(nullptr, which == SCH_WS_NUDGE, model->nx, model->n_modes, n, n_steps, extra,
                &bytes);
    return bytes;
  }
  const int n_jitter = extra;
  carve_cycle(nullptr, which, model->nx, model->n_modes, n, n_steps > 0 ? n_steps : 1, &bytes,
              n_jitter);
  return bytes;
}

int sch_draw_increments(const sch_rng* rng, uint32_t tag, int32_t n, int32_t n_steps,
                        int32_t n_modes, double dt, double* dW, void* stream) {
  if (!rng || !dW || n < 1 || n_steps < 1 || n_modes < 1 || !(dt > 0) || tag > 255)
    return fail(SCH_E_ARG, "bad arguments to sch_draw_increments");
  const int64_t work = static_cast<int64_t>(n) * n_steps * ((n_modes + 1) / 2);
  hipLaunchKernelGGL(k_draw_increments, dim3(grid_for(work, 256)), dim3(256), 0, S(stream),
                     rng->seed, rng->cycle * static_cast<uint32_t>(n_steps), tag,
                     rng->temper_k << 16, n, n_steps, n_modes, std::sqrt(dt), dW);
  CHECK_LAUNCH();
  return SCH_OK;
}

int sch_philox_blocks(uint64_t seed, int32_t n, const uint32_t* ctr, uint32_t* out,
                      void* stream) {
  if (n < 1 || !ctr || !out) return fail(SCH_E_ARG, "bad arguments to sch_philox_blocks");
  hipLaunchKernelGGL(k_philox_blocks, dim3(grid_for(n, 256)), dim3(256), 0, S(stream), seed, n,
                     ctr, out);
  CHECK_LAUNCH();
  return SCH_OK;
}

int sch_velocity(const sch_model* md, int32_t n, const double* m, double* u, void* stream) {
  Tile tl;
  if (int rc = check_model(md, tl)) return rc;
  if (n < 1 || !m || !u || m == u) return fail(SCH_E_ARG, "bad arguments to sch_velocity");
  return launch_helm(*md, tl, n, m, u, 0, S(stream));
}

int sch_init_momentum(const sch_model* md, int32_t n, const double* u, double* m, void* stream) {
  Tile tl;
  if (int rc = check_model(md, tl)) return rc;
  if (n < 1 || !m || !u || m == u) return fail(SCH_E_ARG, "bad arguments to sch_init_momentum");
  return launch_helm(*md, tl, n, u, m, 1, S(stream));
}

int sch_ensemble_step(const sch_model* md, int32_t n, int32_t n_steps, double* m, double* u,
                      const double* dW, const double* dLam, int32_t* status, int32_t* iters,
                      void* stream) {
  Tile tl;
  if (int rc = check_model(md, tl)) return rc;
  if (n < 1 || n_steps < 0 || !m || !u || !dW) return fail(SCH_E_ARG, "bad arguments to sch_ensemble_step");
  if (n_steps == 0) return SCH_OK;
  return launch_window(*md, tl, n, n_steps, m, u, dW, dLam, status, iters, nullptr, S(stream));
}

int sch_observe(const sch_model* md, int32_t n_obs, int32_t n, const double* u, double* out,
                void* stream) {
  if (!md || md->nx < 2 || n_obs < 1 || n < 1 || !u || !out) return fail(SCH_E_ARG, "bad arguments to sch_observe");
  hipLaunchKernelGGL(k_observe, dim3(n), dim3(kWave), 0, S(stream), md->nx, n_obs, u, out);
  CHECK_LAUNCH();
  return SCH_OK;
}

int sch_loglik(const sch_model* md, const sch_obs* ob, int32_t n, const double* u, double* phi,
               void* stream) {
  if (!md || md->nx < 2 || n < 1 || !u || !phi) return fail(SCH_E_ARG, "bad arguments to sch_loglik");
  if (int rc = check_obs(ob)) return rc;
  hipLaunchKernelGGL(k_loglik, dim3(n), dim3(kWave), 0, S(stream), md->nx, ob->n_obs, u, ob->y,
                     ob->sigma, phi);
  CHECK_LAUNCH();
  return SCH_OK;
}

int sch_temper_ess(int32_t n, const double* phi, const double* logw_extra, double* theta,
                   double thr, int32_t n_bisect, double* dtheta, double* w, double* logw_out,
                   double* ess, void* stream) {
  if (n < 1 || n > 65536 || !phi || !theta || !dtheta || !w || !ess || n_bisect < 0 ||
      n_bisect > 200)
    return fail(SCH_E_ARG, "bad arguments to sch_temper_ess");
  hipLaunchKernelGGL(k_temper, dim3(1), dim3(kTB), 0, S(stream), n, phi, logw_extra, theta, thr,
                     n_bisect, dtheta, w, logw_out, ess);
  CHECK_LAUNCH();
  return SCH_OK;
}

int sch_resample(int32_t n, const double* w, const double* u0, const double* cond_ess,
                 double cond_thr, int32_t* idx, int32_t* degenerate, void* workspace,
                 void* stream) {
  if (n < 1 || n > (1 << 24) || !w || !u0 || !idx || !workspace)
    return fail(SCH_E_ARG, "bad arguments to sch_resample");
  hipLaunchKernelGGL(k_resample, dim3(1), dim3(kTB), 0, S(stream), n, w, u0, cond_ess, cond_thr,
                     idx, degenerate, static_cast<unsigned long long*>(workspace));
  CHECK_LAUNCH();
  return SCH_OK;
}

int sch_gather(int32_t n_rows, int64_t row_len, const int32_t* idx, const double* src,
               double* dst, void* stream) {
  if (n_rows < 1 || n_rows > 65535 || row_len < 1 || !idx || !src || !dst || src == dst)
    return fail(SCH_E_ARG, "bad arguments to sch_gather");
  const int gx = static_cast<int>(std::min<int64_t>((row_len + 255) / 256, 64));
  hipLaunchKernelGGL(k_gather, dim3(gx, n_rows), dim3(256), 0, S(stream), n_rows, row_len, idx,
                     src, dst);
  CHECK_LAUNCH();
  return SCH_OK;
}

static int check_jitter_args(const sch_model* md, const sch_obs* ob, const sch_rng* rng,
                             int32_t n, int32_t n_steps, const double* m0, const double* u0,
                             const double* dW, const double* phi, const double* m_end,
                             const double* u_end, const double* theta, double rho,
                             int32_t n_jitter, Tile& tl, const char* who) {
  if (int rc = check_model(md, tl)) return rc;
  if (int rc = check_obs(ob)) return rc;
  if (!rng || n < 1 || n_steps < 1 || !m0 || !u0 || !dW || !phi || !m_end || !u_end || !theta ||
      !(rho >= 0 && rho <= 1) || n_jitter < 0)
    return fail(SCH_E_ARG, "bad arguments to %s", who);
  return SCH_OK;
}

int sch_jitter_pcn(const sch_model* md, const sch_obs* ob, const sch_rng* rng, int32_t n,
                   int32_t n_steps, const double* m0, const double* u0, double* dW,
                   const double* dLambda, double* phi, double* m_end, double* u_end,
                   const double* theta, double rho, int32_t n_jitter, int32_t* n_accept,
                   void* workspace, void* stream) {
  Tile tl;
  if (int rc = check_jitter_args(md, ob, rng, n, n_steps, m0, u0, dW, phi, m_end, u_end, theta,
                                 rho, n_jitter, tl, "sch_jitter_pcn"))
    return rc;
  if (n_jitter > 0 && !workspace) return fail(SCH_E_ARG, "sch_jitter_pcn: workspace is NULL");
  if (n_jitter == 0) return SCH_OK;
  CycleWs W = carve_cycle(workspace, SCH_WS_JITTER, md->nx, md->n_modes, n, n_steps, nullptr,
                          n_jitter);
  return launch_jitter(*md, tl, *ob, rng->seed, rng->cycle, rng->temper_k, n, n_steps, m0, u0,
                       dW, phi, m_end, u_end, theta, rho, n_jitter, n_accept, nullptr, nullptr,
                       W.zeta, W.vacc, dLambda, S(stream));
}

}  // extern "C"

// ---------------------------------------------------------------------------
// The jitter without a workspace: the proposal normals and acceptance
// uniforms go to a device array of the library, one per GPU, held until the
// process ends.  In host code `scratch` names a host-side stand-in, so the
// array's device address is taken with hipGetSymbolAddress once per device
// (with that device current) and only that address is used.
// ---------------------------------------------------------------------------
constexpr size_t kNoAllocScratchBytes = size_t(16) << 20;
static __device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the scratch array on the current device.
int scratch_of_current_device(void** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(SCH_E_ARG, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(SCH_E_HIP, "hipGetSymbolAddress returned NULL for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SCH_OK;
}
}  // namespace

extern "C" {

size_t sch_jitter_pcn_noalloc_max_bytes(void) { return kNoAllocScratchBytes; }

int sch_jitter_pcn_noalloc(const sch_model* md, const sch_obs* ob, const sch_rng* rng, int32_t n,
                           int32_t n_steps, const double* m0, const double* u0, double* dW,
                           const double* dLambda, double* phi, double* m_end, double* u_end,
                           const double* theta, double rho, int32_t n_jitter, int32_t* n_accept,
                           void* stream) {
  Tile tl;
  if (int rc = check_jitter_args(md, ob, rng, n, n_steps, m0, u0, dW, phi, m_end, u_end, theta,
                                 rho, n_jitter, tl, "sch_jitter_pcn_noalloc"))
    return rc;
  if (n_jitter == 0) return SCH_OK;
  size_t need = 0;
  carve_cycle(nullptr, SCH_WS_JITTER, md->nx, md->n_modes, n, n_steps, &need, n_jitter);
  if (need > kNoAllocScratchBytes)
    return fail(SCH_E_SHAPE,
                "sch_jitter_pcn_noalloc: %d moves x %d particles x %d steps x %d modes need %zu "
                "bytes of draws, above the library's %zu-byte scratch array; call sch_jitter_pcn "
                "with a workspace",
                n_jitter, n, n_steps, md->n_modes, need, kNoAllocScratchBytes);
  void* base = nullptr;
  if (int rc = scratch_of_current_device(&base)) return rc;
  CycleWs W = carve_cycle(base, SCH_WS_JITTER, md->nx, md->n_modes, n, n_steps, nullptr,
                          n_jitter);
  return launch_jitter(*md, tl, *ob, rng->seed, rng->cycle, rng->temper_k, n, n_steps, m0, u0,
                       dW, phi, m_end, u_end, theta, rho, n_jitter, n_accept, nullptr, nullptr,
                       W.zeta, W.vacc, dLambda, S(stream));
}

// ---------------------------------------------------------------------------
// Nudging.
// ---------------------------------------------------------------------------
int sch_nudge_grad(const sch_model* md, const sch_obs* ob, int32_t n, int32_t n_steps,
                   const double* m0, const double* u0, const double* dW, const double* dLam,
                   int32_t ce, double* J, double* grad, int32_t* status, void* workspace,
                   void* stream) {
  Tile tl;
  if (int rc = check_model(md, tl)) return rc;
  if (int rc = check_obs(ob)) return rc;
  if (n < 1 || n_steps < 1 || ce < 1 || !m0 || !u0 || !J || !grad || !workspace)
    return fail(SCH_E_ARG, "bad arguments to sch_nudge_grad");
  NudgeWs W = carve_nudge(workspace, false, md->nx, md->n_modes, n, n_steps, ce, nullptr);
  hipStream_t st = S(stream);
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, W.acc, 2);
  return launch_nudge_grad(*md, tl, *ob, n, n_steps, n_steps, m0, u0, dW, dLam, ce, J, grad,
                           status, nullptr, W, st);
}

}  // extern "C"

namespace {
// The stage-wise nudging of section 3.1.3 with the modes-form noise
// (M == null: n_modes controls per step) or the Matern-type noise (M != null:
// one control per cell, nx per step).
// mode (null: all particles warm or cold by warm_start) gives each
// particle's start: SCH_NUDGE_KEEP, _FROM_GIVEN or _FROM_ZERO, the given
// controls being in dLam.
int nudge_run(const sch_model* md, const Tile& tl, const sch_obs* ob, int32_t n, int32_t n_steps,
              double* m, double* u, const double* dW, double* dLam, int32_t warm_start,
              const sch_lbfgs_opts* opts, int32_t ce, double* logG, int32_t* lbfgs_status,
              int32_t* iters, int32_t* evals, int32_t* status, void* workspace, void* stream,
              const MaternDev* M, const int32_t* mode = nullptr) {
  if (!(opts->gtol >= 0) || opts->max_iter < 0 || opts->mem < 1 ||
      opts->mem > kLbfgsMaxMem || opts->max_back < 0 || opts->max_back > 60)
    return fail(SCH_E_ARG, "bad L-BFGS settings");
  hipStream_t st = S(stream);
  const int Q = M ? md->nx : md->n_modes;
  NudgeWs W = carve_nudge(workspace, true, md->nx, Q, n, n_steps, ce, nullptr);
  int* worst = lbfgs_status ? lbfgs_status : W.worst;
  int* its = iters ? iters : W.iters;
  int* evs = evals ? evals : W.evals;
  int* sts = status ? status : W.status;
  const int gb = grid_for(n, 256);
  hipLaunchKernelGGL(k_fill, dim3(gb), dim3(256), 0, st, logG, 0.0, int64_t(n));
  for (int* a : {worst, its, evs, sts})
    hipLaunchKernelGGL(k_fill_i32, dim3(gb), dim3(256), 0, st, a, 0, n);
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, W.acc, 2);
  CHECK_LAUNCH();
  LbfgsParams LP{n, Q, opts->mem, opts->max_iter, opts->max_back, opts->gtol, md->dt};
  const int64_t max_ev = 1 + static_cast<int64_t>(opts->max_iter) * (opts->max_back + 1);
  for (int s = 0; s < n_steps; ++s) {
    hipLaunchKernelGGL(k_lbfgs_init, dim3(gb), dim3(256), 0, st, W.lb, LP,
                       (warm_start || mode) ? dLam + static_cast<size_t>(s) * Q : nullptr,
                       n_steps * Q, mode);
    CHECK_LAUNCH();
    bool done = false;
    for (int64_t ev = 0; ev <= max_ev && !done; ++ev) {
      hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st,
                         reinterpret_cast<int*>(W.lb.n_active), 0, 1);
      {
        TimedScope ts(SCH_TK_NUDGE, st);
        if (int rc = launch_nudge_grad(*md, tl, *ob, n, n_steps - s, 1, m, u, nullptr, W.lb.xt,
                                       ce, W.lb.ft, W.lb.gt, W.lb.est, W.lb.active, W, st, M))
          return rc;
      }
      // one thread per particle for a few modes, one wavefront per particle
      // for one control per cell
      if (Q >= kWave)
        hipLaunchKernelGGL(k_lbfgs_update_w, dim3(grid_for(n, 256 / kWave)), dim3(256), 0, st,
                           W.lb, LP);
      else
        hipLaunchKernelGGL(k_lbfgs_update, dim3(gb), dim3(256), 0, st, W.lb, LP);
      CHECK_LAUNCH();
      unsigned int act = 0;
      HIP_TRY(hipMemcpyAsync(&act, W.lb.n_active, sizeof act, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      timing_flush();
      done = act == 0;
    }
    if (!done) return fail(SCH_E_ARG, "L-BFGS did not stop within its evaluation bound");
    hipLaunchKernelGGL(k_nudge_commit, dim3(gb), dim3(256), 0, st, W.lb, LP, n_steps, s, dW,
                       dLam, W.inc1, logG, worst, its, evs, md->dt);
    CHECK_LAUNCH();
    {
      TimedScope ts(SCH_TK_WINDOW, st);
      if (int rc = launch_window(*md, tl, n, 1, m, u, W.inc1, nullptr, W.tmp, nullptr, W.acc, st,
                                 M))
        return rc;
    }
    hipLaunchKernelGGL(k_status_merge, dim3(gb), dim3(256), 0, st, sts, W.tmp, n);
    CHECK_LAUNCH();
  }
  unsigned long long acc[2] = {0, 0};
  HIP_TRY(hipMemcpyAsync(acc, W.acc, sizeof acc, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  timing_flush();
  g_tm.iters[SCH_TK_NUDGE] += static_cast<long long>(acc[0] + acc[1]);
  return SCH_OK;
}

}  // namespace

extern "C" {

int sch_nudge_run(const sch_model* md, const sch_obs* ob, int32_t n, int32_t n_steps, double* m,
                  double* u, const double* dW, double* dLam, int32_t warm_start,
                  const sch_lbfgs_opts* opts, int32_t ce, double* logG, int32_t* lbfgs_status,
                  int32_t* iters, int32_t* evals, int32_t* status, void* workspace,
                  void* stream) {
  Tile tl;
  if (int rc = check_model(md, tl)) return rc;
  if (int rc = check_obs(ob)) return rc;
  if (n < 1 || n_steps < 1 || ce < 1 || !m || !u || !dW || !dLam || !logG || !opts ||
      !workspace)
    return fail(SCH_E_ARG, "bad arguments to sch_nudge_run");
  return nudge_run(md, tl, ob, n, n_steps, m, u, dW, dLam, warm_start, opts, ce, logG,
                   lbfgs_status, iters, evals, status, workspace, stream, nullptr);
}

// ---------------------------------------------------------------------------
// Filter cycles.
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {
// The bootstrap cycle of section 3.1.1 with the modes-form noise (M == null)
// or the Matern-type noise (M != null: nx cell increments per step).
int bootstrap_cycle(const sch_model* md, const Tile& tl, const sch_obs* ob, uint64_t seed,
                    uint32_t cycle, int32_t n, int32_t n_steps, double ess_frac, double* m,
                    double* u, double* logw, void* workspace, sch_cycle_stats* stats,
                    void* stream, const MaternDev* M) {
  hipStream_t st = S(stream);
  const int nx = md->nx, Q = M ? md->nx : md->n_modes;
  CycleWs W = carve_cycle(workspace, SCH_WS_BOOTSTRAP, nx, Q, n, n_steps, nullptr, 0, M ? 1 : 0);
  *stats = sch_cycle_stats{};
  sch_rng rg{seed, cycle, 0};
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, W.acc, 4);
  {
    TimedScope ts(SCH_TK_OTHER, st);
    if (int rc = sch_draw_increments(&rg, SCH_TAG_FORECAST, n, n_steps, Q, md->dt, W.dW, stream))
      return rc;
  }
  {
    TimedScope ts(SCH_TK_WINDOW, st);
    if (int rc = launch_window(*md, tl, n, n_steps, m, u, W.dW, nullptr, W.status, W.iters, W.acc,
                               st, M))
      return rc;
  }
  {
    TimedScope ts(SCH_TK_OTHER, st);
    if (int rc = sch_loglik(md, ob, n, u, W.phi, stream)) return rc;
    hipLaunchKernelGGL(k_mask_failed, dim3(grid_for(n, 256)), dim3(256), 0, st, n, W.status,
                       W.phi);
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, st, W.scal, 0.0, int64_t(1));  // theta = 0
  }
  {
    TimedScope ts(SCH_TK_TEMPER, st);
    if (int rc = sch_temper_ess(n, W.phi, logw, W.scal + 0, 0.0, 0, W.scal + 1, W.w, logw,
                                W.scal + 2, stream))
      return rc;
  }
  double ess = 0.0;
  unsigned long long its = 0;
  HIP_TRY(hipMemcpyAsync(&ess, W.scal + 2, sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(&its, W.acc, sizeof its, hipMemcpyDeviceToHost, st));
  std::vector<int> status(n);
  HIP_TRY(hipMemcpyAsync(status.data(), W.status, sizeof(int) * n, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  timing_flush();
  g_tm.iters[SCH_TK_WINDOW] += static_cast<long long>(its);
  stats->ess = ess;
  stats->picard_iters = static_cast<int64_t>(its);
  stats->particle_steps = static_cast<int64_t>(n) * n_steps;
  int rc = SCH_OK;
  for (int p = 0; p < n; ++p) stats->n_failed += status[p] != SCH_OK;
  if (!(ess > 0.0)) {
    stats->status = SCH_E_DEGENERATE;
    return fail(SCH_E_DEGENERATE, "all weights vanished in cycle %u", cycle);
  }
  if (ess < ess_frac * n) {
    {
      TimedScope ts(SCH_TK_RESAMPLE, st);
      hipLaunchKernelGGL(k_draw_uniform, dim3(1), dim3(64), 0, st, seed, 0u, cycle,
                         SCH_TAG_RESAMPLE << 24, 0u, W.scal + 3);
      if (int r2 = sch_resample(n, W.w, W.scal + 3, nullptr, 0.0, W.idx, W.degenerate, W.cum, stream))
        return r2;
    }
    TimedScope ts(SCH_TK_GATHER, st);
    if (int r2 = sch_gather(n, nx, W.idx, m, W.scratch, stream)) return r2;
    HIP_TRY(hipMemcpyAsync(m, W.scratch, sizeof(double) * n * nx, hipMemcpyDeviceToDevice, st));
    if (int r2 = sch_gather(n, nx, W.idx, u, W.scratch, stream)) return r2;
    HIP_TRY(hipMemcpyAsync(u, W.scratch, sizeof(double) * n * nx, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n, 256)), dim3(256), 0, st, logw, 0.0, int64_t(n));
    CHECK_LAUNCH();
    stats->resampled = 1;
  }
  HIP_TRY(hipStreamSynchronize(st));
  timing_flush();
  stats->status = rc;
  return SCH_OK;
}
}  // namespace

extern "C" {

int sch_pf_bootstrap_cycle(const sch_model* md, const sch_obs* ob, uint64_t seed, uint32_t cycle,
                           int32_t n, int32_t n_steps, double ess_frac, double* m, double* u,
                           double* logw, void* workspace, sch_cycle_stats* stats,
                           void* stream) {
  Tile tl;
  if (int rc = check_model(md, tl)) return rc;
  if (int rc = check_obs(ob)) return rc;
  if (n < 1 || n > 65535 || n_steps < 1 || !m || !u || !logw || !workspace || !stats)
    return fail(SCH_E_ARG, "bad arguments to sch_pf_bootstrap_cycle");
  return bootstrap_cycle(md, tl, ob, seed, cycle, n, n_steps, ess_frac, m, u, logw, workspace,
                         stats, stream, nullptr);
}

int sch_pf_tempered_cycle(const sch_model* md, const sch_obs* ob, uint64_t seed, uint32_t cycle,
                          int32_t n, int32_t n_steps, double thr, int32_t n_bisect, double rho,
                          int32_t n_jitter, int32_t max_temper, double* m, double* u,
                          void* workspace, sch_cycle_stats* stats, void* stream) {
  Tile tl;
  if (int rc = check_model(md, tl)) return rc;
  if (int rc = check_obs(ob)) return rc;
  if (n < 1 || n > 65535 || n_steps < 1 || !m || !u || !workspace || !stats || n_bisect < 0 ||
      max_temper < 1 || !(rho >= 0 && rho <= 1) || n_jitter < 0)
    return fail(SCH_E_ARG, "bad arguments to sch_pf_tempered_cycle");
  hipStream_t st = S(stream);
  const int nx = md->nx, Q = md->n_modes;
  const size_t state = static_cast<size_t>(n) * nx;
  CycleWs W = carve_cycle(workspace, SCH_WS_TEMPERED, nx, Q, n, n_steps, nullptr, n_jitter);
  *stats = sch_cycle_stats{};
  sch_rng rg{seed, cycle, 0};
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, W.acc, 4);
  {
    TimedScope ts(SCH_TK_GATHER, st);
    HIP_TRY(hipMemcpyAsync(W.m0, m, sizeof(double) * state, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(W.u0, u, sizeof(double) * state, hipMemcpyDeviceToDevice, st));
  }
  {
    TimedScope ts(SCH_TK_OTHER, st);
    if (int rc = sch_draw_increments(&rg, SCH_TAG_FORECAST, n, n_steps, Q, md->dt, W.dW, stream))
      return rc;
  }
  {
    TimedScope ts(SCH_TK_WINDOW, st);
    if (int rc = launch_window(*md, tl, n, n_steps, m, u, W.dW, nullptr, W.status, W.iters, W.acc, st))
      return rc;
  }
  {
    TimedScope ts(SCH_TK_OTHER, st);
    if (int rc = sch_loglik(md, ob, n, u, W.phi, stream)) return rc;
    hipLaunchKernelGGL(k_mask_failed, dim3(grid_for(n, 256)), dim3(256), 0, st, n, W.status,
                       W.phi);
  }
  return temper_loop(*md, tl, *ob, seed, cycle, n, n_steps, thr, n_bisect, rho, n_jitter,
                     max_temper, m, u, nullptr, W, stats, st);
}

}  // extern "C"

namespace {
// Scratch of the nudged cycle: the tempered cycle's, then the nudging's, then
// log G [n]; q controls per step (n_modes, or nx for the Matern-type noise).
size_t nudged_bytes(const sch_model& md, int n, int n_steps, int n_jitter, int ce, bool matern,
                    size_t* a, size_t* b) {
  const int q = matern ? md.nx : md.n_modes;
  carve_cycle(nullptr, SCH_WS_TEMPERED, md.nx, q, n, n_steps, a, n_jitter, matern ? 1 : 0);
  carve_nudge(nullptr, true, md.nx, q, n, n_steps, ce, b);
  return ((*a + 255) & ~size_t(255)) + ((*b + 255) & ~size_t(255)) +
         static_cast<size_t>(n) * sizeof(double) + 256;
}

// The nudged filter's cycle (section 3.1.3, last paragraph, with the
// tempering and jittering of section 3.1.2) with the modes-form noise
// (M == null) or the Matern-type noise (M != null: cells and controls per
// cell).
// mode == null: plain nudging from zero controls; otherwise dLambda holds the
// start controls and mode[p] each particle's start (nudge_run).
int nudged_cycle(const sch_model* md, const Tile& tl, const sch_obs* ob, uint64_t seed,
                 uint32_t cycle, int32_t n, int32_t n_steps, double thr, int32_t n_bisect,
                 double rho, int32_t n_jitter, int32_t max_temper, const sch_lbfgs_opts* opts,
                 int32_t ckpt_every, double* m, double* u, double* dLambda, void* workspace,
                 sch_cycle_stats* stats, void* stream, const MaternDev* M,
                 const int32_t* mode = nullptr) {
  hipStream_t st = S(stream);
  const int nx = md->nx, Q = M ? md->nx : md->n_modes;
  const size_t state = static_cast<size_t>(n) * nx, inc = static_cast<size_t>(n) * n_steps * Q;
  size_t a = 0, b = 0;
  nudged_bytes(*md, n, n_steps, n_jitter, ckpt_every, M != nullptr, &a, &b);
  CycleWs W = carve_cycle(workspace, SCH_WS_TEMPERED, nx, Q, n, n_steps, nullptr, n_jitter,
                          M ? 1 : 0);
  char* nws = static_cast<char*>(workspace) + ((a + 255) & ~size_t(255));
  double* logG = reinterpret_cast<double*>(nws + ((b + 255) & ~size_t(255)));
  *stats = sch_cycle_stats{};
  sch_rng rg{seed, cycle, 0};
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, W.acc, 4);
  if (!mode)
    hipLaunchKernelGGL(k_fill, dim3(grid_for(static_cast<int64_t>(inc), 256)), dim3(256), 0, st,
                       dLambda, 0.0, static_cast<int64_t>(inc));
  CHECK_LAUNCH();
  {
    TimedScope ts(SCH_TK_GATHER, st);
    HIP_TRY(hipMemcpyAsync(W.m0, m, sizeof(double) * state, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(W.u0, u, sizeof(double) * state, hipMemcpyDeviceToDevice, st));
  }
  {
    TimedScope ts(SCH_TK_OTHER, st);
    if (int rc = sch_draw_increments(&rg, SCH_TAG_NUDGE, n, n_steps, Q, md->dt, W.dW, stream))
      return rc;
  }
  // sequential nudging of the window (from zero controls, or as mode says):
  // (m, u) become the nudged window ends, W.status the window statuses
  if (int rc = nudge_run(md, tl, ob, n, n_steps, m, u, W.dW, dLambda, 0, opts, ckpt_every, logG,
                         nullptr, nullptr, nullptr, W.status, nws, stream, M, mode))
    return rc;
  {
    TimedScope ts(SCH_TK_OTHER, st);
    if (int rc = sch_loglik(md, ob, n, u, W.phi, stream)) return rc;
    hipLaunchKernelGGL(k_nudged_potential, dim3(grid_for(n, 256)), dim3(256), 0, st, n, W.phi,
                       logG, W.status, W.phi);
    CHECK_LAUNCH();
  }
  return temper_loop(*md, tl, *ob, seed, cycle, n, n_steps, thr, n_bisect, rho, n_jitter,
                     max_temper, m, u, dLambda, W, stats, st, M);
}
}  // namespace

extern "C" {

size_t sch_nudged_workspace_bytes(const sch_model* md, int32_t n, int32_t n_steps,
                                  int32_t n_jitter, int32_t ckpt_every) {
  if (!md || n < 1 || n_steps < 1 || n_jitter < 0 || ckpt_every < 1) return 0;
  size_t a = 0, b = 0;
  return nudged_bytes(*md, n, n_steps, n_jitter, ckpt_every, false, &a, &b);
}

int sch_pf_nudged_cycle(const sch_model* md, const sch_obs* ob, uint64_t seed, uint32_t cycle,
                        int32_t n, int32_t n_steps, double thr, int32_t n_bisect, double rho,
                        int32_t n_jitter, int32_t max_temper, const sch_lbfgs_opts* opts,
                        int32_t ckpt_every, double* m, double* u, double* dLambda,
                        void* workspace, sch_cycle_stats* stats, void* stream) {
  Tile tl;
  if (int rc = check_model(md, tl)) return rc;
  if (int rc = check_obs(ob)) return rc;
  if (n < 1 || n > 65535 || n_steps < 1 || !m || !u || !dLambda || !workspace || !stats ||
      !opts || n_bisect < 0 || max_temper < 1 || !(rho >= 0 && rho <= 1) || n_jitter < 0 ||
      ckpt_every < 1)
    return fail(SCH_E_ARG, "bad arguments to sch_pf_nudged_cycle");
  return nudged_cycle(md, tl, ob, seed, cycle, n, n_steps, thr, n_bisect, rho, n_jitter,
                      max_temper, opts, ckpt_every, m, u, dLambda, workspace, stats, stream,
                      nullptr);
}

int sch_pf_nudged_cycle_warm(const sch_model* md, const sch_obs* ob, uint64_t seed,
                             uint32_t cycle, int32_t n, int32_t n_steps, double thr,
                             int32_t n_bisect, double rho, int32_t n_jitter, int32_t max_temper,
                             const sch_lbfgs_opts* opts, int32_t ckpt_every, double* m, double* u,
                             double* dLambda, const int32_t* mode, void* workspace,
                             sch_cycle_stats* stats, void* stream) {
  Tile tl;
  if (int rc = check_model(md, tl)) return rc;
  if (int rc = check_obs(ob)) return rc;
  if (n < 1 || n > 65535 || n_steps < 1 || !m || !u || !dLambda || !mode || !workspace ||
      !stats || !opts || n_bisect < 0 || max_temper < 1 || !(rho >= 0 && rho <= 1) ||
      n_jitter < 0 || ckpt_every < 1)
    return fail(SCH_E_ARG, "bad arguments to sch_pf_nudged_cycle_warm");
  return nudged_cycle(md, tl, ob, seed, cycle, n, n_steps, thr, n_bisect, rho, n_jitter,
                      max_temper, opts, ckpt_every, m, u, dLambda, workspace, stats, stream,
                      nullptr, mode);
}

// ---------------------------------------------------------------------------
// Matern-type noise (section 2, eqs. noise_solve and noise_solve2).
// ---------------------------------------------------------------------------
int sch_matern_field(const sch_model* md, const sch_matern* mt, int32_t n, const double* dWc,
                     double* dU, void* stream) {
  Tile tl;
  if (int rc = check_model(md, tl)) return rc;
  MaternDev M;
  if (int rc = make_matern(*md, mt, tl, M)) return rc;
  if (n < 1 || n > 65535 || !dWc || !dU) return fail(SCH_E_ARG, "bad arguments to sch_matern_field");
  const StepParams P = make_params(*md);
  return with_tile(tl, [&]<int PM, int NT, bool FULL>() -> int {
    hipLaunchKernelGGL((k_matern_field<PM, NT, FULL>), dim3(n), dim3(NT), 0, S(stream), P, M, dWc,
                       dU);
    CHECK_LAUNCH();
    return SCH_OK;
  });
}

int sch_ensemble_step_matern(const sch_model* md, const sch_matern* mt, int32_t n,
                             int32_t n_steps, double* m, double* u, const double* dWc,
                             int32_t* status, int32_t* iters, void* stream) {
  Tile tl;
  if (int rc = check_model(md, tl)) return rc;
  MaternDev M;
  if (int rc = make_matern(*md, mt, tl, M)) return rc;
  if (n < 1 || n > 65535 || n_steps < 0 || !m || !u || !dWc)
    return fail(SCH_E_ARG, "bad arguments to sch_ensemble_step_matern");
  if (n_steps == 0) return SCH_OK;
  return launch_window(*md, tl, n, n_steps, m, u, dWc, nullptr, status, iters, nullptr,
                       S(stream), &M);
}

size_t sch_matern_workspace_bytes(int32_t which, const sch_model* md, int32_t n, int32_t n_steps,
                                  int32_t extra) {
  if (!md || n < 1 || n_steps < 1 || extra < 0) return 0;
  size_t bytes = 0;
  if (which == SCH_WS_NUDGE_GRAD || which == SCH_WS_NUDGE) {
    if (extra < 1) return 0;
    carve_nudge(nullptr, which == SCH_WS_NUDGE, md->nx, md->nx, n, n_steps, extra, &bytes);
    return bytes;
  }
  if (which != SCH_WS_JITTER && which != SCH_WS_TEMPERED && which != SCH_WS_BOOTSTRAP) return 0;
  carve_cycle(nullptr, which, md->nx, md->nx, n, n_steps, &bytes, extra, 1);
  return bytes;
}

int sch_nudge_grad_matern(const sch_model* md, const sch_matern* mt, const sch_obs* ob, int32_t n,
                          int32_t n_steps, const double* m0, const double* u0, const double* dWc,
                          const double* dLamc, int32_t ce, double* J, double* grad,
                          int32_t* status, void* workspace, void* stream) {
  Tile tl;
  if (int rc = check_model(md, tl)) return rc;
  if (int rc = check_obs(ob)) return rc;
  MaternDev M;
  if (int rc = make_matern(*md, mt, tl, M)) return rc;
  if (n < 1 || n > 65535 || n_steps < 1 || ce < 1 || !m0 || !u0 || !J || !grad || !workspace)
    return fail(SCH_E_ARG, "bad arguments to sch_nudge_grad_matern");
  NudgeWs W = carve_nudge(workspace, false, md->nx, md->nx, n, n_steps, ce, nullptr);
  hipStream_t st = S(stream);
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, W.acc, 2);
  return launch_nudge_grad(*md, tl, *ob, n, n_steps, n_steps, m0, u0, dWc, dLamc, ce, J, grad,
                           status, nullptr, W, st, &M);
}

int sch_nudge_run_matern(const sch_model* md, const sch_matern* mt, const sch_obs* ob, int32_t n,
                         int32_t n_steps, double* m, double* u, const double* dWc, double* dLamc,
                         int32_t warm_start, const sch_lbfgs_opts* opts, int32_t ce, double* logG,
                         int32_t* lbfgs_status, int32_t* iters, int32_t* evals, int32_t* status,
                         void* workspace, void* stream) {
  Tile tl;
  if (int rc = check_model(md, tl)) return rc;
  if (int rc = check_obs(ob)) return rc;
  MaternDev M;
  if (int rc = make_matern(*md, mt, tl, M)) return rc;
  if (n < 1 || n > 65535 || n_steps < 1 || ce < 1 || !m || !u || !dWc || !dLamc || !logG ||
      !opts || !workspace)
    return fail(SCH_E_ARG, "bad arguments to sch_nudge_run_matern");
  return nudge_run(md, tl, ob, n, n_steps, m, u, dWc, dLamc, warm_start, opts, ce, logG,
                   lbfgs_status, iters, evals, status, workspace, stream, &M);
}

size_t sch_nudged_workspace_bytes_matern(const sch_model* md, int32_t n, int32_t n_steps,
                                         int32_t n_jitter, int32_t ckpt_every) {
  if (!md || n < 1 || n_steps < 1 || n_jitter < 0 || ckpt_every < 1) return 0;
  size_t a = 0, b = 0;
  return nudged_bytes(*md, n, n_steps, n_jitter, ckpt_every, true, &a, &b);
}

int sch_pf_nudged_cycle_matern(const sch_model* md, const sch_matern* mt, const sch_obs* ob,
                               uint64_t seed, uint32_t cycle, int32_t n, int32_t n_steps,
                               double thr, int32_t n_bisect, double rho, int32_t n_jitter,
                               int32_t max_temper, const sch_lbfgs_opts* opts, int32_t ckpt_every,
                               double* m, double* u, double* dLambdac, void* workspace,
                               sch_cycle_stats* stats, void* stream) {
  Tile tl;
  if (int rc = check_model(md, tl)) return rc;
  if (int rc = check_obs(ob)) return rc;
  MaternDev M;
  if (int rc = make_matern(*md, mt, tl, M)) return rc;
  if (n < 1 || n > 65535 || n_steps < 1 || !m || !u || !dLambdac || !workspace || !stats ||
      !opts || n_bisect < 0 || max_temper < 1 || !(rho >= 0 && rho <= 1) || n_jitter < 0 ||
      ckpt_every < 1)
    return fail(SCH_E_ARG, "bad arguments to sch_pf_nudged_cycle_matern");
  return nudged_cycle(md, tl, ob, seed, cycle, n, n_steps, thr, n_bisect, rho, n_jitter,
                      max_temper, opts, ckpt_every, m, u, dLambdac, workspace, stats, stream, &M);
}

}  // extern "C"

namespace {
int jitter_matern(const sch_model* md, const sch_matern* mt, const sch_obs* ob,
                  const sch_rng* rng, int32_t n, int32_t n_steps, const double* m0,
                  const double* u0, double* dWc, double* phi, double* m_end, double* u_end,
                  const double* theta, double rho, int32_t n_jitter, int32_t* n_accept,
                  void* workspace, void* stream, const double* dLamc) {
  Tile tl;
  if (int rc = check_model(md, tl)) return rc;
  if (int rc = check_obs(ob)) return rc;
  MaternDev M;
  if (int rc = make_matern(*md, mt, tl, M)) return rc;
  if (!rng || n < 1 || n > 65535 || n_steps < 1 || !m0 || !u0 || !dWc || !phi || !m_end ||
      !u_end || !theta || !(rho >= 0 && rho <= 1) || n_jitter < 0 ||
      (n_jitter > 0 && !workspace))
    return fail(SCH_E_ARG, "bad arguments to sch_jitter_pcn_matern");
  if (n_jitter == 0) return SCH_OK;
  CycleWs W = carve_cycle(workspace, SCH_WS_JITTER, md->nx, md->nx, n, n_steps, nullptr,
                          n_jitter, 1);
  return launch_jitter(*md, tl, *ob, rng->seed, rng->cycle, rng->temper_k, n, n_steps, m0, u0,
                       dWc, phi, m_end, u_end, theta, rho, n_jitter, n_accept, nullptr, nullptr,
                       W.zeta, nullptr, dLamc, S(stream), &M);
}
}  // namespace

extern "C" {

int sch_jitter_pcn_matern(const sch_model* md, const sch_matern* mt, const sch_obs* ob,
                          const sch_rng* rng, int32_t n, int32_t n_steps, const double* m0,
                          const double* u0, double* dWc, double* phi, double* m_end,
                          double* u_end, const double* theta, double rho, int32_t n_jitter,
                          int32_t* n_accept, void* workspace, void* stream) {
  return jitter_matern(md, mt, ob, rng, n, n_steps, m0, u0, dWc, phi, m_end, u_end, theta, rho,
                       n_jitter, n_accept, workspace, stream, nullptr);
}

int sch_jitter_pcn_matern_ctrl(const sch_model* md, const sch_matern* mt, const sch_obs* ob,
                               const sch_rng* rng, int32_t n, int32_t n_steps, const double* m0,
                               const double* u0, double* dWc, const double* dLamc, double* J,
                               double* m_end, double* u_end, const double* theta, double rho,
                               int32_t n_jitter, int32_t* n_accept, void* workspace,
                               void* stream) {
  if (!dLamc) return fail(SCH_E_ARG, "sch_jitter_pcn_matern_ctrl needs the controls");
  return jitter_matern(md, mt, ob, rng, n, n_steps, m0, u0, dWc, J, m_end, u_end, theta, rho,
                       n_jitter, n_accept, workspace, stream, dLamc);
}

int sch_pf_bootstrap_cycle_matern(const sch_model* md, const sch_matern* mt, const sch_obs* ob,
                                  uint64_t seed, uint32_t cycle, int32_t n, int32_t n_steps,
                                  double ess_frac, double* m, double* u, double* logw,
                                  void* workspace, sch_cycle_stats* stats, void* stream) {
  Tile tl;
  if (int rc = check_model(md, tl)) return rc;
  if (int rc = check_obs(ob)) return rc;
  MaternDev M;
  if (int rc = make_matern(*md, mt, tl, M)) return rc;
  if (n < 1 || n > 65535 || n_steps < 1 || !m || !u || !logw || !workspace || !stats)
    return fail(SCH_E_ARG, "bad arguments to sch_pf_bootstrap_cycle_matern");
  return bootstrap_cycle(md, tl, ob, seed, cycle, n, n_steps, ess_frac, m, u, logw, workspace,
                         stats, stream, &M);
}

// ---------------------------------------------------------------------------
// Gradient-based jitter (pCN-Langevin moves).
// ---------------------------------------------------------------------------
size_t sch_pcnl_workspace_bytes(int32_t which, const sch_model* md, int32_t n, int32_t n_steps,
                                int32_t n_jitter, int32_t ckpt_every) {
  if (!md || n < 1 || n_steps < 1 || n_jitter < 0 || ckpt_every < 1 ||
      (which != SCH_WS_JITTER && which != SCH_WS_TEMPERED))
    return 0;
  size_t a = 0, b = 0;
  if (which == SCH_WS_TEMPERED)
    carve_cycle(nullptr, SCH_WS_TEMPERED, md->nx, md->n_modes, n, n_steps, &a, 0);
  carve_pcnl(nullptr, md->nx, md->n_modes, n, n_steps, n_jitter, ckpt_every, &b);
  return ((a + 255) & ~size_t(255)) + b;
}

int sch_jitter_pcnl(const sch_model* md, const sch_obs* ob, const sch_rng* rng, int32_t n,
                    int32_t n_steps, const double* m0, const double* u0, double* dW, double* phi,
                    double* m_end, double* u_end, const double* theta, double rho,
                    int32_t n_jitter, int32_t ckpt_every, int32_t* n_accept, void* workspace,
                    void* stream) {
  Tile tl;
  if (int rc = check_model(md, tl)) return rc;
  if (int rc = check_obs(ob)) return rc;
  if (!rng || n < 1 || n > 65535 || n_steps < 1 || !m0 || !u0 || !dW || !phi || !m_end ||
      !u_end || !theta || !(rho >= 0 && rho < 1) || n_jitter < 0 || ckpt_every < 1 ||
      (n_jitter > 0 && !workspace))
    return fail(SCH_E_ARG, "bad arguments to sch_jitter_pcnl");
  if (n_jitter == 0) return SCH_OK;
  PcnlWs P = carve_pcnl(workspace, md->nx, md->n_modes, n, n_steps, n_jitter, ckpt_every, nullptr);
  return launch_pcnl(*md, tl, *ob, rng->seed, rng->cycle, rng->temper_k, n, n_steps, m0, u0, dW,
                     phi, m_end, u_end, theta, rho, n_jitter, n_accept, nullptr, P, S(stream));
}

}  // extern "C"

namespace {

// The tempered cycle with a gradient-based jitter (pCNL, or HMC when hmc):
// forecast, likelihood, then the tempering loop with those moves.
int gradient_cycle(const sch_model* md, const Tile& tl, const sch_obs* ob, uint64_t seed,
                   uint32_t cycle, int32_t n, int32_t n_steps, double thr, int32_t n_bisect,
                   double rho, int32_t n_jitter, int32_t max_temper, int32_t ckpt_every,
                   double* m, double* u, void* workspace, sch_cycle_stats* stats, void* stream,
                   bool hmc, double h, int32_t n_leap) {
  hipStream_t st = S(stream);
  const int nx = md->nx, Q = md->n_modes;
  const size_t state = static_cast<size_t>(n) * nx;
  size_t a = 0;
  CycleWs W = carve_cycle(workspace, SCH_WS_TEMPERED, nx, Q, n, n_steps, &a, 0);
  PcnlWs P = carve_pcnl(static_cast<char*>(workspace) + ((a + 255) & ~size_t(255)), nx, Q, n,
                        n_steps, n_jitter, ckpt_every, nullptr, hmc);
  P.h = h;
  P.n_leap = n_leap;
  *stats = sch_cycle_stats{};
  sch_rng rg{seed, cycle, 0};
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, W.acc, 4);
  {
    TimedScope ts(SCH_TK_GATHER, st);
    HIP_TRY(hipMemcpyAsync(W.m0, m, sizeof(double) * state, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(W.u0, u, sizeof(double) * state, hipMemcpyDeviceToDevice, st));
  }
  {
    TimedScope ts(SCH_TK_OTHER, st);
    if (int rc = sch_draw_increments(&rg, SCH_TAG_FORECAST, n, n_steps, Q, md->dt, W.dW, stream))
      return rc;
  }
  {
    TimedScope ts(SCH_TK_WINDOW, st);
    if (int rc = launch_window(*md, tl, n, n_steps, m, u, W.dW, nullptr, W.status, W.iters, W.acc, st))
      return rc;
  }
  {
    TimedScope ts(SCH_TK_OTHER, st);
    if (int rc = sch_loglik(md, ob, n, u, W.phi, stream)) return rc;
    hipLaunchKernelGGL(k_mask_failed, dim3(grid_for(n, 256)), dim3(256), 0, st, n, W.status,
                       W.phi);
  }
  return temper_loop(*md, tl, *ob, seed, cycle, n, n_steps, thr, n_bisect, rho, n_jitter,
                     max_temper, m, u, nullptr, W, stats, st, nullptr, &P);
}

}  // namespace

extern "C" {

int sch_pf_tempered_cycle_pcnl(const sch_model* md, const sch_obs* ob, uint64_t seed,
                               uint32_t cycle, int32_t n, int32_t n_steps, double thr,
                               int32_t n_bisect, double rho, int32_t n_jitter, int32_t max_temper,
                               int32_t ckpt_every, double* m, double* u, void* workspace,
                               sch_cycle_stats* stats, void* stream) {
  Tile tl;
  if (int rc = check_model(md, tl)) return rc;
  if (int rc = check_obs(ob)) return rc;
  if (n < 1 || n > 65535 || n_steps < 1 || !m || !u || !workspace || !stats || n_bisect < 0 ||
      max_temper < 1 || !(rho >= 0 && rho < 1) || n_jitter < 0 || ckpt_every < 1)
    return fail(SCH_E_ARG, "bad arguments to sch_pf_tempered_cycle_pcnl");
  return gradient_cycle(md, tl, ob, seed, cycle, n, n_steps, thr, n_bisect, rho, n_jitter,
                        max_temper, ckpt_every, m, u, workspace, stats, stream, false, 0.0, 0);
}

// ---------------------------------------------------------------------------
// Gradient-based jitter: Hybrid Monte Carlo moves.
// ---------------------------------------------------------------------------
size_t sch_hmc_workspace_bytes(int32_t which, const sch_model* md, int32_t n, int32_t n_steps,
                               int32_t n_jitter, int32_t ckpt_every) {
  if (!md || n < 1 || n_steps < 1 || n_jitter < 0 || ckpt_every < 1 ||
      (which != SCH_WS_JITTER && which != SCH_WS_TEMPERED))
    return 0;
  size_t a = 0, b = 0;
  if (which == SCH_WS_TEMPERED)
    carve_cycle(nullptr, SCH_WS_TEMPERED, md->nx, md->n_modes, n, n_steps, &a, 0);
  carve_pcnl(nullptr, md->nx, md->n_modes, n, n_steps, n_jitter, ckpt_every, &b, true);
  return ((a + 255) & ~size_t(255)) + b;
}

static bool hmc_ok(double h, int32_t n_leap) {
  return h > 0.0 && h < 3.14159 && n_leap >= 1 && n_leap <= 64;
}

int sch_jitter_hmc(const sch_model* md, const sch_obs* ob, const sch_rng* rng, int32_t n,
                   int32_t n_steps, const double* m0, const double* u0, double* dW, double* phi,
                   double* m_end, double* u_end, const double* theta, double h, int32_t n_leap,
                   int32_t n_jitter, int32_t ckpt_every, int32_t* n_accept, void* workspace,
                   void* stream) {
  Tile tl;
  if (int rc = check_model(md, tl)) return rc;
  if (int rc = check_obs(ob)) return rc;
  if (!rng || n < 1 || n > 65535 || n_steps < 1 || !m0 || !u0 || !dW || !phi || !m_end ||
      !u_end || !theta || !hmc_ok(h, n_leap) || n_jitter < 0 || ckpt_every < 1 ||
      (n_jitter > 0 && !workspace))
    return fail(SCH_E_ARG, "bad arguments to sch_jitter_hmc");
  if (n_jitter == 0) return SCH_OK;
  PcnlWs P = carve_pcnl(workspace, md->nx, md->n_modes, n, n_steps, n_jitter, ckpt_every,
                        nullptr, true);
  P.h = h;
  P.n_leap = n_leap;
  return launch_hmc(*md, tl, *ob, rng->seed, rng->cycle, rng->temper_k, n, n_steps, m0, u0, dW,
                    phi, m_end, u_end, theta, n_jitter, n_accept, nullptr, P, S(stream));
}

int sch_pf_tempered_cycle_hmc(const sch_model* md, const sch_obs* ob, uint64_t seed,
                              uint32_t cycle, int32_t n, int32_t n_steps, double thr,
                              int32_t n_bisect, double h, int32_t n_leap, int32_t n_jitter,
                              int32_t max_temper, int32_t ckpt_every, double* m, double* u,
                              void* workspace, sch_cycle_stats* stats, void* stream) {
  Tile tl;
  if (int rc = check_model(md, tl)) return rc;
  if (int rc = check_obs(ob)) return rc;
  if (n < 1 || n > 65535 || n_steps < 1 || !m || !u || !workspace || !stats || n_bisect < 0 ||
      max_temper < 1 || !hmc_ok(h, n_leap) || n_jitter < 0 || ckpt_every < 1)
    return fail(SCH_E_ARG, "bad arguments to sch_pf_tempered_cycle_hmc");
  return gradient_cycle(md, tl, ob, seed, cycle, n, n_steps, thr, n_bisect, 0.0, n_jitter,
                        max_temper, ckpt_every, m, u, workspace, stats, stream, true, h, n_leap);
}

// ---------------------------------------------------------------------------
// The paper's twin experiments (section 4).
// ---------------------------------------------------------------------------
int sch_paper_init(const sch_model* md, uint64_t seed, int32_t n, double* u, void* stream) {
  Tile tl;
  if (int rc = check_model(md, tl)) return rc;
  if (n < 1 || n > 65535 || !u) return fail(SCH_E_ARG, "bad arguments to sch_paper_init");
  const double h = md->L / md->nx;
  const sch_matern smooth{1.0, std::sqrt(h), 3};  // (I - d_xx), load h/2, three solves
  MaternDev M;
  if (int rc = make_matern(*md, &smooth, tl, M)) return rc;
  const StepParams P = make_params(*md);
  return with_tile(tl, [&]<int PM, int NT, bool FULL>() -> int {
    hipLaunchKernelGGL((k_paper_init<PM, NT, FULL>), dim3(n), dim3(NT), 0, S(stream), P, M, seed,
                       u);
    CHECK_LAUNCH();
    return SCH_OK;
  });
}

int sch_ensemble_stats(int32_t n, int32_t nx, const double* u, const double* ua,
                       double* workspace, double* out, void* stream) {
  if (n < 1 || n > 65535 || nx < 1 || !u || !ua || !workspace || !out)
    return fail(SCH_E_ARG, "bad arguments to sch_ensemble_stats");
  hipStream_t st = S(stream);
  double* mean = workspace;
  double* sq = workspace + nx;
  hipLaunchKernelGGL(k_ens_mean, dim3(grid_for(nx, 256)), dim3(256), 0, st, n, nx, u, mean);
  hipLaunchKernelGGL(k_ens_norms, dim3(n), dim3(kWave), 0, st, nx, u, ua, mean, sq);
  hipLaunchKernelGGL(k_ens_final, dim3(1), dim3(kWave), 0, st, n, nx, ua, mean, sq, out);
  CHECK_LAUNCH();
  return SCH_OK;
}

int sch_pf_tempered_cycle_matern(const sch_model* md, const sch_matern* mt, const sch_obs* ob,
                                 uint64_t seed, uint32_t cycle, int32_t n, int32_t n_steps,
                                 double thr, int32_t n_bisect, double rho, int32_t n_jitter,
                                 int32_t max_temper, double* m, double* u, void* workspace,
                                 sch_cycle_stats* stats, void* stream) {
  Tile tl;
  if (int rc = check_model(md, tl)) return rc;
  if (int rc = check_obs(ob)) return rc;
  MaternDev M;
  if (int rc = make_matern(*md, mt, tl, M)) return rc;
  if (n < 1 || n > 65535 || n_steps < 1 || !m || !u || !workspace || !stats || n_bisect < 0 ||
      max_temper < 1 || !(rho >= 0 && rho <= 1) || n_jitter < 0)
    return fail(SCH_E_ARG, "bad arguments to sch_pf_tempered_cycle_matern");
  hipStream_t st = S(stream);
  const int nx = md->nx;
  const size_t state = static_cast<size_t>(n) * nx;
  CycleWs W = carve_cycle(workspace, SCH_WS_TEMPERED, nx, nx, n, n_steps, nullptr, n_jitter, 1);
  *stats = sch_cycle_stats{};
  sch_rng rg{seed, cycle, 0};
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, W.acc, 4);
  {
    TimedScope ts(SCH_TK_GATHER, st);
    HIP_TRY(hipMemcpyAsync(W.m0, m, sizeof(double) * state, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(W.u0, u, sizeof(double) * state, hipMemcpyDeviceToDevice, st));
  }
  {
    TimedScope ts(SCH_TK_OTHER, st);
    // the cell increments: nx per step, N(0, dt) each
    if (int rc = sch_draw_increments(&rg, SCH_TAG_FORECAST, n, n_steps, nx, md->dt, W.dW, stream))
      return rc;
  }
  {
    TimedScope ts(SCH_TK_WINDOW, st);
    if (int rc = launch_window(*md, tl, n, n_steps, m, u, W.dW, nullptr, W.status, W.iters, W.acc,
                               st, &M))
      return rc;
  }
  {
    TimedScope ts(SCH_TK_OTHER, st);
    if (int rc = sch_loglik(md, ob, n, u, W.phi, stream)) return rc;
    hipLaunchKernelGGL(k_mask_failed, dim3(grid_for(n, 256)), dim3(256), 0, st, n, W.status,
                       W.phi);
  }
  return temper_loop(*md, tl, *ob, seed, cycle, n, n_steps, thr, n_bisect, rho, n_jitter,
                     max_temper, m, u, nullptr, W, stats, st, &M);
}

}  // extern "C"

#include "batch_abi.hpp"
#include "mlp_abi.hpp"
