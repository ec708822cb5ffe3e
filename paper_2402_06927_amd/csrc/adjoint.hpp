// adjoint.hpp -- gradient of the nudging objective (section 3.1.3) by the
// discrete adjoint of the implicit-midpoint window, and the batched L-BFGS
// that minimises it stage by stage.
//
// Objective of one particle over a window of S steps from (m^0, u^0):
//   J = Phi(u^S) + sum_{n < CS} ( |dLambda^n|^2 / 2 + dLambda^n . dW^n ) / dt,
// where only the first CS steps carry an increment dW and a control dLambda
// (both zero afterwards).  The second term is minus the log of the discrete
// Girsanov factor of the nudged path.
//
// With s = m^n + m^{n+1} a step solves F(s) = A(dv) s - 2 M m^n = 0 where
// dv = (dt/2) R s + dU^n, R = H^{-1} M.  Writing C(v) f = D(f) v, its
// Jacobian is Jac = A(dv) + (dt/4) D(s) R, and the reverse sweep is
//   lambda_S = M H^{-1} P^T diag(sigma^-2) (P u^S - y),
//   nu = Jac^{-T} lambda_{n+1},   lambda_n = 2 M nu - lambda_{n+1},
//   dJ/d(dU^n) = -(1/2) D(s)^T nu,
//   dJ/d(dLambda^n_q) = xi_q . dJ/d(dU^n) + (dLambda^n_q + dW^n_q) / dt.
// Jac^T nu = lambda is solved by the fixed point
//   nu <- A^{-T} (lambda - (dt/4) M H^{-1} D(s)^T nu)
// to the window's Picard tolerance.  A^T is again periodic tridiagonal with
// rows (c_{i-1}, b_i, a_{i+1}) = (h/6 - mu dt/(2h) + dv_i/4,
// 2h/3 + mu dt/h + (dv_{i+1} - dv_{i-1})/4, h/6 - mu dt/(2h) - dv_i/4).
//
// Memory: the forward pass stores (m, u) at the start of every segment of
// `ckpt_every` steps; the reverse pass recomputes each segment's states from
// its checkpoint into a per-particle segment buffer (the last segment's
// states are kept from the forward pass) and sweeps it backwards.
#pragma once

#include "model.hpp"

namespace sch {

struct NudgeArgs {
  StepParams P;
  int n_steps, ctrl_steps, ckpt_every;
  const double* m0;    // [n][nx]
  const double* u0;    // [n][nx]
  const double* dW;    // [n][ctrl_steps][Q] or null (zero); Matern: [n][ctrl_steps][nx]
  const double* dLam;  // [n][ctrl_steps][Q] or null (zero); Matern: [n][ctrl_steps][nx]
  int n_obs;
  const double* y;
  const double* sigma;
  double* J;           // [n]
  double* grad;        // [n][ctrl_steps][Q]
  int* status;         // [n] or null
  const int* active;   // [n] or null: particles with active[p] == 0 are skipped
  double* ckpt;        // [n][n_segments][2][nx]
  double* seg;         // [n][ckpt_every + 1][2][nx]
  unsigned long long* iters_acc;  // [2]: forward Picard and adjoint fixed-point iterations
  MaternDev M;                    // Matern-type noise (MATERN kernels)
};

// P^T diag(sigma^-2) (P u - y) at the chunk's nodes.  A point in cell e
// (fraction r) adds (1 - r) res to node e and r res to node e + 1; the thread
// walks the points of cells start-1 .. start+cnt-1 (one integer division per
// cell run) and keeps the shares that land on its own nodes.
template <int PMAX, int NT, bool FULL>
__device__ void obs_adjoint(const double (&u)[PMAX], const Chunk& ch, int nx, int n_obs,
                            const double* y, const double* sigma, double (&out)[PMAX],
                            RowLds<NT>& L, int t, int& hs) {
  double hl, hr;
  halo<PMAX, NT, FULL>(u, ch.cnt, L, t, hl, hr, hs);
  const double dn = static_cast<double>(n_obs);
#pragma unroll
  for (int j = 0; j < PMAX; ++j) out[j] = 0.0;
  {
    // the cell left of the chunk (periodic)
    const int64_t e = ch.start == 0 ? nx - 1 : ch.start - 1;
    const int64_t lim = (e + 1) * n_obs, base = e * n_obs;
    for (int64_t o = (base + nx - 1) / nx; o * nx < lim; ++o) {
      const double r = static_cast<double>(o * nx - base) / dn;
      const double s = sigma[o];
      const double res = ((1.0 - r) * hl + r * u[0] - y[o]) / (s * s);
      out[0] += r * res;
    }
  }
  int64_t o = (static_cast<int64_t>(ch.start) * n_obs + nx - 1) / nx;
#pragma unroll
  for (int j = 0; j < PMAX; ++j) {
    if (!FULL && j >= ch.cnt) continue;
    const int64_t node = ch.start + j;
    const int64_t lim = (node + 1) * n_obs, base = node * n_obs;
    const double ur = right_of<PMAX, FULL>(u, j, ch.cnt, hr);
    const bool own_next = (j + 1 < PMAX) && slot_live<PMAX, FULL>(j + 1, ch.cnt);
    for (; o * nx < lim; ++o) {
      const double r = static_cast<double>(o * nx - base) / dn;
      const double s = sigma[o];
      const double res = ((1.0 - r) * u[j] + r * ur - y[o]) / (s * s);
      out[j] += (1.0 - r) * res;
      if (own_next) out[j + 1 < PMAX ? j + 1 : j] += r * res;
    }
  }
}

// (D(s)^T v)_j = (s_{j-1} + s_j)/2 v_{j-1} - (s_j + s_{j+1})/2 v_{j+1}
template <int PMAX, bool FULL>
__device__ __forceinline__ void advect_t(const double (&s)[PMAX], double sl, double sr,
                                         const double (&v)[PMAX], double vl, double vr, int cnt,
                                         double scale, double (&out)[PMAX]) {
#pragma unroll
  for (int j = 0; j < PMAX; ++j) {
    const double sm = left_of<PMAX, FULL>(s, j, sl), sp = right_of<PMAX, FULL>(s, j, cnt, sr);
    const double vm = left_of<PMAX, FULL>(v, j, vl), vp = right_of<PMAX, FULL>(v, j, cnt, vr);
    out[j] = scale * (0.5 * (sm + s[j]) * vm - 0.5 * (s[j] + sp) * vp);
  }
}

// One reverse step: lam holds lambda_{n+1} on entry and lambda_n on exit,
// gdU receives dJ/d(dU^n).  (ma, ua) is the state before the step, (mb, ub)
// after it; noise(0, dv) adds the step's noise field dU^n.  Where the window's two
// LDS arrays exist (free during the reverse sweep), s and lambda_{n+1}, which
// the fixed-point loop only reads, wait there instead of in registers.  PWT
// selects the table form of the Helmholtz solves (solve_helm).
template <int PMAX, int NT, bool FULL, bool PWT, class NoiseF>
__device__ int adjoint_step(const StepParams& P, const HelmConst& K, NoiseF noise,
                            const double* ma, const double* ua, const double* mb,
                            const double* ub, double (&lam)[PMAX], double (&gdU)[PMAX],
                            const Chunk& ch, RowLds<NT>& L, AuxLds<PMAX, NT>& X, int t,
                            Parity& par, int& iters) {
  constexpr bool kL = AuxLds<PMAX, NT>::kInLds;
  const int cnt = ch.cnt;
  const double hdt = 0.5 * P.dt;
  double s[PMAX], dv[PMAX];
#pragma unroll
  for (int j = 0; j < PMAX; ++j) {
    if (slot_live<PMAX, FULL>(j, cnt)) {
      s[j] = ma[ch.start + j] + mb[ch.start + j];
      dv[j] = hdt * (ua[ch.start + j] + ub[ch.start + j]);
    } else {
      s[j] = 0.0;
      dv[j] = 0.0;
    }
  }
  noise(0, dv);  // + dU^n
  double sl, sr, vl, vr;
  halo<PMAX, NT, FULL>(s, cnt, L, t, sl, sr, par.hs);
  halo<PMAX, NT, FULL>(dv, cnt, L, t, vl, vr, par.hs);
  const double ao = P.a_off, ad = P.a_diag;
  auto rowAT = [&](int j, double& a, double& b, double& c) {
    const double vm = left_of<PMAX, FULL>(dv, j, vl);
    const double vp = right_of<PMAX, FULL>(dv, j, cnt, vr);
    a = fma(0.25, dv[j], ao);
    b = fma(0.25, vp - vm, ad);
    c = fma(-0.25, dv[j], ao);
  };
  // s and lambda_{n+1} from LDS (kL), each value laundered so that the
  // loads stay inside the loop instead of being hoisted into registers
  auto s_at = [&](double (&sv)[PMAX]) {
#pragma unroll
    for (int j = 0; j < PMAX; ++j) {
      double x = X.a[1][kL ? j : 0][kL ? t : 0];
      asm volatile("" : "+v"(x));
      sv[j] = x;
    }
  };
  auto lam_at = [&](int j) -> double {
    if constexpr (kL) {
      double x = X.a[0][j][t];
      asm volatile("" : "+v"(x));
      return x;
    } else {
      return lam[j];
    }
  };
  double nu[PMAX], rhs[PMAX];
#pragma unroll
  for (int j = 0; j < PMAX; ++j) {
    nu[j] = 0.0;
    rhs[j] = lam[j];
    if constexpr (kL) {
      X.a[0][j][t] = lam[j];
      X.a[1][j][t] = s[j];
    }
  }
  // the first solve gives A^{-T} lambda; picard_max corrections follow at most
  int status = SCH_E_NONCONVERGED, k = 1;
  double prevd = 0.0;  // the previous iteration's change of nu
  for (; k <= P.picard_max + 1; ++k) {
    double nn[PMAX];
    double xl_unused, xr_unused, grow = 0.0;
    cyclic_solve<PMAX, NT, FULL>(rowAT, [&](int j) { return rhs[j]; }, nn, cnt, L, t, xl_unused,
                                 xr_unused, grow);
    double diff = 0.0, scale = 0.0;
    // bit 0: a non-finite iterate; bit 1: elimination growth above kMaxGrowth
    int bad = grow <= kMaxGrowth ? 0 : 2;
#pragma unroll
    for (int j = 0; j < PMAX; ++j) {
      if (slot_live<PMAX, FULL>(j, cnt)) {
        diff = fmax(diff, fabs(nn[j] - nu[j]));
        scale = fmax(scale, fabs(nn[j]));
        bad |= !isfinite(nn[j]);
      }
      nu[j] = nn[j];
    }
    block_max2_or<NT>(diff, scale, bad, L, t);
    if (bad) {
      status = (bad & 2) ? SCH_E_UNSTABLE : SCH_E_NONFINITE;
      break;
    }
    // the stopping rule of the forward step: the estimated error
    // c / (1 - c) d_k, c = d_k / d_{k-1}, while c < 1/2 (the first change is
    // the first iterate's distance from the zero start)
    const double lim = P.tol * scale;
    const bool done = (k > 1 && 2.0 * diff < prevd) ? diff * diff <= lim * (prevd - diff)
                                                    : diff <= lim;
    prevd = diff;
    if (done) {
      status = SCH_OK;
      break;
    }
    // rhs = lambda - (dt/4) M H^{-1} D(s)^T nu
    double nl, nr, w[PMAX], z[PMAX];
    halo<PMAX, NT, FULL>(nu, cnt, L, t, nl, nr, par.hs);
    if constexpr (kL) {
      double sv[PMAX];
      s_at(sv);
      advect_t<PMAX, FULL>(sv, sl, sr, nu, nl, nr, cnt, 1.0, w);
    } else {
      advect_t<PMAX, FULL>(s, sl, sr, nu, nl, nr, cnt, 1.0, w);
    }
    // M H^{-1} w = H^{-1} M w (the two circulants commute): the mass product
    // folded into the scan form; the bordering values are not used
    double zL, zR, g0, g1, g2;
    solve_helm<PMAX, NT, FULL, true, PWT>(K, w, z, zL, zR, cnt, L, par.slot, t, 0.0, 0.0, 0.0, g0,
                                          g1, g2, 0.0, 0.0);
    par.slot ^= 1;
    const double q = 0.25 * P.dt;
#pragma unroll
    for (int j = 0; j < PMAX; ++j) rhs[j] = fma(-q, z[j], lam_at(j));
  }
  iters += k > P.picard_max + 1 ? P.picard_max + 1 : k;
  // dJ/d(dU) = -(1/2) D(s)^T nu;  lambda_n = 2 M nu - lambda_{n+1}
  double nl, nr, mnu[PMAX];
  halo<PMAX, NT, FULL>(nu, cnt, L, t, nl, nr, par.hs);
  if constexpr (kL) {
    double sv[PMAX];
    s_at(sv);
    advect_t<PMAX, FULL>(sv, sl, sr, nu, nl, nr, cnt, -0.5, gdU);
  } else {
    advect_t<PMAX, FULL>(s, sl, sr, nu, nl, nr, cnt, -0.5, gdU);
  }
  mass_apply<PMAX, NT, FULL>(nu, mnu, P.h, cnt, L, t, 2.0, par.hs);
#pragma unroll
  for (int j = 0; j < PMAX; ++j) lam[j] = mnu[j] - lam_at(j);
  return status;
}

template <int PMAX, bool FULL>
__device__ __forceinline__ void store_state(double* base, int nx, const Chunk& ch,
                                            const double (&m)[PMAX], const double (&u)[PMAX]) {
  store_chunk<PMAX, FULL>(base, ch, m);
  store_chunk<PMAX, FULL>(base + nx, ch, u);
}

// MATERN: the controls dW, dLambda and the gradient are per cell,
// [n][ctrl_steps][nx]; each step's noise is the Matern-type field of the cells
// dW^n + dLambda^n, and the gradient with respect to the cells is the
// transpose of that map applied to dJ/d(dU^n), plus the Girsanov term.
template <int PMAX, int NT, bool FULL, bool MATERN = false>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) k_nudge_grad(const NudgeArgs A, const HelmConst K) {
  __shared__ RowLds<NT> L;
  __shared__ AuxLds<PMAX, NT> X;
  __shared__ double gpart[MATERN ? 1 : 64][MATERN ? 1 : NT / kWave];
  // the table form of the Helmholtz solves where registers are short (the
  // Matern-type noise, 16-node chunks)
  constexpr bool PWT = MATERN || PMAX >= 16;
  const int p = blockIdx.x, t = threadIdx.x;
  if (A.active && A.active[p] == 0) return;  // whole workgroup
  const int nx = A.P.nx, Q = A.P.n_modes, S = A.n_steps, CS = A.ctrl_steps;
  const int nq = MATERN ? nx : Q;  // controls per step
  const int CE = A.ckpt_every, nseg = (S + CE - 1) / CE;
  const Chunk ch = chunk_of<NT>(nx, t);
  const double* dW = A.dW ? A.dW + static_cast<size_t>(p) * CS * nq : nullptr;
  const double* dL = A.dLam ? A.dLam + static_cast<size_t>(p) * CS * nq : nullptr;
  auto incv = [&](int n, int q) -> double {
    if (n >= CS) return 0.0;
    double w = 0.0;
    if (dW) w = dW[n * nq + q];
    if (dL) w += dL[n * nq + q];
    return w;
  };
  Parity par;
  // the noise of step n added to e (uniform across the workgroup: steps past
  // the controlled ones carry none)
  auto step_noise = [&](int n) {
    if constexpr (MATERN) {
      return [&, n](int, double (&e)[PMAX]) {
        if (n >= CS || (!dW && !dL)) return;
        double w[PMAX];
#pragma unroll
        for (int j = 0; j < PMAX; ++j)
          w[j] = slot_live<PMAX, FULL>(j, ch.cnt) ? incv(n, ch.start + j) : 0.0;
        matern_add<PMAX, NT, FULL>(A.M, w, e, ch, L, t, par);
      };
    } else {
      auto inc1 = [&, n](int, int q) { return incv(n, q); };
      return modes_noise<PMAX, FULL>(A.P, ch, inc1);
    }
  };
  double* ck = A.ckpt + static_cast<size_t>(p) * nseg * 2 * nx;
  double* sg = A.seg + static_cast<size_t>(p) * (CE + 1) * 2 * nx;
  double m[PMAX], u[PMAX];
  load_chunk<PMAX, FULL>(A.m0 + static_cast<size_t>(p) * nx, ch, m);
  load_chunk<PMAX, FULL>(A.u0 + static_cast<size_t>(p) * nx, ch, u);
  int fit = 0, ait = 0, st = SCH_OK;

  // forward pass: checkpoints, and every state of the last segment
  for (int c = 0; c < nseg && st == SCH_OK; ++c) {
    const int n0 = c * CE, n1 = min(S, n0 + CE);
    const bool last = c == nseg - 1;
    store_state<PMAX, FULL>(ck + static_cast<size_t>(c) * 2 * nx, nx, ch, m, u);
    if (last) store_state<PMAX, FULL>(sg, nx, ch, m, u);
    for (int n = n0; n < n1 && st == SCH_OK; ++n) {
      st = run_window<PMAX, NT, FULL, true, PWT>(A.P, K, step_noise(n), 1, m, u, ch, L, X, t,
                                                    par, fit);
      if (last) store_state<PMAX, FULL>(sg + static_cast<size_t>(n - n0 + 1) * 2 * nx, nx, ch, m, u);
    }
  }
  double J = INFINITY;
  if (st == SCH_OK) {
    const double phi = block_nll<PMAX, NT, FULL>(u, ch, nx, A.n_obs, A.y, A.sigma, L, t, par.hs);
    double gs = 0.0;
    for (int i = t; i < CS * nq; i += NT) {
      const double l = dL ? dL[i] : 0.0, w = dW ? dW[i] : 0.0;
      gs += 0.5 * l * l + l * w;
    }
    J = phi + block_sum<NT>(gs, L, t) / A.P.dt;
    if (!isfinite(J)) {
      J = INFINITY;
      st = SCH_E_NONFINITE;
    }
  }
  if (st == SCH_OK) {
    // lambda_S = M H^{-1} P^T diag(sigma^-2) (P u^S - y)
    double lam[PMAX];
    {
      double w[PMAX], zL, zR, g0, g1, g2;
      obs_adjoint<PMAX, NT, FULL>(u, ch, nx, A.n_obs, A.y, A.sigma, w, L, t, par.hs);
      // M H^{-1} w as H^{-1} M w (the bordering values are not used)
      solve_helm<PMAX, NT, FULL, true, PWT>(K, w, lam, zL, zR, ch.cnt, L, par.slot, t, 0.0, 0.0,
                                               0.0, g0, g1, g2, 0.0, 0.0);
      par.slot ^= 1;
    }
    const int lane = t & (kWave - 1), wv = t / kWave;
    for (int c = nseg - 1; c >= 0 && st == SCH_OK; --c) {
      const int n0 = c * CE, n1 = min(S, n0 + CE);
      if (c != nseg - 1) {
        load_chunk<PMAX, FULL>(ck + static_cast<size_t>(c) * 2 * nx, ch, m);
        load_chunk<PMAX, FULL>(ck + static_cast<size_t>(c) * 2 * nx + nx, ch, u);
        store_state<PMAX, FULL>(sg, nx, ch, m, u);
        for (int n = n0; n < n1 && st == SCH_OK; ++n) {
          st = run_window<PMAX, NT, FULL, true, PWT>(A.P, K, step_noise(n), 1, m, u, ch, L, X,
                                                        t, par, fit);
          store_state<PMAX, FULL>(sg + static_cast<size_t>(n - n0 + 1) * 2 * nx, nx, ch, m, u);
        }
      }
      for (int n = n1 - 1; n >= n0 && st == SCH_OK; --n) {
        const double* sa = sg + static_cast<size_t>(n - n0) * 2 * nx;
        const double* sb = sa + 2 * nx;
        double gdU[PMAX];
        st = adjoint_step<PMAX, NT, FULL, PWT>(A.P, K, step_noise(n), sa, sa + nx, sb, sb + nx,
                                                  lam, gdU, ch, L, X, t, par, ait);
        if (n >= CS) continue;
        if constexpr (MATERN) {
          double gc[PMAX];
          matern_transpose<PMAX, NT, FULL>(A.M, gdU, gc, ch, L, t, par);
          double* gp = A.grad + (static_cast<size_t>(p) * CS + n) * nx + ch.start;
#pragma unroll
          for (int j = 0; j < PMAX; ++j)
            if (slot_live<PMAX, FULL>(j, ch.cnt)) gp[j] = gc[j] + incv(n, ch.start + j) / A.P.dt;
        } else {
          for (int q = 0; q < Q; ++q) {
            const double* xq = A.P.xi + static_cast<size_t>(q) * nx + ch.start;
            double a = 0.0;
#pragma unroll
            for (int j = 0; j < PMAX; ++j)
              if (slot_live<PMAX, FULL>(j, ch.cnt)) a = fma(xq[j], gdU[j], a);
            a = wave_sum(a);
            if (lane == 0) gpart[q][wv] = a;
          }
          __syncthreads();
          for (int q = t; q < Q; q += NT) {
            double a = 0.0;
#pragma unroll
            for (int i = 0; i < NT / kWave; ++i) a += gpart[q][i];
            A.grad[(static_cast<size_t>(p) * CS + n) * Q + q] = a + incv(n, q) / A.P.dt;
          }
          __syncthreads();
        }
      }
    }
  }
  if (t == 0) {
    A.J[p] = st == SCH_OK ? J : INFINITY;
    if (A.status) A.status[p] = st;
    if (A.iters_acc) {
      atomicAdd(A.iters_acc, static_cast<unsigned long long>(fit));
      atomicAdd(A.iters_acc + 1, static_cast<unsigned long long>(ait));
    }
  }
}

// ---------------------------------------------------------------------------
// Batched L-BFGS, one thread per particle (Q unknowns each).  The state
// machine advances after every evaluation of the objective at the trial
// points x_t (J -> ft, gradient -> gt, evaluation status -> est):
//   phase 0 (start point evaluated): take f, g; then pick a direction;
//   phase 1 (trial evaluated): accept on the Armijo test
//     ft <= f + c1 a g.p + 1e-13 |f| (finite ft, est == 0), store the pair,
//     then pick a direction; else halve a, or stop after max_back halvings.
// Picking a direction first tests |g|_inf <= gtol (1 + |f|) and the iteration
// cap, then runs the two-loop recursion with H0 = gamma I (gamma = s.y/y.y of
// the newest pair, h0 with no pair; a non-descent direction drops the memory
// and uses -h0 g) and sets the trial x + p.  Status: 0 converged, 1 iteration
// cap, 2 line search failed, 3 objective failed at the starting point.
// ---------------------------------------------------------------------------
constexpr int kLbfgsMaxMem = 16;

struct LbfgsState {
  double *x, *g, *p, *xt, *ft, *gt;  // [n][Q]; ft: [n]
  double *f, *gp, *a;                // [n]
  double *S, *Y, *rho;               // [n][mem][Q], [n][mem][Q], [n][mem]
  int *head, *count, *k, *nback, *phase, *lstat, *active, *est, *evals;  // [n]
  unsigned int* n_active;            // [1]
};

struct LbfgsParams {
  int n, Q, mem, max_iter, max_back;
  double gtol, h0;
};

__device__ void lbfgs_direction(const LbfgsState& s, const LbfgsParams& P, int i) {
  const int Q = P.Q, M = P.mem;
  double* x = s.x + static_cast<size_t>(i) * Q;
  double* g = s.g + static_cast<size_t>(i) * Q;
  double* p = s.p + static_cast<size_t>(i) * Q;
  double* xt = s.xt + static_cast<size_t>(i) * Q;
  double* Sm = s.S + static_cast<size_t>(i) * M * Q;
  double* Ym = s.Y + static_cast<size_t>(i) * M * Q;
  double* rho = s.rho + static_cast<size_t>(i) * M;
  const double f = s.f[i];
  double gmax = 0.0;
  for (int q = 0; q < Q; ++q) gmax = fmax(gmax, fabs(g[q]));
  if (gmax <= P.gtol * (1.0 + fabs(f))) {
    s.lstat[i] = 0;
    s.active[i] = 0;
    return;
  }
  if (s.k[i] >= P.max_iter) {
    s.lstat[i] = 1;
    s.active[i] = 0;
    return;
  }
  int head = s.head[i], count = s.count[i];
  double al[kLbfgsMaxMem];
  for (int q = 0; q < Q; ++q) p[q] = -g[q];
  for (int c = 0; c < count; ++c) {
    const int j = (head - 1 - c + M) % M;
    double d = 0.0;
    for (int q = 0; q < Q; ++q) d += Sm[j * Q + q] * p[q];
    al[j] = rho[j] * d;
    for (int q = 0; q < Q; ++q) p[q] -= al[j] * Ym[j * Q + q];
  }
  double gamma = P.h0;
  if (count > 0) {
    const int j = (head - 1 + M) % M;
    double sy = 0.0, yy = 0.0;
    for (int q = 0; q < Q; ++q) {
      sy += Sm[j * Q + q] * Ym[j * Q + q];
      yy += Ym[j * Q + q] * Ym[j * Q + q];
    }
    gamma = sy / yy;
  }
  for (int q = 0; q < Q; ++q) p[q] *= gamma;
  for (int c = count - 1; c >= 0; --c) {
    const int j = (head - 1 - c + M) % M;
    double d = 0.0;
    for (int q = 0; q < Q; ++q) d += Ym[j * Q + q] * p[q];
    const double b = rho[j] * d;
    for (int q = 0; q < Q; ++q) p[q] += (al[j] - b) * Sm[j * Q + q];
  }
  double gp = 0.0;
  for (int q = 0; q < Q; ++q) gp += g[q] * p[q];
  if (!(gp < 0.0)) {
    s.count[i] = 0;
    s.head[i] = 0;
    gp = 0.0;
    for (int q = 0; q < Q; ++q) {
      p[q] = -P.h0 * g[q];
      gp += g[q] * p[q];
    }
  }
  s.gp[i] = gp;
  s.a[i] = 1.0;
  s.nback[i] = 0;
  s.phase[i] = 1;
  for (int q = 0; q < Q; ++q) xt[q] = x[q] + p[q];
}

// Initial state: x = x0 (a [n][stride] array read at offset 0, or zero).
// Start of a stage's L-BFGS.  mode (null: every particle starts from x0, or
// from zero without x0) selects per particle: kNudgeKeep takes x0 as the
// stage's control without any step (the particle is inactive from the
// start), kNudgeFromGiven starts the iteration at x0, kNudgeFromZero at 0.
constexpr int kNudgeKeep = 0, kNudgeFromGiven = 1, kNudgeFromZero = 2;
__global__ void k_lbfgs_init(LbfgsState s, LbfgsParams P, const double* x0, int x0_stride,
                             const int* mode = nullptr) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P.n) return;
  int md = mode ? mode[i] : (x0 ? kNudgeFromGiven : kNudgeFromZero);
  if (md != kNudgeKeep && md != kNudgeFromGiven) md = kNudgeFromZero;
  const bool given = x0 && md != kNudgeFromZero;
  for (int q = 0; q < P.Q; ++q) {
    const double v = given ? x0[static_cast<size_t>(i) * x0_stride + q] : 0.0;
    s.x[static_cast<size_t>(i) * P.Q + q] = v;
    s.xt[static_cast<size_t>(i) * P.Q + q] = v;
  }
  s.head[i] = 0;
  s.count[i] = 0;
  s.k[i] = 0;
  s.nback[i] = 0;
  s.phase[i] = 0;
  s.lstat[i] = md == kNudgeKeep ? 0 : 1;
  s.active[i] = md == kNudgeKeep ? 0 : 1;
  s.evals[i] = 0;
}

__global__ void k_lbfgs_update(LbfgsState s, LbfgsParams P) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P.n || s.active[i] == 0) return;
  const int Q = P.Q, M = P.mem;
  s.evals[i] += 1;
  const double ft = s.ft[i];
  const bool ok = s.est[i] == SCH_OK && isfinite(ft);
  double* x = s.x + static_cast<size_t>(i) * Q;
  double* g = s.g + static_cast<size_t>(i) * Q;
  double* xt = s.xt + static_cast<size_t>(i) * Q;
  const double* gt = s.gt + static_cast<size_t>(i) * Q;
  if (s.phase[i] == 0) {
    if (!ok) {
      s.lstat[i] = 3;
      s.active[i] = 0;
    } else {
      s.f[i] = ft;
      for (int q = 0; q < Q; ++q) g[q] = gt[q];
      lbfgs_direction(s, P, i);
    }
  } else {
    const double f = s.f[i];
    if (ok && ft <= f + 1e-4 * s.a[i] * s.gp[i] + 1e-13 * fabs(f)) {
      const int head = s.head[i];
      double* Sm = s.S + (static_cast<size_t>(i) * M + head) * Q;
      double* Ym = s.Y + (static_cast<size_t>(i) * M + head) * Q;
      double sy = 0.0, ss = 0.0, yy = 0.0;
      for (int q = 0; q < Q; ++q) {
        const double si = xt[q] - x[q], yi = gt[q] - g[q];
        Sm[q] = si;
        Ym[q] = yi;
        sy += si * yi;
        ss += si * si;
        yy += yi * yi;
      }
      if (sy > 1e-10 * sqrt(ss) * sqrt(yy)) {
        s.rho[static_cast<size_t>(i) * M + head] = 1.0 / sy;
        s.head[i] = (head + 1) % M;
        if (s.count[i] < M) s.count[i] += 1;
      }
      for (int q = 0; q < Q; ++q) {
        x[q] = xt[q];
        g[q] = gt[q];
      }
      s.f[i] = ft;
      s.k[i] += 1;
      lbfgs_direction(s, P, i);
    } else if (s.nback[i] >= P.max_back) {
      s.lstat[i] = 2;
      s.active[i] = 0;
    } else {
      const double a = 0.5 * s.a[i];
      s.a[i] = a;
      s.nback[i] += 1;
      const double* p = s.p + static_cast<size_t>(i) * Q;
      for (int q = 0; q < Q; ++q) xt[q] = x[q] + a * p[q];
    }
  }
  if (s.active[i]) atomicAdd(s.n_active, 1u);
}

// The same state machine with one wavefront per particle, for many unknowns
// (one control per cell): each vector loop is strided over the 64 lanes, each
// inner product and the gradient's max norm are wavefront reductions (their
// values uniform across the wavefront), so every lane takes the same
// decisions; lane 0 writes the scalar state.  The steps and tests are those of
// lbfgs_direction / k_lbfgs_update; only the summation order differs.
// Returns whether the particle stays active.
__device__ bool lbfgs_direction_w(const LbfgsState& s, const LbfgsParams& P, int i, int l,
                                  int head, int count, int k, double f) {
  const int Q = P.Q, M = P.mem;
  double* x = s.x + static_cast<size_t>(i) * Q;
  double* g = s.g + static_cast<size_t>(i) * Q;
  double* p = s.p + static_cast<size_t>(i) * Q;
  double* xt = s.xt + static_cast<size_t>(i) * Q;
  const double* Sm = s.S + static_cast<size_t>(i) * M * Q;
  const double* Ym = s.Y + static_cast<size_t>(i) * M * Q;
  const double* rho = s.rho + static_cast<size_t>(i) * M;
  auto dot = [&](const double* a, const double* b) {
    double d = 0.0;
    for (int q = l; q < Q; q += kWave) d = fma(a[q], b[q], d);
    return wave_sum(d);
  };
  double gmax = 0.0;
  for (int q = l; q < Q; q += kWave) gmax = fmax(gmax, fabs(g[q]));
  gmax = wave_max(gmax);
  if (gmax <= P.gtol * (1.0 + fabs(f)) || k >= P.max_iter) {
    if (l == 0) {
      s.lstat[i] = k >= P.max_iter && !(gmax <= P.gtol * (1.0 + fabs(f))) ? 1 : 0;
      s.active[i] = 0;
    }
    return false;
  }
  double al[kLbfgsMaxMem];
  for (int q = l; q < Q; q += kWave) p[q] = -g[q];
  for (int c = 0; c < count; ++c) {
    const int j = (head - 1 - c + M) % M;
    al[j] = rho[j] * dot(Sm + j * Q, p);
    for (int q = l; q < Q; q += kWave) p[q] -= al[j] * Ym[j * Q + q];
  }
  double gamma = P.h0;
  if (count > 0) {
    const int j = (head - 1 + M) % M;
    gamma = dot(Sm + j * Q, Ym + j * Q) / dot(Ym + j * Q, Ym + j * Q);
  }
  for (int q = l; q < Q; q += kWave) p[q] *= gamma;
  for (int c = count - 1; c >= 0; --c) {
    const int j = (head - 1 - c + M) % M;
    const double b = rho[j] * dot(Ym + j * Q, p);
    for (int q = l; q < Q; q += kWave) p[q] += (al[j] - b) * Sm[j * Q + q];
  }
  double gp = dot(g, p);
  if (!(gp < 0.0)) {
    count = 0;
    head = 0;
    for (int q = l; q < Q; q += kWave) p[q] = -P.h0 * g[q];
    gp = dot(g, p);
  }
  if (l == 0) {
    s.head[i] = head;
    s.count[i] = count;
    s.gp[i] = gp;
    s.a[i] = 1.0;
    s.nback[i] = 0;
    s.phase[i] = 1;
  }
  for (int q = l; q < Q; q += kWave) xt[q] = x[q] + p[q];
  return true;
}

__global__ void __launch_bounds__(256) k_lbfgs_update_w(LbfgsState s, LbfgsParams P) {
  const int l = threadIdx.x & (kWave - 1);
  const int i = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (i >= P.n || s.active[i] == 0) return;  // the whole wavefront
  const int Q = P.Q, M = P.mem;
  if (l == 0) s.evals[i] += 1;
  const double ft = s.ft[i];
  const bool ok = s.est[i] == SCH_OK && isfinite(ft);
  double* x = s.x + static_cast<size_t>(i) * Q;
  double* g = s.g + static_cast<size_t>(i) * Q;
  double* xt = s.xt + static_cast<size_t>(i) * Q;
  const double* gt = s.gt + static_cast<size_t>(i) * Q;
  bool act = true;
  if (s.phase[i] == 0) {
    if (!ok) {
      if (l == 0) {
        s.lstat[i] = 3;
        s.active[i] = 0;
      }
      act = false;
    } else {
      if (l == 0) s.f[i] = ft;
      for (int q = l; q < Q; q += kWave) g[q] = gt[q];
      act = lbfgs_direction_w(s, P, i, l, s.head[i], s.count[i], s.k[i], ft);
    }
  } else {
    const double f = s.f[i];
    if (ok && ft <= f + 1e-4 * s.a[i] * s.gp[i] + 1e-13 * fabs(f)) {
      int head = s.head[i], count = s.count[i];
      const int k = s.k[i] + 1;
      double* Sm = s.S + (static_cast<size_t>(i) * M + head) * Q;
      double* Ym = s.Y + (static_cast<size_t>(i) * M + head) * Q;
      double sy = 0.0, ss = 0.0, yy = 0.0;
      for (int q = l; q < Q; q += kWave) {
        const double si = xt[q] - x[q], yi = gt[q] - g[q];
        Sm[q] = si;
        Ym[q] = yi;
        sy = fma(si, yi, sy);
        ss = fma(si, si, ss);
        yy = fma(yi, yi, yy);
      }
      sy = wave_sum(sy);
      ss = wave_sum(ss);
      yy = wave_sum(yy);
      if (sy > 1e-10 * sqrt(ss) * sqrt(yy)) {
        if (l == 0) s.rho[static_cast<size_t>(i) * M + head] = 1.0 / sy;
        head = (head + 1) % M;
        if (count < M) count += 1;
      }
      for (int q = l; q < Q; q += kWave) {
        x[q] = xt[q];
        g[q] = gt[q];
      }
      if (l == 0) {
        s.f[i] = ft;
        s.k[i] = k;
        s.head[i] = head;
        s.count[i] = count;
      }
      act = lbfgs_direction_w(s, P, i, l, head, count, k, ft);
    } else if (s.nback[i] >= P.max_back) {
      if (l == 0) {
        s.lstat[i] = 2;
        s.active[i] = 0;
      }
      act = false;
    } else {
      const double a = 0.5 * s.a[i];
      const double* p = s.p + static_cast<size_t>(i) * Q;
      for (int q = l; q < Q; q += kWave) xt[q] = x[q] + a * p[q];
      if (l == 0) {
        s.a[i] = a;
        s.nback[i] += 1;
      }
    }
  }
  if (act && l == 0) atomicAdd(s.n_active, 1u);
}

// End of a stage: record the control of step n, the increment of the step
// (dW^n + dLambda^n) for the advance, and the log Girsanov term.
__global__ void k_nudge_commit(LbfgsState s, LbfgsParams P, int n_steps, int step,
                               const double* dW, double* dLam, double* inc1, double* logG,
                               int* lbfgs_worst, int* iters, int* evals, double dt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P.n) return;
  const int Q = P.Q;
  double lg = 0.0;
  for (int q = 0; q < Q; ++q) {
    const size_t o = (static_cast<size_t>(i) * n_steps + step) * Q + q;
    const double x = s.x[static_cast<size_t>(i) * Q + q], w = dW[o];
    dLam[o] = x;
    inc1[static_cast<size_t>(i) * Q + q] = w + x;
    lg += 0.5 * x * x / dt + x * w / dt;
  }
  logG[i] -= lg;
  if (s.lstat[i] > lbfgs_worst[i]) lbfgs_worst[i] = s.lstat[i];
  iters[i] += s.k[i];
  evals[i] += s.evals[i];
}

__global__ void k_fill_i32(int* p, int v, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    p[i] = v;
}

// status[i] keeps its first failure; tmp[i] is the status of the latest step.
__global__ void k_status_merge(int* status, const int* tmp, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && status[i] == SCH_OK) status[i] = tmp[i];
}

// Potential of a nudged particle for the tempered weights W~ (section 3.1.3):
// J = phi - log G, +infinity where the nudged window failed or either term
// is not finite.
__global__ void k_nudged_potential(int n, const double* phi, const double* logG,
                                   const int* status, double* J) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = phi[i] - logG[i];
  J[i] = (status[i] == SCH_OK && fabs(v) <= 1.7976931348623157e308) ? v : INFINITY;
}

}  // namespace sch
