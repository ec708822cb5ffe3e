// model.hpp -- kernels of the SCH forward model on gfx950: one workgroup per
// particle, the particle's row of nx nodes split in register chunks over the
// workgroup's threads.  The varying implicit-midpoint systems are solved with
// cyclic_solve(), the constant Helmholtz system with the scan form of
// solve_helm().
#pragma once

#include "device.hpp"
#include "helm.hpp"

namespace sch {

// Per-call constants of the P1 / implicit-midpoint discretisation.
struct StepParams {
  int nx, n_modes, picard_max;
  double h, dt, tol;
  double a_off, a_diag;  // constant parts of the step matrix rows:
                         // h/6 - mu dt/(2h) and 2h/3 + mu dt/h
  const double* xi;      // [n_modes][nx]
};

inline StepParams make_params(const sch_model& md) {
  StepParams P;
  P.nx = md.nx;
  P.n_modes = md.n_modes;
  P.picard_max = md.picard_max;
  P.h = md.L / md.nx;
  P.dt = md.dt;
  P.tol = md.picard_tol;
  P.a_off = P.h / 6.0 - md.mu * md.dt / (2.0 * P.h);
  P.a_diag = 2.0 * P.h / 3.0 + md.mu * md.dt / P.h;
  P.xi = md.xi;
  return P;
}

// Mass-matrix product scale * (M v)_j = scale * (h/6 v_{j-1} + 2h/3 v_j + h/6 v_{j+1})
// with the chunk's halo values hl, hr given.
template <int PMAX, bool FULL>
__device__ __forceinline__ void mass_apply_h(const double (&v)[PMAX], double (&out)[PMAX],
                                             double h, int cnt, double hl, double hr,
                                             double scale) {
  const double c1 = scale * h / 6.0, c0 = scale * 2.0 * h / 3.0;
#pragma unroll
  for (int j = 0; j < PMAX; ++j)
    out[j] = fma(c1, left_of<PMAX, FULL>(v, j, hl) + right_of<PMAX, FULL>(v, j, cnt, hr), c0 * v[j]);
}

// The same with the halo exchanged through LDS.
template <int PMAX, int NT, bool FULL>
__device__ __forceinline__ void mass_apply(const double (&v)[PMAX], double (&out)[PMAX], double h,
                                           int cnt, RowLds<NT>& L, int t, double scale, int& hs) {
  double hl, hr;
  halo<PMAX, NT, FULL>(v, cnt, L, t, hl, hr, hs);
  mass_apply_h<PMAX, FULL>(v, out, h, cnt, hl, hr, scale);
}

// Per-thread solver state carried through a kernel: the halo and record
// buffer parities.
struct Parity {
  int hs = 0, slot = 0;
};

// Two per-node arrays of the window (the explicit part of dv and the previous
// Picard iterate) live in LDS as [slot][thread] when they fit next to the
// solver's LDS (128 KiB for both: a workgroup may hold up to 160 KiB); when
// only one fits, the explicit part goes to LDS and the iterate stays in
// registers; otherwise both do.
template <int PMAX, int NT>
struct AuxLds {
  static constexpr size_t kBytes = static_cast<size_t>(PMAX) * NT * sizeof(double);
  static constexpr bool kInLds = 2 * kBytes <= 131072;  // both arrays
  static constexpr bool kDInLds = kBytes <= 65536;     // the explicit part
  double a[kInLds ? 2 : 1][kDInLds ? PMAX : 1][kDInLds ? NT : 1];
};

// The noise of the modes form: noise(n, e) adds sum_q xi_q inc(n, q) to the
// chunk e, inc(n, q) being the increment dW^n_q (+ dLambda^n_q) of step n,
// mode q.
template <int PMAX, bool FULL, class IncF>
__device__ __forceinline__ auto modes_noise(const StepParams& P, const Chunk& ch, IncF inc) {
  return [&P, ch, inc](int n, double (&e)[PMAX]) {
    for (int q = 0; q < P.n_modes; ++q) {
      const double w = inc(n, q);
      const double* xq = P.xi + static_cast<size_t>(q) * P.nx + ch.start;
#pragma unroll
      for (int j = 0; j < PMAX; ++j)
        if (slot_live<PMAX, FULL>(j, ch.cnt)) e[j] = fma(xq[j], w, e[j]);
    }
  };
}

// Constants of the Matern-type noise (section 2, eq. noise_solve2): the
// operator M + kappa^{-2} K in scan form, the load factor eta sqrt(h) / 2 of
// the cell increments, and the number k of solves.
struct MaternDev {
  HelmConst K;
  double load, h;
  int k;
};

// Adds the Matern-type noise field of one step to e.  w holds the chunk's
// cell increments Delta W_i (cell i = [x_i, x_{i+1}], held by the thread that
// holds node i).  The load vector of Delta W_h is
// b_i = eta sqrt(h) (Delta W_{i-1} + Delta W_i) / 2; then
// (M + kappa^{-2} K) U_1 = b and (M + kappa^{-2} K) U_j = M U_{j-1}, each
// solve in the scan form of solve_helm, the mass products with the bordering
// values of the previous solve as halo (chunks of >= 2 rows) or an exchange.
template <int PMAX, int NT, bool FULL>
__device__ __forceinline__ void matern_add(const MaternDev& M, const double (&w)[PMAX],
                                           double (&e)[PMAX], const Chunk& ch, RowLds<NT>& L,
                                           int t, Parity& par) {
  const int cnt = ch.cnt;
  const bool bordered = FULL || M.K.base >= 2;
  double wl, wr;
  halo<PMAX, NT, FULL>(w, cnt, L, t, wl, wr, par.hs);
  double r[PMAX], U[PMAX];
#pragma unroll
  for (int j = 0; j < PMAX; ++j) r[j] = M.load * (left_of<PMAX, FULL>(w, j, wl) + w[j]);
  double uL = 0.0, uR = 0.0, g0, g1, g2;
  for (int i = 0; i < M.k; ++i) {
    if (i > 0) {
      double hl = uL, hr = uR;
      if (!bordered) halo<PMAX, NT, FULL>(U, cnt, L, t, hl, hr, par.hs);
      mass_apply_h<PMAX, FULL>(U, r, M.h, cnt, hl, hr, 1.0);
    }
    solve_helm<PMAX, NT, FULL, false, true>(M.K, r, U, uL, uR, cnt, L, par.slot, t, 0.0, 0.0, 0.0,
                                            g0, g1, g2);
    par.slot ^= 1;
  }
#pragma unroll
  for (int j = 0; j < PMAX; ++j)
    if (slot_live<PMAX, FULL>(j, cnt)) e[j] += U[j];
}

// The transpose of the map of matern_add (cells Delta W -> field U_k): with
// A = M + kappa^{-2} K and B the load map, T = (A^{-1} M)^{k-1} A^{-1} B, so
// T^T g = B^T (A^{-1} M)^{k-1} A^{-1} g (A and M symmetric): z = A^{-1} g, then
// z = A^{-1} M z k - 1 times, and out_i = load (z_i + z_{i+1}) (cell i feeds the
// load of nodes i and i + 1).
template <int PMAX, int NT, bool FULL>
__device__ __forceinline__ void matern_transpose(const MaternDev& M, const double (&g)[PMAX],
                                                 double (&out)[PMAX], const Chunk& ch,
                                                 RowLds<NT>& L, int t, Parity& par) {
  const int cnt = ch.cnt;
  const bool bordered = FULL || M.K.base >= 2;
  double r[PMAX], z[PMAX];
#pragma unroll
  for (int j = 0; j < PMAX; ++j) r[j] = g[j];
  double zL = 0.0, zR = 0.0, g0, g1, g2;
  for (int i = 0; i < M.k; ++i) {
    if (i > 0) {
      double hl = zL, hr = zR;
      if (!bordered) halo<PMAX, NT, FULL>(z, cnt, L, t, hl, hr, par.hs);
      mass_apply_h<PMAX, FULL>(z, r, M.h, cnt, hl, hr, 1.0);
    }
    solve_helm<PMAX, NT, FULL, false, true>(M.K, r, z, zL, zR, cnt, L, par.slot, t, 0.0, 0.0, 0.0,
                                            g0, g1, g2);
    par.slot ^= 1;
  }
  double hl = zL, hr = zR;
  if (!bordered) halo<PMAX, NT, FULL>(z, cnt, L, t, hl, hr, par.hs);
#pragma unroll
  for (int j = 0; j < PMAX; ++j) out[j] = M.load * (z[j] + right_of<PMAX, FULL>(z, j, cnt, hr));
}

// One assimilation window of n_steps implicit-midpoint steps (eq. fde1) for
// the particle whose chunk is held in m, u.  noise(n, e) adds the step's
// noise increment dU^n to the chunk e (modes_noise, or the Matern-type field).
//
// Each step solves  A(dv) s = 2 M m^n  for s = m^n + m^{n+1}, with
//   A(dv) = M + (mu dt/2) K + (1/2) C(dv),  dv = dt (u^n + u*)/2 + dU^n,
// by Picard iteration on u* (u* = u^n initially, then u* = H^{-1} M m*), until
// the estimated max-norm error of m* (from its change and the observed
// contraction ratio) is at most tol * max|m*|.  Rows of A at node i:
//   a_i = h/6 - mu dt/(2h) - dv_{i-1}/4
//   b_i = 2h/3 + mu dt/h + (dv_{i+1} - dv_{i-1})/4
//   c_i = h/6 - mu dt/(2h) + dv_{i+1}/4
// (the exact P1 integrals of the advective terms of eq. fde1).  The right-
// hand side 2 M m^n is formed row by row inside the solve.  The convergence
// test's workgroup reduction rides on the Helmholtz solve's barrier.  The
// halo of m^n, of the explicit part of dv and of u^n is exchanged once per
// step; inside the iteration the halo of u* comes from the Helmholtz rows at
// the chunk's ends (chunks of at least two rows), so an iteration has two
// barriers: the interface solve and the Helmholtz solve.
// Returns SCH_OK or the status of the first failing step; on non-convergence
// the last iterate is kept, on a non-finite iterate or a system whose
// elimination growth exceeds kMaxGrowth (SCH_E_UNSTABLE) the step's input is
// kept (KEEP) or the state is left undefined (!KEEP, for callers that discard
// a failed window: u^n then need not stay live through the iteration).  PWT
// selects the table form of the Helmholtz solve (solve_helm), which the
// kernels with the Matern-type noise take.
template <int PMAX, int NT, bool FULL, bool KEEP = true, bool PWT = false, class NoiseF>
__device__ int run_window(const StepParams& P, const HelmConst& K, NoiseF noise, int n_steps,
                          double (&m)[PMAX], double (&u)[PMAX], const Chunk& ch, RowLds<NT>& L,
                          AuxLds<PMAX, NT>& X, int t, Parity& par, int& iters) {
  constexpr bool kLds = AuxLds<PMAX, NT>::kInLds, kDLds = AuxLds<PMAX, NT>::kDInLds;
  const int cnt = ch.cnt;
  const double hdt = 0.5 * P.dt;
  // dv is carried as dv/4, the form in which it enters the rows of A (exact:
  // a power-of-two scaling); the products then take no literal operands
  const double hdt4 = 0.25 * hdt;
  const double f1 = P.h / 3.0, f0 = 4.0 * P.h / 3.0;  // 2 M: (h/3, 4h/3, h/3)
  const bool bordered = FULL || K.base >= 2;
  double rD[kDLds ? 1 : PMAX], rP[kLds ? 1 : PMAX];
  // The thread's column of the LDS arrays.  It is laundered once per Picard
  // iteration, so the loads of the step's invariants are redone inside the
  // iteration (not hoisted into registers) and still issue back to back.
  int tx = t;
  auto getD = [&](int j) -> double { if constexpr (kDLds) return X.a[0][j][tx]; else return rD[j]; };
  auto setD = [&](int j, double v) { if constexpr (kDLds) X.a[0][j][tx] = v; else rD[j] = v; };
  auto getP = [&](int j) -> double { if constexpr (kLds) return X.a[1][j][tx]; else return rP[j]; };
  auto setP = [&](int j, double v) { if constexpr (kLds) X.a[1][j][tx] = v; else rP[j] = v; };
  for (int n = 0; n < n_steps; ++n) {
    // (dU^n + dt/2 u^n) / 4 + o, the explicit part of dv / 4 + o
    double eL, eR, mL, mR, uL, uR;
    {
      double e[PMAX];
#pragma unroll
      for (int j = 0; j < PMAX; ++j) e[j] = hdt * u[j];
      noise(n, e);
      // stored with the constant off-diagonal of the step rows added:
      // w = dv/4 + o (o = h/6 - mu dt/(2h)) is then the row's upper entry
#pragma unroll
      for (int j = 0; j < PMAX; ++j) e[j] = fma(e[j], 0.25, P.a_off);
      const double fst[3] = {m[0], e[0], u[0]};
      const double lst[3] = {last_of<PMAX, FULL>(m, cnt), last_of<PMAX, FULL>(e, cnt),
                             last_of<PMAX, FULL>(u, cnt)};
      double fl[3], fr[3];
      exchange<NT, 3>(fst, lst, fl, fr, L, t, par.hs);
      mL = fl[0];
      mR = fr[0];
      eL = fl[1];
      eR = fr[1];
      uL = fl[2];
      uR = fr[2];
#pragma unroll
      for (int j = 0; j < PMAX; ++j) {
        setD(j, e[j]);
        setP(j, m[j]);
      }
    }
    auto fget = [&](int j) -> double {
      return fma(f1, left_of<PMAX, FULL>(m, j, mL) + right_of<PMAX, FULL>(m, j, cnt, mR),
                 f0 * m[j]);
    };

    double us[PMAX];
#pragma unroll
    for (int j = 0; j < PMAX; ++j) us[j] = u[j];
    int status = SCH_E_NONCONVERGED, k = 1;
    double gprev = 0.0;  // the previous iteration's change of m*
    double lim = 0.0;    // tolerance times the first iterate's max |m*|
    double grow = 0.0;   // elimination growth of the step's solves (cyclic_solve)
    for (; k <= P.picard_max; ++k) {
      // Keep the step's invariants (the right-hand side 2 M m^n and the
      // LDS-resident explicit part) out of registers across iterations:
      // hoisting them would cost 64 registers per thread and halve the
      // workgroups a compute unit holds.
#pragma unroll
      for (int j = 0; j < PMAX; ++j) asm volatile("" : "+v"(m[j]));
      asm volatile("" : "+v"(tx));
      double dv[PMAX];
#pragma unroll
      for (int j = 0; j < PMAX; ++j) dv[j] = fma(hdt4, us[j], getD(j));  // dv / 4 + o
      double vl, vr;
      if (bordered) {
        vl = fma(hdt4, uL, eL);
        vr = fma(hdt4, uR, eR);
      } else {
        halo<PMAX, NT, FULL>(dv, cnt, L, t, vl, vr, par.hs);
      }
      // rows (o - v_-, d + v_+ - v_-, o + v_+) from w = v + o:
      // (2o - w_-, d + (w_+ - w_-), w_+)
      const double ao2 = 2.0 * P.a_off, ad = P.a_diag;
      auto rowA = [&](int j, double& a, double& b, double& c) {
        const double vm = left_of<PMAX, FULL>(dv, j, vl);
        const double vp = right_of<PMAX, FULL>(dv, j, cnt, vr);
        a = ao2 - vm;
        b = ad + (vp - vm);
        c = vp;
      };
      double ms[PMAX];
      double sl, sr;  // halo of s = m^n + m*
      cyclic_solve<PMAX, NT, FULL>(rowA, fget, ms, cnt, L, t, sl, sr, grow);
      // max change of m*, and on the first iteration its max size, the scale
      // of the tolerance (later iterates differ from the first by its first
      // correction, about 1e-4 of it at the workloads' steps); a non-finite
      // entry (which fmax would drop) reaches the Helmholtz solve, and
      // solve_helm then reports the change as +infinity, which marks the
      // iterate as failed
      double diff = 0.0, scale = 0.0;
      if (k == 1) {
#pragma unroll
        for (int j = 0; j < PMAX; ++j) {
          ms[j] -= m[j];
          if (slot_live<PMAX, FULL>(j, cnt)) {
            diff = fmax(diff, fabs(ms[j] - getP(j)));
            scale = fmax(scale, fabs(ms[j]));
          }
          setP(j, ms[j]);
        }
        scale = wave_max(scale);
      } else {
#pragma unroll
        for (int j = 0; j < PMAX; ++j) {
          ms[j] -= m[j];
          if (slot_live<PMAX, FULL>(j, cnt)) diff = fmax(diff, fabs(ms[j] - getP(j)));
          setP(j, ms[j]);
        }
      }
      // an upper bound within 2^-20 (a few units of the tolerance's last
      // digit): the test below can only stop later, never earlier
      diff = wave_max_bound(diff);
      // u* = H^{-1} M m* (the mass product folded into the scan form)
      // the growth test rides on the Helmholtz record as a wave-uniform flag
      const double wbad = __any(!(grow <= kMaxGrowth)) ? 1.0 : 0.0;
      double gdiff, gscale, gbad;
      solve_helm<PMAX, NT, FULL, true, PWT>(K, ms, us, uL, uR, cnt, L, par.slot, t, diff, scale,
                                            wbad, gdiff, gscale, gbad, sl - mL, sr - mR);
      par.slot ^= 1;
      if (gbad > 0.0) {
        status = SCH_E_UNSTABLE;
        break;
      }
      if (!(gdiff < INFINITY)) {
        status = SCH_E_NONFINITE;
        break;
      }
      if (k == 1) lim = P.tol * gscale;
      // stop once the iterate's error is within tolerance: for a contraction
      // with ratio c, |m* - m_k| <= c / (1 - c) |m_k - m_{k-1}|; c is the ratio
      // of the last two changes, the bound is used while c < 1/2 (multiplied
      // out: d_k^2 <= lim (d_{k-1} - d_k)), the change itself otherwise
      const bool done = (k > 1 && 2.0 * gdiff < gprev) ? gdiff * gdiff <= lim * (gprev - gdiff)
                                                       : gdiff <= lim;
      gprev = gdiff;
      if (done) {
        status = SCH_OK;
        break;
      }
    }
    iters += k > P.picard_max ? P.picard_max : k;
    if (KEEP && (status == SCH_E_NONFINITE || status == SCH_E_UNSTABLE)) return status;
    // the accepted iterate m* was stored as the last "previous iterate"
#pragma unroll
    for (int j = 0; j < PMAX; ++j) {
      m[j] = getP(j);
      u[j] = us[j];
    }
    if (status != SCH_OK) return status;
  }
  return SCH_OK;
}

// Negative log-likelihood of the particle's velocity chunk (eq. loglikeq):
// each thread takes the observation points that fall in its own cells.
// Point o lies in cell e = floor(o nx / n_obs) at fraction
// r = (o nx - e n_obs) / n_obs; the thread finds its first point with one
// integer division and walks on with integer multiplications only.
// `extra` is a per-thread addend summed into the result (0 for the plain
// likelihood).
template <int PMAX, int NT, bool FULL>
__device__ double block_nll(const double (&u)[PMAX], const Chunk& ch, int nx, int n_obs,
                            const double* y, const double* sigma, RowLds<NT>& L, int t, int& hs,
                            double extra = 0.0) {
  double hl, hr;
  halo<PMAX, NT, FULL>(u, ch.cnt, L, t, hl, hr, hs);
  double acc = 2.0 * extra;
  int64_t o = (static_cast<int64_t>(ch.start) * n_obs + nx - 1) / nx;
  const double dn = static_cast<double>(n_obs);
#pragma unroll
  for (int j = 0; j < PMAX; ++j) {
    if (!FULL && j >= ch.cnt) continue;
    const int64_t node = ch.start + j;
    const int64_t lim = (node + 1) * n_obs, base = node * n_obs;
    const double ur = right_of<PMAX, FULL>(u, j, ch.cnt, hr);
#pragma unroll 1
    for (; o * nx < lim; ++o) {
      const double r = static_cast<double>(o * nx - base) / dn;
      const double pu = (1.0 - r) * u[j] + r * ur;
      const double e = (pu - y[o]) / sigma[o];
      acc += e * e;
    }
  }
  return 0.5 * block_sum<NT>(acc, L, t);
}

// Node e of a row staged in the auxiliary LDS array `slot` as [slot][j][t]
// (the chunk layout of chunk_of: the first nx % NT threads hold one node more).
template <int PMAX, int NT>
__device__ __forceinline__ double staged_at(const AuxLds<PMAX, NT>& X, int slot, int nx, int e) {
  const int base = nx / NT, rem = nx % NT, split = rem * (base + 1);
  if (e < split) return X.a[slot][e % (base + 1)][e / (base + 1)];
  const int f = e - split;
  return X.a[slot][f % base][rem + f / base];
}

// The likelihood of block_nll with the velocity staged in auxiliary LDS
// slot 0: one thread per observation point.
template <int PMAX, int NT>
__device__ double staged_nll(const AuxLds<PMAX, NT>& X, int nx, int n_obs, const double* y,
                             const double* sigma, RowLds<NT>& L, int t, double extra = 0.0) {
  const double dn = static_cast<double>(n_obs);
  double acc = 2.0 * extra;
  for (int o = t; o < n_obs; o += NT) {
    const int64_t num = static_cast<int64_t>(o) * nx;
    const int e = static_cast<int>(num / n_obs);
    const double r = static_cast<double>(num - static_cast<int64_t>(e) * n_obs) / dn;
    const double pu = (1.0 - r) * staged_at(X, 0, nx, e) + r * staged_at(X, 0, nx, e + 1 == nx ? 0 : e + 1);
    const double d = (pu - y[o]) / sigma[o];
    acc += d * d;
  }
  return 0.5 * block_sum<NT>(acc, L, t);
}

template <int PMAX, bool FULL>
__device__ __forceinline__ void load_chunk(const double* g, const Chunk& ch, double (&v)[PMAX]) {
#pragma unroll
  for (int j = 0; j < PMAX; ++j) v[j] = slot_live<PMAX, FULL>(j, ch.cnt) ? g[ch.start + j] : 0.0;
}
template <int PMAX, bool FULL>
__device__ __forceinline__ void store_chunk(double* g, const Chunk& ch, const double (&v)[PMAX]) {
#pragma unroll
  for (int j = 0; j < PMAX; ++j)
    if (slot_live<PMAX, FULL>(j, ch.cnt)) g[ch.start + j] = v[j];
}

// ---------------------------------------------------------------------------
// Kernels.
// ---------------------------------------------------------------------------
struct WindowArgs {
  StepParams P;
  int n_steps;
  double* m;
  double* u;
  const double* dW;    // modes: [n][n_steps][n_modes]; Matern: cells [n][n_steps][nx]
  const double* dLam;
  int* status;
  int* iters;
  unsigned long long* iters_acc;  // optional device accumulator
  MaternDev M;                    // Matern-type noise (MATERN kernels)
};

template <int PMAX, int NT, bool FULL, bool MATERN = false>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) k_window(const WindowArgs A, const HelmConst K) {
  __shared__ RowLds<NT> L;
  __shared__ AuxLds<PMAX, NT> X;
  const int p = blockIdx.x, t = threadIdx.x;
  const Chunk ch = chunk_of<NT>(A.P.nx, t);
  double* mp = A.m + static_cast<size_t>(p) * A.P.nx;
  double* up = A.u + static_cast<size_t>(p) * A.P.nx;
  double m[PMAX], u[PMAX];
  load_chunk<PMAX, FULL>(mp, ch, m);
  load_chunk<PMAX, FULL>(up, ch, u);
  int iters = 0, st;
  Parity par;
  if constexpr (MATERN) {
    const int nx = A.P.nx;
    const double* cells = A.dW + static_cast<size_t>(p) * A.n_steps * nx;
    auto noise = [&](int n, double (&e)[PMAX]) {
      double w[PMAX];
      load_chunk<PMAX, FULL>(cells + static_cast<size_t>(n) * nx, ch, w);
      matern_add<PMAX, NT, FULL>(A.M, w, e, ch, L, t, par);
    };
    st = run_window<PMAX, NT, FULL, true, true>(A.P, K, noise, A.n_steps, m, u, ch, L, X, t, par,
                                                iters);
  } else {
    const int Q = A.P.n_modes;
    const double* dW = A.dW + static_cast<size_t>(p) * A.n_steps * Q;
    const double* dL = A.dLam ? A.dLam + static_cast<size_t>(p) * A.n_steps * Q : nullptr;
    auto inc = [&](int n, int q) {
      double w = dW[n * Q + q];
      if (dL) w += dL[n * Q + q];
      return w;
    };
    st = run_window<PMAX, NT, FULL>(A.P, K, modes_noise<PMAX, FULL>(A.P, ch, inc), A.n_steps, m,
                                    u, ch, L, X, t, par, iters);
  }
  store_chunk<PMAX, FULL>(mp, ch, m);
  store_chunk<PMAX, FULL>(up, ch, u);
  if (t == 0) {
    if (A.status) A.status[p] = st;
    if (A.iters) A.iters[p] = iters;
    if (A.iters_acc) atomicAdd(A.iters_acc, static_cast<unsigned long long>(iters));
  }
}

// v < exp(logr), kept out of line: inlined, the exponential's polynomial
// constants are hoisted to the kernel's start and held (spilled) across the
// window's solver loop.
__device__ __noinline__ bool metropolis_below(double v, double logr) { return v < exp(logr); }

struct JitterArgs {
  StepParams P;
  int n_steps;
  const double* m0;
  const double* u0;
  double* dW;
  double* phi;
  double* m_end;
  double* u_end;
  const double* theta;
  double rho;
  int n_jitter;
  int* n_accept;
  unsigned long long* accept_acc;
  unsigned long long* iters_acc;
  int n_obs;
  const double* y;
  const double* sigma;
  const double* zeta;  // [n_jitter][n][n_steps][n_modes]: sqrt(dt) z of the proposals
  const double* vacc;  // [n_jitter][n]: acceptance uniforms
  const double* dLam;  // [n][n_steps][n_modes] (Matern: [n][n_steps][nx]) fixed controls, or null
  // Matern-type noise (MATERN kernels): the increments are the cells
  // dW [n][n_steps][nx]; proposals and uniforms are drawn in the kernel, the
  // proposal rows go to stage [n][n_steps][nx]
  MaternDev M;
  double* stage;
  uint64_t seed;
  uint32_t cycle, temper_k;
};

// Standard normals of the chunk's cells from one Philox stream: cell i takes
// component i & 1 of the block at counter (c0, c1, (i >> 1) | tag, c3), so
// cells 2k and 2k + 1 share a block; a chunk that starts at an odd cell takes
// the second normal of its first block.  Slots past the chunk get 0.
template <int PMAX, bool FULL>
__device__ __forceinline__ void cell_normals(uint64_t seed, uint32_t c0, uint32_t c1,
                                             uint32_t tag, uint32_t c3, const Chunk& ch,
                                             double (&z)[PMAX]) {
  // the thread's first cell, laundered per call: otherwise the generator's
  // per-thread first-round products, the same for every step, are hoisted
  // out of the callers' step loops and held (in spill slots) across them
  int s0 = ch.start;
  asm volatile("" : "+v"(s0));
  if (!FULL && (s0 & 1)) {
    double za, zb;
    normal2(seed, c0, c1, static_cast<uint32_t>(s0 >> 1) | tag, c3, za, zb);
    z[0] = zb;
#pragma unroll
    for (int j = 1; j < PMAX; j += 2) {
      za = zb = 0.0;
      if (j < ch.cnt) normal2(seed, c0, c1, static_cast<uint32_t>((s0 + j) >> 1) | tag, c3, za, zb);
      z[j] = za;
      if (j + 1 < PMAX) z[j + 1] = j + 1 < ch.cnt ? zb : 0.0;
    }
  } else {
#pragma unroll
    for (int j = 0; j < PMAX; j += 2) {
      double za = 0.0, zb = 0.0;
      if (slot_live<PMAX, FULL>(j, ch.cnt))
        normal2(seed, c0, c1, static_cast<uint32_t>((s0 + j) >> 1) | tag, c3, za, zb);
      z[j] = za;
      z[j + 1] = slot_live<PMAX, FULL>(j + 1, ch.cnt) ? zb : 0.0;
    }
  }
}

// pCN proposal for the chunk's cells of one step (section 3.1.2):
// w_i = rho c_i + sqrt(1 - rho^2) sqrt(dt) z_i, the normals of tag PCN.
template <int PMAX, bool FULL>
__device__ __forceinline__ void pcn_cells(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c3,
                                          const Chunk& ch, double rho, double srho, double sdt,
                                          const double* cur, double (&w)[PMAX]) {
  double z[PMAX];
  cell_normals<PMAX, FULL>(seed, c0, c1, SCH_TAG_PCN << 24, c3, ch, z);
#pragma unroll
  for (int j = 0; j < PMAX; ++j)
    w[j] = slot_live<PMAX, FULL>(j, ch.cnt) ? rho * cur[j] + srho * (sdt * z[j]) : 0.0;
}

// n_jitter pCN moves of one particle's increments (section 3.1.2): proposal,
// window rerun from the window-start state (re-read from global memory for
// every proposal), likelihood and Metropolis accept in one launch.  With
// controls (the nudged filter, section 3.1.3) the window runs with the
// proposal plus the fixed control and the potential is the likelihood plus
// the Girsanov term sum (dLam^2 / 2 + dLam dW') / dt of the proposal.
// MATERN: the increments are the DG0 cell values of the Matern-type noise;
// each thread proposes its own cells step by step inside the window and
// writes them to the stage row, and an acceptance swaps the roles of the
// particle's stage and increment rows (one copy back at the end if needed);
// the per-cell controls are read only in the MCTRL variant, so that the
// variant without them keeps its registers.
template <int PMAX, int NT, bool FULL, bool MATERN = false, bool MCTRL = false>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) k_jitter(const JitterArgs A, const HelmConst K) {
  __shared__ RowLds<NT> L;
  __shared__ AuxLds<PMAX, NT> X;
  extern __shared__ double dyn[];  // modes: [2][n_steps][n_modes]: current increments, proposal
  const int p = blockIdx.x, t = threadIdx.x;
  const int nx = A.P.nx, Q = A.P.n_modes, S = A.n_steps;
  const Chunk ch = chunk_of<NT>(nx, t);
  double* cur;
  double* prop;
  double* dWp;
  if constexpr (MATERN) {
    dWp = A.dW + static_cast<size_t>(p) * S * nx;
    cur = dWp;
    prop = A.stage + static_cast<size_t>(p) * S * nx;
  } else {
    cur = dyn;
    prop = dyn + S * Q;
    dWp = A.dW + static_cast<size_t>(p) * S * Q;
    for (int i = t; i < S * Q; i += NT) cur[i] = dWp[i];
  }
  double phi = A.phi[p];
  const double theta = *A.theta;
  const double srho = sqrt(1.0 - A.rho * A.rho);
  int acc = 0, iters = 0;
  Parity par;
  __syncthreads();
  for (int j = 0; j < A.n_jitter; ++j) {
    const uint32_t w3 = (A.temper_k << 16) | static_cast<uint32_t>(j);
    if constexpr (!MATERN) {
      const double* zj = A.zeta + (static_cast<size_t>(j) * gridDim.x + p) * S * Q;
      for (int i = t; i < S * Q; i += NT) prop[i] = A.rho * cur[i] + srho * zj[i];
      __syncthreads();
    }
    double m[PMAX], u[PMAX];
    load_chunk<PMAX, FULL>(A.m0 + static_cast<size_t>(p) * nx, ch, m);
    load_chunk<PMAX, FULL>(A.u0 + static_cast<size_t>(p) * nx, ch, u);
    const double* lam = (MATERN && !MCTRL) || !A.dLam
                            ? nullptr
                            : A.dLam + static_cast<size_t>(p) * S * (MATERN ? nx : Q);
    int st;
    if constexpr (MATERN) {
      const double sdt = sqrt(A.P.dt);
      const uint32_t step0 = A.cycle * static_cast<uint32_t>(S);
      auto noise = [&](int n, double (&e)[PMAX]) {
        const size_t off = static_cast<size_t>(n) * nx + ch.start;
        double w[PMAX];
        pcn_cells<PMAX, FULL>(A.seed, static_cast<uint32_t>(p), step0 + static_cast<uint32_t>(n),
                              w3, ch, A.rho, srho, sdt, cur + off, w);
#pragma unroll
        for (int jj = 0; jj < PMAX; ++jj)
          if (slot_live<PMAX, FULL>(jj, ch.cnt)) {
            prop[off + jj] = w[jj];
            if (lam) w[jj] += lam[off + jj];  // the window sees dW' + dLambda
          }
        matern_add<PMAX, NT, FULL>(A.M, w, e, ch, L, t, par);
      };
      st = run_window<PMAX, NT, FULL, false, true>(A.P, K, noise, S, m, u, ch, L, X, t, par, iters);
    } else {
      auto inc = [&](int n, int q) {
        double w = prop[n * Q + q];
        if (lam) w += lam[n * Q + q];
        return w;
      };
      st = run_window<PMAX, NT, FULL, false>(A.P, K, modes_noise<PMAX, FULL>(A.P, ch, inc), S, m,
                                             u, ch, L, X, t, par, iters);
    }
    double girs = 0.0;  // this thread's share of the Girsanov term (after the window: not
                        // live across the solver loop)
    if (lam) {
      const double idt = 1.0 / A.P.dt;
      if constexpr (MATERN) {
        // over the thread's own cells, which it wrote to the stage row itself
        for (int n = 0; n < S; ++n) {
          const size_t off = static_cast<size_t>(n) * nx + ch.start;
          for (int jj = 0; jj < ch.cnt; ++jj)
            girs += (0.5 * lam[off + jj] * lam[off + jj] + lam[off + jj] * prop[off + jj]) * idt;
        }
      } else {
        for (int i = t; i < S * Q; i += NT)
          girs += (0.5 * lam[i] * lam[i] + lam[i] * prop[i]) * idt;
      }
    }
    bool accept = false;
    double phin;
    if constexpr (AuxLds<PMAX, NT>::kInLds) {
      // stage the end state (u in slot 0, m in slot 1): no chunk arrays stay
      // live through the likelihood and the copy-out
#pragma unroll
      for (int jj = 0; jj < PMAX; ++jj) {
        X.a[0][jj][t] = u[jj];
        X.a[1][jj][t] = m[jj];
      }
      __syncthreads();
      phin = staged_nll<PMAX, NT>(X, nx, A.n_obs, A.y, A.sigma, L, t, girs);
    } else {
      phin = block_nll<PMAX, NT, FULL>(u, ch, nx, A.n_obs, A.y, A.sigma, L, t, par.hs, girs);
    }
    if (st != SCH_OK || !isfinite(phin)) phin = INFINITY;
    double v;
    if constexpr (MATERN)
      v = uniform1(A.seed, static_cast<uint32_t>(p), A.cycle, SCH_TAG_ACCEPT << 24, w3);
    else
      v = A.vacc[static_cast<size_t>(j) * gridDim.x + p];
    if (phin < INFINITY) {
      const double logr = theta * (phi - phin);
      accept = logr >= 0.0 ? true : metropolis_below(v, logr);
    }
    if (accept) {
      if constexpr (MATERN) {
        double* tmp = cur;
        cur = prop;
        prop = tmp;
      } else {
        for (int i = t; i < S * Q; i += NT) cur[i] = prop[i];
      }
      if constexpr (AuxLds<PMAX, NT>::kInLds) {
        double* me = A.m_end + static_cast<size_t>(p) * nx;
        double* ue = A.u_end + static_cast<size_t>(p) * nx;
        for (int i = t; i < nx; i += NT) {
          me[i] = staged_at(X, 1, nx, i);
          ue[i] = staged_at(X, 0, nx, i);
        }
      } else {
        store_chunk<PMAX, FULL>(A.m_end + static_cast<size_t>(p) * nx, ch, m);
        store_chunk<PMAX, FULL>(A.u_end + static_cast<size_t>(p) * nx, ch, u);
      }
      phi = phin;
      ++acc;
    }
    __syncthreads();
  }
  if constexpr (MATERN) {
    // the accepted increments sit in the stage row after an odd number of
    // swaps: the workgroup copies the row back, consecutive threads on
    // consecutive values (the last move's barrier has made every thread's
    // proposal stores visible)
    if (cur != dWp) {
      const size_t len = static_cast<size_t>(S) * nx;
      for (size_t i = t; i < len; i += NT) dWp[i] = cur[i];
    }
  } else {
    if (acc > 0)
      for (int i = t; i < S * Q; i += NT) dWp[i] = cur[i];
  }
  if (t == 0) {
    A.phi[p] = phi;
    if (A.n_accept) A.n_accept[p] = acc;
    if (A.accept_acc) atomicAdd(A.accept_acc, static_cast<unsigned long long>(acc));
    if (A.iters_acc) atomicAdd(A.iters_acc, static_cast<unsigned long long>(iters));
  }
}

// Initial velocities of the paper's experiments (section 4, eq. init_solve),
// one workgroup per particle: DG0 cell values W_i = sqrt(h) z_i (tag INIT,
// counter (p, 0, pair | tag << 24, 0)), U^{0,3} from |W| by matern_add with
// M = (M + K, load h/2, k = 3), and (alpha, beta) from the block at
// (p, 1, tag << 24, 0): u = alpha^2 U^{0,3} + beta^2.
template <int PMAX, int NT, bool FULL>
__global__ void __launch_bounds__(NT) k_paper_init(const StepParams P, const MaternDev M,
                                                   uint64_t seed, double* u) {
  __shared__ RowLds<NT> L;
  const int p = blockIdx.x, t = threadIdx.x;
  const Chunk ch = chunk_of<NT>(P.nx, t);
  constexpr uint32_t tag = SCH_TAG_INIT << 24;
  double z[PMAX], w[PMAX], e[PMAX];
  cell_normals<PMAX, FULL>(seed, static_cast<uint32_t>(p), 0u, tag, 0u, ch, z);
  const double sh = sqrt(P.h);
#pragma unroll
  for (int j = 0; j < PMAX; ++j) {
    w[j] = fabs(sh * z[j]);
    e[j] = 0.0;
  }
  Parity par;
  matern_add<PMAX, NT, FULL>(M, w, e, ch, L, t, par);
  double a, b;
  normal2(seed, static_cast<uint32_t>(p), 1u, tag, 0u, a, b);
#pragma unroll
  for (int j = 0; j < PMAX; ++j) e[j] = a * a * e[j] + b * b;
  store_chunk<PMAX, FULL>(u + static_cast<size_t>(p) * P.nx, ch, e);
}

// Matern-type noise fields of n rows of cell increments (one workgroup per
// row): out = Delta U_k of matern_add.
template <int PMAX, int NT, bool FULL>
__global__ void __launch_bounds__(NT) k_matern_field(const StepParams P, const MaternDev M,
                                                     const double* cells, double* out) {
  __shared__ RowLds<NT> L;
  const int p = blockIdx.x, t = threadIdx.x;
  const Chunk ch = chunk_of<NT>(P.nx, t);
  double w[PMAX], e[PMAX];
  load_chunk<PMAX, FULL>(cells + static_cast<size_t>(p) * P.nx, ch, w);
#pragma unroll
  for (int j = 0; j < PMAX; ++j) e[j] = 0.0;
  Parity par;
  matern_add<PMAX, NT, FULL>(M, w, e, ch, L, t, par);
  store_chunk<PMAX, FULL>(out + static_cast<size_t>(p) * P.nx, ch, e);
}

// u = H^{-1} M m (mode 0) or m = M^{-1} H u (mode 1) for every particle.
struct HelmArgs {
  StepParams P;
  const double* in;
  double* out;
  int mode;
};

template <int PMAX, int NT, bool FULL>
__global__ void __launch_bounds__(NT) k_helmholtz(const HelmArgs A, const HelmConst K) {
  __shared__ RowLds<NT> L;
  const int p = blockIdx.x, t = threadIdx.x;
  const Chunk ch = chunk_of<NT>(A.P.nx, t);
  double v[PMAX], o[PMAX];
  load_chunk<PMAX, FULL>(A.in + static_cast<size_t>(p) * A.P.nx, ch, v);
  int hs = 0;
  if (A.mode == 0) {
    // the mass product folded into the scan form (the bordering values are
    // not used)
    double uL, uR, g0, g1, g2;
    solve_helm<PMAX, NT, FULL, true>(K, v, o, uL, uR, ch.cnt, L, 0, t, 0.0, 0.0, 0.0, g0, g1, g2,
                                     0.0, 0.0);
  } else {
    // right-hand side H u = M u + alpha^2 K u, then the mass solve
    double hl, hr;
    halo<PMAX, NT, FULL>(v, ch.cnt, L, t, hl, hr, hs);
    double r[PMAX];
#pragma unroll
    for (int j = 0; j < PMAX; ++j)
      r[j] = K.ho * (left_of<PMAX, FULL>(v, j, hl) + right_of<PMAX, FULL>(v, j, ch.cnt, hr)) +
             K.hd * v[j];
    const double mo = A.P.h / 6.0, md = 2.0 * A.P.h / 3.0;
    auto rowM = [&](int, double& a, double& b, double& c) {
      a = mo;
      b = md;
      c = mo;
    };
    double ol, orr;
    cyclic_solve<PMAX, NT, FULL>(rowM, [&](int j) { return r[j]; }, o, ch.cnt, L, t, ol, orr);
  }
  store_chunk<PMAX, FULL>(A.out + static_cast<size_t>(p) * A.P.nx, ch, o);
}

}  // namespace sch
